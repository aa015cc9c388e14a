// Device-scalar slots and vector kernels of the outer iterations.
#pragma once
#include "hdg_internal.hpp"

namespace hdg {

enum {
  SC_RZ = 0, SC_PAP = 1, SC_ALPHA = 2, SC_BETA = 3, SC_RNORM2 = 4, SC_GNORM2 = 5, SC_TMP = 6, SC_GRES = 7,
  SC_HNORM = 8, SC_ONE = 9, SC_COUNT = 16
};
enum { FIN_STORE = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RZ0 = 3, FIN_NORM_INV = 4 };

struct Scratch {
  double* sc = nullptr;        // device scalars [SC_COUNT]
  double* partials = nullptr;  // [2 * 512]
  unsigned* counter = nullptr; // [1], zero between launches
};

void blas_dot(const double* x, const double* y, long n, Scratch& s, int mode, double* out, hipStream_t st);
void blas_dot2_flex(const double* r, const double* z, const double* zold, long n, Scratch& s, hipStream_t st);
void blas_cg_update(double* lam, double* r, const double* p, const double* Ap, long n, Scratch& s,
                    hipStream_t st);
void blas_cg_direction(double* p, const double* z, long n, Scratch& s, hipStream_t st);
void blas_axpy(double* y, const double* x, long n, const double* coef, double sign, hipStream_t st);
void blas_scale(double* y, const double* x, long n, const double* coef, hipStream_t st);
void blas_d2f(const double* x, float* y, long n, hipStream_t st);
void blas_f2d(const float* x, double* y, long n, hipStream_t st);
void blas_copy(double* y, const double* x, long n, hipStream_t st);
template <typename T>
void blas_copy_t(T* y, const T* x, long n, hipStream_t st);
template <typename T>
void blas_fill(T* y, T v, long n, hipStream_t st);
void blas_gmres_rot(double* H, double* cs, double* sn, double* s, int j, int ld, double* sc, hipStream_t st);
void blas_gmres_backsolve(const double* H, const double* s, int j, int ld, double* y, hipStream_t st);
void blas_gmres_combine(double* x, const double* Z, long ldz, int j, const double* y, long n, hipStream_t st);
void blas_set_scalar(double* sc, int slot, const double* src, int negate, hipStream_t st);
void blas_finite(const double* x, long n, int* bad, hipStream_t st);

}  // namespace hdg
