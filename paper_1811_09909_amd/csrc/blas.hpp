// Device-scalar slots and vector kernels of the outer iterations.
#pragma once
#include "hdg_internal.hpp"

namespace hdg {

enum {
  SC_RZ = 0, SC_PAP = 1, SC_ALPHA = 2, SC_BETA = 3, SC_RNORM2 = 4, SC_GNORM2 = 5, SC_TMP = 6, SC_GRES = 7,
  SC_HNORM = 8, SC_RZOLD = 10, SC_HCNT = 11, SC_HIST = 16,
  HIST_MAX = 64,                   // residual norms kept between two host reads
  SC_COUNT = SC_HIST + HIST_MAX
};
// finalisers of a reduction (applied by the one-block finaliser)
enum {
  FIN_STORE = 0,        // *out = s
  FIN_ALPHA = 1,        // pAp = s, alpha = rz / s
  FIN_BETA = 2,         // beta = s / rz, rz = s
  FIN_RZ0 = 3,          // rz = s
  FIN_NORM_INV = 4,     // *out = sqrt(s), tmp = 1 / sqrt(s)
  FIN_BETA_FLEX = 5,    // beta = (s - rzold) / rz, rz = s
  FIN_RNORM = 6,        // rnorm2 = s
  FIN_RNORM_RZOLD = 7,  // rnorm2 = s0, rzold = s1
  FIN_GNORM = 8         // gnorm2 = s
};

constexpr int MAX_RED_BLOCKS = 4096;

struct Scratch {
  double* sc = nullptr;        // device scalars [nrhs][SC_COUNT]
  double* partials = nullptr;  // [nrhs][2 * max(MAX_RED_BLOCKS, blocks of the widest reducing launch)]
  long row = 0;                // partials per right-hand side
  double* pcg = nullptr;       // partials of the fused CG update [nrhs][2 * MAX_RED_BLOCKS]
};

// nrhs: vectors of length n stored one after another; each right-hand side
// has its own scalars (sc + rhs * SC_COUNT) and row of partials.
void blas_finalize(int nb, int nv, int mode, double* out, Scratch& s, hipStream_t st, int nrhs = 1);
void blas_dot(const double* x, const double* y, long n, Scratch& s, int mode, double* out, hipStream_t st,
              int nrhs = 1);
template <typename ZT>
void blas_cg_update2(double* lam, double* r, float* r32, const double* p, const double* Ap, const ZT* z, long n,
                     Scratch& s, hipStream_t st, int nrhs = 1);
template <typename ZT>
void blas_rz(const double* r, const ZT* z, long n, int mode, Scratch& s, hipStream_t st, int nrhs = 1);
// CG iteration with two finalisers instead of four: the update takes alpha
// from the pAp partials (npap per right-hand side, in s.partials) itself and
// keeps its own partials in s.pcg; the r.z reduction's finaliser then also
// does the update's (residual norm and history, rz_old), then beta
// (Polak-Ribiere when flex).  Same sums in the same order as the separate
// finalisers.
template <typename ZT>
void blas_cg_update2_fused(double* lam, double* r, float* r32, const double* p, const double* Ap, const ZT* z,
                           long n, int npap, Scratch& s, hipStream_t st, int nrhs = 1);
template <typename ZT>
void blas_rz_cg(const double* r, const ZT* z, long n, bool flex, Scratch& s, hipStream_t st, int nrhs = 1);
// the same finaliser when the r.z partials (nrz per right-hand side) were
// written by the preconditioner's last sweep
void blas_finalize_cg(long n, int nrz, bool flex, Scratch& s, hipStream_t st, int nrhs = 1);
template <typename ZT>
void blas_cg_dir(double* p, const ZT* z, long n, Scratch& s, hipStream_t st, int nrhs = 1);
template <typename ZT>
void blas_add(double* lam, const ZT* z, long n, hipStream_t st, int nrhs = 1);
void blas_axpy(double* y, const double* x, long n, const double* coef, double sign, hipStream_t st);
void blas_scale(double* y, const double* x, long n, const double* coef, hipStream_t st);
void blas_d2f(const double* x, float* y, long n, hipStream_t st, int nrhs = 1);
void blas_f2d(const float* x, double* y, long n, hipStream_t st, int nrhs = 1);
void blas_copy(double* y, const double* x, long n, hipStream_t st, int nrhs = 1);
template <typename T>
void blas_copy_t(T* y, const T* x, long n, hipStream_t st, int nrhs = 1);
template <typename T>
void blas_fill(T* y, T v, long n, hipStream_t st, int nrhs = 1);
void blas_gmres_rot(double* H, double* cs, double* sn, double* s, int j, int ld, double* sc, hipStream_t st);
void blas_gmres_backsolve(const double* H, const double* s, int j, int ld, double* y, hipStream_t st);
void blas_gmres_combine(double* x, const double* Z, long ldz, int j, const double* y, long n, hipStream_t st);

}  // namespace hdg
