// Internal declarations of the HDG trace multigrid library (host + device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "hdg.h"

namespace hdg {

constexpr int LANES = 64;  // AoSoA block width = one wavefront

inline long pad64(long n) { return (n + LANES - 1) / LANES * LANES; }

// Stored operator blocks (face matrices, face-block inverses, macro-element
// blocks) are AoSoA: 64 items per block, and inside a block the entries of one
// item come in groups of VW = max(1, HDG_VEC_BYTES / sizeof(T)) consecutive
// values, so a lane loads one group and a wavefront one contiguous segment:
//   off(item, e) = (item / 64) * per * 64 + (e / VW) * 64 * VW + (item % 64) * VW + e % VW
// with `per` the item's entry count padded to a multiple of VW.  The default
// (one entry per lane and load) measured fastest on gfx950: wider groups make
// the compiler hoist every load of a face and drop to one wave per SIMD.
#ifndef HDG_VEC_BYTES
#define HDG_VEC_BYTES 4
#endif
template <typename T>
__host__ __device__ constexpr int vw() {
  return HDG_VEC_BYTES / (int)sizeof(T) > 1 ? HDG_VEC_BYTES / (int)sizeof(T) : 1;
}
template <typename T>
__host__ __device__ constexpr long vpad(long cnt) {
  return (cnt + vw<T>() - 1) / vw<T>() * vw<T>();
}
// Packed element maps use their own group width (HDG_PACK_VEC_BYTES, default
// 16: a lane loads 2 doubles or 4 floats at a time; measured on MI355X, the
// FP64 element phase runs 154 -> 116 us at 512^2, k = 4, the FP32 one is
// unchanged): entry e of element T of a map with npk entries (padded to a
// multiple of the width) sits at
//   (T / 64) * npkp * 64 + (e / W) * 64 * W + (T % 64) * W + e % W.
#ifndef HDG_PACK_VEC_BYTES
#define HDG_PACK_VEC_BYTES 16
#endif
template <typename T>
__host__ __device__ constexpr int pvw() {
  return HDG_PACK_VEC_BYTES / (int)sizeof(T) > 1 ? HDG_PACK_VEC_BYTES / (int)sizeof(T) : 1;
}
template <typename T>
__host__ __device__ constexpr long pk_pad(long npk) {
  return (npk + pvw<T>() - 1) / pvw<T>() * pvw<T>();
}
template <typename T>
__host__ __device__ inline long pk_off(long T_, long npk, long e) {
  constexpr int W = pvw<T>();
  return (T_ >> 6) * pk_pad<T>(npk) * LANES + (e / W) * (LANES * W) + (T_ & 63) * W + e % W;
}

template <typename T>
__host__ __device__ inline long aos_off(long item, long per, long e) {
  constexpr int V = vw<T>();
  return (item >> 6) * per * LANES + (e / V) * (LANES * V) + (item & 63) * V + e % V;
}
// start of an item's entries (entry 0); group g then sits at + g * 64 * VW
template <typename T>
__host__ __device__ inline long aos_item(long item, long per) {
  return (item >> 6) * per * LANES + (item & 63) * vw<T>();
}

struct HipError {
  hipError_t err;
  std::string where;
};

#define HDG_CHECK(x)                                                        \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) throw ::hdg::HipError{e_, std::string(#x)};       \
  } while (0)

// ---------------------------------------------------------------------------
// Reference element (host).  Q^k on [0,h]^d, GLL-nodal, Gauss rules with k+2
// points per direction.  All matrices are row-major and already scaled by the
// powers of h of a cell of size h.
struct RefElement {
  int d = 0, k = 0, nv = 0, ne = 0, nf = 0, nl = 0, nq = 0, nc = 0;
  double h = 0;
  std::vector<double> gll, gauss, gw;  // 1D
  std::vector<double> Phi;             // [nq][nv]
  std::vector<double> Wq;              // [nq]
  std::vector<double> B;               // [d][nv][nv]: B[c][i][j] = (d_c phi_j, phi_i)
  std::vector<double> F;               // [d][nv][nl]: <mu_m, phi_i n_c> on faces of normal c
  std::vector<double> G;               // [nv][nl]:   <mu_m, phi_i>
  std::vector<double> E;               // [nv][nv]:   <phi_j, phi_i> on the element boundary
  std::vector<double> H;               // [nl][nl]:   face mass
  std::vector<double> M;               // [nv][nv]:   volume mass
  std::vector<double> Jp;              // [ne][nc]:   P1/Q1 face vertex values -> GLL values
  // primal (IPDG) forms
  std::vector<double> Kst;             // [nv][nv]:   (grad phi_j, grad phi_i)
  std::vector<double> Nn;              // [nv][nv]:   <phi_j, grad phi_i . n> on the element boundary
  std::vector<double> Dn;              // [nv][nl]:   <mu_m, grad phi_i . n>
  std::vector<double> Dnode;           // [d][nv][nv]: d_c phi_j at node a
  // hybridized Raviart-Thomas forms (d = 2; build_rt): nqc coefficients per
  // velocity component, nqv = 2 nqc
  int nqc = 0, nqv = 0;
  std::vector<double> Vq;              // [2][nq][nqc]: component basis at the Gauss points
  std::vector<double> Bd;              // [nqv][nv]:   (phi_j, div v_I)
  std::vector<double> Fr;              // [nqv][nl]:   <mu_m, v_I . n>
  std::vector<double> Vnode;           // [2][nv][nqc]: component basis at the scalar's nodes
  void build(int d, int k, double h);
  void build_rt();
};

void gll_points(int k, std::vector<double>& x);                       // k+1 points on [0,1]
void gauss_points(int n, std::vector<double>& x, std::vector<double>& w);  // on [0,1]

// Device copies of the reference data
struct RefDevice {
  double *Phi = nullptr, *Wq = nullptr, *B = nullptr, *F = nullptr, *G = nullptr, *E = nullptr,
         *H = nullptr, *M = nullptr, *Jp = nullptr;
  double *Kst = nullptr, *Nn = nullptr, *Dn = nullptr, *Dnode = nullptr;  // IPDG handles only
  double *Vq = nullptr, *Bd = nullptr, *Fr = nullptr, *Vnode = nullptr;    // RT-H handles only
};

// ---------------------------------------------------------------------------
// One multigrid level.  The local operators are stored twice: element form
// (row-major [nelem][nl][nl], FP64; input of the next coarsening) and face
// form (AoSoA over interior faces with 16-byte entry groups, see aos_off;
// FP64 and FP32; read by the apply).  Face F holds 2 * S entries, S =
// vpad<T>(nl * ne):
//   entry side * S + j * ne + a  =  A_{T_side}[slot_side * ne + a][j]
// where side 0 is the element below the face along its normal (the face is
// its slot 2c+1), side 1 the element above (slot 2c).  Dinv holds the
// ne x ne row-major block of face F as its vpad<T>(ne * ne) entries.
struct Level {
  int d = 0, n = 0, ne = 0, nl = 0;
  long nelem = 0, nfd = 0, nface = 0, nlam = 0;
  int kind = 2;  // 0: p-transition below, 1: h-transition below, 2: coarsest
  int sweeps = 2;
  double* Aelem = nullptr;  bool own_Aelem = true;
  double* Af64 = nullptr;   float* Af32 = nullptr;
  double* Dinv64 = nullptr; float* Dinv32 = nullptr;
  // Element-major packed form (used instead of Af on the finest level of a
  // p-transition): the upper triangle of each symmetric element map, row by
  // row, AoSoA over elements in groups of 16 bytes (pk_off), and the
  // per-element products z_T = A^e x_T ([nrhs][nelem padded to 64][nl],
  // elem_aos) of the two-phase apply.  `strip`: the one-pass strip apply is
  // used (2D, n a multiple of 64); z then holds its strip-edge products.
  bool packed = false;
  bool strip = false;
  // smoother data beyond Dinv: the Chebyshev smoother's per-step copies of
  // the diagonal blocks scaled by 1 / (root i of its polynomial), and the
  // eigenvalue estimate they come from
  std::vector<double*> cheb64;
  std::vector<float*> cheb32;
  double lmax = 0.0;
  // lanes per macro-element of the fused h-transition kernels: 0 = by the
  // size of the level (four while macro-elements x right-hand sides are
  // few, one above), or forced to 1 or 4 (a tile shape the autotuner tries)
  int lpm = 0;
  double* Ap64 = nullptr;   float* Ap32 = nullptr;
  void* z[2] = {nullptr, nullptr};
  // h-transition to the next level
  long nmacro = 0;
  int nI = 0, ncl = 0;
  double* AIIinv64 = nullptr; float* AIIinv32 = nullptr;  // AoSoA over M, row-major nI x nI
  double* P64 = nullptr;      float* P32 = nullptr;       // AoSoA over M, row-major nI x ncl
  // restriction block R = -A_II^-T A_BI^T J (eq. n_1_Qk: the macro-element
  // share of Q is R^T rho_I); the same array as P when the level operator is
  // symmetric (then R = P), its own array otherwise
  double* R64 = nullptr;      float* R32 = nullptr;
  bool sym = true;  // the level operator is symmetric
  // coarsest direct inverse (dense row-major nlam x nlam)
  double* Ainv64 = nullptr; float* Ainv32 = nullptr;
  // work vectors, [0] = FP64, [1] = FP32
  void* r[2] = {nullptr, nullptr};
  void* e[2] = {nullptr, nullptr};
  void* w[2] = {nullptr, nullptr};
  void* cb[2] = {nullptr, nullptr};
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All run on `st`.
// element.hip (tau_kappa != 0: element T is stabilized with tau * kappa_T,
// kappa per element)
void launch_element_dtn(int d, int k, long nelem, double tau, int tau_kappa, const RefDevice& rd, const double* kqp,
                        double* Aelem, double* W, double* Kinv, double* Minv, hipStream_t st);
void launch_element_load(int d, int k, long nelem, const RefDevice& rd, const double* f, int is_load,
                         const double* W, double* ebuf, hipStream_t st);
void launch_load_pull(int d, int k, int n, const double* ebuf, const double* Aelem, const double* gdir,
                      double* g, hipStream_t st);
void launch_reconstruct(int d, int k, int n, double tau, int tau_kappa, const RefDevice& rd, const double* kqp, const double* lam,
                        const double* gdir, const double* f, int is_load, const double* W, const double* Kinv,
                        const double* Minv, double* b, double* u, double* q, hipStream_t st);
// hybridized IPDG family (eq. IPG_H): A^e, the load map W = L^-T C^T and,
// when X / Linv are given, the recovery blocks X = L^-1 R and L^-1
// (mask: per-element scheme codes, only elements with `code` formed; null: all)
void launch_ipdg_dtn(int d, int k, long nelem, const int* mask, int code, double tau, int tau_kappa, double sf,
                     const RefDevice& rd, const double* kqp, int nq, double* Aelem, double* W, double* X,
                     double* Linv, hipStream_t st);
// hybridized Raviart-Thomas (d = 2, k <= 4): A^e, the load map, and when Xr
// is given the recovery blocks (Xr, Luu for u; Xq, Yq for the nodal flux)
void launch_rt_dtn(int k, long nelem, const int* mask, int code, const RefDevice& rd, const double* kqp,
                   double* Aelem, double* W, double* Xr, double* Luu, double* Xq, double* Yq, hipStream_t st);
// IPDG and RT-H recovery (RT-H elements: mask code rt_code, or all when mask
// is null and Xq is given)
void launch_ipdg_reconstruct(int d, int k, int n, const RefDevice& rd, const double* kqp, int nq, const int* mask,
                             int rt_code, const double* Xq, const double* Yq, const double* lam, const double* gdir,
                             const double* f, int is_load, const double* X, const double* Linv, double* b, double* u,
                             double* q, hipStream_t st);
void launch_grad(int d, int k, long nelem, const RefDevice& rd, const double* kqp, const double* q,
                 const double* qs, double* grad, hipStream_t st);
void launch_mass(int d, int k, long nelem, const RefDevice& rd, const double* u, double* out, hipStream_t st);
void launch_kappa_expand(long nelem, int nq, const double* kappa, int kind, double* kqp, int* bad,
                         hipStream_t st);

// build.hip
void launch_face_major(const Level& L, hipStream_t st);
void launch_pack_sym(const Level& L, hipStream_t st);
// mode 0: omega D_F^-1 (block Jacobi), 1: omega / diag(D_F) (point Jacobi),
// 2: D_F (point Gauss-Seidel), D_F the assembled diagonal block of face F
void launch_dinv(const Level& L, double omega, hipStream_t st, int mode = 0);
void launch_scale_copy(long n, double s, const double* src, double* d64, float* d32, hipStream_t st);
void launch_pgalerkin(int d, int ne, long nelem, const double* Jp, const double* Afine, double* Acoarse,
                      hipStream_t st);
void launch_macro_schur(const Level& fine, Level& coarse, hipStream_t st);
void launch_coarse_inverse(const Level& L, hipStream_t st);

// trace.hip.  Every launcher takes nrhs right-hand sides stored one after
// another (stride: the level's vector length) and runs them in one launch.
// T: vector type; M: storage type of the operator blocks read (the level's
// FP64 or FP32 copy; M = float under T = double on face-major levels only).
template <typename T, typename M = T>
void launch_apply(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc,
                  hipStream_t st, int nrhs = 1);
template <typename T, typename M = T>
void launch_jacobi0(const Level& L, const T* r, T* e, hipStream_t st, int nrhs = 1);
template <typename T>
void launch_prolong_p(const Level& L, int nc, const double* Jp, const T* ec, T* e, hipStream_t st, int nrhs = 1);
template <typename T, typename M = T>
void launch_hcorr(const Level& L, const T* rho, T* e, int do_corr, int do_restrict, T* cb, hipStream_t st,
                  int nrhs = 1);
template <typename T>
void launch_hrestrict(const Level& L, const Level& C, const T* rho, const T* cb, T* rc, hipStream_t st,
                      int nrhs = 1);
template <typename T, typename M = T>
void launch_hprolong(const Level& L, const Level& C, const T* ec, T* e, hipStream_t st, int nrhs = 1);
template <typename T, typename M = T>
void launch_coarse_solve(const Level& L, const T* r, T* e, hipStream_t st, int nrhs = 1);
// one colour pass of multicolour point symmetric Gauss-Seidel on a
// face-major level whose Dinv arrays hold the assembled face blocks: every
// face of colour col (normal col / 2, position parity col % 2) updates its
// values of x in place, in increasing order, or decreasing when backward
template <typename T, typename M = T>
void launch_sgs_color(const Level& L, int col, int backward, T* x, const T* b, hipStream_t st, int nrhs = 1);
template <typename T>
void launch_res_prestrict(const Level& L, const Level& C, const T* x, const T* b, T* rc, T* ec, const double* Jp,
                          hipStream_t st, int nrhs = 1);
// fused 2D h-transition kernels
template <typename T>
void launch_hpre(const Level& L, const T* r, T* e, int do_corr, T* cb, hipStream_t st, int nrhs = 1);
template <typename T>
void launch_hsum(const Level& L, const Level& C, const T* r, const T* cb, T* rc, T* ec, hipStream_t st,
                 int nrhs = 1);
template <typename T>
void launch_hpost(const Level& L, const Level& C, const T* r, const T* ec, const T* eold, T* enew, int do_corr,
                  hipStream_t st, int nrhs = 1);

// single-workgroup coarse tail of the V-cycle (tail.hip)
constexpr int TAIL_MAX_LEVELS = 12;
constexpr int TAIL_ARENA_BYTES = 144 * 1024;
struct TailLevel {
  int n = 0, kind = 2, sweeps = 0;
  long nlam = 0, nface = 0, nmacro = 0;
  const void *Af = nullptr, *Dinv = nullptr, *AIIinv = nullptr, *P = nullptr, *Ainv = nullptr;
  long off_r = 0, off_e = 0, off_w = 0, off_cb = 0;  // element offsets into the LDS arena
};
struct TailArgs {
  int nlev = 0, lc = 0, pre_done = 0;
  TailLevel lev[TAIL_MAX_LEVELS];
  const void* rin = nullptr;
  const void* ein = nullptr;
  void* eout = nullptr;
};
template <typename T>
void launch_tail(const TailArgs& a, hipStream_t st, int nrhs = 1);

// APPLY_SWEEP_DOT: a sweep that also sums v . y (partials, v FP64, passed
// where RES_PRESTRICT takes J_N) for the CG dot product r . z
enum {
  APPLY_Y = 0, APPLY_RES = 1, APPLY_SWEEP = 2, APPLY_RES_PRESTRICT = 3, APPLY_Y_DOT = 4, APPLY_RES_NORM = 5,
  APPLY_SWEEP_DOT = 6
};
struct Scratch;
// Modes with a reduction write per-block partials into red->partials; the
// one-block finaliser runs next, unless nparts is given: then it receives
// the number of partials per right-hand side (their row stride) and the
// caller finalises (e.g. inside the next kernel).
template <typename T, typename M = T>
void launch_apply_red(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc, float* y32,
                      Scratch* red, hipStream_t st, int nrhs = 1, int* nparts = nullptr);

// noalloc.hip: the device address of this device's fixed staging array
// (looked up once per device) and its size in doubles
double* scratch_ptr();
long scratch_capacity();
// api.cpp: staging the load form of hdg_rhs needs, and hdg_rhs with the
// staging buffer given (no allocation)
long rhs_staging_doubles(const hdg_problem* P);
void rhs_with_staging(hdg_problem* P, const double* rhs, int kind, const double* gdir, double* g, double* ebuf);

}  // namespace hdg
