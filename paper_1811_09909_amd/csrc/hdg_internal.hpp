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
  // P^k triangles (unstructured handles only; the UHost reference matrices)
  double *uM = nullptr, *uMinv = nullptr, *uD = nullptr, *uE = nullptr, *uF = nullptr, *uH = nullptr;
  double *uK = nullptr, *uN = nullptr, *uDe = nullptr, *uGn = nullptr;  // IPDG on triangles
};

// ---------------------------------------------------------------------------
// Unstructured triangle meshes (umesh.cpp; host, built once per mesh).
// A level has cells (triangles, or macro-elements of an agglomeration level)
// with slots (their faces; -1: an edge on the domain boundary) and faces with
// m trace values each (k + 1 on the finest level, 2 on P^1 levels).  Face f
// joins cells fcell[2f] < fcell[2f+1] at their slots fslot[2f], fslot[2f+1];
// its chain runs from vertex fstart to fend with length flen.  The
// h-transition arrays describe the agglomeration into the next level.
struct UHostLevel {
  int m = 2;
  bool tri = false;                 // cells are the triangles (three slots each)
  long ncell = 0, nface = 0;
  std::vector<long> sptr;           // [ncell + 1] slot offsets
  std::vector<int> sface;           // [nslot] face of each slot, -1 none
  std::vector<int> fcell, fslot;    // [2 nface]
  std::vector<int> fstart, fend;    // [nface] chain end vertices
  std::vector<double> flen;         // [nface] chain lengths
  // h-transition to the next level (empty on the coarsest)
  long ncoarse = 0;
  std::vector<long> ccptr;          // [ncoarse + 1] fine cells of each coarse cell
  std::vector<int> ccell;
  std::vector<long> iptr;           // [ncoarse + 1] interior faces (E_I) of each coarse cell, ascending
  std::vector<int> iface;
  std::vector<long> bptr;           // [ncoarse + 1] boundary faces (E_B) of each coarse cell, ascending
  std::vector<int> bface, bslot;    // ... and the coarse slot of each one's macro-edge
  std::vector<int> sloc;            // [nslot] local face of every slot in its coarse cell (E_I first)
  std::vector<int> fE;              // [nface] macro-edge of each E_B face, -1 for E_I
  std::vector<double> fJ;           // [4 nface] J block of each E_B face: [fine DOF][macro-edge DOF]
  // (on the coarse level) the finer faces of each macro-edge in chain order
  std::vector<long> eptr;
  std::vector<int> efine;
};

// largest dense local problem of a coarse cell (E_I and E_B values) and the
// largest coarsest level of an unstructured hierarchy
constexpr int UMACRO_MAX_DOFS = 1024;
constexpr int UCOARSE_MAX = 4096;

struct UHost {
  int k = 1, nv = 0, ne = 0;
  long nvert = 0, ntri = 0, nbedge = 0;
  std::vector<double> xy;
  std::vector<int> tri;
  std::vector<int> tbnd;            // [3 ntri] boundary edge of each slot (sorted vertex pairs), -1 interior
  std::vector<int> nmacro;          // macro-elements per agglomeration level (level 1 first)
  std::vector<UHostLevel> lev;      // finest first: P^k triangles, P^1 triangles (k > 1), T_hlevels .. T_1
  // reference triangle (0,0), (1,0), (0,1), nodal P^k at the equispaced
  // lattice, P^k edge traces nodal at GLL points of the edge parameter
  std::vector<double> Mh, Minvh;    // [nv][nv] mass and its inverse
  std::vector<double> Dh;           // [2][nv][nv] (d_r phi_i, phi_j)
  std::vector<double> Eh;           // [3][nv][nv] edge s (from vertex s to s+1, unit parameter): <phi_i, phi_j>
  std::vector<double> Fh;           // [3][nv][ne] <phi_i, mu_a> on edge s, mu in the edge's own direction
  std::vector<double> Hh;           // [ne][ne] <mu_a, mu_b> on the unit parameter
  std::vector<double> Jp;           // [ne][2] P^1 end values -> GLL values
  // primal (IPDG) forms on the reference triangle
  std::vector<double> Kh;           // [2][2][nv][nv] (d_r phi_i, d_r' phi_j)
  std::vector<double> Nh;           // [3][2][nv][nv] edge s: <d_r phi_i, phi_j>
  std::vector<double> De;           // [3][2][nv][ne] edge s: <d_r phi_i, mu_a>
  std::vector<double> Gnode;        // [2][nv][nv] d_r phi_j at node a
  void build_reference(int k);
  void build_mesh(long nvert, const double* xy, long ntri, const int* tri, const double* seeds, int nseeds,
                  int hlevels);
  UHostLevel coarsen(UHostLevel& fine, const std::vector<int>& coarse_of, long ncoarse);
};

// Device copies of an unstructured level's index arrays (set up once per
// mesh) and its per-build storage.  Cell maps are row-major per cell at
// moff[c] (Level.Aelem in FP64, Am32 in FP32); triangle levels also keep
// them AoSoA over triangles in 16-byte groups (pk_off; Level.Af64 / Af32)
// for the element phase of the apply.  z holds the element phase's
// products, one row per (cell, slot, value): face f's value a from its
// side's cell sits at zr[2f + side] + a * zstride (zstride 1: rows of a
// face side are consecutive).
struct ULevel {
  int m = 2;
  bool tri = false;
  long ncell = 0, nrow = 0, nface = 0;
  long* sptr = nullptr;
  int* sface = nullptr;
  int* rcell = nullptr;   // [nrow] cell of each row
  long* moff = nullptr;   // [ncell]
  long msize = 0;         // entries of all cell maps
  long* zr = nullptr;     // [2 nface]
  int zstride = 1;
  int* fcell = nullptr;
  int* fslot = nullptr;
  float* Am32 = nullptr;
  void* z[2] = {nullptr, nullptr};
  // h-transition to the next level
  long ncoarse = 0, nIrow = 0, ncb = 0, nwork = 0, asize = 0, psize = 0;
  long* csptr = nullptr;  // the next level's slot offsets and slot faces
  int* csface = nullptr;
  long *iptr = nullptr, *bptr = nullptr, *ccptr = nullptr;
  int *iface = nullptr, *bface = nullptr, *bslot = nullptr, *ccell = nullptr, *sloc = nullptr;
  int *irc = nullptr, *cbc = nullptr;  // coarse cell of every interior row / restriction-share row
  long *aoff = nullptr, *poff = nullptr, *woff = nullptr;
  int* fE = nullptr;
  double* fJ = nullptr;
  long* eptr = nullptr;   // (coarse level) finer faces of each macro-edge
  int* efine = nullptr;
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
  // unstructured levels: index arrays and element-phase storage (null on
  // the grid levels)
  ULevel* u = nullptr;
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

// Persistent coarse cycle (2D, one right-hand side): the levels from an
// h-level down to the coarsest run in one launch of one workgroup per
// compute unit, phases separated by grid-wide barriers, the vectors in the
// levels' own device buffers.  Each phase is the work item the per-level
// kernels run, in the same lane layout, so the results are theirs bit for
// bit.  sync: [0] arrivals, [32] barrier generation, [64] error flag (a
// barrier wait that ran out of polls; the launch then still ends).
struct GTailLevel {
  int n = 0, kind = 2, sweeps = 0, lpm = 1;
  long nlam = 0, nface = 0, nmacro = 0;
  const void *Af = nullptr, *Dinv = nullptr, *AIIinv = nullptr, *R = nullptr, *P = nullptr, *Ainv = nullptr;
  void *r = nullptr, *e = nullptr, *w = nullptr, *cb = nullptr;
};
struct GTailArgs {
  int nlev = 0, lc = 0;
  GTailLevel lev[TAIL_MAX_LEVELS];
  unsigned* sync = nullptr;
};
// lanes per macro-element the fused 2D transition kernels use on level L
int level_lanes(const Level& L, int nrhs);
#ifndef HDG_GTAIL_NMAX
#define HDG_GTAIL_NMAX 128
#endif
constexpr int GTAIL_NMAX = HDG_GTAIL_NMAX;  // largest grid (elements per direction) the persistent cycle starts on
constexpr int GTAIL_THREADS = 256;
constexpr int GTAIL_SYNC_WORDS = 96;
// workgroups of the persistent launch: one per compute unit, 0 if the
// device cannot hold them all at once
template <typename T>
int gtail_grid();
template <typename T>
void launch_gtail(const GTailArgs& a, int grid, hipStream_t st);

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

// unstructured.hip.  HDG element maps of P^k triangles (A^e row-major
// [ntri][3ne][3ne]) and the load map W ([ntri][nv][3ne], b^e = W^T f for
// nodal f); loads pulled per face; the P^1 Galerkin maps of the triangles;
// per coarse cell the Schur complement, A_II^-1 and P = -A_II^-1 A_IB J
// (eqs. Akm1, n_1_Ik) into the next level's maps; face-block inverses;
// the coarsest dense inverse; AoSoA / FP32 copies of the maps.
// Rec (optional): recovery maps [ntri][3][nv][3ne + nv] taking [Lambda_T; f_T]
// to the nodal q_x, q_y and u of the triangle
void launch_tri_dtn(int k, long ntri, const RefDevice& rd, const double* xy, const int* tri, const double* kappa,
                    double tau, double* Aelem, double* W, double* Rec, hipStream_t st);
// g (gdir: boundary traces [nbedge][ne], lifted with the element maps; may be null)
// the hybridized IPDG family on triangles (eq. IPG_H, s_f = sf): the same
// outputs (recovery: u and q = -kappa grad u at the nodes)
void launch_tri_ipdg_dtn(int k, long ntri, const RefDevice& rd, const double* xy, const int* tri,
                         const double* kappa, double tau, double sf, double* Aelem, double* W, double* Rec,
                         hipStream_t st);
void launch_tri_load(int k, const ULevel& U, const double* W, const double* f, const double* Aelem,
                     const int* tbnd, const double* gdir, double* g, hipStream_t st);
void launch_tri_reconstruct(int k, long ntri, const int* sface, const int* tbnd, const double* Rec,
                            const double* lam, const double* gdir, const double* f, double* u, double* q,
                            hipStream_t st);
void launch_tri_pgalerkin(int k, long ntri, const double* Jp, const double* A0, double* A1, hipStream_t st);
// R (null when the operator is symmetric): the restriction block
// -A_II^-T A_BI^T J of every coarse cell, laid out as P
void launch_uschur(const ULevel& F, const ULevel& C, const double* Afine, double* AIIinv, double* P, double* R,
                   double* Acoarse, double* work, hipStream_t st);
void launch_udinv(const Level& L, hipStream_t st);
void launch_ucoarse_inverse(const Level& L, double* work, hipStream_t st);
// in-place inverse of a dense N x N matrix (row-major) by Gauss-Jordan over
// 64 x 64 blocks, no pivoting; Pb: 4,096 doubles of device scratch
void launch_dense_inverse_blocked(long N, double* A, double* Pb, hipStream_t st);
void launch_umaps(const Level& L, hipStream_t st);
void launch_to_f32(const double* x, float* y, long n, hipStream_t st);
// unstructured trace kernels (dispatched from the launchers above when L.u
// is set)
template <typename T, typename M>
void launch_uapply(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc, float* y32,
                   Scratch* red, hipStream_t st, int nrhs, int* nparts);
template <typename T, typename M>
void launch_ucorr(const Level& L, const T* rho, T* e, int do_corr, int do_restrict, T* cb, hipStream_t st, int nrhs);
template <typename T>
void launch_urestrict(const Level& L, const Level& C, const T* rho, const T* cb, T* rc, hipStream_t st, int nrhs);
template <typename T, typename M>
void launch_uprolong(const Level& L, const Level& C, const T* ec, T* e, hipStream_t st, int nrhs);

// noalloc.hip: the device address of this device's fixed staging array
// (looked up once per device) and its size in doubles
double* scratch_ptr();
long scratch_capacity();
// api.cpp: staging the load form of hdg_rhs needs, and hdg_rhs with the
// staging buffer given (no allocation)
long rhs_staging_doubles(const hdg_problem* P);
// whether the handle forms g from this kind of data (unstructured handles:
// nodal f with zero Dirichlet data only)
bool rhs_supported(const hdg_problem* P, int kind, const double* gdir);
void rhs_with_staging(hdg_problem* P, const double* rhs, int kind, const double* gdir, double* g, double* ebuf);

}  // namespace hdg
