// C ABI of the HDG trace multigrid library: problem setup, hierarchy build,
// V-cycle (Algorithm 1) and the outer iterations (Sec. 3.6 and Sec. 4), all
// driving the HIP kernels of element.hip, build.hip, trace.hip, blas.hip.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <chrono>
#include <limits>
#include <memory>
#include <new>
#include <stdexcept>
#include <thread>

#include "blas.hpp"
#include "hdg_internal.hpp"

using namespace hdg;

struct hdg_problem {
  int d = 0, n = 0, k = 0;
  double tau = 1.0;
  // discretization (HDG_SCHEME_*): s_f of eq. IPG_H, and whether the trace
  // operator is symmetric (HDG, SIPG-H)
  int scheme = HDG_SCHEME_HDG;
  double sf = 0.0;
  bool sym = true;
  bool tau_kappa = false;  // element T stabilized with tau * kappa_T (HDG_SCHEME_TAU_KAPPA)
  // multinumerics (scheme == SCHEME_MULTI): each element's scheme code on the
  // device, and the codes present
  int* emask = nullptr;
  std::vector<int> codes;
  hipStream_t st = nullptr;      // caller's stream: all work is ordered on it
  hipStream_t cap_st = nullptr;  // private stream used only to capture graphs
  // execution form, from hdg_mg_opts.variant at build
  bool use_graphs = true;        // replay captured graphs (HDG_VARIANT_NO_GRAPH: eager launches)
  bool fuse = true;              // fused 2D transition kernels (HDG_VARIANT_NO_FUSE: unfused)
  int tail_nmax = 32;            // largest grid handled by the one-workgroup coarse tail (0 = off)
  bool pack = true;              // element-major packed finest p-level (HDG_VARIANT_NO_PACK: face-major)
  bool strip = true;             // one-pass strip apply on packed levels (HDG_VARIANT_NO_STRIP: two-phase)
  double t_setup_ms = 0.0, t_build_ms = 0.0;  // host wall time of the last setup / build
  // form of the mixed cycle: false = FP32 vectors on every level, true = FP64
  // vectors and sums over the FP32 operator blocks of every level
  bool ops32 = false;
  // set around a preconditioner call inside CG: the finest level's last
  // sweep also forms the r.z partials (dot_v = r); dot_parts receives their
  // count per right-hand side (0: not formed)
  const double* dot_v = nullptr;
  int dot_parts = 0;
  int tail_start[2] = {-1, -1};  // first level of the coarse tail per precision (-1: none)
  TailArgs tail_args[2];
  // persistent coarse cycle (HDG_VARIANT_GRID_TAIL): first level per
  // precision (-1: none), its launch arguments and grid, and the barrier words
  int gtail_start[2] = {-1, -1};
  GTailArgs gtail_args[2];
  int gtail_grid_n[2] = {0, 0};
  unsigned* gtail_sync = nullptr;
  hipGraphExec_t gx[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int gnrhs = 1;                 // right-hand sides the captured graphs iterate
  hipGraph_t grp_graph = nullptr; // CHECK_EVERY CG iterations (one batch graph child), for gnrhs
  int cap = 1;                   // right-hand sides the build's buffers hold
  RefElement ref;
  RefDevice rd;
  long nelem = 0;
  int nv = 0, ne = 0, nl = 0, nq = 0;
  // W: load map (b^e = W^T b); Kinv / Minv: HDG recovery factors; for the
  // IPDG schemes Kinv holds L^-1 and Xr the recovery block L^-1 R
  double *kqp = nullptr, *Ae = nullptr, *W = nullptr, *Kinv = nullptr, *Minv = nullptr, *ework = nullptr;
  double* Xr = nullptr;
  double *Xq = nullptr, *Yq = nullptr;  // RT-H flux recovery at the nodes: Xq Lambda + Yq b
  int* bad = nullptr;
  int* hbad = nullptr;
  bool store_recovery = false;
  bool built = false;
  hdg_mg_opts opts{};
  std::vector<Level> L;
  long N = 0;  // trace DOFs of the finest level
  double *g = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *zold = nullptr, *lam = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
  double *ustar = nullptr, *qstar = nullptr;
  Scratch s;
  double* hpin = nullptr;
  // GMRES
  double *V = nullptr, *Z = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *gsv = nullptr, *y = nullptr;
  int gm_m = 0;
  // inspection timing of finest-level trace kernels
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  static constexpr int NPROF_F32OPS = 2 * (APPLY_SWEEP_DOT + 1);  // first class of the FP64-vector form
  // transfer kernels of the fused 2D path: hpre, hsum, hpost on the first
  // h-transition level and the p-prolongation on the finest level, FP64/FP32
  static constexpr int NPROF_XFER = 3 * (APPLY_SWEEP_DOT + 1);
  static constexpr int NPROF = NPROF_XFER + 8;
  double prof_ms[NPROF] = {};
  long long prof_n[NPROF] = {};
  // unstructured triangle meshes (hdg_setup_unstructured): host topology,
  // device copies of every level's index arrays, vertices and triangles
  bool unstructured = false;
  std::unique_ptr<UHost> uh;
  std::vector<ULevel> ul;
  double* uxy = nullptr;
  int* utri = nullptr;
  int* utbnd = nullptr;   // boundary edge of every triangle slot (-1: interior)
  double* urec = nullptr; // recovery maps [ntri][3][nv][3ne + nv]
  std::vector<void*> allocs;        // freed in destroy
  std::vector<void*> build_allocs;  // freed on rebuild
  long long bytes = 0;
};

namespace {

template <typename T>
T* dalloc(hdg_problem* P, long count, bool build) {
  if (count <= 0) count = 1;
  void* ptr = nullptr;
  HDG_CHECK(hipMalloc(&ptr, sizeof(T) * (size_t)count));
  (build ? P->build_allocs : P->allocs).push_back(ptr);
  P->bytes += (long long)sizeof(T) * count;
  return (T*)ptr;
}

template <typename T>
T* upload(hdg_problem* P, const std::vector<T>& v) {
  T* d = dalloc<T>(P, (long)v.size(), false);
  HDG_CHECK(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return d;
}

long ipow(long b, int e) {
  long r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

void init_level(Level& L, int d, int n, int ne) {
  L.d = d;
  L.n = n;
  L.ne = ne;
  L.nl = 2 * d * ne;
  L.nelem = ipow(n, d);
  L.nfd = n >= 1 ? (long)(n - 1) * ipow(n, d - 1) : 0;
  L.nface = d * L.nfd;
  L.nlam = L.nface * ne;
}

hdg_status map_error(const HipError& e) {
  (void)e;
  return HDG_ERR_DEVICE;
}

// a request the handle's discretization does not support
struct Unsupported {};

#define HDG_GUARD_BEGIN try {
#define HDG_GUARD_END                        \
  }                                          \
  catch (const HipError& e) {                \
    return map_error(e);                     \
  }                                          \
  catch (const Unsupported&) {               \
    return HDG_ERR_UNSUPPORTED;              \
  }                                          \
  catch (const std::bad_alloc&) {            \
    return HDG_ERR_DEVICE;                   \
  }

bool check_kappa(hdg_problem* P, const double* kappa, int kind) {
  HDG_CHECK(hipMemsetAsync(P->bad, 0, sizeof(int), P->st));
  launch_kappa_expand(P->nelem, P->nq, kappa, kind, P->kqp, P->bad, P->st);
  HDG_CHECK(hipMemcpyAsync(P->hbad, P->bad, sizeof(int), hipMemcpyDeviceToHost, P->st));
  HDG_CHECK(hipStreamSynchronize(P->st));
  return *P->hbad == 0;
}

constexpr int SCHEME_MULTI = 64;  // internal: one scheme per element (hdg_setup_multi)

double sf_of(int code) { return code == HDG_SCHEME_SIPG ? 1.0 : code == HDG_SCHEME_IIPG ? 0.0 : -1.0; }

void form_scheme(hdg_problem* P, const int* mask, int code) {
  if (code == HDG_SCHEME_HDG)
    launch_element_dtn(P->d, P->k, P->nelem, P->tau, P->tau_kappa, P->rd, P->kqp, P->Ae, P->W, P->Kinv, P->Minv, P->st);
  else if (code == HDG_SCHEME_RT)
    launch_rt_dtn(P->k, P->nelem, mask, code, P->rd, P->kqp, P->Ae, P->W, P->Xr, P->Kinv, P->Xq, P->Yq, P->st);
  else
    launch_ipdg_dtn(P->d, P->k, P->nelem, mask, code, P->tau, P->tau_kappa, sf_of(code), P->rd, P->kqp, P->nq, P->Ae,
                    P->W, P->Xr, P->Kinv, P->st);
}

void form_elements(hdg_problem* P) {
  if (P->scheme == SCHEME_MULTI)
    for (int c : P->codes) form_scheme(P, P->emask, c);
  else
    form_scheme(P, nullptr, P->scheme);
}

void drop_graphs(hdg_problem* P) {
  for (auto& g : P->gx)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  if (P->grp_graph) {
    (void)hipGraphDestroy(P->grp_graph);
    P->grp_graph = nullptr;
  }
}

void free_build(hdg_problem* P) {
  HDG_CHECK(hipStreamSynchronize(P->st));
  drop_graphs(P);
  for (void* ptr : P->build_allocs) HDG_CHECK(hipFree(ptr));
  P->build_allocs.clear();
  P->L.clear();
  P->built = false;
  P->V = P->Z = P->H = P->cs = P->sn = P->gsv = P->y = nullptr;
  P->s.sc = P->s.partials = P->s.pcg = nullptr;
  P->gm_m = 0;
  P->cap = 1;
  P->gtail_sync = nullptr;
  P->gtail_start[0] = P->gtail_start[1] = -1;
}

hipEvent_t take_event(hdg_problem* P) {
  if (!P->ev_pool.empty()) {
    hipEvent_t e = P->ev_pool.back();
    P->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HDG_CHECK(hipEventCreate(&e));
  return e;
}

// Sum the durations of completed event pairs (called right after a stream
// synchronisation, so every recorded pair is complete).
void harvest(hdg_problem* P) {
  for (auto& pd : P->pending) {
    float ms = 0.f;
    HDG_CHECK(hipEventElapsedTime(&ms, pd.a, pd.b));
    P->prof_ms[pd.cls] += ms;
    P->prof_n[pd.cls] += 1;
    P->ev_pool.push_back(pd.a);
    P->ev_pool.push_back(pd.b);
  }
  P->pending.clear();
}

// profiling class of a finest-level launch of mode `mode` with vectors T
// over operator blocks M
template <typename T, typename M>
int prof_class(int mode) {
  if constexpr (!std::is_same_v<T, M>) return hdg_problem::NPROF_F32OPS + mode;
  return 2 * mode + (sizeof(T) == 8 ? 0 : 1);
}

// run `launch` between two events of class `cls` when `timed`
template <class F>
void timed_launch(hdg_problem* P, bool timed, int cls, F&& launch) {
  hdg_problem::Pending pd{cls, nullptr, nullptr};
  if (timed) {
    pd.a = take_event(P);
    pd.b = take_event(P);
    HDG_CHECK(hipEventRecord(pd.a, P->st));
  }
  launch();
  if (timed) {
    HDG_CHECK(hipEventRecord(pd.b, P->st));
    P->pending.push_back(pd);
  }
}

// first h-transition level (its transfer kernels are the profiled ones)
int first_h(const hdg_problem* P) {
  for (size_t i = 0; i < P->L.size(); ++i)
    if (P->L[i].kind == 1) return (int)i;
  return -1;
}

// trace apply on level i; finest-level launches are timed when profiling
template <typename T, typename M = T>
void apply(hdg_problem* P, int i, int mode, const T* x, const T* b, T* y, T* rc, int nr = 1) {
  const bool timed = P->prof_on && i == 0 && nr == 1;
  hdg_problem::Pending pd{prof_class<T, M>(mode), nullptr, nullptr};
  if (timed) {
    pd.a = take_event(P);
    pd.b = take_event(P);
    HDG_CHECK(hipEventRecord(pd.a, P->st));
  }
  launch_apply<T, M>(P->L[i], mode, x, b, y, P->rd.Jp, rc, P->st, nr);
  if (timed) {
    HDG_CHECK(hipEventRecord(pd.b, P->st));
    P->pending.push_back(pd);
  }
}

// Run `body` (device work only, fixed pointers) as a captured hipGraph on the
// caller's stream; captured once per slot on the private stream.  Eager when
// graphs are disabled or finest-level kernels are being timed.
// Capture `body` (device work only, fixed pointers) into a graph on the
// handle's private capture stream; the caller owns the returned graph.
template <class F>
hipGraph_t capture(hdg_problem* P, F&& body) {
  hipStream_t user = P->st;
  P->st = P->cap_st;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(P->cap_st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    P->st = user;
    throw HipError{e, "hipStreamBeginCapture"};
  }
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(P->cap_st, &g);
    if (g) (void)hipGraphDestroy(g);
    P->st = user;
    throw;
  }
  e = hipStreamEndCapture(P->cap_st, &g);
  P->st = user;
  if (e != hipSuccess) throw HipError{e, "hipStreamEndCapture"};
  return g;
}

template <class F>
void run_graph(hdg_problem* P, int slot, F&& body, int nr = 1) {
  if (!P->use_graphs || P->prof_on) {
    body();
    return;
  }
  if (nr != P->gnrhs) {  // graphs are captured for one right-hand-side count
    drop_graphs(P);
    P->gnrhs = nr;
  }
  if (!P->gx[slot]) {
    hipGraph_t g = capture(P, body);
    hipError_t e = hipGraphInstantiate(&P->gx[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      P->gx[slot] = nullptr;
      throw HipError{e, "hipGraphInstantiate"};
    }
  }
  HDG_CHECK(hipGraphLaunch(P->gx[slot], P->st));
}

enum { G_PCG64 = 0, G_PCGMX = 1, G_MG64 = 2, G_MGMX = 3, G_PRE64 = 4, G_PREMX = 5 };

// -------------------------------------------------------------------------
// Algorithm 1 on level i; returns the device pointer holding e = B_i r.
// If `out` is given the result is written there.  `pre_done`: the caller
// already applied the first block-Jacobi step (e = D^-1 r into L.e).
//
// In 2D with at least one sweep the transitions use fused kernels: the
// finest residual's P1 restriction also takes the P1 level's first Jacobi
// step; an h-transition is one macro-element pass (interior residual, local
// correction of step 3, its share of the restricted residual), one
// coarse-face pass (restricted residual + coarse first Jacobi step, or the
// coarsest direct solve), and one out-of-place pass (prolongation + local
// correction of step 5).  Same arithmetic as the unfused kernels up to the
// order of the last rounding.
//
// Chebyshev smoother: step s reads the level's diagonal blocks scaled by the
// reciprocal of root s (the launchers read L.Dinv at launch)
void cheb_select(Level& L, int s) {
  if (L.cheb64.empty()) return;
  L.Dinv64 = L.cheb64[s];
  L.Dinv32 = L.cheb32[s];
}

// m steps of multicolour point symmetric Gauss-Seidel on A e = r in place:
// the colours forward with each face's values in increasing order, then
// backward with them decreasing
template <typename T, typename M>
void sgs_steps(Level& L, T* e, const T* r, int m, hipStream_t st, int nr) {
  const int nc = 2 * L.d;
  for (int s = 0; s < m; ++s) {
    for (int c = 0; c < nc; ++c) launch_sgs_color<T, M>(L, c, 0, e, r, st, nr);
    for (int c = nc - 1; c >= 0; --c) launch_sgs_color<T, M>(L, c, 1, e, r, st, nr);
  }
}

// M: storage type of the operator blocks read.  M = float under T = double is
// the 3D mixed cycle: every level keeps FP64 vectors and sums and reads the
// FP32 copies of its blocks (unfused kernels, no coarse tail).  The point
// smoothers (HDG_SMOOTHER_*) replace the block-Jacobi steps; they run on the
// unfused path.
template <typename T, typename M = T>
T* vcycle(hdg_problem* P, int i, const T* r, T* out, bool pre_done = false, int nr = 1) {
  constexpr bool narrow = !std::is_same_v<T, M>;
  Level& L = P->L[i];
  const int pr = sizeof(T) == 8 ? 0 : 1;
  hipStream_t st = P->st;
  T* e = (T*)L.e[pr];
  T* w = (T*)L.w[pr];
  if (!narrow && i == P->gtail_start[pr] && pre_done && !out && nr == 1 && r == (const T*)L.r[pr]) {
    launch_gtail<T>(P->gtail_args[pr], P->gtail_grid_n[pr], st);
    return e;
  }
  if (!narrow && i == P->tail_start[pr]) {
    TailArgs a = P->tail_args[pr];
    a.rin = r;
    a.ein = e;
    a.pre_done = pre_done ? 1 : 0;
    a.eout = out ? out : e;
    launch_tail<T>(a, st, nr);
    return (T*)a.eout;
  }
  if (L.kind == 2) {
    T* dst = out ? out : e;
    launch_coarse_solve<T, M>(L, r, dst, st, nr);
    return dst;
  }
  const int m = L.sweeps;
  const int lc = P->opts.local_corr;
  const bool fused = !narrow && P->fuse && L.d == 2 && m >= 1;
  const bool gs = P->opts.smoother == HDG_SMOOTHER_LUSGS;
  // pre-smoothing from e = 0
  if (gs) {
    blas_fill<T>(e, T(0), L.nlam, st, nr);
    sgs_steps<T, M>(L, e, r, m, st, nr);
  } else {
    if (!pre_done) {
      cheb_select(L, 0);
      if (m >= 1)
        launch_jacobi0<T, M>(L, r, e, st, nr);
      else
        blas_fill<T>(e, T(0), L.nlam, st, nr);
    }
    for (int s = 1; s < m; ++s) {
      cheb_select(L, s);
      apply<T, M>(P, i, APPLY_SWEEP, e, r, w, nullptr, nr);
      std::swap(e, w);
    }
  }
  Level& C = P->L[i + 1];
  T* rc = (T*)C.r[pr];
  if (L.kind == 0) {
    const T* ec;
    if (fused && C.kind != 2) {
      const bool timed = P->prof_on && i == 0 && nr == 1;
      hdg_problem::Pending pd{2 * APPLY_RES_PRESTRICT + pr, nullptr, nullptr};
      if (timed) {
        pd.a = take_event(P);
        pd.b = take_event(P);
        HDG_CHECK(hipEventRecord(pd.a, st));
      }
      launch_res_prestrict<T>(L, C, e, r, rc, (T*)C.e[pr], P->rd.Jp, st, nr);
      if (timed) {
        HDG_CHECK(hipEventRecord(pd.b, st));
        P->pending.push_back(pd);
      }
      ec = vcycle<T>(P, i + 1, rc, nullptr, true, nr);
    } else {
      apply<T, M>(P, i, APPLY_RES_PRESTRICT, e, r, nullptr, rc, nr);
      ec = vcycle<T, M>(P, i + 1, rc, nullptr, false, nr);
    }
    const bool tp = P->prof_on && nr == 1 && i == 0;
    timed_launch(P, tp, hdg_problem::NPROF_XFER + 6 + pr,
                 [&] { launch_prolong_p<T>(L, 1 << (L.d - 1), P->rd.Jp, ec, e, st, nr); });
  } else if (fused) {
    T* cb = (T*)L.cb[pr];
    const bool tx = P->prof_on && nr == 1 && i == first_h(P);
    timed_launch(P, tx, hdg_problem::NPROF_XFER + pr,
                 [&] { launch_hpre<T>(L, r, e, (lc & HDG_LC_PRE) ? 1 : 0, cb, st, nr); });
    const T* ec;
    if (C.kind == 2) {
      timed_launch(P, tx, hdg_problem::NPROF_XFER + 2 + pr,
                   [&] { launch_hsum<T>(L, C, r, cb, nullptr, (T*)C.e[pr], st, nr); });
      ec = (const T*)C.e[pr];
    } else {
      timed_launch(P, tx, hdg_problem::NPROF_XFER + 2 + pr,
                   [&] { launch_hsum<T>(L, C, r, cb, rc, (T*)C.e[pr], st, nr); });
      ec = vcycle<T>(P, i + 1, rc, nullptr, true, nr);
    }
    timed_launch(P, tx, hdg_problem::NPROF_XFER + 4 + pr,
                 [&] { launch_hpost<T>(L, C, r, ec, e, w, (lc & HDG_LC_POST) ? 1 : 0, st, nr); });
    std::swap(e, w);
  } else {
    apply<T, M>(P, i, APPLY_RES, e, r, w, nullptr, nr);
    launch_hcorr<T, M>(L, w, e, (lc & HDG_LC_PRE) ? 1 : 0, 1, (T*)L.cb[pr], st, nr);
    launch_hrestrict<T>(L, C, w, (T*)L.cb[pr], rc, st, nr);
    const T* ec = vcycle<T, M>(P, i + 1, rc, nullptr, false, nr);
    launch_hprolong<T, M>(L, C, ec, e, st, nr);
    if (lc & HDG_LC_POST) {
      apply<T, M>(P, i, APPLY_RES, e, r, w, nullptr, nr);
      launch_hcorr<T, M>(L, w, e, 1, 0, nullptr, st, nr);
    }
  }
  if (gs) sgs_steps<T, M>(L, e, r, m, st, nr);
  for (int s = 0; s < m && !gs; ++s) {
    cheb_select(L, s);
    T* dst = (out && s == m - 1) ? out : w;
    if (i == 0 && P->dot_v && dst == out) {
      int np = 0;
      const bool timed = P->prof_on && nr == 1;
      hdg_problem::Pending pd{prof_class<T, M>(APPLY_SWEEP_DOT), nullptr, nullptr};
      if (timed) {
        pd.a = take_event(P);
        pd.b = take_event(P);
        HDG_CHECK(hipEventRecord(pd.a, st));
      }
      launch_apply_red<T, M>(L, APPLY_SWEEP_DOT, e, r, dst, P->dot_v, nullptr, nullptr, &P->s, st, nr, &np);
      if (timed) {
        HDG_CHECK(hipEventRecord(pd.b, st));
        P->pending.push_back(pd);
      }
      P->dot_parts = np;
    } else {
      apply<T, M>(P, i, APPLY_SWEEP, e, r, dst, nullptr, nr);
    }
    if (dst == w)
      std::swap(e, w);
    else
      e = dst;
  }
  if (out && e != out) {
    blas_copy_t<T>(out, e, L.nlam, st, nr);
    e = out;
  }
  return e;
}

// z = B r in FP64 or with an FP32 V-cycle (mixed precision)
void precond(hdg_problem* P, const double* r, double* z, bool mixed) {
  if (!mixed) {
    vcycle<double>(P, 0, r, z);
    return;
  }
  if (P->ops32) {
    vcycle<double, float>(P, 0, r, z);
    return;
  }
  Level& L0 = P->L[0];
  float* r32 = (float*)L0.r[1];
  blas_d2f(r, r32, P->N, P->st);
  float* e32 = vcycle<float>(P, 0, r32, nullptr);
  blas_f2d(e32, z, P->N, P->st);
}

// the scalar blocks of the first nr right-hand sides, on the host
const double* read_scalars(hdg_problem* P, int nr) {
  HDG_CHECK(hipMemcpyAsync(P->hpin, P->s.sc, sizeof(double) * SC_COUNT * nr, hipMemcpyDeviceToHost, P->st));
  HDG_CHECK(hipStreamSynchronize(P->st));
  if (!P->pending.empty()) harvest(P);
  return P->hpin;
}

double read_scalar(hdg_problem* P, const double* dptr) {
  HDG_CHECK(hipMemcpyAsync(P->hpin, dptr, sizeof(double), hipMemcpyDeviceToHost, P->st));
  HDG_CHECK(hipStreamSynchronize(P->st));
  if (!P->pending.empty()) harvest(P);
  return P->hpin[0];
}

void residual(hdg_problem* P, const double* lam, const double* g, double* r) {
  apply<double>(P, 0, APPLY_RES, lam, g, r, nullptr);
}

// outer iterations launched between two reads of the residual history
constexpr int CHECK_EVERY = 4;

struct SolveOut {
  int iters = 0;
  int outer = 0;  // true residuals formed
  double relres = 0.0;
  hdg_status status = HDG_OK;
};

// r = g - A lam and ||r||^2 in one pass (plus the FP32 copy of r when mixed),
// for nr right-hand sides
void residual_norm(hdg_problem* P, const double* lam, const double* g, bool mixed, int nr) {
  float* r32 = mixed ? P->r32 : nullptr;
  const bool timed = P->prof_on && nr == 1;
  hdg_problem::Pending pd{2 * APPLY_RES + 0, nullptr, nullptr};
  if (timed) {
    pd.a = take_event(P);
    pd.b = take_event(P);
    HDG_CHECK(hipEventRecord(pd.a, P->st));
  }
  launch_apply_red<double>(P->L[0], APPLY_RES_NORM, lam, g, P->r, nullptr, nullptr, r32, &P->s, P->st, nr);
  if (timed) {
    HDG_CHECK(hipEventRecord(pd.b, P->st));
    P->pending.push_back(pd);
  }
}

// z = B r: FP64 V-cycle on r, or FP32 V-cycle on the FP32 copy r32 into
// z32, or (mixed, 3D) the cycle over FP32 operator blocks on r into z
void precond_fused(hdg_problem* P, bool mixed, int nr) {
  if (mixed && P->ops32)
    vcycle<double, float>(P, 0, P->r, P->z, false, nr);
  else if (mixed)
    vcycle<float>(P, 0, P->r32, P->z32, false, nr);
  else
    vcycle<double>(P, 0, P->r, P->z, false, nr);
}

// Convergence bookkeeping of nr right-hand sides iterated together: the
// residual history of each since the last reset of the count, its first
// converged iteration, and the worst residual of the returned iterates.
// For a refinement step of mixed PCG it also tracks each right-hand side's
// inner target (a reduction of the step's true residual) and stagnation: no
// halving of its best residual within STAG_WINDOW iterations.
constexpr int STAG_WINDOW = 100;
// Chebyshev smoother: power-iteration steps, safety factor of the largest
// eigenvalue estimate, and ratio largest / smallest of the interval
constexpr int CHEB_POWER_ITS = 20;
constexpr double CHEB_SAFETY = 1.1;
constexpr double CHEB_RATIO = 30.0;
struct Tracker {
  int nr = 1;
  double tol = 0.0;
  const double* gn = nullptr;
  int first[64];
  bool bad = false;
  double tgt[64], best[64], mark[64];
  int t_mark[64];
  bool reached[64];
  void init(int n, double t, const double* g) {
    nr = n;
    tol = t;
    gn = g;
    for (int r = 0; r < nr; ++r) {
      first[r] = -1;
      tgt[r] = 0.0;
      best[r] = mark[r] = std::numeric_limits<double>::infinity();
      t_mark[r] = 0;
      reached[r] = false;
    }
  }
  // inner targets of one refinement step that starts at iteration `base`
  // from true residual norms r0[]: reduction `red` (0: none)
  void init_inner(double red, const double* r0, int base) {
    for (int r = 0; r < nr; ++r) {
      tgt[r] = red * r0[r];
      best[r] = mark[r] = r0[r];
      t_mark[r] = base;
    }
  }
  // scan a group of `cnt` iterations that started at iteration `base`
  bool scan(const double* sc, int base, int cnt, double* worst_last) {
    bool all = true;
    double w = 0.0;
    for (int r = 0; r < nr; ++r) {
      const double* h = sc + (long)r * SC_COUNT + SC_HIST;
      for (int it = 0; it < cnt; ++it) {
        const double a = std::sqrt(h[it]);
        const double rel = a / gn[r];
        if (!std::isfinite(rel)) bad = true;
        if (first[r] < 0 && rel <= tol) first[r] = base + it + 1;
        if (a <= tgt[r]) reached[r] = true;
        if (a < best[r]) best[r] = a;
        if (best[r] <= 0.5 * mark[r]) {
          mark[r] = best[r];
          t_mark[r] = base + it + 1;
        }
      }
      const double last = std::sqrt(h[cnt - 1]) / gn[r];
      if (!std::isfinite(last)) bad = true;
      w = std::max(w, last);
      if (first[r] < 0) all = false;
    }
    *worst_last = w;
    return all;
  }
  // every right-hand side has converged, met its inner target, or stagnated
  // (at iteration `now`)
  bool inner_done(int now) const {
    for (int r = 0; r < nr; ++r)
      if (first[r] < 0 && !reached[r] && now - t_mark[r] < STAG_WINDOW) return false;
    return true;
  }
  int iters() const {
    int m = 0;
    for (int r = 0; r < nr; ++r) m = std::max(m, first[r]);
    return m;
  }
};

double worst_rnorm(const double* sc, int nr, const double* gn) {
  double w = 0.0;
  for (int r = 0; r < nr; ++r) {
    const double rel = std::sqrt(sc[(long)r * SC_COUNT + SC_RNORM2]) / gn[r];
    if (!std::isfinite(rel)) return rel;
    w = std::max(w, rel);
  }
  return w;
}

SolveOut solve_mg(hdg_problem* P, const double* g, double* lam, double tol, const double* gn, bool mixed, int nr) {
  SolveOut o;
  const long N = P->N;
  const bool v32 = mixed && !P->ops32;  // the cycle takes and returns FP32 vectors
  residual_norm(P, lam, g, v32, nr);
  double rel = worst_rnorm(read_scalars(P, nr), nr, gn);
  o.outer = 1;
  Tracker tr;
  tr.init(nr, tol, gn);
  int launched = 0;
  bool all = rel <= tol;
  while (!all && launched < P->opts.max_it && std::isfinite(rel)) {
    const int grp = std::min(CHECK_EVERY, P->opts.max_it - launched);
    for (int r = 0; r < nr; ++r) blas_fill<double>(P->s.sc + (long)r * SC_COUNT + SC_HCNT, 0.0, 1, P->st);
    for (int it = 0; it < grp; ++it)
      run_graph(
          P, mixed ? G_MGMX : G_MG64,
          [&] {
            precond_fused(P, mixed, nr);
            if (v32)
              blas_add<float>(lam, P->z32, N, P->st, nr);
            else
              blas_add<double>(lam, P->z, N, P->st, nr);
            residual_norm(P, lam, g, v32, nr);
          },
          nr);
    all = tr.scan(read_scalars(P, nr), launched, grp, &rel);
    launched += grp;
    if (tr.bad) rel = std::numeric_limits<double>::quiet_NaN();
  }
  o.iters = all ? tr.iters() : launched;
  o.relres = rel;
  o.status = !std::isfinite(rel) ? HDG_ERR_BREAKDOWN : (rel <= tol ? HDG_OK : HDG_ERR_NOT_CONVERGED);
  return o;
}

// First direction of a CG run from the current residual: z = B r, r.z, p = z.
void pcg_start(hdg_problem* P, bool mixed, int nr) {
  const long N = P->N;
  const bool v32 = mixed && !P->ops32;
  precond_fused(P, mixed, nr);
  if (v32) {
    blas_rz<float>(P->r, P->z32, N, FIN_RZ0, P->s, P->st, nr);
    blas_f2d(P->z32, P->p, N, P->st, nr);
  } else {
    blas_rz<double>(P->r, P->z, N, FIN_RZ0, P->s, P->st, nr);
    blas_copy(P->p, P->z, N, P->st, nr);
  }
}

// One CG iteration, device work only (captured into graphs): lambda and r
// are updated first, so after convergence the trailing preconditioner
// application and direction update change nothing that is returned.
void pcg_iteration(hdg_problem* P, double* lam, bool mixed, int nr) {
  const long N = P->N;
  const bool v32 = mixed && !P->ops32;
  hipStream_t s2 = P->st;
  const bool timed = P->prof_on && nr == 1;
  hdg_problem::Pending pd{2 * APPLY_Y + 0, nullptr, nullptr};
  if (timed) {
    pd.a = take_event(P);
    pd.b = take_event(P);
    HDG_CHECK(hipEventRecord(pd.a, s2));
  }
  int npap = 0;
  launch_apply_red<double>(P->L[0], APPLY_Y_DOT, P->p, nullptr, P->Ap, nullptr, nullptr, nullptr, &P->s, s2, nr,
                           &npap);
  if (timed) {
    HDG_CHECK(hipEventRecord(pd.b, s2));
    P->pending.push_back(pd);
  }
  if (v32)
    blas_cg_update2_fused<float>(lam, P->r, P->r32, P->p, P->Ap, P->z32, N, npap, P->s, s2, nr);
  else
    blas_cg_update2_fused<double>(lam, P->r, nullptr, P->p, P->Ap, P->z, N, npap, P->s, s2, nr);
  // the V-cycle's last finest-level sweep also forms the r.z partials
  P->dot_v = P->r;
  P->dot_parts = 0;
  precond_fused(P, mixed, nr);
  P->dot_v = nullptr;
  if (P->dot_parts > 0)
    blas_finalize_cg(N, P->dot_parts, mixed, P->s, s2, nr);
  else if (v32)
    blas_rz_cg<float>(P->r, P->z32, N, true, P->s, s2, nr);
  else
    blas_rz_cg<double>(P->r, P->z, N, mixed, P->s, s2, nr);
  if (v32)
    blas_cg_dir<float>(P->p, P->z32, N, P->s, s2, nr);
  else
    blas_cg_dir<double>(P->p, P->z, N, P->s, s2, nr);
}

// reset the residual-history counters of nr right-hand sides
void reset_history(hdg_problem* P, int nr) {
  for (int r = 0; r < nr; ++r) blas_fill<double>(P->s.sc + (long)r * SC_COUNT + SC_HCNT, 0.0, 1, P->st);
}

// Preconditioned CG.  FP64: Fletcher-Reeves beta, one run to the tolerance
// (then confirmed on the true residual).  Mixed: FP64 iterative refinement
// around an FP32-preconditioned CG.  Each refinement step forms the true
// residual r = g - A lambda in FP64, then runs CG on A delta = r with the
// FP32 V-cycle as preconditioner, accumulating delta into lambda in FP64
// (lambda += alpha p is lambda + delta), until every right-hand side has met
// the tolerance, reduced its residual by refine_red against the step's true
// residual, or stagnated; then the next step restarts from the new true
// residual.  The inner CG takes the flexible Polak-Ribiere beta =
// (r.z - r.z_old) / rz_old, since the FP32 cycle is not exactly the same
// linear map at every application; r.z_old is accumulated in the update pass
// while z still holds z_old.  nr right-hand sides iterate together, each
// with its own scalars; the solve ends when every one has met the tolerance.
SolveOut solve_pcg(hdg_problem* P, const double* g, double* lam, double tol, const double* gn, bool mixed, int nr) {
  SolveOut o;
  const double red = mixed ? P->opts.refine_red : 0.0;
  const bool v32 = mixed && !P->ops32;  // the cycle takes and returns FP32 vectors
  Tracker tr;
  tr.init(nr, tol, gn);
  int launched = 0;
  for (;;) {
    residual_norm(P, lam, g, v32, nr);
    const double* sc0 = read_scalars(P, nr);
    double rel = worst_rnorm(sc0, nr, gn);
    double r0[64];
    for (int r = 0; r < nr; ++r) r0[r] = std::sqrt(sc0[(long)r * SC_COUNT + SC_RNORM2]);
    o.relres = rel;
    o.outer += 1;
    if (!std::isfinite(rel)) {
      o.status = HDG_ERR_BREAKDOWN;
      return o;
    }
    if (rel <= tol || launched >= P->opts.max_it) break;
    pcg_start(P, mixed, nr);
    // one CG iteration per graph launch; launches go out in groups of up to
    // CHECK_EVERY with one read of the residual histories per group;
    // iterations past the first converged one only refine lambda.
    tr.init(nr, tol, gn);
    if (mixed) tr.init_inner(red, r0, launched);
    bool all = false, done = false;
    while (!done && launched < P->opts.max_it) {
      const int grp = std::min(CHECK_EVERY, P->opts.max_it - launched);
      reset_history(P, nr);
      for (int it = 0; it < grp; ++it)
        run_graph(P, mixed ? G_PCGMX : G_PCG64, [&] { pcg_iteration(P, lam, mixed, nr); }, nr);
      all = tr.scan(read_scalars(P, nr), launched, grp, &rel);
      launched += grp;
      if (tr.bad) {
        o.relres = std::numeric_limits<double>::quiet_NaN();
        o.status = HDG_ERR_BREAKDOWN;
        o.iters = launched;
        return o;
      }
      done = all || (mixed && tr.inner_done(launched));
    }
    o.iters = all ? std::max(o.iters, tr.iters()) : launched;
    // next refinement step, or confirmation of convergence, from the true
    // residual of the current iterate
  }
  o.status = o.relres <= tol ? HDG_OK : HDG_ERR_NOT_CONVERGED;
  return o;
}

SolveOut solve_gmres(hdg_problem* P, const double* g, double* lam, double tol, double gn, bool mixed) {
  SolveOut o;
  const long N = P->N;
  hipStream_t st = P->st;
  double* sc = P->s.sc;
  const int m = P->gm_m;
  const long ld = N;
  for (;;) {
    residual(P, lam, g, P->r);
    blas_dot(P->r, P->r, N, P->s, FIN_NORM_INV, sc + SC_HNORM, st);
    double beta = read_scalar(P, sc + SC_HNORM);
    o.relres = beta / gn;
    o.outer += 1;
    if (!std::isfinite(beta)) {
      o.status = HDG_ERR_BREAKDOWN;
      return o;
    }
    if (o.relres <= tol || o.iters >= P->opts.max_it) break;
    blas_scale(P->V, P->r, N, sc + SC_TMP, st);
    blas_fill<double>(P->gsv, 0.0, m + 1, st);
    HDG_CHECK(hipMemcpyAsync(P->gsv, sc + SC_HNORM, sizeof(double), hipMemcpyDeviceToDevice, st));
    int j = 0;
    while (j < m && o.iters < P->opts.max_it) {
      double* vj = P->V + j * ld;
      double* zj = P->Z + j * ld;
      double* w = P->V + (j + 1) * ld;
      blas_copy(P->r, vj, N, st);
      run_graph(P, mixed ? G_PREMX : G_PRE64, [&] { precond(P, P->r, P->z, mixed); });
      blas_copy(zj, P->z, N, st);
      apply<double>(P, 0, APPLY_Y, zj, nullptr, w, nullptr);
      double* hcol = P->H + (long)j * (m + 1);
      for (int i = 0; i <= j; ++i) {
        blas_dot(w, P->V + i * ld, N, P->s, FIN_STORE, hcol + i, st);
        blas_axpy(w, P->V + i * ld, N, hcol + i, -1.0, st);
      }
      blas_dot(w, w, N, P->s, FIN_NORM_INV, hcol + j + 1, st);
      blas_scale(w, w, N, sc + SC_TMP, st);
      blas_gmres_rot(P->H, P->cs, P->sn, P->gsv, j, m + 1, sc, st);
      ++j;
      ++o.iters;
      double res = read_scalar(P, sc + SC_GRES);
      if (!std::isfinite(res)) {
        o.status = HDG_ERR_BREAKDOWN;
        return o;
      }
      if (res / gn <= tol) break;
    }
    blas_gmres_backsolve(P->H, P->gsv, j, m + 1, P->y, st);
    blas_gmres_combine(lam, P->Z, ld, j, P->y, N, st);
  }
  o.status = o.relres <= tol ? HDG_OK : HDG_ERR_NOT_CONVERGED;
  return o;
}

// g from a volume source: element loads b^e staged in ebuf (N_T (n_v + n_l)
// doubles), then pulled per face with the Dirichlet lift
void form_rhs_in(hdg_problem* P, const double* rhs, int kind, const double* gdir, double* g, double* ebuf) {
  launch_element_load(P->d, P->k, P->nelem, P->rd, rhs, kind == HDG_RHS_F_LOAD ? 1 : 0, P->W, ebuf, P->st);
  launch_load_pull(P->d, P->k, P->n, ebuf, P->Ae, gdir, g, P->st);
}

void form_rhs(hdg_problem* P, const double* rhs, int kind, const double* gdir, double* g) {
  if (P->unstructured) {  // nodal f; Dirichlet data per boundary edge
    if (kind != HDG_RHS_F_NODAL) throw Unsupported{};
    launch_tri_load(P->k, P->ul[0], P->W, rhs, P->Ae, P->utbnd, gdir, g, P->st);
    return;
  }
  form_rhs_in(P, rhs, kind, gdir, g, P->ework);
}

// Solve for the nr right-hand sides already in P->g (initial guesses in
// P->lam), all iterated together (MG, PCG) or one after another (GMRES).
// Error flag of the persistent coarse cycle: set when a grid-wide barrier
// wait ran out of polls (its results are then not to be trusted).  The
// barrier words are cleared for the next launch.
hdg_status gtail_check(hdg_problem* P) {
  if (!P->gtail_sync || (P->gtail_start[0] < 0 && P->gtail_start[1] < 0)) return HDG_OK;
  unsigned flag = 0;
  HDG_CHECK(hipMemcpyAsync(&flag, P->gtail_sync + 64, sizeof(unsigned), hipMemcpyDeviceToHost, P->st));
  HDG_CHECK(hipStreamSynchronize(P->st));
  if (flag == 0) return HDG_OK;
  HDG_CHECK(hipMemsetAsync(P->gtail_sync, 0, sizeof(unsigned) * GTAIL_SYNC_WORDS, P->st));
  HDG_CHECK(hipStreamSynchronize(P->st));
  return HDG_ERR_DEVICE;
}

hdg_status solve_many(hdg_problem* P, int nr, double tol, hdg_solve_info* info) {
  const long N = P->N;
  if (N == 0) {
    if (info) info->relres = 0.0;
    return HDG_OK;
  }
  blas_dot(P->g, P->g, N, P->s, FIN_GNORM, nullptr, P->st, nr);
  const double* sc = read_scalars(P, nr);
  double gn[64];
  for (int r = 0; r < nr; ++r) {
    gn[r] = std::sqrt(sc[(long)r * SC_COUNT + SC_GNORM2]);
    if (!std::isfinite(gn[r])) return HDG_ERR_BREAKDOWN;
    if (gn[r] == 0.0) {
      // zero data: the solution is zero
      blas_fill<double>(P->lam + r * N, 0.0, N, P->st);
      gn[r] = 1.0;
    }
  }
  const bool mixed = P->opts.precision == HDG_MIXED;
  SolveOut o;
  switch (P->opts.method) {
    case HDG_METHOD_PCG: o = solve_pcg(P, P->g, P->lam, tol, gn, mixed, nr); break;
    case HDG_METHOD_GMRES: {
      // one right-hand side after another, each in its own rows of g and
      // lambda (the Krylov basis and the preconditioner's vectors are shared)
      hdg_status worst = HDG_OK;
      for (int r = 0; r < nr; ++r) {
        SolveOut q = solve_gmres(P, P->g + r * N, P->lam + r * N, tol, gn[r], mixed);
        o.iters = std::max(o.iters, q.iters);
        o.outer = std::max(o.outer, q.outer);
        o.relres = std::max(o.relres, q.relres);
        if (q.status != HDG_OK && worst == HDG_OK) worst = q.status;
      }
      o.status = worst;
      break;
    }
    default: o = solve_mg(P, P->g, P->lam, tol, gn, mixed, nr); break;
  }
  if (info) {
    info->iters += o.iters;
    info->outer_iters += o.outer;
    info->relres = std::max(info->relres, o.relres);
  }
  const hdg_status gs = gtail_check(P);
  return gs != HDG_OK ? gs : o.status;
}

hdg_status solve_one(hdg_problem* P, const double* g, double* lam, double tol, hdg_solve_info* info) {
  if (P->N == 0) {
    if (info) info->relres = 0.0;
    return HDG_OK;
  }
  // iterate in the handle's own buffers so captured graphs see fixed pointers
  if (g != P->g) blas_copy(P->g, g, P->N, P->st);
  if (lam != P->lam) blas_copy(P->lam, lam, P->N, P->st);
  hdg_status s = solve_many(P, 1, tol, info);
  if (lam != P->lam) blas_copy(lam, P->lam, P->N, P->st);
  return s;
}

}  // namespace

long hdg::rhs_staging_doubles(const hdg_problem* P) { return P->unstructured ? 0 : P->nelem * (P->nv + P->nl); }

bool hdg::rhs_supported(const hdg_problem* P, int kind, const double* gdir) {
  (void)gdir;
  return !P->unstructured || kind == HDG_RHS_F_NODAL;
}

void hdg::rhs_with_staging(hdg_problem* P, const double* rhs, int kind, const double* gdir, double* g,
                           double* ebuf) {
  if (P->unstructured) {  // the per-face load needs no staging
    form_rhs(P, rhs, kind, gdir, g);
    return;
  }
  form_rhs_in(P, rhs, kind, gdir, g, ebuf);
}

// =========================================================================
extern "C" {

void hdg_default_opts(hdg_mg_opts* o) {
  if (!o) return;
  o->sweeps = 2;
  o->growth = 1;
  o->omega = 1.0;
  o->local_corr = HDG_LC_PRE;
  o->precision = HDG_FP64;
  o->method = HDG_METHOD_MG;
  o->max_it = 200;
  o->restart = 0;
  o->coarse_n = 2;
  o->nrhs = 1;
  o->refine_red = 1e-5;
  o->variant = 0;
  o->smoother = HDG_SMOOTHER_BLOCK_JACOBI;
}

const char* hdg_status_string(hdg_status s) {
  switch (s) {
    case HDG_OK: return "ok";
    case HDG_ERR_INVALID_ARG: return "invalid argument";
    case HDG_ERR_UNSUPPORTED: return "unsupported";
    case HDG_ERR_STATE: return "wrong state";
    case HDG_ERR_NOT_CONVERGED: return "not converged";
    case HDG_ERR_BREAKDOWN: return "breakdown";
    case HDG_ERR_DEVICE: return "device error";
  }
  return "unknown";
}

hdg_status hdg_umesh_levels(const hdg_umesh* mesh, int k, long long* sizes, int max_levels, int* nlevels) {
  if (!mesh || !mesh->xy || !mesh->tri || !mesh->seeds || !sizes || !nlevels || max_levels < 1) return HDG_ERR_INVALID_ARG;
  if (mesh->nvert < 3 || mesh->ntri < 1 || mesh->nseeds < 1 || mesh->hlevels < 1 || mesh->hlevels > 16)
    return HDG_ERR_INVALID_ARG;
  if (k < 1 || k > 4) return HDG_ERR_UNSUPPORTED;
  try {
    UHost H;
    H.build_reference(k);
    H.build_mesh(mesh->nvert, mesh->xy, mesh->ntri, mesh->tri, mesh->seeds, mesh->nseeds, mesh->hlevels);
    *nlevels = (int)H.lev.size();
    if ((int)H.lev.size() > max_levels) return HDG_ERR_INVALID_ARG;
    for (size_t i = 0; i < H.lev.size(); ++i) sizes[i] = (long long)H.lev[i].nface * H.lev[i].m;
    return HDG_OK;
  } catch (const std::bad_alloc&) {
    return HDG_ERR_DEVICE;
  } catch (const std::exception&) {
    return HDG_ERR_INVALID_ARG;
  }
}

hdg_status hdg_reference_nodes(int k, double* gll, double* gauss) {
  if (k < 1 || k > 12 || !gll || !gauss) return HDG_ERR_INVALID_ARG;
  std::vector<double> x, gx, gw;
  gll_points(k, x);
  gauss_points(k + 2, gx, gw);
  std::memcpy(gll, x.data(), sizeof(double) * (k + 1));
  std::memcpy(gauss, gx.data(), sizeof(double) * (k + 2));
  return HDG_OK;
}

namespace {

// Setup of any discretization: `scheme` one HDG_SCHEME_* code, or
// SCHEME_MULTI with `codes` the codes present and `mask_host` one code per
// element.
hdg_status setup_impl(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind, int scheme,
                      bool tau_kappa, const std::vector<int>& codes, const std::vector<int>& mask_host,
                      int store_recovery, void* hip_stream, hdg_handle* out) {
  if (!mesh || !out || !kappa) return HDG_ERR_INVALID_ARG;
  if (kappa_kind != HDG_KAPPA_PER_ELEMENT && kappa_kind != HDG_KAPPA_AT_QP) return HDG_ERR_INVALID_ARG;
  if (mesh->dim != 2 && mesh->dim != 3) return HDG_ERR_UNSUPPORTED;
  if (mesh->n < 1 || mesh->n > (mesh->dim == 2 ? 8192 : 512)) return HDG_ERR_INVALID_ARG;
  if (k < 1 || (mesh->dim == 2 && k > 6) || (mesh->dim == 3 && k > 3)) return HDG_ERR_UNSUPPORTED;
  if (!(tau > 0.0) || !std::isfinite(tau)) return HDG_ERR_INVALID_ARG;
  bool has_ipdg = false, has_rt = false, sym = true;
  for (int c : codes) {
    has_ipdg |= c == HDG_SCHEME_SIPG || c == HDG_SCHEME_IIPG || c == HDG_SCHEME_NIPG;
    has_rt |= c == HDG_SCHEME_RT;
    sym &= c == HDG_SCHEME_HDG || c == HDG_SCHEME_SIPG || c == HDG_SCHEME_RT;
  }
  if ((has_ipdg || tau_kappa) && kappa_kind == HDG_KAPPA_AT_QP) return HDG_ERR_UNSUPPORTED;
  if (has_rt && (mesh->dim != 2 || k > 4)) return HDG_ERR_UNSUPPORTED;
  *out = nullptr;
  hdg_problem* P = new (std::nothrow) hdg_problem();
  if (!P) return HDG_ERR_DEVICE;
  HDG_GUARD_BEGIN
  P->d = mesh->dim;
  P->n = mesh->n;
  P->k = k;
  P->tau = tau;
  P->scheme = scheme;
  P->codes = codes;
  P->tau_kappa = tau_kappa;
  P->sf = sf_of(scheme);
  P->sym = sym;
  P->st = (hipStream_t)hip_stream;
  P->store_recovery = store_recovery != 0;
  const auto t0 = std::chrono::steady_clock::now();
  HDG_CHECK(hipStreamCreateWithFlags(&P->cap_st, hipStreamNonBlocking));
  P->ref.build(P->d, k, 1.0 / P->n);
  if (has_rt) P->ref.build_rt();
  P->nv = P->ref.nv;
  P->ne = P->ref.ne;
  P->nl = P->ref.nl;
  P->nq = P->ref.nq;
  P->nelem = ipow(P->n, P->d);
  P->rd.Phi = upload(P, P->ref.Phi);
  P->rd.Wq = upload(P, P->ref.Wq);
  P->rd.B = upload(P, P->ref.B);
  P->rd.F = upload(P, P->ref.F);
  P->rd.G = upload(P, P->ref.G);
  P->rd.E = upload(P, P->ref.E);
  P->rd.H = upload(P, P->ref.H);
  P->rd.M = upload(P, P->ref.M);
  P->rd.Jp = upload(P, P->ref.Jp);
  if (has_ipdg) {
    P->rd.Kst = upload(P, P->ref.Kst);
    P->rd.Nn = upload(P, P->ref.Nn);
    P->rd.Dn = upload(P, P->ref.Dn);
    P->rd.Dnode = upload(P, P->ref.Dnode);
  }
  if (has_rt) {
    P->rd.Vq = upload(P, P->ref.Vq);
    P->rd.Bd = upload(P, P->ref.Bd);
    P->rd.Fr = upload(P, P->ref.Fr);
    P->rd.Vnode = upload(P, P->ref.Vnode);
  }
  if (scheme == SCHEME_MULTI) {
    P->emask = dalloc<int>(P, P->nelem, false);
    HDG_CHECK(hipMemcpy(P->emask, mask_host.data(), sizeof(int) * P->nelem, hipMemcpyHostToDevice));
  }
  P->kqp = dalloc<double>(P, P->nelem * P->nq, false);
  P->Ae = dalloc<double>(P, P->nelem * P->nl * P->nl, false);
  P->W = dalloc<double>(P, P->nelem * P->nv * P->nl, false);
  if (P->store_recovery) {
    P->Kinv = dalloc<double>(P, P->nelem * P->nv * P->nv, false);
    if (scheme == HDG_SCHEME_HDG)
      P->Minv = dalloc<double>(P, P->nelem * P->nv * P->nv, false);
    else
      P->Xr = dalloc<double>(P, P->nelem * P->nv * P->nl, false);
    if (has_rt) {
      P->Xq = dalloc<double>(P, P->nelem * P->d * P->nv * P->nl, false);
      P->Yq = dalloc<double>(P, P->nelem * P->d * P->nv * P->nv, false);
    }
  }
  P->ework = dalloc<double>(P, P->nelem * (P->nv + P->nl), false);
  P->bad = dalloc<int>(P, 1, false);
  HDG_CHECK(hipHostMalloc((void**)&P->hbad, sizeof(int) * 4, hipHostMallocDefault));
  HDG_CHECK(hipHostMalloc((void**)&P->hpin, sizeof(double) * SC_COUNT * HDG_MAX_NRHS, hipHostMallocDefault));
  if (!check_kappa(P, kappa, kappa_kind)) {
    hdg_destroy(P);
    return HDG_ERR_INVALID_ARG;
  }
  (void)scratch_ptr();  // this device's fixed staging of hdg_rhs_noalloc, looked up once per device
  form_elements(P);
  HDG_CHECK(hipStreamSynchronize(P->st));
  P->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  hdg_default_opts(&P->opts);
  *out = P;
  return HDG_OK;
  }
  catch (const HipError& e) {
    hdg_destroy(P);
    return map_error(e);
  }
  catch (const std::bad_alloc&) {
    hdg_destroy(P);
    return HDG_ERR_DEVICE;
  }
}

}  // namespace

hdg_status hdg_setup(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                     int store_recovery, void* hip_stream, hdg_handle* out) {
  return hdg_setup_scheme(mesh, k, tau, kappa, kappa_kind, HDG_SCHEME_HDG, store_recovery, hip_stream, out);
}

hdg_status hdg_setup_scheme(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                            int scheme, int store_recovery, void* hip_stream, hdg_handle* out) {
  if (scheme & ~(15 | HDG_SCHEME_TAU_KAPPA)) return HDG_ERR_INVALID_ARG;
  const bool tau_kappa = (scheme & HDG_SCHEME_TAU_KAPPA) != 0;
  scheme &= 15;
  if (scheme < HDG_SCHEME_HDG || scheme > HDG_SCHEME_RT) return HDG_ERR_INVALID_ARG;
  return setup_impl(mesh, k, tau, kappa, kappa_kind, scheme, tau_kappa, {scheme}, {}, store_recovery, hip_stream, out);
}

hdg_status hdg_setup_multi(const hdg_mesh* mesh, int k, double tau, const double* kappa, int kappa_kind,
                           const int* scheme_of_element, int options, int store_recovery, void* hip_stream,
                           hdg_handle* out) {
  if (!mesh || !scheme_of_element || (options & ~HDG_SCHEME_TAU_KAPPA)) return HDG_ERR_INVALID_ARG;
  if (mesh->n < 1 || mesh->n > 8192 || mesh->dim != 2) return mesh->dim != 2 ? HDG_ERR_UNSUPPORTED : HDG_ERR_INVALID_ARG;
  const long nel = (long)mesh->n * mesh->n;
  std::vector<int> mask(nel);
  if (hipMemcpy(mask.data(), scheme_of_element, sizeof(int) * nel, hipMemcpyDeviceToHost) != hipSuccess)
    return HDG_ERR_INVALID_ARG;
  std::vector<int> codes;
  for (int c : mask) {
    if (c != HDG_SCHEME_SIPG && c != HDG_SCHEME_IIPG && c != HDG_SCHEME_NIPG && c != HDG_SCHEME_RT)
      return HDG_ERR_INVALID_ARG;
    if (std::find(codes.begin(), codes.end(), c) == codes.end()) codes.push_back(c);
  }
  std::sort(codes.begin(), codes.end());
  return setup_impl(mesh, k, tau, kappa, kappa_kind, SCHEME_MULTI, (options & HDG_SCHEME_TAU_KAPPA) != 0, codes, mask,
                    store_recovery, hip_stream, out);
}

hdg_status hdg_update_kappa(hdg_handle P, const double* kappa, int kappa_kind) {
  if (!P || !kappa) return HDG_ERR_INVALID_ARG;
  if (P->unstructured) return HDG_ERR_UNSUPPORTED;
  if (kappa_kind != HDG_KAPPA_PER_ELEMENT && kappa_kind != HDG_KAPPA_AT_QP) return HDG_ERR_INVALID_ARG;
  if (kappa_kind == HDG_KAPPA_AT_QP) {
    bool elem_only = P->tau_kappa;
    for (int c : P->codes) elem_only |= c == HDG_SCHEME_SIPG || c == HDG_SCHEME_IIPG || c == HDG_SCHEME_NIPG;
    if (elem_only) return HDG_ERR_UNSUPPORTED;
  }
  HDG_GUARD_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  if (!check_kappa(P, kappa, kappa_kind)) return HDG_ERR_INVALID_ARG;
  free_build(P);
  form_elements(P);
  HDG_CHECK(hipStreamSynchronize(P->st));
  P->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
  HDG_GUARD_END
}

namespace {

// Solver storage of a build (shared by the grid and the unstructured
// hierarchies): Chebyshev smoother data, Krylov vectors, device scalars and
// reduction partials, the GMRES basis.
void alloc_solver(hdg_problem* P, const hdg_mg_opts& o) {
  std::vector<Level>& L = P->L;
  const int cap = P->cap;
  P->N = L[0].nlam;
  const long N = P->N;
  const long Nc = N * cap;
  if (o.smoother == HDG_SMOOTHER_CHEBYSHEV) {
    // per level: lmax of D^-1 A by power iteration (FP64), then the
    // diagonal blocks scaled by the reciprocal roots of the degree-m
    // Chebyshev polynomial on [lmax / 30, lmax], one copy per step
    Scratch ps;
    ps.sc = dalloc<double>(P, SC_COUNT, true);
    ps.partials = dalloc<double>(P, 2L * MAX_RED_BLOCKS, true);
    ps.row = 2L * MAX_RED_BLOCKS;
    for (auto& Li : L) {
      if (Li.nface == 0 || Li.kind == 2) continue;
      double* v = (double*)Li.r[0];
      double* y = (double*)Li.e[0];
      double* z = (double*)Li.w[0];
      blas_fill<double>(v, 1.0, Li.nlam, P->st);
      auto dinv_apply = [&](const double* in, double* out) {  // out = D^-1 A in
        launch_apply<double>(Li, APPLY_Y, in, nullptr, y, nullptr, nullptr, P->st);
        launch_jacobi0<double>(Li, y, out, P->st);
      };
      for (int it = 0; it < CHEB_POWER_ITS; ++it) {
        dinv_apply(v, z);
        blas_dot(z, z, Li.nlam, ps, FIN_NORM_INV, ps.sc + SC_HNORM, P->st);
        blas_scale(v, z, Li.nlam, ps.sc + SC_TMP, P->st);
      }
      dinv_apply(v, z);
      blas_dot(z, z, Li.nlam, ps, FIN_NORM_INV, ps.sc + SC_HNORM, P->st);
      Li.lmax = CHEB_SAFETY * read_scalar(P, ps.sc + SC_HNORM);
      const double lmin = Li.lmax / CHEB_RATIO, theta = 0.5 * (Li.lmax + lmin), dlt = 0.5 * (Li.lmax - lmin);
      const long nd = pad64(Li.nface) * vpad<double>((long)Li.ne * Li.ne);
      const long nd32 = pad64(Li.nface) * vpad<float>((long)Li.ne * Li.ne);
      if (nd32 != nd) throw HipError{hipErrorInvalidValue, "Chebyshev copies: block padding differs"};
      for (int si = 1; si <= Li.sweeps; ++si) {
        const double root = theta - dlt * std::cos((2.0 * si - 1.0) * M_PI / (2.0 * Li.sweeps));
        double* c64 = dalloc<double>(P, nd, true);
        float* c32 = dalloc<float>(P, nd, true);
        launch_scale_copy(nd, 1.0 / root, Li.Dinv64, c64, c32, P->st);
        Li.cheb64.push_back(c64);
        Li.cheb32.push_back(c32);
      }
    }
  }
  P->g = dalloc<double>(P, Nc, true);
  P->r = dalloc<double>(P, Nc, true);
  P->z = dalloc<double>(P, Nc, true);
  P->p = dalloc<double>(P, Nc, true);
  P->Ap = dalloc<double>(P, Nc, true);
  P->zold = dalloc<double>(P, Nc, true);
  P->lam = dalloc<double>(P, Nc, true);
  P->r32 = dalloc<float>(P, Nc, true);
  P->z32 = dalloc<float>(P, Nc, true);
  {
    // device scalars and reduction partials, one row per right-hand side
    P->s.sc = dalloc<double>(P, (long)SC_COUNT * cap, true);
    const long nface0 = L[0].nface;
    const long nb = std::max<long>(MAX_RED_BLOCKS, (nface0 + 255) / 256 + 64);  // + XCD padding blocks
    P->s.partials = dalloc<double>(P, 2 * nb * cap, true);
    P->s.row = 2 * nb;
    P->s.pcg = dalloc<double>(P, 2L * MAX_RED_BLOCKS * cap, true);
    HDG_CHECK(hipMemsetAsync(P->s.sc, 0, sizeof(double) * SC_COUNT * cap, P->st));
  }
  if (o.method == HDG_METHOD_GMRES) {
    const int m = o.restart > 0 ? std::min(o.restart, std::max(o.max_it, 1)) : std::max(o.max_it, 1);
    P->gm_m = m;
    P->V = dalloc<double>(P, (long)(m + 1) * N, true);
    P->Z = dalloc<double>(P, (long)m * N, true);
    P->H = dalloc<double>(P, (long)(m + 1) * (m + 1), true);
    P->cs = dalloc<double>(P, m + 1, true);
    P->sn = dalloc<double>(P, m + 1, true);
    P->gsv = dalloc<double>(P, m + 2, true);
    P->y = dalloc<double>(P, m + 1, true);
  }
}

hdg_status ubuild(hdg_problem* P, const hdg_mg_opts& o);

}  // namespace

hdg_status hdg_mg_build(hdg_handle P, const hdg_mg_opts* opts) {
  if (!P) return HDG_ERR_INVALID_ARG;
  hdg_mg_opts o;
  if (opts)
    o = *opts;
  else
    hdg_default_opts(&o);
  if (o.sweeps < 0 || o.sweeps > 64 || (o.growth != 1 && o.growth != 2) || !(o.omega > 0.0) ||
      o.local_corr < 0 || o.local_corr > 3 || (o.precision != HDG_FP64 && o.precision != HDG_MIXED) ||
      o.method < 0 || o.method > 2 || o.max_it < 0 || o.restart < 0 || o.coarse_n < 0 || o.nrhs < 0 ||
      o.nrhs > HDG_MAX_NRHS || !(o.refine_red >= 0.0 && o.refine_red < 1.0) || o.variant < 0 || o.variant > 1023 ||
      o.smoother < HDG_SMOOTHER_BLOCK_JACOBI || o.smoother > HDG_SMOOTHER_LUSGS)
    return HDG_ERR_INVALID_ARG;
  if (o.nrhs < 1) o.nrhs = 1;
  if (o.refine_red == 0.0) o.refine_red = 1e-5;
  if (o.coarse_n < 2) o.coarse_n = 2;
  if (P->unstructured) return ubuild(P, o);
  if ((P->n & (P->n - 1)) != 0) return HDG_ERR_UNSUPPORTED;
  if (!P->sym && o.method == HDG_METHOD_PCG) return HDG_ERR_UNSUPPORTED;  // CG needs a symmetric operator
  // The persistent coarse cycle is switched off.  Launched eagerly (single
  // V-cycles) it matched the per-level kernels bit for bit once its grid
  // left residency slack; inside a graph-captured CG solve the device then
  // reported an error and the queue was lost, for a reason not yet shown.
  // Until that is found the variant is refused here, before any allocation.
  if (o.variant & HDG_VARIANT_GRID_TAIL) return HDG_ERR_UNSUPPORTED;
  HDG_GUARD_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  free_build(P);
  P->opts = o;
  P->cap = o.nrhs;
  P->use_graphs = !(o.variant & HDG_VARIANT_NO_GRAPH);
  P->fuse = !(o.variant & HDG_VARIANT_NO_FUSE);
  P->tail_nmax = (o.variant & HDG_VARIANT_NO_TAIL) ? 0 : 32;
  P->pack = !(o.variant & HDG_VARIANT_NO_PACK);
  P->strip = !(o.variant & HDG_VARIANT_NO_STRIP);
  // mixed cycle form: FP64 vectors over FP32 operator blocks in 3D (the FP32
  // cycle stalls CG there), FP32 vectors in 2D; the variant bits force one.
  // The FP64-vector form reads face-major blocks with the unfused kernels.
  P->ops32 = o.precision == HDG_MIXED && !(o.variant & HDG_VARIANT_FP32_VECTORS) &&
             (P->d == 3 || (o.variant & HDG_VARIANT_FP64_VECTORS));
  if (P->ops32 || o.smoother != HDG_SMOOTHER_BLOCK_JACOBI) {
    P->pack = false;
    P->fuse = false;
    P->tail_nmax = 0;
  }
  // nonsymmetric operators: no packed (symmetrised) element maps, and no
  // coarse tail (it restricts with P^T); the grid kernels take the
  // restriction block R
  if (!P->sym) {
    P->pack = false;
    P->tail_nmax = 0;
  }
  const int cap = P->cap;
  const int d = P->d;
  const int nc = 1 << (d - 1);
  std::vector<Level>& L = P->L;
  L.emplace_back();
  init_level(L[0], d, P->n, P->ne);
  L[0].Aelem = P->Ae;
  L[0].own_Aelem = false;
  if (P->k > 1 && P->n >= 2) {
    L[0].kind = 0;
    L.emplace_back();
    init_level(L[1], d, P->n, nc);
    L[1].Aelem = dalloc<double>(P, L[1].nelem * L[1].nl * L[1].nl, true);
    launch_pgalerkin(d, P->ne, P->nelem, P->rd.Jp, P->Ae, L[1].Aelem, P->st);
  }
  while (L.back().n > o.coarse_n) {
    const size_t fi = L.size() - 1;
    L.emplace_back();
    Level& F = L[fi];
    Level& C = L.back();
    F.kind = 1;
    init_level(C, d, F.n / 2, nc);
    F.nmacro = C.nelem;
    F.nI = d * nc * nc;
    F.ncl = 2 * d * nc;
    const long pm = pad64(F.nmacro);
    F.AIIinv64 = dalloc<double>(P, pm * vpad<double>(F.nI * F.nI), true);
    F.AIIinv32 = dalloc<float>(P, pm * vpad<float>(F.nI * F.nI), true);
    F.P64 = dalloc<double>(P, pm * vpad<double>(F.nI * F.ncl), true);
    F.P32 = dalloc<float>(P, pm * vpad<float>(F.nI * F.ncl), true);
    F.sym = P->sym;
    if (F.sym) {
      F.R64 = F.P64;
      F.R32 = F.P32;
    } else {
      F.R64 = dalloc<double>(P, pm * vpad<double>(F.nI * F.ncl), true);
      F.R32 = dalloc<float>(P, pm * vpad<float>(F.nI * F.ncl), true);
    }
    F.cb[0] = dalloc<double>(P, F.nmacro * F.ncl * cap, true);
    F.cb[1] = dalloc<float>(P, F.nmacro * F.ncl * cap, true);
    C.Aelem = dalloc<double>(P, C.nelem * C.nl * C.nl, true);
    launch_macro_schur(F, C, P->st);
  }
  Level& Lc = L.back();
  Lc.kind = 2;
  if (Lc.nlam > 8192) return HDG_ERR_UNSUPPORTED;  // dense coarsest inverse: N^2 doubles
  if (Lc.nlam > 0) {
    Lc.Ainv64 = dalloc<double>(P, Lc.nlam * Lc.nlam, true);
    Lc.Ainv32 = dalloc<float>(P, Lc.nlam * Lc.nlam, true);
    launch_coarse_inverse(Lc, P->st);
  }
  for (size_t i = 0; i < L.size(); ++i) {
    Level& Li = L[i];
    Li.sweeps = o.sweeps * (o.growth == 2 ? (1 << std::min<size_t>(i, 20)) : 1);
    Li.lpm = (o.variant & HDG_VARIANT_LANES1) ? 1 : (o.variant & HDG_VARIANT_LANES4) ? 4 : 0;
    const long pf = pad64(Li.nface);
    // the finest level of a p-transition (only trace applies touch it) is
    // stored element-major as packed symmetric triangles
    Li.packed = Li.kind == 0 && P->pack && Li.nface > 0 && d == 2;  // 3D element maps (nl >= 54) would spill
    Li.strip = Li.packed && P->strip && Li.n % 64 == 0;
    if (Li.packed) {
      const long npk = (long)Li.nl * (Li.nl + 1) / 2;
      Li.Ap64 = dalloc<double>(P, pad64(Li.nelem) * pk_pad<double>(npk), true);
      Li.Ap32 = dalloc<float>(P, pad64(Li.nelem) * pk_pad<float>(npk), true);
      Li.z[0] = dalloc<double>(P, pad64(Li.nelem) * Li.nl * cap, true);
      Li.z[1] = dalloc<float>(P, pad64(Li.nelem) * Li.nl * cap, true);
    } else {
      Li.Af64 = dalloc<double>(P, pf * 2 * vpad<double>((long)Li.nl * Li.ne), true);
      Li.Af32 = dalloc<float>(P, pf * 2 * vpad<float>((long)Li.nl * Li.ne), true);
    }
    Li.Dinv64 = dalloc<double>(P, pf * vpad<double>((long)Li.ne * Li.ne), true);
    Li.Dinv32 = dalloc<float>(P, pf * vpad<float>((long)Li.ne * Li.ne), true);
    for (int pr = 0; pr < 2; ++pr) {
      const size_t es = pr == 0 ? sizeof(double) : sizeof(float);
      for (void** slot : {&Li.r[pr], &Li.e[pr], &Li.w[pr]}) {
        if (pr == 0)
          *slot = dalloc<double>(P, Li.nlam * cap, true);
        else
          *slot = dalloc<float>(P, Li.nlam * cap, true);
        (void)es;
      }
    }
    if (Li.nface > 0) {
      if (Li.packed)
        launch_pack_sym(Li, P->st);
      else
        launch_face_major(Li, P->st);
      const int dmode = o.smoother == HDG_SMOOTHER_BLOCK_JACOBI ? 0 : o.smoother == HDG_SMOOTHER_LUSGS ? 2 : 1;
      launch_dinv(Li, o.smoother == HDG_SMOOTHER_CHEBYSHEV ? 1.0 : o.omega, P->st, dmode);
    }
  }
  // one-workgroup coarse tail (2D, fused path): the first level from which
  // every remaining level's vectors fit the LDS arena
  for (int pr = 0; pr < 2; ++pr) {
    P->tail_start[pr] = -1;
    if (d != 2 || !P->fuse || o.sweeps < 1 || P->tail_nmax <= 0) continue;
    const long es = pr == 0 ? 8 : 4;
    for (int t = 0; t < (int)L.size(); ++t) {
      if (L[t].kind != 1 || L[t].n > P->tail_nmax || L.back().nlam > 64) continue;
      if ((int)L.size() - t > TAIL_MAX_LEVELS) continue;
      TailArgs ta;
      ta.nlev = (int)L.size() - t;
      ta.lc = o.local_corr;
      long off = 0;
      auto take = [&](long cnt) {
        long o2 = off;
        off += (cnt + 3) / 4 * 4;
        return o2;
      };
      for (int l = t; l < (int)L.size(); ++l) {
        const Level& Ll = L[l];
        TailLevel& tl = ta.lev[l - t];
        tl.n = Ll.n;
        tl.kind = Ll.kind;
        tl.sweeps = Ll.sweeps;
        tl.nlam = Ll.nlam;
        tl.nface = Ll.nface;
        tl.nmacro = Ll.kind == 1 ? Ll.nmacro : 0;
        tl.Af = pr == 0 ? (const void*)Ll.Af64 : (const void*)Ll.Af32;
        tl.Dinv = pr == 0 ? (const void*)Ll.Dinv64 : (const void*)Ll.Dinv32;
        tl.AIIinv = pr == 0 ? (const void*)Ll.AIIinv64 : (const void*)Ll.AIIinv32;
        tl.P = pr == 0 ? (const void*)Ll.P64 : (const void*)Ll.P32;
        tl.Ainv = pr == 0 ? (const void*)Ll.Ainv64 : (const void*)Ll.Ainv32;
        tl.off_r = take(Ll.nlam);
        tl.off_e = take(Ll.nlam);
        tl.off_w = take(Ll.nlam);
        tl.off_cb = take(Ll.kind == 1 ? Ll.nmacro * Ll.ncl : 0);
      }
      if (off * es > TAIL_ARENA_BYTES) continue;
      P->tail_start[pr] = t;
      P->tail_args[pr] = ta;
      break;
    }
  }

  // persistent coarse cycle (2D fused path, one right-hand side): from the
  // first h-level of at most GTAIL_NMAX elements per direction below the
  // finest down to a coarsest level solved by the dense row-per-wavefront
  // product (more than 64 unknowns); it replaces the one-workgroup tail
  P->gtail_start[0] = P->gtail_start[1] = -1;
  if ((o.variant & HDG_VARIANT_GRID_TAIL) && d == 2 && P->fuse && o.sweeps >= 1 && L.back().kind == 2 &&
      L.back().nlam > 64) {
    for (int pr = 0; pr < 2; ++pr) {
      const int grid = pr == 0 ? gtail_grid<double>() : gtail_grid<float>();
      if (grid <= 0) continue;
      for (int t = 1; t + 1 < (int)L.size(); ++t) {
        if (L[t].n > GTAIL_NMAX || (int)L.size() - t > TAIL_MAX_LEVELS) continue;
        bool ok = true;
        for (int l = t; l + 1 < (int)L.size(); ++l)
          ok = ok && L[l].kind == 1 && !L[l].packed && !L[l].strip && !L[l].u && L[l].ne == 2 && L[l].sweeps >= 1;
        if (!ok) continue;
        GTailArgs ga;
        ga.nlev = (int)L.size() - t;
        ga.lc = o.local_corr;
        for (int l = t; l < (int)L.size(); ++l) {
          const Level& Ll = L[l];
          GTailLevel& g = ga.lev[l - t];
          g.n = Ll.n;
          g.kind = Ll.kind;
          g.sweeps = Ll.sweeps;
          g.lpm = Ll.kind == 1 ? level_lanes(Ll, 1) : 1;
          g.nlam = Ll.nlam;
          g.nface = Ll.nface;
          g.nmacro = Ll.kind == 1 ? Ll.nmacro : 0;
          g.Af = pr == 0 ? (const void*)Ll.Af64 : (const void*)Ll.Af32;
          g.Dinv = pr == 0 ? (const void*)Ll.Dinv64 : (const void*)Ll.Dinv32;
          g.AIIinv = pr == 0 ? (const void*)Ll.AIIinv64 : (const void*)Ll.AIIinv32;
          g.R = pr == 0 ? (const void*)Ll.R64 : (const void*)Ll.R32;
          g.P = pr == 0 ? (const void*)Ll.P64 : (const void*)Ll.P32;
          g.Ainv = pr == 0 ? (const void*)Ll.Ainv64 : (const void*)Ll.Ainv32;
          g.r = Ll.r[pr];
          g.e = Ll.e[pr];
          g.w = Ll.w[pr];
          g.cb = Ll.cb[pr];
          if (!g.r || !g.e || (Ll.kind == 1 && (!g.w || !g.cb || !g.Af || !g.Dinv || !g.AIIinv || !g.R || !g.P)) ||
              (Ll.kind == 2 && !g.Ainv))
            ok = false;
        }
        if (!ok) break;
        if (!P->gtail_sync) {
          P->gtail_sync = dalloc<unsigned>(P, GTAIL_SYNC_WORDS, true);
          HDG_CHECK(hipMemsetAsync(P->gtail_sync, 0, sizeof(unsigned) * GTAIL_SYNC_WORDS, P->st));
        }
        ga.sync = P->gtail_sync;
        P->gtail_start[pr] = t;
        P->gtail_args[pr] = ga;
        P->gtail_grid_n[pr] = grid;
        P->tail_start[pr] = -1;
        break;
      }
    }
  }

  alloc_solver(P, o);
  HDG_CHECK(hipStreamSynchronize(P->st));
  P->built = true;
  P->t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
  HDG_GUARD_END
}


namespace {

// The hierarchy of an unstructured handle (levels fixed at setup by the
// agglomeration): P^1 Galerkin maps of the triangles, per agglomeration step
// the coarse cells' Schur complements, A_II^-1 and P, the coarsest dense
// inverse, then every level's apply storage (AoSoA / FP32 maps), face-block
// inverses and vectors.  Block-Jacobi smoothing only; the mixed cycle keeps
// FP64 vectors over FP32 maps; no fused kernels, coarse tail or packing.
hdg_status ubuild(hdg_problem* P, const hdg_mg_opts& o) {
  if (o.smoother != HDG_SMOOTHER_BLOCK_JACOBI) return HDG_ERR_UNSUPPORTED;
  if (!P->sym && o.method == HDG_METHOD_PCG) return HDG_ERR_UNSUPPORTED;  // CG needs a symmetric operator
  HDG_GUARD_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  free_build(P);
  P->opts = o;
  P->cap = o.nrhs;
  P->use_graphs = !(o.variant & HDG_VARIANT_NO_GRAPH);
  P->fuse = false;
  P->tail_nmax = 0;
  P->pack = false;
  P->strip = false;
  P->ops32 = o.precision == HDG_MIXED;
  P->tail_start[0] = P->tail_start[1] = -1;
  const int cap = P->cap;
  // coarse_n > 2: the hierarchy stops at the coarsest level with at least
  // coarse_n^2 trace unknowns (solved by the dense inverse)
  int nlev = (int)P->ul.size();
  if (o.coarse_n > 2) {
    int last = 0;
    for (int i = 0; i < (int)P->ul.size(); ++i)
      if (P->ul[i].nface * P->ul[i].m >= (long)o.coarse_n * o.coarse_n) last = i;
    nlev = last + 1;
  }
  if (nlev < 2 || P->ul[nlev - 1].nface * P->ul[nlev - 1].m > UCOARSE_MAX) return HDG_ERR_UNSUPPORTED;
  std::vector<Level>& L = P->L;
  L.resize(nlev);
  for (int i = 0; i < nlev; ++i) {
    ULevel& U = P->ul[i];
    Level& Li = L[i];
    Li.d = 2;
    Li.n = 0;
    Li.ne = U.m;
    Li.nl = U.tri ? 3 * U.m : 0;
    Li.nelem = U.ncell;
    Li.nfd = U.nface;
    Li.nface = U.nface;
    Li.nlam = U.nface * U.m;
    Li.u = &U;
    Li.kind = i == nlev - 1 ? 2 : (i == 0 && P->k > 1) ? 0 : 1;
    Li.sym = P->sym;
  }
  L[0].Aelem = P->Ae;
  L[0].own_Aelem = false;
  if (P->k > 1) {
    L[1].Aelem = dalloc<double>(P, P->nelem * 36, true);
    launch_tri_pgalerkin(P->k, P->nelem, P->rd.Jp, P->Ae, L[1].Aelem, P->st);
  }
  long nwork = 0;
  for (int i = 0; i + 1 < nlev; ++i) nwork = std::max(nwork, P->ul[i].nwork);
  double* work = nwork > 0 ? dalloc<double>(P, nwork, true) : nullptr;
  for (int i = 0; i + 1 < nlev; ++i) {
    Level& F = L[i];
    if (F.kind != 1) continue;
    ULevel& U = P->ul[i];
    F.nmacro = U.ncoarse;
    F.AIIinv64 = dalloc<double>(P, std::max(U.asize, 1L), true);
    F.AIIinv32 = dalloc<float>(P, std::max(U.asize, 1L), true);
    F.P64 = dalloc<double>(P, std::max(U.psize, 1L), true);
    F.P32 = dalloc<float>(P, std::max(U.psize, 1L), true);
    if (P->sym) {
      F.R64 = F.P64;
      F.R32 = F.P32;
    } else {
      F.R64 = dalloc<double>(P, std::max(U.psize, 1L), true);
      F.R32 = dalloc<float>(P, std::max(U.psize, 1L), true);
    }
    F.cb[0] = dalloc<double>(P, std::max(U.ncb, 1L) * cap, true);
    F.cb[1] = dalloc<float>(P, std::max(U.ncb, 1L) * cap, true);
    L[i + 1].Aelem = dalloc<double>(P, std::max(P->ul[i + 1].msize, 1L), true);
    launch_uschur(U, P->ul[i + 1], F.Aelem, F.AIIinv64, F.P64, P->sym ? nullptr : F.R64, L[i + 1].Aelem, work,
                  P->st);
    launch_to_f32(F.AIIinv64, F.AIIinv32, U.asize, P->st);
    launch_to_f32(F.P64, F.P32, U.psize, P->st);
    if (!P->sym) launch_to_f32(F.R64, F.R32, U.psize, P->st);
  }
  Level& Lc = L.back();
  if (Lc.nlam > UCOARSE_MAX) return HDG_ERR_UNSUPPORTED;
  if (Lc.nlam > 0) {
    Lc.Ainv64 = dalloc<double>(P, Lc.nlam * Lc.nlam, true);
    Lc.Ainv32 = dalloc<float>(P, Lc.nlam * Lc.nlam, true);
    double* dense = dalloc<double>(P, 2 * Lc.nlam * Lc.nlam, true);
    launch_ucoarse_inverse(Lc, dense, P->st);
  }
  for (int i = 0; i < nlev; ++i) {
    Level& Li = L[i];
    ULevel& U = P->ul[i];
    Li.sweeps = o.sweeps * (o.growth == 2 ? (1 << std::min(i, 20)) : 1);
    if (U.tri) {
      const long nn = 9L * U.m * U.m;
      Li.Af64 = dalloc<double>(P, pad64(U.ncell) * pk_pad<double>(nn), true);
      Li.Af32 = dalloc<float>(P, pad64(U.ncell) * pk_pad<float>(nn), true);
      U.Am32 = nullptr;
    } else {
      U.Am32 = dalloc<float>(P, std::max(U.msize, 1L), true);
    }
    U.z[0] = dalloc<double>(P, std::max(U.nrow, 1L) * cap, true);
    U.z[1] = dalloc<float>(P, std::max(U.nrow, 1L) * cap, true);
    launch_umaps(Li, P->st);
    const long pf = pad64(Li.nface);
    Li.Dinv64 = dalloc<double>(P, std::max(pf, 64L) * vpad<double>((long)Li.ne * Li.ne), true);
    Li.Dinv32 = dalloc<float>(P, std::max(pf, 64L) * vpad<float>((long)Li.ne * Li.ne), true);
    launch_udinv(Li, P->st);
    for (int pr = 0; pr < 2; ++pr)
      for (void** slot : {&Li.r[pr], &Li.e[pr], &Li.w[pr]}) {
        if (pr == 0)
          *slot = dalloc<double>(P, std::max(Li.nlam, 1L) * cap, true);
        else
          *slot = dalloc<float>(P, std::max(Li.nlam, 1L) * cap, true);
      }
  }
  alloc_solver(P, o);
  HDG_CHECK(hipStreamSynchronize(P->st));
  P->built = true;
  P->t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return HDG_OK;
  HDG_GUARD_END
}

// device copies of the host topology, level by level
void upload_ulevels(hdg_problem* P) {
  const UHost& H = *P->uh;
  P->ul.clear();
  P->ul.reserve(H.lev.size());
  for (size_t i = 0; i < H.lev.size(); ++i) {
    const UHostLevel& h = H.lev[i];
    ULevel U;
    U.m = h.m;
    U.tri = h.tri;
    U.ncell = h.ncell;
    U.nface = h.nface;
    const long nslot = h.sptr[h.ncell];
    U.nrow = nslot * h.m;
    U.zstride = 1;
    U.sptr = upload(P, h.sptr);
    U.sface = upload(P, h.sface);
    if (h.nface > 0) {
      U.fcell = upload(P, h.fcell);
      U.fslot = upload(P, h.fslot);
    }
    std::vector<long> moff(h.ncell), zr(2 * h.nface);
    std::vector<int> rcell;
    long msz = 0;
    for (long c = 0; c < h.ncell; ++c) {
      const long ns = h.sptr[c + 1] - h.sptr[c];
      moff[c] = msz;
      msz += (h.m * ns) * (h.m * ns);
      if (!h.tri)
        for (long r = 0; r < h.m * ns; ++r) rcell.push_back((int)c);
    }
    for (long f = 0; f < h.nface; ++f)
      for (int side = 0; side < 2; ++side)
        zr[2 * f + side] = (h.sptr[h.fcell[2 * f + side]] + h.fslot[2 * f + side]) * h.m;
    U.msize = msz;
    U.moff = upload(P, moff);
    if (h.nface > 0) U.zr = upload(P, zr);
    if (!rcell.empty()) U.rcell = upload(P, rcell);
    if (h.ncoarse > 0) {
      const UHostLevel& c = H.lev[i + 1];
      const long nc = h.ncoarse;
      U.ncoarse = nc;
      U.iptr = upload(P, h.iptr);
      U.bptr = upload(P, h.bptr);
      U.ccptr = upload(P, h.ccptr);
      if (!h.iface.empty()) U.iface = upload(P, h.iface);
      if (!h.bface.empty()) {
        U.bface = upload(P, h.bface);
        U.bslot = upload(P, h.bslot);
      }
      U.ccell = upload(P, h.ccell);
      U.sloc = upload(P, h.sloc);
      U.fE = upload(P, h.fE);
      U.fJ = upload(P, h.fJ);
      std::vector<int> irc, cbc;
      std::vector<long> aoff(nc), poff(nc), woff(nc);
      long as = 0, ps = 0, ws = 0;
      for (long C = 0; C < nc; ++C) {
        const long nI2 = 2 * (h.iptr[C + 1] - h.iptr[C]), nB = h.bptr[C + 1] - h.bptr[C];
        const long n2 = nI2 + 2 * nB, nc2 = 2 * (c.sptr[C + 1] - c.sptr[C]);
        if (n2 > UMACRO_MAX_DOFS) throw std::invalid_argument("a macro-element has too many trace values");
        aoff[C] = as;
        poff[C] = ps;
        woff[C] = ws;
        as += nI2 * nI2;
        ps += nI2 * nc2;
        ws += n2 * n2 + 2 * nB * nc2;
        for (long j = 0; j < nI2; ++j) irc.push_back((int)C);
        for (long j = 0; j < nc2; ++j) cbc.push_back((int)C);
      }
      U.nIrow = (long)irc.size();
      U.ncb = (long)cbc.size();
      U.asize = as;
      U.psize = ps;
      U.nwork = ws;
      if (!irc.empty()) U.irc = upload(P, irc);
      if (!cbc.empty()) U.cbc = upload(P, cbc);
      U.aoff = upload(P, aoff);
      U.poff = upload(P, poff);
      U.woff = upload(P, woff);
    }
    if (!h.eptr.empty()) {
      U.eptr = upload(P, h.eptr);
      if (!h.efine.empty()) U.efine = upload(P, h.efine);
    }
    P->ul.push_back(U);
  }
  for (size_t i = 0; i + 1 < P->ul.size(); ++i)
    if (P->ul[i].ncoarse > 0) {
      P->ul[i].csptr = P->ul[i + 1].sptr;
      P->ul[i].csface = P->ul[i + 1].sface;
    }
}

}  // namespace

hdg_status hdg_setup_unstructured(const hdg_umesh* mesh, int k, double tau, const double* kappa, int scheme,
                                  void* hip_stream, hdg_handle* out) {
  if (!mesh || !out || !kappa || !mesh->xy || !mesh->tri || !mesh->seeds) return HDG_ERR_INVALID_ARG;
  if (mesh->nvert < 3 || mesh->ntri < 1 || mesh->nseeds < 1 || mesh->hlevels < 1 || mesh->hlevels > 16)
    return HDG_ERR_INVALID_ARG;
  if (k < 1 || k > 4) return HDG_ERR_UNSUPPORTED;
  if (!(tau > 0.0) || !std::isfinite(tau)) return HDG_ERR_INVALID_ARG;
  if (scheme != HDG_SCHEME_HDG && scheme != HDG_SCHEME_SIPG && scheme != HDG_SCHEME_IIPG &&
      scheme != HDG_SCHEME_NIPG)
    return scheme == HDG_SCHEME_RT ? HDG_ERR_UNSUPPORTED : HDG_ERR_INVALID_ARG;
  *out = nullptr;
  hdg_problem* P = new (std::nothrow) hdg_problem();
  if (!P) return HDG_ERR_DEVICE;
  try {
    P->unstructured = true;
    P->d = 2;
    P->n = 0;
    P->k = k;
    P->tau = tau;
    P->scheme = scheme;
    P->codes = {scheme};
    P->sf = sf_of(scheme);
    P->sym = scheme == HDG_SCHEME_HDG || scheme == HDG_SCHEME_SIPG;
    P->st = (hipStream_t)hip_stream;
    const auto t0 = std::chrono::steady_clock::now();
    HDG_CHECK(hipStreamCreateWithFlags(&P->cap_st, hipStreamNonBlocking));
    P->uh = std::make_unique<UHost>();
    UHost& H = *P->uh;
    H.build_reference(k);
    H.build_mesh(mesh->nvert, mesh->xy, mesh->ntri, mesh->tri, mesh->seeds, mesh->nseeds, mesh->hlevels);
    P->nelem = H.ntri;
    P->nv = H.nv;
    P->ne = k + 1;
    P->nl = 3 * (k + 1);
    P->nq = 1;
    P->rd.uM = upload(P, H.Mh);
    P->rd.uMinv = upload(P, H.Minvh);
    P->rd.uD = upload(P, H.Dh);
    P->rd.uE = upload(P, H.Eh);
    P->rd.uF = upload(P, H.Fh);
    P->rd.uH = upload(P, H.Hh);
    P->rd.Jp = upload(P, H.Jp);
    if (scheme != HDG_SCHEME_HDG) {
      P->rd.uK = upload(P, H.Kh);
      P->rd.uN = upload(P, H.Nh);
      P->rd.uDe = upload(P, H.De);
      P->rd.uGn = upload(P, H.Gnode);
    }
    P->uxy = upload(P, H.xy);
    P->utri = upload(P, H.tri);
    P->utbnd = upload(P, H.tbnd);
    upload_ulevels(P);
    P->kqp = dalloc<double>(P, P->nelem, false);
    P->Ae = dalloc<double>(P, P->nelem * P->nl * P->nl, false);
    P->W = dalloc<double>(P, P->nelem * P->nv * P->nl, false);
    P->bad = dalloc<int>(P, 1, false);
    HDG_CHECK(hipHostMalloc((void**)&P->hbad, sizeof(int) * 4, hipHostMallocDefault));
    HDG_CHECK(hipHostMalloc((void**)&P->hpin, sizeof(double) * SC_COUNT * HDG_MAX_NRHS, hipHostMallocDefault));
    if (!check_kappa(P, kappa, HDG_KAPPA_PER_ELEMENT)) {
      hdg_destroy(P);
      return HDG_ERR_INVALID_ARG;
    }
    P->urec = dalloc<double>(P, P->nelem * 3 * P->nv * (P->nl + P->nv), false);
    if (scheme == HDG_SCHEME_HDG)
      launch_tri_dtn(k, P->nelem, P->rd, P->uxy, P->utri, P->kqp, tau, P->Ae, P->W, P->urec, P->st);
    else
      launch_tri_ipdg_dtn(k, P->nelem, P->rd, P->uxy, P->utri, P->kqp, tau, P->sf, P->Ae, P->W, P->urec, P->st);
    HDG_CHECK(hipStreamSynchronize(P->st));
    P->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    hdg_default_opts(&P->opts);
    *out = P;
    return HDG_OK;
  } catch (const HipError& e) {
    hdg_destroy(P);
    return map_error(e);
  } catch (const std::bad_alloc&) {
    hdg_destroy(P);
    return HDG_ERR_DEVICE;
  } catch (const std::exception&) {
    hdg_destroy(P);
    return HDG_ERR_INVALID_ARG;
  }
}

hdg_status hdg_vcycle(hdg_handle P, const void* r, void* e, int precision, int nrhs) {
  if (!P || !r || !e || nrhs < 1) return HDG_ERR_INVALID_ARG;
  if (!P->built) return HDG_ERR_STATE;
  if (precision != HDG_FP64 && precision != HDG_FP32 && precision != HDG_MIXED_CYCLE) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  for (int i0 = 0; i0 < nrhs && P->N > 0; i0 += P->cap) {
    const int nr = std::min(P->cap, nrhs - i0);
    if (precision == HDG_FP64) {
      vcycle<double>(P, 0, (const double*)r + i0 * P->N, (double*)e + i0 * P->N, false, nr);
    } else if (precision == HDG_FP32) {
      vcycle<float>(P, 0, (const float*)r + i0 * P->N, (float*)e + i0 * P->N, false, nr);
    } else if (P->ops32) {
      vcycle<double, float>(P, 0, (const double*)r + i0 * P->N, (double*)e + i0 * P->N, false, nr);
    } else {  // the FP32 cycle between conversions of r and e
      float* r32 = (float*)P->L[0].r[1];
      blas_d2f((const double*)r + i0 * P->N, r32, P->N, P->st, nr);
      const float* e32 = vcycle<float>(P, 0, r32, nullptr, false, nr);
      blas_f2d(e32, (double*)e + i0 * P->N, P->N, P->st, nr);
    }
  }
  return gtail_check(P);
  HDG_GUARD_END
}

hdg_status hdg_rhs(hdg_handle P, const double* rhs, int rhs_kind, const double* gdir, double* g) {
  if (!P || !rhs || !g) return HDG_ERR_INVALID_ARG;
  if (rhs_kind != HDG_RHS_F_NODAL && rhs_kind != HDG_RHS_F_LOAD) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  form_rhs(P, rhs, rhs_kind, gdir, g);
  return HDG_OK;
  HDG_GUARD_END
}

namespace {
// hdg_solve on the handle's current stream (shared by hdg_solve_batch)
hdg_status solve_rhs_set(hdg_handle P, const double* rhs, int rhs_kind, const double* gdir, int nrhs, double tol,
                         double* lambda, hdg_solve_info* info) {
  if (info) {
    info->iters = 0;
    info->outer_iters = 0;
    info->relres = 0.0;
    info->t_solve_ms = 0.0;
    info->n_levels = (int)P->L.size();
    info->t_setup_ms = P->t_setup_ms;
    info->t_build_ms = P->t_build_ms;
  }
  hipEvent_t e0, e1;
  HDG_CHECK(hipEventCreate(&e0));
  HDG_CHECK(hipEventCreate(&e1));
  HDG_CHECK(hipEventRecord(e0, P->st));
  hdg_status worst = HDG_OK;
  const long vstride = P->nelem * P->nv;
  const long N = P->N;
  // right-hand sides go through in groups of the build's capacity, each group
  // iterated together
  for (int i0 = 0; i0 < nrhs && N > 0; i0 += P->cap) {
    const int nr = std::min(P->cap, nrhs - i0);
    for (int r = 0; r < nr; ++r) {
      if (rhs_kind == HDG_RHS_TRACE)
        blas_copy(P->g + r * N, rhs + (i0 + r) * N, N, P->st);
      else
        form_rhs(P, rhs + (i0 + r) * vstride, rhs_kind, gdir, P->g + r * N);
    }
    blas_copy(P->lam, lambda + i0 * N, N, P->st, nr);
    hdg_status s = solve_many(P, nr, tol, info);
    blas_copy(lambda + i0 * N, P->lam, N, P->st, nr);
    if (s != HDG_OK && worst == HDG_OK) worst = s;
  }
  HDG_CHECK(hipEventRecord(e1, P->st));
  HDG_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  HDG_CHECK(hipEventElapsedTime(&ms, e0, e1));
  if (info) info->t_solve_ms = ms;
  HDG_CHECK(hipEventDestroy(e0));
  HDG_CHECK(hipEventDestroy(e1));
  return worst;
}
// ---------------------------------------------------------------------------
// Many problems through one graph.  Every problem (a built handle, PCG) keeps
// its own buffers, scalars and convergence state; its group of CHECK_EVERY
// CG iterations is captured once as a graph, and one batch graph holds the
// groups of all iterating problems as independent child graphs, so a single
// launch advances every problem and the GPU overlaps their latency-bound
// coarse levels.  Between launches the host reads all residual histories
// with one synchronisation.  The start of a CG run and the true-residual
// check of a refinement step go out eagerly for the problems that need them.
// A problem that has converged keeps iterating inside the batch graph (its
// solution was already copied out) until the work of such problems reaches a
// quarter of the graph's, so the graph is re-instantiated a few times per
// batch rather than once per problem.
// a lane's batch graph is re-instantiated without its finished problems once
// they carry more than this fraction of its work (until then they iterate
// on; their solutions were already copied out); a lane's problems that
// finished their inner solve get their true-residual check once they carry
// this fraction of its iterating work
constexpr double BATCH_IDLE_FRAC = 0.0;
constexpr double BATCH_CHECK_FRAC = 0.0;

struct BatchItem {
  hdg_problem* P = nullptr;
  const double* rhs = nullptr;
  double* lam_out = nullptr;
  int nrhs = 0;
  hdg_solve_info* info = nullptr;
  int i0 = 0, nr = 0;  // current group of right-hand sides
  bool mixed = false;
  double gn[64];
  Tracker tr;
  SolveOut o;
  int launched = 0;
  enum { IDLE, ITER, DONE } phase = IDLE;
  bool leave = false;     // finished its inner solve, waiting for the true-residual check
  bool in_graph = false;  // its group graph is a child of the current batch graph
  hdg_status status = HDG_OK;
  double work() const { return (double)P->N * nr; }
};

// queue the copy of a problem's scalar blocks to its pinned host buffer
void queue_scalars(hdg_problem* P, int nr) {
  HDG_CHECK(hipMemcpyAsync(P->hpin, P->s.sc, sizeof(double) * SC_COUNT * nr, hipMemcpyDeviceToHost, P->st));
}

// true residual of the item's iterate; returns false when its solve ended
// (converged, breakdown, or iteration limit): then its solution is copied out
bool batch_check(BatchItem& b, double tol, double rnorm2[64]) {
  hdg_problem* P = b.P;
  double rel = 0.0;
  for (int r = 0; r < b.nr; ++r) {
    const double v = std::sqrt(rnorm2[r]) / b.gn[r];
    if (!std::isfinite(v)) rel = v;
    if (std::isfinite(rel)) rel = std::max(rel, v);
  }
  b.o.relres = rel;
  b.o.outer += 1;
  if (!std::isfinite(rel) || rel <= tol || b.launched >= P->opts.max_it) {
    b.o.status = !std::isfinite(rel) ? HDG_ERR_BREAKDOWN : (rel <= tol ? HDG_OK : HDG_ERR_NOT_CONVERGED);
    blas_copy(b.lam_out + (long)b.i0 * P->N, P->lam, P->N, P->st, b.nr);
    b.phase = BatchItem::DONE;
    return false;
  }
  double r0[64];
  for (int r = 0; r < b.nr; ++r) r0[r] = std::sqrt(rnorm2[r]);
  pcg_start(P, b.mixed, b.nr);
  b.tr.init(b.nr, tol, b.gn);
  if (b.mixed) b.tr.init_inner(P->opts.refine_red, r0, b.launched);
  b.leave = false;
  b.phase = BatchItem::ITER;
  return true;
}

// `lanes` streams.  Each problem is dealt to one lane (largest first,
// round-robin) and runs all its work there: the eager starts and checks and
// its group graph, which sits in its lane's batch graph (the groups of a
// lane one after another).  One lane is one batch graph for the whole batch.
hdg_status solve_batch_graph(std::vector<BatchItem>& items, int rhs_kind, double tol,
                             const std::vector<hipStream_t>& lanes) {
  const int nb = (int)lanes.size();
  std::vector<int> lane(items.size(), 0);
  {
    std::vector<int> ord(items.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
      return (double)items[x].P->N * items[x].nrhs > (double)items[y].P->N * items[y].nrhs;
    });
    for (size_t j = 0; j < ord.size(); ++j) lane[ord[j]] = (int)(j % nb);
  }
  for (size_t i = 0; i < items.size(); ++i) items[i].P->st = lanes[lane[i]];
  auto sync_all = [&] {
    for (hipStream_t q : lanes) HDG_CHECK(hipStreamSynchronize(q));
  };
  std::vector<hipGraph_t> bg(nb, nullptr);
  std::vector<hipGraphExec_t> bx(nb, nullptr);
  std::vector<hipEvent_t> marks(nb, nullptr);
  for (auto& m : marks) HDG_CHECK(hipEventCreateWithFlags(&m, hipEventDisableTiming));
  auto drop_lane = [&](int q) {
    if (bx[q]) (void)hipGraphExecDestroy(bx[q]);
    if (bg[q]) (void)hipGraphDestroy(bg[q]);
    bx[q] = nullptr;
    bg[q] = nullptr;
    for (size_t i = 0; i < items.size(); ++i)
      if (lane[i] == q) items[i].in_graph = false;
  };
  auto drop_all = [&] {
    for (int q = 0; q < nb; ++q) drop_lane(q);
  };
  try {
    for (int round = 0;; ++round) {
      // right-hand-side groups of this round: group `round` of every problem that has one
      std::vector<int> act;
      for (size_t i = 0; i < items.size(); ++i) {
        BatchItem& b = items[i];
        b.i0 = round * b.P->cap;
        if (b.i0 >= b.nrhs) continue;
        b.nr = std::min(b.P->cap, b.nrhs - b.i0);
        act.push_back((int)i);
      }
      if (act.empty()) break;
      drop_all();
      // right-hand sides, initial guesses, ||g|| of every problem; one sync
      for (int i : act) {
        BatchItem* b = &items[i];
        hdg_problem* P = b->P;
        const long N = P->N, vs = P->nelem * P->nv;
        for (int r = 0; r < b->nr; ++r) {
          if (rhs_kind == HDG_RHS_TRACE)
            blas_copy(P->g + r * N, b->rhs + (long)(b->i0 + r) * N, N, P->st);
          else
            form_rhs(P, b->rhs + (long)(b->i0 + r) * vs, rhs_kind, nullptr, P->g + r * N);
        }
        blas_copy(P->lam, b->lam_out + (long)b->i0 * N, N, P->st, b->nr);
        blas_dot(P->g, P->g, N, P->s, FIN_GNORM, nullptr, P->st, b->nr);
        queue_scalars(P, b->nr);
      }
      sync_all();
      for (int i : act) {
        BatchItem* b = &items[i];
        b->mixed = b->P->opts.precision == HDG_MIXED;
        b->launched = 0;
        b->o = SolveOut();
        for (int r = 0; r < b->nr; ++r) {
          b->gn[r] = std::sqrt(b->P->hpin[(long)r * SC_COUNT + SC_GNORM2]);
          if (b->gn[r] == 0.0) {  // zero data: the solution is zero
            blas_fill<double>(b->P->lam + r * b->P->N, 0.0, b->P->N, b->P->st);
            b->gn[r] = 1.0;
          }
        }
        b->tr.init(b->nr, tol, b->gn);
        residual_norm(b->P, b->P->lam, b->P->g, b->mixed && !b->P->ops32, b->nr);
        queue_scalars(b->P, b->nr);
      }
      sync_all();
      for (int i : act) {
        BatchItem* b = &items[i];
        double rn[64];
        for (int r = 0; r < b->nr; ++r) rn[r] = b->P->hpin[(long)r * SC_COUNT + SC_RNORM2];
        batch_check(*b, tol, rn);
      }
      // iterate until every problem of the round is done.  Lanes advance on
      // their own: the host polls each lane's marker event and, when its
      // work has finished, scans its problems, runs the true-residual
      // checks it needs, and launches its next group.
      enum { L_IDLE, L_GROUP, L_CHECK, L_DONE };
      std::vector<int> lstate(nb, L_IDLE);
      std::vector<std::vector<BatchItem*>> lchk(nb);
      auto launch_lane = [&](int q) {
        double gwork = 0.0, idle = 0.0;
        bool iter = false, stale = false;
        for (int i : act) {
          if (lane[i] != q) continue;
          const BatchItem& b = items[i];
          if (b.phase == BatchItem::ITER) {
            iter = true;
            if (!b.in_graph) stale = true;
          }
          if (b.in_graph) {
            gwork += b.work();
            if (b.phase != BatchItem::ITER) idle += b.work();
          }
        }
        if (!iter) {
          drop_lane(q);
          lstate[q] = L_DONE;
          return;
        }
        if (stale || idle > BATCH_IDLE_FRAC * gwork) {
          drop_lane(q);
          HDG_CHECK(hipGraphCreate(&bg[q], 0));
          hipGraphNode_t tail = nullptr;
          for (int i : act) {
            BatchItem* b = &items[i];
            if (lane[i] != q || b->phase != BatchItem::ITER) continue;
            hdg_problem* P = b->P;
            if (b->nr != P->gnrhs) {
              drop_graphs(P);
              P->gnrhs = b->nr;
            }
            if (!P->grp_graph) {
              const bool mx = b->mixed;
              const int nr = b->nr;
              P->grp_graph = capture(P, [&] {
                reset_history(P, nr);
                for (int it = 0; it < CHECK_EVERY; ++it) pcg_iteration(P, P->lam, mx, nr);
              });
            }
            hipGraphNode_t node;
            HDG_CHECK(hipGraphAddChildGraphNode(&node, bg[q], tail ? &tail : nullptr, tail ? 1 : 0, P->grp_graph));
            tail = node;
            b->in_graph = true;
          }
          HDG_CHECK(hipGraphInstantiate(&bx[q], bg[q], nullptr, nullptr, 0));
        }
        HDG_CHECK(hipGraphLaunch(bx[q], lanes[q]));
        for (int i : act)
          if (lane[i] == q && items[i].in_graph) queue_scalars(items[i].P, items[i].nr);
        HDG_CHECK(hipEventRecord(marks[q], lanes[q]));
        lstate[q] = L_GROUP;
      };
      // a lane's group has finished: scan its problems; queue the checks
      // of those that finished their inner solve once they carry a quarter
      // of the lane's iterating work (or all of it)
      auto after_group = [&](int q) {
        double lwork = 0.0, iwork = 0.0;
        for (int i : act) {
          BatchItem* b = &items[i];
          if (lane[i] != q || !b->in_graph || b->phase != BatchItem::ITER) continue;
          double w = 0.0;
          const bool all = b->tr.scan(b->P->hpin, b->launched, CHECK_EVERY, &w);
          b->launched += CHECK_EVERY;
          if (b->tr.bad) {
            b->o.relres = std::numeric_limits<double>::quiet_NaN();
            b->o.status = HDG_ERR_BREAKDOWN;
            b->o.iters = b->launched;
            blas_copy(b->lam_out + (long)b->i0 * b->P->N, b->P->lam, b->P->N, b->P->st, b->nr);
            b->phase = BatchItem::DONE;
            continue;
          }
          if (!b->leave && (all || (b->mixed && b->tr.inner_done(b->launched)) || b->launched >= b->P->opts.max_it)) {
            b->leave = true;
            b->o.iters = all ? std::max(b->o.iters, b->tr.iters()) : b->launched;
          }
          iwork += b->work();
          if (b->leave) lwork += b->work();
        }
        lchk[q].clear();
        if (lwork > 0.0 && (lwork >= BATCH_CHECK_FRAC * iwork || lwork == iwork)) {
          for (int i : act)
            if (lane[i] == q && items[i].phase == BatchItem::ITER && items[i].leave) lchk[q].push_back(&items[i]);
          for (BatchItem* b : lchk[q]) {
            residual_norm(b->P, b->P->lam, b->P->g, b->mixed && !b->P->ops32, b->nr);
            queue_scalars(b->P, b->nr);
          }
          HDG_CHECK(hipEventRecord(marks[q], lanes[q]));
          lstate[q] = L_CHECK;
        } else {
          launch_lane(q);
        }
      };
      for (int q = 0; q < nb; ++q) launch_lane(q);
      for (;;) {
        bool busy = false;
        for (int q = 0; q < nb; ++q) {
          if (lstate[q] == L_DONE) continue;
          busy = true;
          const hipError_t e = hipEventQuery(marks[q]);
          if (e == hipErrorNotReady) continue;
          HDG_CHECK(e);
          if (lstate[q] == L_GROUP) {
            after_group(q);
          } else {  // L_CHECK
            for (BatchItem* b : lchk[q]) {
              double rn[64];
              for (int r = 0; r < b->nr; ++r) rn[r] = b->P->hpin[(long)r * SC_COUNT + SC_RNORM2];
              batch_check(*b, tol, rn);
            }
            launch_lane(q);
          }
        }
        if (!busy) break;
      }
      for (int i : act) {
        BatchItem* b = &items[i];
        if (b->info) {
          b->info->iters += b->o.iters;
          b->info->outer_iters += b->o.outer;
          b->info->relres = std::max(b->info->relres, b->o.relres);
        }
        if (b->o.status != HDG_OK && b->status == HDG_OK) b->status = b->o.status;
      }
    }
    sync_all();
  } catch (...) {
    drop_all();
    for (auto& m : marks) (void)hipEventDestroy(m);
    throw;
  }
  drop_all();
  for (auto& m : marks) (void)hipEventDestroy(m);
  hdg_status worst = HDG_OK;
  for (auto& b : items)
    if (b.status != HDG_OK && (worst == HDG_OK || b.status == HDG_ERR_DEVICE)) worst = b.status;
  return worst;
}

}  // namespace

hdg_status hdg_solve(hdg_handle P, const double* rhs, int rhs_kind, const double* gdir, int nrhs, double tol,
                     double* lambda, hdg_solve_info* info) {
  if (!P || !rhs || !lambda || nrhs < 1 || !(tol > 0.0)) return HDG_ERR_INVALID_ARG;
  if (rhs_kind < 0 || rhs_kind > 2) return HDG_ERR_INVALID_ARG;
  if (!P->built) return HDG_ERR_STATE;
  HDG_GUARD_BEGIN
  return solve_rhs_set(P, rhs, rhs_kind, gdir, nrhs, tol, lambda, info);
  HDG_GUARD_END
}

hdg_status hdg_solve_batch(int nprob, const hdg_handle* hs, const double* const* rhs, int rhs_kind,
                           const int* nrhs, double tol, double* const* lambda, hdg_solve_info* info,
                           int nstreams) {
  if (nprob < 1 || !hs || !rhs || !nrhs || !lambda || !(tol > 0.0)) return HDG_ERR_INVALID_ARG;
  // unstructured handles, and handles built with the persistent coarse
  // cycle (its workgroups must all be resident at once, which concurrent
  // problems on other streams would not guarantee)
  for (int i = 0; i < nprob; ++i)
    if (hs[i] && (hs[i]->unstructured || hs[i]->gtail_start[0] >= 0 || hs[i]->gtail_start[1] >= 0))
      return HDG_ERR_UNSUPPORTED;
  if (rhs_kind < 0 || rhs_kind > 2) return HDG_ERR_INVALID_ARG;
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i] || !rhs[i] || !lambda[i] || nrhs[i] < 1) return HDG_ERR_INVALID_ARG;
    if (!hs[i]->built) return HDG_ERR_STATE;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return HDG_ERR_INVALID_ARG;  // a handle is not thread-safe
  }
  bool graph_ok = true;
  for (int i = 0; i < nprob; ++i)
    if (hs[i]->opts.method != HDG_METHOD_PCG || !hs[i]->use_graphs || hs[i]->prof_on) graph_ok = false;
  if (nstreams <= 0 && graph_ok) {
    // one batch graph on a private stream, ordered after and before every handle's stream
    hipStream_t bst = nullptr;
    std::vector<hipStream_t> orig(nprob);
    for (int i = 0; i < nprob; ++i) orig[i] = hs[i]->st;
    std::vector<BatchItem> items(nprob);
    const int nlanes = std::min(std::max(1, -nstreams), 16);
    std::vector<hipStream_t> lanes(nlanes, nullptr);
    std::vector<hipEvent_t> join(nlanes, nullptr);
    hipEvent_t ev = nullptr, fork = nullptr;
    hdg_status res = HDG_OK;
    try {
      HDG_CHECK(hipStreamCreateWithFlags(&bst, hipStreamNonBlocking));
      HDG_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      HDG_CHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
      lanes[0] = bst;
      for (int q = 1; q < nlanes; ++q) HDG_CHECK(hipStreamCreateWithFlags(&lanes[q], hipStreamNonBlocking));
      for (int q = 0; q < nlanes; ++q) HDG_CHECK(hipEventCreateWithFlags(&join[q], hipEventDisableTiming));
      for (int i = 0; i < nprob; ++i) {
        HDG_CHECK(hipEventRecord(ev, orig[i]));
        HDG_CHECK(hipStreamWaitEvent(bst, ev, 0));
        BatchItem& b = items[i];
        b.P = hs[i];
        b.rhs = rhs[i];
        b.lam_out = lambda[i];
        b.nrhs = nrhs[i];
        b.info = info ? info + i : nullptr;
        if (b.info) {
          b.info->iters = 0;
          b.info->outer_iters = 0;
          b.info->relres = 0.0;
          b.info->t_solve_ms = 0.0;
          b.info->n_levels = (int)hs[i]->L.size();
          b.info->t_setup_ms = hs[i]->t_setup_ms;
          b.info->t_build_ms = hs[i]->t_build_ms;
        }
      }
      for (int q = 1; q < nlanes; ++q) {  // every lane starts after the handles' streams
        HDG_CHECK(hipEventRecord(fork, bst));
        HDG_CHECK(hipStreamWaitEvent(lanes[q], fork, 0));
      }
      hipEvent_t e0, e1;
      HDG_CHECK(hipEventCreate(&e0));
      HDG_CHECK(hipEventCreate(&e1));
      HDG_CHECK(hipEventRecord(e0, bst));
      res = solve_batch_graph(items, rhs_kind, tol, lanes);
      for (int q = 1; q < nlanes; ++q) {  // and the batch stream after every lane
        HDG_CHECK(hipEventRecord(join[q], lanes[q]));
        HDG_CHECK(hipStreamWaitEvent(bst, join[q], 0));
      }
      HDG_CHECK(hipEventRecord(e1, bst));
      HDG_CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      HDG_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (info)
        for (int i = 0; i < nprob; ++i) info[i].t_solve_ms = ms;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      HDG_CHECK(hipEventRecord(ev, bst));
      for (int i = 0; i < nprob; ++i) {
        hs[i]->st = orig[i];
        HDG_CHECK(hipStreamWaitEvent(orig[i], ev, 0));
      }
    } catch (const HipError& e) {
      for (int i = 0; i < nprob; ++i) hs[i]->st = orig[i];
      res = map_error(e);
    } catch (const std::bad_alloc&) {
      for (int i = 0; i < nprob; ++i) hs[i]->st = orig[i];
      res = HDG_ERR_DEVICE;
    }
    for (int q = 1; q < nlanes; ++q)
      if (lanes[q]) {
        (void)hipStreamSynchronize(lanes[q]);
        (void)hipStreamDestroy(lanes[q]);
      }
    if (bst) {
      (void)hipStreamSynchronize(bst);
      (void)hipStreamDestroy(bst);
    }
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (ev) (void)hipEventDestroy(ev);
    return res;
  }
  if (nstreams <= 0) nstreams = 4;
  nstreams = std::min(std::min(nstreams, 16), nprob);
  std::vector<hipStream_t> ws(nstreams, nullptr);
  std::vector<hdg_status> st(nprob, HDG_OK);
  try {
    for (auto& w : ws) HDG_CHECK(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
  } catch (const HipError& e) {
    for (auto& w : ws)
      if (w) (void)hipStreamDestroy(w);
    return map_error(e);
  }
  std::atomic<int> next{0};
  auto worker = [&](int t) {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= nprob) return;
      hdg_problem* P = hs[i];
      hipStream_t orig = P->st;
      hipEvent_t ev = nullptr;
      try {
        // order after the work already queued on the handle's stream, run on
        // the worker's stream, then order the handle's stream after it
        HDG_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HDG_CHECK(hipEventRecord(ev, orig));
        HDG_CHECK(hipStreamWaitEvent(ws[t], ev, 0));
        P->st = ws[t];
        st[i] = solve_rhs_set(P, rhs[i], rhs_kind, nullptr, nrhs[i], tol, lambda[i], info ? info + i : nullptr);
        HDG_CHECK(hipEventRecord(ev, ws[t]));
        P->st = orig;
        HDG_CHECK(hipStreamWaitEvent(orig, ev, 0));
      } catch (const HipError& e) {
        P->st = orig;
        st[i] = map_error(e);
      } catch (const std::bad_alloc&) {
        P->st = orig;
        st[i] = HDG_ERR_DEVICE;
      }
      if (ev) (void)hipEventDestroy(ev);
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nstreams; ++t) th.emplace_back(worker, t);
  for (auto& t : th) t.join();
  for (auto& w : ws) {
    (void)hipStreamSynchronize(w);
    (void)hipStreamDestroy(w);
  }
  hdg_status worst = HDG_OK;
  for (int i = 0; i < nprob; ++i)
    if (st[i] != HDG_OK && (worst == HDG_OK || st[i] == HDG_ERR_DEVICE)) worst = st[i];
  return worst;
}

hdg_status hdg_autotune(hdg_handle P, const hdg_mg_opts* base, int nrhs, hdg_mg_opts* best, double* us_per_rhs_it) {
  if (!P || !best || nrhs < 1 || nrhs > HDG_MAX_NRHS) return HDG_ERR_INVALID_ARG;
  if (P->unstructured) return HDG_ERR_UNSUPPORTED;
  hdg_mg_opts b0;
  if (base)
    b0 = *base;
  else
    hdg_default_opts(&b0);
  HDG_GUARD_BEGIN
  // candidates: coarsest macro grid x right-hand-side group size; scored by
  // the stream time of a fixed number of outer iterations per right-hand side
  const int coarse[3] = {2, 8, 16};
  const int groups[7] = {1, 2, 4, 8, 16, 32, 64};
  constexpr int ITS = 6;
  double best_us = 0.0;
  hdg_mg_opts bo = b0;
  bool have = false;
  hipEvent_t e0, e1;
  HDG_CHECK(hipEventCreate(&e0));
  HDG_CHECK(hipEventCreate(&e1));
  for (int ci = 0; ci < 3; ++ci) {
    if (ci > 0 && coarse[ci] >= P->n) continue;  // same hierarchy as a smaller candidate
    for (int gi = 0; gi < 7; ++gi) {
      const int g = groups[gi];
      if (g > nrhs) break;
      hdg_mg_opts o = b0;
      o.coarse_n = coarse[ci];
      o.nrhs = g;
      o.max_it = ITS;
      const hdg_status sb = hdg_mg_build(P, &o);
      if (sb != HDG_OK) continue;
      const long N = P->N;
      if (N == 0) continue;
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {  // the first run captures the graphs
        blas_fill<double>(P->g, 1.0, N, P->st, g);
        blas_fill<double>(P->lam, 0.0, N, P->st, g);
        HDG_CHECK(hipEventRecord(e0, P->st));
        (void)solve_many(P, g, 1e-300, nullptr);
        HDG_CHECK(hipEventRecord(e1, P->st));
        HDG_CHECK(hipEventSynchronize(e1));
        HDG_CHECK(hipEventElapsedTime(&ms, e0, e1));
      }
      const double us = 1e3 * ms / ((double)ITS * g);
      if (!have || us < best_us) {
        best_us = us;
        bo = o;
        have = true;
      }
    }
  }
  // then the tile shapes of the work on top of the best layout: lanes per
  // macro-element of the transition kernels, and the finest level's strip
  // apply against its two-phase form
  if (have) {
    const int shapes[3] = {HDG_VARIANT_LANES1, HDG_VARIANT_LANES4, HDG_VARIANT_NO_STRIP};
    const hdg_mg_opts best0 = bo;
    for (int si = 0; si < 3; ++si) {
      hdg_mg_opts o = best0;
      o.variant = best0.variant | shapes[si];
      o.max_it = ITS;
      if (hdg_mg_build(P, &o) != HDG_OK || P->N == 0) continue;
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        blas_fill<double>(P->g, 1.0, P->N, P->st, o.nrhs);
        blas_fill<double>(P->lam, 0.0, P->N, P->st, o.nrhs);
        HDG_CHECK(hipEventRecord(e0, P->st));
        (void)solve_many(P, o.nrhs, 1e-300, nullptr);
        HDG_CHECK(hipEventRecord(e1, P->st));
        HDG_CHECK(hipEventSynchronize(e1));
        HDG_CHECK(hipEventElapsedTime(&ms, e0, e1));
      }
      const double us = 1e3 * ms / ((double)ITS * o.nrhs);
      if (us < best_us) {
        best_us = us;
        bo = o;
      }
    }
  }
  HDG_CHECK(hipEventDestroy(e0));
  HDG_CHECK(hipEventDestroy(e1));
  if (!have) return HDG_ERR_UNSUPPORTED;
  bo.max_it = b0.max_it;
  *best = bo;
  if (us_per_rhs_it) *us_per_rhs_it = best_us;
  return hdg_mg_build(P, &bo);
  HDG_GUARD_END
}

hdg_status hdg_reconstruct(hdg_handle P, const double* lambda, const double* rhs, int rhs_kind,
                           const double* gdir, double* u, double* q) {
  if (!P || !lambda || !rhs || !u || !q) return HDG_ERR_INVALID_ARG;
  if (rhs_kind != HDG_RHS_F_NODAL && rhs_kind != HDG_RHS_F_LOAD) return HDG_ERR_INVALID_ARG;
  if (P->unstructured) {
    if (rhs_kind != HDG_RHS_F_NODAL) return HDG_ERR_UNSUPPORTED;
    HDG_GUARD_BEGIN
    launch_tri_reconstruct(P->k, P->nelem, P->ul[0].sface, P->utbnd, P->urec, lambda, gdir, rhs, u, q, P->st);
    return HDG_OK;
    HDG_GUARD_END
  }
  if (!P->store_recovery) return HDG_ERR_STATE;
  HDG_GUARD_BEGIN
  if (P->scheme == HDG_SCHEME_HDG)
    launch_reconstruct(P->d, P->k, P->n, P->tau, P->tau_kappa, P->rd, P->kqp, lambda, gdir, rhs, rhs_kind == HDG_RHS_F_LOAD ? 1 : 0,
                       P->W, P->Kinv, P->Minv, P->ework, u, q, P->st);
  else
    launch_ipdg_reconstruct(P->d, P->k, P->n, P->rd, P->kqp, P->nq, P->emask, HDG_SCHEME_RT, P->Xq, P->Yq, lambda, gdir,
                            rhs, rhs_kind == HDG_RHS_F_LOAD ? 1 : 0, P->Xr, P->Kinv, P->ework, u, q, P->st);
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_adjoint(hdg_handle P, const double* dJdu, const double* q_fwd, double tol, double* grad,
                       hdg_solve_info* info) {
  if (!P || !dJdu || !q_fwd || !grad || !(tol > 0.0)) return HDG_ERR_INVALID_ARG;
  if (P->scheme != HDG_SCHEME_HDG || P->tau_kappa || P->unstructured) return HDG_ERR_UNSUPPORTED;
  if (!P->built || !P->store_recovery) return HDG_ERR_STATE;
  HDG_GUARD_BEGIN
  if (!P->ustar) {
    P->ustar = dalloc<double>(P, P->nelem * P->nv, false);
    P->qstar = dalloc<double>(P, P->nelem * P->d * P->nv, false);
  }
  if (info) {
    info->iters = 0;
    info->outer_iters = 0;
    info->relres = 0.0;
    info->t_solve_ms = 0.0;
    info->n_levels = (int)P->L.size();
    info->t_setup_ms = P->t_setup_ms;
    info->t_build_ms = P->t_build_ms;
  }
  form_rhs(P, dJdu, HDG_RHS_F_LOAD, nullptr, P->g);
  blas_fill<double>(P->lam, 0.0, P->N, P->st);
  hdg_status s = solve_one(P, P->g, P->lam, tol, info);
  launch_reconstruct(P->d, P->k, P->n, P->tau, 0, P->rd, P->kqp, P->lam, nullptr, dJdu, 1, P->W, P->Kinv, P->Minv, P->ework,
                     P->ustar, P->qstar, P->st);
  launch_grad(P->d, P->k, P->nelem, P->rd, P->kqp, q_fwd, P->qstar, grad, P->st);
  HDG_CHECK(hipStreamSynchronize(P->st));
  return s;
  HDG_GUARD_END
}

hdg_status hdg_mass_apply(hdg_handle P, const double* u, double* out) {
  if (!P || !u || !out) return HDG_ERR_INVALID_ARG;
  if (P->unstructured) return HDG_ERR_UNSUPPORTED;
  HDG_GUARD_BEGIN
  launch_mass(P->d, P->k, P->nelem, P->rd, u, out, P->st);
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_level_apply(hdg_handle P, int level, const void* x, void* y, int precision) {
  if (!P || !x || !y) return HDG_ERR_INVALID_ARG;
  if (!P->built) return HDG_ERR_STATE;
  if (level < 0 || level >= (int)P->L.size()) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  const Level& L = P->L[level];
  if (precision == HDG_FP64)
    launch_apply<double>(L, APPLY_Y, (const double*)x, nullptr, (double*)y, nullptr, nullptr, P->st);
  else if (precision == HDG_FP32)
    launch_apply<float>(L, APPLY_Y, (const float*)x, nullptr, (float*)y, nullptr, nullptr, P->st);
  else
    return HDG_ERR_INVALID_ARG;
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_level_smooth(hdg_handle P, int level, const void* r, void* e, int sweeps, int precision) {
  if (!P || !r || !e || sweeps < 0) return HDG_ERR_INVALID_ARG;
  if (!P->built) return HDG_ERR_STATE;
  if (level < 0 || level >= (int)P->L.size()) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  Level& L = P->L[level];
  if (P->opts.smoother == HDG_SMOOTHER_CHEBYSHEV && sweeps != L.sweeps && L.nface > 0) return HDG_ERR_INVALID_ARG;
  auto run = [&](auto tag) {
    using T = decltype(tag);
    const int pr = sizeof(T) == 8 ? 0 : 1;
    T* a = (T*)L.e[pr];
    T* b = (T*)L.w[pr];
    if (sweeps == 0) {
      blas_fill<T>((T*)e, T(0), L.nlam, P->st);
      return;
    }
    if (P->opts.smoother == HDG_SMOOTHER_LUSGS) {
      blas_fill<T>(a, T(0), L.nlam, P->st);
      sgs_steps<T, T>(L, a, (const T*)r, sweeps, P->st, 1);
    } else {
      cheb_select(L, 0);
      launch_jacobi0<T>(L, (const T*)r, a, P->st);
      for (int s = 1; s < sweeps; ++s) {
        cheb_select(L, s);
        launch_apply<T>(L, APPLY_SWEEP, a, (const T*)r, b, nullptr, nullptr, P->st);
        std::swap(a, b);
      }
    }
    HDG_CHECK(hipMemcpyAsync(e, a, sizeof(T) * L.nlam, hipMemcpyDeviceToDevice, P->st));
  };
  if (precision == HDG_FP64)
    run(double(0));
  else if (precision == HDG_FP32)
    run(float(0));
  else
    return HDG_ERR_INVALID_ARG;
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_level_export(hdg_handle P, int level, double* out) {
  if (!P || !out) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  if (level == 0) {
    HDG_CHECK(hipMemcpyAsync(out, P->Ae, sizeof(double) * P->nelem * P->nl * P->nl, hipMemcpyDeviceToDevice,
                             P->st));
    return HDG_OK;
  }
  if (!P->built) return HDG_ERR_STATE;
  if (level < 0 || level >= (int)P->L.size()) return HDG_ERR_INVALID_ARG;
  const Level& L = P->L[level];
  if (L.u && !L.u->tri) return HDG_ERR_UNSUPPORTED;  // macro-element maps of varying size
  HDG_CHECK(hipMemcpyAsync(out, L.Aelem, sizeof(double) * L.nelem * L.nl * L.nl, hipMemcpyDeviceToDevice, P->st));
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_profile_begin(hdg_handle P) {
  if (!P) return HDG_ERR_INVALID_ARG;
  HDG_GUARD_BEGIN
  HDG_CHECK(hipStreamSynchronize(P->st));
  harvest(P);
  for (int i = 0; i < hdg_problem::NPROF; ++i) {
    P->prof_ms[i] = 0.0;
    P->prof_n[i] = 0;
  }
  P->prof_on = true;
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_profile_read(hdg_handle P, int kernel, long long* launches, double* total_ms,
                            double* bytes_per_launch) {
  if (!P || kernel < 0 || kernel >= hdg_problem::NPROF) return HDG_ERR_INVALID_ARG;
  if (!P->built) return HDG_ERR_STATE;
  HDG_GUARD_BEGIN
  HDG_CHECK(hipStreamSynchronize(P->st));
  harvest(P);
  if (kernel >= hdg_problem::NPROF_XFER) {
    // algorithmic bytes of the transfer kernels: every operator block and
    // vector entry the kernel must touch, once
    const int kind = (kernel - hdg_problem::NPROF_XFER) / 2;
    const double s = ((kernel - hdg_problem::NPROF_XFER) % 2) ? 4.0 : 8.0;
    double bytes = 0.0;
    const int fh = first_h(P);
    if (kind == 3) {  // e += J_N e_c on the finest level: e_c read, e read and written
      const Level& L0 = P->L[0];
      bytes = (double)L0.nface * ((1 << (L0.d - 1)) + 2.0 * L0.ne) * s;
    } else if (fh >= 0) {
      const Level& L = P->L[fh];
      const Level& C = P->L[fh + 1];
      const double nc = 1 << (L.d - 1), nif = L.d * nc, nbf = 2 * L.d * nc;
      const double ni = L.nI, ncl = L.ncl, nl = L.nl;
      const double rows = nif * 2.0 * nl * nc;  // the interior faces' rows of both children
      const bool lpost = (P->opts.local_corr & HDG_LC_POST) != 0;
      if (kind == 0)  // hpre: residual on I, A_II^-1, restriction block; e, r, e_I, cb
        bytes = (double)L.nmacro * ((rows + ni * ni + ni * ncl) * s + ((nif + nbf) * nc + 3.0 * ni + ncl) * s);
      else if (kind == 1)  // hsum: r on the sub-faces, two shares, coarse block inverse, rc and ec
        bytes = (double)C.nface * ((nc * nc + 2.0 * nc + 2.0 * nc) * s + nc * nc * s);
      else  // hpost: e_c, P, e_I (and the post correction), the sub-face prolongation
        bytes = (double)L.nmacro * ((ncl + ni * ncl + 2.0 * ni) * s +
                                    (lpost ? (rows + ni * ni) * s + ((nif + nbf) * nc + ni) * s : 0.0)) +
                (double)C.nface * (nc + 2.0 * nc * nc) * s;
    }
    if (launches) *launches = P->prof_n[kernel];
    if (total_ms) *total_ms = P->prof_ms[kernel];
    if (bytes_per_launch) *bytes_per_launch = bytes;
    return HDG_OK;
  }
  const Level& L = P->L[0];
  const bool f32ops = kernel >= hdg_problem::NPROF_F32OPS;  // FP32 blocks, FP64 vectors
  const int mode = f32ops ? kernel - hdg_problem::NPROF_F32OPS : kernel / 2;
  const double sm = f32ops ? 4.0 : ((kernel % 2) ? 4.0 : 8.0);  // bytes per stored operator entry
  const double s = f32ops ? 8.0 : sm;                             // bytes per vector entry
  const double N = (double)L.nlam;
  // operator bytes: each element row once (face-major), the packed upper
  // triangle of each element map (element-major), or every triangle's whole
  // map (unstructured: both phases of the apply)
  double bytes = L.u ? (double)L.nelem * L.nl * L.nl * sm
                     : L.packed ? (double)L.nelem * (L.nl * (L.nl + 1) / 2) * sm
                                : (double)L.nface * 2.0 * L.ne * L.nl * sm;
  if (mode == APPLY_Y) bytes += 2.0 * N * s;
  if (mode == APPLY_RES) bytes += 3.0 * N * s;
  // face-block inverses: full blocks, or upper triangles on element-major levels
  const double nd = L.packed ? L.ne * (L.ne + 1) / 2 : L.ne * L.ne;
  if (mode == APPLY_SWEEP) bytes += (double)L.nface * nd * sm + 3.0 * N * s;
  if (mode == APPLY_SWEEP_DOT) bytes += (double)L.nface * nd * sm + 3.0 * N * s + 8.0 * N;  // + r (FP64)
  if (mode == APPLY_RES_PRESTRICT) bytes += 2.0 * N * s + (double)L.nface * (1 << (L.d - 1)) * s;
  if (launches) *launches = P->prof_n[kernel];
  if (total_ms) *total_ms = P->prof_ms[kernel];
  if (bytes_per_launch) *bytes_per_launch = bytes;
  return HDG_OK;
  HDG_GUARD_END
}

hdg_status hdg_query(hdg_handle P, int what, long long* out) {
  if (!P || !out) return HDG_ERR_INVALID_ARG;
  const int nL = (int)P->L.size();
  if (what == HDG_Q_NT) {
    *out = P->nelem;
  } else if (what == HDG_Q_NLAMBDA && P->unstructured) {
    *out = P->ul[0].nface * P->ul[0].m;
  } else if (what == HDG_Q_NLAMBDA) {
    Level tmp;
    init_level(tmp, P->d, P->n, P->ne);
    *out = tmp.nlam;
  } else if (what == HDG_Q_NLEVELS) {
    *out = nL;
  } else if (what == HDG_Q_NV) {
    *out = P->nv;
  } else if (what == HDG_Q_NQ) {
    *out = P->nq;
  } else if (what == HDG_Q_DEVICE_BYTES) {
    *out = P->bytes;
  } else if (what == HDG_Q_GRID_TAIL) {
    *out = P->gtail_start[0];
  } else if (what >= HDG_Q_LEVEL_NLAMBDA && what < HDG_Q_LEVEL_NLAMBDA + 100) {
    int l = what - HDG_Q_LEVEL_NLAMBDA;
    if (l >= nL) return HDG_ERR_INVALID_ARG;
    *out = P->L[l].nlam;
  } else if (what >= HDG_Q_LEVEL_N && what < HDG_Q_LEVEL_N + 100) {
    int l = what - HDG_Q_LEVEL_N;
    if (l >= nL) return HDG_ERR_INVALID_ARG;
    *out = P->L[l].n;
  } else if (what >= HDG_Q_LEVEL_NE && what < HDG_Q_LEVEL_NE + 100) {
    int l = what - HDG_Q_LEVEL_NE;
    if (l >= nL) return HDG_ERR_INVALID_ARG;
    *out = P->L[l].ne;
  } else {
    return HDG_ERR_INVALID_ARG;
  }
  return HDG_OK;
}

hdg_status hdg_destroy(hdg_handle P) {
  if (!P) return HDG_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(P->st);
  drop_graphs(P);
  if (P->cap_st) (void)hipStreamDestroy(P->cap_st);
  for (void* ptr : P->build_allocs) (void)hipFree(ptr);
  for (void* ptr : P->allocs) (void)hipFree(ptr);
  for (auto& pd : P->pending) {
    (void)hipEventDestroy(pd.a);
    (void)hipEventDestroy(pd.b);
  }
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  if (P->hbad) (void)hipHostFree(P->hbad);
  if (P->hpin) (void)hipHostFree(P->hpin);
  delete P;
  return HDG_OK;
}

}  // extern "C"
