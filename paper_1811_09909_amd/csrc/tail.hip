// Coarse tail of the V-cycle in one workgroup (gfx950, 2D).
//
// Below a few thousand trace unknowns every level of Algorithm 1 is a handful
// of tiny launches whose fixed cost (a few microseconds each) dwarfs their
// work.  This kernel runs the whole remaining cycle -- smoothing, local
// corrections, restrictions, the coarsest direct solve, prolongations --
// from one level down in a single workgroup: the residual, correction and
// scratch vectors of every tail level live in LDS, the level operators are
// read through the caches, and phases are separated by workgroup barriers.
// Each step is the same per-face / per-macro-element work item the grid
// kernels use, so results match them up to rounding order.
#include "hdg_internal.hpp"
#include "trace_dev.hpp"

namespace hdg {

namespace {

using namespace dev;

constexpr int TAIL_THREADS = 512;

template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS) tail_kernel(TailArgs a) {
  __shared__ __align__(16) unsigned char arena_raw[TAIL_ARENA_BYTES];
  T* arena = reinterpret_cast<T*>(arena_raw);
  constexpr int D = 2, NC = 2;
  const int tid = threadIdx.x, nt = TAIL_THREADS;
  const TailLevel& L0 = a.lev[0];
  T* r0 = arena + L0.off_r;
  T* e0 = arena + L0.off_e;
  // one workgroup per right-hand side (stored one after another)
  const long roff = blockIdx.y * L0.nlam;
  for (long i = tid; i < L0.nlam; i += nt) {
    r0[i] = reinterpret_cast<const T*>(a.rin)[roff + i];
    if (a.pre_done) e0[i] = reinterpret_cast<const T*>(a.ein)[roff + i];
  }
  __syncthreads();
  if (!a.pre_done) {
    const T* Dv = reinterpret_cast<const T*>(L0.Dinv);
    for (long F = tid; F < L0.nface; F += nt) jacobi0_item<NC, T>(F, Dv, r0, e0);
    __syncthreads();
  }
  int cur[TAIL_MAX_LEVELS];
  // restriction side of the cycle
  for (int l = 0; l + 1 < a.nlev; ++l) {
    const TailLevel& L = a.lev[l];
    const TailLevel& C = a.lev[l + 1];
    T* r = arena + L.off_r;
    T* eb[2] = {arena + L.off_e, arena + L.off_w};
    T* cb = arena + L.off_cb;
    const T* Af = reinterpret_cast<const T*>(L.Af);
    const T* Dv = reinterpret_cast<const T*>(L.Dinv);
    const T* Ai = reinterpret_cast<const T*>(L.AIIinv);
    const T* Pm = reinterpret_cast<const T*>(L.P);
    int c = 0;
    for (int s = 1; s < L.sweeps; ++s) {
      for (long F = tid; F < L.nface; F += nt) face_item<D, NC, T, APPLY_SWEEP>(F, L.n, Af, Dv, eb[c], r, eb[1 - c]);
      __syncthreads();
      c = 1 - c;
    }
    for (long M = tid; M < L.nmacro; M += nt) hpre_item<D, T>(M, L.n, Af, Ai, Pm, r, eb[c], a.lc & HDG_LC_PRE, cb);
    __syncthreads();
    T* rc = arena + C.off_r;
    T* ec = arena + C.off_e;
    if (C.kind == 2) {
      for (long F = tid; F < C.nface; F += nt) hsum_item<D, T>(F, L.n, r, cb, nullptr, rc, nullptr);
      __syncthreads();
      const T* Ainv = reinterpret_cast<const T*>(C.Ainv);
      const int N = (int)C.nlam;
      for (int i = tid; i < N; i += nt) {
        acc_t<T> sacc = 0;
        for (int j = 0; j < N; ++j) sacc += acc_t<T>(Ainv[i * N + j]) * rc[j];
        ec[i] = T(sacc);
      }
    } else {
      const T* Dc = reinterpret_cast<const T*>(C.Dinv);
      for (long F = tid; F < C.nface; F += nt) hsum_item<D, T>(F, L.n, r, cb, Dc, rc, ec);
    }
    __syncthreads();
    cur[l] = c;
  }
  cur[a.nlev - 1] = 0;
  // prolongation side
  for (int l = a.nlev - 2; l >= 0; --l) {
    const TailLevel& L = a.lev[l];
    const TailLevel& C = a.lev[l + 1];
    T* r = arena + L.off_r;
    T* eb[2] = {arena + L.off_e, arena + L.off_w};
    const T* Af = reinterpret_cast<const T*>(L.Af);
    const T* Dv = reinterpret_cast<const T*>(L.Dinv);
    const T* Ai = reinterpret_cast<const T*>(L.AIIinv);
    const T* Pm = reinterpret_cast<const T*>(L.P);
    const T* ec = arena + (cur[l + 1] == 0 ? C.off_e : C.off_w);
    int c = cur[l];
    for (long M = tid; M < L.nmacro; M += nt)
      hpost_m_item<D, T>(M, L.n, Af, Ai, Pm, r, ec, eb[c], eb[1 - c], a.lc & HDG_LC_POST);
    for (long F = tid; F < C.nface; F += nt) hpost_f_item<D, T>(F, L.n, ec, eb[c], eb[1 - c]);
    __syncthreads();
    c = 1 - c;
    for (int s = 0; s < L.sweeps; ++s) {
      for (long F = tid; F < L.nface; F += nt) face_item<D, NC, T, APPLY_SWEEP>(F, L.n, Af, Dv, eb[c], r, eb[1 - c]);
      __syncthreads();
      c = 1 - c;
    }
    cur[l] = c;
  }
  const T* res = arena + (cur[0] == 0 ? L0.off_e : L0.off_w);
  for (long i = tid; i < L0.nlam; i += nt) reinterpret_cast<T*>(a.eout)[roff + i] = res[i];
}

}  // namespace

template <typename T>
void launch_tail(const TailArgs& a, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL((tail_kernel<T>), dim3(1, nrhs), dim3(TAIL_THREADS), 0, st, a);
  HDG_CHECK(hipGetLastError());
}
template void launch_tail<double>(const TailArgs&, hipStream_t, int);
template void launch_tail<float>(const TailArgs&, hipStream_t, int);

}  // namespace hdg
