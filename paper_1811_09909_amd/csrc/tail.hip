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

// Grid-wide barrier of the persistent coarse cycle.  Thread 0 of every
// workgroup publishes the workgroup's writes (agent-scope release: the
// per-XCD L2s are written back), arrives on the counter, and waits for the
// generation to move; the last arrival resets the counter and moves it.
// The wait is bounded: after GTAIL_SPIN_MAX polls the error flag is set and
// the workgroup goes on, so every launch ends; the host reports the flag.
constexpr unsigned GTAIL_SPIN_MAX = 1u << 14;  // well under a second per launch even if every wait ran out

__device__ inline void grid_barrier(unsigned* sync, unsigned nblocks, unsigned& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned arrived = __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&sync[32], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned polls = 0;
      while (__hip_atomic_load(&sync[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (++polls > GTAIL_SPIN_MAX) {
          __hip_atomic_store(&sync[64], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();
  }
  ++gen;
  __syncthreads();
}

// the pre-coarse macro-element work of one level (lpm lanes per
// macro-element, as the per-level kernel of that level runs it)
template <typename T>
__device__ inline void gt_hpre(const GTailLevel& L, long gt, long gs, const T* r, T* e, int corr) {
  const T* Af = (const T*)L.Af;
  const T* Ai = (const T*)L.AIIinv;
  const T* R = (const T*)L.R;
  T* cb = (T*)L.cb;
  if (L.lpm == 4) {
    for (long t = gt; t < 4 * L.nmacro; t += gs) hpreL_item<T, 4>(t / 4, (int)(t % 4), L.n, Af, Ai, R, r, e, corr, cb);
  } else if (L.lpm == 2) {
    for (long t = gt; t < 2 * L.nmacro; t += gs) hpreL_item<T, 2>(t / 2, (int)(t % 2), L.n, Af, Ai, R, r, e, corr, cb);
  } else {
    for (long M = gt; M < L.nmacro; M += gs) hpre_item<2, T>(M, L.n, Af, Ai, R, r, e, corr, cb);
  }
}

template <typename T>
__device__ inline void gt_hpost(const GTailLevel& L, const GTailLevel& C, long gt, long gs, const T* r, const T* ec,
                                const T* eold, T* enew, int corr) {
  const T* Af = (const T*)L.Af;
  const T* Ai = (const T*)L.AIIinv;
  const T* Pm = (const T*)L.P;
  if (L.lpm == 4) {
    for (long t = gt; t < 4 * L.nmacro; t += gs)
      hpostL_m_item<T, 4>(t / 4, (int)(t % 4), L.n, Af, Ai, Pm, r, ec, eold, enew, corr);
  } else if (L.lpm == 2) {
    for (long t = gt; t < 2 * L.nmacro; t += gs)
      hpostL_m_item<T, 2>(t / 2, (int)(t % 2), L.n, Af, Ai, Pm, r, ec, eold, enew, corr);
  } else {
    for (long M = gt; M < L.nmacro; M += gs) hpost_m_item<2, T>(M, L.n, Af, Ai, Pm, r, ec, eold, enew, corr);
  }
  for (long F = gt; F < C.nface; F += gs) hpost_f_item<2, T>(F, L.n, ec, eold, enew);
}

// The V-cycle from level lev[0] (its first block-Jacobi step already in
// lev[0].e, as the transition above leaves it) down to the coarsest and back;
// the result ends in lev[0].e (2 m buffer swaps per level).
template <typename T>
__global__ void __launch_bounds__(GTAIL_THREADS) gtail_kernel(GTailArgs a) {
  constexpr int D = 2, NC = 2;
  const long gt = (long)blockIdx.x * GTAIL_THREADS + threadIdx.x;
  const long gs = (long)gridDim.x * GTAIL_THREADS;
  const unsigned nb = gridDim.x;
  __shared__ unsigned gen0;
  if (threadIdx.x == 0) gen0 = __hip_atomic_load(&a.sync[32], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned gen = gen0;
  // restriction side; the pre-smoothing leaves level l's iterate in e when
  // its sweep count m is odd (m - 1 swaps), in w otherwise
  for (int l = 0; l + 1 < a.nlev; ++l) {
    const GTailLevel L = a.lev[l];
    const GTailLevel C = a.lev[l + 1];
    const T* r = (const T*)L.r;
    T* e = (T*)L.e;
    T* w = (T*)L.w;
    const T* Af = (const T*)L.Af;
    const T* Dv = (const T*)L.Dinv;
    for (int s = 1; s < L.sweeps; ++s) {
      for (long F = gt; F < L.nface; F += gs) face_item<D, NC, T, APPLY_SWEEP>(F, L.n, Af, Dv, e, r, w);
      grid_barrier(a.sync, nb, gen);
      T* t = e;
      e = w;
      w = t;
    }
    gt_hpre<T>(L, gt, gs, r, e, a.lc & HDG_LC_PRE);
    grid_barrier(a.sync, nb, gen);
    const T* cb = (const T*)L.cb;
    if (C.kind == 2) {
      T* rc = (T*)C.r;
      for (long F = gt; F < C.nface; F += gs) hsum_item<D, T>(F, L.n, r, cb, nullptr, rc, nullptr);
      grid_barrier(a.sync, nb, gen);
      // e_c = A_c^-1 r_c: one wavefront per row, lanes strided over the
      // columns, FP64 sums reduced down the wavefront
      const int N = (int)C.nlam;
      const T* Ainv = (const T*)C.Ainv;
      T* ec = (T*)C.e;
      const int lane = threadIdx.x & 63;
      for (long row = gt >> 6; row < N; row += gs >> 6) {
        double sacc = 0.0;
        for (int j = lane; j < N; j += 64) sacc += (double)Ainv[row * N + j] * (double)rc[j];
        for (int o = 32; o > 0; o >>= 1) sacc += __shfl_down(sacc, o, 64);
        if (lane == 0) ec[row] = (T)sacc;
      }
    } else {
      for (long F = gt; F < C.nface; F += gs)
        hsum_item<D, T>(F, L.n, r, cb, (const T*)C.Dinv, (T*)C.r, (T*)C.e);
    }
    grid_barrier(a.sync, nb, gen);
  }
  // prolongation side: the coarse correction ec, then e + I ec (with the
  // local correction) into the other buffer and m post-sweeps; 2 m swaps in
  // all, so each level's result ends in its e
  const T* ec = (const T*)a.lev[a.nlev - 1].e;
  for (int l = a.nlev - 2; l >= 0; --l) {
    const GTailLevel L = a.lev[l];
    const GTailLevel C = a.lev[l + 1];
    const T* r = (const T*)L.r;
    const bool odd = (L.sweeps - 1) & 1;
    T* e = odd ? (T*)L.w : (T*)L.e;
    T* w = odd ? (T*)L.e : (T*)L.w;
    gt_hpost<T>(L, C, gt, gs, r, ec, e, w, a.lc & HDG_LC_POST);
    grid_barrier(a.sync, nb, gen);
    {
      T* t = e;
      e = w;
      w = t;
    }
    const T* Af = (const T*)L.Af;
    const T* Dv = (const T*)L.Dinv;
    for (int s = 0; s < L.sweeps; ++s) {
      for (long F = gt; F < L.nface; F += gs) face_item<D, NC, T, APPLY_SWEEP>(F, L.n, Af, Dv, e, r, w);
      if (l > 0 || s + 1 < L.sweeps) grid_barrier(a.sync, nb, gen);
      T* t = e;
      e = w;
      w = t;
    }
    ec = e;
  }
}

}  // namespace

template <typename T>
void launch_tail(const TailArgs& a, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL((tail_kernel<T>), dim3(1, nrhs), dim3(TAIL_THREADS), 0, st, a);
  HDG_CHECK(hipGetLastError());
}
template void launch_tail<double>(const TailArgs&, hipStream_t, int);
template void launch_tail<float>(const TailArgs&, hipStream_t, int);

template <typename T>
int gtail_grid() {
  int dev = 0, ncu = 0, per_cu = 0;
  HDG_CHECK(hipGetDevice(&dev));
  HDG_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HDG_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gtail_kernel<T>, GTAIL_THREADS, 0));
  // half as many workgroups as compute units: at this kernel's register count
  // one workgroup fills a compute unit, and the dispatcher spreads
  // workgroups over shader engines whose usable compute units need not be
  // equal in number, so a grid of one per compute unit could leave one
  // workgroup unplaced while the others wait for it at a barrier
  return (ncu >= 2 && per_cu >= 1) ? ncu / 2 : 0;
}
template <typename T>
void launch_gtail(const GTailArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((gtail_kernel<T>), dim3((unsigned)grid), dim3(GTAIL_THREADS), 0, st, a);
  HDG_CHECK(hipGetLastError());
}
template int gtail_grid<double>();
template int gtail_grid<float>();
template void launch_gtail<double>(const GTailArgs&, int, hipStream_t);
template void launch_gtail<float>(const GTailArgs&, int, hipStream_t);

}  // namespace hdg
