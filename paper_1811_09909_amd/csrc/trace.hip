// Trace-space kernels of the V-cycle (gfx950): matrix-free trace apply
// (eq. trace_linear_system, unassembled element DtN maps pulled per face),
// face-block Jacobi (Sec. 4.1), p-transfers (eqs. n_g1_Ik, n_g1_Qk),
// local correction (eq. localCorrection), h-transfers (eqs. n_1_Ik, n_1_Qk)
// and the coarsest direct solve (Algorithm 1, B_1 = A_1^-1).
//
// Face-major levels: one lane per interior face.  The rows of the two
// element maps that touch a face are one face-major AoSoA item, so every
// matrix load of a wavefront is one contiguous segment; the trace vector is
// gathered through the caches.  The finest level of a p-transition in 2D is
// element-major (packed symmetric maps): strip_kernel forms the element
// products of a 64 x 8 strip in LDS and finishes the faces inside the strip,
// shface_kernel the faces on strip edges.  The macro-element kernels of the
// h-transitions take 1, 2 or 4 lanes per macro-element.  No atomics: every
// output is written by exactly one lane, so results are bitwise
// reproducible.
#include "hdg_internal.hpp"
#include "blas.hpp"
#include "reduce.hpp"
#include "trace_dev.hpp"

namespace hdg {

namespace {

using namespace dev;

// -------------------------------------------------------------------------
// y = A x | y = b - A x | y = x + Dinv (b - A x) | rc = Jp^T (b - A x)
// Modes with a reduction (APPLY_Y_DOT: partial sums of x.y; APPLY_RES_NORM:
// of ||y||^2, and y32 = (float) y when given) write one partial per block;
// the caller launches the one-block finaliser.
// Minimum waves per SIMD the register allocation of the trace apply is held to
#ifndef HDG_APPLY_WPE
#define HDG_APPLY_WPE 1
#endif

// The trace apply of face-major levels with CH lanes per face (3D, k = 3:
// 3,072 block entries per face, and only 95,232 faces at 32^3, so one lane
// per face leaves under two waves per SIMD to hide the memory latency).
// Wave w of a workgroup takes rows w*RA .. of the 64 faces of the group (one
// per lane, so every block load of a wave is one contiguous 512-byte
// segment), loads a slot's rows into registers before summing them, and
// sums each row in the order of the one-lane form (face_acc), so results
// match it bit for bit.  Modes that need a whole face's residual (the
// block-Jacobi update, the p-restriction and its coarse first step) pass it
// through LDS.  Each workgroup walks the face groups blockIdx.x, +gridDim.x,
// ... of its right-hand side (blockIdx.y) and writes one partial sum.
template <int D, int NE, typename T, int MODE, typename M, int CH>
__global__ void __launch_bounds__(256) apply_mc_kernel(int n, const M* __restrict__ Af, const M* __restrict__ Dinv,
                                                       const T* __restrict__ x, const T* __restrict__ bvec,
                                                       T* __restrict__ y, const double* __restrict__ Jp,
                                                       T* __restrict__ rc, float* __restrict__ y32,
                                                       double* __restrict__ partials) {
  static_assert(CH * 64 == 256 && NE % CH == 0, "one wave per chunk of rows");
  constexpr bool RED = (MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM || MODE == APPLY_SWEEP_DOT);
  constexpr int NC = 1 << (D - 1);
  constexpr int RA = NE / CH, RC = (NC + CH - 1) / CH;
  constexpr int NL = 2 * D * NE;
  constexpr long S = vpad<M>(NL * NE);
  using A = acc_t<T>;
  __shared__ A sres[64][NE + 1];
  __shared__ A srcv[64][NC + 1];
  const int rhs = blockIdx.y;
  {
    const long sN = trace_len<D>(n, NE), sC = trace_len<D>(n, NC);
    x += rhs * sN;
    bvec = off(bvec, rhs * sN);
    y = off(y, rhs * (MODE == APPLY_RES_PRESTRICT ? sC : sN));
    rc = off(rc, rhs * sC);
    y32 = off(y32, rhs * sN);
    if (MODE == APPLY_SWEEP_DOT) Jp += rhs * sN;
  }
  const long nface = D * nface_dir<D>(n);
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  double part = 0.0;
  for (long fg = blockIdx.x; fg * 64 < nface; fg += gridDim.x) {
    const long F = fg * 64 + lane;
    const bool live = F < nface;
    A acc[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) acc[r] = A(0);
    if (live) {
      int g[3] = {0, 0, 0};
      const int cn = decode_face<D>(F, n, g);
      const M* Mbase = Af + aos_item<M>(F, 2 * S);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        int e[3] = {g[0], g[1], g[2]};
        e[cn] = g[cn] - 1 + side;
        const M* Mx = Mbase + side * S * LANES;
#pragma unroll
        for (int sl = 0; sl < 2 * D; ++sl) {
          const int cc = sl / 2, sd = sl % 2;
          const int p = e[cc] + sd;
          if (p == 0 || p == n) continue;
          int fgc[3] = {e[0], e[1], e[2]};
          fgc[cc] = p;
          const T* xf = x + face_id<D>(cc, fgc, n) * NE;
          M v[NE][RA];
#pragma unroll
          for (int bb = 0; bb < NE; ++bb)
#pragma unroll
            for (int r = 0; r < RA; ++r) v[bb][r] = Mx[aos_off<M>(0, 0, (sl * NE + bb) * NE + c * RA + r)];
          A xs[NE];
#pragma unroll
          for (int bb = 0; bb < NE; ++bb) xs[bb] = xf[bb];
#pragma unroll
          for (int bb = 0; bb < NE; ++bb)
#pragma unroll
            for (int r = 0; r < RA; ++r) acc[r] += A(v[bb][r]) * xs[bb];
        }
      }
    }
    if (MODE == APPLY_Y || MODE == APPLY_RES || MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM) {
      if (live)
#pragma unroll
        for (int r = 0; r < RA; ++r) {
          const long i = F * NE + c * RA + r;
          if (MODE == APPLY_Y) {
            y[i] = T(acc[r]);
          } else if (MODE == APPLY_RES) {
            y[i] = T(A(bvec[i]) - acc[r]);
          } else if (MODE == APPLY_Y_DOT) {
            y[i] = T(acc[r]);
            part += (double)x[i] * (double)T(acc[r]);
          } else {
            const T vv = T(A(bvec[i]) - acc[r]);
            y[i] = vv;
            if (y32) y32[i] = (float)vv;
            part += (double)vv * (double)vv;
          }
        }
    } else {
      // the face's whole residual through LDS
      if (live)
#pragma unroll
        for (int r = 0; r < RA; ++r) sres[lane][c * RA + r] = A(bvec[F * NE + c * RA + r]) - acc[r];
      __syncthreads();
      if (MODE == APPLY_SWEEP || MODE == APPLY_SWEEP_DOT) {
        if (live) {
          const M* Db = Dinv + aos_item<M>(F, vpad<M>(NE * NE));
#pragma unroll
          for (int r = 0; r < RA; ++r) {
            const int a = c * RA + r;
            M dv[NE];
#pragma unroll
            for (int bb = 0; bb < NE; ++bb) dv[bb] = Db[aos_off<M>(0, 0, a * NE + bb)];
            A s = A(x[F * NE + a]);
#pragma unroll
            for (int bb = 0; bb < NE; ++bb) s += A(dv[bb]) * sres[lane][bb];
            y[F * NE + a] = T(s);
            if (MODE == APPLY_SWEEP_DOT) part += Jp[F * NE + a] * (double)T(s);
          }
        }
      } else {  // APPLY_RES_PRESTRICT: J_N^T res, then the coarse first step
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const int vv = c * RC + r;
          if (live && vv < NC) {
            A s = A(0);
#pragma unroll
            for (int a = 0; a < NE; ++a) s += A(Jp[a * NC + vv]) * sres[lane][a];
            rc[F * NC + vv] = T(s);
            srcv[lane][vv] = A(T(s));
          }
        }
        if (y) {
          __syncthreads();
#pragma unroll
          for (int r = 0; r < RC; ++r) {
            const int vv = c * RC + r;
            if (live && vv < NC) {
              const M* Db = Dinv + aos_item<M>(F, vpad<M>(NC * NC));
              A s = A(0);
#pragma unroll
              for (int bb = 0; bb < NC; ++bb) s += A(Db[aos_off<M>(0, 0, vv * NC + bb)]) * srcv[lane][bb];
              y[F * NC + vv] = T(s);
            }
          }
        }
      }
      __syncthreads();  // sres / srcv are reused by the next face group
    }
  }
  if constexpr (RED) {
    __shared__ double sh[4];
    const double sum = block_sum_t<256>(part, sh);
    if (threadIdx.x == 0) partials[(long)rhs * gridDim.x + blockIdx.x] = sum;
  }
}

// ZS: the level is stored element-major; Af then points to the per-element
// products z of the first phase (elem_apply_kernel) and each face only adds
// its two elements' rows.  M: storage type of the operator blocks (T, or
// FP32 blocks under FP64 vectors on the finest level of the mixed cycle).
template <int D, int NE, typename T, int MODE, bool ZS = false, typename M = T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HDG_APPLY_WPE))) apply_kernel(int n, const M* __restrict__ Af, const M* __restrict__ Dinv,
                                                    const T* __restrict__ x, const T* __restrict__ bvec,
                                                    T* __restrict__ y, const double* __restrict__ Jp,
                                                    T* __restrict__ rc, float* __restrict__ y32,
                                                    double* __restrict__ partials, int nrhs) {
  constexpr bool RED = (MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM || MODE == APPLY_SWEEP_DOT);
  constexpr int NC = 1 << (D - 1);
  int rhs;
  unsigned slot;
  const long F = xcd_face_rhs<D>(n, nrhs, blockIdx.x, threadIdx.x, &rhs, &slot);
  if (!RED && F < 0) return;
  {
    const long sN = trace_len<D>(n, NE), sC = trace_len<D>(n, NC);
    x += rhs * sN;
    bvec = off(bvec, rhs * sN);
    y = off(y, rhs * (MODE == APPLY_RES_PRESTRICT ? sC : sN));
    rc = off(rc, rhs * sC);
    y32 = off(y32, rhs * sN);
    if (MODE == APPLY_SWEEP_DOT) Jp += rhs * sN;
    if (ZS) {
      long nelem = 1;
      for (int a = 0; a < D; ++a) nelem *= n;
      Af += rhs * ((nelem + 63) / 64 * 64) * (2 * D * NE);
    }
  }
  double part = 0.0;
  if (F >= 0) {
  using A = acc_t<T>;
  A acc[NE];
  if constexpr (ZS)
    face_acc_z<D, NE, T>(F, n, Af, acc);
  else
    face_acc<D, NE, T, M>(F, n, Af, x, acc);
  face_finish<D, NE, T, MODE, ZS, M>(F, acc, Dinv, x, bvec, y, Jp, rc, y32, part);
  }  // F >= 0
  if constexpr (RED) {
    __shared__ double sh[4];
    const double s = block_sum_t<256>(part, sh);
    if (threadIdx.x == 0) partials[slot] = s;
  }
}

// e = Dinv r (first sweep from e = 0); blocks stored as M
template <int NE, typename T, bool DSYM, typename M = T>
__global__ void jacobi0_kernel(long nface, int nrhs, const M* __restrict__ Dinv, const T* __restrict__ r,
                               T* __restrict__ e) {
  int rhs;
  const long b = xcd_block_rhs((nface + 255) / 256, nrhs, blockIdx.x, &rhs);
  const long F = b * 256 + threadIdx.x;
  if (b < 0 || F >= nface) return;
  r += rhs * nface * NE;
  e += rhs * nface * NE;
  jacobi0_item<NE, T, DSYM, M>(F, Dinv, r, e);
}

// e = Dinv r with CH lanes per face (as apply_mc_kernel: wave w takes rows
// w*RA .. of the 64 faces of its group, row sums in the order of
// jacobi0_item)
template <int NE, typename T, typename M, int CH>
__global__ void __launch_bounds__(256) jacobi0_mc_kernel(long nface, const M* __restrict__ Dinv,
                                                         const T* __restrict__ r, T* __restrict__ e) {
  constexpr int RA = NE / CH;
  using A = acc_t<T>;
  r += blockIdx.y * nface * NE;
  e += blockIdx.y * nface * NE;
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  for (long fg = blockIdx.x; fg * 64 < nface; fg += gridDim.x) {
    const long F = fg * 64 + lane;
    if (F >= nface) continue;
    A rv[NE];
#pragma unroll
    for (int b = 0; b < NE; ++b) rv[b] = r[F * NE + b];
    const M* Db = Dinv + aos_item<M>(F, vpad<M>(NE * NE));
#pragma unroll
    for (int k = 0; k < RA; ++k) {
      const int a = c * RA + k;
      M dv[NE];
#pragma unroll
      for (int b = 0; b < NE; ++b) dv[b] = Db[aos_off<M>(0, 0, a * NE + b)];
      A s = A(0);
#pragma unroll
      for (int b = 0; b < NE; ++b) s += A(dv[b]) * rv[b];
      e[F * NE + a] = T(s);
    }
  }
}

// One colour pass of multicolour point symmetric Gauss-Seidel (the LU-SGS
// smoother of Sec. 4.1 in a parallel order).  Colour col holds the faces of
// normal direction col / 2 at grid positions p (1 .. n-1) with p % 2 ==
// col % 2: no two of them bound a common element, so no face's row involves
// another one's values and every face of the colour updates at once.  One
// lane per face: acc = (A x)_F with the current values, then point updates of
// the face's values in increasing order (decreasing when backward), each
// followed by the change of the remaining rows through the face's own block
// D_F (held in Dblk).
template <int D, int NE, typename T, typename M = T>
__global__ void __launch_bounds__(256) sgs_color_kernel(int n, int col, int backward, const M* __restrict__ Af,
                                                        const M* __restrict__ Dblk, T* x, const T* __restrict__ b) {
  const int c = col / 2, par = col % 2;
  const long np = par ? n / 2 : (n - 1) / 2;  // positions p in 1 .. n-1 with p % 2 == par
  long nt = np;
  for (int a = 1; a < D; ++a) nt *= n;
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= nt) return;
  {
    const long sN = trace_len<D>(n, NE);
    x += blockIdx.y * sN;
    b += blockIdx.y * sN;
  }
  int g[3] = {0, 0, 0};
  long rem = t / np;
  g[c] = 2 * (int)(t % np) + (par ? 1 : 2);
  for (int a = 0; a < D; ++a)
    if (a != c) {
      g[a] = (int)(rem % n);
      rem /= n;
    }
  const long F = face_id<D>(c, g, n);
  using A = acc_t<T>;
  A acc[NE];
  face_acc<D, NE, T, M>(F, n, Af, x, acc);
  A xs[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) xs[a] = x[F * NE + a];
  const M* blk = Dblk + aos_item<M>(F, vpad<M>(NE * NE));
  constexpr int V = vw<M>();
#pragma unroll
  for (int ii = 0; ii < NE; ++ii) {
    const int a = backward ? NE - 1 - ii : ii;
    const A dx = (A(b[F * NE + a]) - acc[a]) / A(blk[((a * NE + a) / V) * (LANES * V) + (a * NE + a) % V]);
    xs[a] += dx;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = q * NE + a;  // D_F[q][a]: row q, column a
      acc[q] += A(blk[(e / V) * (LANES * V) + e % V]) * dx;
    }
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) x[F * NE + a] = T(xs[a]);
}

// first phase of the element-major apply: z_T = A^e x_T for every element
template <int D, int NE, typename T>
__global__ void __launch_bounds__(256) elem_apply_kernel(int n, const T* __restrict__ Ap, const T* __restrict__ x,
                                                         T* __restrict__ z, int nrhs) {
  long nelem = 1;
  for (int a = 0; a < D; ++a) nelem *= n;
  int rhs;
  const long Tq = xcd_elem_rhs(nelem, nrhs, blockIdx.x, threadIdx.x, &rhs);
  if (Tq < 0) return;
  x += rhs * trace_len<D>(n, NE);
  z += rhs * ((nelem + 63) / 64 * 64) * (2 * D * NE);
  elem_item<D, NE, T>(Tq, n, Ap, x, z);
}

// One-pass apply of an element-major level in 2D (n a multiple of 64).  A
// workgroup owns a strip of 64 x SH elements (one wavefront per grid row, so
// a wavefront's matrix loads are one AoSoA block):
//   phase 1: z_T = A^e x_T per element, into LDS;
//   phase 2: every face whose two elements lie in the strip is finished from
//            LDS (T- rows first, as face_acc_z adds them); each lane takes its
//            element's right and top face.
// The products of the faces on the strip's edge go to zsh ([nrhs][2 sides]
// [NE][nshp]; side 0 = T-, 1 = T+), which shface_kernel finishes.  Faces on
// strip edges: x = 64 m (m = 1 .. n/64-1, index (m-1) n + row) first, then
// y = SH m (index NV + (m-1) n + column).  Workgroups go to the 8 XCDs in
// contiguous bands of strips (right-hand side fastest after the XCD).
// Requires x != y: a strip's outputs may be read as another strip's inputs.
template <int NE, typename T, int MODE, int SH>
__global__ void __launch_bounds__(64 * SH) strip_kernel(int n, const T* __restrict__ Ap, const T* __restrict__ Dinv,
                                                        const T* __restrict__ x, const T* __restrict__ bvec,
                                                        T* __restrict__ y, const double* __restrict__ Jp,
                                                        T* __restrict__ rc, float* __restrict__ y32,
                                                        T* __restrict__ zsh, long nshp, int nbt,
                                                        double* __restrict__ partials, int nrhs) {
  constexpr int D = 2, NC = 2, NL = 4 * NE, NT = 64 * SH;
  constexpr bool RED = (MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM || MODE == APPLY_SWEEP_DOT);
  using A = acc_t<T>;
  __shared__ __align__(16) T zs[NL * NT];
  const int nsx = n / 64, nsy = n / SH;
  const unsigned nstrip = (unsigned)nsx * (unsigned)nsy;
  const unsigned C = (nstrip + 7u) / 8u;
  const unsigned p = blockIdx.x, xj = p & 7u, m = p >> 3;
  const int rhs = (int)(m % (unsigned)nrhs);
  const unsigned w = m / (unsigned)nrhs;
  const unsigned sidx = xj * C + w;
  const long slot = (long)rhs * nbt + xj + 8u * w;
  if (w >= C || sidx >= nstrip) {  // whole workgroup out of range
    if (RED && w < C && threadIdx.x == 0) partials[slot] = 0.0;
    return;
  }
  const int sy = (int)(sidx / (unsigned)nsx), sx = (int)(sidx - (unsigned)sy * (unsigned)nsx);
  const int tid = threadIdx.x, j = tid & 63, rr = tid >> 6;
  const int ex = sx * 64 + j, ey = sy * SH + rr;
  {
    const long sN = trace_len<D>(n, NE), sC = trace_len<D>(n, NC);
    x += rhs * sN;
    bvec = off(bvec, rhs * sN);
    y = off(y, rhs * (MODE == APPLY_RES_PRESTRICT ? sC : sN));
    rc = off(rc, rhs * sC);
    y32 = off(y32, rhs * sN);
    if (MODE == APPLY_SWEEP_DOT) Jp += rhs * sN;
    zsh += rhs * (2L * NE) * nshp;
  }
  {
    A acc[NL];
    elem_prod<D, NE, T>((long)ey * n + ex, n, Ap, x, acc);
#pragma unroll
    for (int i = 0; i < NL; ++i) zs[i * NT + tid] = T(acc[i]);
  }
  __syncthreads();
  const long nfd = (long)(n - 1) * n, NV = (long)(nsx - 1) * n;
  double part = 0.0;
  A acc[NE];
  // right face (normal x at ex + 1): slot 1 of this element, slot 0 of the next
  if (ex + 1 < n) {
    if (j < 63) {
      const long F = (long)ex + (long)(n - 1) * ey;
#pragma unroll
      for (int a = 0; a < NE; ++a) acc[a] = A(zs[(NE + a) * NT + tid]) + A(zs[a * NT + tid + 1]);
      face_finish<D, NE, T, MODE, true>(F, acc, Dinv, x, bvec, y, Jp, rc, y32, part);
    } else {
      const long q = (long)sx * n + ey;  // edge x = 64 (sx + 1)
#pragma unroll
      for (int a = 0; a < NE; ++a) zsh[(long)a * nshp + q] = zs[(NE + a) * NT + tid];
    }
  }
  // top face (normal y at ey + 1): slot 3 of this element, slot 2 of the one above
  if (ey + 1 < n) {
    if (rr < SH - 1) {
      const long F = nfd + ex + (long)n * ey;
#pragma unroll
      for (int a = 0; a < NE; ++a) acc[a] = A(zs[(3 * NE + a) * NT + tid]) + A(zs[(2 * NE + a) * NT + tid + 64]);
      face_finish<D, NE, T, MODE, true>(F, acc, Dinv, x, bvec, y, Jp, rc, y32, part);
    } else {
      const long q = NV + (long)sy * n + ex;  // edge y = SH (sy + 1)
#pragma unroll
      for (int a = 0; a < NE; ++a) zsh[(long)a * nshp + q] = zs[(3 * NE + a) * NT + tid];
    }
  }
  // left and bottom strip edges inside the domain: this element is T+
  if (j == 0 && ex > 0) {
    const long q = (long)(sx - 1) * n + ey;
#pragma unroll
    for (int a = 0; a < NE; ++a) zsh[(long)(NE + a) * nshp + q] = zs[a * NT + tid];
  }
  if (rr == 0 && ey > 0) {
    const long q = NV + (long)(sy - 1) * n + ex;
#pragma unroll
    for (int a = 0; a < NE; ++a) zsh[(long)(NE + a) * nshp + q] = zs[(2 * NE + a) * NT + tid];
  }
  if constexpr (RED) {  // the reduction reuses the product area once every lane is done with it
    __syncthreads();
    const double s = block_sum_t<NT>(part, reinterpret_cast<double*>(zs));
    if (threadIdx.x == 0) partials[slot] = s;
  }
}

// Faces on strip edges: (A x)_F = T- product + T+ product from zsh, then the
// mode's output.  Lane t of block b takes horizontal edge face b*256 + t
// (consecutive face ids: coalesced) and, for t < vpb, vertical edge face
// b*vpb + t: those are a grid column apart, so each one's loads are
// scattered, and they are spread thinly over all blocks.  Grid (blocks,
// nrhs); partials after the strip blocks' ones.
// lanes per block of the strip-edge kernel
#ifndef HDG_SHF_TPB
#define HDG_SHF_TPB 256
#endif
constexpr int SHF_TPB = HDG_SHF_TPB;

template <int NE, typename T, int MODE, int SH>
__device__ inline void shface_one(long q, int n, long NV, const T* __restrict__ Dinv, const T* x,
                                  const T* __restrict__ bvec, T* __restrict__ y, const double* __restrict__ Jp,
                                  T* __restrict__ rc, float* __restrict__ y32, const T* __restrict__ zsh, long nshp,
                                  double& part) {
  using A = acc_t<T>;
  long F;
  if (q < NV) {
    const long mm = q / n, row = q - mm * n;  // x = 64 (mm + 1)
    F = 64 * (mm + 1) - 1 + (long)(n - 1) * row;
  } else {
    const long h = q - NV, mm = h / n, col = h - mm * n;  // y = SH (mm + 1)
    F = (long)(n - 1) * n + col + (long)n * (SH * (mm + 1) - 1);
  }
  A acc[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = A(zsh[(long)a * nshp + q]) + A(zsh[(long)(NE + a) * nshp + q]);
  face_finish<2, NE, T, MODE, true>(F, acc, Dinv, x, bvec, y, Jp, rc, y32, part);
}

template <int NE, typename T, int MODE, int SH>
__global__ void __launch_bounds__(SHF_TPB) shface_kernel(int n, const T* __restrict__ Dinv, const T* __restrict__ x,
                                                     const T* __restrict__ bvec, T* __restrict__ y,
                                                     const double* __restrict__ Jp, T* __restrict__ rc,
                                                     float* __restrict__ y32, const T* __restrict__ zsh, long nshp,
                                                     int vpb, int nbt, int nb0, double* __restrict__ partials) {
  constexpr int D = 2, NC = 2;
  constexpr bool RED = (MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM || MODE == APPLY_SWEEP_DOT);
  const int rhs = blockIdx.y;
  const long nsx = n / 64, nsy = n / SH;
  const long NV = (nsx - 1) * n, NH = (nsy - 1) * n;
  {
    const long sN = trace_len<D>(n, NE), sC = trace_len<D>(n, NC);
    x += rhs * sN;
    bvec = off(bvec, rhs * sN);
    y = off(y, rhs * (MODE == APPLY_RES_PRESTRICT ? sC : sN));
    rc = off(rc, rhs * sC);
    y32 = off(y32, rhs * sN);
    if (MODE == APPLY_SWEEP_DOT) Jp += rhs * sN;
    zsh += rhs * (2L * NE) * nshp;
  }
  double part = 0.0;
  if ((int)threadIdx.x < vpb) {
    const long v = (long)blockIdx.x * vpb + threadIdx.x;
    if (v < NV) shface_one<NE, T, MODE, SH>(v, n, NV, Dinv, x, bvec, y, Jp, rc, y32, zsh, nshp, part);
  }
  const long h = blockIdx.x * (long)SHF_TPB + threadIdx.x;
  if (h < NH) shface_one<NE, T, MODE, SH>(NV + h, n, NV, Dinv, x, bvec, y, Jp, rc, y32, zsh, nshp, part);
  if constexpr (RED) {
    __shared__ double sh[SHF_TPB / 64];
    const double s = block_sum_t<SHF_TPB>(part, sh);
    if (threadIdx.x == 0) partials[(long)rhs * nbt + nb0 + blockIdx.x] = s;
  }
}

// e += J_N ec on every face (p-prolongation)
template <int NE, int NC, typename T>
__global__ void prolong_p_kernel(long nface, const double* __restrict__ Jp, const T* __restrict__ ec,
                                 T* __restrict__ e) {
  const long F = blockIdx.x * 256L + threadIdx.x;
  if (F >= nface) return;
  ec += blockIdx.y * nface * NC;
  e += blockIdx.y * nface * NE;
  using A = acc_t<T>;
  A cv[NC];
#pragma unroll
  for (int v = 0; v < NC; ++v) cv[v] = ec[F * NC + v];
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    A s = e[F * NE + a];
#pragma unroll
    for (int v = 0; v < NC; ++v) s += A(Jp[a * NC + v]) * cv[v];
    e[F * NE + a] = T(s);
  }
}

// Local correction and the macro-element part of the restriction:
//   e_I += A_II^-1 rho_I            (eq. localCorrection, when do_corr)
//   cb_M = R_M^T rho_I = -J^T A_BI A_II^-1 rho_I   (eq. n_1_Qk, when do_restrict;
//   the launcher passes the restriction block R, which is P on symmetric levels)
// CH lanes share a macro-element: wavefront w of the grid covers the 64
// macro-elements of group w / CH (one per lane, so the AoSoA blocks are read
// coalesced) and takes chunk w % CH of the work: rows c*RI .. of A_II^-1 and
// outputs c*RJ .. of the restriction.  Each row and output is still summed
// by one lane in the order of the one-lane form.
template <int D, typename T, typename M, int CH>
__global__ void __launch_bounds__(256) hcorr_kernel(int n, const M* __restrict__ AIIinv, const M* __restrict__ P,
                                                    const T* __restrict__ rho, T* __restrict__ e, int do_corr,
                                                    int do_restrict, T* __restrict__ cb) {
  constexpr int NC = 1 << (D - 1);
  constexpr int NIF = D * NC;  // interior faces per macro-element
  constexpr int NI = NIF * NC;
  constexpr int NCL = 2 * D * NC;
  constexpr int RI = (NI + CH - 1) / CH;
  constexpr int RJ = (NCL + CH - 1) / CH;
  const int nm = n / 2;
  long nmacro = 1;
  for (int a = 0; a < D; ++a) nmacro *= nm;
  const long t = blockIdx.x * 256L + threadIdx.x;
  const long w = t >> 6;
  const int c = (int)(w % CH);
  const long Mi = (w / CH) * 64 + (t & 63);
  if (Mi >= nmacro) return;
  {
    const long sF = trace_len<D>(n, NC);
    rho += blockIdx.y * sF;
    e += blockIdx.y * sF;
    cb = off(cb, blockIdx.y * nmacro * NCL);
  }
  int m[3] = {0, 0, 0};
  decode_elem<D>(Mi, nm, m);
  using A = acc_t<T>;
  A rI[NI];
#pragma unroll
  for (int i = 0; i < NIF; ++i) {
    const long f = macro_iface<D>(m, i, n);
#pragma unroll
    for (int a = 0; a < NC; ++a) rI[i * NC + a] = rho[f * NC + a];
  }
  if (do_corr) {
    const M* Ab = AIIinv + aos_item<M>(Mi, vpad<M>(NI * NI));
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int i = c * RI + r;
      if (i < NI) {
        // the whole row first: its loads stay in flight together
        M v[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) v[j] = Ab[aos_off<M>(0, 0, i * NI + j)];
        A s = A(0);
#pragma unroll
        for (int j = 0; j < NI; ++j) s += A(v[j]) * rI[j];
        const long f = macro_iface<D>(m, i / NC, n) * NC + i % NC;
        e[f] = T(A(e[f]) + s);
      }
    }
  }
  if (do_restrict) {
    const M* Pb = P + aos_item<M>(Mi, vpad<M>(NI * NCL));
#pragma unroll
    for (int r = 0; r < RJ; ++r) {
      const int J = c * RJ + r;
      if (J < NCL) {
        M v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = Pb[aos_off<M>(0, 0, i * NCL + J)];
        A s = A(0);
#pragma unroll
        for (int i = 0; i < NI; ++i) s += A(v[i]) * rI[i];
        cb[Mi * NCL + J] = T(s);
      }
    }
  }
}

// rc_F = J^T rho_B(F) + cb_{M-}(slot 2c+1) + cb_{M+}(slot 2c)   (eq. n_1_Qk)
template <int D, typename T>
__global__ void hrestrict_kernel(int n, const T* __restrict__ rho, const T* __restrict__ cb, T* __restrict__ rc) {
  constexpr int NC = 1 << (D - 1);
  constexpr int NS = NC;
  constexpr int NCL = 2 * D * NC;
  const int nm = n / 2;
  const long ncf = D * nface_dir<D>(nm);
  const long Fc = blockIdx.x * 256L + threadIdx.x;
  if (Fc >= ncf) return;
  {
    long nmacro = 1;
    for (int a = 0; a < D; ++a) nmacro *= nm;
    rho += blockIdx.y * trace_len<D>(n, NC);
    cb += blockIdx.y * nmacro * NCL;
    rc += blockIdx.y * ncf * NC;
  }
  int G[3] = {0, 0, 0};
  const int c = decode_face<D>(Fc, nm, G);
  using A = acc_t<T>;
  A out[NC];
#pragma unroll
  for (int V = 0; V < NC; ++V) out[V] = A(0);
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const long f = subface<D>(c, G, t, n);
#pragma unroll
    for (int v = 0; v < NC; ++v) {
      const A rv = rho[f * NC + v];
#pragma unroll
      for (int V = 0; V < NC; ++V) out[V] += A(jh_weight<D>(t, v, V)) * rv;
    }
  }
  int mm[3] = {G[0], G[1], G[2]};
  mm[c] = G[c] - 1;
  const long Mm = elem_id<D>(mm, nm);
  mm[c] = G[c];
  const long Mp = elem_id<D>(mm, nm);
#pragma unroll
  for (int V = 0; V < NC; ++V) {
    out[V] += A(cb[Mm * NCL + (2 * c + 1) * NC + V]);
    out[V] += A(cb[Mp * NCL + (2 * c) * NC + V]);
    rc[Fc * NC + V] = T(out[V]);
  }
}

// e_I += P_M ec_M per macro-element (blocks [0, nbm)), e_B += J ec per coarse
// face (blocks [nbm, ...))   (eq. n_1_Ik)
template <int D, typename T, typename M, int CH>
__global__ void __launch_bounds__(256) hprolong_kernel(int n, long nbm, const M* __restrict__ P,
                                                       const T* __restrict__ ec, T* __restrict__ e) {
  constexpr int NC = 1 << (D - 1);
  constexpr int NIF = D * NC;
  constexpr int NI = NIF * NC;
  constexpr int NCL = 2 * D * NC;
  using A = acc_t<T>;
  const int nm = n / 2;
  ec += blockIdx.y * trace_len<D>(nm, NC);
  e += blockIdx.y * trace_len<D>(n, NC);
  if (blockIdx.x < nbm) {
    long nmacro = 1;
    for (int a = 0; a < D; ++a) nmacro *= nm;
    // CH lanes per macro-element, rows c*RI .. of P for chunk c (as hcorr)
    constexpr int RI = (NI + CH - 1) / CH;
    const long t = blockIdx.x * 256L + threadIdx.x;
    const long w = t >> 6;
    const int c = (int)(w % CH);
    const long Mi = (w / CH) * 64 + (t & 63);
    if (Mi >= nmacro) return;
    int m[3] = {0, 0, 0};
    decode_elem<D>(Mi, nm, m);
    A cv[NCL];
#pragma unroll
    for (int sl = 0; sl < 2 * D; ++sl) {
      const int cc = sl / 2, sd = sl % 2;
      const int p = m[cc] + sd;
      if (p == 0 || p == nm) {
#pragma unroll
        for (int V = 0; V < NC; ++V) cv[sl * NC + V] = A(0);
      } else {
        int G[3] = {m[0], m[1], m[2]};
        G[cc] = p;
        const long Fc = face_id<D>(cc, G, nm);
#pragma unroll
        for (int V = 0; V < NC; ++V) cv[sl * NC + V] = ec[Fc * NC + V];
      }
    }
    const M* Pb = P + aos_item<M>(Mi, vpad<M>(NI * NCL));
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int i = c * RI + r;
      if (i < NI) {
        const long f = macro_iface<D>(m, i / NC, n) * NC + i % NC;
        M v[NCL];
#pragma unroll
        for (int J = 0; J < NCL; ++J) v[J] = Pb[aos_off<M>(0, 0, i * NCL + J)];
        A s = e[f];
#pragma unroll
        for (int J = 0; J < NCL; ++J) s += A(v[J]) * cv[J];
        e[f] = T(s);
      }
    }
  } else {
    const long ncf = D * nface_dir<D>(nm);
    const long Fc = (blockIdx.x - nbm) * 256L + threadIdx.x;
    if (Fc >= ncf) return;
    int G[3] = {0, 0, 0};
    const int c = decode_face<D>(Fc, nm, G);
    A cv[NC];
#pragma unroll
    for (int V = 0; V < NC; ++V) cv[V] = ec[Fc * NC + V];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const long f = subface<D>(c, G, t, n);
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        A s = e[f * NC + v];
#pragma unroll
        for (int V = 0; V < NC; ++V) s += A(jh_weight<D>(t, v, V)) * cv[V];
        e[f * NC + v] = T(s);
      }
    }
  }
}

template <typename T, typename M = T>
__global__ void coarse_solve_kernel(int N, const M* __restrict__ Ainv, const T* __restrict__ r, T* __restrict__ e) {
  r += blockIdx.y * (long)N;
  e += blockIdx.y * (long)N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    acc_t<T> s = 0;
    for (int j = 0; j < N; ++j) s += acc_t<T>(Ainv[i * N + j]) * r[j];
    e[i] = T(s);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) hpre_kernel(int n, int nrhs, const T* __restrict__ Af,
                                                   const T* __restrict__ AIIinv, const T* __restrict__ P,
                                                   const T* __restrict__ r, T* __restrict__ e, int do_corr,
                                                   T* __restrict__ cb) {
  const long nmacro = (long)(n / 2) * (n / 2);
  int rhs;
  const long b = xcd_block_rhs((nmacro + 255) / 256, nrhs, blockIdx.x, &rhs);
  const long M = b * 256 + threadIdx.x;
  if (b < 0) return;
  r += rhs * trace_len<2>(n, 2);
  e += rhs * trace_len<2>(n, 2);
  cb += rhs * nmacro * 8;
  if (M < nmacro) hpre_item<2, T>(M, n, Af, AIIinv, P, r, e, do_corr, cb);
}

// L = 2 or 4 lanes per macro-element (latency-bound levels)
template <typename T, int L>
__global__ void __launch_bounds__(256) hpreL_kernel(int n, int nrhs, const T* __restrict__ Af,
                                                    const T* __restrict__ AIIinv, const T* __restrict__ P,
                                                    const T* __restrict__ r, T* __restrict__ e, int do_corr,
                                                    T* __restrict__ cb) {
  const long nmacro = (long)(n / 2) * (n / 2);
  int rhs;
  const long b = xcd_block_rhs((L * nmacro + 255) / 256, nrhs, blockIdx.x, &rhs);
  const long t = b * 256 + threadIdx.x;
  const long M = t / L;
  if (b < 0) return;
  r += rhs * trace_len<2>(n, 2);
  e += rhs * trace_len<2>(n, 2);
  cb += rhs * nmacro * 8;
  if (M < nmacro) hpreL_item<T, L>(M, (int)(t % L), n, Af, AIIinv, P, r, e, do_corr, cb);
}

template <int D, typename T>
__global__ void hsum_kernel(int n, int nrhs, const T* __restrict__ r, const T* __restrict__ cb,
                            const T* __restrict__ Dc, T* __restrict__ rc, T* __restrict__ ec) {
  constexpr int NC = 1 << (D - 1);
  const long ncf = D * nface_dir<D>(n / 2);
  int rhs;
  const long b = xcd_block_rhs((ncf + 255) / 256, nrhs, blockIdx.x, &rhs);
  const long Fc = b * 256 + threadIdx.x;
  if (b < 0) return;
  long nmacro = 1;
  for (int a = 0; a < D; ++a) nmacro *= n / 2;
  r += rhs * trace_len<D>(n, NC);
  cb += rhs * nmacro * 2 * D * NC;
  rc = off(rc, rhs * ncf * NC);
  ec = off(ec, rhs * ncf * NC);
  if (Fc < ncf) hsum_item<D, T>(Fc, n, r, cb, Dc, rc, ec);
}

// LPM lanes per macro-element in the macro part (1, or 2 / 4 on latency-bound
// 2D levels)
template <int D, typename T, int LPM>
__global__ void __launch_bounds__(256) hpost_kernel(int n, long nbm, long nbf, int nrhs, const T* __restrict__ Af,
                                                    const T* __restrict__ AIIinv, const T* __restrict__ P,
                                                    const T* __restrict__ r, const T* __restrict__ ec,
                                                    const T* __restrict__ eold, T* __restrict__ enew, int do_corr) {
  int rhs;
  const long b = xcd_block_rhs(nbm + nbf, nrhs, blockIdx.x, &rhs);
  if (b < 0) return;
  {
    constexpr int NC = 1 << (D - 1);
    const long sF = trace_len<D>(n, NC);
    r += rhs * sF;
    eold += rhs * sF;
    enew += rhs * sF;
    ec += rhs * trace_len<D>(n / 2, NC);
  }
  if (b < nbm) {
    const long nmacro = (long)(n / 2) * (n / 2);
    const long t = b * 256 + threadIdx.x;
    if constexpr (LPM > 1) {
      if (t / LPM < nmacro) hpostL_m_item<T, LPM>(t / LPM, (int)(t % LPM), n, Af, AIIinv, P, r, ec, eold, enew, do_corr);
    } else {
      if (t < nmacro) hpost_m_item<D, T>(t, n, Af, AIIinv, P, r, ec, eold, enew, do_corr);
    }
  } else {
    const long ncf = D * nface_dir<D>(n / 2);
    const long Fc = (b - nbm) * 256 + threadIdx.x;
    if (Fc < ncf) hpost_f_item<D, T>(Fc, n, ec, eold, enew);
  }
}

// Coarsest level reached from an h-transition: r_c by the restriction sum
// and e_c = A_1^-1 r_c, in one workgroup (N <= 64)
template <int D, typename T>
__global__ void hsum_solve_kernel(int n, int N, const T* __restrict__ r, const T* __restrict__ cb,
                                  const T* __restrict__ Ainv, T* __restrict__ ec) {
  constexpr int NC = 1 << (D - 1);
  constexpr int NCL = 2 * D * NC;
  using A = acc_t<T>;
  __shared__ T rcs[64];
  const int nm = n / 2;
  const long ncf = D * nface_dir<D>(nm);
  {
    long nmacro = 1;
    for (int a = 0; a < D; ++a) nmacro *= nm;
    r += blockIdx.y * trace_len<D>(n, NC);
    cb += blockIdx.y * nmacro * NCL;
    ec += blockIdx.y * (long)N;
  }
  for (long Fc = threadIdx.x; Fc < ncf; Fc += blockDim.x) {
    int G[3] = {0, 0, 0};
    const int c = decode_face<D>(Fc, nm, G);
    A out[NC];
#pragma unroll
    for (int V = 0; V < NC; ++V) out[V] = A(0);
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const long f = subface<D>(c, G, t, n);
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        const A rv = r[f * NC + v];
#pragma unroll
        for (int V = 0; V < NC; ++V) out[V] += A(jh_weight<D>(t, v, V)) * rv;
      }
    }
    int mm[3] = {G[0], G[1], G[2]};
    mm[c] = G[c] - 1;
    const long Mm = elem_id<D>(mm, nm);
    mm[c] = G[c];
    const long Mp = elem_id<D>(mm, nm);
#pragma unroll
    for (int V = 0; V < NC; ++V)
      rcs[Fc * NC + V] = T(out[V] + A(cb[Mm * NCL + (2 * c + 1) * NC + V]) + A(cb[Mp * NCL + (2 * c) * NC + V]));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    A s = A(0);
    for (int j = 0; j < N; ++j) s += A(Ainv[i * N + j]) * rcs[j];
    ec[i] = T(s);
  }
}

// e = A_1^-1 r for a larger coarsest level: one wavefront per row
template <typename T, typename M = T>
__global__ void coarse_gemv_kernel(int N, const M* __restrict__ Ainv, const T* __restrict__ r, T* __restrict__ e) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= N) return;
  r += blockIdx.y * (long)N;
  e += blockIdx.y * (long)N;
  // columns lane, lane + 64, ... summed in that order; the loads of GU
  // consecutive terms go out before any is added (one at a time they were
  // a chain of memory round trips)
  constexpr int GU = 8;
  double s = 0.0;
  for (int j0 = lane; j0 < N; j0 += 64 * GU) {
    double a[GU], b[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int j = j0 + 64 * u < N ? j0 + 64 * u : N - 1;  // past the end: a valid column, not added
      a[u] = (double)Ainv[(long)row * N + j];
      b[u] = (double)r[j];
    }
#pragma unroll
    for (int u = 0; u < GU; ++u)
      if (j0 + 64 * u < N) s += a[u] * b[u];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) e[row] = (T)s;
}

inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }
// lanes per macro-element of the 3D local-correction / restriction /
// prolongation kernels (NI = 48 rows of A_II^-1 and P: 4 each; 24 restriction
// outputs: 2 each), and the blocks of 256 lanes that cover nmacro of them
constexpr int MACRO_CH3 = 12;
inline unsigned macro_blocks(long nmacro, int ch) { return (unsigned)(((nmacro + 63) / 64 * ch * 64 + 255) / 256); }

// macro-element kernels use 4 lanes per macro-element up to MULTI_LANE_MAX
// macro-elements times right-hand sides (latency-bound levels), 2 lanes up to
// MULTI_LANE2_MAX, one lane above (bandwidth-bound); HDG_MULTI_LANE_MAX and
// HDG_MULTI_LANE2_MAX override at build time.  Two lanes on the 256^2-macro
// level of the 512^2 workload measured no faster than one, so that band is
// empty by default.
#ifndef HDG_MULTI_LANE_MAX
#define HDG_MULTI_LANE_MAX 16384
#endif
#ifndef HDG_MULTI_LANE2_MAX
#define HDG_MULTI_LANE2_MAX 0
#endif
constexpr long MULTI_LANE_MAX = HDG_MULTI_LANE_MAX;  // macro-elements times right-hand sides
constexpr long MULTI_LANE2_MAX = HDG_MULTI_LANE2_MAX;
inline int lanes_per_macro(long nmacro, int nrhs) {
  const long w = nmacro * nrhs;
  return w <= MULTI_LANE_MAX ? 4 : w <= MULTI_LANE2_MAX ? 2 : 1;
}

// grid of xcd_block_rhs for nb blocks per right-hand side
inline unsigned xcd_rhs_grid(long nb, int nrhs) {
  return nrhs == 1 ? (unsigned)nb : (unsigned)(8 * ((nb + 7) / 8) * nrhs);
}

// grid of the XCD-aware face launches (see xcd_face): 8 chunks of C blocks
// per normal direction
// workgroups of the multi-lane apply: one per group of 64 faces, at most
// MAX_RED_BLOCKS (the workgroups then walk several groups)
inline unsigned mc_grid(long nface) {
  const long g = (nface + 63) / 64;
  return (unsigned)(g < MAX_RED_BLOCKS ? g : MAX_RED_BLOCKS);
}

inline unsigned xcd_grid(int d, int n) {
  long nfd = n - 1;
  for (int a = 1; a < d; ++a) nfd *= n;
  const long nbh = (nfd + 255) / 256;
  return (unsigned)(8L * d * ((nbh + 7) / 8));
}

template <typename F>
void dispatch_d_ne(int d, int ne, F&& f) {
#define HDG_CASE(DD, NN)                                                            \
  if (d == DD && ne == NN) {                                                        \
    f(std::integral_constant<int, DD>{}, std::integral_constant<int, NN>{});        \
    return;                                                                         \
  }
  HDG_CASE(2, 2) HDG_CASE(2, 3) HDG_CASE(2, 4) HDG_CASE(2, 5) HDG_CASE(2, 6) HDG_CASE(2, 7)
  HDG_CASE(3, 4) HDG_CASE(3, 9) HDG_CASE(3, 16)
#undef HDG_CASE
  throw HipError{hipErrorInvalidValue, "unsupported (d, ne)"};
}

// face sizes of the 2D levels (k = 1 .. 6)
template <typename F>
void dispatch_ne_2d(int ne, F&& f) {
  switch (ne) {
    case 2: f(std::integral_constant<int, 2>{}); return;
    case 3: f(std::integral_constant<int, 3>{}); return;
    case 4: f(std::integral_constant<int, 4>{}); return;
    case 5: f(std::integral_constant<int, 5>{}); return;
    case 6: f(std::integral_constant<int, 6>{}); return;
    case 7: f(std::integral_constant<int, 7>{}); return;
  }
  throw HipError{hipErrorInvalidValue, "unsupported face size"};
}

// rows of elements per strip of the one-pass element-major apply (the LDS
// products of a 64 x SH strip: 40 KiB for 512 lanes in FP32 at k = 4, 80 KiB
// in FP64; gfx950 gives a workgroup up to 160 KiB)
#ifndef HDG_STRIP_ROWS32
#define HDG_STRIP_ROWS32 8
#endif
#ifndef HDG_STRIP_ROWS64
#define HDG_STRIP_ROWS64 8
#endif
template <typename T>
constexpr int strip_rows() {
  return sizeof(T) == 4 ? HDG_STRIP_ROWS32 : HDG_STRIP_ROWS64;
}

// one-pass element-major apply (strip_kernel + shface_kernel); returns the
// number of partial sums per right-hand side
template <typename T, int MODE>
int launch_strips(const Level& L, const T* Dv, const T* x, const T* b, T* y, const double* Jp, T* rc, float* y32,
                  double* partials, hipStream_t st, int nrhs) {
  constexpr int SH = strip_rows<T>();
  const T* Ap = sizeof(T) == 8 ? (const T*)L.Ap64 : (const T*)L.Ap32;
  T* zsh = (T*)L.z[sizeof(T) == 8 ? 0 : 1];
  const int n = L.n;
  const long nsx = n / 64, nsy = n / SH;
  const long NV = (nsx - 1) * n, NH = (nsy - 1) * n;
  const long nsh = NV + NH, nshp = pad64(nsh);
  const long C = (nsx * nsy + 7) / 8;
  const long nbs = 8 * C, nbh = (NH + SHF_TPB - 1) / SHF_TPB;
  const int vpb = nbh > 0 ? (int)((NV + nbh - 1) / nbh) : 0;
  const int nbt = (int)(nbs + nbh);
  if (vpb > SHF_TPB || (NV > 0 && nbh == 0))
    throw HipError{hipErrorInvalidValue, "strip apply: edge faces do not fit the edge kernel"};
  if (x == y || 2 * L.ne * nshp > pad64(L.nelem) * L.nl)
    throw HipError{hipErrorInvalidValue, "strip apply: in-place output or edge buffer too small"};
  dispatch_ne_2d(L.ne, [&](auto NE_) {
    constexpr int NE = decltype(NE_)::value;
    hipLaunchKernelGGL((strip_kernel<NE, T, MODE, SH>), dim3((unsigned)(nbs * nrhs)), dim3(64 * SH), 0, st, n, Ap,
                       Dv, x, b, y, Jp, rc, y32, zsh, nshp, nbt, partials, nrhs);
    if (nbh > 0)
      hipLaunchKernelGGL((shface_kernel<NE, T, MODE, SH>), dim3((unsigned)nbh, nrhs), dim3(SHF_TPB), 0, st, n, Dv, x, b,
                         y, Jp, rc, y32, zsh, nshp, vpb, nbt, (int)nbs, partials);
  });
  HDG_CHECK(hipGetLastError());
  return nbt;
}

// first phase of the element-major apply on a packed level
template <typename T>
void launch_elem_phase(const Level& L, const T* x, hipStream_t st, int nrhs) {
  const T* Ap = sizeof(T) == 8 ? (const T*)L.Ap64 : (const T*)L.Ap32;
  T* z = (T*)L.z[sizeof(T) == 8 ? 0 : 1];
  const long C = ((L.nelem + 255) / 256 + 7) / 8;
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int D = decltype(D_)::value, NE = decltype(NE_)::value;
    hipLaunchKernelGGL((elem_apply_kernel<D, NE, T>), dim3((unsigned)(8 * C * nrhs)), dim3(256), 0, st, L.n, Ap, x, z,
                       nrhs);
  });
  HDG_CHECK(hipGetLastError());
}

}  // namespace

template <typename T, typename M>
void launch_apply(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc,
                  hipStream_t st, int nrhs) {
  launch_apply_red<T, M>(L, mode, x, b, y, Jp, rc, nullptr, nullptr, st, nrhs);
}

template <typename T, typename M>
void launch_apply_red(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc, float* y32,
                      Scratch* red, hipStream_t st, int nrhs, int* nparts) {
  if (L.nface == 0) return;
  if (L.u) {
    launch_uapply<T, M>(L, mode, x, b, y, Jp, rc, y32, red, st, nrhs, nparts);
    return;
  }
  double* partials = red ? red->partials : nullptr;
  const M* Af = nullptr;
  const M* Dv = nullptr;
  if constexpr (sizeof(M) == 8) {
    Af = (const M*)L.Af64;
    Dv = (const M*)L.Dinv64;
  } else {
    Af = (const M*)L.Af32;
    Dv = (const M*)L.Dinv32;
  }
  unsigned g1 = xcd_grid(L.d, L.n);
  if constexpr (!std::is_same_v<T, M>) {
    if (L.packed || !Af || !Dv)
      throw HipError{hipErrorInvalidValue, "narrow operator blocks under wider vectors: face-major levels only"};
  } else if (L.strip) {
    int nbt = 0;
    switch (mode) {
      case APPLY_Y: nbt = launch_strips<T, APPLY_Y>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs); break;
      case APPLY_RES: nbt = launch_strips<T, APPLY_RES>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs); break;
      case APPLY_SWEEP: nbt = launch_strips<T, APPLY_SWEEP>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs); break;
      case APPLY_RES_PRESTRICT:
        nbt = launch_strips<T, APPLY_RES_PRESTRICT>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs);
        break;
      case APPLY_Y_DOT: nbt = launch_strips<T, APPLY_Y_DOT>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs); break;
      case APPLY_RES_NORM:
        nbt = launch_strips<T, APPLY_RES_NORM>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs);
        break;
      case APPLY_SWEEP_DOT:
        nbt = launch_strips<T, APPLY_SWEEP_DOT>(L, Dv, x, b, y, Jp, rc, y32, partials, st, nrhs);
        break;
      default: throw HipError{hipErrorInvalidValue, "apply mode"};
    }
    if (mode == APPLY_SWEEP_DOT && !(red && nparts))
      throw HipError{hipErrorInvalidValue, "sweep with dot product: partials are finished by the caller"};
    if (red && mode == APPLY_SWEEP_DOT) {
      if (nbt > red->row) throw HipError{hipErrorInvalidValue, "strip apply: too many partial sums"};
      *nparts = nbt;
    }
    if (red && (mode == APPLY_Y_DOT || mode == APPLY_RES_NORM)) {
      if (nbt > red->row) throw HipError{hipErrorInvalidValue, "strip apply: too many partial sums"};
      if (nparts)
        *nparts = nbt;
      else
        blas_finalize(nbt, 1, mode == APPLY_Y_DOT ? FIN_ALPHA : FIN_RNORM, nullptr, *red, st, nrhs);
    }
    return;
  }
  if (!L.packed && L.d == 3 && L.ne == 16) {  // face-major 3D k = 3: four lanes per face
    const unsigned g = mc_grid(L.nface);
    if (red && (mode == APPLY_Y_DOT || mode == APPLY_RES_NORM || mode == APPLY_SWEEP_DOT) && (long)g > red->row)
      throw HipError{hipErrorInvalidValue, "trace apply: too many partial sums"};
#define HDG_MC(MM)                                                                                                 \
  hipLaunchKernelGGL((apply_mc_kernel<3, 16, T, MM, M, 4>), dim3(g, nrhs), dim3(256), 0, st, L.n, Af, Dv, x, b, y,   \
                     Jp, rc, y32, partials)
    switch (mode) {
      case APPLY_Y: HDG_MC(APPLY_Y); break;
      case APPLY_RES: HDG_MC(APPLY_RES); break;
      case APPLY_SWEEP: HDG_MC(APPLY_SWEEP); break;
      case APPLY_RES_PRESTRICT: HDG_MC(APPLY_RES_PRESTRICT); break;
      case APPLY_Y_DOT: HDG_MC(APPLY_Y_DOT); break;
      case APPLY_RES_NORM: HDG_MC(APPLY_RES_NORM); break;
      case APPLY_SWEEP_DOT: HDG_MC(APPLY_SWEEP_DOT); break;
      default: throw HipError{hipErrorInvalidValue, "apply mode"};
    }
#undef HDG_MC
    HDG_CHECK(hipGetLastError());
    if (mode == APPLY_SWEEP_DOT) {
      if (!(red && nparts))
        throw HipError{hipErrorInvalidValue, "sweep with dot product: partials are finished by the caller"};
      *nparts = (int)g;
    }
    if (red && (mode == APPLY_Y_DOT || mode == APPLY_RES_NORM)) {
      if (nparts)
        *nparts = (int)g;
      else
        blas_finalize((int)g, 1, mode == APPLY_Y_DOT ? FIN_ALPHA : FIN_RNORM, nullptr, *red, st, nrhs);
    }
    return;
  }
  const T* Zs = nullptr;
  if constexpr (std::is_same_v<T, M>) {
    if (L.packed) launch_elem_phase<T>(L, x, st, nrhs);
    Zs = L.packed ? (const T*)L.z[sizeof(T) == 8 ? 0 : 1] : nullptr;
  }
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int D = decltype(D_)::value, NE = decltype(NE_)::value;
#define HDG_AK(MM)                                                                                                 \
  if constexpr (std::is_same_v<T, M>) {                                                                            \
    if (L.packed)                                                                                                  \
      hipLaunchKernelGGL((apply_kernel<D, NE, T, MM, true>), dim3(g1 * (unsigned)nrhs), dim3(256), 0, st, L.n, Zs,   \
                         Dv, x, b, y, Jp, rc, y32, partials, nrhs);                                                \
    else                                                                                                           \
      hipLaunchKernelGGL((apply_kernel<D, NE, T, MM>), dim3(g1 * (unsigned)nrhs), dim3(256), 0, st, L.n, Af, Dv, x,  \
                         b, y, Jp, rc, y32, partials, nrhs);                                                       \
  } else {                                                                                                         \
    hipLaunchKernelGGL((apply_kernel<D, NE, T, MM, false, M>), dim3(g1 * (unsigned)nrhs), dim3(256), 0, st, L.n, Af, \
                       Dv, x, b, y, Jp, rc, y32, partials, nrhs);                                                  \
  }
    switch (mode) {
      case APPLY_Y: HDG_AK(APPLY_Y); break;
      case APPLY_RES: HDG_AK(APPLY_RES); break;
      case APPLY_SWEEP: HDG_AK(APPLY_SWEEP); break;
      case APPLY_RES_PRESTRICT: HDG_AK(APPLY_RES_PRESTRICT); break;
      case APPLY_Y_DOT: HDG_AK(APPLY_Y_DOT); break;
      case APPLY_RES_NORM: HDG_AK(APPLY_RES_NORM); break;
      case APPLY_SWEEP_DOT: HDG_AK(APPLY_SWEEP_DOT); break;
      default: throw HipError{hipErrorInvalidValue, "apply mode"};
    }
#undef HDG_AK
  });
  HDG_CHECK(hipGetLastError());
  if (mode == APPLY_SWEEP_DOT) {
    if (!(red && nparts))
      throw HipError{hipErrorInvalidValue, "sweep with dot product: partials are finished by the caller"};
    *nparts = (int)g1;
  }
  if (red && (mode == APPLY_Y_DOT || mode == APPLY_RES_NORM)) {
    if (nparts)
      *nparts = (int)g1;
    else
      blas_finalize((int)g1, 1, mode == APPLY_Y_DOT ? FIN_ALPHA : FIN_RNORM, nullptr, *red, st, nrhs);
  }
}

// residual of level L restricted to P1 on the same faces (level C), and when
// ec is given the first block-Jacobi step of C on it
template <typename T>
void launch_res_prestrict(const Level& L, const Level& C, const T* x, const T* b, T* rc, T* ec, const double* Jp,
                          hipStream_t st, int nrhs) {
  if (L.nface == 0) return;
  const T* Af = sizeof(T) == 8 ? (const T*)L.Af64 : (const T*)L.Af32;
  const T* Dc = sizeof(T) == 8 ? (const T*)C.Dinv64 : (const T*)C.Dinv32;
  if (L.strip) {
    launch_strips<T, APPLY_RES_PRESTRICT>(L, Dc, x, b, ec, Jp, rc, nullptr, nullptr, st, nrhs);
    return;
  }
  if (!L.packed && L.d == 3 && L.ne == 16) {
    hipLaunchKernelGGL((apply_mc_kernel<3, 16, T, APPLY_RES_PRESTRICT, T, 4>), dim3(mc_grid(L.nface), nrhs), dim3(256),
                       0, st, L.n, Af, Dc, x, b, ec, Jp, rc, nullptr, nullptr);
    HDG_CHECK(hipGetLastError());
    return;
  }
  if (L.packed) launch_elem_phase<T>(L, x, st, nrhs);
  const T* Zs = L.packed ? (const T*)L.z[sizeof(T) == 8 ? 0 : 1] : nullptr;
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int D = decltype(D_)::value, NE = decltype(NE_)::value;
    if (L.packed)
      hipLaunchKernelGGL((apply_kernel<D, NE, T, APPLY_RES_PRESTRICT, true>),
                         dim3(xcd_grid(L.d, L.n) * (unsigned)nrhs), dim3(256), 0, st, L.n, Zs, Dc, x, b, ec, Jp, rc,
                         nullptr, nullptr, nrhs);
    else
      hipLaunchKernelGGL((apply_kernel<D, NE, T, APPLY_RES_PRESTRICT>), dim3(xcd_grid(L.d, L.n) * (unsigned)nrhs),
                         dim3(256), 0, st, L.n, Af, Dc, x, b, ec, Jp, rc, nullptr, nullptr, nrhs);
  });
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_jacobi0(const Level& L, const T* r, T* e, hipStream_t st, int nrhs) {
  if (L.nface == 0) return;
  const M* Dv = sizeof(M) == 8 ? (const M*)L.Dinv64 : (const M*)L.Dinv32;
  if (!L.packed && L.ne == 16) {  // 3D k = 3 face blocks: four lanes per face
    hipLaunchKernelGGL((jacobi0_mc_kernel<16, T, M, 4>), dim3(mc_grid(L.nface), nrhs), dim3(256), 0, st, L.nface, Dv,
                       r, e);
    HDG_CHECK(hipGetLastError());
    return;
  }
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int NE = decltype(NE_)::value;
    const dim3 g(xcd_rhs_grid(nblk(L.nface), nrhs));
    if constexpr (std::is_same_v<T, M>) {
      if (L.packed)
        hipLaunchKernelGGL((jacobi0_kernel<NE, T, true>), g, dim3(256), 0, st, L.nface, nrhs, Dv, r, e);
      else
        hipLaunchKernelGGL((jacobi0_kernel<NE, T, false>), g, dim3(256), 0, st, L.nface, nrhs, Dv, r, e);
    } else {
      if (L.packed) throw HipError{hipErrorInvalidValue, "narrow operator blocks: face-major levels only"};
      hipLaunchKernelGGL((jacobi0_kernel<NE, T, false, M>), g, dim3(256), 0, st, L.nface, nrhs, Dv, r, e);
    }
  });
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void launch_prolong_p(const Level& L, int nc, const double* Jp, const T* ec, T* e, hipStream_t st, int nrhs) {
  if (L.nface == 0) return;
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int D = decltype(D_)::value, NE = decltype(NE_)::value;
    constexpr int NC = 1 << (D - 1);
    hipLaunchKernelGGL((prolong_p_kernel<NE, NC, T>), dim3(nblk(L.nface), nrhs), dim3(256), 0, st, L.nface, Jp, ec,
                       e);
  });
  (void)nc;
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_hcorr(const Level& L, const T* rho, T* e, int do_corr, int do_restrict, T* cb, hipStream_t st, int nrhs) {
  if (L.u) {
    launch_ucorr<T, M>(L, rho, e, do_corr, do_restrict, cb, st, nrhs);
    return;
  }
  const M* Ai = sizeof(M) == 8 ? (const M*)L.AIIinv64 : (const M*)L.AIIinv32;
  const M* P = sizeof(M) == 8 ? (const M*)L.R64 : (const M*)L.R32;  // restriction block
  if (L.d == 2)
    hipLaunchKernelGGL((hcorr_kernel<2, T, M, 1>), dim3(nblk(L.nmacro), nrhs), dim3(256), 0, st, L.n, Ai, P, rho, e,
                       do_corr, do_restrict, cb);
  else
    hipLaunchKernelGGL((hcorr_kernel<3, T, M, MACRO_CH3>), dim3(macro_blocks(L.nmacro, MACRO_CH3), nrhs), dim3(256), 0,
                       st, L.n, Ai, P, rho, e, do_corr, do_restrict, cb);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void launch_hrestrict(const Level& L, const Level& C, const T* rho, const T* cb, T* rc, hipStream_t st, int nrhs) {
  if (L.u) {
    launch_urestrict<T>(L, C, rho, cb, rc, st, nrhs);
    return;
  }
  if (C.nface == 0) return;
  if (L.d == 2)
    hipLaunchKernelGGL((hrestrict_kernel<2, T>), dim3(nblk(C.nface), nrhs), dim3(256), 0, st, L.n, rho, cb, rc);
  else
    hipLaunchKernelGGL((hrestrict_kernel<3, T>), dim3(nblk(C.nface), nrhs), dim3(256), 0, st, L.n, rho, cb, rc);
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_hprolong(const Level& L, const Level& C, const T* ec, T* e, hipStream_t st, int nrhs) {
  if (L.u) {
    launch_uprolong<T, M>(L, C, ec, e, st, nrhs);
    return;
  }
  const M* P = sizeof(M) == 8 ? (const M*)L.P64 : (const M*)L.P32;
  const long nbf = nblk(C.nface);
  if (L.d == 2) {
    const long nbm = nblk(L.nmacro);
    hipLaunchKernelGGL((hprolong_kernel<2, T, M, 1>), dim3((unsigned)(nbm + nbf), nrhs), dim3(256), 0, st, L.n, nbm, P,
                       ec, e);
  } else {
    const long nbm = macro_blocks(L.nmacro, MACRO_CH3);
    hipLaunchKernelGGL((hprolong_kernel<3, T, M, MACRO_CH3>), dim3((unsigned)(nbm + nbf), nrhs), dim3(256), 0, st,
                       L.n, nbm, P, ec, e);
  }
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_coarse_solve(const Level& L, const T* r, T* e, hipStream_t st, int nrhs) {
  if (L.nlam == 0) return;
  const M* Ai = sizeof(M) == 8 ? (const M*)L.Ainv64 : (const M*)L.Ainv32;
  if (L.nlam > 64) {
    hipLaunchKernelGGL((coarse_gemv_kernel<T, M>), dim3((unsigned)((L.nlam + 3) / 4), nrhs), dim3(256), 0, st,
                       (int)L.nlam, Ai, r, e);
    HDG_CHECK(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL((coarse_solve_kernel<T, M>), dim3(1, nrhs), dim3(64), 0, st, (int)L.nlam, Ai, r, e);
  HDG_CHECK(hipGetLastError());
}


int level_lanes(const Level& L, int nrhs) { return L.lpm > 0 ? L.lpm : lanes_per_macro(L.nmacro, nrhs); }

template <typename T>
void launch_hpre(const Level& L, const T* r, T* e, int do_corr, T* cb, hipStream_t st, int nrhs) {
  const T* Af = sizeof(T) == 8 ? (const T*)L.Af64 : (const T*)L.Af32;
  const T* Ai = sizeof(T) == 8 ? (const T*)L.AIIinv64 : (const T*)L.AIIinv32;
  const T* P = sizeof(T) == 8 ? (const T*)L.R64 : (const T*)L.R32;  // restriction block
  const int lpm = L.lpm > 0 ? L.lpm : lanes_per_macro(L.nmacro, nrhs);
  if (lpm == 4)
    hipLaunchKernelGGL((hpreL_kernel<T, 4>), dim3(xcd_rhs_grid(nblk(4 * L.nmacro), nrhs)), dim3(256), 0, st, L.n, nrhs,
                       Af, Ai, P, r, e, do_corr, cb);
  else if (lpm == 2)
    hipLaunchKernelGGL((hpreL_kernel<T, 2>), dim3(xcd_rhs_grid(nblk(2 * L.nmacro), nrhs)), dim3(256), 0, st, L.n, nrhs,
                       Af, Ai, P, r, e, do_corr, cb);
  else
    hipLaunchKernelGGL((hpre_kernel<T>), dim3(xcd_rhs_grid(nblk(L.nmacro), nrhs)), dim3(256), 0, st, L.n, nrhs, Af,
                       Ai, P, r, e, do_corr, cb);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void launch_hsum(const Level& L, const Level& C, const T* r, const T* cb, T* rc, T* ec, hipStream_t st, int nrhs) {
  if (C.kind == 2 && C.nlam <= 64) {
    const T* Ai = sizeof(T) == 8 ? (const T*)C.Ainv64 : (const T*)C.Ainv32;
    hipLaunchKernelGGL((hsum_solve_kernel<2, T>), dim3(1, nrhs), dim3(64), 0, st, L.n, (int)C.nlam, r, cb, Ai, ec);
  } else if (C.kind == 2) {
    // restricted residual into C.r, then the dense coarsest solve
    hipLaunchKernelGGL((hsum_kernel<2, T>), dim3(xcd_rhs_grid(nblk(C.nface), nrhs)), dim3(256), 0, st, L.n, nrhs, r,
                       cb, (const T*)nullptr, (T*)C.r[sizeof(T) == 8 ? 0 : 1], (T*)nullptr);
    HDG_CHECK(hipGetLastError());
    launch_coarse_solve<T>(C, (const T*)C.r[sizeof(T) == 8 ? 0 : 1], ec, st, nrhs);
  } else {
    const T* Dc = ec ? (sizeof(T) == 8 ? (const T*)C.Dinv64 : (const T*)C.Dinv32) : nullptr;
    hipLaunchKernelGGL((hsum_kernel<2, T>), dim3(xcd_rhs_grid(nblk(C.nface), nrhs)), dim3(256), 0, st, L.n, nrhs, r,
                       cb, Dc, rc, ec);
  }
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void launch_hpost(const Level& L, const Level& C, const T* r, const T* ec, const T* eold, T* enew, int do_corr,
                  hipStream_t st, int nrhs) {
  const T* Af = sizeof(T) == 8 ? (const T*)L.Af64 : (const T*)L.Af32;
  const T* Ai = sizeof(T) == 8 ? (const T*)L.AIIinv64 : (const T*)L.AIIinv32;
  const T* P = sizeof(T) == 8 ? (const T*)L.P64 : (const T*)L.P32;
  const long nbf = nblk(C.nface);
  const int lpm = L.lpm > 0 ? L.lpm : lanes_per_macro(L.nmacro, nrhs);
  if (lpm == 4) {
    const long nbm = nblk(4 * L.nmacro);
    hipLaunchKernelGGL((hpost_kernel<2, T, 4>), dim3(xcd_rhs_grid(nbm + nbf, nrhs)), dim3(256), 0, st, L.n, nbm, nbf,
                       nrhs, Af, Ai, P, r, ec, eold, enew, do_corr);
  } else if (lpm == 2) {
    const long nbm = nblk(2 * L.nmacro);
    hipLaunchKernelGGL((hpost_kernel<2, T, 2>), dim3(xcd_rhs_grid(nbm + nbf, nrhs)), dim3(256), 0, st, L.n, nbm, nbf,
                       nrhs, Af, Ai, P, r, ec, eold, enew, do_corr);
  } else {
    const long nbm = nblk(L.nmacro);
    hipLaunchKernelGGL((hpost_kernel<2, T, 1>), dim3(xcd_rhs_grid(nbm + nbf, nrhs)), dim3(256), 0, st, L.n, nbm, nbf,
                       nrhs, Af, Ai, P, r, ec, eold, enew, do_corr);
  }
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_sgs_color(const Level& L, int col, int backward, T* x, const T* b, hipStream_t st, int nrhs) {
  if (L.nface == 0) return;
  if (L.packed) throw HipError{hipErrorInvalidValue, "Gauss-Seidel smoother: face-major levels only"};
  const M* Af = sizeof(M) == 8 ? (const M*)L.Af64 : (const M*)L.Af32;
  const M* Db = sizeof(M) == 8 ? (const M*)L.Dinv64 : (const M*)L.Dinv32;
  const long np = (col % 2) ? L.n / 2 : (L.n - 1) / 2;
  long nt = np;
  for (int a = 1; a < L.d; ++a) nt *= L.n;
  if (nt == 0) return;
  dispatch_d_ne(L.d, L.ne, [&](auto D_, auto NE_) {
    constexpr int D = decltype(D_)::value, NE = decltype(NE_)::value;
    hipLaunchKernelGGL((sgs_color_kernel<D, NE, T, M>), dim3(nblk(nt), nrhs), dim3(256), 0, st, L.n, col, backward, Af,
                       Db, x, b);
  });
  HDG_CHECK(hipGetLastError());
}

// operator-reading launchers also for FP32 operator blocks under FP64 vectors
#define HDG_INST_M(T, M)                                                                                          \
  template void launch_apply<T, M>(const Level&, int, const T*, const T*, T*, const double*, T*, hipStream_t, int); \
  template void launch_apply_red<T, M>(const Level&, int, const T*, const T*, T*, const double*, T*, float*,       \
                                       Scratch*, hipStream_t, int, int*);                                         \
  template void launch_jacobi0<T, M>(const Level&, const T*, T*, hipStream_t, int);                               \
  template void launch_hcorr<T, M>(const Level&, const T*, T*, int, int, T*, hipStream_t, int);                   \
  template void launch_hprolong<T, M>(const Level&, const Level&, const T*, T*, hipStream_t, int);                \
  template void launch_coarse_solve<T, M>(const Level&, const T*, T*, hipStream_t, int);                        \
  template void launch_sgs_color<T, M>(const Level&, int, int, T*, const T*, hipStream_t, int);
HDG_INST_M(double, double)
HDG_INST_M(float, float)
HDG_INST_M(double, float)
#undef HDG_INST_M

#define HDG_INST(T)                                                                                              \
  template void launch_prolong_p<T>(const Level&, int, const double*, const T*, T*, hipStream_t, int);            \
  template void launch_hrestrict<T>(const Level&, const Level&, const T*, const T*, T*, hipStream_t, int);        \
  template void launch_hpre<T>(const Level&, const T*, T*, int, T*, hipStream_t, int);                            \
  template void launch_res_prestrict<T>(const Level&, const Level&, const T*, const T*, T*, T*, const double*,      \
                                        hipStream_t, int);                                                        \
  template void launch_hsum<T>(const Level&, const Level&, const T*, const T*, T*, T*, hipStream_t, int);         \
  template void launch_hpost<T>(const Level&, const Level&, const T*, const T*, const T*, T*, int, hipStream_t, int);
HDG_INST(double)
HDG_INST(float)
#undef HDG_INST

}  // namespace hdg
