// Hierarchy construction kernels (gfx950), all in FP64:
//  * face-major copies of the element matrices for the trace apply,
//  * assembled face-block inverses for block-Jacobi (Sec. 4.1),
//  * p-level Galerkin operator J_N^T A^e J_N per element (eq. ANm1),
//  * per coarse macro-element: assembly of the 2^d children on the interior
//    faces I and boundary faces B of the macro-element, A_II^-1,
//    S = A_BB - A_BI A_II^-1 A_IB, coarse matrix J^T S J (eq. Akm1) and the
//    prolongation block P = -A_II^-1 A_IB J (eq. n_1_Ik).  On symmetric levels
//    (HDG, SIPG-H) A_BI is taken as A_IB^T and the restriction is Q = I^T
//    (eq. n_1_Qk); otherwise A_BI is read from the children and the
//    restriction block R = -A_II^-T A_BI^T J is formed as well,
//  * dense inverse of the coarsest operator (Algorithm 1, B_1 = A_1^-1).
#include "hdg_internal.hpp"
#include "mfma_dev.hpp"

namespace hdg {

namespace {

inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

__device__ inline long nfd_of(int d, int n) {
  long v = n - 1;
  for (int a = 1; a < d; ++a) v *= n;
  return v;
}

__device__ inline int decode_face_rt(int d, long F, int n, int* g) {
  long nfd = nfd_of(d, n);
  int c = (int)(F / nfd);
  long r = F % nfd;
  for (int a = 0; a < d; ++a) {
    int ext = a == c ? n - 1 : n;
    g[a] = (int)(r % ext) + (a == c ? 1 : 0);
    r /= ext;
  }
  return c;
}

__device__ inline long elem_rt(int d, const int* e, int n) {
  long T = 0;
  for (int a = d - 1; a >= 0; --a) T = T * n + e[a];
  return T;
}

// Af[F, side, j, a] = A_{T_side}[slot_side*ne + a][j] (FP64 and FP32 copies)
__global__ void face_major_kernel(int d, int n, int ne, long nface, const double* __restrict__ Aelem,
                                  double* __restrict__ Af64, float* __restrict__ Af32) {
  const int nl = 2 * d * ne;
  const long per = 2L * nl * ne;
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= nface * per) return;
  const long F = t / per;
  long r = t % per;
  const int side = (int)(r / (nl * ne));
  r %= nl * ne;
  const int j = (int)(r / ne), a = (int)(r % ne);
  int g[3] = {0, 0, 0};
  const int c = decode_face_rt(d, F, n, g);
  int e[3] = {g[0], g[1], g[2]};
  e[c] = g[c] - 1 + side;
  const long T = elem_rt(d, e, n);
  const int slot = side == 0 ? 2 * c + 1 : 2 * c;
  const double v = Aelem[(T * nl + slot * ne + a) * nl + j];
  const long ent = (long)j * ne + a;
  const long s64 = vpad<double>((long)nl * ne), s32 = vpad<float>((long)nl * ne);
  Af64[aos_off<double>(F, 2 * s64, side * s64 + ent)] = v;
  Af32[aos_off<float>(F, 2 * s32, side * s32 + ent)] = (float)v;
}

// Per face, from the assembled diagonal block D_F = A_{T-}[F,F] + A_{T+}[F,F]
// (Sec. 4.1 smoothers): mode 0, omega * D_F^-1 (block Jacobi; sym: stored
// as the upper triangle, row by row, of the symmetrized inverse); mode 1,
// omega / diag(D_F) as a diagonal block (point Jacobi); mode 2, D_F itself
// (the in-face updates of point Gauss-Seidel).
template <int NE>
__global__ void dinv_kernel(int d, int n, long nface, double omega, const double* __restrict__ Aelem,
                            double* __restrict__ D64, float* __restrict__ D32, int sym, int mode) {
  const long F = blockIdx.x * 256L + threadIdx.x;
  if (F >= nface) return;
  const int nl = 2 * d * NE;
  int g[3] = {0, 0, 0};
  const int c = decode_face_rt(d, F, n, g);
  double A[NE * NE];
  for (int i = 0; i < NE * NE; ++i) A[i] = 0.0;
  for (int side = 0; side < 2; ++side) {
    int e[3] = {g[0], g[1], g[2]};
    e[c] = g[c] - 1 + side;
    const long T = elem_rt(d, e, n);
    const int slot = side == 0 ? 2 * c + 1 : 2 * c;
    for (int a = 0; a < NE; ++a)
      for (int b = 0; b < NE; ++b) A[a * NE + b] += Aelem[(T * nl + slot * NE + a) * nl + slot * NE + b];
  }
  if (mode != 0) {
    for (int i = 0; i < NE * NE; ++i) {
      double v = A[i];
      if (mode == 1) v = (i % (NE + 1) == 0) ? omega / A[i] : 0.0;
      D64[aos_off<double>(F, vpad<double>(NE * NE), i)] = v;
      D32[aos_off<float>(F, vpad<float>(NE * NE), i)] = (float)v;
    }
    return;
  }
  // Gauss-Jordan, SPD block: no pivoting
  for (int k = 0; k < NE; ++k) {
    const double p = 1.0 / A[k * NE + k];
    for (int j = 0; j < NE; ++j)
      if (j != k) A[k * NE + j] *= p;
    for (int i = 0; i < NE; ++i) {
      if (i == k) continue;
      const double f = A[i * NE + k];
      for (int j = 0; j < NE; ++j)
        if (j != k) A[i * NE + j] -= f * A[k * NE + j];
      A[i * NE + k] = -f * p;
    }
    A[k * NE + k] = p;
  }
  if (sym) {
    constexpr int NP = NE * (NE + 1) / 2;
    int idx = 0;
    for (int i = 0; i < NE; ++i)
      for (int j = i; j < NE; ++j, ++idx) {
        const double v = omega * 0.5 * (A[i * NE + j] + A[j * NE + i]);
        D64[aos_off<double>(F, vpad<double>(NP), idx)] = v;
        D32[aos_off<float>(F, vpad<float>(NP), idx)] = (float)v;
      }
    return;
  }
  for (int i = 0; i < NE * NE; ++i) {
    const double v = omega * A[i];
    D64[aos_off<double>(F, vpad<double>(NE * NE), i)] = v;
    D32[aos_off<float>(F, vpad<float>(NE * NE), i)] = (float)v;
  }
}

// dst = s * src in FP64 and its FP32 copy (per-step copies of a level's
// diagonal blocks for the Chebyshev smoother)
__global__ void scale_copy_kernel(long n, double s, const double* __restrict__ src, double* __restrict__ d64,
                                  float* __restrict__ d32) {
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= n) return;
  const double v = s * src[i];
  d64[i] = v;
  d32[i] = (float)v;
}

// Ac[(s1,v1),(s2,v2)] = sum_a Jp[a][v1] (sum_b A[(s1,a),(s2,b)] Jp[b][v2]),
// a lane per entry (2D: the lanes of a wave share their rows of A)
__global__ void pgalerkin_kernel(int d, int ne, long nelem, const double* __restrict__ Jp,
                                 const double* __restrict__ Af, double* __restrict__ Ac) {
  const int nc = 1 << (d - 1);
  const int nl = 2 * d * ne, ncl = 2 * d * nc;
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= nelem * ncl * ncl) return;
  const long T = t / (ncl * ncl);
  const int r = (int)(t % (ncl * ncl));
  const int I = r / ncl, J = r % ncl;
  const int s1 = I / nc, v1 = I % nc, s2 = J / nc, v2 = J % nc;
  double s = 0.0;
  for (int a = 0; a < ne; ++a) {
    double inner = 0.0;
    for (int b = 0; b < ne; ++b) inner += Af[(T * nl + s1 * ne + a) * nl + s2 * ne + b] * Jp[b * nc + v2];
    s += Jp[a * nc + v1] * inner;
  }
  Ac[t] = s;
}

// The same product by rows (3D, where a lane per entry re-reads 256 entries
// of A): a workgroup takes 256 / nl elements; first a lane per row of A forms
// that row of T = A blockdiag(Jp) in LDS (each row of A read once, in order),
// then a lane per output entry sums blockdiag(Jp)^T T.  The sums run in the
// same order as in the entry-by-entry form.
constexpr int PG_MAX_J = 64;  // ne * nc of the supported (d, k)
__global__ void __launch_bounds__(256) pgalerkin_rows_kernel(int d, int ne, long nelem, const double* __restrict__ Jp,
                                                        const double* __restrict__ Af, double* __restrict__ Ac) {
  extern __shared__ double sT[];  // [256 / nl][nl][ncl]
  __shared__ double sJ[PG_MAX_J];
  const int nc = 1 << (d - 1);
  const int nl = 2 * d * ne, ncl = 2 * d * nc;
  const int epw = 256 / nl;
  const long T0 = blockIdx.x * (long)epw;
  const int tid = threadIdx.x;
  for (int i = tid; i < ne * nc; i += 256) sJ[i] = Jp[i];
  __syncthreads();
  {
    const int e = tid / nl, r = tid % nl;
    if (e < epw && T0 + e < nelem) {
      const double* row = Af + ((T0 + e) * nl + r) * (long)nl;
      double* trow = sT + (e * nl + r) * ncl;
      for (int s2 = 0; s2 < 2 * d; ++s2) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b = 0; b < ne; ++b) {
          const double x = row[s2 * ne + b];
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (v < nc) acc[v] += x * sJ[b * nc + v];
        }
        for (int v = 0; v < nc; ++v) trow[s2 * nc + v] = acc[v];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < epw * ncl * ncl; idx += 256) {
    const int e = idx / (ncl * ncl), rr = idx % (ncl * ncl);
    if (T0 + e >= nelem) break;
    const int I = rr / ncl, J = rr % ncl, s1 = I / nc, v1 = I % nc;
    double s = 0.0;
    for (int a = 0; a < ne; ++a) s += sJ[a * nc + v1] * sT[(e * nl + s1 * ne + a) * ncl + J];
    Ac[(T0 + e) * ncl * ncl + rr] = s;
  }
}

template <int N>
__device__ void gj_lds(double* A, int tid, int nt) {
  __shared__ double pv;
  for (int k = 0; k < N; ++k) {
    __syncthreads();
    if (tid == 0) pv = 1.0 / A[k * N + k];
    __syncthreads();
    const double p = pv;
    for (int j = tid; j < N; j += nt)
      if (j != k) A[k * N + j] *= p;
    __syncthreads();
    for (int idx = tid; idx < N * N; idx += nt) {
      const int i = idx / N, j = idx % N;
      if (i != k && j != k) A[idx] -= A[i * N + k] * A[k * N + j];
    }
    __syncthreads();
    for (int i = tid; i < N; i += nt)
      if (i != k) A[i * N + k] = -A[i * N + k] * p;
    if (tid == 0) A[k * N + k] = p;
  }
  __syncthreads();
}

// one workgroup per coarse macro-element
template <int D, int NT>
__global__ void __launch_bounds__(NT) macro_schur_kernel(int n, const double* __restrict__ Achild,
                                                         double* __restrict__ Acoarse, double* __restrict__ Ai64,
                                                         float* __restrict__ Ai32, double* __restrict__ P64,
                                                         float* __restrict__ P32, double* __restrict__ R64,
                                                         float* __restrict__ R32) {
  constexpr int NC = 1 << (D - 1);    // DOFs per (sub)face
  constexpr int NS = NC;              // sub-faces per macro-face
  constexpr int NLC = 2 * D * NC;     // child local size == coarse local size
  constexpr int NI = D * NS * NC;     // interior DOFs of the macro-element
  constexpr int NB = 2 * D * NS * NC; // boundary DOFs of the macro-element
  __shared__ double sII[NI * NI];
  __shared__ double sIB[NI * NB];
  __shared__ double sBB[NB * NB];
  __shared__ double sY[NI * NLC];
  __shared__ int map[(1 << D) * NLC];
  __shared__ int bsrc[NB];      // B DOF -> (child, child-local DOF) that holds it
  __shared__ int isrc[2 * NI];  // I DOF -> its two (child, child-local DOF)
  constexpr int CB = 32;        // 3D: columns of A_IB per matrix-core block
  __shared__ double sX[D == 3 ? NI * CB : 1];
  const bool nonsym = R64 != nullptr;
  const int tid = threadIdx.x;
  const int nm = n / 2;
  const long M = blockIdx.x;
  int m[3] = {0, 0, 0};
  {
    long r = M;
    for (int a = 0; a < D; ++a) {
      m[a] = (int)(r % nm);
      r /= nm;
    }
  }
  // child-local DOF -> macro DOF (>= 0: I index, < 0: -(B index) - 1)
  for (int idx = tid; idx < (1 << D) * NLC; idx += NT) {
    const int ch = idx / NLC, l = idx % NLC;
    const int sl = l / NC, v = l % NC;
    const int c = sl / 2, sd = sl % 2;
    const int q = ((ch >> c) & 1) + sd;  // position inside the macro-element along c
    int t = 0, j = 0;
    for (int a = 0; a < D; ++a)
      if (a != c) {
        t |= ((ch >> a) & 1) << j;
        ++j;
      }
    if (q == 1) {
      map[idx] = (c * NS + t) * NC + v;
      isrc[2 * map[idx] + ((ch >> c) & 1)] = idx;
    } else {
      map[idx] = -(((2 * c + (q == 2 ? 1 : 0)) * NS + t) * NC + v) - 1;
      bsrc[-map[idx] - 1] = idx;
    }
  }
  auto child_elem = [&](int ch) {
    long T = 0;
    for (int a = D - 1; a >= 0; --a) T = T * n + 2 * m[a] + ((ch >> a) & 1);
    return T;
  };
  for (int idx = tid; idx < NI * NI; idx += NT) sII[idx] = 0.0;
  for (int idx = tid; idx < NI * NB; idx += NT) sIB[idx] = 0.0;
  for (int idx = tid; idx < NB * NB; idx += NT) sBB[idx] = 0.0;
  __syncthreads();
  for (int ch = 0; ch < (1 << D); ++ch) {
    int e[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) e[a] = 2 * m[a] + ((ch >> a) & 1);
    long T = 0;
    for (int a = D - 1; a >= 0; --a) T = T * n + e[a];
    const double* Ac = Achild + T * NLC * NLC;
    for (int idx = tid; idx < NLC * NLC; idx += NT) {
      const int r = idx / NLC, s = idx % NLC;
      const int mr = map[ch * NLC + r], ms = map[ch * NLC + s];
      const double v = Ac[idx];
      if (mr >= 0 && ms >= 0)
        sII[mr * NI + ms] += v;
      else if (mr >= 0 && ms < 0)
        sIB[mr * NB + (-ms - 1)] += v;
      else if (mr < 0 && ms < 0)
        sBB[(-mr - 1) * NB + (-ms - 1)] += v;
    }
    __syncthreads();
  }
  if constexpr (NI % 16 == 0)
    gj_inverse_blocked<NI, NT>(sII);
  else
    gj_lds<NI>(sII, tid, NT);
  // J: coarse DOF (S, V) -> B DOF (S*NS + t, v) with weight jw(t, v, V)
  auto jw = [](int t, int v, int V) {
    double w = 1.0;
    for (int j = 0; j < D - 1; ++j) {
      double s = 0.5 * (((t >> j) & 1) + ((v >> j) & 1));
      w *= ((V >> j) & 1) ? s : 1.0 - s;
    }
    return w;
  };
  // Y = A_IB J  (NI x NLC)
  for (int idx = tid; idx < NI * NLC; idx += NT) {
    const int i = idx / NLC, J = idx % NLC;
    const int S = J / NC, V = J % NC;
    double s = 0.0;
    for (int t = 0; t < NS; ++t)
      for (int v = 0; v < NC; ++v) s += sIB[i * NB + (S * NS + t) * NC + v] * jw(t, v, V);
    sY[idx] = s;
  }
  __syncthreads();
  // P = -A_II^-1 Y, written AoSoA over macro-elements
  for (int idx = tid; idx < NI * NLC; idx += NT) {
    const int i = idx / NLC, J = idx % NLC;
    double s = 0.0;
    for (int l = 0; l < NI; ++l) s += sII[i * NI + l] * sY[l * NLC + J];
    P64[aos_off<double>(M, vpad<double>(NI * NLC), idx)] = -s;
    P32[aos_off<float>(M, vpad<float>(NI * NLC), idx)] = (float)(-s);
  }
  for (int idx = tid; idx < NI * NI; idx += NT) {
    Ai64[aos_off<double>(M, vpad<double>(NI * NI), idx)] = sII[idx];
    Ai32[aos_off<float>(M, vpad<float>(NI * NI), idx)] = (float)sII[idx];
  }
  __syncthreads();
  if constexpr (D == 3) {
    // by blocks of CB columns on the matrix cores: X = A_II^-1 A_IB(:, block),
    // then S(:, block) = A_BB - A_IB^T X (symmetric levels) or X written back
    // in place of A_IB(:, block) (nonsymmetric levels: Z = A_II^-1 A_IB)
    static_assert(NB % CB == 0, "whole column blocks");
    for (int j0 = 0; j0 < NB; j0 += CB) {
      wg_mfma<NI, CB, NI, NT>([&](int i, int l) { return sII[i * NI + l]; },
                              [&](int l, int j) { return sIB[l * NB + j0 + j]; },
                              [&](int i, int j, double v) { sX[i * CB + j] = v; });
      __syncthreads();
      if (!nonsym)
        wg_mfma<NB, CB, NI, NT>([&](int i, int l) { return sIB[l * NB + i]; },
                                [&](int l, int j) { return sX[l * CB + j]; },
                                [&](int i, int j, double v) { sBB[i * NB + j0 + j] -= v; });
      else
        for (int idx = tid; idx < NI * CB; idx += NT) sIB[(idx / CB) * NB + j0 + idx % CB] = sX[idx];
      __syncthreads();
    }
  } else if (!nonsym) {
    // S = A_BB - A_IB^T A_II^-1 A_IB, column j owned by one thread
    for (int j = tid; j < NB; j += NT) {
      double x[NI];
      for (int i = 0; i < NI; ++i) {
        double s = 0.0;
        for (int l = 0; l < NI; ++l) s += sII[i * NI + l] * sIB[l * NB + j];
        x[i] = s;
      }
      for (int i = 0; i < NB; ++i) {
        double s = 0.0;
        for (int l = 0; l < NI; ++l) s += sIB[l * NB + i] * x[l];
        sBB[i * NB + j] -= s;
      }
    }
  } else {
    // Z = A_II^-1 A_IB in place of A_IB, one column per thread
    for (int j = tid; j < NB; j += NT) {
      double x[NI];
      for (int i = 0; i < NI; ++i) {
        double s = 0.0;
        for (int l = 0; l < NI; ++l) s += sII[i * NI + l] * sIB[l * NB + j];
        x[i] = s;
      }
      for (int i = 0; i < NI; ++i) sIB[i * NB + j] = x[i];
    }
  }
  if (nonsym) {
    __syncthreads();
    // S = A_BB - A_BI Z: row i of A_BI lives in the one child that holds B DOF i
    for (int idx = tid; idx < NB * NB; idx += NT) {
      const int i = idx / NB, j = idx % NB;
      const int ch = bsrc[i] / NLC, r = bsrc[i] % NLC;
      const double* Ac = Achild + child_elem(ch) * NLC * NLC + r * NLC;
      double s = 0.0;
      for (int l = 0; l < NLC; ++l) {
        const int ms = map[ch * NLC + l];
        if (ms >= 0) s += Ac[l] * sIB[ms * NB + j];
      }
      sBB[idx] -= s;
    }
    // Y2 = A_BI^T J (into Y): column l of A_BI gathers the B rows of the two
    // children that hold I DOF l
    for (int idx = tid; idx < NI * NLC; idx += NT) {
      const int l = idx / NLC, J = idx % NLC;
      const int S = J / NC, V = J % NC;
      double s = 0.0;
      for (int side = 0; side < 2; ++side) {
        const int ch = isrc[2 * l + side] / NLC, cl = isrc[2 * l + side] % NLC;
        const double* Ac = Achild + child_elem(ch) * NLC * NLC;
        for (int r = 0; r < NLC; ++r) {
          const int mr = map[ch * NLC + r];
          if (mr >= 0) continue;
          const int i = -mr - 1;
          if (i / (NS * NC) != S) continue;
          s += Ac[r * NLC + cl] * jw((i / NC) % NS, i % NC, V);
        }
      }
      sY[idx] = s;
    }
    __syncthreads();
    // R = -A_II^-T Y2, written AoSoA over macro-elements like P
    for (int idx = tid; idx < NI * NLC; idx += NT) {
      const int i = idx / NLC, J = idx % NLC;
      double s = 0.0;
      for (int l = 0; l < NI; ++l) s += sII[l * NI + i] * sY[l * NLC + J];
      R64[aos_off<double>(M, vpad<double>(NI * NLC), idx)] = -s;
      R32[aos_off<float>(M, vpad<float>(NI * NLC), idx)] = (float)(-s);
    }
  }
  __syncthreads();
  // T1 = S J (NB x NLC) into sIB, then A_coarse = J^T T1
  for (int idx = tid; idx < NB * NLC; idx += NT) {
    const int i = idx / NLC, J = idx % NLC;
    const int S = J / NC, V = J % NC;
    double s = 0.0;
    for (int t = 0; t < NS; ++t)
      for (int v = 0; v < NC; ++v) s += sBB[i * NB + (S * NS + t) * NC + v] * jw(t, v, V);
    sIB[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < NLC * NLC; idx += NT) {
    const int I = idx / NLC, J = idx % NLC;
    const int S = I / NC, V = I % NC;
    double s = 0.0;
    for (int t = 0; t < NS; ++t)
      for (int v = 0; v < NC; ++v) s += jw(t, v, V) * sIB[((S * NS + t) * NC + v) * NLC + J];
    Acoarse[M * NLC * NLC + idx] = s;
  }
}

// dense assembly and inverse of the coarsest operator (n = 2), one workgroup
__global__ void coarse_inverse_kernel(int d, int n, int ne, int N, const double* __restrict__ Aelem,
                                      double* __restrict__ Ai64, float* __restrict__ Ai32) {
  __shared__ double A[64 * 64];
  __shared__ double pv;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nl = 2 * d * ne;
  long nelem = 1;
  for (int a = 0; a < d; ++a) nelem *= n;
  for (int idx = tid; idx < N * N; idx += nt) A[idx] = 0.0;
  __syncthreads();
  for (long T = 0; T < nelem; ++T) {
    int e[3] = {0, 0, 0};
    long r = T;
    for (int a = 0; a < d; ++a) {
      e[a] = (int)(r % n);
      r /= n;
    }
    for (int idx = tid; idx < nl * nl; idx += nt) {
      const int i = idx / nl, j = idx % nl;
      long gi = -1, gj = -1;
      for (int pass = 0; pass < 2; ++pass) {
        const int l = pass == 0 ? i : j;
        const int sl = l / ne, a = l % ne;
        const int c = sl / 2, sd = sl % 2;
        const int p = e[c] + sd;
        long gid = -1;
        if (p > 0 && p < n) {
          int g[3] = {e[0], e[1], e[2]};
          g[c] = p;
          long idx2 = 0, stride = 1;
          for (int aa = 0; aa < d; ++aa) {
            if (aa == c) {
              idx2 += (long)(g[aa] - 1) * stride;
              stride *= n - 1;
            } else {
              idx2 += (long)g[aa] * stride;
              stride *= n;
            }
          }
          gid = (c * nfd_of(d, n) + idx2) * ne + a;
        }
        if (pass == 0)
          gi = gid;
        else
          gj = gid;
      }
      if (gi >= 0 && gj >= 0) A[gi * N + gj] += Aelem[(T * nl + i) * nl + j];
    }
    __syncthreads();
  }
  for (int k = 0; k < N; ++k) {
    __syncthreads();
    if (tid == 0) pv = 1.0 / A[k * N + k];
    __syncthreads();
    const double p = pv;
    for (int j = tid; j < N; j += nt)
      if (j != k) A[k * N + j] *= p;
    __syncthreads();
    for (int idx = tid; idx < N * N; idx += nt) {
      const int i = idx / N, j = idx % N;
      if (i != k && j != k) A[idx] -= A[i * N + k] * A[k * N + j];
    }
    __syncthreads();
    for (int i = tid; i < N; i += nt)
      if (i != k) A[i * N + k] = -A[i * N + k] * p;
    if (tid == 0) A[k * N + k] = p;
  }
  __syncthreads();
  for (int idx = tid; idx < N * N; idx += nt) {
    Ai64[idx] = A[idx];
    Ai32[idx] = (float)A[idx];
  }
}

// Dense assembly of a level operator: elements of one colour (parity of
// their coordinates) share no face, so a pass adds without conflicts.
__global__ void dense_assemble_kernel(int d, int n, int ne, int color, long N, const double* __restrict__ Aelem,
                                      double* __restrict__ A) {
  const int nl = 2 * d * ne;
  long nelem = 1;
  for (int a = 0; a < d; ++a) nelem *= n;
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= nelem * nl * nl) return;
  const long T = t / (nl * nl);
  const int ij = (int)(t % (nl * nl));
  int e[3] = {0, 0, 0};
  long r = T;
  int col = 0;
  for (int a = 0; a < d; ++a) {
    e[a] = (int)(r % n);
    r /= n;
    col |= (e[a] & 1) << a;
  }
  if (col != color) return;
  long gid[2];
  const int loc[2] = {ij / nl, ij % nl};
  for (int pass = 0; pass < 2; ++pass) {
    const int l = loc[pass];
    const int sl = l / ne, a = l % ne;
    const int c = sl / 2, sd = sl % 2;
    const int p = e[c] + sd;
    gid[pass] = -1;
    if (p > 0 && p < n) {
      long idx2 = 0, stride = 1;
      for (int aa = 0; aa < d; ++aa) {
        const int g = aa == c ? p : e[aa];
        if (aa == c) {
          idx2 += (long)(g - 1) * stride;
          stride *= n - 1;
        } else {
          idx2 += (long)g * stride;
          stride *= n;
        }
      }
      gid[pass] = (c * nfd_of(d, n) + idx2) * ne + a;
    }
  }
  if (gid[0] >= 0 && gid[1] >= 0) A[gid[0] * N + gid[1]] += Aelem[T * nl * nl + ij];
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) b[i] = (float)a[i];
}

// Ap[T][e] for the packed upper triangle (i <= j, row by row) of the
// symmetrised element map (A + A^T) / 2, AoSoA over elements
__global__ void pack_sym_kernel(long nelem, int nl, const double* __restrict__ Aelem, double* __restrict__ Ap64,
                                float* __restrict__ Ap32) {
  const int npk = nl * (nl + 1) / 2;
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= nelem * npk) return;
  const long T = t / npk;
  int e = (int)(t % npk);
  int i = 0;
  while (e >= nl - i) {
    e -= nl - i;
    ++i;
  }
  const int j = i + e;
  const double* A = Aelem + T * (long)nl * nl;
  const double v = 0.5 * (A[i * nl + j] + A[j * nl + i]);
  Ap64[pk_off<double>(T, npk, t % npk)] = v;
  Ap32[pk_off<float>(T, npk, t % npk)] = (float)v;
}

}  // namespace

void launch_pack_sym(const Level& L, hipStream_t st) {
  const long npk = (long)L.nl * (L.nl + 1) / 2;
  hipLaunchKernelGGL(pack_sym_kernel, dim3(nblk(L.nelem * npk)), dim3(256), 0, st, L.nelem, L.nl, L.Aelem, L.Ap64,
                     L.Ap32);
  HDG_CHECK(hipGetLastError());
}

void launch_face_major(const Level& L, hipStream_t st) {
  if (L.nface == 0) return;
  long tot = L.nface * 2L * L.nl * L.ne;
  hipLaunchKernelGGL(face_major_kernel, dim3(nblk(tot)), dim3(256), 0, st, L.d, L.n, L.ne, L.nface, L.Aelem,
                     L.Af64, L.Af32);
  HDG_CHECK(hipGetLastError());
}

void launch_dinv(const Level& L, double omega, hipStream_t st, int mode) {
  if (L.nface == 0) return;
  if (mode != 0 && L.packed) throw HipError{hipErrorInvalidValue, "point smoother data: face-major levels only"};
#define HDG_DCASE(NN)                                                                                     \
  case NN:                                                                                                \
    hipLaunchKernelGGL((dinv_kernel<NN>), dim3(nblk(L.nface)), dim3(256), 0, st, L.d, L.n, L.nface, omega, \
                       L.Aelem, L.Dinv64, L.Dinv32, L.packed ? 1 : 0, mode);                              \
    break;
  switch (L.ne) {
    HDG_DCASE(2) HDG_DCASE(3) HDG_DCASE(4) HDG_DCASE(5) HDG_DCASE(6) HDG_DCASE(7) HDG_DCASE(9) HDG_DCASE(16)
    default:
      throw HipError{hipErrorInvalidValue, "unsupported face size"};
  }
#undef HDG_DCASE
  HDG_CHECK(hipGetLastError());
}

void launch_pgalerkin(int d, int ne, long nelem, const double* Jp, const double* Afine, double* Acoarse,
                      hipStream_t st) {
  const int nc = 1 << (d - 1), ncl = 2 * d * nc, nl = 2 * d * ne;
  if (nelem <= 0) return;
  if (d == 2) {
    hipLaunchKernelGGL(pgalerkin_kernel, dim3(nblk(nelem * ncl * ncl)), dim3(256), 0, st, d, ne, nelem, Jp, Afine,
                       Acoarse);
  } else {
    if (nl > 256 || ne * nc > PG_MAX_J) throw HipError{hipErrorInvalidValue, "p-Galerkin: element too large"};
    const int epw = 256 / nl;
    const long nb = (nelem + epw - 1) / epw;
    const size_t lds = (size_t)epw * nl * ncl * sizeof(double);
    hipLaunchKernelGGL(pgalerkin_rows_kernel, dim3((unsigned)nb), dim3(256), lds, st, d, ne, nelem, Jp, Afine,
                       Acoarse);
  }
  HDG_CHECK(hipGetLastError());
}

void launch_macro_schur(const Level& fine, Level& coarse, hipStream_t st) {
  if (fine.d == 2)
    hipLaunchKernelGGL((macro_schur_kernel<2, 64>), dim3((unsigned)fine.nmacro), dim3(64), 0, st, fine.n,
                       fine.Aelem, coarse.Aelem, fine.AIIinv64, fine.AIIinv32, fine.P64, fine.P32,
                       fine.sym ? nullptr : fine.R64, fine.sym ? nullptr : fine.R32);
  else
    hipLaunchKernelGGL((macro_schur_kernel<3, 256>), dim3((unsigned)fine.nmacro), dim3(256), 0, st, fine.n,
                       fine.Aelem, coarse.Aelem, fine.AIIinv64, fine.AIIinv32, fine.P64, fine.P32,
                       fine.sym ? nullptr : fine.R64, fine.sym ? nullptr : fine.R32);
  HDG_CHECK(hipGetLastError());
}

void launch_coarse_inverse(const Level& L, hipStream_t st) {
  if (L.nlam == 0) return;
  if (L.nlam > 64) {
    // dense assembly, then the blocked Gauss-Jordan inverse (FP64)
    const long N = L.nlam;
    double *A = nullptr, *B = nullptr;
    HDG_CHECK(hipMalloc((void**)&A, sizeof(double) * N * N));
    HDG_CHECK(hipMalloc((void**)&B, sizeof(double) * N * N));
    HDG_CHECK(hipMemsetAsync(A, 0, sizeof(double) * N * N, st));
    const long tot = L.nelem * L.nl * L.nl;
    for (int color = 0; color < (1 << L.d); ++color)
      hipLaunchKernelGGL(dense_assemble_kernel, dim3(nblk(tot)), dim3(256), 0, st, L.d, L.n, L.ne, color, N, L.Aelem,
                         A);
    launch_dense_inverse_blocked(N, A, B, st);  // B (N * N >= 4,096 doubles) holds the pivot blocks
    HDG_CHECK(hipMemcpyAsync(L.Ainv64, A, sizeof(double) * N * N, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, st, A, L.Ainv32, N * N);
    HDG_CHECK(hipGetLastError());
    HDG_CHECK(hipStreamSynchronize(st));
    HDG_CHECK(hipFree(A));
    HDG_CHECK(hipFree(B));
    return;
  }
  hipLaunchKernelGGL(coarse_inverse_kernel, dim3(1), dim3(256), 0, st, L.d, L.n, L.ne, (int)L.nlam, L.Aelem,
                     L.Ainv64, L.Ainv32);
  HDG_CHECK(hipGetLastError());
}

}  // namespace hdg

namespace hdg {
void launch_scale_copy(long n, double s, const double* src, double* d64, float* d32, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, s, src, d64, d32);
  HDG_CHECK(hipGetLastError());
}
}  // namespace hdg
