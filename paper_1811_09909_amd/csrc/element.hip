// Element-local kernels of the HDG discretization (gfx950).
//
// For each element T the local problem of eqs. HDG / HDG_flux reads
//   A_T Q - B^T U + F Lambda = 0,      B Q + tau E U = tau G Lambda + b_T,
// with A_T = blockdiag_c(Mk), Mk = (kappa^-1 phi_j, phi_i)_T, B = [B_c],
// B_c[i][j] = (d_c phi_j, phi_i), F = [F_c], G, E, H the face integrals.
// Eliminating Q with the SPD blocks Mk gives the SPD volume Schur complement
//   K = sum_c B_c Mk^-1 B_c^T + tau E,   Z = tau G + sum_c B_c Mk^-1 F_c,
// and the element DtN map of the condensed trace system (Sec. 2, static
// condensation; eq. trace_linear_system):
//   A^e = tau H + sum_c F_c^T Mk^-1 F_c - Z^T K^-1 Z,   b^e = (K^-1 Z)^T b_T.
// Local recovery: U = K^-1 (Z Lambda + b), Q_c = Mk^-1 (B_c^T U - F_c Lambda).
// F_c only touches the two face slots of normal c, which keeps the LDS
// footprint of a 3D k=3 element at 144 KB.
#include "hdg_internal.hpp"
#include "mfma_dev.hpp"

namespace hdg {

namespace {

template <int D, int K>
struct Dims {
  static constexpr int P1 = K + 1;
  static constexpr int NV = D == 2 ? P1 * P1 : P1 * P1 * P1;
  static constexpr int NE = D == 2 ? P1 : P1 * P1;
  static constexpr int NF = 2 * D;
  static constexpr int NL = NF * NE;
  static constexpr int NQ = D == 2 ? (K + 2) * (K + 2) : (K + 2) * (K + 2) * (K + 2);
  static constexpr int SA = (2 * NV * NV > NV * NL) ? 2 * NV * NV : NV * NL;
};

// In-place Gauss-Jordan inverse of an SPD N x N matrix in LDS (no
// pivoting) with the matrix held in registers: lane (ti, tj) of a G x G lane
// grid (G * G = NT) owns the BS x BS block at rows ti * BS, columns tj * BS
// (BS = ceil(N / G); entries past N act as identity).  Each step publishes
// the pivot row and column through LDS, double-buffered, so one barrier per
// step suffices; every lane then updates its own block.
template <int N, int NT>
__device__ void gj_inverse_reg(double* A) {
  static_assert(NT == 64 || NT == 256, "lane grid of 8 x 8 or 16 x 16");
  constexpr int G = NT == 64 ? 8 : 16;
  constexpr int BS = (N + G - 1) / G;
  __shared__ double rowb[2][G * BS], colb[2][G * BS];
  const int tid = threadIdx.x, ti = tid / G, tj = tid % G;
  double a[BS][BS];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < BS; ++r)
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int i = ti * BS + r, j = tj * BS + c;
      a[r][c] = (i < N && j < N) ? A[i * N + j] : (i == j ? 1.0 : 0.0);
    }
  for (int k = 0; k < N; ++k) {
    const int buf = k & 1, kb = k / BS, kr = k % BS;
    if (ti == kb)
#pragma unroll
      for (int c = 0; c < BS; ++c)
#pragma unroll
        for (int r = 0; r < BS; ++r)
          if (r == kr) rowb[buf][tj * BS + c] = a[r][c];
    if (tj == kb)
#pragma unroll
      for (int r = 0; r < BS; ++r)
#pragma unroll
        for (int c = 0; c < BS; ++c)
          if (c == kr) colb[buf][ti * BS + r] = a[r][c];
    __syncthreads();
    const double p = 1.0 / rowb[buf][k];
#pragma unroll
    for (int r = 0; r < BS; ++r) {
      const int i = ti * BS + r;
      const double ci = colb[buf][i];
#pragma unroll
      for (int c = 0; c < BS; ++c) {
        const int j = tj * BS + c;
        const double rj = rowb[buf][j] * p;
        if (i == k)
          a[r][c] = j == k ? p : rj;
        else if (j == k)
          a[r][c] = -ci * p;
        else
          a[r][c] -= ci * rj;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < BS; ++r)
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int i = ti * BS + r, j = tj * BS + c;
      if (i < N && j < N) A[i * N + j] = a[r][c];
    }
  __syncthreads();
}

// the blocked form where the size allows it (3D, k = 3: 64 x 64)
template <int N, int NT>
__device__ inline void gj_inverse(double* A) {
  if constexpr (N % 16 == 0 && N >= 32 && NT >= 64)
    gj_inverse_blocked<N, NT>(A);
  else
    gj_inverse_reg<N, NT>(A);
}

// lanes per element of the 2D element kernel
#ifndef HDG_ELEM_NT2
#define HDG_ELEM_NT2 256
#endif
// lanes per element of the 3D, k = 3 element kernels (HDG and IPDG)
#ifndef HDG_ELEM_NT3
#define HDG_ELEM_NT3 1024
#endif

// In 2D the Schur-complement route is followed by one step of iterative
// refinement on the full local system.  Forming A^e as
// tau H + F^T Mk^-1 F - Z^T K^-1 Z subtracts terms of size kappa to leave a
// result of size tau h, so its rounding error grows like eps kappa / (tau h)
// (4e-10 at kappa = 680, h = 1/512).  Instead the local solution
// X = [Q; U] = L^-1 R for every trace DOF is computed by that route, its
// residual R - L X is formed directly, one correction is solved by the same
// route, and A^e = tau H - S^T X = tau H - sum_c F_c^T Q_c - tau G^T U; the
// refined X is backward stable and A^e comes out to a few eps like a pivoted
// LU of L.  (3D elements keep the plain route: their LDS budget is spent, and
// the smooth 3D coefficient keeps kappa / (tau h) small.)
//
// Every dense product runs on the matrix cores (wg_mfma); the two
// Gauss-Jordan inverses stay on the vector units.  Mk^-1 and K^-1 are
// symmetric, so their rows are read as columns (consecutive lanes then read
// consecutive LDS words).
template <int D, int K, int NT>
__global__ void __launch_bounds__(NT) element_dtn_kernel(long nelem, double tau0, int tau_kappa,
                                                         const double* __restrict__ Phi,
                                                         const double* __restrict__ Wq,
                                                         const double* __restrict__ Bm,
                                                         const double* __restrict__ Fm,
                                                         const double* __restrict__ Gm,
                                                         const double* __restrict__ Em,
                                                         const double* __restrict__ Hm,
                                                         const double* __restrict__ kqp, double* __restrict__ Aelem,
                                                         double* __restrict__ Wout, double* __restrict__ Kinv_out,
                                                         double* __restrict__ Minv_out) {
  using Dm = Dims<D, K>;
  constexpr int NV = Dm::NV, NE = Dm::NE, NL = Dm::NL, NQ = Dm::NQ;
  constexpr int N2 = 2 * NE;
  constexpr bool REF = (D == 2);
  constexpr int NX = REF ? (D + 1) * NV * NL : 1;
  __shared__ double sA[Dm::SA];      // Mk^-1 | Y   (plain route, later: W)
  __shared__ double sK[NV * NV];     // K -> K^-1
  __shared__ double sZ[NV * NL];     // Z
  __shared__ double sW[NQ];          // w_q / kappa_q
  __shared__ double sX[NX];          // refined route: Q_0 .. Q_{D-1}, U  ([(D+1) NV][NL])
  __shared__ double sR[NX];          // refined route: residual / correction
  const long T = blockIdx.x;
  if (T >= nelem) return;
  const int tid = threadIdx.x;
  const double tau = tau_kappa ? tau0 * kqp[T * NQ] : tau0;  // tau_T = tau kappa_T (per-element kappa)
  double* sM = sA;
  double* sY = sA + NV * NV;
  double* Ae = Aelem + T * (long)NL * NL;

  for (int q = tid; q < NQ; q += NT) sW[q] = Wq[q] / kqp[T * NQ + q];
  __syncthreads();
  // Mk = Phi^T diag(w/kappa) Phi
  wg_mfma<NV, NV, NQ, NT>([&](int i, int q) { return Phi[q * NV + i] * sW[q]; },
                          [&](int q, int j) { return Phi[q * NV + j]; },
                          [&](int i, int j, double v) { sM[i * NV + j] = v; });
  // K = tau E, Z = tau G, A^e = tau H
  for (int idx = tid; idx < NV * NV; idx += NT) sK[idx] = tau * Em[idx];
  for (int idx = tid; idx < NV * NL; idx += NT) sZ[idx] = tau * Gm[idx];
  if (!REF)
    for (int idx = tid; idx < NL * NL; idx += NT) Ae[idx] = tau * Hm[idx];
  gj_inverse<NV, NT>(sM);
  if (Minv_out)
    for (int idx = tid; idx < NV * NV; idx += NT) Minv_out[T * NV * NV + idx] = sM[idx];

  for (int c = 0; c < D; ++c) {
    const double* Bc = Bm + (long)c * NV * NV;
    const double* Fc = Fm + (long)c * NV * NL;
    const int col0 = 2 * c * NE;
    // Y = Mk^-1 B_c^T ; K += B_c Y
    __syncthreads();
    wg_mfma<NV, NV, NV, NT>([&](int i, int l) { return sM[l * NV + i]; },
                            [&](int l, int j) { return Bc[j * NV + l]; },
                            [&](int i, int j, double v) { sY[i * NV + j] = v; });
    __syncthreads();
    wg_mfma<NV, NV, NV, NT>([&](int i, int l) { return Bc[i * NV + l]; },
                            [&](int l, int j) { return sY[l * NV + j]; },
                            [&](int i, int j, double v) { sK[i * NV + j] += v; });
    __syncthreads();
    // Y(:, 0:2NE) = Mk^-1 F_c(:, slots of normal c)
    wg_mfma<NV, N2, NV, NT>([&](int i, int l) { return sM[l * NV + i]; },
                            [&](int l, int j) { return Fc[l * NL + col0 + j]; },
                            [&](int i, int j, double v) { sY[i * N2 + j] = v; });
    __syncthreads();
    // Z(:, slots c) += B_c Y ; A^e(slots c, slots c) += F_c^T Y
    wg_mfma<NV, N2, NV, NT>([&](int i, int l) { return Bc[i * NV + l]; },
                            [&](int l, int j) { return sY[l * N2 + j]; },
                            [&](int i, int j, double v) { sZ[i * NL + col0 + j] += v; });
    if (!REF)
      wg_mfma<N2, N2, NV, NT>([&](int i, int l) { return Fc[l * NL + col0 + i]; },
                              [&](int l, int j) { return sY[l * N2 + j]; },
                              [&](int i, int j, double v) { Ae[(col0 + i) * NL + col0 + j] += v; });
  }
  __syncthreads();
  gj_inverse<NV, NT>(sK);
  if (Kinv_out)
    for (int idx = tid; idx < NV * NV; idx += NT) Kinv_out[T * NV * NV + idx] = sK[idx];
  if constexpr (!REF) {
    // W = K^-1 Z (into sA) ; A^e -= Z^T W
    double* sWm = sA;
    wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sK[l * NV + i]; },
                            [&](int l, int j) { return sZ[l * NL + j]; },
                            [&](int i, int j, double v) { sWm[i * NL + j] = v; });
    __syncthreads();
    wg_mfma<NL, NL, NV, NT>([&](int i, int l) { return sZ[l * NL + i]; },
                            [&](int l, int j) { return sWm[l * NL + j]; },
                            [&](int i, int j, double v) { Ae[i * NL + j] -= v; });
    for (int idx = tid; idx < NV * NL; idx += NT) Wout[T * NV * NL + idx] = sWm[idx];
  } else {
    double* sU = sX + D * NV * NL;
    double* rU = sR + D * NV * NL;
    // U = K^-1 Z
    wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sK[l * NV + i]; },
                            [&](int l, int j) { return sZ[l * NL + j]; },
                            [&](int i, int j, double v) { sU[i * NL + j] = v; });
    __syncthreads();
    // Q_c = Mk^-1 (B_c^T U - F_c)
    for (int c = 0; c < D; ++c) {
      const double* Bc = Bm + (long)c * NV * NV;
      const double* Fc = Fm + (long)c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return Bc[l * NV + i]; },
                              [&](int l, int j) { return sU[l * NL + j]; },
                              [&](int i, int j, double v) { sZ[i * NL + j] = v - Fc[i * NL + j]; });
      __syncthreads();
      double* Qc = sX + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sM[l * NV + i]; },
                              [&](int l, int j) { return sZ[l * NL + j]; },
                              [&](int i, int j, double v) { Qc[i * NL + j] = v; });
      __syncthreads();
    }
    // Mk itself again (into Y) for the residual
    wg_mfma<NV, NV, NQ, NT>([&](int i, int q) { return Phi[q * NV + i] * sW[q]; },
                            [&](int q, int j) { return Phi[q * NV + j]; },
                            [&](int i, int j, double v) { sY[i * NV + j] = v; });
    __syncthreads();
    // residual of the local system for R = [-F; tau G]:
    //   r_c = -F_c - Mk Q_c + B_c^T U,   r_u = tau G - sum_c B_c Q_c - tau E U
    // (each entry is accumulated by one lane, which reads back only its own
    // writes between the products)
    for (int c = 0; c < D; ++c) {
      const double* Bc = Bm + (long)c * NV * NV;
      const double* Fc = Fm + (long)c * NV * NL;
      const double* Qc = sX + c * NV * NL;
      double* rc = sR + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return Bc[l * NV + i]; },
                              [&](int l, int j) { return sU[l * NL + j]; },
                              [&](int i, int j, double v) { rc[i * NL + j] = v - Fc[i * NL + j]; });
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sY[l * NV + i]; },
                              [&](int l, int j) { return Qc[l * NL + j]; },
                              [&](int i, int j, double v) { rc[i * NL + j] -= v; });
    }
    wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return tau * Em[i * NV + l]; },
                            [&](int l, int j) { return sU[l * NL + j]; },
                            [&](int i, int j, double v) { rU[i * NL + j] = tau * Gm[i * NL + j] - v; });
    for (int c = 0; c < D; ++c) {
      const double* Bc = Bm + (long)c * NV * NV;
      const double* Qc = sX + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return Bc[i * NV + l]; },
                              [&](int l, int j) { return Qc[l * NL + j]; },
                              [&](int i, int j, double v) { rU[i * NL + j] -= v; });
    }
    __syncthreads();
    // correction by the same route: y_c = Mk^-1 r_c (in place via Z),
    // dU = K^-1 (r_u - sum_c B_c y_c), dQ_c = y_c + Mk^-1 B_c^T dU
    for (int c = 0; c < D; ++c) {
      double* rc = sR + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sM[l * NV + i]; },
                              [&](int l, int j) { return rc[l * NL + j]; },
                              [&](int i, int j, double v) { sZ[i * NL + j] = v; });
      __syncthreads();
      for (int idx = tid; idx < NV * NL; idx += NT) rc[idx] = sZ[idx];
      __syncthreads();
    }
    for (int c = 0; c < D; ++c) {
      const double* Bc = Bm + (long)c * NV * NV;
      const double* yc = sR + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return Bc[i * NV + l]; },
                              [&](int l, int j) { return yc[l * NL + j]; },
                              [&](int i, int j, double v) { sZ[i * NL + j] = (c == 0 ? rU[i * NL + j] : sZ[i * NL + j]) - v; });
    }
    __syncthreads();
    wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sK[l * NV + i]; },
                            [&](int l, int j) { return sZ[l * NL + j]; },
                            [&](int i, int j, double v) { rU[i * NL + j] = v; });  // dU
    __syncthreads();
    for (int c = 0; c < D; ++c) {
      const double* Bc = Bm + (long)c * NV * NV;
      // t = B_c^T dU (into Z), then Q_c += y_c + Mk^-1 t
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return Bc[l * NV + i]; },
                              [&](int l, int j) { return rU[l * NL + j]; },
                              [&](int i, int j, double v) { sZ[i * NL + j] = v; });
      __syncthreads();
      double* Qc = sX + c * NV * NL;
      const double* yc = sR + c * NV * NL;
      wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sM[l * NV + i]; },
                              [&](int l, int j) { return sZ[l * NL + j]; },
                              [&](int i, int j, double v) { Qc[i * NL + j] += yc[i * NL + j] + v; });
      __syncthreads();
    }
    for (int idx = tid; idx < NV * NL; idx += NT) sU[idx] += rU[idx];
    __syncthreads();
    // A^e = tau H - tau G^T U - sum_c F_c^T Q_c
    wg_mfma<NL, NL, NV, NT>([&](int i, int l) { return tau * Gm[l * NL + i]; },
                            [&](int l, int j) { return sU[l * NL + j]; },
                            [&](int i, int j, double v) { Ae[i * NL + j] = tau * Hm[i * NL + j] - v; });
    for (int c = 0; c < D; ++c) {
      const double* Fc = Fm + (long)c * NV * NL;
      const double* Qc = sX + c * NV * NL;
      wg_mfma<NL, NL, NV, NT>([&](int i, int l) { return Fc[l * NL + i]; },
                              [&](int l, int j) { return Qc[l * NL + j]; },
                              [&](int i, int j, double v) { Ae[i * NL + j] -= v; });
    }
    for (int idx = tid; idx < NV * NL; idx += NT) Wout[T * NV * NL + idx] = sU[idx];
  }
}

// Element maps of the hybridized IPDG family (eq. IPG_H), one workgroup per
// element.  With kappa the element's value (face terms included) and
// s_f = 1, 0, -1 for SIPG-H, IIPG-H, NIPG-H, rows for the test function:
//   L = kappa (K - s_f N - N^T) + tau E,   R = tau G - s_f kappa D,
//   C = tau G^T - kappa D^T                (the conservation rows),
//   A^e = tau H - C L^-1 R,  load map W = L^-T C^T (b^e = W^T b),
//   recovery X = L^-1 R (u = X Lambda + L^-1 b).
// At tau = (p+1)(p+2)/h_min the symmetric part of L is positive definite
// for every s_f, so every leading minor of L is nonzero and Gauss-Jordan
// without pivoting applies.  The products run on the matrix cores; the
// operands R and C^T are formed as they are read.
template <int D, int K, int NT>
__global__ void __launch_bounds__(NT) ipdg_dtn_kernel(long nelem, const int* __restrict__ mask, int code,
                                                      double tau0, int tau_kappa, double sf, int nq,
                                                      const double* __restrict__ kqp,
                                                      const double* __restrict__ Kst,
                                                      const double* __restrict__ Nn,
                                                      const double* __restrict__ Dn,
                                                      const double* __restrict__ Gm,
                                                      const double* __restrict__ Em,
                                                      const double* __restrict__ Hm, double* __restrict__ Aelem,
                                                      double* __restrict__ Wout, double* __restrict__ Xout,
                                                      double* __restrict__ Linv_out) {
  using Dm = Dims<D, K>;
  constexpr int NV = Dm::NV, NL = Dm::NL;
  __shared__ double sL[NV * NV];  // L -> L^-1
  __shared__ double sX[NV * NL];  // X = L^-1 R
  const long T = blockIdx.x;
  if (T >= nelem) return;
  if (mask && mask[T] != code) return;
  const int tid = threadIdx.x;
  const double kap = kqp[T * nq];
  const double tau = tau_kappa ? tau0 * kap : tau0;
  double* Ae = Aelem + T * (long)NL * NL;
  for (int idx = tid; idx < NV * NV; idx += NT) {
    const int i = idx / NV, j = idx % NV;
    sL[idx] = kap * (Kst[idx] - sf * Nn[idx] - Nn[j * NV + i]) + tau * Em[idx];
  }
  gj_inverse<NV, NT>(sL);
  if (Linv_out)
    for (int idx = tid; idx < NV * NV; idx += NT) Linv_out[T * NV * NV + idx] = sL[idx];
  wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sL[i * NV + l]; },
                          [&](int l, int j) { return tau * Gm[l * NL + j] - sf * kap * Dn[l * NL + j]; },
                          [&](int i, int j, double v) { sX[i * NL + j] = v; });
  __syncthreads();
  if (Xout)
    for (int idx = tid; idx < NV * NL; idx += NT) Xout[T * NV * NL + idx] = sX[idx];
  wg_mfma<NL, NL, NV, NT>([&](int i, int l) { return tau * Gm[l * NL + i] - kap * Dn[l * NL + i]; },
                          [&](int l, int j) { return sX[l * NL + j]; },
                          [&](int i, int j, double v) { Ae[i * NL + j] = tau * Hm[i * NL + j] - v; });
  wg_mfma<NV, NL, NV, NT>([&](int i, int l) { return sL[l * NV + i]; },
                          [&](int l, int j) { return tau * Gm[l * NL + j] - kap * Dn[l * NL + j]; },
                          [&](int i, int j, double v) { Wout[(T * NV + i) * NL + j] = v; });
}

// Element maps of the hybridized Raviart-Thomas method (eqs. mixed_local1/2,
// d = 2), one workgroup per element.  The local system in (Q, U),
//   L = [[Mq, -Bd], [Bd^T, 0]],  R = [-Fr; 0],  S = [Fr; 0],
// Mq = blockdiag_c(Vq_c^T diag(w / kappa) Vq_c), is inverted in LDS
// (Gauss-Jordan in the natural order: the Mq pivots, then those of
// Bd^T Mq^-1 Bd, all positive), and with L^-1 = [[Lqq, Lqu], [Luq, Luu]]:
//   A^e = -S^T L^-1 R = Fr^T Lqq Fr,       load map W = Lqu^T Fr,
//   u = Xr Lambda + Luu b,  Xr = -Luq Fr,
//   flux at the nodes  Xq Lambda + Yq b,  Xq = -Vn Lqq Fr,  Yq = Vn Lqu,
// Vn the velocity basis at the scalar's nodes.  `mask`: element scheme codes
// (only elements with code `code` are formed), or null for all.
template <int K, int NT>
__global__ void __launch_bounds__(NT) rt_dtn_kernel(long nelem, const int* __restrict__ mask, int code,
                                                    const double* __restrict__ Wq, const double* __restrict__ kqp,
                                                    const double* __restrict__ Vq, const double* __restrict__ Bd,
                                                    const double* __restrict__ Fr, const double* __restrict__ Vn,
                                                    double* __restrict__ Aelem, double* __restrict__ Wout,
                                                    double* __restrict__ Xr, double* __restrict__ Luu_out,
                                                    double* __restrict__ Xq, double* __restrict__ Yq) {
  using Dm = Dims<2, K>;
  constexpr int NV = Dm::NV, NL = Dm::NL, NQ = Dm::NQ;
  constexpr int NQC = (K + 2) * (K + 1), NQV = 2 * NQC, N = NQV + NV;
  __shared__ double sL[N * N];       // L -> L^-1
  __shared__ double sT[NQV * NL];    // T = Lqq Fr
  __shared__ double sW[NQ];          // w_q / kappa_q
  const long T = blockIdx.x;
  if (T >= nelem) return;
  if (mask && mask[T] != code) return;
  const int tid = threadIdx.x;
  for (int q = tid; q < NQ; q += NT) sW[q] = Wq[q] / kqp[T * NQ + q];
  for (int idx = tid; idx < N * N; idx += NT) {
    const int i = idx / N, j = idx % N;
    double v = 0.0;
    if (i < NQV && j >= NQV)
      v = -Bd[i * NV + (j - NQV)];
    else if (i >= NQV && j < NQV)
      v = Bd[j * NV + (i - NQV)];
    sL[idx] = v;
  }
  __syncthreads();
  for (int c = 0; c < 2; ++c) {
    const double* V = Vq + (long)c * NQ * NQC;
    wg_mfma<NQC, NQC, NQ, NT>([&](int i, int q) { return V[q * NQC + i] * sW[q]; },
                              [&](int q, int j) { return V[q * NQC + j]; },
                              [&](int i, int j, double v) { sL[(c * NQC + i) * N + c * NQC + j] = v; });
  }
  gj_inverse_reg<N, NT>(sL);
  if (Luu_out)
    for (int idx = tid; idx < NV * NV; idx += NT)
      Luu_out[T * NV * NV + idx] = sL[(NQV + idx / NV) * N + NQV + idx % NV];
  // T = Lqq Fr
  wg_mfma<NQV, NL, NQV, NT>([&](int i, int l) { return sL[i * N + l]; },
                            [&](int l, int j) { return Fr[l * NL + j]; },
                            [&](int i, int j, double v) { sT[i * NL + j] = v; });
  __syncthreads();
  double* Ae = Aelem + T * (long)NL * NL;
  wg_mfma<NL, NL, NQV, NT>([&](int i, int l) { return Fr[l * NL + i]; },
                           [&](int l, int j) { return sT[l * NL + j]; },
                           [&](int i, int j, double v) { Ae[i * NL + j] = v; });
  // W = Lqu^T Fr: W[a][l] = sum_q L[q][NQV + a] Fr[q][l]
  wg_mfma<NV, NL, NQV, NT>([&](int a, int q) { return sL[q * N + NQV + a]; },
                           [&](int q, int l) { return Fr[q * NL + l]; },
                           [&](int a, int l, double v) { Wout[(T * NV + a) * NL + l] = v; });
  if (Xr) {
    // Xr = -Luq Fr
    wg_mfma<NV, NL, NQV, NT>([&](int a, int q) { return sL[(NQV + a) * N + q]; },
                             [&](int q, int l) { return Fr[q * NL + l]; },
                             [&](int a, int l, double v) { Xr[(T * NV + a) * NL + l] = -v; });
    // flux maps at the nodes, one velocity component at a time
    for (int c = 0; c < 2; ++c) {
      const double* V = Vn + (long)c * NV * NQC;
      wg_mfma<NV, NL, NQC, NT>([&](int a, int I) { return V[a * NQC + I]; },
                               [&](int I, int l) { return sT[(c * NQC + I) * NL + l]; },
                               [&](int a, int l, double v) { Xq[((T * 2 + c) * NV + a) * NL + l] = -v; });
      wg_mfma<NV, NV, NQC, NT>([&](int a, int I) { return V[a * NQC + I]; },
                               [&](int I, int j) { return sL[(c * NQC + I) * N + NQV + j]; },
                               [&](int a, int j, double v) { Yq[((T * 2 + c) * NV + a) * NV + j] = v; });
    }
  }
}

// b = M f (or f itself when it is already a load), per (element, node)
template <int NV>
__global__ void load_vec_kernel(long nelem, const double* __restrict__ M, const double* __restrict__ f,
                                int is_load, double* __restrict__ b) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nelem * NV) return;
  long T = t / NV;
  int i = (int)(t % NV);
  if (is_load) {
    b[t] = f[t];
    return;
  }
  double s = 0.0;
  for (int j = 0; j < NV; ++j) s += M[i * NV + j] * f[T * NV + j];
  b[t] = s;
}

// b^e = W^T b per (element, local trace DOF)
template <int NV, int NL>
__global__ void load_elem_kernel(long nelem, const double* __restrict__ W, const double* __restrict__ b,
                                 double* __restrict__ ebuf) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nelem * NL) return;
  long T = t / NL;
  int r = (int)(t % NL);
  double s = 0.0;
  for (int i = 0; i < NV; ++i) s += W[(T * NV + i) * NL + r] * b[T * NV + i];
  ebuf[t] = s;
}

// element coordinates <-> index, face ids (interior / boundary)
template <int D>
__device__ inline void elem_coords(long T, int n, int* e) {
  for (int a = 0; a < D; ++a) {
    e[a] = (int)(T % n);
    T /= n;
  }
}

template <int D>
__device__ inline long elem_index(const int* e, int n) {
  long T = 0;
  for (int a = D - 1; a >= 0; --a) T = T * n + e[a];
  return T;
}

// interior face id of direction c at grid coordinates g (g[c] = position 1..n-1)
template <int D>
__device__ inline long iface_id(int c, const int* g, int n) {
  long idx = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    if (a == c) {
      idx += (long)(g[a] - 1) * stride;
      stride *= (n - 1);
    } else {
      idx += (long)g[a] * stride;
      stride *= n;
    }
  }
  long nfd = (long)(n - 1);
  for (int a = 1; a < D; ++a) nfd *= n;
  return c * nfd + idx;
}

template <int D>
__device__ inline long bface_id(int c, int side, const int* g, int n) {
  long idx = 0, stride = 1;
  for (int a = 0; a < D; ++a)
    if (a != c) {
      idx += (long)g[a] * stride;
      stride *= n;
    }
  long blk = 1;
  for (int a = 1; a < D; ++a) blk *= n;
  return (2 * c + side) * blk + idx;
}

// g_F = b^e_{T-}[slot 2c+1] + b^e_{T+}[slot 2c] - (Dirichlet lift)
template <int D, int NE>
__global__ void load_pull_kernel(int n, const double* __restrict__ ebuf, const double* __restrict__ Aelem,
                                 const double* __restrict__ gdir, double* __restrict__ g) {
  constexpr int NL = 2 * D * NE;
  long nfd = (long)(n - 1);
  for (int a = 1; a < D; ++a) nfd *= n;
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= D * nfd * NE) return;
  long F = t / NE;
  int a = (int)(t % NE);
  int c = (int)(F / nfd);
  long r = F % nfd;
  int gco[3] = {0, 0, 0};
  for (int dd = 0; dd < D; ++dd) {
    int ext = dd == c ? n - 1 : n;
    gco[dd] = (int)(r % ext) + (dd == c ? 1 : 0);
    r /= ext;
  }
  double s = 0.0;
  for (int side = 0; side < 2; ++side) {
    int e[3] = {gco[0], gco[1], gco[2]};
    e[c] = gco[c] - 1 + side;
    long T = elem_index<D>(e, n);
    int row = (side == 0 ? 2 * c + 1 : 2 * c) * NE + a;
    s += ebuf[T * NL + row];
    if (gdir) {
      for (int sl = 0; sl < 2 * D; ++sl) {
        int cc = sl / 2, sd = sl % 2;
        int p = e[cc] + sd;
        if (p == 0 || p == n) {
          int fg[3] = {e[0], e[1], e[2]};
          long bid = bface_id<D>(cc, p == n ? 1 : 0, fg, n);
          for (int b = 0; b < NE; ++b) s -= Aelem[(T * NL + row) * NL + sl * NE + b] * gdir[bid * NE + b];
        }
      }
    }
  }
  g[t] = s;
}

// Local recovery, one workgroup per element.  X = [Q; U] solves the local
// system L X = R Lambda + [0; b]: first by the Schur-complement route with
// the stored inverses (U = W Lambda + K^-1 b, Q_c = Mk^-1 (B_c^T U - F_c
// Lambda)), then one step of refinement on the full system: the residuals
//   r_c = -F_c Lambda - Mk Q_c + B_c^T U,
//   r_u = tau G Lambda + b - sum_c B_c Q_c - tau E U
// (Mk applied as Phi^T diag(w / kappa) Phi) are corrected by the same route,
// dU = K^-1 (r_u - sum_c B_c Mk^-1 r_c), dQ_c = Mk^-1 (r_c + B_c^T dU).  On
// elements with large kappa / (tau h) the first solution carries an error of
// eps kappa / (tau h) (the route cancels terms of size kappa); after the step
// it is backward stable.
template <int D, int K, int NT>
__global__ void __launch_bounds__(NT) reconstruct_kernel(int n, double tau0, int tau_kappa,
                                                         const double* __restrict__ Phi,
                                                         const double* __restrict__ Wq,
                                                         const double* __restrict__ kqp,
                                                         const double* __restrict__ Bm,
                                                         const double* __restrict__ Fm,
                                                         const double* __restrict__ Gm,
                                                         const double* __restrict__ Em,
                                                         const double* __restrict__ lam,
                                                         const double* __restrict__ gdir,
                                                         const double* __restrict__ b,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ Kinv,
                                                         const double* __restrict__ Minv, double* __restrict__ u,
                                                         double* __restrict__ q) {
  using Dm = Dims<D, K>;
  constexpr int NV = Dm::NV, NE = Dm::NE, NL = Dm::NL, NQ = Dm::NQ;
  __shared__ double sL[NL], sU[NV], sT[D * NV], sQ[D * NV], sY[D * NV], sR[NV], sP[NQ];
  const long T = blockIdx.x;
  const int tid = threadIdx.x;
  const double tau = tau_kappa ? tau0 * kqp[T * NQ] : tau0;
  const double* Mi = Minv + T * (long)NV * NV;
  const double* Ki = Kinv + T * (long)NV * NV;
  int e[3] = {0, 0, 0};
  elem_coords<D>(T, n, e);
  for (int idx = tid; idx < NL; idx += NT) {
    int sl = idx / NE, a = idx % NE;
    int c = sl / 2, sd = sl % 2;
    int gco[3] = {e[0], e[1], e[2]};
    int p = e[c] + sd;
    gco[c] = p;
    double v = 0.0;
    if (p == 0 || p == n) {
      if (gdir) v = gdir[bface_id<D>(c, p == n ? 1 : 0, gco, n) * NE + a];
    } else {
      v = lam[iface_id<D>(c, gco, n) * NE + a];
    }
    sL[idx] = v;
  }
  __syncthreads();
  // U = W Lambda + K^-1 b
  for (int i = tid; i < NV; i += NT) {
    double s = 0.0;
    for (int j = 0; j < NL; ++j) s += W[(T * NV + i) * NL + j] * sL[j];
    for (int j = 0; j < NV; ++j) s += Ki[i * NV + j] * b[T * NV + j];
    sU[i] = s;
  }
  __syncthreads();
  // Q_c = Mk^-1 (B_c^T U - F_c Lambda)
  for (int idx = tid; idx < D * NV; idx += NT) {
    const int c = idx / NV, i = idx % NV;
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Bm[(c * NV + j) * NV + i] * sU[j];
    for (int j = 0; j < NL; ++j) s -= Fm[(c * NV + i) * NL + j] * sL[j];
    sT[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < D * NV; idx += NT) {
    const int c = idx / NV, i = idx % NV;
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Mi[i * NV + j] * sT[c * NV + j];
    sQ[idx] = s;
  }
  __syncthreads();
  // residual of the second equation
  for (int i = tid; i < NV; i += NT) {
    double s = b[T * NV + i];
    for (int j = 0; j < NL; ++j) s += tau * Gm[i * NL + j] * sL[j];
    for (int j = 0; j < NV; ++j) s -= tau * Em[i * NV + j] * sU[j];
    for (int c = 0; c < D; ++c)
      for (int j = 0; j < NV; ++j) s -= Bm[(c * NV + i) * NV + j] * sQ[c * NV + j];
    sR[i] = s;
  }
  // residual of the first equations: r_c = -F_c Lambda + B_c^T U - Mk Q_c,
  // with Mk Q_c = Phi^T (w / kappa * (Phi Q_c)), one direction at a time
  for (int c = 0; c < D; ++c) {
    __syncthreads();
    for (int qp = tid; qp < NQ; qp += NT) {
      double s = 0.0;
      for (int j = 0; j < NV; ++j) s += Phi[qp * NV + j] * sQ[c * NV + j];
      sP[qp] = s * Wq[qp] / kqp[T * NQ + qp];
    }
    __syncthreads();
    for (int i = tid; i < NV; i += NT) {
      double s = 0.0;
      for (int j = 0; j < NV; ++j) s += Bm[(c * NV + j) * NV + i] * sU[j];
      for (int j = 0; j < NL; ++j) s -= Fm[(c * NV + i) * NL + j] * sL[j];
      for (int qp = 0; qp < NQ; ++qp) s -= Phi[qp * NV + i] * sP[qp];
      sT[c * NV + i] = s;
    }
  }
  __syncthreads();
  // y_c = Mk^-1 r_c ; Q_c += y_c
  for (int idx = tid; idx < D * NV; idx += NT) {
    const int c = idx / NV, i = idx % NV;
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Mi[i * NV + j] * sT[c * NV + j];
    sY[idx] = s;
    sQ[idx] += s;
  }
  __syncthreads();
  // dU = K^-1 (r_u - sum_c B_c y_c)
  for (int i = tid; i < NV; i += NT) {
    double s = sR[i];
    for (int c = 0; c < D; ++c)
      for (int j = 0; j < NV; ++j) s -= Bm[(c * NV + i) * NV + j] * sY[c * NV + j];
    sP[i] = s;  // NQ >= NV
  }
  __syncthreads();
  for (int i = tid; i < NV; i += NT) {
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Ki[i * NV + j] * sP[j];
    sR[i] = s;  // dU
  }
  __syncthreads();
  // Q_c += Mk^-1 B_c^T dU ; U += dU
  for (int idx = tid; idx < D * NV; idx += NT) {
    const int c = idx / NV, i = idx % NV;
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Bm[(c * NV + j) * NV + i] * sR[j];
    sT[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < D * NV; idx += NT) {
    const int c = idx / NV, i = idx % NV;
    double s = 0.0;
    for (int j = 0; j < NV; ++j) s += Mi[i * NV + j] * sT[c * NV + j];
    sQ[idx] += s;
  }
  for (int i = tid; i < NV; i += NT) sU[i] += sR[i];
  __syncthreads();
  for (int i = tid; i < NV; i += NT) u[T * NV + i] = sU[i];
  for (int i = tid; i < D * NV; i += NT) q[T * D * NV + i] = sQ[i];
}

// Local recovery of the IPDG family and of RT-H, one workgroup per element:
// u = X Lambda + Y b (IPDG: X = L^-1 R, Y = L^-1; RT-H: X = -Luq Fr,
// Y = Luu), then for IPDG q_c = -kappa d_c u at the nodes (each component
// of grad u lies in Q^k, so its nodal values represent it), for RT-H
// elements (code rt_code in mask, or all when mask is null and Xq is given)
// the flux field at the nodes, Xq Lambda + Yq b.
template <int D, int K, int NT>
__global__ void __launch_bounds__(NT) ipdg_reconstruct_kernel(int n, int nq, const int* __restrict__ mask, int rt_code,
                                                              const double* __restrict__ Xq,
                                                              const double* __restrict__ Yq,
                                                              const double* __restrict__ kqp,
                                                              const double* __restrict__ Dnode,
                                                              const double* __restrict__ lam,
                                                              const double* __restrict__ gdir,
                                                              const double* __restrict__ b,
                                                              const double* __restrict__ X,
                                                              const double* __restrict__ Linv,
                                                              double* __restrict__ u, double* __restrict__ q) {
  using Dm = Dims<D, K>;
  constexpr int NV = Dm::NV, NE = Dm::NE, NL = Dm::NL;
  __shared__ double sL[NL], sU[NV];
  const long T = blockIdx.x;
  const int tid = threadIdx.x;
  int e[3] = {0, 0, 0};
  elem_coords<D>(T, n, e);
  for (int idx = tid; idx < NL; idx += NT) {
    int sl = idx / NE, a = idx % NE;
    int c = sl / 2, sd = sl % 2;
    int gco[3] = {e[0], e[1], e[2]};
    int p = e[c] + sd;
    gco[c] = p;
    double v = 0.0;
    if (p == 0 || p == n) {
      if (gdir) v = gdir[bface_id<D>(c, p == n ? 1 : 0, gco, n) * NE + a];
    } else {
      v = lam[iface_id<D>(c, gco, n) * NE + a];
    }
    sL[idx] = v;
  }
  __syncthreads();
  const double* Xe = X + T * (long)NV * NL;
  const double* Li = Linv + T * (long)NV * NV;
  for (int i = tid; i < NV; i += NT) {
    double s = 0.0;
    for (int j = 0; j < NL; ++j) s += Xe[i * NL + j] * sL[j];
    for (int j = 0; j < NV; ++j) s += Li[i * NV + j] * b[T * NV + j];
    sU[i] = s;
  }
  __syncthreads();
  const double kap = kqp[T * nq];
  const bool rt = Xq && (!mask || mask[T] == rt_code);
  for (int idx = tid; idx < D * NV; idx += NT) {
    double s = 0.0;
    if (rt) {  // RT-H element: the flux field at the nodes, Xq Lambda + Yq b
      for (int j = 0; j < NL; ++j) s += Xq[(T * D * NV + idx) * NL + j] * sL[j];
      for (int j = 0; j < NV; ++j) s += Yq[(T * D * NV + idx) * NV + j] * b[T * NV + j];
      q[T * D * NV + idx] = s;
    } else {
      const int c = idx / NV, a = idx % NV;
      for (int j = 0; j < NV; ++j) s += Dnode[(c * NV + a) * NV + j] * sU[j];
      q[T * D * NV + idx] = -kap * s;
    }
  }
  for (int i = tid; i < NV; i += NT) u[T * NV + i] = sU[i];
}

// dJ/dlog kappa_T = -sum_c (q*_c)^T Mk q_c, evaluated at the Gauss points.
template <int D, int K, int NT>
__global__ void __launch_bounds__(NT) grad_kernel(long nelem, const double* __restrict__ Phi,
                                                  const double* __restrict__ Wq, const double* __restrict__ kqp,
                                                  const double* __restrict__ q, const double* __restrict__ qs,
                                                  double* __restrict__ grad) {
  using Dm = Dims<D, K>;
  constexpr int NV = Dm::NV, NQ = Dm::NQ;
  __shared__ double red[NT];
  const long T = blockIdx.x;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int Q = tid; Q < NQ; Q += NT) {
    double s = 0.0;
    for (int c = 0; c < D; ++c) {
      double a = 0.0, b = 0.0;
      for (int i = 0; i < NV; ++i) {
        a += Phi[Q * NV + i] * q[(T * D + c) * NV + i];
        b += Phi[Q * NV + i] * qs[(T * D + c) * NV + i];
      }
      s += a * b;
    }
    acc += Wq[Q] / kqp[T * NQ + Q] * s;
  }
  red[tid] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) grad[T] = -red[0];
}

__global__ void kappa_expand_kernel(long nelem, int nq, const double* __restrict__ kappa, int kind,
                                    double* __restrict__ kqp, int* bad) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nelem * nq) return;
  double v = kind == HDG_KAPPA_PER_ELEMENT ? kappa[t / nq] : kappa[t];
  if (!(v > 0.0) || !(v < INFINITY)) atomicOr(bad, 1);
  kqp[t] = v;
}

template <typename F>
void dispatch_dk(int d, int k, F&& f) {
  if (d == 2) {
    switch (k) {
      case 1: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{}); return;
      case 2: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{}); return;
      case 3: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{}); return;
      case 4: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{}); return;
      case 5: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 5>{}); return;
      case 6: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 6>{}); return;
    }
  } else {
    switch (k) {
      case 1: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{}); return;
      case 2: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{}); return;
      case 3: f(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}); return;
    }
  }
  throw HipError{hipErrorInvalidValue, "unsupported (d, k)"};
}

}  // namespace

void launch_element_dtn(int d, int k, long nelem, double tau, int tau_kappa, const RefDevice& rd, const double* kqp,
                        double* Aelem, double* W, double* Kinv, double* Minv, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    constexpr int NT = D == 2 ? HDG_ELEM_NT2 : (K == 3 ? HDG_ELEM_NT3 : 256);
    hipLaunchKernelGGL((element_dtn_kernel<D, K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, nelem, tau,
                       tau_kappa, rd.Phi, rd.Wq, rd.B, rd.F, rd.G, rd.E, rd.H, kqp, Aelem, W, Kinv, Minv);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_ipdg_dtn(int d, int k, long nelem, const int* mask, int code, double tau, int tau_kappa, double sf,
                     const RefDevice& rd, const double* kqp, int nq, double* Aelem, double* W, double* X,
                     double* Linv, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    constexpr int NT = (D == 3 && K == 3) ? HDG_ELEM_NT3 : 256;
    hipLaunchKernelGGL((ipdg_dtn_kernel<D, K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, nelem, mask, code, tau,
                       tau_kappa, sf, nq, kqp,
                       rd.Kst, rd.Nn, rd.Dn, rd.G, rd.E, rd.H, Aelem, W, X, Linv);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_rt_dtn(int k, long nelem, const int* mask, int code, const RefDevice& rd, const double* kqp,
                   double* Aelem, double* W, double* Xr, double* Luu, double* Xq, double* Yq, hipStream_t st) {
  auto go = [&](auto K_) {
    constexpr int K = decltype(K_)::value;
    constexpr int NT = 256;
    hipLaunchKernelGGL((rt_dtn_kernel<K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, nelem, mask, code, rd.Wq, kqp,
                       rd.Vq, rd.Bd, rd.Fr, rd.Vnode, Aelem, W, Xr, Luu, Xq, Yq);
  };
  switch (k) {
    case 1: go(std::integral_constant<int, 1>{}); break;
    case 2: go(std::integral_constant<int, 2>{}); break;
    case 3: go(std::integral_constant<int, 3>{}); break;
    case 4: go(std::integral_constant<int, 4>{}); break;
    default: throw HipError{hipErrorInvalidValue, "RT-H: k in 1..4"};
  }
  HDG_CHECK(hipGetLastError());
}

void launch_ipdg_reconstruct(int d, int k, int n, const RefDevice& rd, const double* kqp, int nq, const int* mask,
                             int rt_code, const double* Xq, const double* Yq, const double* lam, const double* gdir,
                             const double* f, int is_load, const double* X, const double* Linv, double* b, double* u,
                             double* q, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    using Dm = Dims<D, K>;
    long nelem = 1;
    for (int a = 0; a < D; ++a) nelem *= n;
    long n1 = nelem * Dm::NV;
    hipLaunchKernelGGL((load_vec_kernel<Dm::NV>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, nelem,
                       rd.M, f, is_load, b);
    constexpr int NT = 64;
    hipLaunchKernelGGL((ipdg_reconstruct_kernel<D, K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, n, nq, mask,
                       rt_code, Xq, Yq, kqp, rd.Dnode, lam, gdir, b, X, Linv, u, q);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_element_load(int d, int k, long nelem, const RefDevice& rd, const double* f, int is_load,
                         const double* W, double* ebuf, hipStream_t st) {
  // ebuf must hold nelem*(NV + NL) doubles: b then b^e
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    using Dm = Dims<D, K>;
    double* b = ebuf + nelem * Dm::NL;
    long n1 = nelem * Dm::NV, n2 = nelem * Dm::NL;
    hipLaunchKernelGGL((load_vec_kernel<Dm::NV>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, nelem,
                       rd.M, f, is_load, b);
    hipLaunchKernelGGL((load_elem_kernel<Dm::NV, Dm::NL>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st,
                       nelem, W, b, ebuf);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_load_pull(int d, int k, int n, const double* ebuf, const double* Aelem, const double* gdir,
                      double* g, hipStream_t st) {
  if (n < 2) return;
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    using Dm = Dims<D, K>;
    long nfd = n - 1;
    for (int a = 1; a < D; ++a) nfd *= n;
    long tot = D * nfd * Dm::NE;
    hipLaunchKernelGGL((load_pull_kernel<D, Dm::NE>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n,
                       ebuf, Aelem, gdir, g);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_reconstruct(int d, int k, int n, double tau, int tau_kappa, const RefDevice& rd, const double* kqp, const double* lam,
                        const double* gdir, const double* f, int is_load, const double* W, const double* Kinv,
                        const double* Minv, double* b, double* u, double* q, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    using Dm = Dims<D, K>;
    long nelem = 1;
    for (int a = 0; a < D; ++a) nelem *= n;
    long n1 = nelem * Dm::NV;
    hipLaunchKernelGGL((load_vec_kernel<Dm::NV>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, nelem,
                       rd.M, f, is_load, b);
    constexpr int NT = 64;
    hipLaunchKernelGGL((reconstruct_kernel<D, K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, n, tau, tau_kappa,
                       rd.Phi,
                       rd.Wq, kqp, rd.B, rd.F, rd.G, rd.E, lam, gdir, b, W, Kinv, Minv, u, q);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_grad(int d, int k, long nelem, const RefDevice& rd, const double* kqp, const double* q,
                 const double* qs, double* grad, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    constexpr int NT = 64;
    hipLaunchKernelGGL((grad_kernel<D, K, NT>), dim3((unsigned)nelem), dim3(NT), 0, st, nelem, rd.Phi, rd.Wq, kqp,
                       q, qs, grad);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_mass(int d, int k, long nelem, const RefDevice& rd, const double* u, double* out, hipStream_t st) {
  dispatch_dk(d, k, [&](auto D_, auto K_) {
    constexpr int D = decltype(D_)::value, K = decltype(K_)::value;
    using Dm = Dims<D, K>;
    long n1 = nelem * Dm::NV;
    hipLaunchKernelGGL((load_vec_kernel<Dm::NV>), dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, nelem,
                       rd.M, u, 0, out);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_kappa_expand(long nelem, int nq, const double* kappa, int kind, double* kqp, int* bad,
                         hipStream_t st) {
  long tot = nelem * nq;
  hipLaunchKernelGGL(kappa_expand_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nelem, nq, kappa,
                     kind, kqp, bad);
  HDG_CHECK(hipGetLastError());
}

}  // namespace hdg
