// Kernels of the unstructured-mesh path (gfx950): HDG element maps of P^k
// triangles (Sec. 2, static condensation), loads, the P^1 Galerkin maps of
// the p-coarsening (eq. ANm1), the per-macro-element Schur complements of the
// agglomeration levels (eqs. trace_partition, Akm1, n_1_Ik, n_1_Qk; Sec.
// 3.1.2), face-block inverses (Sec. 4.1), the coarsest dense inverse
// (Algorithm 1, B_1 = A_1^-1), and the trace apply, local correction and
// transfers of the V-cycle on cells with explicit connectivity.
//
// Apply in two phases: the element phase forms z = A_c x_c for every cell c
// (one lane per triangle on triangle levels, reading maps AoSoA over
// triangles; one lane per map row on agglomeration levels), the face phase
// adds each face's two cell rows and finishes the mode (residual, block-
// Jacobi update, p-restriction, dot products) exactly as on the grid levels.
// No atomics: every output has one writer, so results are reproducible.
#include "hdg_internal.hpp"
#include "blas.hpp"
#include "reduce.hpp"
#include "trace_dev.hpp"
#include "mfma_dev.hpp"

namespace hdg {

namespace {

using namespace dev;

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

// ---------------------------------------------------------------------------
// Element maps of P^k triangles.  With the local unknowns [q_x, q_y, u] the
// local matrix is L = [[M/kappa (per component), B], [C, tau E]] (B_c =
// -(d_c phi_i, phi_j), C_c = -(d_c phi_i, phi_j) + <n_c phi_i, phi_j>), R =
// [-F; tau G], S = [F; tau G]; eliminating q first leaves the SPD block
//   K = tau E - sum_c C_c Mk^-1 B_c,
// so that L^-1 R = [Q; X], K X = tau G + sum_c C_c Mk^-1 F_c, Q_c = -Mk^-1
// (F_c + B_c X), and A^e = tau H - S^T L^-1 R = tau H - sum_c F_c^T Q_c -
// tau G^T X.  The load b^e = S^T L^-1 [0; M_T f] = (tau G^T - sum_c F_c^T
// Mk^-1 B_c) K^-1 M_T f is stored as W = its transpose map.  Geometry is
// affine: M_T = det M^, D_c = det sum_r (J^-1)_{rc} D^_r, edge integrals
// scale with the edge length; trace values of an edge run from its lower to
// its higher vertex, so a slot whose own direction is the reverse reads the
// reference columns k - a.  One wavefront per triangle.
template <int K>
__global__ void __launch_bounds__(64) tri_dtn_kernel(long ntri, const double* __restrict__ Mh,
                                                     const double* __restrict__ Minvh,
                                                     const double* __restrict__ Dh, const double* __restrict__ Eh,
                                                     const double* __restrict__ Fh, const double* __restrict__ Hh,
                                                     const double* __restrict__ xy, const int* __restrict__ tri,
                                                     const double* __restrict__ kappa, double tau,
                                                     double* __restrict__ Aelem, double* __restrict__ W,
                                                     double* __restrict__ Rec) {
  constexpr int NV = (K + 1) * (K + 2) / 2, NE = K + 1, NL = 3 * NE, RL = NV + NL + NV;
  __shared__ double sMi[NV * NV];
  __shared__ double sD[2][NV * NV];
  __shared__ double sC[2][NV * NV];
  __shared__ double sF[2][NV * NL];
  __shared__ double sG[NV * NL];
  __shared__ double sMB[2][NV * NV];
  __shared__ double sMF[2][NV * NL];
  __shared__ double sK[NV * RL];
  __shared__ double sS[NL * NV];
  __shared__ double fac[NV];
  const long t = blockIdx.x;
  if (t >= ntri) return;
  const int tid = threadIdx.x;
  int vid[3];
  double px[3], py[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    vid[s] = tri[3 * t + s];
    px[s] = xy[2 * vid[s]];
    py[s] = xy[2 * vid[s] + 1];
  }
  const double j00 = px[1] - px[0], j01 = px[2] - px[0], j10 = py[1] - py[0], j11 = py[2] - py[0];
  const double det = j00 * j11 - j01 * j10;
  // J^-1 = [[j11, -j01], [-j10, j00]] / det; Ji[r][c]
  const double Ji[2][2] = {{j11 / det, -j01 / det}, {-j10 / det, j00 / det}};
  double ell[3], nx[3], ny[3];
  int flip[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int s1 = (s + 1) % 3;
    const double dx = px[s1] - px[s], dy = py[s1] - py[s];
    ell[s] = sqrt(dx * dx + dy * dy);
    nx[s] = dy / ell[s];
    ny[s] = -dx / ell[s];
    flip[s] = vid[s] > vid[s1];
  }
  const double kap = kappa[t];
  for (int idx = tid; idx < NV * NV; idx += 64) {
    sMi[idx] = (kap / det) * Minvh[idx];
    double nc0 = 0.0, nc1 = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      nc0 += nx[s] * ell[s] * Eh[s * NV * NV + idx];
      nc1 += ny[s] * ell[s] * Eh[s * NV * NV + idx];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double dc = det * (Ji[0][c] * Dh[idx] + Ji[1][c] * Dh[NV * NV + idx]);
      sD[c][idx] = dc;
      sC[c][idx] = -dc + (c == 0 ? nc0 : nc1);
    }
  }
  for (int idx = tid; idx < NV * NL; idx += 64) {
    const int i = idx / NL, l = idx % NL, s = l / NE, a = l % NE;
    const double fr = ell[s] * Fh[(s * NV + i) * NE + (flip[s] ? NE - 1 - a : a)];
    sF[0][idx] = nx[s] * fr;
    sF[1][idx] = ny[s] * fr;
    sG[idx] = fr;
  }
  __syncthreads();
  for (int idx = tid; idx < NV * NV; idx += 64) {
    const int i = idx / NV, j = idx % NV;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double acc = 0.0;
      for (int m = 0; m < NV; ++m) acc += sMi[i * NV + m] * sD[c][m * NV + j];
      sMB[c][idx] = -acc;
    }
  }
  for (int idx = tid; idx < NV * NL; idx += 64) {
    const int i = idx / NL, l = idx % NL;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double acc = 0.0;
      for (int m = 0; m < NV; ++m) acc += sMi[i * NV + m] * sF[c][m * NL + l];
      sMF[c][idx] = acc;
    }
  }
  __syncthreads();
  // [K | tau G + sum_c C_c Mk^-1 F_c | M_T]
  for (int idx = tid; idx < NV * RL; idx += 64) {
    const int i = idx / RL, j = idx % RL;
    double v;
    if (j < NV) {
      double e = 0.0;
#pragma unroll
      for (int s = 0; s < 3; ++s) e += ell[s] * Eh[(s * NV + i) * NV + j];
      v = tau * e;
      for (int c = 0; c < 2; ++c)
        for (int m = 0; m < NV; ++m) v -= sC[c][i * NV + m] * sMB[c][m * NV + j];
    } else if (j < NV + NL) {
      const int l = j - NV;
      v = tau * sG[i * NL + l];
      for (int c = 0; c < 2; ++c)
        for (int m = 0; m < NV; ++m) v += sC[c][i * NV + m] * sMF[c][m * NL + l];
    } else {
      v = det * Mh[i * NV + (j - NV - NL)];
    }
    sK[idx] = v;
  }
  __syncthreads();
  // Gauss-Jordan on the SPD block K (no pivoting)
  for (int p = 0; p < NV; ++p) {
    const double piv = sK[p * RL + p];
    if (tid < NV) fac[tid] = sK[tid * RL + p] / piv;
    __syncthreads();
    for (int idx = tid; idx < NV * RL; idx += 64) {
      const int r = idx / RL, c = idx % RL;
      if (r != p && c > p) sK[idx] -= fac[r] * sK[p * RL + c];
    }
    __syncthreads();
    for (int c = p + 1 + tid; c < RL; c += 64) sK[p * RL + c] /= piv;
    __syncthreads();
  }
  // Y_c = Mk^-1 F_c + Mk^-1 B_c X (= -Q_c), in place of sMF
  for (int idx = tid; idx < NV * NL; idx += 64) {
    const int i = idx / NL, l = idx % NL;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double acc = sMF[c][idx];
      for (int m = 0; m < NV; ++m) acc += sMB[c][i * NV + m] * sK[m * RL + NV + l];
      sMF[c][idx] = acc;
    }
  }
  // S_u = tau G^T - sum_c F_c^T Mk^-1 B_c  [NL][NV]
  for (int idx = tid; idx < NL * NV; idx += 64) {
    const int l = idx / NV, i = idx % NV;
    double acc = tau * sG[i * NL + l];
    for (int c = 0; c < 2; ++c)
      for (int m = 0; m < NV; ++m) acc -= sF[c][m * NL + l] * sMB[c][m * NV + i];
    sS[idx] = acc;
  }
  __syncthreads();
  double* Ae = Aelem + t * NL * NL;
  for (int idx = tid; idx < NL * NL; idx += 64) {
    const int l = idx / NL, lp = idx % NL, s = l / NE, sp = lp / NE;
    double v = (s == sp) ? tau * ell[s] * Hh[(l % NE) * NE + (lp % NE)] : 0.0;
    for (int i = 0; i < NV; ++i)
      v += sF[0][i * NL + l] * sMF[0][i * NL + lp] + sF[1][i * NL + l] * sMF[1][i * NL + lp] -
           tau * sG[i * NL + l] * sK[i * RL + NV + lp];
    Ae[idx] = v;
  }
  double* Wt = W + t * NV * NL;
  for (int idx = tid; idx < NV * NL; idx += 64) {
    const int j = idx / NL, l = idx % NL;
    double v = 0.0;
    for (int i = 0; i < NV; ++i) v += sS[l * NV + i] * sK[i * RL + NV + NL + j];
    Wt[idx] = v;
  }
  if (!Rec) return;
  // recovery: u = X [Lambda; f], q_c = -Y_c Lambda - Mk^-1 B_c X_M f
  constexpr int RC = NL + NV;
  double* Rt = Rec + t * 3 * NV * RC;
  for (int idx = tid; idx < NV * RC; idx += 64) {
    const int i = idx / RC, col = idx % RC;
    Rt[2 * NV * RC + idx] = sK[i * RL + NV + col];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double v;
      if (col < NL) {
        v = -sMF[c][i * NL + col];
      } else {
        v = 0.0;
        for (int m = 0; m < NV; ++m) v -= sMB[c][i * NV + m] * sK[m * RL + NV + col];
      }
      Rt[c * NV * RC + idx] = v;
    }
  }
}

// Element maps of the hybridized IPDG family on P^k triangles (eq. IPG_H):
// with rows for the test function, L = kappa (K - s_f N - N^T) + tau E,
// R = tau G - s_f kappa D, C = tau G^T - kappa D^T (K the stiffness matrix,
// N_ij = <phi_j, grad phi_i . n>, D_il = <mu_l, grad phi_i . n>); L X =
// [R | M_T] by Gauss-Jordan without pivoting (the symmetric part of L is
// positive definite at tau = (p+1)(p+2)/h_min), A^e = tau H - C X_R, the
// load map (C X_M)^T and the recovery maps u = X [Lambda; f], q_c = -kappa
// d_c u at the nodes.  Geometry as in tri_dtn_kernel: gradients through
// J^-1, edge integrals scaled by the length, reversed slots read the
// reference columns k - a.
template <int K>
__global__ void __launch_bounds__(64) tri_ipdg_dtn_kernel(
    long ntri, const double* __restrict__ Mh, const double* __restrict__ Kh, const double* __restrict__ Nh,
    const double* __restrict__ De, const double* __restrict__ Eh, const double* __restrict__ Fh,
    const double* __restrict__ Hh, const double* __restrict__ Gn, const double* __restrict__ xy,
    const int* __restrict__ tri, const double* __restrict__ kappa, double tau, double sf,
    double* __restrict__ Aelem, double* __restrict__ W, double* __restrict__ Rec) {
  constexpr int NV = (K + 1) * (K + 2) / 2, NE = K + 1, NL = 3 * NE, RL = NV + NL + NV;
  __shared__ double sL[NV * RL];
  __shared__ double sC[NL * NV];
  __shared__ double fac[NV];
  const long t = blockIdx.x;
  if (t >= ntri) return;
  const int tid = threadIdx.x;
  int vid[3];
  double px[3], py[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    vid[s] = tri[3 * t + s];
    px[s] = xy[2 * vid[s]];
    py[s] = xy[2 * vid[s] + 1];
  }
  const double j00 = px[1] - px[0], j01 = px[2] - px[0], j10 = py[1] - py[0], j11 = py[2] - py[0];
  const double det = j00 * j11 - j01 * j10;
  const double Ji[2][2] = {{j11 / det, -j01 / det}, {-j10 / det, j00 / det}};
  double ell[3], gn[3][2];
  int flip[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int s1 = (s + 1) % 3;
    const double dx = px[s1] - px[s], dy = py[s1] - py[s];
    ell[s] = sqrt(dx * dx + dy * dy);
    const double nx = dy / ell[s], ny = -dx / ell[s];
#pragma unroll
    for (int r = 0; r < 2; ++r) gn[s][r] = Ji[r][0] * nx + Ji[r][1] * ny;  // d/dxi_r weight of grad . n
    flip[s] = vid[s] > vid[s1];
  }
  double G[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int rp = 0; rp < 2; ++rp) G[r][rp] = Ji[r][0] * Ji[rp][0] + Ji[r][1] * Ji[rp][1];
  const double kap = kappa[t];
  for (int idx = tid; idx < NV * RL; idx += 64) {
    const int i = idx / RL, j = idx % RL;
    double v;
    if (j < NV) {
      double kk = 0.0, nij = 0.0, nji = 0.0, e = 0.0;
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int rp = 0; rp < 2; ++rp) kk += G[r][rp] * Kh[((r * 2 + rp) * NV + i) * NV + j];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          nij += ell[s] * gn[s][r] * Nh[((s * 2 + r) * NV + i) * NV + j];
          nji += ell[s] * gn[s][r] * Nh[((s * 2 + r) * NV + j) * NV + i];
        }
        e += ell[s] * Eh[(s * NV + i) * NV + j];
      }
      v = kap * (det * kk - sf * nij - nji) + tau * e;
    } else if (j < NV + NL) {
      const int l = j - NV, s = l / NE, a = l % NE, ap = flip[s] ? NE - 1 - a : a;
      double dv = 0.0;
#pragma unroll
      for (int r = 0; r < 2; ++r) dv += gn[s][r] * De[((s * 2 + r) * NV + i) * NE + ap];
      dv *= ell[s];
      const double gv = ell[s] * Fh[(s * NV + i) * NE + ap];
      v = tau * gv - sf * kap * dv;
      sC[l * NV + i] = tau * gv - kap * dv;
    } else {
      v = det * Mh[i * NV + (j - NV - NL)];
    }
    sL[idx] = v;
  }
  __syncthreads();
  for (int p = 0; p < NV; ++p) {
    const double piv = sL[p * RL + p];
    if (tid < NV) fac[tid] = sL[tid * RL + p] / piv;
    __syncthreads();
    for (int idx = tid; idx < NV * RL; idx += 64) {
      const int r = idx / RL, c = idx % RL;
      if (r != p && c > p) sL[idx] -= fac[r] * sL[p * RL + c];
    }
    __syncthreads();
    for (int c = p + 1 + tid; c < RL; c += 64) sL[p * RL + c] /= piv;
    __syncthreads();
  }
  double* Ae = Aelem + t * NL * NL;
  for (int idx = tid; idx < NL * NL; idx += 64) {
    const int l = idx / NL, lp = idx % NL, s = l / NE, sp = lp / NE;
    double v = (s == sp) ? tau * ell[s] * Hh[(l % NE) * NE + (lp % NE)] : 0.0;
    for (int i = 0; i < NV; ++i) v -= sC[l * NV + i] * sL[i * RL + NV + lp];
    Ae[idx] = v;
  }
  double* Wt = W + t * NV * NL;
  for (int idx = tid; idx < NV * NL; idx += 64) {
    const int j = idx / NL, l = idx % NL;
    double v = 0.0;
    for (int i = 0; i < NV; ++i) v += sC[l * NV + i] * sL[i * RL + NV + NL + j];
    Wt[idx] = v;
  }
  if (!Rec) return;
  constexpr int RC = NL + NV;
  double* Rt = Rec + t * 3 * NV * RC;
  for (int idx = tid; idx < NV * RC; idx += 64) {
    const int a = idx / RC, col = idx % RC;
    Rt[2 * NV * RC + idx] = sL[a * RL + NV + col];
    double g0 = 0.0, g1 = 0.0;  // d_xi0 u, d_xi1 u at node a
    for (int m = 0; m < NV; ++m) {
      const double x = sL[m * RL + NV + col];
      g0 += Gn[(0 * NV + a) * NV + m] * x;
      g1 += Gn[(1 * NV + a) * NV + m] * x;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) Rt[c * NV * RC + idx] = -kap * (Ji[0][c] * g0 + Ji[1][c] * g1);
  }
}

// u, q (nodal) of every triangle from its traces (interior: lambda; boundary
// edges: gdir or 0) and f
template <int K>
__global__ void tri_reconstruct_kernel(long ntri, const int* __restrict__ sface, const int* __restrict__ tbnd,
                                       const double* __restrict__ Rec, const double* __restrict__ lam,
                                       const double* __restrict__ gdir, const double* __restrict__ f,
                                       double* __restrict__ u, double* __restrict__ q) {
  constexpr int NV = (K + 1) * (K + 2) / 2, NE = K + 1, NL = 3 * NE, RC = NL + NV;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= ntri) return;
  double v[RC];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int fc = sface[3 * t + s], b = tbnd[3 * t + s];
#pragma unroll
    for (int a = 0; a < NE; ++a)
      v[s * NE + a] = fc >= 0 ? lam[(long)fc * NE + a] : (gdir && b >= 0 ? gdir[(long)b * NE + a] : 0.0);
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) v[NL + j] = f[t * NV + j];
  const double* R = Rec + t * 3 * NV * RC;
  for (int r = 0; r < 3 * NV; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < RC; ++c) acc += R[r * RC + c] * v[c];
    if (r < 2 * NV)
      q[t * 2 * NV + r] = acc;
    else
      u[t * NV + r - 2 * NV] = acc;
  }
}

// g_F = sum over the face's two triangles of W^T f (rows of the face's slot)
template <int K>
__global__ void tri_load_kernel(long nface, const int* __restrict__ fcell, const int* __restrict__ fslot,
                                const double* __restrict__ W, const double* __restrict__ f,
                                const double* __restrict__ Aelem, const int* __restrict__ tbnd,
                                const double* __restrict__ gdir, double* __restrict__ g) {
  constexpr int NV = (K + 1) * (K + 2) / 2, NE = K + 1, NL = 3 * NE;
  const long F = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (F >= nface) return;
  double acc[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = 0.0;
  for (int side = 0; side < 2; ++side) {
    const long c = fcell[2 * F + side];
    const int s = fslot[2 * F + side];
    const double* Wc = W + c * NV * NL + s * NE;
    const double* fc = f + c * NV;
    for (int j = 0; j < NV; ++j) {
      const double fj = fc[j];
#pragma unroll
      for (int a = 0; a < NE; ++a) acc[a] += Wc[j * NL + a] * fj;
    }
    if (!gdir) continue;
    // Dirichlet lift: - A^e[face rows][boundary edge columns] g_D
    for (int sp = 0; sp < 3; ++sp) {
      const int b = tbnd[3 * c + sp];
      if (b < 0) continue;
      const double* Ac = Aelem + c * NL * NL + (s * NE) * NL + sp * NE;
#pragma unroll
      for (int a = 0; a < NE; ++a)
        for (int bb = 0; bb < NE; ++bb) acc[a] -= Ac[a * NL + bb] * gdir[(long)b * NE + bb];
    }
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) g[F * NE + a] = acc[a];
}

// P^1 maps of the triangles: A1 = Jb^T A0 Jb, Jb = diag(J_N, J_N, J_N)
__global__ void tri_pgalerkin_kernel(long ntri, int ne, const double* __restrict__ Jp, const double* __restrict__ A0,
                                     double* __restrict__ A1) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= ntri * 36) return;
  const long t = idx / 36;
  const int e = (int)(idx % 36), r = e / 6, c = e % 6;
  const int s = r / 2, v = r % 2, sp = c / 2, vp = c % 2;
  const int nl = 3 * ne;
  const double* A = A0 + t * nl * nl;
  double acc = 0.0;
  for (int a = 0; a < ne; ++a) {
    double row = 0.0;
    for (int b = 0; b < ne; ++b) row += A[(s * ne + a) * nl + sp * ne + b] * Jp[b * 2 + vp];
    acc += Jp[a * 2 + v] * row;
  }
  A1[idx] = acc;
}

// ---------------------------------------------------------------------------
// One coarse cell C of an agglomeration step per workgroup: assemble its
// fine cells' maps over its interior faces (E_I) and boundary faces (E_B),
// sweep the E_I pivots (partial Gauss-Jordan inversion: the SPD block A_II
// is never pivoted) to
//   [[A_II^-1, A_II^-1 A_IB], [-A_BI A_II^-1, A_BB - A_BI A_II^-1 A_IB]],
// then P = -A_II^-1 A_IB J_C (eq. n_1_Ik) and the coarse map J_C^T S J_C
// (eq. Akm1).  Work space per cell: its dense local matrix and S J_C.

__global__ void __launch_bounds__(256) uschur_kernel(
    long ncoarse, const long* __restrict__ ccptr, const int* __restrict__ ccell, const long* __restrict__ fsptr,
    const int* __restrict__ sloc, const long* __restrict__ fmoff, const long* __restrict__ iptr,
    const long* __restrict__ bptr, const int* __restrict__ bface, const int* __restrict__ bslot,
    const double* __restrict__ fJ, const long* __restrict__ csptr, const long* __restrict__ cmoff,
    const long* __restrict__ aoff, const long* __restrict__ poff, const long* __restrict__ woff,
    const double* __restrict__ Afine, double* __restrict__ AIIinv, double* __restrict__ P,
    double* __restrict__ R, double* __restrict__ Acoarse, double* __restrict__ work) {
  __shared__ double prow[UMACRO_MAX_DOFS], pcol[UMACRO_MAX_DOFS];
  const long C = blockIdx.x;
  if (C >= ncoarse) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nI = (int)(iptr[C + 1] - iptr[C]), nB = (int)(bptr[C + 1] - bptr[C]);
  const int n2 = 2 * (nI + nB), nI2 = 2 * nI, nc2 = 2 * (int)(csptr[C + 1] - csptr[C]);
  double* Wm = work + woff[C];
  double* T1 = Wm + (long)n2 * n2;
  for (long idx = tid; idx < (long)n2 * n2; idx += nt) Wm[idx] = 0.0;
  __syncthreads();
  for (long q = ccptr[C]; q < ccptr[C + 1]; ++q) {
    const int x = ccell[q];
    const long s0 = fsptr[x];
    const int nr = 2 * (int)(fsptr[x + 1] - s0);
    const double* A = Afine + fmoff[x];
    for (int idx = tid; idx < nr * nr; idx += nt) {
      const int r = idx / nr, c = idx % nr;
      const int lr = sloc[s0 + r / 2], lc = sloc[s0 + c / 2];
      if (lr >= 0 && lc >= 0) Wm[(long)(2 * lr + r % 2) * n2 + 2 * lc + c % 2] += A[idx];
    }
    __syncthreads();
  }
  for (int p = 0; p < nI2; ++p) {
    for (int j = tid; j < n2; j += nt) {
      prow[j] = Wm[(long)p * n2 + j];
      pcol[j] = Wm[(long)j * n2 + p];
    }
    __syncthreads();
    const double d = 1.0 / prow[p];
    for (long idx = tid; idx < (long)n2 * n2; idx += nt) {
      const int i = (int)(idx / n2), j = (int)(idx % n2);
      if (i == p && j == p)
        Wm[idx] = d;
      else if (i == p)
        Wm[idx] = prow[j] * d;
      else if (j == p)
        Wm[idx] = -pcol[i] * d;
      else
        Wm[idx] -= pcol[i] * prow[j] * d;
    }
    __syncthreads();
  }
  const long b0 = bptr[C];
  for (int idx = tid; idx < nI2 * nI2; idx += nt) AIIinv[aoff[C] + idx] = Wm[(long)(idx / nI2) * n2 + idx % nI2];
  for (int idx = tid; idx < nI2 * nc2; idx += nt) {
    const int i = idx / nc2, q2 = idx % nc2, q = q2 / 2, j = q2 % 2;
    double s = 0.0;
    for (int b = 0; b < nB; ++b) {
      if (bslot[b0 + b] != q) continue;
      const long f = bface[b0 + b];
      s += Wm[(long)i * n2 + nI2 + 2 * b] * fJ[4 * f + j] + Wm[(long)i * n2 + nI2 + 2 * b + 1] * fJ[4 * f + 2 + j];
    }
    P[poff[C] + idx] = -s;
    if (R) {  // restriction block from the swept lower-left block -A_BI A_II^-1
      double sr = 0.0;
      for (int b = 0; b < nB; ++b) {
        if (bslot[b0 + b] != q) continue;
        const long f = bface[b0 + b];
        sr += Wm[(long)(nI2 + 2 * b) * n2 + i] * fJ[4 * f + j] + Wm[(long)(nI2 + 2 * b + 1) * n2 + i] * fJ[4 * f + 2 + j];
      }
      R[poff[C] + idx] = sr;
    }
  }
  for (int idx = tid; idx < 2 * nB * nc2; idx += nt) {
    const int r = idx / nc2, q2 = idx % nc2, q = q2 / 2, j = q2 % 2;
    double s = 0.0;
    for (int b = 0; b < nB; ++b) {
      if (bslot[b0 + b] != q) continue;
      const long f = bface[b0 + b];
      const double* Srow = Wm + (long)(nI2 + r) * n2 + nI2;
      s += Srow[2 * b] * fJ[4 * f + j] + Srow[2 * b + 1] * fJ[4 * f + 2 + j];
    }
    T1[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < nc2 * nc2; idx += nt) {
    const int q2 = idx / nc2, c2 = idx % nc2, q = q2 / 2, j = q2 % 2;
    double s = 0.0;
    for (int b = 0; b < nB; ++b) {
      if (bslot[b0 + b] != q) continue;
      const long f = bface[b0 + b];
      s += fJ[4 * f + j] * T1[(long)(2 * b) * nc2 + c2] + fJ[4 * f + 2 + j] * T1[(long)(2 * b + 1) * nc2 + c2];
    }
    Acoarse[cmoff[C] + idx] = s;
  }
}

// face-block inverses D_F^-1 of the assembled diagonal blocks (SPD: Gauss-
// Jordan without pivoting), AoSoA over faces in FP64 and FP32
template <int NE>
__global__ void udinv_kernel(long nface, const int* __restrict__ fcell, const int* __restrict__ fslot,
                             const long* __restrict__ sptr, const long* __restrict__ moff,
                             const double* __restrict__ A, double* __restrict__ D64, float* __restrict__ D32) {
  const long F = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (F >= nface) return;
  double a[NE][2 * NE];
#pragma unroll
  for (int i = 0; i < NE; ++i)
#pragma unroll
    for (int j = 0; j < 2 * NE; ++j) a[i][j] = (j - NE == i) ? 1.0 : 0.0;
  for (int side = 0; side < 2; ++side) {
    const long c = fcell[2 * F + side];
    const int s = fslot[2 * F + side];
    const int nr = NE * (int)(sptr[c + 1] - sptr[c]);
    const double* Ac = A + moff[c];
#pragma unroll
    for (int i = 0; i < NE; ++i)
#pragma unroll
      for (int j = 0; j < NE; ++j) a[i][j] += Ac[(long)(s * NE + i) * nr + s * NE + j];
  }
#pragma unroll
  for (int p = 0; p < NE; ++p) {
    const double d = 1.0 / a[p][p];
#pragma unroll
    for (int j = 0; j < 2 * NE; ++j) a[p][j] *= d;
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      if (r == p) continue;
      const double f = a[r][p];
#pragma unroll
      for (int j = 0; j < 2 * NE; ++j) a[r][j] -= f * a[p][j];
    }
  }
#pragma unroll
  for (int i = 0; i < NE; ++i)
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      D64[aos_off<double>(F, vpad<double>(NE * NE), i * NE + j)] = a[i][NE + j];
      D32[aos_off<float>(F, vpad<float>(NE * NE), i * NE + j)] = (float)a[i][NE + j];
    }
}

// dense coarsest operator, one row per thread (face F's value a), from the
// cell maps of both its cells
__global__ void udense_kernel(long nface, int m, const int* __restrict__ fcell, const int* __restrict__ fslot,
                              const long* __restrict__ sptr, const int* __restrict__ sface,
                              const long* __restrict__ moff, const double* __restrict__ A, double* __restrict__ Ad) {
  const long row = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long N = nface * m;
  if (row >= N) return;
  const long F = row / m;
  const int a = (int)(row % m);
  double* out = Ad + row * N;
  for (long j = 0; j < N; ++j) out[j] = 0.0;
  for (int side = 0; side < 2; ++side) {
    const long c = fcell[2 * F + side];
    const int s = fslot[2 * F + side];
    const int ns = (int)(sptr[c + 1] - sptr[c]), nr = m * ns;
    const double* Ac = A + moff[c] + (long)(s * m + a) * nr;
    for (int sp = 0; sp < ns; ++sp) {
      const int g = sface[sptr[c] + sp];
      if (g < 0) continue;
      for (int b = 0; b < m; ++b) out[(long)g * m + b] += Ac[sp * m + b];
    }
  }
}

// in-place inverse of a dense SPD N x N matrix by N pivot sweeps (one
// workgroup), written to the FP64 and FP32 inverses
__global__ void __launch_bounds__(256) udense_inverse_kernel(int N, double* __restrict__ A, double* __restrict__ Ai64,
                                                             float* __restrict__ Ai32) {
  __shared__ double prow[UCOARSE_MAX], pcol[UCOARSE_MAX];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int p = 0; p < N; ++p) {
    for (int j = tid; j < N; j += nt) {
      prow[j] = A[(long)p * N + j];
      pcol[j] = A[(long)j * N + p];
    }
    __syncthreads();
    const double d = 1.0 / prow[p];
    for (long idx = tid; idx < (long)N * N; idx += nt) {
      const int i = (int)(idx / N), j = (int)(idx % N);
      if (i == p && j == p)
        A[idx] = d;
      else if (i == p)
        A[idx] = prow[j] * d;
      else if (j == p)
        A[idx] = -pcol[i] * d;
      else
        A[idx] -= pcol[i] * prow[j] * d;
    }
    __syncthreads();
  }
  for (long idx = tid; idx < (long)N * N; idx += nt) {
    Ai64[idx] = A[idx];
    Ai32[idx] = (float)A[idx];
  }
}

// Blocked Gauss-Jordan inverse of a large dense coarsest operator, in place
// in A (row-major, leading dimension N), by 64 x 64 blocks; entries past N
// act as the identity.  Block step p: P = A_pp^-1 (one workgroup), then
// A_pj <- P A_pj, A_ij -= A_ip A_pj (i, j != p), A_ip <- -A_ip P and
// A_pp <- P, every block product on the matrix cores.  Four launches per
// block step instead of one per pivot; no pivoting, the same elimination as
// the pivot-by-pivot sweep up to the rounding order.
constexpr int UBK = 64;

__device__ inline double ublk_get(const double* A, long N, long i, long j) {
  return (i < N && j < N) ? A[i * N + j] : (i == j ? 1.0 : 0.0);
}

__global__ void __launch_bounds__(256) ublk_pivot_kernel(long N, int p, const double* __restrict__ A,
                                                         double* __restrict__ Pb) {
  __shared__ double s[UBK * UBK];
  const long r0 = (long)p * UBK;
  for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) s[idx] = ublk_get(A, N, r0 + idx / UBK, r0 + idx % UBK);
  gj_inverse_blocked<UBK, 256>(s);  // starts and ends with a barrier
  for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) Pb[idx] = s[idx];
}

// A_pj <- P A_pj for every column block j != p (workgroup j)
__global__ void __launch_bounds__(256) ublk_row_kernel(long N, int p, const double* __restrict__ Pb,
                                                       double* __restrict__ A) {
  const int jb = blockIdx.x;
  if (jb == p) return;
  __shared__ double sP[UBK * UBK], sB[UBK * UBK];
  const long r0 = (long)p * UBK, c0 = (long)jb * UBK;
  for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) {
    sP[idx] = Pb[idx];
    sB[idx] = ublk_get(A, N, r0 + idx / UBK, c0 + idx % UBK);
  }
  __syncthreads();
  wg_mfma<UBK, UBK, UBK, 256>([&](int i, int k) { return sP[i * UBK + k]; },
                              [&](int k, int j) { return sB[k * UBK + j]; },
                              [&](int i, int j, double v) {
                                if (r0 + i < N && c0 + j < N) A[(r0 + i) * N + c0 + j] = v;
                              });
}

// A_ij -= A_ip A_pj for i, j != p (workgroup (j, i))
__global__ void __launch_bounds__(256) ublk_trail_kernel(long N, int p, double* __restrict__ A) {
  const int ib = blockIdx.y, jb = blockIdx.x;
  if (ib == p || jb == p) return;
  __shared__ double sL[UBK * UBK], sR[UBK * UBK];
  const long r0 = (long)ib * UBK, c0 = (long)jb * UBK, k0 = (long)p * UBK;
  for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) {
    sL[idx] = ublk_get(A, N, r0 + idx / UBK, k0 + idx % UBK);
    sR[idx] = ublk_get(A, N, k0 + idx / UBK, c0 + idx % UBK);
  }
  __syncthreads();
  wg_mfma<UBK, UBK, UBK, 256>([&](int i, int k) { return sL[i * UBK + k]; },
                              [&](int k, int j) { return sR[k * UBK + j]; },
                              [&](int i, int j, double v) {
                                if (r0 + i < N && c0 + j < N) A[(r0 + i) * N + c0 + j] -= v;
                              });
}

// A_ip <- -A_ip P for i != p, A_pp <- P (workgroup i)
__global__ void __launch_bounds__(256) ublk_col_kernel(long N, int p, const double* __restrict__ Pb,
                                                       double* __restrict__ A) {
  const int ib = blockIdx.x;
  const long r0 = (long)ib * UBK, c0 = (long)p * UBK;
  if (ib == p) {
    for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) {
      const long i = r0 + idx / UBK, j = c0 + idx % UBK;
      if (i < N && j < N) A[i * N + j] = Pb[idx];
    }
    return;
  }
  __shared__ double sP[UBK * UBK], sB[UBK * UBK];
  for (int idx = threadIdx.x; idx < UBK * UBK; idx += 256) {
    sP[idx] = Pb[idx];
    sB[idx] = ublk_get(A, N, r0 + idx / UBK, c0 + idx % UBK);
  }
  __syncthreads();
  wg_mfma<UBK, UBK, UBK, 256>([&](int i, int k) { return sB[i * UBK + k]; },
                              [&](int k, int j) { return sP[k * UBK + j]; },
                              [&](int i, int j, double v) {
                                if (r0 + i < N && c0 + j < N) A[(r0 + i) * N + c0 + j] = -v;
                              });
}

// row-major triangle maps -> AoSoA over triangles in 16-byte groups (FP64
// and FP32)
__global__ void tri_aos_kernel(long ntri, int nn, const double* __restrict__ A, double* __restrict__ A64,
                               float* __restrict__ A32) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= ntri * nn) return;
  const long t = idx / nn;
  const int e = (int)(idx % nn);
  A64[pk_off<double>(t, nn, e)] = A[idx];
  A32[pk_off<float>(t, nn, e)] = (float)A[idx];
}

__global__ void f32_kernel(const double* __restrict__ x, float* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// ---------------------------------------------------------------------------
// trace kernels
// element phase, triangle levels: workgroup b takes the 64 triangles
// 64 b .. 64 b + 63 (one per lane) and its CH waves split their 3 NE rows
// (wave w: rows w RA .., RA = ceil(3 NE / CH)), so that every map load of a
// wave is one contiguous segment and a level of 2 10^5 triangles still
// gives each SIMD enough waves to hide the memory latency; each lane
// gathers its triangle's traces itself.  The products go through LDS and
// leave as one contiguous block (z row-major per triangle), so that the
// face phase reads each side's values as one short segment.
template <int NE, typename T, typename M, int CH>
__global__ void __launch_bounds__(64 * CH) utri_phase_kernel(long ntri, long nrow, long N,
                                                             const int* __restrict__ sface, const M* __restrict__ Af,
                                                             const T* __restrict__ x, T* __restrict__ z) {
  constexpr int NL = 3 * NE, RA = (NL + CH - 1) / CH;
  using A = acc_t<T>;
  __shared__ T zs[LANES * NL];
  const int lane = threadIdx.x % LANES, w = threadIdx.x / LANES;
  const long t0 = blockIdx.x * (long)LANES, t = t0 + lane;
  const int rhs = blockIdx.y;
  x += rhs * N;
  z += rhs * nrow;
  if (t < ntri) {
    A xs[NL];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int f = sface[3 * t + s];
#pragma unroll
      for (int b = 0; b < NE; ++b) xs[s * NE + b] = f >= 0 ? A(x[(long)f * NE + b]) : A(0);
    }
    constexpr int V = pvw<M>();
    const M* blk = Af + (t / LANES) * pk_pad<M>(NL * NL) * LANES + (t % LANES) * V;
#pragma unroll
    for (int rr = 0; rr < RA; ++rr) {
      const int r = w * RA + rr;
      if (r < NL) {
        A acc = A(0);
#pragma unroll
        for (int j = 0; j < NL; ++j) {
          const int e = r * NL + j;
          acc += A(blk[(e / V) * (LANES * V) + e % V]) * xs[j];
        }
        zs[lane * NL + r] = T(acc);
      }
    }
  }
  __syncthreads();
  const long cnt = (ntri - t0 < LANES ? ntri - t0 : LANES) * NL;
  for (long i = threadIdx.x; i < cnt; i += LANES * CH) z[t0 * NL + i] = zs[i];
}

// element phase, agglomeration levels: one lane per map row
template <typename T, typename M>
__global__ void __launch_bounds__(256) ucell_phase_kernel(long nrow, long N, int m, const int* __restrict__ rcell,
                                                          const long* __restrict__ sptr,
                                                          const int* __restrict__ sface,
                                                          const long* __restrict__ moff, const M* __restrict__ Am,
                                                          const T* __restrict__ x, T* __restrict__ z) {
  using A = acc_t<T>;
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g >= nrow) return;
  const int rhs = blockIdx.y;
  x += rhs * N;
  z += rhs * nrow;
  const long c = rcell[g];
  const long s0 = sptr[c];
  const int ns = (int)(sptr[c + 1] - s0), nr = m * ns;
  const long lr = g - s0 * m;
  const M* row = Am + moff[c] + lr * nr;
  A acc = A(0);
  for (int sp = 0; sp < ns; ++sp) {
    const int f = sface[s0 + sp];
    if (f < 0) continue;
    for (int b = 0; b < m; ++b) acc += A(row[sp * m + b]) * A(x[(long)f * m + b]);
  }
  z[g] = T(acc);
}

// face phase: acc = z rows of both cells, then the mode's output; the
// workgroups walk the faces blockIdx.x * 256, + gridDim.x * 256, ... and
// write one partial sum each (reducing modes)
template <int NE, typename T, int MODE, typename M>
__global__ void __launch_bounds__(256) uface_kernel(long nface, long nrow, const long* __restrict__ zr, int zs,
                                                    const T* __restrict__ z, const M* __restrict__ Dinv,
                                                    const T* __restrict__ x, const T* __restrict__ bvec,
                                                    T* __restrict__ y, const double* __restrict__ Jp,
                                                    T* __restrict__ rc, float* __restrict__ y32,
                                                    double* __restrict__ partials) {
  constexpr bool RED = (MODE == APPLY_Y_DOT || MODE == APPLY_RES_NORM || MODE == APPLY_SWEEP_DOT);
  using A = acc_t<T>;
  const int rhs = blockIdx.y;
  {
    const long sN = nface * NE, sC = nface * 2;
    x += rhs * sN;
    bvec = off(bvec, rhs * sN);
    y = off(y, rhs * (MODE == APPLY_RES_PRESTRICT ? sC : sN));
    rc = off(rc, rhs * sC);
    y32 = off(y32, rhs * sN);
    if (MODE == APPLY_SWEEP_DOT) Jp += rhs * sN;
    z += rhs * nrow;
  }
  double part = 0.0;
  for (long F = blockIdx.x * 256L + threadIdx.x; F < nface; F += (long)gridDim.x * 256L) {
    const T* z0 = z + zr[2 * F];
    const T* z1 = z + zr[2 * F + 1];
    A acc[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) acc[a] = A(z0[a * zs]) + A(z1[a * zs]);
    face_finish<2, NE, T, MODE, false, M>(F, acc, Dinv, x, bvec, y, Jp, rc, y32, part);
  }
  if constexpr (RED) {
    __shared__ double sh[4];
    const double s = block_sum_t<256>(part, sh);
    if (threadIdx.x == 0) partials[(long)rhs * gridDim.x + blockIdx.x] = s;
  }
}

// local correction and restriction share of each coarse cell (eqs.
// localCorrection, n_1_Qk): rows [0, nIrow) are interior values (w =
// A_II^-1 rho_I; e_I += w when do_corr), rows [nIrow, nIrow + ncb) the
// coarse cell's share R^T rho_I of the restricted residual (R = P: the
// operator is symmetric)
template <typename T, typename M>
__global__ void __launch_bounds__(256) ucorr_kernel(long nIrow, long ncb, long N, const int* __restrict__ irc,
                                                    const int* __restrict__ cbc, const long* __restrict__ iptr,
                                                    const int* __restrict__ iface, const long* __restrict__ csptr,
                                                    const long* __restrict__ aoff, const long* __restrict__ poff,
                                                    const M* __restrict__ Ai, const M* __restrict__ R,
                                                    const T* __restrict__ rho, T* __restrict__ e, int do_corr,
                                                    int do_restrict, T* __restrict__ cb) {
  using A = acc_t<T>;
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  rho += rhs * N;
  e += rhs * N;
  if (g < nIrow) {
    if (!do_corr) return;
    const long C = irc[g];
    const long i0 = iptr[C];
    const int nI2 = 2 * (int)(iptr[C + 1] - i0);
    const long li = g - 2 * i0;
    const M* row = Ai + aoff[C] + li * nI2;
    A w = A(0);
    for (int j = 0; j < nI2; ++j) w += A(row[j]) * A(rho[2L * iface[i0 + j / 2] + j % 2]);
    const long dof = 2L * iface[i0 + li / 2] + li % 2;
    e[dof] = T(A(e[dof]) + w);
    return;
  }
  const long h = g - nIrow;
  if (h >= ncb || !do_restrict) return;
  const long C = cbc[h];
  const long i0 = iptr[C];
  const int nI2 = 2 * (int)(iptr[C + 1] - i0);
  const int nc2 = 2 * (int)(csptr[C + 1] - csptr[C]);
  const long q2 = h - 2 * csptr[C];
  const M* col = R + poff[C] + q2;
  A s = A(0);
  for (int j = 0; j < nI2; ++j) s += A(col[(long)j * nc2]) * A(rho[2L * iface[i0 + j / 2] + j % 2]);
  cb[rhs * ncb + h] = T(s);
}

// restricted residual on every macro-edge E (eq. n_1_Qk): J^T rho_B over its
// finer faces plus the shares of its two coarse cells
template <typename T>
__global__ void urestrict_kernel(long ncf, long N, long Nc, long ncb, const long* __restrict__ eptr,
                                 const int* __restrict__ efine, const double* __restrict__ fJ,
                                 const long* __restrict__ czr, const T* __restrict__ rho, const T* __restrict__ cb,
                                 T* __restrict__ rc) {
  using A = acc_t<T>;
  const long E = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (E >= ncf) return;
  const int rhs = blockIdx.y;
  rho += rhs * N;
  cb += rhs * ncb;
  rc += rhs * Nc;
  A s0 = A(0), s1 = A(0);
  for (long q = eptr[E]; q < eptr[E + 1]; ++q) {
    const long f = efine[q];
    const A r0 = A(rho[2 * f]), r1 = A(rho[2 * f + 1]);
    s0 += A(fJ[4 * f + 0]) * r0 + A(fJ[4 * f + 2]) * r1;
    s1 += A(fJ[4 * f + 1]) * r0 + A(fJ[4 * f + 3]) * r1;
  }
  const long z0 = czr[2 * E], z1 = czr[2 * E + 1];
  rc[2 * E] = T(s0 + A(cb[z0]) + A(cb[z1]));
  rc[2 * E + 1] = T(s1 + A(cb[z0 + 1]) + A(cb[z1 + 1]));
}

// prolongation (eq. n_1_Ik): interior values e_I += P e_c of their coarse
// cell (rows [0, nIrow)), boundary faces e_B += J e_E (one lane per face)
template <typename T, typename M>
__global__ void __launch_bounds__(256) uprolong_kernel(long nIrow, long nface, long N, long Nc,
                                                       const int* __restrict__ irc, const long* __restrict__ iptr,
                                                       const int* __restrict__ iface, const long* __restrict__ csptr,
                                                       const int* __restrict__ csface, const long* __restrict__ poff,
                                                       const M* __restrict__ P, const int* __restrict__ fE,
                                                       const double* __restrict__ fJ, const T* __restrict__ ec,
                                                       T* __restrict__ e) {
  using A = acc_t<T>;
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  e += rhs * N;
  ec += rhs * Nc;
  if (g < nIrow) {
    const long C = irc[g];
    const long i0 = iptr[C], c0 = csptr[C];
    const int nc2 = 2 * (int)(csptr[C + 1] - c0);
    const long li = g - 2 * i0;
    const M* row = P + poff[C] + li * nc2;
    A s = A(0);
    for (int q2 = 0; q2 < nc2; ++q2) s += A(row[q2]) * A(ec[2L * csface[c0 + q2 / 2] + q2 % 2]);
    const long dof = 2L * iface[i0 + li / 2] + li % 2;
    e[dof] = T(A(e[dof]) + s);
    return;
  }
  const long f = g - nIrow;
  if (f >= nface) return;
  const int E = fE[f];
  if (E < 0) return;
  const A c0 = A(ec[2L * E]), c1 = A(ec[2L * E + 1]);
  e[2 * f] = T(A(e[2 * f]) + A(fJ[4 * f + 0]) * c0 + A(fJ[4 * f + 1]) * c1);
  e[2 * f + 1] = T(A(e[2 * f + 1]) + A(fJ[4 * f + 2]) * c0 + A(fJ[4 * f + 3]) * c1);
}

template <typename F>
void dispatch_k(int k, F&& f) {
  switch (k) {
    case 1: f(std::integral_constant<int, 1>{}); return;
    case 2: f(std::integral_constant<int, 2>{}); return;
    case 3: f(std::integral_constant<int, 3>{}); return;
    case 4: f(std::integral_constant<int, 4>{}); return;
  }
  throw HipError{hipErrorInvalidValue, "triangle degree"};
}

template <typename F>
void dispatch_m(int m, F&& f) {
  switch (m) {
    case 2: f(std::integral_constant<int, 2>{}); return;
    case 3: f(std::integral_constant<int, 3>{}); return;
    case 4: f(std::integral_constant<int, 4>{}); return;
    case 5: f(std::integral_constant<int, 5>{}); return;
  }
  throw HipError{hipErrorInvalidValue, "face size"};
}

}  // namespace

// ---------------------------------------------------------------------------
void launch_tri_dtn(int k, long ntri, const RefDevice& rd, const double* xy, const int* tri, const double* kappa,
                    double tau, double* Aelem, double* W, double* Rec, hipStream_t st) {
  if (ntri == 0) return;
  dispatch_k(k, [&](auto K_) {
    constexpr int K = decltype(K_)::value;
    hipLaunchKernelGGL((tri_dtn_kernel<K>), dim3((unsigned)ntri), dim3(64), 0, st, ntri, rd.uM, rd.uMinv, rd.uD,
                       rd.uE, rd.uF, rd.uH, xy, tri, kappa, tau, Aelem, W, Rec);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_tri_ipdg_dtn(int k, long ntri, const RefDevice& rd, const double* xy, const int* tri,
                         const double* kappa, double tau, double sf, double* Aelem, double* W, double* Rec,
                         hipStream_t st) {
  if (ntri == 0) return;
  dispatch_k(k, [&](auto K_) {
    constexpr int K = decltype(K_)::value;
    hipLaunchKernelGGL((tri_ipdg_dtn_kernel<K>), dim3((unsigned)ntri), dim3(64), 0, st, ntri, rd.uM, rd.uK, rd.uN,
                       rd.uDe, rd.uE, rd.uF, rd.uH, rd.uGn, xy, tri, kappa, tau, sf, Aelem, W, Rec);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_tri_load(int k, const ULevel& U, const double* W, const double* f, const double* Aelem,
                     const int* tbnd, const double* gdir, double* g, hipStream_t st) {
  if (U.nface == 0) return;
  dispatch_k(k, [&](auto K_) {
    constexpr int K = decltype(K_)::value;
    hipLaunchKernelGGL((tri_load_kernel<K>), dim3(nb256(U.nface)), dim3(256), 0, st, U.nface, U.fcell, U.fslot, W, f,
                       Aelem, tbnd, gdir, g);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_tri_reconstruct(int k, long ntri, const int* sface, const int* tbnd, const double* Rec,
                            const double* lam, const double* gdir, const double* f, double* u, double* q,
                            hipStream_t st) {
  if (ntri == 0) return;
  dispatch_k(k, [&](auto K_) {
    constexpr int K = decltype(K_)::value;
    hipLaunchKernelGGL((tri_reconstruct_kernel<K>), dim3(nb256(ntri)), dim3(256), 0, st, ntri, sface, tbnd, Rec, lam,
                       gdir, f, u, q);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_tri_pgalerkin(int k, long ntri, const double* Jp, const double* A0, double* A1, hipStream_t st) {
  if (ntri == 0) return;
  hipLaunchKernelGGL(tri_pgalerkin_kernel, dim3(nb256(ntri * 36)), dim3(256), 0, st, ntri, k + 1, Jp, A0, A1);
  HDG_CHECK(hipGetLastError());
}

void launch_uschur(const ULevel& F, const ULevel& C, const double* Afine, double* AIIinv, double* P, double* R,
                   double* Acoarse, double* work, hipStream_t st) {
  if (F.ncoarse == 0) return;
  hipLaunchKernelGGL(uschur_kernel, dim3((unsigned)F.ncoarse), dim3(256), 0, st, F.ncoarse, F.ccptr, F.ccell, F.sptr,
                     F.sloc, F.moff, F.iptr, F.bptr, F.bface, F.bslot, F.fJ, C.sptr, C.moff, F.aoff, F.poff, F.woff,
                     Afine, AIIinv, P, R, Acoarse, work);
  HDG_CHECK(hipGetLastError());
}

void launch_udinv(const Level& L, hipStream_t st) {
  const ULevel& U = *L.u;
  if (U.nface == 0) return;
  dispatch_m(U.m, [&](auto M_) {
    constexpr int NE = decltype(M_)::value;
    hipLaunchKernelGGL((udinv_kernel<NE>), dim3(nb256(U.nface)), dim3(256), 0, st, U.nface, U.fcell, U.fslot, U.sptr,
                       U.moff, L.Aelem, L.Dinv64, L.Dinv32);
  });
  HDG_CHECK(hipGetLastError());
}

void launch_dense_inverse_blocked(long N, double* A, double* Pb, hipStream_t st) {
  if (N <= 0) return;
  if (N > 64L * 65535) throw HipError{hipErrorInvalidValue, "dense inverse too large"};
  const int nbk = (int)((N + UBK - 1) / UBK);
  for (int p = 0; p < nbk; ++p) {
    hipLaunchKernelGGL(ublk_pivot_kernel, dim3(1), dim3(256), 0, st, N, p, A, Pb);
    hipLaunchKernelGGL(ublk_row_kernel, dim3(nbk), dim3(256), 0, st, N, p, Pb, A);
    hipLaunchKernelGGL(ublk_trail_kernel, dim3(nbk, nbk), dim3(256), 0, st, N, p, A);
    hipLaunchKernelGGL(ublk_col_kernel, dim3(nbk), dim3(256), 0, st, N, p, Pb, A);
  }
  HDG_CHECK(hipGetLastError());
}

void launch_ucoarse_inverse(const Level& L, double* work, hipStream_t st) {
  const ULevel& U = *L.u;
  const long N = L.nlam;
  if (N == 0) return;
  if (N > UCOARSE_MAX) throw HipError{hipErrorInvalidValue, "coarsest level too large for the dense inverse"};
  hipLaunchKernelGGL(udense_kernel, dim3(nb256(N)), dim3(256), 0, st, U.nface, U.m, U.fcell, U.fslot, U.sptr,
                     U.sface, U.moff, L.Aelem, work);
  if (N <= 512) {
    hipLaunchKernelGGL(udense_inverse_kernel, dim3(1), dim3(256), 0, st, (int)N, work, L.Ainv64, L.Ainv32);
  } else {  // work holds two N x N buffers: A, then the pivot-block inverse
    double* A = work;
    launch_dense_inverse_blocked(N, A, work + N * N, st);
    HDG_CHECK(hipMemcpyAsync(L.Ainv64, A, sizeof(double) * N * N, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(f32_kernel, dim3(1024), dim3(256), 0, st, A, L.Ainv32, N * N);
  }
  HDG_CHECK(hipGetLastError());
}

void launch_umaps(const Level& L, hipStream_t st) {
  const ULevel& U = *L.u;
  if (U.tri) {
    const int nn = 9 * U.m * U.m;
    hipLaunchKernelGGL(tri_aos_kernel, dim3(nb256(U.ncell * nn)), dim3(256), 0, st, U.ncell, nn, L.Aelem, L.Af64,
                       L.Af32);
  } else if (U.msize > 0) {
    hipLaunchKernelGGL(f32_kernel, dim3(1024), dim3(256), 0, st, L.Aelem, U.Am32, U.msize);
  }
  HDG_CHECK(hipGetLastError());
}

void launch_to_f32(const double* x, float* y, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(f32_kernel, dim3(1024), dim3(256), 0, st, x, y, n);
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_uapply(const Level& L, int mode, const T* x, const T* b, T* y, const double* Jp, T* rc, float* y32,
                   Scratch* red, hipStream_t st, int nrhs, int* nparts) {
  const ULevel& U = *L.u;
  if (U.nface == 0) return;
  const bool rmode = mode == APPLY_Y_DOT || mode == APPLY_RES_NORM || mode == APPLY_SWEEP_DOT;
  T* z = (T*)U.z[sizeof(T) == 8 ? 0 : 1];
  if (U.tri) {
    const M* Af = sizeof(M) == 8 ? (const M*)L.Af64 : (const M*)L.Af32;
    const unsigned nb = (unsigned)((U.ncell + LANES - 1) / LANES);
    dispatch_m(U.m, [&](auto M_) {
      constexpr int NE = decltype(M_)::value;
      constexpr int CH = NE == 2 ? 3 : 4;
      hipLaunchKernelGGL((utri_phase_kernel<NE, T, M, CH>), dim3(nb, nrhs), dim3(64 * CH), 0, st, U.ncell, U.nrow,
                         L.nlam, U.sface, Af, x, z);
    });
  } else {
    const M* Am = sizeof(M) == 8 ? (const M*)L.Aelem : (const M*)U.Am32;
    hipLaunchKernelGGL((ucell_phase_kernel<T, M>), dim3(nb256(U.nrow), nrhs), dim3(256), 0, st, U.nrow, L.nlam, U.m,
                       U.rcell, U.sptr, U.sface, U.moff, Am, x, z);
  }
  HDG_CHECK(hipGetLastError());
  const M* Dv = sizeof(M) == 8 ? (const M*)L.Dinv64 : (const M*)L.Dinv32;
  const unsigned g = (unsigned)std::min<long>(nb256(U.nface), MAX_RED_BLOCKS);
  if (red && rmode && (long)g > red->row) throw HipError{hipErrorInvalidValue, "trace apply: too many partial sums"};
  double* partials = red ? red->partials : nullptr;
  dispatch_m(U.m, [&](auto M_) {
    constexpr int NE = decltype(M_)::value;
#define HDG_UF(MM)                                                                                                \
  hipLaunchKernelGGL((uface_kernel<NE, T, MM, M>), dim3(g, nrhs), dim3(256), 0, st, U.nface, U.nrow, U.zr, U.zstride, z, Dv, x, \
                     b, y, Jp, rc, y32, partials)
    switch (mode) {
      case APPLY_Y: HDG_UF(APPLY_Y); break;
      case APPLY_RES: HDG_UF(APPLY_RES); break;
      case APPLY_SWEEP: HDG_UF(APPLY_SWEEP); break;
      case APPLY_RES_PRESTRICT: HDG_UF(APPLY_RES_PRESTRICT); break;
      case APPLY_Y_DOT: HDG_UF(APPLY_Y_DOT); break;
      case APPLY_RES_NORM: HDG_UF(APPLY_RES_NORM); break;
      case APPLY_SWEEP_DOT: HDG_UF(APPLY_SWEEP_DOT); break;
      default: throw HipError{hipErrorInvalidValue, "apply mode"};
    }
#undef HDG_UF
  });
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
}

template <typename T, typename M>
void launch_ucorr(const Level& L, const T* rho, T* e, int do_corr, int do_restrict, T* cb, hipStream_t st, int nrhs) {
  const ULevel& U = *L.u;
  const long rows = U.nIrow + U.ncb;
  if (rows == 0) return;
  const M* Ai = sizeof(M) == 8 ? (const M*)L.AIIinv64 : (const M*)L.AIIinv32;
  const M* R = sizeof(M) == 8 ? (const M*)L.R64 : (const M*)L.R32;
  hipLaunchKernelGGL((ucorr_kernel<T, M>), dim3(nb256(rows), nrhs), dim3(256), 0, st, U.nIrow, U.ncb, L.nlam, U.irc,
                     U.cbc, U.iptr, U.iface, U.csptr, U.aoff, U.poff, Ai, R, rho, e, do_corr, do_restrict, cb);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void launch_urestrict(const Level& L, const Level& C, const T* rho, const T* cb, T* rc, hipStream_t st, int nrhs) {
  const ULevel& U = *L.u;
  const ULevel& Uc = *C.u;
  if (Uc.nface == 0) return;
  hipLaunchKernelGGL((urestrict_kernel<T>), dim3(nb256(Uc.nface), nrhs), dim3(256), 0, st, Uc.nface, L.nlam, C.nlam,
                     U.ncb, Uc.eptr, Uc.efine, U.fJ, Uc.zr, rho, cb, rc);
  HDG_CHECK(hipGetLastError());
}

template <typename T, typename M>
void launch_uprolong(const Level& L, const Level& C, const T* ec, T* e, hipStream_t st, int nrhs) {
  const ULevel& U = *L.u;
  const ULevel& Uc = *C.u;
  const M* P = sizeof(M) == 8 ? (const M*)L.P64 : (const M*)L.P32;
  const long rows = U.nIrow + U.nface;
  if (rows == 0) return;
  hipLaunchKernelGGL((uprolong_kernel<T, M>), dim3(nb256(rows), nrhs), dim3(256), 0, st, U.nIrow, U.nface, L.nlam,
                     C.nlam, U.irc, U.iptr, U.iface, Uc.sptr, Uc.sface, U.poff, P, U.fE, U.fJ, ec, e);
  HDG_CHECK(hipGetLastError());
}

#define HDG_UINST_M(T, M)                                                                                         \
  template void launch_uapply<T, M>(const Level&, int, const T*, const T*, T*, const double*, T*, float*, Scratch*, \
                                    hipStream_t, int, int*);                                                      \
  template void launch_ucorr<T, M>(const Level&, const T*, T*, int, int, T*, hipStream_t, int);                   \
  template void launch_uprolong<T, M>(const Level&, const Level&, const T*, T*, hipStream_t, int);
HDG_UINST_M(double, double)
HDG_UINST_M(double, float)
HDG_UINST_M(float, float)
#undef HDG_UINST_M
template void launch_urestrict<double>(const Level&, const Level&, const double*, const double*, double*, hipStream_t,
                                       int);
template void launch_urestrict<float>(const Level&, const Level&, const float*, const float*, float*, hipStream_t,
                                      int);

}  // namespace hdg
