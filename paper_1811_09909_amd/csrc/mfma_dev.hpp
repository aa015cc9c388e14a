// Workgroup-level FP64 matrix-core helpers shared by the element and the
// macro-element kernels (gfx950, v_mfma_f64_16x16x4f64): dense products of
// operands held in LDS or read through the caches, and a blocked in-place
// Gauss-Jordan inverse whose block updates run on the matrix cores.
#pragma once

#include <hip/hip_runtime.h>

namespace hdg {

typedef double mf_d4 __attribute__((ext_vector_type(4)));

// One 16 x 16 output tile of sum_k a(i, k) b(k, j) over K = 16 on the matrix
// cores (four v_mfma_f64_16x16x4f64); lane l supplies a(l % 16, k0 + l / 16)
// and b(k0 + l / 16, l % 16) and receives rows l / 16 + 4 r of column l % 16.
template <typename FA, typename FB>
__device__ inline mf_d4 tile16(FA a, FB b) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, l4 = lane >> 4;
  mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(l16, k0 + l4), b(k0 + l4, l16), acc, 0, 0, 0);
  return acc;
}

// In-place Gauss-Jordan inverse of an N x N matrix in LDS without pivoting
// (SPD matrices, and the local matrices of the nonsymmetric schemes, whose
// leading blocks are invertible), N a multiple of 16, by 16 x 16 blocks:
// step p inverts the diagonal block in the registers of wave 0 (lane holds
// four entries of one row; pivot rows and columns travel by shuffles, no
// barrier), then A_pj <- P A_pj, A_ij -= A_ip A_pj (i, j != p),
// A_ip <- -A_ip P and A_pp <- P with P the block inverse, every block
// product a 16 x 16 x 16 MFMA tile.  Four barriers per block step instead of
// one per pivot; the same elimination as the pivot-by-pivot sweep up to the
// rounding order.
template <int N, int NT>
__device__ void gj_inverse_blocked(double* A) {
  static_assert(N % 16 == 0, "16 x 16 blocks");
  constexpr int NB = N / 16, NW = NT / 64;
  __shared__ double Pv[256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, l4 = lane >> 4;
  for (int p = 0; p < NB; ++p) {
    __syncthreads();
    if (wave == 0) {
      const int i = lane >> 2, cq = lane & 3;
      double v[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) v[m] = A[(p * 16 + i) * N + p * 16 + 4 * cq + m];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int km = k & 3;  // register of column k (selected without indexing, so v stays in registers)
        const double vk = km == 0 ? v[0] : km == 1 ? v[1] : km == 2 ? v[2] : v[3];
        const double piv = __shfl(vk, 4 * k + (k >> 2), 64);
        const double pinv = 1.0 / piv;
        const double cik = __shfl(vk, 4 * i + (k >> 2), 64);
        double rk[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) rk[m] = __shfl(v[m], 4 * k + cq, 64);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int j = 4 * cq + m;
          if (i == k)
            v[m] = (j == k) ? pinv : rk[m] * pinv;
          else if (j == k)
            v[m] = -cik * pinv;
          else
            v[m] -= cik * rk[m] * pinv;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) Pv[i * 16 + 4 * cq + m] = v[m];
    }
    __syncthreads();
    // pivot block row: A_pj <- P A_pj (each tile read and written by one wave)
    for (int jb = wave; jb < NB; jb += NW) {
      if (jb == p) continue;
      const mf_d4 acc = tile16([](int i, int k) { return Pv[i * 16 + k]; },
                               [A, p, jb](int k, int j) { return A[(p * 16 + k) * N + jb * 16 + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) A[(p * 16 + l4 + 4 * r) * N + jb * 16 + l16] = acc[r];
    }
    __syncthreads();
    // trailing blocks: A_ij -= A_ip A_pj
    for (int t = wave; t < NB * NB; t += NW) {
      const int ib = t / NB, jb = t % NB;
      if (ib == p || jb == p) continue;
      const mf_d4 acc = tile16([A, p, ib](int i, int k) { return A[(ib * 16 + i) * N + p * 16 + k]; },
                               [A, p, jb](int k, int j) { return A[(p * 16 + k) * N + jb * 16 + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) A[(ib * 16 + l4 + 4 * r) * N + jb * 16 + l16] -= acc[r];
    }
    __syncthreads();
    // pivot block column: A_ip <- -A_ip P; pivot block: P
    for (int ib = wave; ib < NB; ib += NW) {
      if (ib == p) continue;
      const mf_d4 acc = tile16([A, p, ib](int i, int k) { return A[(ib * 16 + i) * N + p * 16 + k]; },
                               [](int k, int j) { return Pv[k * 16 + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) A[(ib * 16 + l4 + 4 * r) * N + p * 16 + l16] = -acc[r];
    }
    for (int idx = threadIdx.x; idx < 256; idx += NT) A[(p * 16 + idx / 16) * N + p * 16 + idx % 16] = Pv[idx];
  }
  __syncthreads();
}

// k-steps of a product tile unrolled (loads of several steps in flight)
#ifndef HDG_WG_MFMA_UNROLL
#define HDG_WG_MFMA_UNROLL 4
#endif

// Dense product on the matrix cores, shared by the workgroup's wavefronts:
// for every (i, j) of an M x N output, s = sum_k a(i, k) b(k, j), and
// c(i, j, s) is called once, by the lane that holds the entry.  Output tiles
// of 16 x 16 go to the wavefronts round-robin; each is accumulated by
// v_mfma_f64_16x16x4f64 over K in steps of 4 (indices past M, N or K read
// as 0).  Lane l supplies a(i0 + l % 16, k0 + l / 16) and
// b(k0 + l / 16, j0 + l % 16) and receives rows i0 + l / 16 + 4 r (r = 0..3)
// of column j0 + l % 16.  The tile loop is uniform over a wavefront, so every
// lane issues every MFMA.
template <int M, int N, int K, int NT, typename FA, typename FB, typename FC>
__device__ inline void wg_mfma(FA a, FB b, FC c) {
  constexpr int TM = (M + 15) / 16, TN = (N + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  for (int t = wave; t < TM * TN; t += NT / 64) {
    const int i0 = (t / TN) * 16, j0 = (t % TN) * 16;
    const int ia = i0 + l16, jb = j0 + l16;
    mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll HDG_WG_MFMA_UNROLL
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + l4;
      const double av = (ia < M && k < K) ? a(ia, k) : 0.0;
      const double bv = (jb < N && k < K) ? b(k, jb) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + l4 + 4 * r;
      if (i < M && jb < N) c(i, jb, acc[r]);
    }
  }
}

}  // namespace hdg
