// Vector kernels of the outer iterations (fixed point, CG, GMRES; Sec. 3.6
// and Sec. 4).
//
// Reductions: every block writes one partial sum (wavefront shuffles, then
// LDS) with plain stores, and a one-block finaliser launched next sums the
// partials in block order and updates the device scalars.  The grid depends
// only on the vector length, so sums are reproducible.  No device-scope
// fences or atomics: on MI355X the eight XCDs' L2 caches are not coherent
// with each other, so a per-block release fence costs an L2 write-back and a
// per-block atomic on one counter serialises; the kernel boundary is the
// cheap synchronisation point.
//
// Several right-hand sides: vectors of length n stored one after another,
// blockIdx.y selects one; each has its own scalar block (sc + rhs * SC_COUNT)
// and its own row of partials ([rhs][blocks]); the finaliser runs one block
// per right-hand side.
#include "blas.hpp"
#include "hdg_internal.hpp"
#include "reduce.hpp"

namespace hdg {

namespace {

constexpr int RB = 256;  // reduction block size
constexpr int RPT = 4;   // elements per thread per pass (independent loads in flight)

__device__ inline double block_sum(double v, double* sh) { return block_sum_t<RB>(v, sh); }

// Per-thread share of a fixed-order sum of partials: terms i = tid, tid + RB,
// tid + 2 RB, ... < cnt added in that order (so the block sum that follows is
// the same as a plain strided loop's), with the loads of PU consecutive
// terms issued before any is added.  The partials come from workgroups on
// every XCD, so each load waits on the memory side: one at a time would
// chain those waits.  nv values per index, component v.
constexpr int PU = 8;
__device__ inline double strided_sum(const double* __restrict__ p, int cnt, int nv, int v) {
  double a = 0.0;
  for (int i0 = threadIdx.x; i0 < cnt; i0 += PU * RB) {
    double x[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int i = i0 + u * RB;
      x[u] = i < cnt ? p[(long)nv * i + v] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PU; ++u)
      if (i0 + u * RB < cnt) a += x[u];
  }
  return a;
}

__global__ void __launch_bounds__(RB) dot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                 long n, double* __restrict__ partials) {
  __shared__ double sh[RB / 64];
  x += blockIdx.y * n;
  y += blockIdx.y * n;
  partials += blockIdx.y * (long)gridDim.x;
  double v = 0.0;
  for (long base = blockIdx.x * (long)RB * RPT; base < n; base += (long)gridDim.x * RB * RPT) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const long i = base + u * RB + threadIdx.x;
      if (i < n) v += x[i] * y[i];
    }
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// sum partials[nv * i + v] over i < nb (fixed order) and apply the finaliser
__global__ void __launch_bounds__(RB) finalize_kernel(const double* __restrict__ partials, int nb, int nv, int mode,
                                                      double* sc, double* out) {
  __shared__ double sh[RB / 64];
  partials += blockIdx.x * (long)nb * nv;
  sc += blockIdx.x * (long)SC_COUNT;
  if (out) out += blockIdx.x;
  double tot[2] = {0.0, 0.0};
  for (int v = 0; v < nv; ++v) {
    tot[v] = block_sum(strided_sum(partials, nb, nv, v), sh);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double t0 = tot[0], t1 = tot[1];
  // a zero denominator only occurs once the residual is exactly zero: the
  // step is then zero instead of 0/0
  switch (mode) {
    case FIN_STORE: *out = t0; break;
    case FIN_ALPHA:
      sc[SC_PAP] = t0;
      sc[SC_ALPHA] = t0 != 0.0 ? sc[SC_RZ] / t0 : 0.0;
      break;
    case FIN_BETA:
      sc[SC_BETA] = sc[SC_RZ] != 0.0 ? t0 / sc[SC_RZ] : 0.0;
      sc[SC_RZ] = t0;
      break;
    case FIN_BETA_FLEX:
      sc[SC_BETA] = sc[SC_RZ] != 0.0 ? (t0 - sc[SC_RZOLD]) / sc[SC_RZ] : 0.0;
      sc[SC_RZ] = t0;
      break;
    case FIN_RZ0: sc[SC_RZ] = t0; break;
    case FIN_GNORM: sc[SC_GNORM2] = t0; break;
    case FIN_NORM_INV:
      *out = sqrt(t0);
      sc[SC_TMP] = t0 > 0.0 ? 1.0 / sqrt(t0) : 0.0;
      break;
    case FIN_RNORM:
    case FIN_RNORM_RZOLD: {
      sc[SC_RNORM2] = t0;
      if (mode == FIN_RNORM_RZOLD) sc[SC_RZOLD] = t1;
      // history of squared residual norms since the host last reset the count
      const int c = (int)sc[SC_HCNT];
      if (c >= 0 && c < HIST_MAX) sc[SC_HIST + c] = t0;
      sc[SC_HCNT] = (double)(c + 1);
      break;
    }
  }
}

// Fused CG update (one pass over the vectors):
//   lam += alpha p ; r -= alpha Ap ; r32 = (float) r (mixed only)
//   partial sums of r.r and r.z_old, where z still holds the previous
//   preconditioned residual.
// With papp: alpha = rz / pAp is formed in every block from the pAp
// partials of the apply (npap per right-hand side, summed in the
// finaliser's order); block 0 also stores pAp and alpha.
template <typename ZT>
__global__ void __launch_bounds__(RB) cg_update2_kernel(double* __restrict__ lam, double* __restrict__ r,
                                                        float* __restrict__ r32, const double* __restrict__ p,
                                                        const double* __restrict__ Ap, const ZT* __restrict__ z,
                                                        long n, double* __restrict__ partials, double* sc,
                                                        const double* __restrict__ papp, int npap) {
  __shared__ double sh[RB / 64];
  __shared__ double alpha_sh;
  {
    const long o = blockIdx.y * n;
    lam += o;
    r += o;
    r32 = r32 ? r32 + o : r32;
    p += o;
    Ap += o;
    z += o;
    partials += blockIdx.y * 2L * gridDim.x;
    sc += blockIdx.y * (long)SC_COUNT;
  }
  double alpha;
  if (papp) {
    papp += blockIdx.y * (long)npap;
    const double t0 = block_sum(strided_sum(papp, npap, 1, 0), sh);
    if (threadIdx.x == 0) {
      const double al = t0 != 0.0 ? sc[SC_RZ] / t0 : 0.0;
      alpha_sh = al;
      if (blockIdx.x == 0) {
        sc[SC_PAP] = t0;
        sc[SC_ALPHA] = al;
      }
    }
    __syncthreads();
    alpha = alpha_sh;
  } else {
    alpha = sc[SC_ALPHA];
  }
  double rr = 0.0, rz = 0.0;
  for (long base = blockIdx.x * (long)RB * RPT; base < n; base += (long)gridDim.x * RB * RPT) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const long i = base + u * RB + threadIdx.x;
      if (i < n) {
        lam[i] += alpha * p[i];
        const double ri = r[i] - alpha * Ap[i];
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
        rr += ri * ri;
        rz += ri * (double)z[i];
      }
    }
  }
  const double sa = block_sum(rr, sh);
  __syncthreads();
  const double sb = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sa;
    partials[2 * blockIdx.x + 1] = sb;
  }
}

// finaliser of a fused CG iteration: residual norm (and history) and rz_old
// from the update's partials, then beta from the r.z partials
__global__ void __launch_bounds__(RB) finalize_cg_kernel(const double* __restrict__ pcg, int ncg,
                                                         const double* __restrict__ prz, int nrz, int flex,
                                                         double* sc) {
  __shared__ double sh[RB / 64];
  pcg += blockIdx.x * 2L * ncg;
  prz += blockIdx.x * (long)nrz;
  sc += blockIdx.x * (long)SC_COUNT;
  double t[3];
  // the three per-thread shares first (all their loads in flight), then the
  // three block sums in the same order as before
  const double a0 = strided_sum(pcg, ncg, 2, 0);
  const double a1 = strided_sum(pcg, ncg, 2, 1);
  const double a2 = strided_sum(prz, nrz, 1, 0);
  const double a[3] = {a0, a1, a2};
  for (int v = 0; v < 3; ++v) {
    t[v] = block_sum(a[v], sh);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  sc[SC_RNORM2] = t[0];
  sc[SC_RZOLD] = t[1];
  const int c = (int)sc[SC_HCNT];
  if (c >= 0 && c < HIST_MAX) sc[SC_HIST + c] = t[0];
  sc[SC_HCNT] = (double)(c + 1);
  if (flex)
    sc[SC_BETA] = sc[SC_RZ] != 0.0 ? (t[2] - sc[SC_RZOLD]) / sc[SC_RZ] : 0.0;
  else
    sc[SC_BETA] = sc[SC_RZ] != 0.0 ? t[2] / sc[SC_RZ] : 0.0;
  sc[SC_RZ] = t[2];
}

// partial sums of r.z (z FP64 or FP32)
template <typename ZT>
__global__ void __launch_bounds__(RB) rz_kernel(const double* __restrict__ r, const ZT* __restrict__ z, long n,
                                                double* __restrict__ partials) {
  __shared__ double sh[RB / 64];
  r += blockIdx.y * n;
  z += blockIdx.y * n;
  partials += blockIdx.y * (long)gridDim.x;
  double v = 0.0;
  for (long base = blockIdx.x * (long)RB * RPT; base < n; base += (long)gridDim.x * RB * RPT) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const long i = base + u * RB + threadIdx.x;
      if (i < n) v += r[i] * (double)z[i];
    }
  }
  const double s = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p
template <typename ZT>
__global__ void cg_dir_kernel(double* __restrict__ p, const ZT* __restrict__ z, long n, const double* sc) {
  p += blockIdx.y * n;
  z += blockIdx.y * n;
  const double beta = sc[blockIdx.y * (long)SC_COUNT + SC_BETA];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) p[i] = (double)z[i] + beta * p[i];
}

// lam += z (z FP64 or FP32)
template <typename ZT>
__global__ void add_kernel(double* __restrict__ lam, const ZT* __restrict__ z, long n) {
  lam += blockIdx.y * n;
  z += blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) lam[i] += (double)z[i];
}

// y += sign * x, or y += sign * (*coef) * x when coef is given
__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, long n, const double* coef,
                            double sign) {
  const double a = coef ? sign * (*coef) : sign;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] += a * x[i];
}

// y = (*coef) * x
__global__ void scale_kernel(double* __restrict__ y, const double* __restrict__ x, long n, const double* coef) {
  const double a = *coef;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = a * x[i];
}

template <typename A, typename B>
__global__ void convert_kernel(const A* __restrict__ x, B* __restrict__ y, long n) {
  x += blockIdx.y * n;
  y += blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = (B)x[i];
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ y, T v, long n) {
  y += blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = v;
}

template <typename T>
__global__ void copy_t_kernel(T* __restrict__ y, const T* __restrict__ x, long n) {
  y += blockIdx.y * n;
  x += blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = x[i];
}

// GMRES: apply old rotations to column j of H, make a new one, update s.
// H column-major with leading dimension ld; cs, sn, s device arrays.
__global__ void gmres_rot_kernel(double* H, double* cs, double* sn, double* s, int j, int ld, double* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* h = H + (long)j * ld;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * h[i] + sn[i] * h[i + 1];
    h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
    h[i] = t;
  }
  const double den = hypot(h[j], h[j + 1]);
  if (den == 0.0) {
    cs[j] = 1.0;
    sn[j] = 0.0;
  } else {
    cs[j] = h[j] / den;
    sn[j] = h[j + 1] / den;
  }
  h[j] = den;
  h[j + 1] = 0.0;
  s[j + 1] = -sn[j] * s[j];
  s[j] = cs[j] * s[j];
  sc[SC_GRES] = fabs(s[j + 1]);
}

// back substitution H(0:j,0:j) y = s(0:j)
__global__ void gmres_backsolve_kernel(const double* H, const double* s, int j, int ld, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = j - 1; i >= 0; --i) {
    double v = s[i];
    for (int l = i + 1; l < j; ++l) v -= H[(long)l * ld + i] * y[l];
    y[i] = v / H[(long)i * ld + i];
  }
}

// x += sum_i y_i Z_i  (Z: j vectors of length n, stride ldz)
__global__ void gmres_combine_kernel(double* __restrict__ x, const double* __restrict__ Z, long ldz, int j,
                                     const double* __restrict__ y, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) {
    double v = x[i];
    for (int l = 0; l < j; ++l) v += y[l] * Z[l * ldz + i];
    x[i] = v;
  }
}

inline unsigned gs(long n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// the grid depends only on n, so sums are reproducible run to run
inline unsigned rg(long n) {
  long b = (n + RB * RPT - 1) / (RB * RPT);
  if (b > MAX_RED_BLOCKS) b = MAX_RED_BLOCKS;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void blas_finalize(int nb, int nv, int mode, double* out, Scratch& s, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(RB), 0, st, s.partials, nb, nv, mode, s.sc, out);
  HDG_CHECK(hipGetLastError());
}

void blas_dot(const double* x, const double* y, long n, Scratch& s, int mode, double* out, hipStream_t st,
              int nrhs) {
  const unsigned nb = rg(n);
  hipLaunchKernelGGL(dot_kernel, dim3(nb, nrhs), dim3(RB), 0, st, x, y, n, s.partials);
  HDG_CHECK(hipGetLastError());
  blas_finalize((int)nb, 1, mode, out, s, st, nrhs);
}

template <typename ZT>
void blas_cg_update2(double* lam, double* r, float* r32, const double* p, const double* Ap, const ZT* z, long n,
                     Scratch& s, hipStream_t st, int nrhs) {
  const unsigned nb = rg(n);
  hipLaunchKernelGGL((cg_update2_kernel<ZT>), dim3(nb, nrhs), dim3(RB), 0, st, lam, r, r32, p, Ap, z, n, s.partials,
                     s.sc, nullptr, 0);
  HDG_CHECK(hipGetLastError());
  blas_finalize((int)nb, 2, FIN_RNORM_RZOLD, nullptr, s, st, nrhs);
}

template <typename ZT>
void blas_cg_update2_fused(double* lam, double* r, float* r32, const double* p, const double* Ap, const ZT* z,
                           long n, int npap, Scratch& s, hipStream_t st, int nrhs) {
  const unsigned nb = rg(n);
  hipLaunchKernelGGL((cg_update2_kernel<ZT>), dim3(nb, nrhs), dim3(RB), 0, st, lam, r, r32, p, Ap, z, n, s.pcg, s.sc,
                     s.partials, npap);
  HDG_CHECK(hipGetLastError());
}
template void blas_cg_update2_fused<double>(double*, double*, float*, const double*, const double*, const double*,
                                            long, int, Scratch&, hipStream_t, int);
template void blas_cg_update2_fused<float>(double*, double*, float*, const double*, const double*, const float*,
                                           long, int, Scratch&, hipStream_t, int);

template <typename ZT>
void blas_rz_cg(const double* r, const ZT* z, long n, bool flex, Scratch& s, hipStream_t st, int nrhs) {
  const unsigned nb = rg(n);
  hipLaunchKernelGGL((rz_kernel<ZT>), dim3(nb, nrhs), dim3(RB), 0, st, r, z, n, s.partials);
  HDG_CHECK(hipGetLastError());
  hipLaunchKernelGGL(finalize_cg_kernel, dim3(nrhs), dim3(RB), 0, st, s.pcg, (int)nb, s.partials, (int)nb,
                     flex ? 1 : 0, s.sc);
  HDG_CHECK(hipGetLastError());
}
template void blas_rz_cg<double>(const double*, const double*, long, bool, Scratch&, hipStream_t, int);

void blas_finalize_cg(long n, int nrz, bool flex, Scratch& s, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL(finalize_cg_kernel, dim3(nrhs), dim3(RB), 0, st, s.pcg, (int)rg(n), s.partials, nrz,
                     flex ? 1 : 0, s.sc);
  HDG_CHECK(hipGetLastError());
}
template void blas_rz_cg<float>(const double*, const float*, long, bool, Scratch&, hipStream_t, int);
template void blas_cg_update2<double>(double*, double*, float*, const double*, const double*, const double*, long,
                                      Scratch&, hipStream_t, int);
template void blas_cg_update2<float>(double*, double*, float*, const double*, const double*, const float*, long,
                                     Scratch&, hipStream_t, int);

template <typename ZT>
void blas_rz(const double* r, const ZT* z, long n, int mode, Scratch& s, hipStream_t st, int nrhs) {
  const unsigned nb = rg(n);
  hipLaunchKernelGGL((rz_kernel<ZT>), dim3(nb, nrhs), dim3(RB), 0, st, r, z, n, s.partials);
  HDG_CHECK(hipGetLastError());
  blas_finalize((int)nb, 1, mode, nullptr, s, st, nrhs);
}
template void blas_rz<double>(const double*, const double*, long, int, Scratch&, hipStream_t, int);
template void blas_rz<float>(const double*, const float*, long, int, Scratch&, hipStream_t, int);

template <typename ZT>
void blas_cg_dir(double* p, const ZT* z, long n, Scratch& s, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL((cg_dir_kernel<ZT>), dim3(gs(n), nrhs), dim3(256), 0, st, p, z, n, s.sc);
  HDG_CHECK(hipGetLastError());
}
template void blas_cg_dir<double>(double*, const double*, long, Scratch&, hipStream_t, int);
template void blas_cg_dir<float>(double*, const float*, long, Scratch&, hipStream_t, int);

template <typename ZT>
void blas_add(double* lam, const ZT* z, long n, hipStream_t st, int nrhs) {
  hipLaunchKernelGGL((add_kernel<ZT>), dim3(gs(n), nrhs), dim3(256), 0, st, lam, z, n);
  HDG_CHECK(hipGetLastError());
}
template void blas_add<double>(double*, const double*, long, hipStream_t, int);
template void blas_add<float>(double*, const float*, long, hipStream_t, int);

void blas_axpy(double* y, const double* x, long n, const double* coef, double sign, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3(gs(n)), dim3(256), 0, st, y, x, n, coef, sign);
  HDG_CHECK(hipGetLastError());
}

void blas_scale(double* y, const double* x, long n, const double* coef, hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(gs(n)), dim3(256), 0, st, y, x, n, coef);
  HDG_CHECK(hipGetLastError());
}

void blas_d2f(const double* x, float* y, long n, hipStream_t st, int nrhs) {
  if (n <= 0) return;
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(gs(n), nrhs), dim3(256), 0, st, x, y, n);
  HDG_CHECK(hipGetLastError());
}

void blas_f2d(const float* x, double* y, long n, hipStream_t st, int nrhs) {
  if (n <= 0) return;
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(gs(n), nrhs), dim3(256), 0, st, x, y, n);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void blas_copy_t(T* y, const T* x, long n, hipStream_t st, int nrhs) {
  if (n <= 0) return;
  hipLaunchKernelGGL((copy_t_kernel<T>), dim3(gs(n), nrhs), dim3(256), 0, st, y, x, n);
  HDG_CHECK(hipGetLastError());
}
template void blas_copy_t<double>(double*, const double*, long, hipStream_t, int);
template void blas_copy_t<float>(float*, const float*, long, hipStream_t, int);

void blas_copy(double* y, const double* x, long n, hipStream_t st, int nrhs) {
  blas_copy_t<double>(y, x, n, st, nrhs);
}

template <typename T>
void blas_fill(T* y, T v, long n, hipStream_t st, int nrhs) {
  if (n <= 0) return;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(gs(n), nrhs), dim3(256), 0, st, y, v, n);
  HDG_CHECK(hipGetLastError());
}
template void blas_fill<double>(double*, double, long, hipStream_t, int);
template void blas_fill<float>(float*, float, long, hipStream_t, int);
template void blas_fill<unsigned>(unsigned*, unsigned, long, hipStream_t, int);
template void blas_fill<int>(int*, int, long, hipStream_t, int);

void blas_gmres_rot(double* H, double* cs, double* sn, double* s, int j, int ld, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(gmres_rot_kernel, dim3(1), dim3(64), 0, st, H, cs, sn, s, j, ld, sc);
  HDG_CHECK(hipGetLastError());
}

void blas_gmres_backsolve(const double* H, const double* s, int j, int ld, double* y, hipStream_t st) {
  hipLaunchKernelGGL(gmres_backsolve_kernel, dim3(1), dim3(64), 0, st, H, s, j, ld, y);
  HDG_CHECK(hipGetLastError());
}

void blas_gmres_combine(double* x, const double* Z, long ldz, int j, const double* y, long n, hipStream_t st) {
  hipLaunchKernelGGL(gmres_combine_kernel, dim3(gs(n)), dim3(256), 0, st, x, Z, ldz, j, y, n);
  HDG_CHECK(hipGetLastError());
}

}  // namespace hdg
