// Vector kernels of the outer iterations (fixed point, CG, GMRES; Sec. 3.6
// and Sec. 4): dot products with a deterministic two-level reduction
// (wavefront shuffles, one partial per block, the last block to finish sums
// the partials in block order), fused CG updates whose scalars never leave
// the device, precision conversions, and the small GMRES Hessenberg work.
#include "hdg_internal.hpp"
#include "blas.hpp"

namespace hdg {

namespace {

constexpr int RB = 256;     // reduction block size
constexpr int RG = 512;     // reduction grid (fixed -> reproducible sums)

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < RB / 64; ++w) s += sh[w];
  return s;
}

// Sum partials in block order in the last block; apply the finaliser.
__device__ inline bool last_block(unsigned* counter) {
  __shared__ bool last;
  __threadfence();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  return last;
}

__device__ inline double sum_partials(const double* partials, int np, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += RB)
    v += __hip_atomic_load(partials + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // fixed order: each thread sums a fixed strided subset, then the block tree
  return block_sum(v, sh);
}

// out_slots: dot(x, y) finalised according to mode
__global__ void __launch_bounds__(RB) dot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                 long n, double* __restrict__ partials, unsigned* counter,
                                                 double* sc, int mode, double* out) {
  __shared__ double sh[RB / 64];
  double v = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) v += x[i] * y[i];
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (!last_block(counter)) return;
  __syncthreads();
  double tot = sum_partials(partials, gridDim.x, sh);
  if (threadIdx.x == 0) {
    *counter = 0u;
    switch (mode) {
      case FIN_STORE: *out = tot; break;
      case FIN_ALPHA:  // alpha = rz / pAp
        sc[SC_PAP] = tot;
        sc[SC_ALPHA] = sc[SC_RZ] / tot;
        break;
      case FIN_BETA:   // beta = rz_new / rz ; rz = rz_new
        sc[SC_BETA] = tot / sc[SC_RZ];
        sc[SC_RZ] = tot;
        break;
      case FIN_RZ0: sc[SC_RZ] = tot; break;
      case FIN_NORM_INV:  // out <- ||x||, SC_TMP <- 1/||x||
        *out = sqrt(tot);
        sc[SC_TMP] = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
        break;
    }
  }
}

// flexible CG direction scalar: beta = (rz_new - r.z_old) / rz ; rz = rz_new
__global__ void __launch_bounds__(RB) dot2_kernel(const double* __restrict__ r, const double* __restrict__ z,
                                                  const double* __restrict__ zold, long n,
                                                  double* __restrict__ partials, unsigned* counter, double* sc) {
  __shared__ double sh[RB / 64];
  double a = 0.0, b = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
    a += r[i] * z[i];
    b += r[i] * zold[i];
  }
  double sa = block_sum(a, sh);
  __syncthreads();
  double sb = block_sum(b, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sa;
    partials[2 * blockIdx.x + 1] = sb;
  }
  if (!last_block(counter)) return;
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  if (threadIdx.x == 0)
    for (unsigned i = 0; i < gridDim.x; ++i) {
      ta += __hip_atomic_load(partials + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tb += __hip_atomic_load(partials + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  if (threadIdx.x == 0) {
    *counter = 0u;
    sc[SC_BETA] = (ta - tb) / sc[SC_RZ];
    sc[SC_RZ] = ta;
  }
}

// lam += alpha p ; r -= alpha Ap ; rnorm2 = r.r
__global__ void __launch_bounds__(RB) cg_update_kernel(double* __restrict__ lam, double* __restrict__ r,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ Ap, long n,
                                                       double* __restrict__ partials, unsigned* counter,
                                                       double* sc) {
  __shared__ double sh[RB / 64];
  const double alpha = sc[SC_ALPHA];
  double v = 0.0;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) {
    lam[i] += alpha * p[i];
    const double ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    v += ri * ri;
  }
  double s = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (!last_block(counter)) return;
  __syncthreads();
  double tot = sum_partials(partials, gridDim.x, sh);
  if (threadIdx.x == 0) {
    *counter = 0u;
    sc[SC_RNORM2] = tot;
  }
}

// p = z + beta p
__global__ void cg_direction_kernel(double* __restrict__ p, const double* __restrict__ z, long n,
                                    const double* sc) {
  const double beta = sc[SC_BETA];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) p[i] = z[i] + beta * p[i];
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
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = (B)x[i];
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ y, T v, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = v;
}

__global__ void copy_kernel(double* __restrict__ y, const double* __restrict__ x, long n) {
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

__global__ void set_scalar_kernel(double* sc, int slot, const double* src, int mode) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (mode == 0) sc[slot] = *src;
    else sc[slot] = -(*src);
  }
}

__global__ void finite_kernel(const double* __restrict__ x, long n, int* bad) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L)
    if (!isfinite(x[i])) atomicOr(bad, 1);
}

inline unsigned gs(long n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

inline unsigned rg(long n) {
  long b = (n + RB - 1) / RB;
  if (b > RG) b = RG;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void blas_dot(const double* x, const double* y, long n, Scratch& s, int mode, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(rg(n)), dim3(RB), 0, st, x, y, n, s.partials, s.counter, s.sc, mode, out);
  HDG_CHECK(hipGetLastError());
}

void blas_dot2_flex(const double* r, const double* z, const double* zold, long n, Scratch& s, hipStream_t st) {
  hipLaunchKernelGGL(dot2_kernel, dim3(rg(n)), dim3(RB), 0, st, r, z, zold, n, s.partials, s.counter, s.sc);
  HDG_CHECK(hipGetLastError());
}

void blas_cg_update(double* lam, double* r, const double* p, const double* Ap, long n, Scratch& s,
                    hipStream_t st) {
  hipLaunchKernelGGL(cg_update_kernel, dim3(rg(n)), dim3(RB), 0, st, lam, r, p, Ap, n, s.partials, s.counter, s.sc);
  HDG_CHECK(hipGetLastError());
}

void blas_cg_direction(double* p, const double* z, long n, Scratch& s, hipStream_t st) {
  hipLaunchKernelGGL(cg_direction_kernel, dim3(gs(n)), dim3(256), 0, st, p, z, n, s.sc);
  HDG_CHECK(hipGetLastError());
}

void blas_axpy(double* y, const double* x, long n, const double* coef, double sign, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3(gs(n)), dim3(256), 0, st, y, x, n, coef, sign);
  HDG_CHECK(hipGetLastError());
}

void blas_scale(double* y, const double* x, long n, const double* coef, hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(gs(n)), dim3(256), 0, st, y, x, n, coef);
  HDG_CHECK(hipGetLastError());
}

void blas_d2f(const double* x, float* y, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(gs(n)), dim3(256), 0, st, x, y, n);
  HDG_CHECK(hipGetLastError());
}

void blas_f2d(const float* x, double* y, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(gs(n)), dim3(256), 0, st, x, y, n);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
__global__ void copy_t_kernel(T* __restrict__ y, const T* __restrict__ x, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256L) y[i] = x[i];
}

template <typename T>
void blas_copy_t(T* y, const T* x, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((copy_t_kernel<T>), dim3(gs(n)), dim3(256), 0, st, y, x, n);
  HDG_CHECK(hipGetLastError());
}
template void blas_copy_t<double>(double*, const double*, long, hipStream_t);
template void blas_copy_t<float>(float*, const float*, long, hipStream_t);

void blas_copy(double* y, const double* x, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(gs(n)), dim3(256), 0, st, y, x, n);
  HDG_CHECK(hipGetLastError());
}

template <typename T>
void blas_fill(T* y, T v, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(gs(n)), dim3(256), 0, st, y, v, n);
  HDG_CHECK(hipGetLastError());
}
template void blas_fill<double>(double*, double, long, hipStream_t);
template void blas_fill<float>(float*, float, long, hipStream_t);
template void blas_fill<unsigned>(unsigned*, unsigned, long, hipStream_t);
template void blas_fill<int>(int*, int, long, hipStream_t);

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

void blas_set_scalar(double* sc, int slot, const double* src, int negate, hipStream_t st) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, st, sc, slot, src, negate);
  HDG_CHECK(hipGetLastError());
}

void blas_finite(const double* x, long n, int* bad, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(finite_kernel, dim3(gs(n)), dim3(256), 0, st, x, n, bad);
  HDG_CHECK(hipGetLastError());
}

}  // namespace hdg
