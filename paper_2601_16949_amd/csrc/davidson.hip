// Kernels of the block-Davidson solver for the lowest eigenpairs of A (the TI-TDA eigenproblem,
// eq. casida_tda) and of the eigenstate populations (eq. populations).  All vectors are real FP64
// of length n = o*v, stored one after another ([count][n]).  The products A v come from the
// sigma kernels of the propagation (Coulomb and exchange partial slabs of FP32 or split-BF16
// stage copies) plus the diagonal D = e_a - e_i; everything else here is FP64.  Reductions are
// per-block partial sums added in a fixed order, so every result is reproducible.
#include <algorithm>

#include "common.h"

namespace rttda {
namespace {

constexpr int DV_THREADS = 256;
constexpr int DV_COMBINE_MAX = 16;  // vectors formed per combine launch (register accumulators)

__device__ __forceinline__ double dv_block_sum(double x, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < DV_THREADS / 64; ++w) t += sh[w];
  return t;
}

// W[j][e] = D[e] V[j][e] + sum_k P[k][j][e]: the nslab partial slabs of nb slices (fixed order)
__global__ __launch_bounds__(DV_THREADS) void k_dv_apply(long long n, int nb, int nslab, const double *__restrict__ D,
                                                         const float *__restrict__ P, const double *__restrict__ V,
                                                         double *__restrict__ W) {
  const long long total = (long long)nb * n;
  for (long long idx = blockIdx.x * (long long)DV_THREADS + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * DV_THREADS) {
    const long long e = idx % n;
    double s = D[e] * V[idx];
    for (int k = 0; k < nslab; ++k) s += (double)P[(size_t)k * total + idx];
    W[idx] = s;
  }
}

// out[i * nt + j] = <V_i, T_j> for i < m, j < nt: one workgroup per pair
__global__ __launch_bounds__(DV_THREADS) void k_dv_dots(long long n, int nt, const double *__restrict__ V,
                                                        const double *__restrict__ T, double *__restrict__ out) {
  __shared__ double sh[DV_THREADS / 64];
  const int i = blockIdx.x / nt, j = blockIdx.x % nt;
  const double *a = V + (size_t)i * n, *b = T + (size_t)j * n;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < n; e += DV_THREADS) acc += a[e] * b[e];
  const double t = dv_block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// out[j][e] = sum_i C[i][j] V[i][e] (mode 0) or out[j][e] -= that sum (mode 1), j < nc <= 16;
// C is [m][ldc] row-major
__global__ __launch_bounds__(DV_THREADS) void k_dv_combine(long long n, int m, const double *__restrict__ V, int nc,
                                                           const double *__restrict__ C, int ldc, int mode,
                                                           double *__restrict__ out) {
  extern __shared__ double cs[];  // [m][nc]
  for (int t = threadIdx.x; t < m * nc; t += DV_THREADS) cs[t] = C[(t / nc) * ldc + t % nc];
  __syncthreads();
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS) {
    double acc[DV_COMBINE_MAX];
#pragma unroll
    for (int j = 0; j < DV_COMBINE_MAX; ++j) acc[j] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double x = V[(size_t)i * n + e];
#pragma unroll
      for (int j = 0; j < DV_COMBINE_MAX; ++j)
        if (j < nc) acc[j] += cs[i * nc + j] * x;
    }
#pragma unroll
    for (int j = 0; j < DV_COMBINE_MAX; ++j)
      if (j < nc) {
        double *o = out + (size_t)j * n + e;
        *o = mode ? *o - acc[j] : acc[j];
      }
  }
}

// R[j] = AX[j] - theta[j] X[j]; part[j][block] = block sum of R[j]^2 (grid.y = j)
__global__ __launch_bounds__(DV_THREADS) void k_dv_resid(long long n, const double *__restrict__ X,
                                                         const double *__restrict__ AX,
                                                         const double *__restrict__ theta, double *__restrict__ R,
                                                         double *__restrict__ part) {
  __shared__ double sh[DV_THREADS / 64];
  const int j = blockIdx.y;
  const double th = theta[j];
  const size_t off = (size_t)j * n;
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS) {
    const double r = AX[off + e] - th * X[off + e];
    R[off + e] = r;
    acc += r * r;
  }
  const double t = dv_block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = t;
}

// Davidson correction with the diagonal preconditioner: T[j] = R[j] / (theta[j] - diag(A)), the
// denominator kept at least 1e-3 in magnitude (grid.y = j)
// (R and T may be the same array: each element is read, then written, by one thread)
__global__ __launch_bounds__(DV_THREADS) void k_dv_precond(long long n, const double *R,
                                                           const double *__restrict__ theta,
                                                           const double *__restrict__ D, double *T) {
  const int j = blockIdx.y;
  const double th = theta[j];
  const size_t off = (size_t)j * n;
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS) {
    double den = th - D[e];
    if (fabs(den) < 1e-3) den = den < 0.0 ? -1e-3 : 1e-3;
    T[off + e] = R[off + e] / den;
  }
}

// part[block] = block sum of T^2
__global__ __launch_bounds__(DV_THREADS) void k_dv_norm2(long long n, const double *__restrict__ T,
                                                         double *__restrict__ part) {
  __shared__ double sh[DV_THREADS / 64];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS)
    acc += T[e] * T[e];
  const double t = dv_block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out = s T
__global__ __launch_bounds__(DV_THREADS) void k_dv_scale(long long n, double s, const double *__restrict__ T,
                                                         double *__restrict__ out) {
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS)
    out[e] = s * T[e];
}

// Diagonal of A (the Davidson preconditioner): diag[i][a] = D[i][a] + 2 sum_Q B_ov^Q[i][a]^2
// - cx sum_Q B_oo^Q[i][i] B_vv^Q[a][a], FP64 sums over Q in order
template <typename T>
__global__ __launch_bounds__(DV_THREADS) void k_dv_diag(int o, int v, int nq, const T *__restrict__ Bov,
                                                        const T *__restrict__ Boo, const T *__restrict__ Bvv, double cx,
                                                        const double *__restrict__ D, double *__restrict__ diag) {
  const long long n = (long long)o * v;
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS) {
    const int i = (int)(e / v), a = (int)(e - (long long)i * v);
    double j = 0.0, x = 0.0;
    for (int q = 0; q < nq; ++q) {
      const double b = (double)(float)Bov[(size_t)q * n + e];
      j += b * b;
      x += (double)(float)Boo[((size_t)q * o + i) * o + i] * (double)(float)Bvv[((size_t)q * v + a) * v + a];
    }
    diag[e] = D[e] + 2.0 * j - cx * x;
  }
}

// unit vector e_idx into V (n entries)
__global__ __launch_bounds__(DV_THREADS) void k_dv_unit(long long n, long long idx, double *__restrict__ V) {
  for (long long e = blockIdx.x * (long long)DV_THREADS + threadIdx.x; e < n; e += (long long)gridDim.x * DV_THREADS)
    V[e] = e == idx ? 1.0 : 0.0;
}

inline int dv_grid(long long n) {
  return (int)std::min<long long>(DV_BLOCKS_MAX, std::max<long long>(1, (n + DV_THREADS - 1) / DV_THREADS));
}

}  // namespace

int dv_blocks(long long n) { return dv_grid(n); }

hipError_t launch_dv_apply(hipStream_t s, long long n, int nb, int nslab, const double *D, const float *P,
                           const double *V, double *W) {
  hipLaunchKernelGGL(k_dv_apply, dim3(dv_grid((long long)nb * n)), dim3(DV_THREADS), 0, s, n, nb, nslab, D, P, V, W);
  return hipGetLastError();
}
hipError_t launch_dv_dots(hipStream_t s, long long n, int m, const double *V, int nt, const double *T, double *out) {
  if (m <= 0 || nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dv_dots, dim3(m * nt), dim3(DV_THREADS), 0, s, n, nt, V, T, out);
  return hipGetLastError();
}
hipError_t launch_dv_combine(hipStream_t s, long long n, int m, const double *V, int nc, const double *C, int ldc,
                             int mode, double *out) {
  if (m <= 0 || nc <= 0) return hipSuccess;
  if (nc > DV_COMBINE_MAX || m > DV_SPACE_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dv_combine, dim3(dv_grid(n)), dim3(DV_THREADS), (size_t)m * nc * sizeof(double), s, n, m, V,
                     nc, C, ldc, mode, out);
  return hipGetLastError();
}
hipError_t launch_dv_resid(hipStream_t s, long long n, int nc, const double *X, const double *AX, const double *theta,
                           double *R, double *part) {
  hipLaunchKernelGGL(k_dv_resid, dim3(dv_grid(n), nc), dim3(DV_THREADS), 0, s, n, X, AX, theta, R, part);
  return hipGetLastError();
}
hipError_t launch_dv_precond(hipStream_t s, long long n, int nc, const double *R, const double *theta,
                             const double *D, double *T) {
  hipLaunchKernelGGL(k_dv_precond, dim3(dv_grid(n), nc), dim3(DV_THREADS), 0, s, n, R, theta, D, T);
  return hipGetLastError();
}
hipError_t launch_dv_norm2(hipStream_t s, long long n, const double *T, double *part) {
  hipLaunchKernelGGL(k_dv_norm2, dim3(dv_grid(n)), dim3(DV_THREADS), 0, s, n, T, part);
  return hipGetLastError();
}
hipError_t launch_dv_scale(hipStream_t s, long long n, double scale, const double *T, double *out) {
  hipLaunchKernelGGL(k_dv_scale, dim3(dv_grid(n)), dim3(DV_THREADS), 0, s, n, scale, T, out);
  return hipGetLastError();
}
hipError_t launch_dv_diag(hipStream_t s, int b_dtype, int o, int v, int nq, const void *Bov, const void *Boo,
                          const void *Bvv, double cx, const double *D, double *diag) {
  const long long n = (long long)o * v;
  if (b_dtype == RTTDA_BF16)
    hipLaunchKernelGGL((k_dv_diag<__hip_bfloat16>), dim3(dv_grid(n)), dim3(DV_THREADS), 0, s, o, v, nq,
                       static_cast<const __hip_bfloat16 *>(Bov), static_cast<const __hip_bfloat16 *>(Boo),
                       static_cast<const __hip_bfloat16 *>(Bvv), cx, D, diag);
  else
    hipLaunchKernelGGL((k_dv_diag<float>), dim3(dv_grid(n)), dim3(DV_THREADS), 0, s, o, v, nq,
                       static_cast<const float *>(Bov), static_cast<const float *>(Boo),
                       static_cast<const float *>(Bvv), cx, D, diag);
  return hipGetLastError();
}
hipError_t launch_dv_unit(hipStream_t s, long long n, long long idx, double *V) {
  hipLaunchKernelGGL(k_dv_unit, dim3(dv_grid(n)), dim3(DV_THREADS), 0, s, n, idx, V);
  return hipGetLastError();
}

}  // namespace rttda
