// Bandwidth- and latency-bound kernels of the RT-TDA step on gfx950:
// dipole blocks, Coulomb GEMV pair, FP64 field/trace, stage scalars, RK4 epilogue, kick.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace rttda {

namespace {

__device__ __forceinline__ float load_b(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float load_b(const __hip_bfloat16 *p, size_t i) { return __bfloat162float(p[i]); }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ------------------------------------------------------------------------------------------------
// mu_d = sum_k d_k mu_k, split into the oo, ov and vv blocks, one copy per right-hand side.
// ------------------------------------------------------------------------------------------------
__global__ void k_mu_blocks(const double *__restrict__ mu, const DevPulse *__restrict__ pulses, int o, int v,
                            int R, double *__restrict__ moo, double *__restrict__ mov, double *__restrict__ mvv) {
  const long long n = o + v, nn = n * n, total = (long long)R * nn;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / nn);
    const long long pq = e - r * nn;
    const int p = (int)(pq / n), q = (int)(pq - p * n);
    const double *d = pulses[r].dir;
    const double m = d[0] * mu[pq] + d[1] * mu[nn + pq] + d[2] * mu[2 * nn + pq];
    if (p < o && q < o)
      moo[(size_t)r * o * o + (size_t)p * o + q] = m;
    else if (p < o)
      mov[(size_t)r * o * v + (size_t)p * v + (q - o)] = m;
    else if (q >= o)
      mvv[(size_t)r * v * v + (size_t)(p - o) * v + (q - o)] = m;
  }
}

// D_ia = e_a - e_i (diagonal of A, eq. A_matrix_element2).
__global__ void k_gaps(const double *__restrict__ e_occ, const double *__restrict__ e_virt, int o, int v,
                       double *__restrict__ D) {
  const long long total = (long long)o * v;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e / v), a = (int)(e - (long long)i * v);
    D[e] = e_virt[a] - e_occ[i];
  }
}

__global__ void k_to_f32(const double *__restrict__ c, long long n, float *__restrict__ x) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    x[e] = (float)c[e];
}

__device__ __forceinline__ void split_bf16(double x, __hip_bfloat16 &hi, __hip_bfloat16 &lo) {
  hi = __float2bfloat16((float)x);
  lo = __float2bfloat16((float)(x - (double)__bfloat162float(hi)));
}

__global__ void k_to_bf16x2(const double *__restrict__ c, long long n, float *__restrict__ x,
                            __hip_bfloat16 *__restrict__ hi, __hip_bfloat16 *__restrict__ lo) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    x[e] = (float)c[e];
    split_bf16(c[e], hi[e], lo[e]);
  }
}

// ------------------------------------------------------------------------------------------------
// Coulomb, first product: d[Q][s] = sum_ia B_ov[Q][ia] X[s][ia]   (B streamed once from HBM)
// Block = QT rows of B x ST slices x one ia chunk; the chunk partials dpart[chunk][Q][s] are summed
// in a fixed order by the second product.  Vector path: 4 consecutive ia per lane and load (needs
// ov % 4 == 0 so that every B row starts 16/8-byte aligned); scalar path otherwise.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ float4 load_b4(const float *p, size_t i) {
  return *reinterpret_cast<const float4 *>(p + i);
}
__device__ __forceinline__ float4 load_b4(const __hip_bfloat16 *p, size_t i) {
  const uint2 u = *reinterpret_cast<const uint2 *>(p + i);  // element 2k in the low half of word k
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}

// Sum 64 per-lane values over the wave with 63 exchanges: at each halving step a lane keeps the
// half of its values selected by its lane bit and adds the partner's copy of that half.  On exit
// lane l holds the wave total of value l.
template <int K>
__device__ __forceinline__ void transpose_sum_step(float (&v)[64], int lane) {
  const bool up = (lane & K) != 0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float send = up ? v[j] : v[j + K];
    const float keep = up ? v[j + K] : v[j];
    v[j] = keep + __shfl_xor(send, K, 64);
  }
  if constexpr (K > 1) transpose_sum_step<K / 2>(v, lane);
}

__device__ __forceinline__ float wave_transpose_sum64(float (&v)[64], int lane) {
  transpose_sum_step<32>(v, lane);
  return v[0];
}

// One 16-byte load of a B row: EPL values widened to FP32 (FP32: four; BF16: four from an 8-byte load,
// or eight)
template <int EPL>
__device__ __forceinline__ void load_row(const float *p, size_t i, float (&x)[EPL]) {
  static_assert(EPL == 4, "FP32 rows: four values per 16-byte load");
  const float4 t = *reinterpret_cast<const float4 *>(p + i);
  x[0] = t.x, x[1] = t.y, x[2] = t.z, x[3] = t.w;
}
template <int EPL>
__device__ __forceinline__ void load_row(const __hip_bfloat16 *p, size_t i, float (&x)[EPL]) {
  static_assert(EPL == 4 || EPL == 8, "BF16 rows: four or eight values per load");
  if constexpr (EPL == 4) {
    const float4 t = load_b4(p, i);
    x[0] = t.x, x[1] = t.y, x[2] = t.z, x[3] = t.w;
  } else {
    const uint4 u = *reinterpret_cast<const uint4 *>(p + i);  // element 2k in the low half of word k
    const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[2 * k] = __uint_as_float(w[k] << 16);
      x[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
    }
  }
}

// VEC: EPL consecutive ia per lane and load (4: 16 bytes of FP32 or 8 of BF16; 8: 16 bytes of BF16,
// needs ov % 8 == 0); scalar path otherwise
template <typename TB, int QT, int ST, bool VEC, int EPL = 4>
__global__ __launch_bounds__(256) void k_gemv1(const TB *__restrict__ B, const float *__restrict__ X, int nq, int ov,
                                               int ns, int echunk, float *__restrict__ dpart) {
  static_assert(QT * ST <= 64, "one reduced value per lane");
  const int q0 = blockIdx.x * QT, s0 = blockIdx.y * ST;
  const int e0 = blockIdx.z * echunk, e1 = min(ov, e0 + echunk);
  const int nqv = min(QT, nq - q0), nsv = min(ST, ns - s0);
  float acc[QT][ST];
#pragma unroll
  for (int a = 0; a < QT; ++a)
#pragma unroll
    for (int b = 0; b < ST; ++b) acc[a][b] = 0.f;
  if constexpr (VEC) {
    for (int e = e0 + EPL * (int)threadIdx.x; e < e1; e += 256 * EPL) {
      float xs[ST][EPL];
#pragma unroll
      for (int b = 0; b < ST; ++b)
#pragma unroll
        for (int g = 0; g < EPL / 4; ++g) {
          const float4 t = b < nsv ? *reinterpret_cast<const float4 *>(X + (size_t)(s0 + b) * ov + e + 4 * g)
                                   : make_float4(0, 0, 0, 0);
          xs[b][4 * g] = t.x, xs[b][4 * g + 1] = t.y, xs[b][4 * g + 2] = t.z, xs[b][4 * g + 3] = t.w;
        }
      // all QT rows' loads issued before any of their products (rows past nq read row q0)
      float bq[QT][EPL];
#pragma unroll
      for (int a = 0; a < QT; ++a) load_row<EPL>(B, (size_t)(q0 + (a < nqv ? a : 0)) * ov + e, bq[a]);
#pragma unroll
      for (int a = 0; a < QT; ++a) {
        if (a < nqv) {
#pragma unroll
          for (int b = 0; b < ST; ++b) {
            float t = acc[a][b];
#pragma unroll
            for (int k = 0; k < EPL; ++k) t = fmaf(bq[a][k], xs[b][k], t);
            acc[a][b] = t;
          }
        }
      }
    }
  } else {
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
      float xs[ST];
#pragma unroll
      for (int b = 0; b < ST; ++b) xs[b] = b < nsv ? X[(size_t)(s0 + b) * ov + e] : 0.f;
#pragma unroll
      for (int a = 0; a < QT; ++a) {
        if (a < nqv) {
          const float bq = load_b(B, (size_t)(q0 + a) * ov + e);
#pragma unroll
          for (int b = 0; b < ST; ++b) acc[a][b] = fmaf(bq, xs[b], acc[a][b]);
        }
      }
    }
  }
  float vals[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) vals[k] = k < QT * ST ? acc[k / ST][k % ST] : 0.f;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ float red[4][64];
  red[wave][lane] = wave_transpose_sum64(vals, lane);
  __syncthreads();
  if (threadIdx.x < QT * ST) {
    const int k = threadIdx.x, a = k / ST, b = k % ST;
    if (a < nqv && b < nsv)
      dpart[((size_t)blockIdx.z * nq + q0 + a) * ns + s0 + b] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
  }
}

// Sum of the ia-chunk partials into chunk slot 0: dpart[0][q][s] = sum_k dpart[k][q][s] (fixed order).
__global__ void k_dsum(float *__restrict__ dpart, int n, int nes) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    float d = dpart[e];
    for (int k = 1; k < nes; ++k) d += dpart[(size_t)k * n + e];
    dpart[e] = d;
  }
}

// ------------------------------------------------------------------------------------------------
// Coulomb, second product: P[split][s][ia] = 2 sum_{Q in split} B_ov[Q][ia] d[Q][s]
// One thread per ia (coalesced along ia), d staged in LDS.
// ------------------------------------------------------------------------------------------------
template <typename TB, int ST>
__global__ __launch_bounds__(256) void k_gemv2(const TB *__restrict__ B, const float *__restrict__ dvec, int nq,
                                               int ov, int ns, int nsplit, float *__restrict__ P) {
  constexpr int QCH = 64;
  __shared__ float dsh[QCH][ST];
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int s0 = blockIdx.y * ST, sp = blockIdx.z;
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  float acc[ST];
#pragma unroll
  for (int b = 0; b < ST; ++b) acc[b] = 0.f;
  for (int qc = qa; qc < qb; qc += QCH) {
    const int nqc = min(QCH, qb - qc);
    __syncthreads();
    for (int k = threadIdx.x; k < QCH * ST; k += 256) {
      const int qq = k / ST, b = k % ST;
      dsh[qq][b] = (qq < nqc && s0 + b < ns) ? dvec[(size_t)(qc + qq) * ns + s0 + b] : 0.f;
    }
    __syncthreads();
    if (e < ov) {
      for (int qq = 0; qq < nqc; ++qq) {
        const float bq = load_b(B, (size_t)(qc + qq) * ov + e);
#pragma unroll
        for (int b = 0; b < ST; ++b) acc[b] += bq * dsh[qq][b];
      }
    }
  }
  if (e < ov) {
#pragma unroll
    for (int b = 0; b < ST; ++b)
      if (s0 + b < ns) P[((size_t)sp * ns + s0 + b) * ov + e] = 2.f * acc[b];
  }
}

// Vector form (ov % EPL == 0): a block covers 64 EPL consecutive ia, EPL per lane (16 bytes of B:
// four FP32 or eight BF16 values), and its four waves take every fourth Q of the split's range
// (wave w: Q = qa + w, qa + w + 4, ...), with eight B rows in flight per lane; the wave partials
// meet in LDS and are summed in wave order.  Each slice's sum depends only on its own d values, so
// a batch and a single RHS give the same bits.
template <typename TB, int ST, int EPL>
__global__ __launch_bounds__(256) void k_gemv2v(const TB *__restrict__ B, const float *__restrict__ dvec, int nq,
                                                int ov, int ns, int nsplit, float *__restrict__ P) {
  constexpr int QCH = 64, U = 8;
  __shared__ float dsh[QCH][ST];
  __shared__ float4 red[4][ST][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * (64 * EPL) + EPL * lane;
  const int s0 = blockIdx.y * ST, sp = blockIdx.z;
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const bool live = e < ov;  // ov % EPL == 0: the lane's EPL ia are all inside or all outside
  float acc[ST][EPL];
#pragma unroll
  for (int b = 0; b < ST; ++b)
#pragma unroll
    for (int k = 0; k < EPL; ++k) acc[b][k] = 0.f;
  for (int qc = qa; qc < qb; qc += QCH) {
    const int nqc = min(QCH, qb - qc);
    __syncthreads();
    for (int k = threadIdx.x; k < QCH * ST; k += 256) {
      const int qq = k / ST, b = k % ST;
      dsh[qq][b] = (qq < nqc && s0 + b < ns) ? dvec[(size_t)(qc + qq) * ns + s0 + b] : 0.f;
    }
    __syncthreads();
    if (live) {
      int qq = wave;
      for (; qq + 4 * (U - 1) < nqc; qq += 4 * U) {
        float bq[U][EPL];
#pragma unroll
        for (int u = 0; u < U; ++u) load_row<EPL>(B, (size_t)(qc + qq + 4 * u) * ov + e, bq[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int b = 0; b < ST; ++b) {
            const float d = dsh[qq + 4 * u][b];
#pragma unroll
            for (int k = 0; k < EPL; ++k) acc[b][k] = fmaf(bq[u][k], d, acc[b][k]);
          }
      }
      for (; qq < nqc; qq += 4) {
        float bq[EPL];
        load_row<EPL>(B, (size_t)(qc + qq) * ov + e, bq);
#pragma unroll
        for (int b = 0; b < ST; ++b) {
          const float d = dsh[qq][b];
#pragma unroll
          for (int k = 0; k < EPL; ++k) acc[b][k] = fmaf(bq[k], d, acc[b][k]);
        }
      }
    }
  }
  // wave partials through LDS, four values per lane at a time; wave w stores slices w, w + 4, ...
#pragma unroll
  for (int g = 0; g < EPL / 4; ++g) {
    __syncthreads();
#pragma unroll
    for (int b = 0; b < ST; ++b)
      red[wave][b][lane] = make_float4(acc[b][4 * g], acc[b][4 * g + 1], acc[b][4 * g + 2], acc[b][4 * g + 3]);
    __syncthreads();
    for (int b = wave; b < ST; b += 4) {
      if (!live || s0 + b >= ns) continue;
      const float4 r0 = red[0][b][lane], r1 = red[1][b][lane], r2 = red[2][b][lane], r3 = red[3][b][lane];
      float4 t;
      t.x = 2.f * ((r0.x + r1.x) + (r2.x + r3.x));
      t.y = 2.f * ((r0.y + r1.y) + (r2.y + r3.y));
      t.z = 2.f * ((r0.z + r1.z) + (r2.z + r3.z));
      t.w = 2.f * ((r0.w + r1.w) + (r2.w + r3.w));
      *reinterpret_cast<float4 *>(P + ((size_t)sp * ns + s0 + b) * ov + e + 4 * g) = t;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Field product (FP64), eqs. sc2-sc5 in factorised form, on the FP64 matrix cores:
//   F_p = X_p mu_vv - mu_oo X_p + sqrt2 mu_ov c0_p      (p = 0, 1: the real and imaginary planes)
// plus per-block partial sums g_p = sqrt2 <mu_ov, X_p>, <X, F> and |X|^2.
// One block per (RHS, 16 x 16 tile of (i, a)); 8 waves: waves 0-3 form plane 0, waves 4-7 plane 1,
// each over a quarter of the contraction index (b for X mu_vv, j for mu_oo X) with
// v_mfma_f64_16x16x4 (operands read straight from memory, four K steps' loads issued before their
// MFMAs); the quarters are added in a fixed order through LDS.
// f64 16x16x4 operand layout: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the result
// element t of lane l is D[4 t + l / 16][l % 16].
// ------------------------------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(512) void k_field(const double *__restrict__ X, const double *__restrict__ X0,
                                               const double *__restrict__ moo, const double *__restrict__ mov,
                                               const double *__restrict__ mvv, int o, int v,
                                               double *__restrict__ F, double *__restrict__ part) {
  __shared__ double red[8][4][64];
  __shared__ double sums[2][4];
  const int at = blockIdx.x, it = blockIdx.y, r = blockIdx.z;
  const int nbf = gridDim.x * gridDim.y, blk = it * gridDim.x + at;
  const int i0 = it * FT_I, a0 = at * FT_A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p = wave >> 2, q = wave & 3;
  const int m = lane & 15, g = lane >> 4;
  const size_t ov = (size_t)o * v;
  const double *Xp = X + ((size_t)r * 2 + p) * ov;
  const double *moo_r = moo + (size_t)r * o * o;
  const double *mov_r = mov + (size_t)r * ov;
  const double *mvv_r = mvv + (size_t)r * v * v;
  const int i = i0 + m, a = a0 + m;  // this lane's operand row (A) and column (B)
  d4v acc = {0.0, 0.0, 0.0, 0.0};

  // X_p mu_vv over b in this wave's quarter [bq, be)
  {
    const int kq = (((v + 3) / 4) + 3) / 4 * 4;
    const int bq = q * kq, be = min(v, bq + kq);
    for (int b0 = bq; b0 < be; b0 += 16) {
      double xa[4], mb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + 4 * u + g;
        xa[u] = (i < o && b < be) ? Xp[(size_t)i * v + b] : 0.0;
        mb[u] = (b < be && a < v) ? mvv_r[(size_t)b * v + a] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], mb[u], acc, 0, 0, 0);
    }
  }
  // - mu_oo X_p over j in this wave's quarter [jq, je)
  {
    const int kq = (((o + 3) / 4) + 3) / 4 * 4;
    const int jq = q * kq, je = min(o, jq + kq);
    for (int j0 = jq; j0 < je; j0 += 16) {
      double ma[4], xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = j0 + 4 * u + g;
        ma[u] = (i < o && j < je) ? -moo_r[(size_t)i * o + j] : 0.0;
        xb[u] = (j < je && a < v) ? Xp[(size_t)j * v + a] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[u], xb[u], acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) red[wave][t][lane] = acc[t];
  __syncthreads();
  // plane leaders (waves 0 and 4): add the quarters, + sqrt2 mu_ov c0_p, outputs, partial sums
  if (q == 0) {
    const double c0p = X0[2 * r + p];
    double pg = 0.0, ptr = 0.0, pnr = 0.0;
    double *Fp = F + ((size_t)r * 2 + p) * ov;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ii = i0 + 4 * t + g, aa = a0 + m;
      if (ii < o && aa < v) {
        const size_t ia = (size_t)ii * v + aa;
        const double mo = mov_r[ia], x = Xp[ia];
        const double f = ((red[wave][t][lane] + red[wave + 1][t][lane]) + (red[wave + 2][t][lane] + red[wave + 3][t][lane])) +
                         SQRT2 * mo * c0p;
        Fp[ia] = f;
        pg += SQRT2 * mo * x;
        ptr += x * f;
        pnr += x * x;
      }
    }
    pg = wave_sum(pg);
    ptr = wave_sum(ptr);
    pnr = wave_sum(pnr);
    if (lane == 0) {
      sums[p][0] = p == 0 ? pg : 0.0;
      sums[p][1] = p == 1 ? pg : 0.0;
      sums[p][2] = ptr;
      sums[p][3] = pnr;
    }
  }
  __syncthreads();
  if (tid < 4) part[((size_t)r * nbf + blk) * PART_STRIDE + tid] = sums[0][tid] + sums[1][tid];
}

// ------------------------------------------------------------------------------------------------
// Stage scalars (one block): pulse fields E_r(t_stage), the ground-row product g, the trace and
// norm samples with the norm guard, and the RK4 update of c0 (dc0/dt = -i(-E g) = i E g).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scalar(int R, int nbf, int stage, int mode, double dt,
                                                const DevPulse *__restrict__ pulses, DevState *__restrict__ st,
                                                const double *__restrict__ part, double *__restrict__ sc,
                                                double *__restrict__ c0, double *__restrict__ acc0,
                                                double *__restrict__ xs0, double *__restrict__ out,
                                                double *__restrict__ normref, double *__restrict__ s0) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const long long step = st->step;
  const long long k = step - st->step0;
  double *trace = st->trace;
  double *norms = st->norms;
  const double node = (stage == 0) ? 0.0 : (stage == 3 ? 1.0 : 0.5);
  // the field kernel's per-block partial sums of each RHS, 64 RHS at a time: wave w adds those of
  // RHS r0 + w, r0 + w + 4, ... (lanes over blocks, then a fixed shuffle tree)
  __shared__ double tot[64][PART_STRIDE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r0 = 0; r0 < R; r0 += 64) {
    const int nr0 = min(64, R - r0);
    for (int rr = wave; rr < nr0; rr += (int)(blockDim.x >> 6)) {
      const double *pp = part + (size_t)(r0 + rr) * nbf * PART_STRIDE;
      double s_0 = 0.0, s_1 = 0.0, s_2 = 0.0, s_3 = 0.0;
      for (int b = lane; b < nbf; b += 64) {
        s_0 += pp[(size_t)b * PART_STRIDE + 0];
        s_1 += pp[(size_t)b * PART_STRIDE + 1];
        s_2 += pp[(size_t)b * PART_STRIDE + 2];
        s_3 += pp[(size_t)b * PART_STRIDE + 3];
      }
      s_0 = wave_sum(s_0);
      s_1 = wave_sum(s_1);
      s_2 = wave_sum(s_2);
      s_3 = wave_sum(s_3);
      if (lane == 0) {
        tot[rr][0] = s_0;
        tot[rr][1] = s_1;
        tot[rr][2] = s_2;
        tot[rr][3] = s_3;
      }
    }
    __syncthreads();
    for (int r = r0 + (int)threadIdx.x; r < r0 + nr0; r += blockDim.x) {
      const double g0 = tot[r - r0][0], g1 = tot[r - r0][1], tr = tot[r - r0][2], nr = tot[r - r0][3];
      double E = 0.0;
      if (mode & SM_EFIELD)
        E = pulse_field(pulses[r], ((double)step + node) * dt);
      else if (mode & SM_KEEP_E)
        E = sc[r * SC_STRIDE + SC_E];
      sc[r * SC_STRIDE + SC_GRE] = g0;
      sc[r * SC_STRIDE + SC_GIM] = g1;
      sc[r * SC_STRIDE + SC_E] = E;
      // X0 of this stage (c0 at stage 0, else the stage value)
      const double x0r = (stage == 0) ? c0[2 * r] : xs0[2 * r];
      const double x0i = (stage == 0) ? c0[2 * r + 1] : xs0[2 * r + 1];
      if (mode & (SM_TRACE | SM_OUT)) {
        const double t = tr + (x0r * g0 + x0i * g1);
        const double n2 = nr + (x0r * x0r + x0i * x0i);
        if (mode & SM_OUT) out[r] = t;
        if (mode & SM_TRACE) {
          if (trace) trace[k * R + r] = t;
          if (norms) norms[k * R + r] = n2;
          if (k == 0 && !st->keep_ref) {
            normref[r] = n2;
          } else if (!(n2 <= 2.0 * normref[r])) {  // also catches NaN
            bad = 1;
          }
        }
      }
      if (mode & SM_SIGMA0) {
        s0[2 * r] = -E * g0;
        s0[2 * r + 1] = -E * g1;
      }
      if (mode & SM_C0) {
        // k0 = -i * (H X)_0 = -i * (-E g) = i E g
        const double kr = -E * g1, ki = E * g0;
        const double cr = c0[2 * r], ci = c0[2 * r + 1];
        if (stage == 0) {
          acc0[2 * r] = cr + dt / 6.0 * kr;
          acc0[2 * r + 1] = ci + dt / 6.0 * ki;
          xs0[2 * r] = cr + 0.5 * dt * kr;
          xs0[2 * r + 1] = ci + 0.5 * dt * ki;
        } else if (stage == 1) {
          acc0[2 * r] += dt / 3.0 * kr;
          acc0[2 * r + 1] += dt / 3.0 * ki;
          xs0[2 * r] = cr + 0.5 * dt * kr;
          xs0[2 * r + 1] = ci + 0.5 * dt * ki;
        } else if (stage == 2) {
          acc0[2 * r] += dt / 3.0 * kr;
          acc0[2 * r + 1] += dt / 3.0 * ki;
          xs0[2 * r] = cr + dt * kr;
          xs0[2 * r + 1] = ci + dt * ki;
        } else {
          c0[2 * r] = acc0[2 * r] + dt / 6.0 * kr;
          c0[2 * r + 1] = acc0[2 * r + 1] + dt / 6.0 * ki;
        }
      }
    }
    __syncthreads();
  }
  // energy sample: the epilogue's per-block partial sums of each RHS, added lane-wise then by a
  // fixed shuffle tree (one wave per RHS)
  if ((mode & SM_ENERGY) && st->energy) {
    const long long nbe = st->nbe;
    for (int r = wave; r < R; r += (int)(blockDim.x >> 6)) {
      double e = 0.0;
      for (long long b = lane; b < nbe; b += 64) e += st->epart[(size_t)r * nbe + b];
      e = wave_sum(e);
      if (lane == 0) st->energy[k * R + r] = e;
    }
  }
  if (threadIdx.x == 0) {
    if (bad && st->bad_step < 0) st->bad_step = step;
    if (mode & SM_INC) st->step = step + 1;
  }
}

// ------------------------------------------------------------------------------------------------
// Symplectic split-operator step (Propagation Algorithm subsection: X = q + i p, dq/dt = H p,
// dp/dt = -H q; second order, kick-drift-kick):
//   drift:  q <- q + dt (H p_h)                    at t_n + dt/2
//   kick:   p <- p_h - dt/2 (H q);  p_h <- p - dt/2 (H q)   at t_n + dt   (two half kicks merged)
// with H x = D x + (Coulomb + exchange partials of x) - E F_x on one real plane and ground element
// (H x)_0 = -E g_x.  c holds (q, p) at whole steps; W (the stage buffer) holds the work state
// (q, p_h).  The FP32 (+ BF16 hi/lo) copy of the next plane to multiply goes to x32 [R][o][v].
// One thread per (r, i, a); the ground element of RHS r by the thread with ia == 0.
// ------------------------------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256) void k_sso_update(int R, int o, int v, int nslab, int mode, int use_field, double dt,
                                                    const double *__restrict__ D, const float *__restrict__ P,
                                                    const double *__restrict__ F, const double *__restrict__ sc,
                                                    double *__restrict__ c, double *__restrict__ c0,
                                                    double *__restrict__ W, double *__restrict__ W0,
                                                    float *__restrict__ x32, __hip_bfloat16 *__restrict__ xhi,
                                                    __hip_bfloat16 *__restrict__ xlo) {
  const size_t ov = (size_t)o * v;
  const size_t total = (size_t)R * ov;
  const size_t slab = total;  // one plane per RHS: floats per partial slab
  const int pl = (mode == SSO_DRIFT) ? 1 : 0;  // plane of the multiplied vector
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ov, ia = e - r * ov;
    const size_t iq = r * 2 * ov + ia, ip = iq + ov;
    const double x = (mode == SSO_KICK_FIRST) ? c[iq] : W[pl ? ip : iq];
    double psum = 0.0;
    int sl = 0;
    for (; sl + 8 <= nslab; sl += 8) {
      float a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = P[(sl + u) * slab + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) psum += (double)a[u];
    }
    for (; sl < nslab; ++sl) psum += (double)P[sl * slab + e];
    const double E = sc[r * SC_STRIDE + SC_E];
    double hx = D[ia] * x + psum;
    if (use_field) hx -= E * F[pl ? ip : iq];
    double nxt;
    if (mode == SSO_DRIFT) {
      const double qn = c[iq] + dt * hx;
      c[iq] = qn;
      W[iq] = qn;
      nxt = qn;
    } else if (mode == SSO_KICK) {
      const double pn = W[ip] - 0.5 * dt * hx;
      c[ip] = pn;
      nxt = pn - 0.5 * dt * hx;
      W[ip] = nxt;
    } else {
      W[iq] = x;
      nxt = c[ip] - 0.5 * dt * hx;
      W[ip] = nxt;
    }
    x32[e] = (float)nxt;
    if (PREC == 1) split_bf16(nxt, xhi[e], xlo[e]);
    if (ia == 0) {
      const double h0 = use_field ? -E * sc[r * SC_STRIDE + (pl ? SC_GIM : SC_GRE)] : 0.0;
      if (mode == SSO_DRIFT) {
        const double q0 = c0[2 * r] + dt * h0;
        c0[2 * r] = q0;
        W0[2 * r] = q0;
      } else if (mode == SSO_KICK) {
        const double p0 = W0[2 * r + 1] - 0.5 * dt * h0;
        c0[2 * r + 1] = p0;
        W0[2 * r + 1] = p0 - 0.5 * dt * h0;
      } else {
        W0[2 * r] = c0[2 * r];
        W0[2 * r + 1] = c0[2 * r + 1] - 0.5 * dt * h0;
      }
    }
  }
}

// FP32 (+ BF16 hi/lo) copy of one plane of c into x32 [R][o][v].
template <int PREC>
__global__ void k_plane_copy(int R, size_t ov, int plane, const double *__restrict__ c, float *__restrict__ x32,
                             __hip_bfloat16 *__restrict__ xhi, __hip_bfloat16 *__restrict__ xlo) {
  const size_t total = (size_t)R * ov;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ov, ia = e - r * ov;
    const double x = c[(r * 2 + plane) * ov + ia];
    x32[e] = (float)x;
    if (PREC == 1) split_bf16(x, xhi[e], xlo[e]);
  }
}

// ------------------------------------------------------------------------------------------------
// Lanczos iteration on A (stability guard: the RK4 step is stable for rho(A) dt below ~2.8).
// Vectors of length ov in FP64; A v = D v + (Coulomb + exchange partials of v) for one real
// slice.  Block partial sums go to part[blockIdx.x] and are added in a fixed order on the host.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double x, double *sh) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

// start vector: a fixed pseudo-random vector (SplitMix64 of the index), part = |v|^2
__global__ __launch_bounds__(256) void k_lz_init(long long n, double *__restrict__ v, double *__restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    unsigned long long z = (unsigned long long)e + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double x = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    v[e] = x;
    acc += x * x;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w = A v - beta vprev, part = <w, v>
__global__ __launch_bounds__(256) void k_lz_apply(long long n, int nslab, const double *__restrict__ D,
                                                  const float *__restrict__ P, const double *__restrict__ v,
                                                  const double *__restrict__ vprev, double beta,
                                                  double *__restrict__ w, double *__restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    double s = D[e] * v[e];
    for (int k = 0; k < nslab; ++k) s += (double)P[(size_t)k * n + e];
    s -= beta * vprev[e];
    w[e] = s;
    acc += s * v[e];
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w -= alpha v, part = |w|^2
__global__ __launch_bounds__(256) void k_lz_orth(long long n, const double *__restrict__ v, double alpha,
                                                 double *__restrict__ w, double *__restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const double x = w[e] - alpha * v[e];
    w[e] = x;
    acc += x * x;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// vprev = v; v = w * scale; FP32 (+ BF16 hi/lo) copy of v for the next product
template <int PREC>
__global__ __launch_bounds__(256) void k_lz_next(long long n, double scale, const double *__restrict__ w,
                                                 double *__restrict__ v, double *__restrict__ vprev,
                                                 float *__restrict__ x32, __hip_bfloat16 *__restrict__ xhi,
                                                 __hip_bfloat16 *__restrict__ xlo, int shift) {
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    if (shift) vprev[e] = v[e];
    const double x = w[e] * scale;
    v[e] = x;
    x32[e] = (float)x;
    if (PREC == 1) split_bf16(x, xhi[e], xlo[e]);
  }
}

// ------------------------------------------------------------------------------------------------
// RK4 epilogue (FP64): sigma = D X + sum of Coulomb/exchange partials - E F;  k = -i sigma;
// stage accumulation into acc, next stage input (FP64 + FP32 or BF16 hi/lo copy), c at stage 4.
// One thread per (r, i, a), both planes.
// ------------------------------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256) void k_epilogue(int R, int o, int v, int nslab, int stage, int mode, int use_field,
                                                  double dt, const double *__restrict__ D,
                                                  const float *__restrict__ P, const double *__restrict__ F,
                                                  const double *__restrict__ sc, const double *__restrict__ Xin,
                                                  double *__restrict__ c, double *__restrict__ acc,
                                                  double *__restrict__ xs64, float *__restrict__ x32,
                                                  __hip_bfloat16 *__restrict__ xhi, __hip_bfloat16 *__restrict__ xlo,
                                                  double *__restrict__ s_out, double *__restrict__ epart) {
  const size_t ov = (size_t)o * v;
  const size_t slab = 2 * (size_t)R * ov;  // floats per partial slab
  const size_t r = blockIdx.y;             // one RHS per block row
  double en = 0.0;                         // this thread's part of <X, A X> (both planes)
  for (size_t ia = blockIdx.x * (size_t)blockDim.x + threadIdx.x; ia < ov; ia += (size_t)gridDim.x * blockDim.x) {
    const size_t i0 = r * 2 * ov + ia, i1 = i0 + ov;
    const double x0 = Xin[i0], x1 = Xin[i1];
    const double d = D[ia];
    // partial slabs: eight independent loads in flight per plane, summed in a fixed order
    double p0 = 0.0, p1 = 0.0;
    int sl = 0;
    for (; sl + 8 <= nslab; sl += 8) {
      float a[8], b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] = P[(sl + u) * slab + i0];
        b[u] = P[(sl + u) * slab + i1];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        p0 += (double)a[u];
        p1 += (double)b[u];
      }
    }
    for (; sl < nslab; ++sl) {
      p0 += (double)P[sl * slab + i0];
      p1 += (double)P[sl * slab + i1];
    }
    double s0v = d * x0 + p0, s1v = d * x1 + p1;
    if (epart) en += x0 * s0v + x1 * s1v;
    if (mode == EP_ENERGY) continue;
    if (use_field) {
      const double E = sc[r * SC_STRIDE + SC_E];
      s0v -= E * F[i0];
      s1v -= E * F[i1];
    }
    if (mode == EP_SIGMA) {
      s_out[i0] = s0v;
      s_out[i1] = s1v;
      continue;
    }
    // k = -i sigma: Re k = Im sigma, Im k = -Re sigma
    const double k0 = s1v, k1 = -s0v;
    double n0, n1;
    if (stage == 0) {
      acc[i0] = x0 + dt / 6.0 * k0;
      acc[i1] = x1 + dt / 6.0 * k1;
      n0 = x0 + 0.5 * dt * k0;
      n1 = x1 + 0.5 * dt * k1;
    } else if (stage == 3) {
      n0 = acc[i0] + dt / 6.0 * k0;
      n1 = acc[i1] + dt / 6.0 * k1;
      c[i0] = n0;
      c[i1] = n1;
    } else {
      acc[i0] += dt / 3.0 * k0;
      acc[i1] += dt / 3.0 * k1;
      const double h = (stage == 1) ? 0.5 * dt : dt;
      n0 = c[i0] + h * k0;
      n1 = c[i1] + h * k1;
    }
    if (stage != 3) {
      xs64[i0] = n0;
      xs64[i1] = n1;
    }
    x32[i0] = (float)n0;
    x32[i1] = (float)n1;
    if (PREC == 1) {
      split_bf16(n0, xhi[i0], xlo[i0]);
      split_bf16(n1, xhi[i1], xlo[i1]);
    }
  }
  if (epart) {  // block sum in a fixed order: waves, then the four wave totals
    __shared__ double ws[4];
    en = wave_sum(en);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = en;
    __syncthreads();
    if (threadIdx.x == 0) epart[r * gridDim.x + blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
  }
}

// First-order delta kick X <- X + i kappa M X for RHS with a delta pulse.
__global__ void k_kick(int R, int ov, const DevPulse *__restrict__ pulses, const double *__restrict__ F,
                       const double *__restrict__ sc, double *__restrict__ c, double *__restrict__ c0) {
  const size_t total = (size_t)R * ov;
  const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (size_t e = gid; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ov, ia = e - r * ov;
    if (pulses[r].kind != RTTDA_PULSE_DELTA) continue;
    const double kap = pulses[r].e0;
    const size_t i0 = r * 2 * ov + ia, i1 = i0 + ov;
    const double f0 = F[i0], f1 = F[i1];
    c[i0] -= kap * f1;
    c[i1] += kap * f0;
  }
  if (gid < (size_t)R && pulses[gid].kind == RTTDA_PULSE_DELTA) {
    const double kap = pulses[gid].e0;
    const double g0 = sc[gid * SC_STRIDE + SC_GRE], g1 = sc[gid * SC_STRIDE + SC_GIM];
    c0[2 * gid] -= kap * g1;
    c0[2 * gid + 1] += kap * g0;
  }
}

// One Taylor term of the unitary kick exp(i kappa M) X for the RHS with PULSE_DELTA_EXACT:
// given F = (M T)_C and g = (M T)_0 of the previous term T, the next term is (i kappa / j) M T;
// it replaces T and is added to the state (c, c0).
__global__ void k_kick_term(int R, int ov, const DevPulse *__restrict__ pulses, const double *__restrict__ F,
                            const double *__restrict__ sc, double inv_j, double *__restrict__ T,
                            double *__restrict__ T0, double *__restrict__ c, double *__restrict__ c0) {
  const size_t total = (size_t)R * ov;
  const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  for (size_t e = gid; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ov, ia = e - r * ov;
    if (pulses[r].kind != RTTDA_PULSE_DELTA_EXACT) continue;
    const double s = pulses[r].e0 * inv_j;
    const size_t i0 = r * 2 * ov + ia, i1 = i0 + ov;
    const double t0 = -s * F[i1], t1 = s * F[i0];
    T[i0] = t0;
    T[i1] = t1;
    c[i0] += t0;
    c[i1] += t1;
  }
  if (gid < (size_t)R && pulses[gid].kind == RTTDA_PULSE_DELTA_EXACT) {
    const double s = pulses[gid].e0 * inv_j;
    const double t0 = -s * sc[gid * SC_STRIDE + SC_GIM], t1 = s * sc[gid * SC_STRIDE + SC_GRE];
    T0[2 * gid] = t0;
    T0[2 * gid + 1] = t1;
    c0[2 * gid] += t0;
    c0[2 * gid + 1] += t1;
  }
}

__global__ void k_set_state(DevState *st, long long step0, double *trace, double *norms, double *corr, double *pops,
                            const double *popU, int popk, double *energy, const double *epart, long long nbe,
                            int resume) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->step = step0;
    st->step0 = step0;
    if (!resume) st->bad_step = -1;
    st->keep_ref = resume;
    st->energy = energy;
    st->epart = epart;
    st->nbe = nbe;
    st->trace = trace;
    st->norms = norms;
    st->corr = corr;
    st->pops = pops;
    st->popU = popU;
    st->popk = popk;
  }
}

// Eigenstate populations (eq. populations) at k = step - step0: pops[k][r][I] = |<U_I, X_r>|^2
// with real unit vectors U_I over the amplitudes c_ia (both planes); one block per (RHS, state),
// blocks past the state count return at once, a fixed-order block reduction.
__global__ __launch_bounds__(256) void k_pop(int R, size_t ov, const double *__restrict__ X,
                                             const DevState *__restrict__ st) {
  __shared__ double sh[2][4];
  double *pops = st->pops;
  const int K = (int)st->popk, r = blockIdx.x, I = blockIdx.y;
  if (pops == nullptr || I >= K) return;
  const double *u = st->popU + (size_t)I * ov, *x = X + (size_t)r * 2 * ov;
  double re = 0.0, im = 0.0;
  for (size_t e = threadIdx.x; e < ov; e += 256) {
    re += u[e] * x[e];
    im += u[e] * x[ov + e];
  }
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wave] = re;
    sh[1][wave] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]), b = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    const long long k = st->step - st->step0;
    pops[(k * R + r) * K + I] = a * a + b * b;
  }
}

// Time-correlation function (eq. time_correlation_function): corr[k][r] = <Xref_r | X_r>
// = conj(x0ref) x0 + sum_ia conj(Xref_ia) X_ia at k = step - step0, one block per RHS (the two
// planes of length ov and the ground amplitude), a fixed-order block reduction.
__global__ __launch_bounds__(256) void k_corr(int R, size_t ov, const double *__restrict__ X,
                                              const double *__restrict__ X0, const double *__restrict__ xref,
                                              const double *__restrict__ xref0, const DevState *__restrict__ st) {
  __shared__ double sh[2][4];
  double *corr = st->corr;
  if (corr == nullptr) return;
  const int r = blockIdx.x;
  const double *x = X + (size_t)r * 2 * ov, *y = xref + (size_t)r * 2 * ov;
  double re = 0.0, im = 0.0;
  for (size_t e = threadIdx.x; e < ov; e += 256) {
    const double a0 = y[e], a1 = y[ov + e], b0 = x[e], b1 = x[ov + e];
    re += a0 * b0 + a1 * b1;
    im += a0 * b1 - a1 * b0;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wave] = re;
    sh[1][wave] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double g0 = xref0[2 * r], g1 = xref0[2 * r + 1], c0 = X0[2 * r], c1 = X0[2 * r + 1];
    const long long k = st->step - st->step0;
    corr[(k * R + r) * 2] = (g0 * c0 + g1 * c1) + ((sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]));
    corr[(k * R + r) * 2 + 1] = (g0 * c1 - g1 * c0) + ((sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]));
  }
}

inline int grid_for(long long n, int block = 256, int cap = 8192) {
  long long g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_mu_blocks(hipStream_t s, const double *mu, const DevPulse *pulses, int o, int v, int R,
                            double *moo, double *mov, double *mvv) {
  const long long n = (long long)(o + v) * (o + v) * R;
  hipLaunchKernelGGL(k_mu_blocks, dim3(grid_for(n)), dim3(256), 0, s, mu, pulses, o, v, R, moo, mov, mvv);
  return hipGetLastError();
}

hipError_t launch_gaps(hipStream_t s, const double *e_occ, const double *e_virt, int o, int v, double *D) {
  hipLaunchKernelGGL(k_gaps, dim3(grid_for((long long)o * v)), dim3(256), 0, s, e_occ, e_virt, o, v, D);
  return hipGetLastError();
}

hipError_t launch_to_f32(hipStream_t s, const double *c, long long n, float *x32) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, c, n, x32);
  return hipGetLastError();
}

hipError_t launch_to_bf16x2(hipStream_t s, const double *c, long long n, float *x32, __hip_bfloat16 *hi,
                            __hip_bfloat16 *lo) {
  hipLaunchKernelGGL(k_to_bf16x2, dim3(grid_for(n)), dim3(256), 0, s, c, n, x32, hi, lo);
  return hipGetLastError();
}

int gemv1_chunks(int nq, int ov) {
  // independent of the slice count, so that a batch and a single RHS sum d identically
  if (nq <= 0 || ov <= 0) return 1;
  // as many ia chunks as keep the grid within one round of three workgroups per CU (the occupancy
  // of the six- and eight-slice forms' registers), so that no second, partly filled round follows
  const int blocks = (nq + 7) / 8;
  int es = std::max(1, std::min({768 / blocks, GEMV1_CHUNKS_MAX, ov / 2048}));
  const int echunk = (((ov + es - 1) / es) + 1023) / 1024 * 1024;
  return (ov + echunk - 1) / echunk;
}

template <typename TB, int ST>
static void gemv1_go(hipStream_t s, const TB *B, const float *X, int nq, int ov, int ns, int nes, float *dpart) {
  constexpr int QT = 8;
  const bool vec = (ov % 4) == 0;
  const int echunk = nes == 1 ? ov : (((ov + nes - 1) / nes) + 1023) / 1024 * 1024;
  dim3 grid((nq + QT - 1) / QT, (ns + ST - 1) / ST, nes);
  bool done = false;
  if constexpr (std::is_same<TB, __hip_bfloat16>::value) {
    if (ov % 8 == 0) {  // 16-byte loads of eight BF16 values
      hipLaunchKernelGGL((k_gemv1<TB, QT, ST, true, 8>), grid, dim3(256), 0, s, B, X, nq, ov, ns, echunk, dpart);
      done = true;
    }
  }
  if (done) {
  } else if (vec)
    hipLaunchKernelGGL((k_gemv1<TB, QT, ST, true>), grid, dim3(256), 0, s, B, X, nq, ov, ns, echunk, dpart);
  else
    hipLaunchKernelGGL((k_gemv1<TB, QT, ST, false>), grid, dim3(256), 0, s, B, X, nq, ov, ns, echunk, dpart);
  if (nes > 1) {
    const int n = nq * ns;
    hipLaunchKernelGGL(k_dsum, dim3(grid_for(n)), dim3(256), 0, s, dpart, n, nes);
  }
}

template <typename TB>
static void gemv1_st(hipStream_t s, const TB *B, const float *X, int nq, int ov, int ns, int nes, float *dpart) {
  if (ns <= 2) gemv1_go<TB, 2>(s, B, X, nq, ov, ns, nes, dpart);
  else if (ns <= 4) gemv1_go<TB, 4>(s, B, X, nq, ov, ns, nes, dpart);
  else if (ns <= 6) gemv1_go<TB, 6>(s, B, X, nq, ov, ns, nes, dpart);
  else gemv1_go<TB, 8>(s, B, X, nq, ov, ns, nes, dpart);
}

hipError_t launch_gemv1(hipStream_t s, int b_dtype, const void *B, const float *X, int nq, int ov, int ns, int nes,
                        float *dpart) {
  if (b_dtype == RTTDA_BF16)
    gemv1_st(s, static_cast<const __hip_bfloat16 *>(B), X, nq, ov, ns, nes, dpart);
  else
    gemv1_st(s, static_cast<const float *>(B), X, nq, ov, ns, nes, dpart);
  return hipGetLastError();
}

hipError_t launch_gemv2(hipStream_t s, int b_dtype, const void *B, const float *dvec, int nq, int ov, int ns,
                        int nsplit, float *P) {
  constexpr int ST = 8;
  dim3 grid((ov + 255) / 256, (ns + ST - 1) / ST, nsplit);
  if (b_dtype == RTTDA_BF16 && ov % 8 == 0) {
    dim3 g8((ov + 511) / 512, (ns + ST - 1) / ST, nsplit);
    hipLaunchKernelGGL((k_gemv2v<__hip_bfloat16, ST, 8>), g8, dim3(256), 0, s,
                       static_cast<const __hip_bfloat16 *>(B), dvec, nq, ov, ns, nsplit, P);
    return hipGetLastError();
  }
  if (ov % 4 == 0) {
    if (b_dtype == RTTDA_BF16)
      hipLaunchKernelGGL((k_gemv2v<__hip_bfloat16, ST, 4>), grid, dim3(256), 0, s,
                         static_cast<const __hip_bfloat16 *>(B), dvec, nq, ov, ns, nsplit, P);
    else
      hipLaunchKernelGGL((k_gemv2v<float, ST, 4>), grid, dim3(256), 0, s, static_cast<const float *>(B), dvec, nq,
                         ov, ns, nsplit, P);
    return hipGetLastError();
  }
  if (b_dtype == RTTDA_BF16)
    hipLaunchKernelGGL((k_gemv2<__hip_bfloat16, ST>), grid, dim3(256), 0, s, static_cast<const __hip_bfloat16 *>(B),
                       dvec, nq, ov, ns, nsplit, P);
  else
    hipLaunchKernelGGL((k_gemv2<float, ST>), grid, dim3(256), 0, s, static_cast<const float *>(B), dvec, nq, ov, ns,
                       nsplit, P);
  return hipGetLastError();
}

hipError_t launch_field(hipStream_t s, const double *X, const double *X0, const double *moo, const double *mov,
                        const double *mvv, int o, int v, int R, double *F, double *part) {
  dim3 grid(field_blocks_a(v), field_blocks_i(o), R);
  hipLaunchKernelGGL(k_field, grid, dim3(512), 0, s, X, X0, moo, mov, mvv, o, v, F, part);
  return hipGetLastError();
}

hipError_t launch_scalar(hipStream_t s, int R, int nbf, int stage, int mode, double dt, const DevPulse *pulses,
                         DevState *st, const double *part, double *sc, double *c0, double *acc0, double *xs0,
                         double *out, double *normref, double *s0) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(256), 0, s, R, nbf, stage, mode, dt, pulses, st, part, sc, c0, acc0,
                     xs0, out, normref, s0);
  return hipGetLastError();
}

hipError_t launch_epilogue(hipStream_t s, int prec, int R, int o, int v, int nslab, int stage, int mode,
                           int use_field, double dt, const double *D, const float *P, const double *F,
                           const double *sc, const double *Xin, double *c, double *acc, double *xs64, float *x32,
                           __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, double *s_out, double *epart) {
  dim3 grid(epilogue_blocks((long long)o * v), R);
  if (prec == RTTDA_PREC_MIXED_BF16)
    hipLaunchKernelGGL((k_epilogue<1>), grid, dim3(256), 0, s, R, o, v, nslab, stage, mode, use_field, dt, D, P, F,
                       sc, Xin, c, acc, xs64, x32, xhi, xlo, s_out, epart);
  else
    hipLaunchKernelGGL((k_epilogue<0>), grid, dim3(256), 0, s, R, o, v, nslab, stage, mode, use_field, dt, D, P, F,
                       sc, Xin, c, acc, xs64, x32, xhi, xlo, s_out, epart);
  return hipGetLastError();
}

int epilogue_blocks(long long ov) { return (int)std::min<long long>((ov + 255) / 256, EP_BX_MAX); }

hipError_t launch_sso_update(hipStream_t s, int prec, int R, int o, int v, int nslab, int mode, int use_field,
                             double dt, const double *D, const float *P, const double *F, const double *sc, double *c,
                             double *c0, double *W, double *W0, float *x32, __hip_bfloat16 *xhi,
                             __hip_bfloat16 *xlo) {
  const long long n = (long long)R * o * v;
  dim3 grid(grid_for(n, 256, 65536));
  if (prec == RTTDA_PREC_MIXED_BF16)
    hipLaunchKernelGGL((k_sso_update<1>), grid, dim3(256), 0, s, R, o, v, nslab, mode, use_field, dt, D, P, F, sc, c,
                       c0, W, W0, x32, xhi, xlo);
  else
    hipLaunchKernelGGL((k_sso_update<0>), grid, dim3(256), 0, s, R, o, v, nslab, mode, use_field, dt, D, P, F, sc, c,
                       c0, W, W0, x32, xhi, xlo);
  return hipGetLastError();
}

hipError_t launch_plane_copy(hipStream_t s, int prec, int R, size_t ov, int plane, const double *c, float *x32,
                             __hip_bfloat16 *xhi, __hip_bfloat16 *xlo) {
  const long long n = (long long)R * (long long)ov;
  dim3 grid(grid_for(n, 256, 65536));
  if (prec == RTTDA_PREC_MIXED_BF16)
    hipLaunchKernelGGL((k_plane_copy<1>), grid, dim3(256), 0, s, R, ov, plane, c, x32, xhi, xlo);
  else
    hipLaunchKernelGGL((k_plane_copy<0>), grid, dim3(256), 0, s, R, ov, plane, c, x32, xhi, xlo);
  return hipGetLastError();
}

int lz_blocks(long long n) { return (int)std::min<long long>(LZ_BLOCKS_MAX, std::max<long long>(1, (n + 255) / 256)); }

hipError_t launch_lz_init(hipStream_t s, long long n, double *v, double *part) {
  hipLaunchKernelGGL(k_lz_init, dim3(lz_blocks(n)), dim3(256), 0, s, n, v, part);
  return hipGetLastError();
}
hipError_t launch_lz_apply(hipStream_t s, long long n, int nslab, const double *D, const float *P, const double *v,
                           const double *vprev, double beta, double *w, double *part) {
  hipLaunchKernelGGL(k_lz_apply, dim3(lz_blocks(n)), dim3(256), 0, s, n, nslab, D, P, v, vprev, beta, w, part);
  return hipGetLastError();
}
hipError_t launch_lz_orth(hipStream_t s, long long n, const double *v, double alpha, double *w, double *part) {
  hipLaunchKernelGGL(k_lz_orth, dim3(lz_blocks(n)), dim3(256), 0, s, n, v, alpha, w, part);
  return hipGetLastError();
}
hipError_t launch_lz_next(hipStream_t s, int prec, long long n, double scale, const double *w, double *v,
                          double *vprev, float *x32, __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, int shift) {
  if (prec == RTTDA_PREC_MIXED_BF16)
    hipLaunchKernelGGL((k_lz_next<1>), dim3(lz_blocks(n)), dim3(256), 0, s, n, scale, w, v, vprev, x32, xhi, xlo,
                       shift);
  else
    hipLaunchKernelGGL((k_lz_next<0>), dim3(lz_blocks(n)), dim3(256), 0, s, n, scale, w, v, vprev, x32, xhi, xlo,
                       shift);
  return hipGetLastError();
}

hipError_t launch_kick(hipStream_t s, int R, int ov, const DevPulse *pulses, const double *F, const double *sc,
                       double *c, double *c0) {
  const long long n = (long long)R * ov;
  hipLaunchKernelGGL(k_kick, dim3(grid_for(n)), dim3(256), 0, s, R, ov, pulses, F, sc, c, c0);
  return hipGetLastError();
}

hipError_t launch_kick_term(hipStream_t s, int R, int ov, const DevPulse *pulses, const double *F, const double *sc,
                            double inv_j, double *T, double *T0, double *c, double *c0) {
  const long long n = (long long)R * ov;
  hipLaunchKernelGGL(k_kick_term, dim3(grid_for(n)), dim3(256), 0, s, R, ov, pulses, F, sc, inv_j, T, T0, c, c0);
  return hipGetLastError();
}

hipError_t launch_set_state(hipStream_t s, DevState *st, long long step0, double *trace, double *norms,
                            double *corr, double *pops, const double *popU, int popk, double *energy,
                            const double *epart, long long nbe, int resume) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, step0, trace, norms, corr, pops, popU, popk, energy,
                     epart, nbe, resume);
  return hipGetLastError();
}

// Kick spectra on a frequency grid (eq. fourier_transform, with the half-Hann window that
// equals a full Hann window on the mirrored record): for a dipole trace (kind 0)
//   S_s(w) = w sum_n h_n (mu_n - mu_0) sin(w t_n) dt / kappa,
// for the time-correlation function (kind 1)
//   S_s(w) = w Re sum_n h_n R_n exp(i w t_n) dt,
// with h_n = (1 + cos(pi n / N)) / 2, t_n = n dt, n = 0..N.  One thread per (frequency, signal);
// average: out[w] = the mean over the signals (eq. spectrum_average) instead of out[s][w].
__global__ __launch_bounds__(256) void k_spectrum(int kind, const double *__restrict__ sig, int n_t, int nsig, double dt,
                                                  double kappa, int n_w, double w0, double dw, int average,
                                                  double *__restrict__ out) {
  const int w_idx = blockIdx.x * 256 + threadIdx.x;
  if (w_idx >= n_w) return;
  const double w = w0 + dw * w_idx;
  const int N = n_t - 1;
  double mean = 0.0;
  for (int s = 0; s < nsig; ++s) {
    double acc = 0.0;
    const double base = kind == 0 ? sig[s] : 0.0;
    for (int n = 0; n < n_t; ++n) {
      const double h = N > 0 ? 0.5 * (1.0 + cos(M_PI * (double)n / N)) : 1.0;
      double sn, cs;
      sincos(w * (n * dt), &sn, &cs);
      if (kind == 0)
        acc += h * (sig[(size_t)n * nsig + s] - base) * sn;
      else
        acc += h * (sig[((size_t)n * nsig + s) * 2] * cs - sig[((size_t)n * nsig + s) * 2 + 1] * sn);
    }
    const double val = kind == 0 ? w * acc * dt / kappa : w * acc * dt;
    if (average)
      mean += val;
    else
      out[(size_t)s * n_w + w_idx] = val;
  }
  if (average) out[w_idx] = mean / nsig;
}

hipError_t launch_spectrum(hipStream_t s, int kind, const double *sig, int n_t, int nsig, double dt, double kappa,
                           int n_w, double w0, double dw, int average, double *out) {
  hipLaunchKernelGGL(k_spectrum, dim3((n_w + 255) / 256), dim3(256), 0, s, kind, sig, n_t, nsig, dt, kappa, n_w, w0, dw,
                     average, out);
  return hipGetLastError();
}

hipError_t launch_pop(hipStream_t s, int R, size_t ov, const double *X, const DevState *st) {
  hipLaunchKernelGGL(k_pop, dim3(R, POP_MAX), dim3(256), 0, s, R, ov, X, st);
  return hipGetLastError();
}

hipError_t launch_corr(hipStream_t s, int R, size_t ov, const double *X, const double *X0, const double *xref,
                       const double *xref0, const DevState *st) {
  hipLaunchKernelGGL(k_corr, dim3(R), dim3(256), 0, s, R, ov, X, X0, xref, xref0, st);
  return hipGetLastError();
}

}  // namespace rttda
