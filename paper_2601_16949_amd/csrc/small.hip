// Small problems, where a step is bound by the gaps between dependent launches rather than by
// any bandwidth (o v up to 2048, at most 64 right-hand sides): each RK4 stage is two launches.
//  * k_small_2e: the Coulomb and exchange parts of sigma for one slice and a range of Q in one
//    workgroup.  Every Q term of J = 2 sum_Q B^Q <B^Q, X> needs only its own d_Q, so no grid-wide
//    step separates the two Coulomb products here; the exchange term B_oo^Q X B_vv^Q goes through
//    the workgroup's LDS (FP32 FMA: at these sizes the matrix cores would idle on latency anyway).
//    Each workgroup writes one partial slab J - c_x K for its Q range.
//  * k_small_epi: the whole stage epilogue of all right-hand sides in one workgroup: the field
//    product F = X mu_vv - mu_oo X + sqrt2 mu_ov c0 (FP64), the stage scalars (pulse field, ground
//    row g, trace, norm and guard, energy, c0 update), sigma = D X + sum of slabs - E F, and the RK4
//    stage update with the next stage's FP32 (and BF16 hi/lo) copies.  Block reductions run in a
//    fixed order, so results are reproducible run to run.
#include "common.h"

namespace rttda {
namespace {

__device__ __forceinline__ float bload(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float bload(const __hip_bfloat16 *p, size_t i) { return __bfloat162float(p[i]); }

template <typename T>
__device__ __forceinline__ T wsum(T x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ void split_hl(double x, __hip_bfloat16 &hi, __hip_bfloat16 &lo) {
  hi = __float2bfloat16((float)x);
  lo = __float2bfloat16((float)(x - (double)__bfloat162float(hi)));
}

constexpr int EPT2 = SMALL_OV_MAX / 256;  // elements per thread of k_small_2e

// sum_k x[k sx] y[k sy] for k < n as four interleaved partial sums (four independent LDS reads and
// FMAs in flight instead of one dependent chain), added in a fixed order
template <typename T>
__device__ __forceinline__ T dot4(const T *x, int sx, const T *y, int sy, int n) {
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    a0 += x[k * sx] * y[k * sy];
    a1 += x[(k + 1) * sx] * y[(k + 1) * sy];
    a2 += x[(k + 2) * sx] * y[(k + 2) * sy];
    a3 += x[(k + 3) * sx] * y[(k + 3) * sy];
  }
  for (; k < n; ++k) a0 += x[k * sx] * y[k * sy];
  return (a0 + a1) + (a2 + a3);
}

// grid (nsplit, ns), 256 threads; dynamic LDS: X slice, W, B_vv^Q and B_oo^Q (floats)
template <typename TB>
__global__ __launch_bounds__(256) void k_small_2e(const TB *__restrict__ Bov, const TB *__restrict__ Boo,
                                                  const TB *__restrict__ Bvv, const float *__restrict__ X, int o,
                                                  int v, int nq, int ns, int nsplit, float cx,
                                                  float *__restrict__ P) {
  extern __shared__ float sm2[];
  __shared__ float red[4];
  const int sp = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ov = o * v;
  float *Xs = sm2, *W = sm2 + ov, *Vs = W + ov, *Os = Vs + v * v;
  const float *Xg = X + (size_t)s * ov;
  for (int e = tid; e < ov; e += 256) Xs[e] = Xg[e];
  __syncthreads();
  float J[EPT2], K[EPT2];
#pragma unroll
  for (int k = 0; k < EPT2; ++k) J[k] = K[k] = 0.f;
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  for (int q = qa; q < qb; ++q) {
    const TB *Bq = Bov + (size_t)q * ov;
    const TB *Vq = Bvv + (size_t)q * v * v;
    const TB *Oq = Boo + (size_t)q * o * o;
    for (int e = tid; e < v * v; e += 256) Vs[e] = bload(Vq, e);  // coalesced staging of this Q's factors
    for (int e = tid; e < o * o; e += 256) Os[e] = bload(Oq, e);
    float bq[EPT2];
    float pd = 0.f;
#pragma unroll
    for (int k = 0; k < EPT2; ++k) {
      const int e = tid + 256 * k;
      bq[k] = e < ov ? bload(Bq, e) : 0.f;
      if (e < ov) pd += bq[k] * Xs[e];
    }
    pd = wsum(pd);
    if (lane == 0) red[wave] = pd;
    __syncthreads();
    const float d = (red[0] + red[1]) + (red[2] + red[3]);
#pragma unroll
    for (int k = 0; k < EPT2; ++k) {
      const int e = tid + 256 * k;
      if (e < ov) {
        J[k] += 2.f * d * bq[k];
        const int i = e / v, a = e - i * v;
        W[e] = dot4(Xs + i * v, 1, Vs + a, v, v);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT2; ++k) {
      const int e = tid + 256 * k;
      if (e < ov) {
        const int i = e / v, a = e - i * v;
        K[k] += dot4(Os + i * o, 1, W + a, v, o);
      }
    }
    __syncthreads();  // W, red and the staged factors are rewritten by the next Q
  }
  float *Pp = P + ((size_t)sp * ns + s) * ov;
#pragma unroll
  for (int k = 0; k < EPT2; ++k) {
    const int e = tid + 256 * k;
    if (e < ov) Pp[e] = J[k] - cx * K[k];
  }
}

constexpr int NTE = 512;                  // threads of k_small_epi (two waves per SIMD: no register spills)
constexpr int EPT = SMALL_OV_MAX / NTE;   // (i, a) elements per thread of k_small_epi

// One workgroup of NTE threads; the right-hand sides one after another.  The RHS's two planes of
// X and its dipole blocks are staged in LDS (dynamic, SMALL_LDS_DOUBLES), so the field product's
// dot products read LDS; the partial slabs are read sixteen at a time.
template <int PREC>
__global__ __launch_bounds__(NTE) void k_small_epi(int R, int o, int v, int nslab, int stage, int use_field,
                                                    int want_trace, double dt, const DevPulse *__restrict__ pulses,
                                                    DevState *__restrict__ st, const double *__restrict__ D,
                                                    const float *__restrict__ P, const double *__restrict__ moo,
                                                    const double *__restrict__ mov, const double *__restrict__ mvv,
                                                    const double *__restrict__ Xin, double *__restrict__ c,
                                                    double *__restrict__ c0, double *__restrict__ acc,
                                                    double *__restrict__ acc0, double *__restrict__ xs64,
                                                    double *__restrict__ xs0, float *__restrict__ x32,
                                                    __hip_bfloat16 *__restrict__ xhi, __hip_bfloat16 *__restrict__ xlo,
                                                    double *__restrict__ normref) {
  __shared__ double red[NTE / 64][5];
  __shared__ double tot[5];
  __shared__ int bad;
  extern __shared__ double lds_e[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ov = o * v;
  double *Xl = lds_e;            // [2][o][v] this RHS's stage input
  double *Ml = Xl + 2 * ov;      // [v][v] mu_vv
  double *Ol = Ml + v * v;       // [o][o] mu_oo
  const size_t slab = 2 * (size_t)R * ov;
  const long long step = st->step, k = step - st->step0;
  // stage -1: the sample of the state c itself (trace, norm, guard, energy) with no update, as the
  // last sample of a call; the same sums as a stage 0, so that a run split into calls gives the
  // same samples as one call
  const bool sample = stage < 0;
  const double node = (stage <= 0) ? 0.0 : (stage == 3 ? 1.0 : 0.5);
  const bool need_f = use_field || want_trace;
  if (tid == 0) bad = 0;
  for (int r = 0; r < R; ++r) {
    const double E = use_field ? pulse_field(pulses[r], ((double)step + node) * dt) : 0.0;
    const double *X0 = stage <= 0 ? c0 : xs0;
    const double x0r = X0[2 * r], x0i = X0[2 * r + 1];
    const double *moo_r = moo + (size_t)r * o * o, *mov_r = mov + (size_t)r * ov, *mvv_r = mvv + (size_t)r * v * v;
    if (need_f) {
      for (int e = tid; e < 2 * ov; e += NTE) Xl[e] = Xin[(size_t)r * 2 * ov + e];
      for (int e = tid; e < v * v; e += NTE) Ml[e] = mvv_r[e];
      for (int e = tid; e < o * o; e += NTE) Ol[e] = moo_r[e];
      __syncthreads();
    }
    double sg[EPT][2];
    double pg0 = 0.0, pg1 = 0.0, ptr = 0.0, pnr = 0.0, pen = 0.0;
#pragma unroll
    for (int kk = 0; kk < EPT; ++kk) {
      const int ia = tid + NTE * kk;
      sg[kk][0] = sg[kk][1] = 0.0;
      if (ia >= ov) continue;
      const int i = ia / v, a = ia - i * v;
      const size_t i0 = (size_t)r * 2 * ov + ia, i1 = i0 + ov;
      const double x[2] = {Xin[i0], Xin[i1]};
      double ps0 = 0.0, ps1 = 0.0;
      int sl = 0;
      for (; sl + 16 <= nslab; sl += 16) {  // sixteen slabs' loads in flight, added in order
        float a[16], b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          a[u] = P[(sl + u) * slab + i0];
          b[u] = P[(sl + u) * slab + i1];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          ps0 += (double)a[u];
          ps1 += (double)b[u];
        }
      }
      for (; sl < nslab; ++sl) {
        ps0 += (double)P[sl * slab + i0];
        ps1 += (double)P[sl * slab + i1];
      }
      const double d = D[ia];
      double s0 = d * x[0] + ps0, s1 = d * x[1] + ps1;
      pen += x[0] * s0 + x[1] * s1;
      if (need_f) {
        const double mo = mov_r[ia];
        double f[2];
        for (int p = 0; p < 2; ++p) {
          const double *Xp = Xl + p * ov;
          const double t = dot4(Xp + i * v, 1, Ml + a, v, v) - dot4(Ol + i * o, 1, Xp + a, v, o);
          f[p] = t + SQRT2 * mo * (p == 0 ? x0r : x0i);
        }
        pg0 += SQRT2 * mo * x[0];
        pg1 += SQRT2 * mo * x[1];
        ptr += x[0] * f[0] + x[1] * f[1];
        pnr += x[0] * x[0] + x[1] * x[1];
        s0 -= E * f[0];
        s1 -= E * f[1];
      }
      sg[kk][0] = s0;
      sg[kk][1] = s1;
    }
    // block totals of g (two planes), <X|F>, |X|^2 and <X, A X>, in a fixed order
    const double pv[5] = {pg0, pg1, ptr, pnr, pen};
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const double w = wsum(pv[t]);
      if (lane == 0) red[wave][t] = w;
    }
    __syncthreads();
    if (tid < 5) {
      double a = 0.0;
      for (int w = 0; w < NTE / 64; ++w) a += red[w][tid];
      tot[tid] = a;
    }
    __syncthreads();
    const double g0 = tot[0], g1 = tot[1];
    if (tid == 0) {
      if (want_trace) {
        const double t = tot[2] + (x0r * g0 + x0i * g1);
        const double n2 = tot[3] + (x0r * x0r + x0i * x0i);
        if (st->trace) st->trace[k * R + r] = t;
        if (st->norms) st->norms[k * R + r] = n2;
        if (k == 0 && !st->keep_ref) {
          normref[r] = n2;
        } else if (!(n2 <= 2.0 * normref[r])) {
          bad = 1;
        }
        if (st->energy) st->energy[k * R + r] = tot[4];
      }
      if (use_field && !sample) {  // c0: k0 = -i (H X)_0 = i E g
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
    // RK4 stage update of this RHS's amplitudes (k = -i sigma: Re k = Im sigma, Im k = -Re sigma)
#pragma unroll
    for (int kk = 0; kk < EPT; ++kk) {
      const int ia = tid + NTE * kk;
      if (sample || ia >= ov) continue;
      const size_t i0 = (size_t)r * 2 * ov + ia, i1 = i0 + ov;
      const double k0 = sg[kk][1], k1 = -sg[kk][0];
      double n0, n1;
      if (stage == 0) {
        const double x0 = Xin[i0], x1 = Xin[i1];
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
        split_hl(n0, xhi[i0], xlo[i0]);
        split_hl(n1, xhi[i1], xlo[i1]);
      }
    }
    __syncthreads();  // red and tot are reused by the next RHS
  }
  if (tid == 0) {
    if (bad && st->bad_step < 0) st->bad_step = step;
    if (stage == 3) st->step = step + 1;
  }
}

}  // namespace

hipError_t prepare_small() {
  const int bytes = SMALL_LDS_DOUBLES * (int)sizeof(double);
  const void *fn[] = {reinterpret_cast<const void *>(&k_small_epi<0>), reinterpret_cast<const void *>(&k_small_epi<1>),
                      reinterpret_cast<const void *>(&k_small_2e<float>),
                      reinterpret_cast<const void *>(&k_small_2e<__hip_bfloat16>)};
  for (const void *f : fn) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_small_2e(hipStream_t s, int b_dtype, const void *Bov, const void *Boo, const void *Bvv,
                           const float *X, int o, int v, int nq, int ns, int nsplit, float cx, float *P) {
  const int ov = o * v;
  if (ov > SMALL_OV_MAX || nsplit < 1) return hipErrorInvalidValue;
  const dim3 grid(nsplit, ns);
  const size_t lds = ((size_t)2 * ov + (size_t)v * v + (size_t)o * o) * sizeof(float);
  if (b_dtype == RTTDA_BF16)
    hipLaunchKernelGGL(k_small_2e<__hip_bfloat16>, grid, dim3(256), lds, s,
                       static_cast<const __hip_bfloat16 *>(Bov), static_cast<const __hip_bfloat16 *>(Boo),
                       static_cast<const __hip_bfloat16 *>(Bvv), X, o, v, nq, ns, nsplit, cx, P);
  else
    hipLaunchKernelGGL(k_small_2e<float>, grid, dim3(256), lds, s, static_cast<const float *>(Bov),
                       static_cast<const float *>(Boo), static_cast<const float *>(Bvv), X, o, v, nq, ns, nsplit, cx,
                       P);
  return hipGetLastError();
}

hipError_t launch_small_epi(hipStream_t s, int prec, int R, int o, int v, int nslab, int stage, int use_field,
                            int want_trace, double dt, const DevPulse *pulses, DevState *st, const double *D,
                            const float *P, const double *moo, const double *mov, const double *mvv,
                            const double *Xin, double *c, double *c0, double *acc, double *acc0, double *xs64,
                            double *xs0, float *x32, __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, double *normref) {
  if (!small_shape_ok(o, v) || R > SMALL_R_MAX) return hipErrorInvalidValue;
  const size_t lds = (size_t)(2 * o * v + v * v + o * o) * sizeof(double);
  if (prec == RTTDA_PREC_MIXED_BF16)
    hipLaunchKernelGGL(k_small_epi<1>, dim3(1), dim3(NTE), lds, s, R, o, v, nslab, stage, use_field, want_trace, dt,
                       pulses, st, D, P, moo, mov, mvv, Xin, c, c0, acc, acc0, xs64, xs0, x32, xhi, xlo, normref);
  else
    hipLaunchKernelGGL(k_small_epi<0>, dim3(1), dim3(NTE), lds, s, R, o, v, nslab, stage, use_field, want_trace, dt,
                       pulses, st, D, P, moo, mov, mvv, Xin, c, c0, acc, acc0, xs64, xs0, x32, xhi, xlo, normref);
  return hipGetLastError();
}

}  // namespace rttda
