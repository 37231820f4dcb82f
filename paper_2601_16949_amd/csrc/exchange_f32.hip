// Exchange contraction on gfx950 matrix cores, FP32:
//   P[split][s][i][c] = scale * sum_{Q in split} (B_oo^Q X_s B_vv^Q)[i][c]
// for every slice s (one real plane of one right-hand side; slices stacked as rows).
//
// Order of the two products per Q: W = X_s B_vv^Q first (the large o x v x v product, B_vv^Q
// streamed through LDS once per workgroup), then K_s += B_oo^Q W (o x o x v).  W never leaves the
// matrix-core accumulators: its 16x16 output blocks are fed straight back as the B operand of the
// second product, because the accumulator layout (row 4g + t of a block in register t of lane
// group g) equals the operand layout once the K index of that product is permuted the same way
// for both operands.  The same permutation lets every operand fragment come from one 16-byte LDS
// read (4 consecutive K values per lane).
//
// v_mfma_f32_16x16x4_f32 operand layout (lane l = 16 g + n):
//   A[m = n][k = g], B[k = g][n], D[m = 4 g + t][n] in accumulator register t.
#include "common.h"

namespace rttda {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;       // K chunk (virtual index a) per LDS stage
constexpr int XP = KC + 4;   // LDS row pitch (floats) of the X and B_vv tiles

template <int O16, int WS, int WC>
struct Cfg {
  static constexpr int KS = 2 * WS;   // slices per workgroup (2 waves along slices)
  static constexpr int NT = 32 * WC;  // columns per workgroup (2 waves along columns)
  static constexpr int JB = O16 / 16;
  static constexpr int OP = O16 + 4;  // LDS pitch of the B_oo tile
  static constexpr size_t LDS = (size_t)(KS * O16 * XP + NT * XP + O16 * OP) * sizeof(float);
};

template <int O16, int WS, int WC>
__global__ __launch_bounds__(256, 1) void k_exchange_f32(const float *__restrict__ Boo,
                                                         const float *__restrict__ Bvv,
                                                         const float *__restrict__ X, int o, int v, int nq, int ns,
                                                         int n_sg, int n_ct, int nsplit, float scale,
                                                         float *__restrict__ P) {
  using C = Cfg<O16, WS, WC>;
  constexpr int KS = C::KS, NT = C::NT, JB = C::JB, OP = C::OP;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  float *Xs = lds;                  // [KS*O16][XP]
  float *Bs = Xs + KS * O16 * XP;   // [NT][XP]
  float *Os = Bs + NT * XP;         // [O16][OP]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int ws = wave >> 1, wc = wave & 1;

  const int bid = blockIdx.x;
  const int sg = bid % n_sg;
  const int ct = (bid / n_sg) % n_ct;
  const int sp = bid / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * KS, c_base = ct * NT;
  const bool vec = (v & 3) == 0;

  f4 Kacc[WS][JB][WC];
#pragma unroll
  for (int a = 0; a < WS; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int c = 0; c < WC; ++c) Kacc[a][b][c] = f4{0.f, 0.f, 0.f, 0.f};

  for (int q = qa; q < qb; ++q) {
    __syncthreads();
    const float *Oq = Boo + (size_t)q * o * o;
    for (int e = tid; e < O16 * O16; e += 256) {
      const int i = e / O16, j = e - i * O16;
      Os[i * OP + j] = (i < o && j < o) ? Oq[(size_t)i * o + j] : 0.f;
    }
    const float *Vq = Bvv + (size_t)q * v * v;

    f4 Wacc[WS][JB][WC];
#pragma unroll
    for (int a = 0; a < WS; ++a)
#pragma unroll
      for (int b = 0; b < JB; ++b)
#pragma unroll
        for (int c = 0; c < WC; ++c) Wacc[a][b][c] = f4{0.f, 0.f, 0.f, 0.f};

    for (int a0 = 0; a0 < v; a0 += KC) {
      __syncthreads();
      // X tile: rows (slice, j) of this workgroup's slices, columns a0 .. a0+KC
      for (int e = tid; e < KS * O16 * (KC / 4); e += 256) {
        const int row = e / (KC / 4), k4 = (e - row * (KC / 4)) * 4;
        const int sl = s_base + row / O16, j = row % O16, a = a0 + k4;
        f4 val = f4{0.f, 0.f, 0.f, 0.f};
        if (sl < ns && j < o) {
          const float *src = X + ((size_t)sl * o + j) * v + a;
          if (vec && a < v) {
            val = *reinterpret_cast<const f4 *>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) val[t] = (a + t < v) ? src[t] : 0.f;
          }
        }
        *reinterpret_cast<f4 *>(&Xs[row * XP + k4]) = val;
      }
      // B_vv tile: rows c of this workgroup's columns, columns a0 .. a0+KC (B_vv symmetric)
      for (int e = tid; e < NT * (KC / 4); e += 256) {
        const int cl = e / (KC / 4), k4 = (e - cl * (KC / 4)) * 4;
        const int cc = c_base + cl, a = a0 + k4;
        f4 val = f4{0.f, 0.f, 0.f, 0.f};
        if (cc < v) {
          const float *src = Vq + (size_t)cc * v + a;
          if (vec && a < v) {
            val = *reinterpret_cast<const f4 *>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) val[t] = (a + t < v) ? src[t] : 0.f;
          }
        }
        *reinterpret_cast<f4 *>(&Bs[cl * XP + k4]) = val;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; kk += 16) {
        f4 bf[WC];
#pragma unroll
        for (int cb = 0; cb < WC; ++cb)
          bf[cb] = *reinterpret_cast<const f4 *>(&Bs[((wc * WC + cb) * 16 + n) * XP + kk + 4 * g]);
        f4 af[WS][JB];
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
            af[si][jb] = *reinterpret_cast<const f4 *>(&Xs[((ws * WS + si) * O16 + jb * 16 + n) * XP + kk + 4 * g]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int si = 0; si < WS; ++si)
#pragma unroll
            for (int jb = 0; jb < JB; ++jb)
#pragma unroll
              for (int cb = 0; cb < WC; ++cb)
                Wacc[si][jb][cb] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(af[si][jb][t], bf[cb][t], Wacc[si][jb][cb], 0, 0, 0);
      }
    }
    // K += B_oo^Q W.  Step (jb, t): lane (g, n) supplies W[j = 16 jb + 4 g + t][c] (its own
    // accumulator register t) and B_oo[i][j] for the same j (B_oo symmetric: read row i).
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      f4 ar[JB];
#pragma unroll
      for (int ib = 0; ib < JB; ++ib) ar[ib] = *reinterpret_cast<const f4 *>(&Os[(ib * 16 + n) * OP + jb * 16 + 4 * g]);
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int si = 0; si < WS; ++si)
#pragma unroll
            for (int cb = 0; cb < WC; ++cb)
              Kacc[si][ib][cb] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ib][t], Wacc[si][jb][cb][t], Kacc[si][ib][cb], 0, 0, 0);
    }
  }

  float *Pp = P + (size_t)sp * ns * o * v;
#pragma unroll
  for (int si = 0; si < WS; ++si) {
    const int sl = s_base + ws * WS + si;
    if (sl >= ns) continue;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
      for (int cb = 0; cb < WC; ++cb) {
        const int c = c_base + (wc * WC + cb) * 16 + n;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = ib * 16 + 4 * g + t;
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[si][ib][cb][t];
        }
      }
  }
}

template <int O16, int WS, int WC>
hipError_t launch_xf32(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void * /*Xlo*/, int o,
                       int v, int nq, int ns, int nsplit, float scale, float *P) {
  using C = Cfg<O16, WS, WC>;
  if (o > O16) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  dim3 grid(n_sg * n_ct * nsplit);
  hipLaunchKernelGGL((k_exchange_f32<O16, WS, WC>), grid, dim3(256), C::LDS, s, static_cast<const float *>(Boo),
                     static_cast<const float *>(Bvv), static_cast<const float *>(X), o, v, nq, ns, n_sg, n_ct, nsplit,
                     scale, P);
  return hipGetLastError();
}

template <int O16, int WS, int WC>
hipError_t prepare_xf32() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_f32<O16, WS, WC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)Cfg<O16, WS, WC>::LDS);
}

#define XF32(O16, WS, WC)                                                                              \
  ExchangeVariant {                                                                                    \
    RTTDA_PREC_FP32, O16, Cfg<O16, WS, WC>::KS, Cfg<O16, WS, WC>::NT, "f32_o" #O16 "_ws" #WS "_wc" #WC, \
        &launch_xf32<O16, WS, WC>, Cfg<O16, WS, WC>::LDS, &prepare_xf32<O16, WS, WC>                  \
  }

const ExchangeVariant kF32Variants[] = {
    XF32(16, 1, 1),  XF32(16, 2, 2), XF32(16, 4, 2),  XF32(32, 2, 2),  XF32(32, 4, 2), XF32(48, 2, 2),
    XF32(48, 3, 2),  XF32(48, 4, 1), XF32(64, 1, 2),  XF32(64, 3, 2),  XF32(64, 2, 2), XF32(64, 3, 1),
    XF32(80, 2, 2),  XF32(96, 1, 2), XF32(96, 2, 1),  XF32(112, 1, 2), XF32(128, 1, 2), XF32(128, 1, 1),
};

}  // namespace

int exchange_f32_variant_count() { return (int)(sizeof(kF32Variants) / sizeof(kF32Variants[0])); }
const ExchangeVariant *exchange_f32_variant(int k) { return &kF32Variants[k]; }

}  // namespace rttda
