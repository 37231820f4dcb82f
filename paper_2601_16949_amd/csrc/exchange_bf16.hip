// Exchange contraction on gfx950 matrix cores, split BF16 precision:
//   P[split][s][i][c] = scale * sum_{Q in split} (B_oo^Q X_s B_vv^Q)[i][c]
// with B stored exactly in BF16 and X = X_hi + X_lo (two BF16 planes, about 16 significant bits).
// Both products are taken as two BF16 products with FP32 accumulation:
//   W   = X_hi B_vv^Q + X_lo B_vv^Q               (FP32 accumulators)
//   K  += B_oo^Q W_hi + B_oo^Q W_lo,  W_hi = bf16(W), W_lo = bf16(W - W_hi)
// The structure follows the FP32 kernel: W = X B_vv^Q first with B_vv^Q tiles staged in LDS, then
// the accumulator blocks of W feed the second product directly (no LDS round trip), using the
// freedom to permute the K index of a product consistently in both operands.
//
// v_mfma_f32_32x32x16_bf16 (lane l = 32 h + m): the lane supplies eight K values of row m of A and
// of column m of B; the 32x32 result sits in 16 registers, register t of lane (h, n) holding
// D[8 (t/4) + 4 h + t%4][n].  32x32 blocks need half the operand bytes per flop of 16x16 blocks,
// which keeps LDS traffic well under its bandwidth at the BF16 rate.
//   W product: lane's K values are a = k0 + 8 h + e (e = 0..7): one 16-byte LDS read per operand.
//   K product: for W block jb and half u, lane's K values are j = 32 jb + 8 (t/4) + 4 h + t%4 for
//              t = 8u .. 8u+7, i.e. its own accumulator registers t of that block.
#include "common.h"

namespace rttda {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;      // K chunk (virtual index a) per LDS stage = two MFMA K steps
constexpr int XP = KC + 8;  // LDS pitch (bf16 elements) of the X and B_vv tiles (80 bytes)

template <int O32, int WS, int WC>
struct CfgB {
  static constexpr int KS = 2 * WS;          // slices per workgroup (2 waves along slices)
  static constexpr int NT = 64 * WC;         // columns per workgroup (2 waves along columns)
  static constexpr int JB = O32 / 32;        // 32-row blocks per slice
  static constexpr bool OS_LDS = O32 <= 128; // B_oo^Q tile in LDS (else read from L2)
  static constexpr int OP = O32 + 4;         // LDS pitch of the B_oo tile (bf16)
  static constexpr size_t LDS =
      (size_t)(2 * KS * O32 * XP + NT * XP + (OS_LDS ? O32 * OP : 0)) * sizeof(__bf16);
};

__device__ __forceinline__ bf8 ld8(const __bf16 *p) { return *reinterpret_cast<const bf8 *>(p); }
__device__ __forceinline__ bf4 ld4(const __bf16 *p) { return *reinterpret_cast<const bf4 *>(p); }

__device__ __forceinline__ bf8 cat(bf4 a, bf4 b) {
  return bf8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

// copy 8 consecutive bf16 (16 bytes) from global to LDS, zero beyond `lim` elements
__device__ __forceinline__ void stage8(__bf16 *dst, const __bf16 *src, int lim, bool vec) {
  if (vec && lim >= 8) {
    *reinterpret_cast<us8 *>(dst) = *reinterpret_cast<const us8 *>(src);
  } else {
    const unsigned short *s = reinterpret_cast<const unsigned short *>(src);
    us8 val = us8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (t < lim) val[t] = s[t];
    *reinterpret_cast<us8 *>(dst) = val;
  }
}

__device__ __forceinline__ f16v zero16() {
  f16v z;
#pragma unroll
  for (int t = 0; t < 16; ++t) z[t] = 0.f;
  return z;
}

template <int O32, int WS, int WC>
__global__ __launch_bounds__(256, 1) void k_exchange_bf16(const __bf16 *__restrict__ Boo,
                                                          const __bf16 *__restrict__ Bvv,
                                                          const __bf16 *__restrict__ Xh,
                                                          const __bf16 *__restrict__ Xl, int o, int v, int nq, int ns,
                                                          int n_sg, int n_ct, int nsplit, float scale,
                                                          float *__restrict__ P) {
  using C = CfgB<O32, WS, WC>;
  constexpr int KS = C::KS, NT = C::NT, JB = C::JB, OP = C::OP;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsb[];
  __bf16 *Xhs = ldsb;                 // [KS*O32][XP]
  __bf16 *Xls = Xhs + KS * O32 * XP;  // [KS*O32][XP]
  __bf16 *Bs = Xls + KS * O32 * XP;   // [NT][XP]
  __bf16 *Os = Bs + NT * XP;          // [O32][OP] (only if OS_LDS)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, m = lane & 31;
  const int ws = wave >> 1, wc = wave & 1;
  const int bid = blockIdx.x;
  const int sg = bid % n_sg;
  const int ct = (bid / n_sg) % n_ct;
  const int sp = bid / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * KS, c_base = ct * NT;
  const bool vec = (v & 7) == 0;
  const bool ovec = (o & 3) == 0;

  f16v Kacc[WS][JB][WC];
#pragma unroll
  for (int a = 0; a < WS; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int c = 0; c < WC; ++c) Kacc[a][b][c] = zero16();

  for (int q = qa; q < qb; ++q) {
    const __bf16 *Oq = Boo + (size_t)q * o * o;
    if constexpr (C::OS_LDS) {
      __syncthreads();
      const unsigned short *src = reinterpret_cast<const unsigned short *>(Oq);
      unsigned short *dst = reinterpret_cast<unsigned short *>(Os);
      for (int e = tid; e < O32 * O32; e += 256) {
        const int i = e / O32, j = e - i * O32;
        dst[i * OP + j] = (i < o && j < o) ? src[(size_t)i * o + j] : (unsigned short)0;
      }
    }
    const __bf16 *Vq = Bvv + (size_t)q * v * v;

    f16v Wacc[WS][JB][WC];
#pragma unroll
    for (int a = 0; a < WS; ++a)
#pragma unroll
      for (int b = 0; b < JB; ++b)
#pragma unroll
        for (int c = 0; c < WC; ++c) Wacc[a][b][c] = zero16();

    for (int a0 = 0; a0 < v; a0 += KC) {
      __syncthreads();
      for (int e = tid; e < KS * O32 * (KC / 8); e += 256) {
        const int row = e / (KC / 8), k8 = (e - row * (KC / 8)) * 8;
        const int sl = s_base + row / O32, j = row % O32, a = a0 + k8;
        __bf16 *dh = &Xhs[row * XP + k8];
        __bf16 *dl = &Xls[row * XP + k8];
        if (sl < ns && j < o && a < v) {
          const size_t off = ((size_t)sl * o + j) * v + a;
          stage8(dh, Xh + off, v - a, vec);
          stage8(dl, Xl + off, v - a, vec);
        } else {
          *reinterpret_cast<us8 *>(dh) = us8{0, 0, 0, 0, 0, 0, 0, 0};
          *reinterpret_cast<us8 *>(dl) = us8{0, 0, 0, 0, 0, 0, 0, 0};
        }
      }
      for (int e = tid; e < NT * (KC / 8); e += 256) {
        const int cl = e / (KC / 8), k8 = (e - cl * (KC / 8)) * 8;
        const int cc = c_base + cl, a = a0 + k8;
        __bf16 *d = &Bs[cl * XP + k8];
        if (cc < v && a < v)
          stage8(d, Vq + (size_t)cc * v + a, v - a, vec);
        else
          *reinterpret_cast<us8 *>(d) = us8{0, 0, 0, 0, 0, 0, 0, 0};
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; kk += 16) {
        bf8 bf[WC];
#pragma unroll
        for (int cb = 0; cb < WC; ++cb) bf[cb] = ld8(&Bs[((wc * WC + cb) * 32 + m) * XP + kk + 8 * h]);
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb) {
            const int row = (ws * WS + si) * O32 + jb * 32 + m;
            const bf8 ah = ld8(&Xhs[row * XP + kk + 8 * h]);
            const bf8 al = ld8(&Xls[row * XP + kk + 8 * h]);
#pragma unroll
            for (int cb = 0; cb < WC; ++cb) {
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bf[cb], Wacc[si][jb][cb], 0, 0, 0);
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bf[cb], Wacc[si][jb][cb], 0, 0, 0);
            }
          }
      }
    }
    // K += B_oo^Q (W_hi + W_lo) over W blocks jb and halves u
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        bf8 wh[WS][WC], wl[WS][WC];
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int cb = 0; cb < WC; ++cb)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float w = Wacc[si][jb][cb][8 * u + e];
              const __bf16 hi = (__bf16)w;
              wh[si][cb][e] = hi;
              wl[si][cb][e] = (__bf16)(w - (float)hi);
            }
        const int j0 = jb * 32 + 16 * u + 4 * h;  // j of register 8u (and j0 + 8 of register 8u + 4)
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          const int i = ib * 32 + m;
          bf8 ar;
          if constexpr (C::OS_LDS) {
            ar = cat(ld4(&Os[i * OP + j0]), ld4(&Os[i * OP + j0 + 8]));
          } else {
            // B_oo^Q straight from L2: rows i < o, columns j < o (zero padding beyond)
            const unsigned short *src = reinterpret_cast<const unsigned short *>(Oq);
            us8 uu = us8{0, 0, 0, 0, 0, 0, 0, 0};
            if (i < o) {
#pragma unroll
              for (int p = 0; p < 2; ++p) {
                const int jj = j0 + 8 * p;
                if (ovec && jj + 3 < o) {
                  const us4 w4 = *reinterpret_cast<const us4 *>(src + (size_t)i * o + jj);
#pragma unroll
                  for (int t = 0; t < 4; ++t) uu[4 * p + t] = w4[t];
                } else {
#pragma unroll
                  for (int t = 0; t < 4; ++t) uu[4 * p + t] = (jj + t < o) ? src[(size_t)i * o + jj + t] : 0;
                }
              }
            }
            ar = __builtin_bit_cast(bf8, uu);
          }
#pragma unroll
          for (int si = 0; si < WS; ++si)
#pragma unroll
            for (int cb = 0; cb < WC; ++cb) {
              Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, wh[si][cb], Kacc[si][ib][cb], 0, 0, 0);
              Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, wl[si][cb], Kacc[si][ib][cb], 0, 0, 0);
            }
        }
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
        const int c = c_base + (wc * WC + cb) * 32 + m;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int i = ib * 32 + 8 * (t / 4) + 4 * h + (t % 4);
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[si][ib][cb][t];
        }
      }
  }
}

template <int O32, int WS, int WC>
hipError_t launch_xbf16(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o, int v,
                        int nq, int ns, int nsplit, float scale, float *P) {
  using C = CfgB<O32, WS, WC>;
  if (o > O32) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  dim3 grid(n_sg * n_ct * nsplit);
  hipLaunchKernelGGL((k_exchange_bf16<O32, WS, WC>), grid, dim3(256), C::LDS, s, static_cast<const __bf16 *>(Boo),
                     static_cast<const __bf16 *>(Bvv), static_cast<const __bf16 *>(X),
                     static_cast<const __bf16 *>(Xlo), o, v, nq, ns, n_sg, n_ct, nsplit, scale, P);
  return hipGetLastError();
}

template <int O32, int WS, int WC>
hipError_t prepare_xbf16() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_bf16<O32, WS, WC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgB<O32, WS, WC>::LDS);
}

#define XBF(O32, WS, WC)                                                                                     \
  ExchangeVariant {                                                                                          \
    RTTDA_PREC_MIXED_BF16, O32, CfgB<O32, WS, WC>::KS, CfgB<O32, WS, WC>::NT,                                \
        "bf16x2_o" #O32 "_ws" #WS "_wc" #WC, &launch_xbf16<O32, WS, WC>, CfgB<O32, WS, WC>::LDS,             \
        &prepare_xbf16<O32, WS, WC>                                                                          \
  }

const ExchangeVariant kBf16Variants[] = {
    XBF(32, 1, 2),  XBF(32, 2, 2),  XBF(32, 4, 1),  XBF(64, 1, 2),  XBF(64, 2, 1),  XBF(64, 3, 1),
    XBF(96, 1, 2),  XBF(96, 2, 1),  XBF(128, 1, 2), XBF(128, 1, 1), XBF(160, 1, 1), XBF(192, 1, 1),
    XBF(224, 1, 1), XBF(256, 1, 1),
};

}  // namespace

int exchange_bf16_variant_count() { return (int)(sizeof(kBf16Variants) / sizeof(kBf16Variants[0])); }
const ExchangeVariant *exchange_bf16_variant(int k) { return &kBf16Variants[k]; }

}  // namespace rttda
