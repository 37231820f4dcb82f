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

template <int O32, int WS, int WC, int KC>
struct CfgB {
  static constexpr int KS = 2 * WS;          // slices per workgroup (2 waves along slices)
  static constexpr int NT = 64 * WC;         // columns per workgroup (2 waves along columns)
  static constexpr int JB = O32 / 32;        // 32-row blocks per slice
  static constexpr int XP = KC + 8;          // LDS pitch (bf16) of X and B_vv tiles
  static constexpr bool OS_LDS = O32 <= 64;  // B_oo^Q tile in LDS (else fragments read from L2)
  static constexpr int OP = O32 + 4;         // LDS pitch of the B_oo tile (bf16)
  static constexpr int XT = KS * O32 * (KC / 8);  // 16-byte vectors per X plane chunk
  static constexpr int BT = NT * (KC / 8);        // 16-byte vectors per B_vv chunk
  static constexpr int XR = (XT + 255) / 256, BR = (BT + 255) / 256;
  static constexpr int OR = (O32 * O32 / 4 + 255) / 256;  // 8-byte vectors of B_oo per thread
  static constexpr int XS = KS * O32 * XP, BS = NT * XP, OS = OS_LDS ? O32 * OP : 0;  // bf16 per buffer
  static constexpr size_t LDS = (size_t)(2 * (2 * XS + BS) + 2 * OS) * sizeof(__bf16);
};

__device__ __forceinline__ bf8 ld8(const __bf16 *p) { return *reinterpret_cast<const bf8 *>(p); }
__device__ __forceinline__ bf4 ld4(const __bf16 *p) { return *reinterpret_cast<const bf4 *>(p); }

__device__ __forceinline__ bf8 cat(bf4 a, bf4 b) {
  return bf8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

// 8 consecutive bf16 from global, zero beyond `lim` elements
__device__ __forceinline__ us8 fetch8(const __bf16 *src, int lim, bool vec) {
  if (vec && lim >= 8) return *reinterpret_cast<const us8 *>(src);
  const unsigned short *s = reinterpret_cast<const unsigned short *>(src);
  us8 val = us8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < 8; ++t)
    if (t < lim) val[t] = s[t];
  return val;
}

__device__ __forceinline__ f16v zero16() {
  f16v z;
#pragma unroll
  for (int t = 0; t < 16; ++t) z[t] = 0.f;
  return z;
}

template <int O32, int WS, int WC, int KC>
__global__ __launch_bounds__(256, 1) void k_exchange_bf16(const __bf16 *__restrict__ Boo,
                                                          const __bf16 *__restrict__ Bvv,
                                                          const __bf16 *__restrict__ Xh,
                                                          const __bf16 *__restrict__ Xl, int o, int v, int nq, int ns,
                                                          int n_sg, int n_ct, int nsplit, float scale,
                                                          float *__restrict__ P) {
  using C = CfgB<O32, WS, WC, KC>;
  constexpr int KS = C::KS, NT = C::NT, JB = C::JB, XP = C::XP, OP = C::OP;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsb[];
  __bf16 *Xh0 = ldsb;                 // [2][KS*O32][XP]
  __bf16 *Xl0 = Xh0 + 2 * C::XS;      // [2][KS*O32][XP]
  __bf16 *Bs0 = Xl0 + 2 * C::XS;      // [2][NT][XP]
  __bf16 *Os0 = Bs0 + 2 * C::BS;      // [2][O32][OP] (only if OS_LDS)

  // XCD-aware logical block id (hardware deals workgroups to the 8 XCDs round robin)
  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  const int sg = lb % n_sg;
  const int ct = (lb / n_sg) % n_ct;
  const int sp = lb / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * KS, c_base = ct * NT;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, m = lane & 31;
  const int ws = wave >> 1, wc = wave & 1;
  const bool vec = (v & 7) == 0;
  const bool ovec = (o & 3) == 0;
  const int nkc = (v + KC - 1) / KC;
  const int NC = (qb - qa) * nkc;
  // column blocks entirely beyond v (last column tile) skip their MFMAs (wave-uniform)
  bool cvalid[WC];
#pragma unroll
  for (int cb = 0; cb < WC; ++cb) cvalid[cb] = c_base + (wc * WC + cb) * 32 < v;

  struct Regs {
    us8 xh[C::XR], xl[C::XR], b[C::BR];
    us4 o[C::OS_LDS ? C::OR : 1];
  };
  Regs R0, R1;

  auto gload = [&](Regs &RR, int c) {
    us8 *xhr = RR.xh;
    us8 *xlr = RR.xl;
    us8 *brr = RR.b;
    us4 *orr = RR.o;
    const int q = qa + c / nkc, kc = c % nkc, a0 = kc * KC;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + 256 * r;
      us8 vh = us8{0, 0, 0, 0, 0, 0, 0, 0}, vl = vh;
      if (e < C::XT) {
        const int row = e / (KC / 8), k8 = (e - row * (KC / 8)) * 8;
        const int sl = s_base + row / O32, j = row % O32, a = a0 + k8;
        if (sl < ns && j < o && a < v) {
          const size_t off = ((size_t)sl * o + j) * v + a;
          vh = fetch8(Xh + off, v - a, vec);
          vl = fetch8(Xl + off, v - a, vec);
        }
      }
      xhr[r] = vh;
      xlr[r] = vl;
    }
    const __bf16 *Vq = Bvv + (size_t)q * v * v;
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + 256 * r;
      us8 val = us8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < C::BT) {
        const int cl = e / (KC / 8), k8 = (e - cl * (KC / 8)) * 8;
        const int cc = c_base + cl, a = a0 + k8;
        if (cc < v && a < v) val = fetch8(Vq + (size_t)cc * v + a, v - a, vec);  // row cc of symmetric B_vv^Q
      }
      brr[r] = val;
    }
    if constexpr (C::OS_LDS) {
      if (kc == 0) {
        const unsigned short *Oq = reinterpret_cast<const unsigned short *>(Boo + (size_t)q * o * o);
#pragma unroll
        for (int r = 0; r < C::OR; ++r) {
          const int e = tid + 256 * r;  // 4-element group of the O32 x O32 tile
          const int i = (4 * e) / O32, j0 = (4 * e) % O32;
          us4 val = us4{0, 0, 0, 0};
          if (4 * e < O32 * O32 && i < o) {
#pragma unroll
            for (int t = 0; t < 4; ++t) val[t] = (j0 + t < o) ? Oq[(size_t)i * o + j0 + t] : (unsigned short)0;
          }
          orr[r] = val;
        }
      }
    }
  };
  auto lstore = [&](const Regs &RR, int c) {
    const us8 *xhr = RR.xh;
    const us8 *xlr = RR.xl;
    const us8 *brr = RR.b;
    const us4 *orr = RR.o;
    const int kc = c % nkc, qi = c / nkc;
    __bf16 *Xhs = Xh0 + (c & 1) * C::XS;
    __bf16 *Xls = Xl0 + (c & 1) * C::XS;
    __bf16 *Bs = Bs0 + (c & 1) * C::BS;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + 256 * r;
      if (e < C::XT) {
        const int row = e / (KC / 8), k8 = (e - row * (KC / 8)) * 8;
        *reinterpret_cast<us8 *>(&Xhs[row * XP + k8]) = xhr[r];
        *reinterpret_cast<us8 *>(&Xls[row * XP + k8]) = xlr[r];
      }
    }
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + 256 * r;
      if (e < C::BT) {
        const int cl = e / (KC / 8), k8 = (e - cl * (KC / 8)) * 8;
        *reinterpret_cast<us8 *>(&Bs[cl * XP + k8]) = brr[r];
      }
    }
    if constexpr (C::OS_LDS) {
      if (kc == 0) {
        __bf16 *Os = Os0 + (qi & 1) * C::OS;
#pragma unroll
        for (int r = 0; r < C::OR; ++r) {
          const int e = tid + 256 * r;
          if (4 * e < O32 * O32) *reinterpret_cast<us4 *>(&Os[((4 * e) / O32) * OP + (4 * e) % O32]) = orr[r];
        }
      }
    }
  };

  f16v Kacc[WS][JB][WC], Wacc[WS][JB][WC];
#pragma unroll
  for (int a = 0; a < WS; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int c = 0; c < WC; ++c) {
        Kacc[a][b][c] = zero16();
        Wacc[a][b][c] = zero16();
      }

  auto compute = [&](int c) {
    const int kc = c % nkc, qi = c / nkc;
    const __bf16 *Xhs = Xh0 + (c & 1) * C::XS;
    const __bf16 *Xls = Xl0 + (c & 1) * C::XS;
    const __bf16 *Bs = Bs0 + (c & 1) * C::BS;
    const int klim = v - kc * KC;  // valid K values in this chunk (>= 1)
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      if (kk < klim) {
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
              if (!cvalid[cb]) continue;
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bf[cb], Wacc[si][jb][cb], 0, 0, 0);
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bf[cb], Wacc[si][jb][cb], 0, 0, 0);
            }
          }
      }
    }
    if (kc == nkc - 1) {
      // K += B_oo^Q (W_hi + W_lo) over W blocks jb and halves u
      const __bf16 *Os = Os0 + (qi & 1) * C::OS;
      const unsigned short *Oq = reinterpret_cast<const unsigned short *>(Boo + (size_t)(qa + qi) * o * o);
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
              us8 uu = us8{0, 0, 0, 0, 0, 0, 0, 0};
              if (i < o) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                  const int jj = j0 + 8 * p;
                  if (ovec && jj + 3 < o) {
                    const us4 w4 = *reinterpret_cast<const us4 *>(Oq + (size_t)i * o + jj);
#pragma unroll
                    for (int t = 0; t < 4; ++t) uu[4 * p + t] = w4[t];
                  } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) uu[4 * p + t] = (jj + t < o) ? Oq[(size_t)i * o + jj + t] : 0;
                  }
                }
              }
              ar = __builtin_bit_cast(bf8, uu);
            }
#pragma unroll
            for (int si = 0; si < WS; ++si)
#pragma unroll
              for (int cb = 0; cb < WC; ++cb) {
                if (!cvalid[cb]) continue;
                Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, wh[si][cb], Kacc[si][ib][cb], 0, 0, 0);
                Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, wl[si][cb], Kacc[si][ib][cb], 0, 0, 0);
              }
          }
        }
#pragma unroll
      for (int a = 0; a < WS; ++a)
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
          for (int cc = 0; cc < WC; ++cc) Wacc[a][b][cc] = zero16();
    }
  };

  // two register sets: chunk c + 2 is in flight while chunk c runs on the matrix cores
  if (NC > 0) {
    gload(R0, 0);
    lstore(R0, 0);
    __syncthreads();
  }
  if (NC > 1) gload(R1, 1);
  for (int c = 0; c < NC; c += 2) {
    if (c + 2 < NC) gload(R0, c + 2);
    compute(c);
    if (c + 1 < NC) lstore(R1, c + 1);
    __syncthreads();
    if (c + 1 >= NC) break;
    if (c + 3 < NC) gload(R1, c + 3);
    compute(c + 1);
    if (c + 2 < NC) lstore(R0, c + 2);
    __syncthreads();
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

template <int O32, int WS, int WC, int KC>
hipError_t launch_xbf16(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o, int v,
                        int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgB<O32, WS, WC, KC>;
  if (o > O32) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_bf16<O32, WS, WC, KC>), grid, dim3(256), C::LDS, s, static_cast<const __bf16 *>(Boo),
                     static_cast<const __bf16 *>(Bvv), static_cast<const __bf16 *>(X),
                     static_cast<const __bf16 *>(Xlo), o, v, nq, ns, n_sg, n_ct, nsplit, scale, P);
  return hipGetLastError();
}

template <int O32, int WS, int WC, int KC>
hipError_t prepare_xbf16() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_bf16<O32, WS, WC, KC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgB<O32, WS, WC, KC>::LDS);
}

// ------------------------------------------------------------------------------------------------
// Large o: W handed through LDS.  One slice per workgroup, NW waves; the (32-row, 32-column)
// blocks of W and of K are dealt to the waves round robin.  Per Q, W = X B_vv^Q is accumulated
// as above, split into BF16 hi/lo planes and written to LDS as Ws[c][j] (j contiguous), and after
// a barrier each wave forms its K blocks from B_oo^Q (read straight from L2) and Ws.  The next
// Q's chunk barriers separate these LDS reads from the next writes of Ws.
// ------------------------------------------------------------------------------------------------
template <int O32, int NT, int NW, int KC>
struct CfgW {
  static constexpr int JB = O32 / 32, CB = NT / 32, NB = JB * CB;
  static constexpr int WB = (NB + NW - 1) / NW;   // blocks per wave
  static constexpr int NTH = 64 * NW;
  static constexpr int XP = KC + 8;
  static constexpr int WP = O32 + 8;              // LDS pitch of Ws rows (bf16)
  static constexpr int XT = O32 * (KC / 8), BT = NT * (KC / 8);
  static constexpr int XR = (XT + NTH - 1) / NTH, BR = (BT + NTH - 1) / NTH;
  static constexpr int XS = O32 * XP, BS = NT * XP, WS_ = NT * WP;
  static constexpr size_t LDS = (size_t)(2 * (2 * XS + BS) + 2 * WS_) * sizeof(__bf16);
};

template <int O32, int NT, int NW, int KC>
__global__ __launch_bounds__(64 * NW, 1) void k_exchange_bf16w(const __bf16 *__restrict__ Boo,
                                                               const __bf16 *__restrict__ Bvv,
                                                               const __bf16 *__restrict__ Xh,
                                                               const __bf16 *__restrict__ Xl, int o, int v, int nq,
                                                               int ns, int n_sg, int n_ct, int nsplit, float scale,
                                                               float *__restrict__ P) {
  using C = CfgW<O32, NT, NW, KC>;
  constexpr int CB = C::CB, NB = C::NB, WB = C::WB, XP = C::XP, WP = C::WP, NTH = C::NTH;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsw[];
  __bf16 *Xh0 = ldsw;                 // [2][O32][XP]
  __bf16 *Xl0 = Xh0 + 2 * C::XS;      // [2][O32][XP]
  __bf16 *Bs0 = Xl0 + 2 * C::XS;      // [2][NT][XP]
  __bf16 *Wh = Bs0 + 2 * C::BS;       // [NT][WP]
  __bf16 *Wl = Wh + C::WS_;           // [NT][WP]

  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  const int sl = lb % n_sg;  // one slice per workgroup
  const int ct = (lb / n_sg) % n_ct;
  const int sp = lb / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int c_base = ct * NT;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, m = lane & 31;
  const bool vec = (v & 7) == 0;
  const bool ovec = (o & 3) == 0;
  const int nkc = (v + KC - 1) / KC;
  const int NC = (qb - qa) * nkc;

  struct Regs {
    us8 xh[C::XR], xl[C::XR], b[C::BR];
  };
  Regs R0, R1;
  auto gload = [&](Regs &RR, int c) {
    const int q = qa + c / nkc, kc = c % nkc, a0 = kc * KC;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + NTH * r;
      us8 vh = us8{0, 0, 0, 0, 0, 0, 0, 0}, vl = vh;
      if (e < C::XT) {
        const int j = e / (KC / 8), k8 = (e - j * (KC / 8)) * 8, a = a0 + k8;
        if (j < o && a < v) {
          const size_t off = ((size_t)sl * o + j) * v + a;
          vh = fetch8(Xh + off, v - a, vec);
          vl = fetch8(Xl + off, v - a, vec);
        }
      }
      RR.xh[r] = vh;
      RR.xl[r] = vl;
    }
    const __bf16 *Vq = Bvv + (size_t)q * v * v;
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + NTH * r;
      us8 val = us8{0, 0, 0, 0, 0, 0, 0, 0};
      if (e < C::BT) {
        const int cl = e / (KC / 8), k8 = (e - cl * (KC / 8)) * 8;
        const int cc = c_base + cl, a = a0 + k8;
        if (cc < v && a < v) val = fetch8(Vq + (size_t)cc * v + a, v - a, vec);
      }
      RR.b[r] = val;
    }
  };
  auto lstore = [&](const Regs &RR, int c) {
    __bf16 *Xhs = Xh0 + (c & 1) * C::XS;
    __bf16 *Xls = Xl0 + (c & 1) * C::XS;
    __bf16 *Bs = Bs0 + (c & 1) * C::BS;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + NTH * r;
      if (e < C::XT) {
        const int j = e / (KC / 8), k8 = (e - j * (KC / 8)) * 8;
        *reinterpret_cast<us8 *>(&Xhs[j * XP + k8]) = RR.xh[r];
        *reinterpret_cast<us8 *>(&Xls[j * XP + k8]) = RR.xl[r];
      }
    }
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + NTH * r;
      if (e < C::BT) {
        const int cl = e / (KC / 8), k8 = (e - cl * (KC / 8)) * 8;
        *reinterpret_cast<us8 *>(&Bs[cl * XP + k8]) = RR.b[r];
      }
    }
  };

  f16v Kacc[WB], Wacc[WB];
#pragma unroll
  for (int b = 0; b < WB; ++b) {
    Kacc[b] = zero16();
    Wacc[b] = zero16();
  }

  auto compute = [&](int c) {
    const int kc = c % nkc, qi = c / nkc;
    const __bf16 *Xhs = Xh0 + (c & 1) * C::XS;
    const __bf16 *Xls = Xl0 + (c & 1) * C::XS;
    const __bf16 *Bs = Bs0 + (c & 1) * C::BS;
    const int klim = v - kc * KC;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      if (kk < klim) {
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          const int blk = wave + NW * b;
          if (blk < NB && c_base + (blk % CB) * 32 < v) {
            const int jb = blk / CB, cb = blk % CB;
            const bf8 bf = ld8(&Bs[(cb * 32 + m) * XP + kk + 8 * h]);
            const bf8 ah = ld8(&Xhs[(jb * 32 + m) * XP + kk + 8 * h]);
            const bf8 al = ld8(&Xls[(jb * 32 + m) * XP + kk + 8 * h]);
            Wacc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bf, Wacc[b], 0, 0, 0);
            Wacc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bf, Wacc[b], 0, 0, 0);
          }
        }
      }
    }
    if (kc == nkc - 1) {
      // W (hi/lo) to LDS as Ws[c][j]: register t of lane (h, n) holds W[32 jb + 8 p + 4 h + r][32 cb + n]
#pragma unroll
      for (int b = 0; b < WB; ++b) {
        const int blk = wave + NW * b;
        if (blk < NB) {
          const int jb = blk / CB, cb = blk % CB;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            bf4 hv, lv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float w = Wacc[b][4 * p + r];
              const __bf16 hi = (__bf16)w;
              hv[r] = hi;
              lv[r] = (__bf16)(w - (float)hi);
            }
            const int off = (cb * 32 + m) * WP + jb * 32 + 8 * p + 4 * h;
            *reinterpret_cast<bf4 *>(&Wh[off]) = hv;
            *reinterpret_cast<bf4 *>(&Wl[off]) = lv;
          }
          Wacc[b] = zero16();
        }
      }
      __syncthreads();
      const unsigned short *Oq = reinterpret_cast<const unsigned short *>(Boo + (size_t)(qa + qi) * o * o);
#pragma unroll
      for (int b = 0; b < WB; ++b) {
        const int blk = wave + NW * b;
        if (blk < NB && c_base + (blk % CB) * 32 < v) {
          const int ib = blk / CB, cb = blk % CB;
          const int i = ib * 32 + m;
#pragma unroll 4
          for (int j0 = 0; j0 < O32; j0 += 16) {
            const int jj = j0 + 8 * h;
            us8 uu = us8{0, 0, 0, 0, 0, 0, 0, 0};
            if (i < o) {
              if (ovec && jj + 7 < o) {
                const us4 w0 = *reinterpret_cast<const us4 *>(Oq + (size_t)i * o + jj);
                const us4 w1 = *reinterpret_cast<const us4 *>(Oq + (size_t)i * o + jj + 4);
                uu = us8{w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
              } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) uu[t] = (jj + t < o) ? Oq[(size_t)i * o + jj + t] : 0;
              }
            }
            const bf8 ar = __builtin_bit_cast(bf8, uu);
            const bf8 bh = ld8(&Wh[(cb * 32 + m) * WP + jj]);
            const bf8 bl = ld8(&Wl[(cb * 32 + m) * WP + jj]);
            Kacc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bh, Kacc[b], 0, 0, 0);
            Kacc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar, bl, Kacc[b], 0, 0, 0);
          }
        }
      }
    }
  };

  if (NC > 0) {
    gload(R0, 0);
    lstore(R0, 0);
    __syncthreads();
  }
  if (NC > 1) gload(R1, 1);
  for (int c = 0; c < NC; c += 2) {
    if (c + 2 < NC) gload(R0, c + 2);
    compute(c);
    if (c + 1 < NC) lstore(R1, c + 1);
    __syncthreads();
    if (c + 1 >= NC) break;
    if (c + 3 < NC) gload(R1, c + 3);
    compute(c + 1);
    if (c + 2 < NC) lstore(R0, c + 2);
    __syncthreads();
  }

  float *Pp = P + (size_t)sp * ns * o * v;
#pragma unroll
  for (int b = 0; b < WB; ++b) {
    const int blk = wave + NW * b;
    if (blk < NB) {
      const int ib = blk / CB, cb = blk % CB;
      const int c = c_base + cb * 32 + m;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int i = ib * 32 + 8 * (t / 4) + 4 * h + (t % 4);
        if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[b][t];
      }
    }
  }
}

template <int O32, int NT, int NW, int KC>
hipError_t launch_xbf16w(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o,
                         int v, int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgW<O32, NT, NW, KC>;
  if (o > O32) return hipErrorInvalidValue;
  const int n_sg = ns, n_ct = (v + NT - 1) / NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_bf16w<O32, NT, NW, KC>), grid, dim3(C::NTH), C::LDS, s,
                     static_cast<const __bf16 *>(Boo), static_cast<const __bf16 *>(Bvv),
                     static_cast<const __bf16 *>(X), static_cast<const __bf16 *>(Xlo), o, v, nq, ns, n_sg, n_ct, nsplit,
                     scale, P);
  return hipGetLastError();
}

template <int O32, int NT, int NW, int KC>
hipError_t prepare_xbf16w() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_bf16w<O32, NT, NW, KC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgW<O32, NT, NW, KC>::LDS);
}

#define XBW(O32, NT, NW, KC)                                                                              \
  ExchangeVariant {                                                                                       \
    RTTDA_PREC_MIXED_BF16, O32, 1, NT, "bf16x2w_o" #O32 "_nt" #NT "_nw" #NW "_kc" #KC,                    \
        &launch_xbf16w<O32, NT, NW, KC>, CfgW<O32, NT, NW, KC>::LDS, &prepare_xbf16w<O32, NT, NW, KC>     \
  }

#define XBF(O32, WS, WC, KC)                                                                             \
  ExchangeVariant {                                                                                      \
    RTTDA_PREC_MIXED_BF16, O32, CfgB<O32, WS, WC, KC>::KS, CfgB<O32, WS, WC, KC>::NT,                    \
        "bf16x2_o" #O32 "_ws" #WS "_wc" #WC "_kc" #KC, &launch_xbf16<O32, WS, WC, KC>,                   \
        CfgB<O32, WS, WC, KC>::LDS, &prepare_xbf16<O32, WS, WC, KC>                                      \
  }

const ExchangeVariant kBf16Variants[] = {
    XBF(32, 1, 2, 32), XBF(32, 2, 2, 32), XBF(32, 4, 1, 32), XBF(64, 1, 2, 32), XBF(64, 2, 1, 32),
    XBF(64, 3, 1, 32), XBF(96, 1, 1, 32), XBF(128, 1, 1, 32), XBF(160, 1, 1, 16),
    XBW(96, 64, 4, 32),  XBW(128, 64, 4, 32), XBW(128, 128, 8, 16), XBW(160, 64, 4, 32), XBW(160, 128, 8, 16),
    XBW(192, 64, 4, 32), XBW(192, 128, 8, 16), XBW(224, 64, 8, 16), XBW(256, 64, 4, 16),
    XBW(256, 64, 8, 16),
};

}  // namespace

int exchange_bf16_variant_count() { return (int)(sizeof(kBf16Variants) / sizeof(kBf16Variants[0])); }
const ExchangeVariant *exchange_bf16_variant(int k) { return &kBf16Variants[k]; }

}  // namespace rttda
