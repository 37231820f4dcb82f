// Exchange contraction on gfx950 matrix cores, FP32:
//   P[split][s][i][c] = scale * sum_{Q in split} (B_oo^Q X_s B_vv^Q)[i][c]
// for every slice s (one real plane of one right-hand side; slices stacked as rows).
//
// Order of the two products per Q: W = X_s B_vv^Q first (the large o x v x v product), then
// K_s += B_oo^Q W (o x o x v).  W never leaves the matrix-core accumulators: its 16x16 output
// blocks are fed straight back as the B operand of the second product, because the accumulator
// layout (row 4g + t of a block in register t of lane group g) equals the operand layout once
// the K index of that product is permuted the same way for both operands.  The same permutation
// lets every operand fragment come from one 16-byte LDS read (4 consecutive K values per lane).
//
// Pipelining: the (Q, K-chunk) sequence of a workgroup is one flat stream of chunks.  While the
// matrix cores work on chunk c from one LDS buffer, the global loads of chunk c+2 (X rows,
// B_vv^Q rows and, at a Q boundary, the next B_oo^Q) are in flight into one register set and
// chunk c+1 waits in the other; after the MFMAs chunk c+1 lands in the other LDS buffer, so one
// barrier per chunk suffices and each global load has two chunks of MFMA work to arrive.
// Block order: workgroups sharing a B_vv^Q tile (same Q range and columns, different slices)
// get consecutive logical ids on the same XCD, so the tile is fetched once into that XCD's L2.
//
// v_mfma_f32_16x16x4_f32 operand layout (lane l = 16 g + n):
//   A[m = n][k = g], B[k = g][n], D[m = 4 g + t][n] in accumulator register t.
#include "common.h"

namespace rttda {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int O16, int WS, int WC, int KC>
struct Cfg {
  static constexpr int KS = 2 * WS;   // slices per workgroup (2 waves along slices)
  static constexpr int NT = 32 * WC;  // columns per workgroup (2 waves along columns)
  static constexpr int JB = O16 / 16;
  static constexpr int XP = KC + 4;   // LDS row pitch (floats) of X and B_vv tiles
  static constexpr int OP = O16 + 4;  // LDS row pitch of the B_oo tile
  static constexpr int XT = KS * O16 * (KC / 4);  // float4 per X chunk
  static constexpr int BT = NT * (KC / 4);        // float4 per B_vv chunk
  static constexpr int XR = (XT + 255) / 256, BR = (BT + 255) / 256, OR = (O16 * O16 + 255) / 256;
  static constexpr bool OS_LDS = O16 <= 80;       // B_oo^Q in LDS (else fragments read from L2)
  static constexpr int XS = KS * O16 * XP, BS = NT * XP, OS = OS_LDS ? O16 * OP : 0;  // floats per buffer
  static constexpr size_t LDS = (size_t)(2 * (XS + BS) + 2 * OS) * sizeof(float);
};

template <int O16, int WS, int WC, int KC>
__global__ __launch_bounds__(256, 1) void k_exchange_f32(const float *__restrict__ Boo,
                                                         const float *__restrict__ Bvv,
                                                         const float *__restrict__ X, int o, int v, int nq, int ns,
                                                         int n_sg, int n_ct, int nsplit, float scale,
                                                         float *__restrict__ P) {
  using C = Cfg<O16, WS, WC, KC>;
  constexpr int KS = C::KS, NT = C::NT, JB = C::JB, XP = C::XP, OP = C::OP;
  extern __shared__ __attribute__((aligned(16))) float lds[];
  float *Xs0 = lds;
  float *Bs0 = Xs0 + 2 * C::XS;
  float *Os0 = Bs0 + 2 * C::BS;

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
  const int g = lane >> 4, n = lane & 15;
  const int ws = wave >> 1, wc = wave & 1;
  const bool vec = (v & 3) == 0;
  const int nkc = (v + KC - 1) / KC;
  const int NC = (qb - qa) * nkc;
  // column blocks entirely beyond v (last column tile) skip their MFMAs (wave-uniform)
  bool cvalid[WC];
#pragma unroll
  for (int cb = 0; cb < WC; ++cb) cvalid[cb] = c_base + (wc * WC + cb) * 16 < v;

  struct Regs {
    f4 x[C::XR], b[C::BR];
    float o[C::OS_LDS ? C::OR : 1];
  };
  Regs R0, R1;

  auto gload = [&](Regs &RR, int c) {
    f4 *xr = RR.x;
    f4 *br = RR.b;
    float *orr = RR.o;
    const int q = qa + c / nkc, kc = c % nkc, a0 = kc * KC;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + 256 * r;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (e < C::XT) {
        const int row = e / (KC / 4), k4 = (e - row * (KC / 4)) * 4;
        const int sl = s_base + row / O16, j = row % O16, a = a0 + k4;
        if (sl < ns && j < o && a < v) {
          const float *src = X + ((size_t)sl * o + j) * v + a;
          if (vec) {
            val = *reinterpret_cast<const f4 *>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) val[t] = (a + t < v) ? src[t] : 0.f;
          }
        }
      }
      xr[r] = val;
    }
    const float *Vq = Bvv + (size_t)q * v * v;
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + 256 * r;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (e < C::BT) {
        const int cl = e / (KC / 4), k4 = (e - cl * (KC / 4)) * 4;
        const int cc = c_base + cl, a = a0 + k4;
        if (cc < v && a < v) {
          const float *src = Vq + (size_t)cc * v + a;  // row cc of the symmetric B_vv^Q
          if (vec) {
            val = *reinterpret_cast<const f4 *>(src);
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) val[t] = (a + t < v) ? src[t] : 0.f;
          }
        }
      }
      br[r] = val;
    }
    if (C::OS_LDS && kc == 0) {
      const float *Oq = Boo + (size_t)q * o * o;
#pragma unroll
      for (int r = 0; r < C::OR; ++r) {
        const int e = tid + 256 * r;
        const int i = e / O16, j = e - (e / O16) * O16;
        orr[r] = (e < O16 * O16 && i < o && j < o) ? Oq[(size_t)i * o + j] : 0.f;
      }
    }
  };
  auto lstore = [&](const Regs &RR, int c) {
    const f4 *xr = RR.x;
    const f4 *br = RR.b;
    const float *orr = RR.o;
    const int kc = c % nkc, qi = c / nkc;
    float *Xs = Xs0 + (c & 1) * C::XS;
    float *Bs = Bs0 + (c & 1) * C::BS;
#pragma unroll
    for (int r = 0; r < C::XR; ++r) {
      const int e = tid + 256 * r;
      if (e < C::XT) {
        const int row = e / (KC / 4), k4 = (e - row * (KC / 4)) * 4;
        *reinterpret_cast<f4 *>(&Xs[row * XP + k4]) = xr[r];
      }
    }
#pragma unroll
    for (int r = 0; r < C::BR; ++r) {
      const int e = tid + 256 * r;
      if (e < C::BT) {
        const int cl = e / (KC / 4), k4 = (e - cl * (KC / 4)) * 4;
        *reinterpret_cast<f4 *>(&Bs[cl * XP + k4]) = br[r];
      }
    }
    if (C::OS_LDS && kc == 0) {
      float *Os = Os0 + (qi & 1) * C::OS;
#pragma unroll
      for (int r = 0; r < C::OR; ++r) {
        const int e = tid + 256 * r;
        if (e < O16 * O16) Os[(e / O16) * OP + (e % O16)] = orr[r];
      }
    }
  };

  f4 Kacc[WS][JB][WC], Wacc[WS][JB][WC];
#pragma unroll
  for (int a = 0; a < WS; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int c = 0; c < WC; ++c) {
        Kacc[a][b][c] = f4{0.f, 0.f, 0.f, 0.f};
        Wacc[a][b][c] = f4{0.f, 0.f, 0.f, 0.f};
      }

  auto compute = [&](int c) {
    const int kc = c % nkc, qi = c / nkc;
    const float *Xs = Xs0 + (c & 1) * C::XS;
    const float *Bs = Bs0 + (c & 1) * C::BS;
    const int klim = v - kc * KC;  // valid K values in this chunk (>= 1)
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      if (kk < klim) {
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
                if (cvalid[cb])
                  Wacc[si][jb][cb] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(af[si][jb][t], bf[cb][t], Wacc[si][jb][cb], 0, 0, 0);
      }
    }
    if (kc == nkc - 1) {
      // K += B_oo^Q W.  Step (jb, t): lane (g, n) supplies W[j = 16 jb + 4 g + t][c] (its own
      // accumulator register t) and B_oo[i][j] for the same j (B_oo symmetric: read row i).
      const float *Os = Os0 + (qi & 1) * C::OS;
      const float *Oq = Boo + (size_t)(qa + qi) * o * o;
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        f4 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          if constexpr (C::OS_LDS) {
            ar[ib] = *reinterpret_cast<const f4 *>(&Os[(ib * 16 + n) * OP + jb * 16 + 4 * g]);
          } else {
            const int i = ib * 16 + n, j0 = jb * 16 + 4 * g;
            f4 val = f4{0.f, 0.f, 0.f, 0.f};
            if (i < o) {
              if ((o & 3) == 0 && j0 + 3 < o) {
                val = *reinterpret_cast<const f4 *>(Oq + (size_t)i * o + j0);
              } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) val[t] = (j0 + t < o) ? Oq[(size_t)i * o + j0 + t] : 0.f;
              }
            }
            ar[ib] = val;
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ib = 0; ib < JB; ++ib)
#pragma unroll
            for (int si = 0; si < WS; ++si)
#pragma unroll
              for (int cb = 0; cb < WC; ++cb)
                if (cvalid[cb])
                  Kacc[si][ib][cb] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ib][t], Wacc[si][jb][cb][t], Kacc[si][ib][cb], 0, 0, 0);
      }
#pragma unroll
      for (int a = 0; a < WS; ++a)
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
          for (int cc = 0; cc < WC; ++cc) Wacc[a][b][cc] = f4{0.f, 0.f, 0.f, 0.f};
    }
  };

  // two register sets: chunk c + 2 is in flight from global memory while chunk c runs on the
  // matrix cores and chunk c + 1 waits in registers for its LDS buffer
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
        const int c = c_base + (wc * WC + cb) * 16 + n;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = ib * 16 + 4 * g + t;
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[si][ib][cb][t];
        }
      }
  }
}

template <int O16, int WS, int WC, int KC>
hipError_t launch_xf32(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void * /*Xlo*/, int o,
                       int v, int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = Cfg<O16, WS, WC, KC>;
  if (o > O16) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_f32<O16, WS, WC, KC>), grid, dim3(256), C::LDS, s, static_cast<const float *>(Boo),
                     static_cast<const float *>(Bvv), static_cast<const float *>(X), o, v, nq, ns, n_sg, n_ct, nsplit,
                     scale, P);
  return hipGetLastError();
}

template <int O16, int WS, int WC, int KC>
hipError_t prepare_xf32() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_f32<O16, WS, WC, KC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)Cfg<O16, WS, WC, KC>::LDS);
}

#define XF32(O16, WS, WC, KC)                                                                           \
  ExchangeVariant {                                                                                     \
    RTTDA_PREC_FP32, O16, Cfg<O16, WS, WC, KC>::KS, Cfg<O16, WS, WC, KC>::NT,                           \
        "f32_o" #O16 "_ws" #WS "_wc" #WC "_kc" #KC, &launch_xf32<O16, WS, WC, KC>,                      \
        Cfg<O16, WS, WC, KC>::LDS, &prepare_xf32<O16, WS, WC, KC>                                       \
  }

const ExchangeVariant kF32Variants[] = {
    XF32(16, 1, 1, 32), XF32(16, 2, 2, 32), XF32(16, 4, 2, 32), XF32(32, 2, 2, 32), XF32(32, 1, 2, 64),
    XF32(48, 1, 2, 32), XF32(48, 1, 2, 64), XF32(48, 2, 2, 32), XF32(48, 2, 2, 16), XF32(64, 1, 2, 32),
    XF32(64, 1, 2, 64), XF32(64, 1, 2, 16), XF32(64, 3, 1, 32), XF32(64, 1, 4, 32), XF32(64, 1, 1, 64),
    XF32(80, 1, 2, 32), XF32(96, 1, 2, 32), XF32(112, 1, 1, 16), XF32(128, 1, 2, 16), XF32(128, 1, 1, 32),
};

}  // namespace

int exchange_f32_variant_count() { return (int)(sizeof(kF32Variants) / sizeof(kF32Variants[0])); }
const ExchangeVariant *exchange_f32_variant(int k) { return &kF32Variants[k]; }

}  // namespace rttda
