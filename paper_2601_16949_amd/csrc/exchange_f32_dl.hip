// Exchange contraction, FP32, with direct global->LDS loads (gfx950 global_load_lds_dwordx4):
//   P[split][s][i][c] = scale * sum_{Q in split} (B_oo^Q X_s B_vv^Q)[i][c]
//
// Same two-product structure as exchange_f32.hip (W = X_s B_vv^Q in matrix-core accumulators,
// then K += B_oo^Q W with the accumulators used directly as the second operand).  What differs
// is the data path: the X and B_vv tiles of a 16-wide K chunk and the B_oo^Q tile travel from
// global memory straight into LDS, 16 bytes per lane, without passing through registers.  That
// frees the prefetch registers (higher occupancy) and lets the kernel keep two chunks in flight:
// chunk c+2 is requested into one of three LDS buffers while chunk c is multiplied, and an
// explicit vmcnt wait (counting this wave's outstanding load instructions) followed by a barrier
// makes chunk c+1 visible.  Every lane of every load instruction is active: lanes whose element
// lies outside the matrices read a 256-byte zero page, so the instruction counts behind the
// vmcnt waits are exact.
//
// LDS tiles are unpadded rows of 16 floats (four 16-byte chunks); the chunk position inside a
// row is XOR-swizzled with bits of the row index so that the 16-byte fragment reads of the MFMA
// operands (rows n = 0..15 at one logical chunk) spread over all banks.  B_oo^Q rows (o16 floats)
// are swizzled the same way with the low row bits.
#include <type_traits>

#include "common.h"

namespace rttda {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __attribute__((aligned(256))) float g_zero_page[64];  // 256 zero bytes (zero-initialised)

constexpr int KC = 16;  // K values per chunk: one 64-byte LDS row

// XOR swizzle of the four 16-byte chunks of a 64-byte row by row bits 1-2 (the 16x16 operand
// reads of this kernel: 16 rows at one logical chunk per lane group); measured conflict-free
// enough (0.4 conflict cycles per LDS instruction) where the variant with bit 3 mixed in, which
// suits the 32-row BF16 reads, gives 4
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }

template <int O16>
__device__ __forceinline__ int swz_o(int i) {
  return (O16 % 32 == 0) ? (i & 7) : (i & 3);
}

__device__ __forceinline__ void dma16(const float *src, float *lds_row0) {
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src), (lds_void *)lds_row0, 16, 0, 0);
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier for this kernel's LDS protocol: this wave's LDS reads are complete
// (lgkmcnt 0) and the loads that must be visible were waited for explicitly with wait_vm; the
// loads of later chunks stay in flight (a __syncthreads fence would drain them, vmcnt 0).  The
// asm statement's memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xF | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0) only
  asm volatile("s_barrier" ::: "memory");
}

template <int O16, int WS, int WC>
struct CfgD {
  static constexpr int KS = 2 * WS, NT = 32 * WC, JB = O16 / 16;
  static constexpr int XROWS = KS * O16;
  static constexpr int NXW = XROWS / 64;  // X load instructions per wave (16 rows each, 4 waves)
  static constexpr int NBW = NT / 64;     // B_vv load instructions per wave
  static constexpr int OCH = O16 * O16 / 4;                 // 16-byte chunks of the B_oo tile
  static constexpr int NOW = (OCH + 255) / 256;             // B_oo load instructions per wave
  static constexpr int XS = XROWS * KC, BS = NT * KC;       // floats per buffer
  static constexpr int OS = NOW * 256 * 4;                  // floats (padded to whole instructions)
  static constexpr size_t LDS = (size_t)(3 * (XS + BS) + OS) * sizeof(float);
  static_assert(XROWS % 64 == 0 && NT % 64 == 0, "tile must split into whole load instructions");
};

// PIPE: the operand fragments of chunk c+1 are read from LDS into a second register set right
// after the barrier that publishes chunk c+1, and the MFMAs of chunk c then run on fragments that
// are already in registers; without PIPE each chunk's fragments are read after the barrier and the
// MFMAs wait for them (all waves at the same moment, since the barrier aligns them).
// OCC: workgroups per CU the register budget is sized for (2, or 3 where three fit the LDS).
template <int O16, int WS, int WC, bool PIPE, int OCC>
__global__ __launch_bounds__(256, OCC) void k_exchange_f32_dl(const float *__restrict__ Boo,
                                                         const float *__restrict__ Bvv,
                                                         const float *__restrict__ X, int o, int v, int nq, int ns,
                                                         int n_sg, int n_ct, int nsplit, float scale,
                                                         float *__restrict__ P) {
  using C = CfgD<O16, WS, WC>;
  constexpr int JB = C::JB, NXW = C::NXW, NBW = C::NBW, NOW = C::NOW, NXB = NXW + NBW;
  extern __shared__ __attribute__((aligned(16))) float ldsd[];
  float *Xs0 = ldsd;                 // [3][XROWS][16]
  float *Bs0 = Xs0 + 3 * C::XS;      // [3][NT][16]
  float *Os = Bs0 + 3 * C::BS;       // [O16][O16] (+ padding)

  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  const int sg = lb % n_sg;
  const int ct = (lb / n_sg) % n_ct;
  const int sp = lb / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * C::KS, c_base = ct * C::NT;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int ws = wave >> 1, wc = wave & 1;
  const int nkc = (v + KC - 1) / KC;
  const int NC = (qb - qa) * nkc;
  int nvalid = 0;  // column blocks of this wave inside [0, v): WC, or fewer in the last tile
#pragma unroll
  for (int cb = 0; cb < WC; ++cb) nvalid += (c_base + (wc * WC + cb) * 16 < v) ? 1 : 0;
  // (nvalid is wave-uniform)
  // the zero page's address stays in registers for the whole kernel (re-deriving it inside the
  // loop puts a scalar memory load among the LDS reads, which forces full LDS waits)
  const float *zp = g_zero_page;
  asm volatile("" : "+s"(zp));

  // this lane's row / logical chunk inside each of its load instructions
  const int lrow = lane >> 2;  // 0..15 within a 16-row block

  auto issue = [&](int c) {
    const int q = qa + c / nkc, kc = c % nkc, a0 = kc * KC;
    float *Xs = Xs0 + (c % 3) * C::XS;
    float *Bs = Bs0 + (c % 3) * C::BS;
#pragma unroll
    for (int k = 0; k < NXW; ++k) {
      const int r0 = (wave * NXW + k) * 16, r = r0 + lrow;
      const int a = a0 + 4 * ((lane & 3) ^ swz(r));
      const int sl = s_base + r / O16, j = r % O16;
      const float *src = (sl < ns && j < o && a < v) ? X + ((size_t)sl * o + j) * v + a : zp;
      dma16(src, Xs + r0 * KC);
    }
    const float *Vq = Bvv + (size_t)q * v * v;
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int r0 = (wave * NBW + k) * 16, r = r0 + lrow;
      const int a = a0 + 4 * ((lane & 3) ^ swz(r));
      const int cc = c_base + r;
      const float *src = (cc < v && a < v) ? Vq + (size_t)cc * v + a : zp;  // row cc of symmetric B_vv
      dma16(src, Bs + r0 * KC);
    }
  };
  auto issue_os = [&](int q) {
    const float *Oq = Boo + (size_t)q * o * o;
#pragma unroll
    for (int k = 0; k < NOW; ++k) {
      const int e0 = (wave * NOW + k) * 64, e = e0 + lane;  // 16-byte chunk index in the tile
      const int i = e / (O16 / 4), p = e % (O16 / 4);
      const int jc = 4 * (p ^ swz_o<O16>(i));
      const float *src = (e < C::OCH && i < o && jc < o) ? Oq + (size_t)i * o + jc : zp;
      dma16(src, Os + e0 * 4);
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

  struct Frag {
    f4 bf[WC];
    f4 af[WS][JB];
  };
  auto read_frags = [&](int c, Frag &F) {
    const float *Xs = Xs0 + (c % 3) * C::XS;
    const float *Bs = Bs0 + (c % 3) * C::BS;
#pragma unroll
    for (int cb = 0; cb < WC; ++cb) {
      const int r = (wc * WC + cb) * 16 + n;
      F.bf[cb] = *reinterpret_cast<const f4 *>(&Bs[r * KC + 4 * (g ^ swz(r))]);
    }
#pragma unroll
    for (int si = 0; si < WS; ++si)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int r = (ws * WS + si) * O16 + jb * 16 + n;
        F.af[si][jb] = *reinterpret_cast<const f4 *>(&Xs[r * KC + 4 * (g ^ swz(r))]);
      }
  };
  // MFMAs of chunk c on fragments in registers, then (last chunk of a Q) K += B_oo^Q W
  auto mfma_n = [&](auto ncb_tag, int c, const Frag &F) {
    constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int si = 0; si < WS; ++si)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            Wacc[si][jb][cb] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(F.af[si][jb][t], F.bf[cb][t], Wacc[si][jb][cb], 0, 0, 0);
    if (c % nkc == nkc - 1) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        f4 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          const int i = ib * 16 + n;
          ar[ib] = *reinterpret_cast<const f4 *>(&Os[i * O16 + 4 * ((jb * 4 + g) ^ swz_o<O16>(i))]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ib = 0; ib < JB; ++ib)
#pragma unroll
            for (int si = 0; si < WS; ++si)
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
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
  auto mfma_chunk = [&](int c, const Frag &F) {
    if (nvalid == WC) {
      mfma_n(std::integral_constant<int, WC>{}, c, F);
    } else {
      if constexpr (WC >= 4) {
        if (nvalid == 3) mfma_n(std::integral_constant<int, 3>{}, c, F);
      }
      if constexpr (WC >= 3) {
        if (nvalid == 2) mfma_n(std::integral_constant<int, 2>{}, c, F);
      }
      if constexpr (WC >= 2) {
        if (nvalid == 1) mfma_n(std::integral_constant<int, 1>{}, c, F);
      }
    }
  };

  // NCB = number of this wave's column blocks inside [0, v) (wave-uniform; only the last column
  // tile has fewer than WC): the MFMA loops are specialised on it instead of testing each block
  auto compute_n = [&](auto ncb_tag, int c) {
    constexpr int NCB = decltype(ncb_tag)::value;
    const int kc = c % nkc;
    const float *Xs = Xs0 + (c % 3) * C::XS;
    const float *Bs = Bs0 + (c % 3) * C::BS;
    {
      f4 bf[WC];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int r = (wc * WC + cb) * 16 + n;
        bf[cb] = *reinterpret_cast<const f4 *>(&Bs[r * KC + 4 * (g ^ swz(r))]);
      }
      f4 af[WS][JB];
#pragma unroll
      for (int si = 0; si < WS; ++si)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int r = (ws * WS + si) * O16 + jb * 16 + n;
          af[si][jb] = *reinterpret_cast<const f4 *>(&Xs[r * KC + 4 * (g ^ swz(r))]);
        }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              Wacc[si][jb][cb] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(af[si][jb][t], bf[cb][t], Wacc[si][jb][cb], 0, 0, 0);
    }
    if (kc == nkc - 1) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        f4 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          const int i = ib * 16 + n;
          ar[ib] = *reinterpret_cast<const f4 *>(&Os[i * O16 + 4 * ((jb * 4 + g) ^ swz_o<O16>(i))]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ib = 0; ib < JB; ++ib)
#pragma unroll
            for (int si = 0; si < WS; ++si)
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
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
  // nvalid == 0: this wave's columns lie beyond v; it only takes part in loads and barriers
  auto compute = [&](int c) {
    static_assert(WC >= 1 && WC <= 4, "column blocks per wave");
    if (nvalid == WC) {
      compute_n(std::integral_constant<int, WC>{}, c);
    } else {
      if constexpr (WC >= 4) {
        if (nvalid == 3) compute_n(std::integral_constant<int, 3>{}, c);
      }
      if constexpr (WC >= 3) {
        if (nvalid == 2) compute_n(std::integral_constant<int, 2>{}, c);
      }
      if constexpr (WC >= 2) {
        if (nvalid == 1) compute_n(std::integral_constant<int, 1>{}, c);
      }
    }
  };

  if constexpr (PIPE) {
    Frag F0, F1;  // two named sets (a dynamically indexed pair would live in scratch memory)
    if (NC > 0) {
      issue_os(qa);
      issue(0);
      if (NC > 1) {
        issue(1);
        wait_vm<NXB>();  // B_oo^Q and chunk 0 have landed
      } else {
        wait_vm<0>();
      }
      lds_barrier();
      read_frags(0, F0);
    }
    auto step = [&](int c, const Frag &cur, Frag &nxt) {
      const bool more2 = c + 2 < NC;
      if (more2) issue(c + 2);  // its buffer's fragments were read before the previous barrier
      if (c + 1 < NC) {
        if (more2) wait_vm<NXB>(); else wait_vm<0>();  // chunk c+1 (and any B_oo^Q) has landed
        lds_barrier();  // also: every wave is past the MFMAs of chunk c-1 (and their B_oo reads)
        if (c > 0 && c % nkc == 0) issue_os(qa + c / nkc);  // needed at chunk c + nkc - 1 >= c + 2
        read_frags(c + 1, nxt);
        __builtin_amdgcn_sched_barrier(0);
      }
      mfma_chunk(c, cur);
    };
    for (int c = 0; c < NC; c += 2) {
      step(c, F0, F1);
      if (c + 1 < NC) step(c + 1, F1, F0);
    }
  } else {
  if (NC > 0) {
    issue_os(qa);
    issue(0);
    if (NC > 1) {
      issue(1);
      wait_vm<NXB>();  // B_oo^Q and chunk 0 have landed
    } else {
      wait_vm<0>();
    }
    lds_barrier();
  }
  for (int c = 0; c < NC; ++c) {
    const bool os_now = (c > 0) && (c % nkc == 0);  // the previous Q's K product is behind the last barrier
    const bool more = c + 2 < NC;
    if (os_now) issue_os(qa + c / nkc);
    if (more) issue(c + 2);
    compute(c);
    // chunk c+1 must have landed; younger loads (this iteration's) may stay in flight
    if (os_now) {
      if (more) wait_vm<NOW + NXB>(); else wait_vm<NOW>();
    } else {
      if (more) wait_vm<NXB>(); else wait_vm<0>();
    }
    lds_barrier();
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

template <int O16, int WS, int WC, bool PIPE, int OCC>
hipError_t launch_xf32dl(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *, int o, int v,
                         int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgD<O16, WS, WC>;
  if (o > O16 || (v & 3) != 0 || (o & 3) != 0 || v < 3 * KC) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_f32_dl<O16, WS, WC, PIPE, OCC>), grid, dim3(256), C::LDS, s, static_cast<const float *>(Boo),
                     static_cast<const float *>(Bvv), static_cast<const float *>(X), o, v, nq, ns, n_sg, n_ct, nsplit,
                     scale, P);
  return hipGetLastError();
}

template <int O16, int WS, int WC, bool PIPE, int OCC>
hipError_t prepare_xf32dl() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_f32_dl<O16, WS, WC, PIPE, OCC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgD<O16, WS, WC>::LDS);
}

#define XDL(O16, WS, WC, PIPE, OCC, NAME)                                                                \
  ExchangeVariant {                                                                                      \
    RTTDA_PREC_FP32, O16, CfgD<O16, WS, WC>::KS, CfgD<O16, WS, WC>::NT, NAME,                            \
        &launch_xf32dl<O16, WS, WC, PIPE, OCC>, CfgD<O16, WS, WC>::LDS,                                  \
        &prepare_xf32dl<O16, WS, WC, PIPE, OCC>, 3 * KC, 4, 4                                            \
  }
#define XDL2(O16, WS, WC)                                                                                \
  XDL(O16, WS, WC, false, 2, "f32dl_o" #O16 "_ws" #WS "_wc" #WC),                                        \
      XDL(O16, WS, WC, true, 2, "f32dlp_o" #O16 "_ws" #WS "_wc" #WC)

// (the register-pipelined form of the larger tiles would spill, so those have only the plain form;
// o64 ws1 wc2 already fits three workgroups per CU: 134 registers, 52 KiB of LDS)
const ExchangeVariant kF32DlVariants[] = {
    XDL2(32, 1, 2), XDL2(32, 2, 2), XDL2(48, 2, 2), XDL2(64, 1, 2),
    XDL(64, 2, 2, false, 2, "f32dl_o64_ws2_wc2"), XDL(64, 1, 4, false, 2, "f32dl_o64_ws1_wc4"),
    XDL(96, 1, 2, false, 2, "f32dl_o96_ws1_wc2"),
};

}  // namespace

int exchange_f32dl_variant_count() { return (int)(sizeof(kF32DlVariants) / sizeof(kF32DlVariants[0])); }
const ExchangeVariant *exchange_f32dl_variant(int k) { return &kF32DlVariants[k]; }

}  // namespace rttda
