// Exchange contraction, split BF16 precision, with direct global->LDS loads (gfx950
// global_load_lds): same arithmetic as exchange_bf16.hip (X = X_hi + X_lo, W = X B_vv^Q in FP32
// accumulators of v_mfma_f32_32x32x16_bf16, W split into hi/lo for K += B_oo^Q W), same data
// path as exchange_f32_dl.hip:
//  * the X_hi, X_lo and B_vv tiles of a 32-wide K chunk go from global memory straight into one
//    of three LDS buffers (16 bytes per lane); chunk c+2 is in flight while chunk c is multiplied;
//  * the B_oo^Q tile goes into LDS with the 4-byte form (rows of o bf16 need only o even);
//  * every lane of every load instruction is active (out-of-range lanes read a zero page) so the
//    explicit vmcnt waits count exactly; the workgroup barrier waits only for LDS reads;
//  * 16-byte chunks of the 64-byte LDS rows are XOR-swizzled with row bits so that the operand
//    reads (rows m = 0..31 at one logical chunk) spread over the banks.
#include <type_traits>

#include "common.h"

namespace rttda {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __attribute__((aligned(256))) unsigned int g_zero_page_b[64];  // 256 zero bytes

constexpr int KC = 32;  // bf16 per chunk row: 64 bytes = four 16-byte chunks

// XOR swizzle of the four 16-byte chunks of a 64-byte row: the 16-byte reads of 8 consecutive rows
// (one 128-byte bank sweep) and of 16 consecutive rows (one 256-byte sweep) at one logical chunk all
// land in distinct bank groups
__device__ __forceinline__ int swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }
__device__ __forceinline__ int swz_o(int i) { return i & 3; }

__device__ __forceinline__ void dma16(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)lds_base, 16, 0, 0);
}
__device__ __forceinline__ void dma4(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)lds_base, 4, 0, 0);
}

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// LDS reads of this wave are done; loads of later chunks stay in flight (see exchange_f32_dl.hip)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xF | (7 << 4) | (0 << 8) | (3 << 14));
  asm volatile("s_barrier" ::: "memory");
}

__device__ __forceinline__ f16v zero16() {
  f16v z;
#pragma unroll
  for (int t = 0; t < 16; ++t) z[t] = 0.f;
  return z;
}

// NW waves per workgroup: NWS rows of waves over the slices (2, or 1 for odd slice counts such
// as the split operator's R real slices), NW/NWS columns of waves over the B_vv columns; NB LDS
// buffers (chunks c+1 .. c+NB-2 are in flight while chunk c is multiplied)
template <int O32, int WS, int WC, int NW = 4, int NB = 3, int NWS = 2>
struct CfgBD {
  static constexpr int NWC = NW / NWS, NTH = 64 * NW;
  static constexpr int KS = NWS * WS, NT = 32 * WC * NWC, JB = O32 / 32;
  static constexpr int XROWS = KS * O32;
  static constexpr int NXW = XROWS / (16 * NW);  // per plane: 16-byte load instructions per wave
  static constexpr int NBW = NT / (16 * NW);
  static constexpr int ODW = O32 * O32 / 2;            // dwords of the B_oo tile
  static constexpr int NOW = (ODW + NTH - 1) / NTH;    // 4-byte load instructions per wave
  static constexpr int XS = XROWS * KC, BS = NT * KC;  // bf16 per buffer and plane
  static constexpr int OS = NOW * NTH * 2;             // bf16 (padded to whole instructions)
  static constexpr size_t LDS = (size_t)(NB * (2 * XS + BS) + OS) * 2;
  static_assert(NW == 4 || NW == 8, "four or eight waves");
  static_assert(NB == 3 || NB == 4, "three or four LDS buffers");
  static_assert(XROWS % (16 * NW) == 0 && NT % (16 * NW) == 0, "tile must split into whole load instructions");
};

// PIPE: half-chunk software pipeline.  The fragments of one 16-wide K step are read from LDS
// while the matrix cores work on the other step, and the barrier that publishes chunk c+1 sits
// between the two steps of chunk c, so every LDS read has a batch of MFMAs to hide behind; the
// loop is specialised once on the number of valid column blocks (no branches on it inside).
template <int O32, int WS, int WC, bool PIPE, int NW, int NB, int NWS>
__global__ __launch_bounds__(64 * NW, 8 / NW) void k_exchange_bf16_dl(const __bf16 *__restrict__ Boo,
                                                             const __bf16 *__restrict__ Bvv,
                                                             const __bf16 *__restrict__ Xh,
                                                             const __bf16 *__restrict__ Xl, int o, int v, int nq,
                                                             int ns, int n_sg, int n_ct, int nsplit, float scale,
                                                             float *__restrict__ P) {
  using C = CfgBD<O32, WS, WC, NW, NB, NWS>;
  constexpr int JB = C::JB, NXW = C::NXW, NBW = C::NBW, NOW = C::NOW, NXB = 2 * NXW + NBW;
  static_assert(PIPE || (NW == 4 && NB == 3), "the plain loop has four waves and three buffers");
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsbd[];
  __bf16 *Xh0 = ldsbd;               // [NB][XROWS][32]
  __bf16 *Xl0 = Xh0 + NB * C::XS;    // [NB][XROWS][32]
  __bf16 *Bs0 = Xl0 + NB * C::XS;    // [NB][NT][32]
  __bf16 *Os = Bs0 + NB * C::BS;     // [O32][O32] (+ padding)

  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  const int sg = lb % n_sg;
  const int ct = (lb / n_sg) % n_ct;
  const int sp = lb / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * C::KS, c_base = ct * C::NT;

  // (the pipelined loop holds the wave index in a scalar register, and with it the LDS destinations
  // of the loads; in the plain loop that moves more values into vector registers than fit)
  const int tid = threadIdx.x, lane = tid & 63, wave = PIPE ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  const int h = lane >> 5, m = lane & 31;
  const int ws = wave / C::NWC, wc = wave % C::NWC;
  const int nkc = (v + KC - 1) / KC;
  const int NC = (qb - qa) * nkc;
  int nvalid = 0;
#pragma unroll
  for (int cb = 0; cb < WC; ++cb) nvalid += (c_base + (wc * WC + cb) * 32 < v) ? 1 : 0;
  // (nvalid is wave-uniform)
  // the zero page's address stays in registers for the whole kernel (re-deriving it inside the
  // loop puts a scalar memory load among the LDS reads, which forces full LDS waits)
  const void *zp = g_zero_page_b;
  asm volatile("" : "+s"(zp));
  const int lrow = lane >> 2;

  // loads of the chunk (Q index q, K chunk kc) into LDS buffer buf; with live false (chunks past
  // the end, pipelined loop) the B_vv lanes read the zero page
  auto issue_at = [&](int q, int kc, int buf, bool live) {
    const int a0 = kc * KC;
#pragma unroll
    for (int k = 0; k < NXW; ++k) {
      const int r0 = (wave * NXW + k) * 16, r = r0 + lrow;
      const int a = a0 + 8 * ((lane & 3) ^ swz(r));
      const int sl = s_base + r / O32, j = r % O32;
      const bool ok = sl < ns && j < o && a < v;
      const size_t off = ((size_t)sl * o + j) * v + a;
      dma16(ok ? (const void *)(Xh + off) : zp, Xh0 + buf * C::XS + r0 * KC);
      dma16(ok ? (const void *)(Xl + off) : zp, Xl0 + buf * C::XS + r0 * KC);
    }
    const __bf16 *Vq = Bvv + (size_t)(live ? q : 0) * v * v;
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int r0 = (wave * NBW + k) * 16, r = r0 + lrow;
      const int a = a0 + 8 * ((lane & 3) ^ swz(r));
      const int cc = c_base + r;
      const bool ok = live && cc < v && a < v;
      dma16(ok ? (const void *)(Vq + (size_t)cc * v + a) : zp,
              Bs0 + buf * C::BS + r0 * KC);
    }
  };
  auto issue = [&](int c) { issue_at(qa + c / nkc, c % nkc, c % 3, true); };
  auto issue_os = [&](int q) {
    const __bf16 *Oq = Boo + (size_t)q * o * o;
    // (once per Q: the per-lane addresses are recomputed here rather than held in registers
    // through the loop, which the pipelined form has none to spare for)
    int ln = lane;
    if constexpr (PIPE) asm volatile("" : "+v"(ln));
#pragma unroll
    for (int k = 0; k < NOW; ++k) {
      const int d0 = (wave * NOW + k) * 64, d = d0 + ln;  // dword index in the tile
      const int i = d / (O32 / 2), w = d % (O32 / 2);
      const int jl = 2 * (4 * ((w >> 2) ^ swz_o(i)) + (w & 3));  // logical column (bf16)
      const bool ok = d < C::ODW && i < o && jl < o;
      dma4(ok ? (const void *)(Oq + (size_t)i * o + jl) : zp, Os + 2 * d0);
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

  // B_oo row i, logical columns j .. j+3 (one 8-byte half of a swizzled 16-byte chunk)
  auto os4 = [&](int i, int j) -> bf4 {
    const int ch = (j >> 3) ^ swz_o(i);
    return *reinterpret_cast<const bf4 *>(&Os[i * O32 + 8 * ch + (j & 7)]);
  };

  // K += B_oo^Q W for the Q whose last chunk was just multiplied (W split into hi + lo), then W = 0
  auto compute_k = [&](auto ncb_tag) {
    constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        bf8 wh[WS][WC], wl[WS][WC];
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float w = Wacc[si][jb][cb][8 * u + e];
              const __bf16 hi = (__bf16)w;
              wh[si][cb][e] = hi;
              wl[si][cb][e] = (__bf16)(w - (float)hi);
            }
        const int j0 = jb * 32 + 16 * u + 4 * h;
        bf8 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          const int i = ib * 32 + m;
          const bf4 lo4 = os4(i, j0), hi4 = os4(i, j0 + 8);
          ar[ib] = bf8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]};
        }
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int si = 0; si < WS; ++si)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ib], wh[si][cb], Kacc[si][ib][cb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int si = 0; si < WS; ++si)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              Kacc[si][ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ib], wl[si][cb], Kacc[si][ib][cb], 0, 0, 0);
      }
#pragma unroll
    for (int a = 0; a < WS; ++a)
#pragma unroll
      for (int b = 0; b < JB; ++b)
#pragma unroll
        for (int cc = 0; cc < WC; ++cc) Wacc[a][b][cc] = zero16();
  };
  auto compute_n = [&](auto ncb_tag, int c) {
    constexpr int NCB = decltype(ncb_tag)::value;
    const int kc = c % nkc, buf = c % 3;
    const __bf16 *Xhs = Xh0 + buf * C::XS;
    const __bf16 *Xls = Xl0 + buf * C::XS;
    const __bf16 *Bs = Bs0 + buf * C::BS;
    const int klim = v - kc * KC;
    // each K step's operand fragments are read into registers before its MFMAs (one LDS wait per
    // K step instead of one per fragment); the next step's reads overlap these MFMAs
#pragma unroll
    for (int u = 0; u < 2; ++u) {  // two MFMA K steps of 16 per chunk
      bf8 bf[WC], ah[WS][JB], al[WS][JB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int r = (wc * WC + cb) * 32 + m;
        bf[cb] = *reinterpret_cast<const bf8 *>(&Bs[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
      }
#pragma unroll
      for (int si = 0; si < WS; ++si)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int r = (ws * WS + si) * O32 + jb * 32 + m;
          const int co = r * KC + 8 * ((2 * u + h) ^ swz(r));
          ah[si][jb] = *reinterpret_cast<const bf8 *>(&Xhs[co]);
          al[si][jb] = *reinterpret_cast<const bf8 *>(&Xls[co]);
        }
      __builtin_amdgcn_sched_barrier(0);
      if (16 * u < klim) {
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[si][jb], bf[cb], Wacc[si][jb][cb], 0, 0, 0);
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
              Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[si][jb], bf[cb], Wacc[si][jb][cb], 0, 0, 0);
      }
    }
    if (kc == nkc - 1) compute_k(ncb_tag);
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
    struct Frag {
      bf8 b[WC], h[WS][JB], l[WS][JB];
    };
    // operand fragments of K step u (0 or 1) of chunk c
    auto read_frag = [&](auto ncb_tag, int buf, int u, Frag &F) {
      constexpr int NCB = decltype(ncb_tag)::value;
      const __bf16 *Xhs = Xh0 + buf * C::XS;
      const __bf16 *Xls = Xl0 + buf * C::XS;
      const __bf16 *Bs = Bs0 + buf * C::BS;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int r = (wc * WC + cb) * 32 + m;
        F.b[cb] = *reinterpret_cast<const bf8 *>(&Bs[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
      }
      if constexpr (NCB > 0) {
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb) {
            const int r = (ws * WS + si) * O32 + jb * 32 + m;
            const int co = r * KC + 8 * ((2 * u + h) ^ swz(r));
            F.h[si][jb] = *reinterpret_cast<const bf8 *>(&Xhs[co]);
            F.l[si][jb] = *reinterpret_cast<const bf8 *>(&Xls[co]);
          }
      }
    };
    // half of K step F: the X_hi products (part 0) or the X_lo products (part 1)
    auto mfma_w = [&](auto ncb_tag, const Frag &F, int part) {
      constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
      for (int si = 0; si < WS; ++si)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(part ? F.l[si][jb] : F.h[si][jb], F.b[cb],
                                                                       Wacc[si][jb][cb], 0, 0, 0);
    };
    // Per chunk c, after the barrier that publishes it: issue the loads of chunk c+NB-1 (into chunk
    // c-1's buffer), read K step 0's fragments (F0), run K step 1 of chunk c-1 (F1, read before the
    // barrier) and, at the end of a Q, its K product while they arrive, then the X_hi half of K
    // step 0, then read K step 1's fragments into F1 while the X_lo half runs.  Every LDS wait is
    // then a wait for all outstanding reads.  Chunks past the end are issued too (zero page), so
    // the loads need no branch; the B_oo^Q tile of the Q that starts at chunk s is loaded at chunk
    // s+1, after the barrier behind which every wave finished the previous Q's K product, ahead of
    // that chunk's own loads so that the per-chunk wait count stays the same.
    auto main_loop = [&](auto ncb_tag) {
      constexpr int NCB = decltype(ncb_tag)::value;
      Frag F0, F1;
#pragma unroll
      for (int cb = 0; cb < WC; ++cb) F1.b[cb] = bf8{};  // "K step 1 of chunk -1": adds zero
#pragma unroll
      for (int si = 0; si < WS; ++si)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) F1.h[si][jb] = F1.l[si][jb] = bf8{};
      if (NC == 0) return;
      issue_os(qa);
#pragma unroll
      for (int b = 0; b < NB - 1; ++b) issue_at(qa, b, b, true);  // NC >= nkc >= 3 >= NB - 1
      const bool tail1 = 16 < v - (nkc - 1) * KC;  // K step 1 of a Q's last chunk lies inside [0, v)
      int kcc = 0, qc = qa, buf = 0;               // chunk c's K chunk, Q index and LDS buffer
      for (int c = 0; c < NC; ++c) {
        wait_vm<(NB - 2) * NXB>();  // chunk c (and a B_oo^Q tile issued before it) has landed
        lds_barrier();   // publishes chunk c; every wave has read chunk c-1 and run the last K product
        if (kcc == 1 && c > 1) issue_os(qc);  // chunk c-1 opened Q qc; the K product before it is done
        {
          const bool wrap = kcc + NB - 1 >= nkc;  // chunk c+NB-1 (nkc >= 3: at most one Q ahead)
          issue_at(wrap ? qc + 1 : qc, wrap ? kcc + NB - 1 - nkc : kcc + NB - 1, buf == 0 ? NB - 1 : buf - 1,
                   c + NB - 1 < NC);
        }
        __builtin_amdgcn_sched_barrier(0);
        read_frag(ncb_tag, buf, 0, F0);
        __builtin_amdgcn_sched_barrier(0);
        if (c > 0 && (kcc != 0 || tail1)) {  // K step 1 of chunk c-1
          mfma_w(ncb_tag, F1, 0);
          mfma_w(ncb_tag, F1, 1);
        }
        if constexpr (NCB > 0) {
          if (c > 0 && kcc == 0) compute_k(ncb_tag);  // chunk c-1 closed its Q
        }
        __builtin_amdgcn_sched_barrier(0);
        mfma_w(ncb_tag, F0, 0);
        __builtin_amdgcn_sched_barrier(0);
        read_frag(ncb_tag, buf, 1, F1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_w(ncb_tag, F0, 1);
        if (++kcc == nkc) { kcc = 0; ++qc; }
        buf = buf == NB - 1 ? 0 : buf + 1;
      }
      if (tail1) {
        mfma_w(ncb_tag, F1, 0);
        mfma_w(ncb_tag, F1, 1);
      }
      if constexpr (NCB > 0) compute_k(ncb_tag);
      wait_vm<0>();  // no LDS write may still be in flight when the workgroup ends
    };
    if (nvalid == WC) {
      main_loop(std::integral_constant<int, WC>{});
    } else {
      if constexpr (WC >= 4) {
        if (nvalid == 3) main_loop(std::integral_constant<int, 3>{});
      }
      if constexpr (WC >= 3) {
        if (nvalid == 2) main_loop(std::integral_constant<int, 2>{});
      }
      if constexpr (WC >= 2) {
        if (nvalid == 1) main_loop(std::integral_constant<int, 1>{});
      }
      if (nvalid == 0) main_loop(std::integral_constant<int, 0>{});
    }
  } else {
  if (NC > 0) {
    issue_os(qa);
    issue(0);
    if (NC > 1) {
      issue(1);
      wait_vm<NXB>();
    } else {
      wait_vm<0>();
    }
    lds_barrier();
  }
  for (int c = 0; c < NC; ++c) {
    const bool os_now = (c > 0) && (c % nkc == 0);
    const bool more = c + 2 < NC;
    if (os_now) issue_os(qa + c / nkc);
    if (more) issue(c + 2);
    compute(c);
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
        const int c = c_base + (wc * WC + cb) * 32 + m;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int i = ib * 32 + 8 * (t / 4) + 4 * h + (t % 4);
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[si][ib][cb][t];
        }
      }
  }
}

template <int O32, int WS, int WC, bool PIPE, int NW, int NB, int NWS>
hipError_t launch_xbf16dl(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o,
                          int v, int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgBD<O32, WS, WC, NW, NB, NWS>;
  if (o > O32 || (v & 7) != 0 || (o & 1) != 0 || v < 3 * KC) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_bf16_dl<O32, WS, WC, PIPE, NW, NB, NWS>), grid, dim3(C::NTH), C::LDS, s,
                     static_cast<const __bf16 *>(Boo), static_cast<const __bf16 *>(Bvv),
                     static_cast<const __bf16 *>(X), static_cast<const __bf16 *>(Xlo), o, v, nq, ns, n_sg, n_ct,
                     nsplit, scale, P);
  return hipGetLastError();
}

template <int O32, int WS, int WC, bool PIPE, int NW, int NB, int NWS>
hipError_t prepare_xbf16dl() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_bf16_dl<O32, WS, WC, PIPE, NW, NB, NWS>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgBD<O32, WS, WC, NW, NB, NWS>::LDS);
}

#define XBDS(O32, WS, WC, PIPE, NW, NB, NWS, NAME)                                                          \
  ExchangeVariant {                                                                                         \
    RTTDA_PREC_MIXED_BF16, O32, CfgBD<O32, WS, WC, NW, NB, NWS>::KS, CfgBD<O32, WS, WC, NW, NB, NWS>::NT,    \
        NAME, &launch_xbf16dl<O32, WS, WC, PIPE, NW, NB, NWS>, CfgBD<O32, WS, WC, NW, NB, NWS>::LDS,        \
        &prepare_xbf16dl<O32, WS, WC, PIPE, NW, NB, NWS>, 3 * KC, 8, 2, 1, false, PIPE ? 2 : 1              \
  }
#define XBD(O32, WS, WC, PIPE, NW, NB, NAME) XBDS(O32, WS, WC, PIPE, NW, NB, 2, NAME)
#define XBD2(O32, WS, WC)                                                                                   \
  XBD(O32, WS, WC, false, 4, 3, "bf16x2dl_o" #O32 "_ws" #WS "_wc" #WC),                                     \
      XBD(O32, WS, WC, true, 4, 3, "bf16x2dlp_o" #O32 "_ws" #WS "_wc" #WC)

// ------------------------------------------------------------------------------------------------
// 64-wide K chunks with two LDS buffers (k64).  A chunk carries four MFMA K steps of 16, so the
// per-chunk barrier, wait and load issue fall on twice the matrix work of the 32-wide chunks above;
// chunk c+1 streams into the buffer chunk c-1 used while chunk c is multiplied.  Rows of 128 bytes
// hold eight 16-byte chunks, XOR-swizzled with (r >> 1) & 7 so that the 16 rows a quarter-wave
// reads at one logical chunk fall in 16 distinct bank groups.  The B_oo^Q tiles alternate between
// two LDS slots, so the next Q's tile loads while this Q's chunks run (it is issued at the Q's
// second chunk, once every wave has finished the previous Q's K product; hence v > 64).  Within a
// chunk the fragments of K step u+1 are read while the X_lo half of step u runs; every LDS wait is
// then a wait for all outstanding reads with matrix work queued ahead of it.  K steps that lie
// wholly past v in a Q's last chunk skip their matrix work.
// ------------------------------------------------------------------------------------------------
constexpr int KC64 = 64;

__device__ __forceinline__ int swz8(int r) { return (r >> 1) & 7; }

template <int O32, int WC, int NW, int NWS>
struct CfgK64 {
  static constexpr int NWC = NW / NWS, NTH = 64 * NW;
  static constexpr int KS = NWS, NT = 32 * WC * NWC, JB = O32 / 32;
  static constexpr int XROWS = KS * O32;
  static constexpr int NXW = XROWS / (8 * NW);  // per plane: 16-byte load instructions per wave (8 rows each)
  static constexpr int NBW = NT / (8 * NW);
  static constexpr int ODW = O32 * O32 / 2;             // dwords of a B_oo tile
  static constexpr int NOW = (ODW + NTH - 1) / NTH;     // 4-byte load instructions per wave
  static constexpr int XS = XROWS * KC64, BS = NT * KC64;  // bf16 per buffer and plane
  static constexpr int OS = NOW * NTH * 2;              // bf16 per B_oo slot (whole instructions)
  static constexpr size_t LDS = (size_t)(2 * (2 * XS + BS) + 2 * OS) * 2;
  static_assert(XROWS % (8 * NW) == 0 && NT % (8 * NW) == 0, "tile must split into whole load instructions");
  static_assert(LDS <= 160 * 1024, "LDS");
};

template <int O32, int WC, int NW, int NWS>
__global__ __launch_bounds__(64 * NW, 1) void k_exchange_bf16_k64(const __bf16 *__restrict__ Boo,
                                                                 const __bf16 *__restrict__ Bvv,
                                                                 const __bf16 *__restrict__ Xh,
                                                                 const __bf16 *__restrict__ Xl, int o, int v, int nq,
                                                                 int ns, int n_sg, int n_ct, int nsplit, float scale,
                                                                 float *__restrict__ P) {
  using C = CfgK64<O32, WC, NW, NWS>;
  constexpr int JB = C::JB, NXW = C::NXW, NBW = C::NBW, NOW = C::NOW;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsk[];
  __bf16 *Xh0 = ldsk;              // [2][XROWS][64]
  __bf16 *Xl0 = Xh0 + 2 * C::XS;   // [2][XROWS][64]
  __bf16 *Bs0 = Xl0 + 2 * C::XS;   // [2][NT][64]
  __bf16 *Os0 = Bs0 + 2 * C::BS;   // [2][O32][O32] (+ padding)

  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  const int sg = lb % n_sg;
  const int ct = (lb / n_sg) % n_ct;
  const int sp = lb / (n_sg * n_ct);
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * C::KS, c_base = ct * C::NT;

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = lane >> 5, m = lane & 31;
  const int ws = wave / C::NWC, wc = wave % C::NWC;
  const int nkc = (v + KC64 - 1) / KC64;
  const int klast = v - (nkc - 1) * KC64;  // valid K values in a Q's last chunk (1..64)
  const int NC = (qb - qa) * nkc;
  int nvalid = 0;
#pragma unroll
  for (int cb = 0; cb < WC; ++cb) nvalid += (c_base + (wc * WC + cb) * 32 < v) ? 1 : 0;
  const void *zp = g_zero_page_b;
  asm volatile("" : "+s"(zp));
  const int lrow = lane >> 3, lch = lane & 7;

  // loads of chunk (Q index q, K chunk kc) into LDS buffer buf; live false: B_vv lanes read the zero page
  auto issue_at = [&](int q, int kc, int buf, bool live) {
    const int a0 = kc * KC64;
#pragma unroll
    for (int k = 0; k < NXW; ++k) {
      const int r0 = (wave * NXW + k) * 8, r = r0 + lrow;
      const int a = a0 + 8 * (lch ^ swz8(r));
      const int sl = s_base + r / O32, j = r % O32;
      const bool ok = live && sl < ns && j < o && a < v;
      const size_t off = ((size_t)sl * o + j) * v + a;
      dma16(ok ? (const void *)(Xh + off) : zp, Xh0 + buf * C::XS + r0 * KC64);
      dma16(ok ? (const void *)(Xl + off) : zp, Xl0 + buf * C::XS + r0 * KC64);
    }
    const __bf16 *Vq = Bvv + (size_t)(live ? q : 0) * v * v;
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int r0 = (wave * NBW + k) * 8, r = r0 + lrow;
      const int a = a0 + 8 * (lch ^ swz8(r));
      const int cc = c_base + r;
      const bool ok = live && cc < v && a < v;
      dma16(ok ? (const void *)(Vq + (size_t)cc * v + a) : zp, Bs0 + buf * C::BS + r0 * KC64);
    }
  };
  auto issue_os = [&](int q, int slot) {
    const __bf16 *Oq = Boo + (size_t)q * o * o;
    int ln = lane;
    asm volatile("" : "+v"(ln));
#pragma unroll
    for (int k = 0; k < NOW; ++k) {
      const int d0 = (wave * NOW + k) * 64, d = d0 + ln;
      const int i = d / (O32 / 2), w = d % (O32 / 2);
      const int jl = 2 * (4 * ((w >> 2) ^ swz_o(i)) + (w & 3));
      const bool ok = d < C::ODW && i < o && jl < o;
      dma4(ok ? (const void *)(Oq + (size_t)i * o + jl) : zp, Os0 + slot * C::OS + 2 * d0);
    }
  };

  f16v Kacc[JB][WC], Wacc[JB][WC];
#pragma unroll
  for (int b = 0; b < JB; ++b)
#pragma unroll
    for (int c = 0; c < WC; ++c) {
      Kacc[b][c] = zero16();
      Wacc[b][c] = zero16();
    }

  auto compute_k = [&](auto ncb_tag, int slot) {
    constexpr int NCB = decltype(ncb_tag)::value;
    const __bf16 *Os = Os0 + slot * C::OS;
    auto os4 = [&](int i, int j) -> bf4 {
      const int ch = (j >> 3) ^ swz_o(i);
      return *reinterpret_cast<const bf4 *>(&Os[i * O32 + 8 * ch + (j & 7)]);
    };
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        bf8 wh[WC], wl[WC];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float w = Wacc[jb][cb][8 * u + e];
            const __bf16 hi = (__bf16)w;
            wh[cb][e] = hi;
            wl[cb][e] = (__bf16)(w - (float)hi);
          }
        const int j0 = jb * 32 + 16 * u + 4 * h;
        bf8 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib) {
          const int i = ib * 32 + m;
          const bf4 lo4 = os4(i, j0), hi4 = os4(i, j0 + 8);
          ar[ib] = bf8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]};
        }
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            Kacc[ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ib], wh[cb], Kacc[ib][cb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            Kacc[ib][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ar[ib], wl[cb], Kacc[ib][cb], 0, 0, 0);
      }
#pragma unroll
    for (int b = 0; b < JB; ++b)
#pragma unroll
      for (int cc = 0; cc < WC; ++cc) Wacc[b][cc] = zero16();
  };

  struct Frag {
    bf8 b[WC], h[JB], l[JB];
  };
  // operand fragments of K step u (0..3) of the chunk in buffer buf
  auto read_frag = [&](auto ncb_tag, int buf, int u, Frag &F) {
    constexpr int NCB = decltype(ncb_tag)::value;
    const __bf16 *Xhs = Xh0 + buf * C::XS;
    const __bf16 *Xls = Xl0 + buf * C::XS;
    const __bf16 *Bs = Bs0 + buf * C::BS;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int r = (wc * WC + cb) * 32 + m;
      F.b[cb] = *reinterpret_cast<const bf8 *>(&Bs[r * KC64 + 8 * ((2 * u + h) ^ swz8(r))]);
    }
    if constexpr (NCB > 0) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int r = ws * O32 + jb * 32 + m;
        const int co = r * KC64 + 8 * ((2 * u + h) ^ swz8(r));
        F.h[jb] = *reinterpret_cast<const bf8 *>(&Xhs[co]);
        F.l[jb] = *reinterpret_cast<const bf8 *>(&Xls[co]);
      }
    }
  };
  auto mfma_w = [&](auto ncb_tag, const Frag &F, int part) {
    constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        Wacc[jb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(part ? F.l[jb] : F.h[jb], F.b[cb], Wacc[jb][cb], 0,
                                                               0, 0);
  };
  // Chunk c: after the barrier that publishes it, issue chunk c+1's loads (into chunk c-1's buffer)
  // and, at the second chunk of a Q, the next Q's B_oo tile (into the slot the previous Q's K
  // product read before this barrier); read step 0, run step 3 of chunk c-1 (read before the
  // barrier) and, if chunk c-1 closed its Q, the K product; then steps 0..2 of chunk c, each step's
  // X_hi half, the next step's reads, its X_lo half.  Step 3's reads end the chunk.  (Lanes of K
  // values past v were filled from the zero page, so the reads need no branch.)
  auto main_loop = [&](auto ncb_tag) {
    constexpr int NCB = decltype(ncb_tag)::value;
    Frag F0, F1;
#pragma unroll
    for (int cb = 0; cb < WC; ++cb) F1.b[cb] = bf8{};
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) F1.h[jb] = F1.l[jb] = bf8{};
    if (NC == 0) return;
    issue_os(qa, 0);
    issue_at(qa, 0, 0, true);
    int kcc = 0, qc = qa, buf = 0;
    bool prev3 = false;  // step 3 of chunk c-1 lies inside [0, v)
    for (int c = 0; c < NC; ++c) {
      wait_vm<0>();   // chunk c (and every B_oo tile issued so far) has landed
      lds_barrier();  // publishes chunk c; chunk c-1's buffer and the older B_oo slot are free
      {
        const bool wrap = kcc + 1 == nkc;
        issue_at(wrap ? qc + 1 : qc, wrap ? 0 : kcc + 1, buf ^ 1, c + 1 < NC);
      }
      if (kcc == 1 && qc + 1 < qb) issue_os(qc + 1, (qc + 1 - qa) & 1);
      const bool last = kcc == nkc - 1;
      const bool s1 = !last || klast > 16, s2 = !last || klast > 32;
      __builtin_amdgcn_sched_barrier(0);
      read_frag(ncb_tag, buf, 0, F0);
      __builtin_amdgcn_sched_barrier(0);
      if (prev3) {  // step 3 of chunk c-1
        mfma_w(ncb_tag, F1, 0);
        mfma_w(ncb_tag, F1, 1);
      }
      if constexpr (NCB > 0) {
        if (c > 0 && kcc == 0) compute_k(ncb_tag, (qc - 1 - qa) & 1);  // chunk c-1 closed Q qc-1
      }
      __builtin_amdgcn_sched_barrier(0);
      mfma_w(ncb_tag, F0, 0);
      __builtin_amdgcn_sched_barrier(0);
      read_frag(ncb_tag, buf, 1, F1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_w(ncb_tag, F0, 1);
      __builtin_amdgcn_sched_barrier(0);
      if (s1) mfma_w(ncb_tag, F1, 0);
      __builtin_amdgcn_sched_barrier(0);
      read_frag(ncb_tag, buf, 2, F0);
      __builtin_amdgcn_sched_barrier(0);
      if (s1) mfma_w(ncb_tag, F1, 1);
      __builtin_amdgcn_sched_barrier(0);
      if (s2) mfma_w(ncb_tag, F0, 0);
      __builtin_amdgcn_sched_barrier(0);
      read_frag(ncb_tag, buf, 3, F1);
      __builtin_amdgcn_sched_barrier(0);
      if (s2) mfma_w(ncb_tag, F0, 1);
      prev3 = !last || klast > 48;
      if (++kcc == nkc) { kcc = 0; ++qc; }
      buf ^= 1;
    }
    if (prev3) {
      mfma_w(ncb_tag, F1, 0);
      mfma_w(ncb_tag, F1, 1);
    }
    if constexpr (NCB > 0) compute_k(ncb_tag, (qb - 1 - qa) & 1);
    wait_vm<0>();
  };
  if (nvalid == WC) {
    main_loop(std::integral_constant<int, WC>{});
  } else {
    if constexpr (WC >= 4) {
      if (nvalid == 3) main_loop(std::integral_constant<int, 3>{});
    }
    if constexpr (WC >= 3) {
      if (nvalid == 2) main_loop(std::integral_constant<int, 2>{});
    }
    if constexpr (WC >= 2) {
      if (nvalid == 1) main_loop(std::integral_constant<int, 1>{});
    }
    if (nvalid == 0) main_loop(std::integral_constant<int, 0>{});
  }

  float *Pp = P + (size_t)sp * ns * o * v;
  const int sl = s_base + ws;
  if (sl < ns) {
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
      for (int cb = 0; cb < WC; ++cb) {
        const int c = c_base + (wc * WC + cb) * 32 + m;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int i = ib * 32 + 8 * (t / 4) + 4 * h + (t % 4);
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[ib][cb][t];
        }
      }
  }
}

template <int O32, int WC, int NW, int NWS>
hipError_t launch_xbf16k64(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o,
                           int v, int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgK64<O32, WC, NW, NWS>;
  if (o > O32 || (v & 7) != 0 || (o & 1) != 0 || v <= KC64) return hipErrorInvalidValue;
  const int n_sg = (ns + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_bf16_k64<O32, WC, NW, NWS>), grid, dim3(C::NTH), C::LDS, s,
                     static_cast<const __bf16 *>(Boo), static_cast<const __bf16 *>(Bvv),
                     static_cast<const __bf16 *>(X), static_cast<const __bf16 *>(Xlo), o, v, nq, ns, n_sg, n_ct,
                     nsplit, scale, P);
  return hipGetLastError();
}

template <int O32, int WC, int NW, int NWS>
hipError_t prepare_xbf16k64() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_bf16_k64<O32, WC, NW, NWS>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgK64<O32, WC, NW, NWS>::LDS);
}

#define XBK64(O32, WC, NW, NWS, NAME)                                                                        \
  ExchangeVariant {                                                                                          \
    RTTDA_PREC_MIXED_BF16, O32, CfgK64<O32, WC, NW, NWS>::KS, CfgK64<O32, WC, NW, NWS>::NT, NAME,              \
        &launch_xbf16k64<O32, WC, NW, NWS>, CfgK64<O32, WC, NW, NWS>::LDS, &prepare_xbf16k64<O32, WC, NW, NWS>, \
        KC64 + 8, 8, 2, 1, false, 2                                                                          \
  }

const ExchangeVariant kBf16DlVariants[] = {
    XBD2(32, 1, 1), XBD2(32, 2, 1), XBD2(64, 1, 1), XBD2(64, 1, 2), XBD2(64, 2, 1),
    // eight waves (2 x 4) per workgroup, one workgroup per CU: the X tile of a chunk serves twice
    // the columns, and with four buffers three chunks are in flight
    XBD(64, 1, 2, true, 8, 3, "bf16x2dlp_o64_ws1_wc2_w8"), XBD(64, 1, 2, true, 8, 4, "bf16x2dlp_o64_ws1_wc2_w8b4"),
    XBD(32, 2, 2, true, 8, 4, "bf16x2dlp_o32_ws2_wc2_w8b4"),
    // one slice per workgroup, four columns of waves (odd slice counts: no idle slice row)
    XBDS(64, 1, 2, true, 4, 3, 1, "bf16x2dlp_o64_ws1_wc2_s1"), XBDS(64, 1, 1, true, 4, 3, 1, "bf16x2dlp_o64_ws1_wc1_s1"),
    // 64-wide K chunks, two buffers: eight waves (2 slices x 4 column groups) and four (one slice)
    XBK64(64, 2, 8, 2, "bf16x2k64_o64_wc2_w8"), XBK64(64, 1, 8, 2, "bf16x2k64_o64_wc1_w8"),
    XBK64(32, 2, 8, 2, "bf16x2k64_o32_wc2_w8"), XBK64(64, 2, 4, 1, "bf16x2k64_o64_wc2_w4s1"),
};

}  // namespace

int exchange_bf16dl_variant_count() { return (int)(sizeof(kBf16DlVariants) / sizeof(kBf16DlVariants[0])); }
const ExchangeVariant *exchange_bf16dl_variant(int k) { return &kBf16DlVariants[k]; }

}  // namespace rttda
