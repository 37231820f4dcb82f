// Exchange contraction for large o in split BF16 precision, as two batched GEMMs per chunk of Q
// instead of one fused kernel (the fused kernels keep W = X B_vv^Q on chip, which forces a
// workgroup tile of one slice's rows and re-reads all of X for every (Q, column tile); at large o
// that re-read traffic, not the matrix cores, sets the time):
//
//   (A) W^Q = X B_vv^Q for all stacked rows r = (slice, i) of X at once, with X = X_hi + X_lo and
//       FP32 accumulation on v_mfma_f32_32x32x16_bf16; the workgroup tile is 256 virtual columns x
//       256 rows, and the result is stored transposed, W^T[Q][c][r], as BF16 hi and lo planes.
//   (B) P[ks][s] (+)= scale * sum_{Q in split ks} B_oo^Q W_s^Q with W = W_hi + W_lo: a GEMM whose
//       reduction index runs over (Q, j); the slab of split ks is stored by the first chunk and
//       read-modified-written (same thread, fixed order) by later chunks.
//
// The exchange term is the c_x sum_Q B^Q_ij B^Q_ab part of the DF hybrid A (section "Real-Time
// TDA", the A matrix elements with the exact-exchange fraction c_x).  Both kernels stage operand
// tiles with gfx950 global_load_lds (16 bytes per lane) into three XOR-swizzled LDS buffers; loads
// of chunk c+2 are in flight while chunk c is multiplied; waits count vmcnt explicitly and the
// barrier drains only LDS reads.  Needs o % 8 == 0 and v % 8 == 0 (16-byte rows).
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace rttda {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

__device__ __attribute__((aligned(256))) unsigned int g_zero_page_g[64];  // 256 zero bytes

constexpr int KC = 32;  // bf16 per chunk row: 64 bytes = four 16-byte chunks

// XOR swizzle of the four 16-byte chunks of a 64-byte row: the 16-byte reads of 8 consecutive rows
// (one 128-byte bank sweep) and of 16 consecutive rows (one 256-byte sweep) at one logical chunk all
// land in distinct bank groups
__device__ __forceinline__ int swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }

__device__ __forceinline__ void dma16(const void *src, void *lds_base) {
  __builtin_amdgcn_global_load_lds(src, (lds_void *)lds_base, 16, 0, 0);
}

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

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

// logical workgroup id: consecutive ids on one XCD (hardware deals workgroups round robin)
__device__ __forceinline__ int xcd_local_id() {
  const int per_xcd = (int)gridDim.x / 8;
  return (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
}

// ---------------------------------------------------------------------------------------------
// (A) W^T[qq][c][r] = sum_b B_vv^(q0+qq)[c][b] X[r][b]      (B_vv symmetric: row c = column c)
// Waves: NWC along c x NWR along r; each wave CB x RB blocks of 32 x 32.
// ---------------------------------------------------------------------------------------------
template <int NWC, int NWR, int CB, int RB>
struct CfgA {
  static constexpr int NW = NWC * NWR, NT = 64 * NW;
  static constexpr int TC = NWC * CB * 32, TR = NWR * RB * 32;
  static constexpr int NA = TC / (16 * NW), NB = TR / (16 * NW);  // 16-byte loads per wave and chunk
  static constexpr int AS = TC * KC, BS = TR * KC;                 // bf16 per buffer (B: per plane)
  static constexpr size_t LDS = (size_t)3 * (AS + 2 * BS) * 2;
  static constexpr int NL = NA + 2 * NB;  // load instructions per wave and chunk
  static_assert(TC % (16 * NW) == 0 && TR % (16 * NW) == 0, "tiles split into whole load instructions");
  static_assert(LDS <= 160 * 1024, "LDS");
};

template <int NWC, int NWR, int CB, int RB, bool RT_MAJOR>
__global__ __launch_bounds__(64 * NWC * NWR, 1) void k_xgemm_w(const __bf16 *__restrict__ Bvv,
                                                               const __bf16 *__restrict__ Xh,
                                                               const __bf16 *__restrict__ Xl, int v, int M, int q0,
                                                               int nqc, int n_ct, int n_rt, __bf16 *__restrict__ Wh,
                                                               __bf16 *__restrict__ Wl) {
  using C = CfgA<NWC, NWR, CB, RB>;
  constexpr int NA = C::NA, NB = C::NB, NL = C::NL;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsa[];
  __bf16 *As0 = ldsa;              // [3][TC][32]  B_vv rows
  __bf16 *Xh0 = As0 + 3 * C::AS;   // [3][TR][32]
  __bf16 *Xl0 = Xh0 + 3 * C::BS;   // [3][TR][32]

  // Tile order: with RT_MAJOR the row tile varies slowest, so each XCD (a contiguous range of
  // logical ids) works on one or two row tiles of X, which then stay in its L2, and streams
  // B_vv; otherwise the tiles of one (Q, column tile) are adjacent and share B_vv^Q in L2.
  const int lb = xcd_local_id();
  if (lb >= nqc * n_ct * n_rt) return;
  int rt, ct, qq;
  if constexpr (RT_MAJOR) {
    ct = lb % n_ct;
    qq = (lb / n_ct) % nqc;
    rt = lb / (n_ct * nqc);
  } else {
    rt = lb % n_rt;
    ct = (lb / n_rt) % n_ct;
    qq = lb / (n_rt * n_ct);
  }
  const int c_base = ct * C::TC, r_base = rt * C::TR;
  const __bf16 *Vq = Bvv + (size_t)(q0 + qq) * v * v;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, m = lane & 31, lrow = lane >> 2;
  const int wc = wave / NWR, wr = wave % NWR;
  const int nkc = (v + KC - 1) / KC;
  int nvalid = 0;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) nvalid += (c_base + (wc * CB + cb) * 32 < v) ? 1 : 0;
  if (r_base + wr * RB * 32 >= M) nvalid = 0;  // no rows of this wave exist
  // (nvalid is wave-uniform)
  // the zero page's address stays in registers for the whole kernel (re-deriving it inside the
  // loop puts a scalar memory load among the LDS reads, which forces full LDS waits)
  const void *zp = g_zero_page_g;
  asm volatile("" : "+s"(zp));

  auto issue = [&](int kc) {
    const int a0 = kc * KC, buf = kc % 3;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int r0 = (wave * NA + k) * 16, r = r0 + lrow;
      const int a = a0 + 8 * ((lane & 3) ^ swz(r));
      const int cc = c_base + r;
      const bool ok = cc < v && a < v;
      dma16(ok ? (const void *)(Vq + (size_t)cc * v + a) : zp, As0 + buf * C::AS + r0 * KC);
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int r0 = (wave * NB + k) * 16, r = r0 + lrow;
      const int a = a0 + 8 * ((lane & 3) ^ swz(r));
      const int rr = r_base + r;
      const bool ok = rr < M && a < v;
      const size_t off = (size_t)rr * v + a;
      dma16(ok ? (const void *)(Xh + off) : zp, Xh0 + buf * C::BS + r0 * KC);
      dma16(ok ? (const void *)(Xl + off) : zp, Xl0 + buf * C::BS + r0 * KC);
    }
  };

  f16v acc[CB][RB];
#pragma unroll
  for (int a = 0; a < CB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[a][b] = zero16();

  struct Frag {
    bf8 a[CB], xh[RB], xl[RB];
  };
  // part 0: the B_vv fragments and X_hi; part 1: X_lo (used by the second half of the MFMAs)
  auto read_part = [&](int kc, int u, int part, Frag &F) {
    const int buf = kc % 3;
    if (part == 0) {
      const __bf16 *As = As0 + buf * C::AS;
      const __bf16 *Xhs = Xh0 + buf * C::BS;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int r = (wc * CB + cb) * 32 + m;
        F.a[cb] = *reinterpret_cast<const bf8 *>(&As[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int r = (wr * RB + rb) * 32 + m;
        F.xh[rb] = *reinterpret_cast<const bf8 *>(&Xhs[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
      }
    } else {
      const __bf16 *Xls = Xl0 + buf * C::BS;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int r = (wr * RB + rb) * 32 + m;
        F.xl[rb] = *reinterpret_cast<const bf8 *>(&Xls[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
      }
    }
  };
  // one half of a K step's products: X_hi (part 0) or X_lo (part 1) against the B_vv fragments
  auto mfma_part = [&](auto ncb_tag, const Frag &F, int part) {
    constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
        acc[cb][rb] =
            __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.a[cb], part ? F.xl[rb] : F.xh[rb], acc[cb][rb], 0, 0, 0);
  };

  // The pipelined loop, specialised on this wave's count of valid column blocks (wave-uniform;
  // only the last column tile has fewer than CB).  Choosing the specialisation once, outside the
  // loop, keeps branches out of it.  Waves without valid blocks (NCB = 0) still take part in
  // every load and barrier.  Per chunk kc, after the barrier that publishes it: issue the loads of
  // chunk kc+2, read K step 0's fragments (F0), run K step 1 of chunk kc-1 (F1, read before the
  // barrier) while they arrive, then the X_hi half of K step 0, then read K step 1's fragments
  // into F1 while the X_lo half runs (at most 8 LDS reads are outstanding at any wait, inside
  // the wait counter's range).  Chunks past the end (kc >= nkc) are issued too: their addresses
  // fall outside [0, v), so they load the zero page into a consumed buffer, which keeps the loop
  // free of branches around the loads.
  auto main_loop = [&](auto ncb_tag) {
    Frag F0, F1;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) F1.a[cb] = bf8{};  // "K step 1 of chunk -1": adds zero
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) F1.xh[rb] = F1.xl[rb] = bf8{};
    issue(0);
    issue(1);
    for (int kc = 0; kc < nkc; ++kc) {
      wait_vm<NL>();  // chunk kc has landed (chunk kc+1 may be in flight)
      lds_barrier();  // publishes chunk kc; every wave has read chunk kc-1's buffer
      issue(kc + 2);  // into chunk kc-1's buffer, two chunks ahead of its use
      __builtin_amdgcn_sched_barrier(0);
      read_part(kc, 0, 0, F0);
      read_part(kc, 0, 1, F0);
      __builtin_amdgcn_sched_barrier(0);
      // second K step of chunk kc-1 (a full chunk: only the last chunk can end inside a step)
      mfma_part(ncb_tag, F1, 0);
      mfma_part(ncb_tag, F1, 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_part(ncb_tag, F0, 0);  // K step 0 of a chunk always lies inside [0, v)
      __builtin_amdgcn_sched_barrier(0);
      read_part(kc, 1, 0, F1);
      read_part(kc, 1, 1, F1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_part(ncb_tag, F0, 1);
    }
    if (16 < v - (nkc - 1) * KC) {
      mfma_part(ncb_tag, F1, 0);
      mfma_part(ncb_tag, F1, 1);
    }
    wait_vm<0>();  // no LDS write may still be in flight when the workgroup ends
  };
  static_assert(CB >= 1 && CB <= 4, "column blocks per wave");
  if (nvalid == CB) {
    main_loop(std::integral_constant<int, CB>{});
  } else if (nvalid == 0) {
    main_loop(std::integral_constant<int, 0>{});
  } else {
    if constexpr (CB >= 4) {
      if (nvalid == 3) main_loop(std::integral_constant<int, 3>{});
    }
    if constexpr (CB >= 3) {
      if (nvalid == 2) main_loop(std::integral_constant<int, 2>{});
    }
    if constexpr (CB >= 2) {
      if (nvalid == 1) main_loop(std::integral_constant<int, 1>{});
    }
  }

  // store W^T as hi/lo planes: register t of lane (32h + m) holds row c = 8(t/4) + 4h + t%4,
  // column r = m of the block, so each register store covers 32 consecutive r
  __bf16 *Whq = Wh + (size_t)qq * v * M;
  __bf16 *Wlq = Wl + (size_t)qq * v * M;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int r = r_base + (wr * RB + rb) * 32 + m;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = c_base + (wc * CB + cb) * 32 + 8 * (t / 4) + 4 * h + (t % 4);
        if (c < v && r < M) {
          const float w = acc[cb][rb][t];
          const __bf16 hi = (__bf16)w;
          Whq[(size_t)c * M + r] = hi;
          Wlq[(size_t)c * M + r] = (__bf16)(w - (float)hi);
        }
      }
    }
}

// ---------------------------------------------------------------------------------------------
// (B) P[ks][s][i][c] (+)= scale * sum_{qq in split ks} sum_j B_oo^(q0+qq)[i][j] W^T[qq][c][s*o + j]
// Waves: NWM along i x NWN along c; each wave MB x NB blocks.  Reduction chunks run over (qq, j).
// ---------------------------------------------------------------------------------------------
template <int NWM, int NWN, int MB, int NB>
struct CfgB {
  static constexpr int NW = NWM * NWN, NT = 64 * NW;
  static constexpr int TM = NWM * MB * 32, TN = NWN * NB * 32;
  static constexpr int NA = TM / (16 * NW), NBL = TN / (16 * NW);
  static constexpr int AS = TM * KC, BS = TN * KC;
  static constexpr size_t LDS = (size_t)3 * (AS + 2 * BS) * 2;
  static constexpr int NL = NA + 2 * NBL;
  static_assert(TM % (16 * NW) == 0 && TN % (16 * NW) == 0, "tiles split into whole load instructions");
  static_assert(LDS <= 160 * 1024, "LDS");
};

template <int NWM, int NWN, int MB, int NB>
__global__ __launch_bounds__(64 * NWM * NWN, 1) void k_boo_w(const __bf16 *__restrict__ Boo,
                                                             const __bf16 *__restrict__ Wh,
                                                             const __bf16 *__restrict__ Wl, int o, int v, int ns,
                                                             int q0, int nqc, int nsplit, int n_ct, int accumulate,
                                                             float scale, float *__restrict__ P) {
  using C = CfgB<NWM, NWN, MB, NB>;
  constexpr int NA = C::NA, NBL = C::NBL, NL = C::NL;
  extern __shared__ __attribute__((aligned(16))) __bf16 ldsb[];
  __bf16 *As0 = ldsb;              // [3][TM][32]  B_oo rows
  __bf16 *Wh0 = As0 + 3 * C::AS;   // [3][TN][32]
  __bf16 *Wl0 = Wh0 + 3 * C::BS;

  const int lb = xcd_local_id();
  if (lb >= ns * n_ct * nsplit) return;
  const int ct = lb % n_ct, sl = (lb / n_ct) % ns, ks = lb / (n_ct * ns);
  const int qa = (int)((long long)ks * nqc / nsplit), qb = (int)((long long)(ks + 1) * nqc / nsplit);
  const int c_base = ct * C::TN, M = ns * o;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, m = lane & 31, lrow = lane >> 2;
  const int wm = wave / NWN, wn = wave % NWN;
  const int nkj = (o + KC - 1) / KC;
  const int NC = (qb - qa) * nkj;
  int nvalid = 0;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) nvalid += (c_base + (wn * NB + nb) * 32 < v) ? 1 : 0;
  if (wm * MB * 32 >= o) nvalid = 0;
  // (nvalid is wave-uniform)
  // the zero page's address stays in registers for the whole kernel (re-deriving it inside the
  // loop puts a scalar memory load among the LDS reads, which forces full LDS waits)
  const void *zp = g_zero_page_g;
  asm volatile("" : "+s"(zp));

  auto issue = [&](int c) {  // chunks c >= NC (past the end) load the zero page
    const bool live = c < NC;
    const int qq = live ? qa + c / nkj : qa, j0 = (c % nkj) * KC, buf = c % 3;
    const __bf16 *Oq = Boo + (size_t)(q0 + qq) * o * o;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int r0 = (wave * NA + k) * 16, r = r0 + lrow;
      const int j = j0 + 8 * ((lane & 3) ^ swz(r));
      const bool ok = live && r < o && j < o;
      dma16(ok ? (const void *)(Oq + (size_t)r * o + j) : zp, As0 + buf * C::AS + r0 * KC);
    }
    const size_t wq = (size_t)qq * v * M + (size_t)sl * o;
#pragma unroll
    for (int k = 0; k < NBL; ++k) {
      const int r0 = (wave * NBL + k) * 16, r = r0 + lrow;
      const int j = j0 + 8 * ((lane & 3) ^ swz(r));
      const int cc = c_base + r;
      const bool ok = live && cc < v && j < o;
      const size_t off = wq + (size_t)cc * M + j;
      dma16(ok ? (const void *)(Wh + off) : zp, Wh0 + buf * C::BS + r0 * KC);
      dma16(ok ? (const void *)(Wl + off) : zp, Wl0 + buf * C::BS + r0 * KC);
    }
  };

  f16v acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = zero16();

  // Same pipeline as the first kernel (see there): K step 0's fragments are read right after the
  // barrier while K step 1 of the previous chunk runs; K step 1's are read during the W_lo half of
  // K step 0.  Steps past o read zero rows of the B_oo tile and add nothing.
  struct Frag {
    bf8 a[MB], wh[NB], wl[NB];
  };
  auto read_step = [&](int c, int u, Frag &F) {
    const int buf = c % 3;
    const __bf16 *As = As0 + buf * C::AS;
    const __bf16 *Whs = Wh0 + buf * C::BS;
    const __bf16 *Wls = Wl0 + buf * C::BS;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int r = (wm * MB + mb) * 32 + m;
      F.a[mb] = *reinterpret_cast<const bf8 *>(&As[r * KC + 8 * ((2 * u + h) ^ swz(r))]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int r = (wn * NB + nb) * 32 + m;
      const int co = r * KC + 8 * ((2 * u + h) ^ swz(r));
      F.wh[nb] = *reinterpret_cast<const bf8 *>(&Whs[co]);
      F.wl[nb] = *reinterpret_cast<const bf8 *>(&Wls[co]);
    }
  };
  auto mfma_part = [&](auto nnb_tag, const Frag &F, int part) {
    constexpr int NNB = decltype(nnb_tag)::value;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
        acc[mb][nb] =
            __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.a[mb], part ? F.wl[nb] : F.wh[nb], acc[mb][nb], 0, 0, 0);
  };
  auto main_loop = [&](auto nnb_tag) {
    Frag F0, F1;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) F1.a[mb] = bf8{};
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) F1.wh[nb] = F1.wl[nb] = bf8{};
    issue(0);
    issue(1);
    for (int c = 0; c < NC; ++c) {
      wait_vm<NL>();  // chunk c has landed (chunk c+1 may be in flight)
      lds_barrier();
      issue(c + 2);  // into chunk c-1's buffer
      __builtin_amdgcn_sched_barrier(0);
      read_step(c, 0, F0);
      __builtin_amdgcn_sched_barrier(0);
      mfma_part(nnb_tag, F1, 0);  // K step 1 of chunk c-1 (zero fragments before chunk 0)
      mfma_part(nnb_tag, F1, 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_part(nnb_tag, F0, 0);
      __builtin_amdgcn_sched_barrier(0);
      read_step(c, 1, F1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_part(nnb_tag, F0, 1);
    }
    mfma_part(nnb_tag, F1, 0);
    mfma_part(nnb_tag, F1, 1);
    wait_vm<0>();  // no LDS write may still be in flight when the workgroup ends
  };
  static_assert(NB >= 1 && NB <= 4, "column blocks per wave");
  if (nvalid == NB) {
    main_loop(std::integral_constant<int, NB>{});
  } else if (nvalid == 0) {
    main_loop(std::integral_constant<int, 0>{});
  } else {
    if constexpr (NB >= 4) {
      if (nvalid == 3) main_loop(std::integral_constant<int, 3>{});
    }
    if constexpr (NB >= 3) {
      if (nvalid == 2) main_loop(std::integral_constant<int, 2>{});
    }
    if constexpr (NB >= 2) {
      if (nvalid == 1) main_loop(std::integral_constant<int, 1>{});
    }
  }

  // a split with no Q in this chunk still stores its (zero) slab on the first chunk
  float *Pp = P + ((size_t)ks * ns + sl) * o * v;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = c_base + (wn * NB + nb) * 32 + m;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int i = (wm * MB + mb) * 32 + 8 * (t / 4) + 4 * h + (t % 4);
        if (i < o && c < v) {
          float *dst = Pp + (size_t)i * v + c;
          const float val = scale * acc[mb][nb][t];
          *dst = accumulate ? *dst + val : val;
        }
      }
    }
}

// ---------------------------------------------------------------------------------------------
// Host side: the chunk loop.  W hi/lo for `qc` values of Q take qc * v * M * 4 bytes of scratch.
// ---------------------------------------------------------------------------------------------
template <int NWC, int NWR, int CB, int RB, bool RT_MAJOR, int NWM, int NWN, int MB, int NB>
hipError_t launch_xgemm(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o,
                        int v, int nq, int ns, int nsplit, float scale, float *P, void *scratch,
                        size_t scratch_bytes) {
  using CA = CfgA<NWC, NWR, CB, RB>;
  using CBf = CfgB<NWM, NWN, MB, NB>;
  if (o > CBf::TM || (o & 7) != 0 || (v & 7) != 0 || nq <= 0 || scratch == nullptr) return hipErrorInvalidValue;
  const int M = ns * o;
  const size_t per_q = (size_t)v * M * 2 * sizeof(__bf16);
  int qc = (int)std::min<size_t>((size_t)nq, scratch_bytes / per_q);
  if (qc < 1) return hipErrorInvalidValue;
  // equal chunks: fewer launches of nearly equal size
  const int nchunk = (nq + qc - 1) / qc;
  qc = (nq + nchunk - 1) / nchunk;
  __bf16 *Wh = static_cast<__bf16 *>(scratch);
  __bf16 *Wl = Wh + (size_t)qc * v * M;
  const int n_ct = (v + CA::TC - 1) / CA::TC, n_rt = (M + CA::TR - 1) / CA::TR;
  const int n_ctb = (v + CBf::TN - 1) / CBf::TN;
  for (int q0 = 0; q0 < nq; q0 += qc) {
    const int nqc = std::min(qc, nq - q0);
    const int ta = nqc * n_ct * n_rt;
    hipLaunchKernelGGL((k_xgemm_w<NWC, NWR, CB, RB, RT_MAJOR>), dim3((ta + 7) / 8 * 8), dim3(CA::NT), CA::LDS, s,
                       static_cast<const __bf16 *>(Bvv), static_cast<const __bf16 *>(X),
                       static_cast<const __bf16 *>(Xlo), v, M, q0, nqc, n_ct, n_rt, Wh, Wl);
    const int tb = ns * n_ctb * nsplit;
    hipLaunchKernelGGL((k_boo_w<NWM, NWN, MB, NB>), dim3((tb + 7) / 8 * 8), dim3(CBf::NT), CBf::LDS, s,
                       static_cast<const __bf16 *>(Boo), Wh, Wl, o, v, ns, q0, nqc, nsplit, n_ctb, q0 > 0 ? 1 : 0,
                       scale, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NWC, int NWR, int CB, int RB, bool RT_MAJOR, int NWM, int NWN, int MB, int NB>
hipError_t prepare_xgemm() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_xgemm_w<NWC, NWR, CB, RB, RT_MAJOR>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgA<NWC, NWR, CB, RB>::LDS);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_boo_w<NWM, NWN, MB, NB>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)CfgB<NWM, NWN, MB, NB>::LDS);
}

#define XGM(NWC, NWR, CB, RB, RTM, NWM, NWN, MB, NB, NAME)                                                   \
  ExchangeVariant {                                                                                          \
    RTTDA_PREC_MIXED_BF16, CfgB<NWM, NWN, MB, NB>::TM, 1, CfgA<NWC, NWR, CB, RB>::TC, NAME,                  \
        &launch_xgemm<NWC, NWR, CB, RB, RTM, NWM, NWN, MB, NB>,                                              \
        std::max(CfgA<NWC, NWR, CB, RB>::LDS, CfgB<NWM, NWN, MB, NB>::LDS),                                  \
        &prepare_xgemm<NWC, NWR, CB, RB, RTM, NWM, NWN, MB, NB>, 2 * KC, 8, 8, XGEMM_O_MIN, true            \
  }

const ExchangeVariant kGemmVariants[] = {
    XGM(2, 4, 4, 2, true, 4, 2, 2, 2, "bf16x2gemm_a256x256w8r_b256x128w8"),
    XGM(2, 4, 4, 2, false, 4, 2, 2, 2, "bf16x2gemm_a256x256w8_b256x128w8"),
    XGM(2, 4, 4, 2, true, 4, 2, 2, 4, "bf16x2gemm_a256x256w8r_b256x256w8"),
    XGM(2, 4, 4, 2, false, 4, 2, 2, 4, "bf16x2gemm_a256x256w8_b256x256w8"),
    XGM(2, 4, 4, 2, true, 4, 1, 2, 2, "bf16x2gemm_a256x256w8r_b256x64w4"),
    XGM(2, 4, 4, 2, false, 4, 1, 2, 2, "bf16x2gemm_a256x256w8_b256x64w4"),
};

}  // namespace

int exchange_gemm_variant_count() { return (int)(sizeof(kGemmVariants) / sizeof(kGemmVariants[0])); }
const ExchangeVariant *exchange_gemm_variant(int k) { return &kGemmVariants[k]; }

}  // namespace rttda
