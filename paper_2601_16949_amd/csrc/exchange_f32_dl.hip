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
//
// Paired slices (OH > 0): a kernel slice of O16 rows holds two real slices of at most OH rows each
// (rows [0, OH) and [OH, 2 OH)), so that o = 40 runs as 80-row tiles instead of two 48-row ones.
// The K product then takes the block-diagonal operand diag(B_oo^Q, B_oo^Q): its tile is the
// OT x OT B_oo^Q tile (OT = OH rounded up to 16), each fragment read with the row and column
// inside their halves and zeroed where the halves differ, and 16 x 16 tile pairs that lie wholly
// off the diagonal blocks are skipped at compile time.
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

// NWS rows of waves over the slices (2, or 1 for odd slice counts such as the split operator's
// R real slices), 4 / NWS columns of waves over the B_vv columns
// (with OH > 0, KS counts kernel slices, each a pair of real slices)
template <int O16, int WS, int WC, int NB = 3, int NWS = 2, int OH = 0>
struct CfgD {
  static constexpr int NWC = 4 / NWS;
  static constexpr int KS = NWS * WS, NT = 16 * WC * NWC, JB = O16 / 16;
  static constexpr int XROWS = KS * O16;
  static constexpr int XROWSP = (XROWS + 63) / 64 * 64;  // rows loaded (whole instructions; the rest zero)
  static constexpr int NXW = XROWSP / 64;  // X load instructions per wave (16 rows each, 4 waves)
  static constexpr int NBW = NT / 64;      // B_vv load instructions per wave
  static constexpr int OT = OH ? (OH + 15) / 16 * 16 : O16;  // rows and columns of the B_oo tile
  static constexpr int OCH = OT * OT / 4;                    // 16-byte chunks of the B_oo tile
  static constexpr int NOW = (OCH + 255) / 256;              // B_oo load instructions per wave
  static constexpr int XS = XROWSP * KC, BS = NT * KC;       // floats per buffer
  static constexpr int OS = NOW * 256 * 4;                   // floats (padded to whole instructions)
  static constexpr size_t LDS = (size_t)(NB * (XS + BS) + OS) * sizeof(float);  // NB chunk buffers
  static_assert(NT % 64 == 0, "tile must split into whole load instructions");
  static_assert(OH == 0 || (OH % 4 == 0 && 2 * OH <= O16), "paired slices: 16-byte B_oo chunks, both halves in the tile");
};

// paired slices: does the 16 x 16 tile pair (ib, jb) of diag(B_oo, B_oo) meet a diagonal block?
template <int OH>
__host__ __device__ constexpr bool pair_tile_live(int ib, int jb) {
  if (OH == 0) return true;
  for (int h = 0; h < 2; ++h) {
    const int lo = h * OH, hi = (h + 1) * OH;
    if (16 * ib < hi && 16 * ib + 16 > lo && 16 * jb < hi && 16 * jb + 16 > lo) return true;
  }
  return false;
}

// PIPE: 0 reads each chunk's fragments after its barrier and waits for them before its MFMAs;
// 1 is the half-chunk software pipeline (described at the loop) over three chunk buffers, loads
// issued two chunks ahead; 2 the same over two buffers, loads one chunk ahead (less LDS, so four
// workgroups fit a CU).
// OCC: workgroups per CU the register budget is sized for (2, or 3 where three fit the LDS).
template <int O16, int WS, int WC, int PIPE, int OCC, int NWS, int OH = 0>
__global__ __launch_bounds__(256, OCC) void k_exchange_f32_dl(const float *__restrict__ Boo,
                                                         const float *__restrict__ Bvv,
                                                         const float *__restrict__ X, int o, int v, int nq, int ns,
                                                         int n_sg, int n_ct, int nsplit, int xres, float scale,
                                                         float *__restrict__ P) {
  constexpr int NB = PIPE == 2 ? 2 : 3;
  using C = CfgD<O16, WS, WC, NB, NWS, OH>;
  constexpr int JB = C::JB, NXW = C::NXW, NBW = C::NBW, NOW = C::NOW, NXB = NXW + NBW, OT = C::OT;
  extern __shared__ __attribute__((aligned(16))) float ldsd[];
  float *Xs0 = ldsd;                 // [NB][XROWS][16]
  float *Bs0 = Xs0 + NB * C::XS;     // [NB][NT][16]
  float *Os = Bs0 + NB * C::BS;      // [OT][OT] (+ padding)

  const int total = n_sg * n_ct * nsplit;
  const int per_xcd = (int)gridDim.x / 8;
  const int lb = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (lb >= total) return;
  // Workgroup order over (slice group, column tile, Q split), consecutive ids on one XCD.  Slice
  // groups fastest: the workgroups of an XCD that run together share their B_vv^Q tiles in its L2
  // (the choice when X is small).  xres: slice groups slowest, so that an XCD holds the X tiles of
  // a few slice groups in its L2 and streams B_vv instead (the choice when X outgrows the L2).
  int sg, ct, sp;
  if (xres) {
    sp = lb % nsplit;
    ct = (lb / nsplit) % n_ct;
    sg = lb / (nsplit * n_ct);
  } else {
    sg = lb % n_sg;
    ct = (lb / n_sg) % n_ct;
    sp = lb / (n_sg * n_ct);
  }
  const int qa = (int)((long long)sp * nq / nsplit), qb = (int)((long long)(sp + 1) * nq / nsplit);
  const int s_base = sg * C::KS, c_base = ct * C::NT;

  // (the two-buffer form holds the wave index in a scalar register, and with it the LDS destinations)
  const int tid = threadIdx.x, lane = tid & 63, wave = PIPE == 2 ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int ws = wave / C::NWC, wc = wave % C::NWC;
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

  // loads of the chunk (Q index q, K chunk kc) into LDS buffer buf; with live false (chunks past
  // the end, pipelined loop) the B_vv lanes read the zero page
  auto issue_at = [&](int q, int kc, int buf, bool live) {
    const int a0 = kc * KC;
    float *Xs = Xs0 + buf * C::XS;
    float *Bs = Bs0 + buf * C::BS;
#pragma unroll
    for (int k = 0; k < NXW; ++k) {
      const int r0 = (wave * NXW + k) * 16, r = r0 + lrow;
      const int a = a0 + 4 * ((lane & 3) ^ swz(r));
      int sl = s_base + r / O16, j = r % O16;
      bool rv = true;
      if constexpr (OH > 0) {  // kernel slice s_base + r / O16 = real slices 2s (rows < OH) and 2s + 1
        const int hf = j / OH;
        sl = 2 * sl + hf;
        j -= hf * OH;
        rv = hf < 2 && r < C::XROWS;
      }
      const float *src = (rv && sl < ns && j < o && a < v) ? X + ((size_t)sl * o + j) * v + a : zp;
      dma16(src, Xs + r0 * KC);
    }
    const float *Vq = Bvv + (size_t)(live ? q : 0) * v * v;
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
      const int r0 = (wave * NBW + k) * 16, r = r0 + lrow;
      const int a = a0 + 4 * ((lane & 3) ^ swz(r));
      const int cc = c_base + r;
      const float *src = (live && cc < v && a < v) ? Vq + (size_t)cc * v + a : zp;  // row cc of symmetric B_vv
      dma16(src, Bs + r0 * KC);
    }
  };
  auto issue = [&](int c) { issue_at(qa + c / nkc, c % nkc, c % 3, true); };
  auto issue_os = [&](int q) {
    const float *Oq = Boo + (size_t)q * o * o;
    // (once per Q: with two buffers the per-lane addresses are recomputed here rather than held in
    // registers through the loop)
    int ln = lane;
    if constexpr (PIPE == 2) asm volatile("" : "+v"(ln));
#pragma unroll
    for (int k = 0; k < NOW; ++k) {
      const int e0 = (wave * NOW + k) * 64, e = e0 + ln;  // 16-byte chunk index in the tile
      const int i = e / (OT / 4), p = e % (OT / 4);
      const int jc = 4 * (p ^ swz_o<OT>(i));
      const float *src = (e < C::OCH && i < o && jc < o) ? Oq + (size_t)i * o + jc : zp;
      dma16(src, Os + e0 * 4);
    }
  };

  // K-product operand: the B_oo^Q entries of rows ib*16 + n, columns jb*16 + 4g .. +3 (with paired
  // slices, of diag(B_oo^Q, B_oo^Q): the tile entry inside the halves, zero across them)
  auto boo_frag = [&](int ib, int jb) __attribute__((always_inline)) -> f4 {
    const int i = ib * 16 + n;
    if constexpr (OH == 0) {
      return *reinterpret_cast<const f4 *>(&Os[i * O16 + 4 * ((jb * 4 + g) ^ swz_o<O16>(i))]);
    } else {
      const int j = jb * 16 + 4 * g;
      const int hi = i / OH, hj = j / OH, ii = i - hi * OH, jj = j - hj * OH;
      const f4 e = *reinterpret_cast<const f4 *>(&Os[ii * OT + 4 * ((jj >> 2) ^ swz_o<OT>(ii))]);
      return (hi == hj && hi < 2) ? e : f4{0.f, 0.f, 0.f, 0.f};
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
        for (int ib = 0; ib < JB; ++ib)
          if (pair_tile_live<OH>(ib, jb)) ar[ib] = boo_frag(ib, jb);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ib = 0; ib < JB; ++ib)
            if (pair_tile_live<OH>(ib, jb)) {
#pragma unroll
              for (int si = 0; si < WS; ++si)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                  Kacc[si][ib][cb] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ib][t], Wacc[si][jb][cb][t], Kacc[si][ib][cb], 0, 0, 0);
            }
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
    // Half-chunk software pipeline.  A chunk's MFMAs split into half 0 (row blocks jb < JH) and
    // half 1 (jb >= JH).  Per chunk c, after the barrier that publishes it: issue the loads of
    // chunk c+2, read chunk c's B_vv fragments and half-0 X fragments, run half 1 of chunk c-1
    // (fragments read before the barrier) and, at the end of a Q, its K product while they
    // arrive, then half 0 of chunk c in two parts with the half-1 reads between them.  Every LDS
    // wait is then a wait for all outstanding reads.  The chunk, K-chunk and Q counters advance
    // incrementally (no divisions in the loop); chunks past the end are issued too (zero page for
    // B_vv) so the loads need no branch; the B_oo^Q tile of the Q that starts at chunk s is loaded
    // at chunk s+1, after the barrier behind which every wave finished the previous Q's K product,
    // ahead of that chunk's own loads so that the per-chunk wait count stays the same.
    constexpr int JH = (JB + 1) / 2;  // row blocks of half 0
    struct FragB {
      f4 b[WC];
    };
    struct FragA {
      f4 a[WS][JH];
    };
    auto read_b = [&](auto ncb_tag, int buf, FragB &F) __attribute__((always_inline)) {
      constexpr int NCB = decltype(ncb_tag)::value;
      const float *Bs = Bs0 + buf * C::BS;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int r = (wc * WC + cb) * 16 + n;
        F.b[cb] = *reinterpret_cast<const f4 *>(&Bs[r * KC + 4 * (g ^ swz(r))]);
      }
    };
    auto read_a = [&](auto ncb_tag, auto half_tag, int buf, FragA &F) __attribute__((always_inline)) {
      constexpr int NCB = decltype(ncb_tag)::value, HF = decltype(half_tag)::value;
      const float *Xs = Xs0 + buf * C::XS;
      if constexpr (NCB > 0) {
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jj = 0; jj < JH; ++jj) {
            const int jb = HF * JH + jj;
            if (jb < JB) {
              const int r = (ws * WS + si) * O16 + jb * 16 + n;
              F.a[si][jj] = *reinterpret_cast<const f4 *>(&Xs[r * KC + 4 * (g ^ swz(r))]);
            }
          }
      }
    };
    // W += X B_vv for one half's row blocks, K values t0 <= t < t1 of the chunk
    auto mfma_half = [&](auto ncb_tag, auto half_tag, const FragB &B, const FragA &A, auto t0_tag, auto t1_tag) __attribute__((always_inline)) {
      constexpr int NCB = decltype(ncb_tag)::value, HF = decltype(half_tag)::value;
      constexpr int t0 = decltype(t0_tag)::value, t1 = decltype(t1_tag)::value;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < t0 || t >= t1) continue;
#pragma unroll
        for (int si = 0; si < WS; ++si)
#pragma unroll
          for (int jj = 0; jj < JH; ++jj) {
            const int jb = HF * JH + jj;
            if (jb < JB) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb)
                Wacc[si][jb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[si][jj][t], B.b[cb][t], Wacc[si][jb][cb], 0, 0, 0);
            }
          }
      }
    };
    // K += B_oo^Q W for the Q whose last chunk was just multiplied, then W = 0
    auto compute_k = [&](auto ncb_tag) __attribute__((always_inline)) {
      constexpr int NCB = decltype(ncb_tag)::value;
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        f4 ar[JB];
#pragma unroll
        for (int ib = 0; ib < JB; ++ib)
          if (pair_tile_live<OH>(ib, jb)) ar[ib] = boo_frag(ib, jb);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int ib = 0; ib < JB; ++ib)
            if (pair_tile_live<OH>(ib, jb)) {
#pragma unroll
              for (int si = 0; si < WS; ++si)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                  Kacc[si][ib][cb] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ib][t], Wacc[si][jb][cb][t], Kacc[si][ib][cb], 0, 0, 0);
            }
      }
#pragma unroll
      for (int a = 0; a < WS; ++a)
#pragma unroll
        for (int b = 0; b < JB; ++b)
#pragma unroll
          for (int cc = 0; cc < WC; ++cc) Wacc[a][b][cc] = f4{0.f, 0.f, 0.f, 0.f};
    };
    using H0 = std::integral_constant<int, 0>;
    using H1 = std::integral_constant<int, 1>;
    using T0 = std::integral_constant<int, 0>;
    using T2 = std::integral_constant<int, 2>;
    using T4 = std::integral_constant<int, 4>;
    auto main_loop = [&](auto ncb_tag) __attribute__((always_inline)) {
      constexpr int NCB = decltype(ncb_tag)::value;
      if (NC == 0) return;
      FragB B0, B1;
      FragA A0, A1;
      issue_os(qa);
      issue_at(qa, 0, 0, true);
      if constexpr (NB == 3) issue_at(qa, 1, 1, true);  // NC >= nkc >= 3
      // the chunk NB-1 ahead of chunk c: (Q index, K chunk, buffer), advanced one chunk per iteration
      int q2 = qa, kc2 = NB - 1, b2 = NB - 1;
      int kcc = 0, qc = qa, buf = 0;  // chunk c's K chunk, Q index and LDS buffer
      auto step = [&](int c, FragB &Bc, const FragB &Bp) __attribute__((always_inline)) {
        // chunk c (and a B_oo^Q tile issued before it) has landed; with three buffers chunk c+1
        // may still be in flight
        if constexpr (NB == 3) wait_vm<NXB>(); else wait_vm<0>();
        lds_barrier();   // publishes chunk c; every wave has read chunk c-1 and run the last K product
        if (kcc == 1 && c > 1) issue_os(qc);  // chunk c-1 opened Q qc; the K product before it is done
        issue_at(q2, kc2, b2, c + NB - 1 < NC);  // into chunk c-1's buffer
        if (++kc2 == nkc) { kc2 = 0; ++q2; }
        b2 = b2 == NB - 1 ? 0 : b2 + 1;
        __builtin_amdgcn_sched_barrier(0);
        read_b(ncb_tag, buf, Bc);
        read_a(ncb_tag, H0{}, buf, A0);
        __builtin_amdgcn_sched_barrier(0);
        if (c > 0) {
          mfma_half(ncb_tag, H1{}, Bp, A1, T0{}, T4{});  // chunk c-1, half 1
          if constexpr (NCB > 0) {
            if (kcc == 0) compute_k(ncb_tag);  // chunk c-1 closed its Q
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        mfma_half(ncb_tag, H0{}, Bc, A0, T0{}, T2{});
        __builtin_amdgcn_sched_barrier(0);
        read_a(ncb_tag, H1{}, buf, A1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_half(ncb_tag, H0{}, Bc, A0, T2{}, T4{});
        if (++kcc == nkc) { kcc = 0; ++qc; }
        buf = buf == NB - 1 ? 0 : buf + 1;
      };
      for (int c = 0; c < NC; c += 2) {
        step(c, B0, B1);
        if (c + 1 < NC) step(c + 1, B1, B0);
      }
      if (NC & 1)  // chunk NC-1, half 1 (a select between the two sets would put them in memory)
        mfma_half(ncb_tag, H1{}, B0, A1, T0{}, T4{});
      else
        mfma_half(ncb_tag, H1{}, B1, A1, T0{}, T4{});
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
    const int ks = s_base + ws * WS + si;  // kernel slice
    if ((OH ? 2 * ks : ks) >= ns) continue;
#pragma unroll
    for (int ib = 0; ib < JB; ++ib)
#pragma unroll
      for (int cb = 0; cb < WC; ++cb) {
        const int c = c_base + (wc * WC + cb) * 16 + n;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int i = ib * 16 + 4 * g + t, sl = ks;
          if constexpr (OH > 0) {
            const int hf = i / OH;
            sl = 2 * ks + hf;
            i -= hf * OH;
            if (hf >= 2 || sl >= ns) continue;
          }
          if (i < o && c < v) Pp[((size_t)sl * o + i) * v + c] = scale * Kacc[si][ib][cb][t];
        }
      }
  }
}

template <int O16, int WS, int WC, int PIPE, int OCC, int NWS, int OH = 0>
hipError_t launch_xf32dl(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *, int o, int v,
                         int nq, int ns, int nsplit, float scale, float *P, void *, size_t) {
  using C = CfgD<O16, WS, WC, PIPE == 2 ? 2 : 3, NWS, OH>;
  if (o > (OH ? OH : O16) || (v & 3) != 0 || (o & 3) != 0 || v < 3 * KC) return hipErrorInvalidValue;
  const int nks = OH ? (ns + 1) / 2 : ns;  // kernel slices
  const int n_sg = (nks + C::KS - 1) / C::KS, n_ct = (v + C::NT - 1) / C::NT;
  const int total = n_sg * n_ct * nsplit;
  // X (all slices) beyond half of an XCD's 4 MiB L2: keep X resident per XCD, stream B_vv
  const int xres = (size_t)ns * o * v * sizeof(float) > (size_t)(2u << 20) ? 1 : 0;
  dim3 grid((total + 7) / 8 * 8);
  hipLaunchKernelGGL((k_exchange_f32_dl<O16, WS, WC, PIPE, OCC, NWS, OH>), grid, dim3(256), C::LDS, s,
                     static_cast<const float *>(Boo), static_cast<const float *>(Bvv), static_cast<const float *>(X), o,
                     v, nq, ns, n_sg, n_ct, nsplit, xres, scale, P);
  return hipGetLastError();
}

template <int O16, int WS, int WC, int PIPE, int OCC, int NWS, int OH = 0>
hipError_t prepare_xf32dl() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_exchange_f32_dl<O16, WS, WC, PIPE, OCC, NWS, OH>),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)CfgD<O16, WS, WC, PIPE == 2 ? 2 : 3, NWS, OH>::LDS);
}

#define XDLS(O16, WS, WC, PIPE, OCC, NWS, NAME)                                                          \
  ExchangeVariant {                                                                                      \
    RTTDA_PREC_FP32, O16, CfgD<O16, WS, WC, 3, NWS>::KS, CfgD<O16, WS, WC, 3, NWS>::NT, NAME,            \
        &launch_xf32dl<O16, WS, WC, PIPE, OCC, NWS>, CfgD<O16, WS, WC, PIPE == 2 ? 2 : 3, NWS>::LDS,      \
        &prepare_xf32dl<O16, WS, WC, PIPE, OCC, NWS>, 3 * KC, 4, 4, 1, false, PIPE ? 2 : 1              \
  }
#define XDL(O16, WS, WC, PIPE, OCC, NAME) XDLS(O16, WS, WC, PIPE, OCC, 2, NAME)
#define XDL2(O16, WS, WC)                                                                                \
  XDL(O16, WS, WC, 0, 2, "f32dl_o" #O16 "_ws" #WS "_wc" #WC),                                            \
      XDL(O16, WS, WC, 1, 2, "f32dlp_o" #O16 "_ws" #WS "_wc" #WC)

// paired slices: o16 is the half size OH, ks counts real slices (two per kernel slice)
#define XDLP(O16, WS, WC, OCC, OH, NAME)                                                                 \
  ExchangeVariant {                                                                                      \
    RTTDA_PREC_FP32, OH, 2 * CfgD<O16, WS, WC, 3, 2, OH>::KS, CfgD<O16, WS, WC, 3, 2, OH>::NT, NAME,     \
        &launch_xf32dl<O16, WS, WC, 1, OCC, 2, OH>, CfgD<O16, WS, WC, 3, 2, OH>::LDS,                    \
        &prepare_xf32dl<O16, WS, WC, 1, OCC, 2, OH>, 3 * KC, 4, 4, 1, false, 2                            \
  }

// (o64 ws1 wc2 fits three workgroups per CU in both forms: at most 152 registers, 52 KiB of LDS)
const ExchangeVariant kF32DlVariants[] = {
    XDL2(32, 1, 2), XDL2(32, 2, 2), XDL2(48, 2, 2), XDL2(64, 1, 2), XDL2(64, 2, 2), XDL2(64, 1, 4), XDL2(96, 1, 2),
    XDL(64, 1, 2, 2, 4, "f32dlq_o64_ws1_wc2"),
    // one slice per workgroup, four columns of waves (odd slice counts: no idle slice row)
    XDLS(64, 1, 2, 1, 2, 1, "f32dlp_o64_ws1_wc2_s1"), XDLS(64, 1, 1, 1, 2, 1, "f32dlp_o64_ws1_wc1_s1"),
    // two slices of up to 40 rows in one 80-row tile
    XDLP(80, 1, 2, 2, 40, "f32dlp_p40_ws1_wc2"), XDLP(80, 1, 4, 1, 40, "f32dlp_p40_ws1_wc4"),
    XDLP(80, 2, 2, 1, 40, "f32dlp_p40_ws2_wc2"),
};

}  // namespace

int exchange_f32dl_variant_count() { return (int)(sizeof(kF32DlVariants) / sizeof(kF32DlVariants[0])); }
const ExchangeVariant *exchange_f32dl_variant(int k) { return &kF32DlVariants[k]; }

}  // namespace rttda
