// Host runtime of the RT-TDA library: argument validation, workspace layout, the RK4 step
// sequence (direct launches or replay of a captured HIP graph) and the C ABI.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace rttda {
int exchange_f32_variant_count();
const ExchangeVariant *exchange_f32_variant(int k);
int exchange_bf16_variant_count();
const ExchangeVariant *exchange_bf16_variant(int k);
int exchange_f32dl_variant_count();
const ExchangeVariant *exchange_f32dl_variant(int k);
int exchange_bf16dl_variant_count();
const ExchangeVariant *exchange_bf16dl_variant(int k);
int exchange_gemm_variant_count();
const ExchangeVariant *exchange_gemm_variant(int k);
}  // namespace rttda

using namespace rttda;

static_assert(sizeof(DevPulse) == sizeof(rttda_pulse), "pulse layout");
static_assert(offsetof(DevPulse, dir) == offsetof(rttda_pulse, dir), "pulse layout");

namespace {

thread_local std::string g_last_error;

rttda_status fail(rttda_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
rttda_status fail(rttda_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail(RTTDA_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

constexpr int MAX_RHS = 4096;
constexpr int SJ_MAX = 8;    // Coulomb second-product Q splits
constexpr int SK_MAX = 768;  // exchange Q splits
// exchange flops per stage (at the largest RHS count) from which the Coulomb pair gets its own stream
constexpr double OVERLAP_MIN_FLOPS = 5e10;
constexpr int SMALL_SPLITS = 64;
// slices (2 max_rhs) from which the Coulomb pair runs on the matrix cores
constexpr int COUL_MFMA_MIN_SLICES = 32;
// the exchange's partial K slabs (one per split) take at most this much workspace, or 32 slabs
constexpr size_t SK_SLAB_BYTES = (size_t)256 << 20;
constexpr size_t ALIGN = 256;

inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

struct Layout {
  size_t D, moo, mov, mvv, xs64, xs0, acc, acc0, F, part, sc, x32, xhi, xlo, dvec, P, pulses, state, normref;
  size_t xref, xref0;  // reference state of the time-correlation output (state at the start of a call)
  size_t epart;        // per-block partial sums of the energy output ([R][EP_BX_MAX] FP64)
  size_t scratch, scratch_bytes;  // W hi/lo of the large-o exchange path (0 bytes when it does not apply)
  size_t lz, lzp;                 // Lanczos guard: three FP64 vectors of ov, block partial sums
  size_t total;
  int nbf;
  int sk_max, sj_max;
};

// slab_bytes: workspace for the exchange's partial K slabs (at least 32 slabs); gemm_scratch: carve
// the W scratch of the large-o GEMM exchange path where that path applies
Layout make_layout(int o, int v, int nq, int R, int prec, size_t slab_bytes = SK_SLAB_BYTES,
                   bool gemm_scratch = true) {
  Layout L{};
  const size_t ov = (size_t)o * v;
  const size_t ns = 2 * (size_t)R;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += up(bytes > 0 ? bytes : 1);
    return at;
  };
  L.nbf = field_blocks_a(v) * field_blocks_i(o);
  L.sj_max = nq > 0 ? std::min(SJ_MAX, nq) : 0;
  L.sk_max = nq > 0 ? std::min({SK_MAX, nq, (int)std::max<size_t>(32, slab_bytes / (ns * ov * 4))}) : 0;
  L.D = take(ov * 8);
  L.moo = take((size_t)R * o * o * 8);
  L.mov = take((size_t)R * ov * 8);
  L.mvv = take((size_t)R * v * v * 8);
  L.xs64 = take(ns * ov * 8);
  L.xs0 = take(ns * 8);
  L.acc = take(ns * ov * 8);
  L.acc0 = take(ns * 8);
  L.F = take(ns * ov * 8);
  L.part = take((size_t)R * L.nbf * PART_STRIDE * 8);
  L.sc = take((size_t)R * SC_STRIDE * 8);
  L.x32 = take(ns * ov * 4);  // FP32 stage copy (Coulomb input; exchange input in FP32 mode)
  L.xhi = take(prec == RTTDA_PREC_MIXED_BF16 ? ns * ov * 2 : 0);
  L.xlo = take(prec == RTTDA_PREC_MIXED_BF16 ? ns * ov * 2 : 0);
  L.dvec = take((size_t)GEMV1_CHUNKS_MAX * std::max(nq, 1) * ns * 4);
  L.P = take((size_t)(L.sj_max + L.sk_max) * ns * ov * 4);
  L.pulses = take((size_t)R * sizeof(DevPulse));
  L.state = take(sizeof(DevState));
  L.normref = take((size_t)R * 8);
  L.xref = take(ns * ov * 8);
  L.xref0 = take(ns * 8);
  L.epart = take((size_t)R * EP_BX_MAX * 8);
  L.scratch_bytes = 0;
  if (gemm_scratch && prec == RTTDA_PREC_MIXED_BF16 && nq > 0 && o >= XGEMM_O_MIN && o <= 256 && o % 8 == 0 &&
      v % 8 == 0) {
    const size_t per_q = (size_t)v * ns * o * 4;  // W hi + lo for one Q at the largest RHS count
    L.scratch_bytes = std::min((size_t)nq * per_q, std::max(per_q, XGEMM_SCRATCH_MAX));
  }
  L.scratch = take(L.scratch_bytes);
  L.lz = take(3 * ov * 8);
  L.lzp = take((size_t)LZ_BLOCKS_MAX * 8);
  L.total = off;
  return L;
}

struct Profiler {
  static constexpr int CLASSES = 4;
  static constexpr size_t CAP = 2048;  // event pairs kept per class before folding
  bool on = false;
  std::vector<hipEvent_t> start[CLASSES], stop[CLASSES];
  size_t used[CLASSES] = {0, 0, 0, 0};
  int64_t launches[CLASSES] = {0, 0, 0, 0};
  double ms[CLASSES] = {0, 0, 0, 0};

  hipError_t fold(int k) {
    if (used[k] == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(stop[k][used[k] - 1]);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < used[k]; ++i) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, start[k][i], stop[k][i]);
      if (e != hipSuccess) return e;
      ms[k] += t;
    }
    used[k] = 0;
    return hipSuccess;
  }
  hipError_t begin(int k, hipStream_t s) {
    if (used[k] == CAP) {
      hipError_t e = fold(k);
      if (e != hipSuccess) return e;
    }
    if (start[k].size() <= used[k]) {
      hipEvent_t a, b;
      hipError_t e = hipEventCreate(&a);
      if (e == hipSuccess) e = hipEventCreate(&b);
      if (e != hipSuccess) return e;
      start[k].push_back(a);
      stop[k].push_back(b);
    }
    return hipEventRecord(start[k][used[k]], s);
  }
  hipError_t end(int k, hipStream_t s) {
    hipError_t e = hipEventRecord(stop[k][used[k]], s);
    ++used[k];
    ++launches[k];
    return e;
  }
  void reset() {
    for (int k = 0; k < CLASSES; ++k) {
      used[k] = 0;
      launches[k] = 0;
      ms[k] = 0;
    }
  }
  void destroy() {
    for (int k = 0; k < CLASSES; ++k) {
      for (auto e : start[k]) (void)hipEventDestroy(e);
      for (auto e : stop[k]) (void)hipEventDestroy(e);
      start[k].clear();
      stop[k].clear();
    }
  }
};

enum { PC_EXCHANGE = 0, PC_COULOMB = 1, PC_FIELD = 2, PC_EPILOGUE = 3 };

struct GraphEntry {
  bool valid = false;
  // key
  int nrhs = 0, steps = 0, mode = 0, integ = 0;
  double dt = 0;
  const void *c0 = nullptr, *c = nullptr;
  bool trace = false, norms = false, corr = false, pops = false, energy = false;
  hipGraphExec_t exec = nullptr;
};

// Variant tables: register-staged variants first, then direct-to-LDS variants
const ExchangeVariant *variant_of(int prec, int k) {
  if (k < 0) return nullptr;
  if (prec == RTTDA_PREC_FP32) {
    const int n1 = exchange_f32_variant_count();
    if (k < n1) return exchange_f32_variant(k);
    k -= n1;
    return k < exchange_f32dl_variant_count() ? exchange_f32dl_variant(k) : nullptr;
  }
  const int n2 = exchange_bf16_variant_count();
  if (k < n2) return exchange_bf16_variant(k);
  k -= n2;
  const int n3 = exchange_bf16dl_variant_count();
  if (k < n3) return exchange_bf16dl_variant(k);
  k -= n3;
  return k < exchange_gemm_variant_count() ? exchange_gemm_variant(k) : nullptr;
}
int variant_count(int prec) {
  return prec == RTTDA_PREC_FP32
             ? exchange_f32_variant_count() + exchange_f32dl_variant_count()
             : exchange_bf16_variant_count() + exchange_bf16dl_variant_count() + exchange_gemm_variant_count();
}
// a variant runs on a context when it holds the shape and, if it needs one, the workspace has scratch
bool usable(const ExchangeVariant *x, int o, int v, const Layout &L) {
  return x && x->applies(o, v) && (!x->scratch || L.scratch_bytes > 0);
}

}  // namespace

struct rttda_ctx {
  rttda_desc d{};
  hipStream_t stream = nullptr;
  int o = 0, v = 0, nq = 0, R = 0, prec = 0;
  size_t ov = 0;
  Layout L{};
  char *ws = nullptr;
  // launch configuration
  int xvar = -1;  // 0-based exchange variant
  int sk = 0, sj = 0;
  int use_graph = 1, steps_per_graph = 8;
  int qchunk = 0;  // Q per chunk of the GEMM exchange path, 0 = as many as the scratch holds
  // second stream for the Coulomb pair, which then runs alongside the exchange (HBM-bound next to
  // MFMA-bound work); fork and join through two events, also inside a captured graph
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int overlap = 2;  // 1: Coulomb pair on the second stream, 2: in order on the context's stream
  // small problems: the stage's Coulomb + exchange slabs in one launch (small_splits slabs) and the
  // RK4 stage epilogue in one single-workgroup launch
  int small = 0, small_splits = 0;
  // Coulomb pair on the matrix cores (batches of many slices) instead of the vector-unit GEMVs
  int coul_mfma = 0;
  double *corr_next = nullptr;  // time-correlation output of the next propagate call
  double *energy_next = nullptr;  // energy output of the next propagate call
  double *pops_next = nullptr;  // populations output of the next propagate call, its vectors and count
  const double *popU_next = nullptr;
  int popk_next = 0;
  // host staging for pulses (pinned)
  DevPulse *h_pulses = nullptr;
  hipEvent_t upload_ev = nullptr;
  GraphEntry graph;
  Profiler prof;

  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  double *D() const { return at<double>(L.D); }
  double *moo() const { return at<double>(L.moo); }
  double *mov() const { return at<double>(L.mov); }
  double *mvv() const { return at<double>(L.mvv); }
  double *xs64() const { return at<double>(L.xs64); }
  double *xs0() const { return at<double>(L.xs0); }
  double *acc() const { return at<double>(L.acc); }
  double *acc0() const { return at<double>(L.acc0); }
  double *F() const { return at<double>(L.F); }
  double *part() const { return at<double>(L.part); }
  double *sc() const { return at<double>(L.sc); }
  float *x32() const { return at<float>(L.x32); }
  __hip_bfloat16 *xhi() const { return at<__hip_bfloat16>(L.xhi); }
  __hip_bfloat16 *xlo() const { return at<__hip_bfloat16>(L.xlo); }
  float *dvec() const { return at<float>(L.dvec); }
  float *P() const { return at<float>(L.P); }
  void *scratch() const { return L.scratch_bytes ? static_cast<void *>(ws + L.scratch) : nullptr; }
  double *lz() const { return at<double>(L.lz); }
  double *lzp() const { return at<double>(L.lzp); }
  DevPulse *pulses() const { return at<DevPulse>(L.pulses); }
  DevState *state() const { return at<DevState>(L.state); }
  double *normref() const { return at<double>(L.normref); }
  double *xref() const { return at<double>(L.xref); }
  double *xref0() const { return at<double>(L.xref0); }
  double *epart() const { return at<double>(L.epart); }
};

namespace {

rttda_status validate_desc(const rttda_desc *d, bool need_ptrs) {
  if (!d) return fail(RTTDA_E_INVAL, "desc is NULL");
  if (d->n_occ < 1 || d->n_virt < 1 || d->n_aux < 0)
    return fail(RTTDA_E_INVAL, "bad sizes o=%d v=%d n_aux=%d (need o,v >= 1, n_aux >= 0)", d->n_occ, d->n_virt,
                d->n_aux);
  if ((long long)d->n_occ * d->n_virt > (1LL << 31) / 8)
    return fail(RTTDA_E_UNSUPPORTED, "o*v=%lld too large", (long long)d->n_occ * d->n_virt);
  if (d->max_rhs < 1 || d->max_rhs > MAX_RHS)
    return fail(RTTDA_E_INVAL, "max_rhs=%d outside 1..%d", d->max_rhs, MAX_RHS);
  if (d->precision == RTTDA_PREC_FP32) {
    if (d->b_dtype != RTTDA_F32) return fail(RTTDA_E_INVAL, "PREC_FP32 needs b_dtype RTTDA_F32");
  } else if (d->precision == RTTDA_PREC_MIXED_BF16) {
    if (d->b_dtype != RTTDA_BF16) return fail(RTTDA_E_INVAL, "PREC_MIXED_BF16 needs b_dtype RTTDA_BF16");
  } else {
    return fail(RTTDA_E_INVAL, "unknown precision %d", d->precision);
  }
  if (!std::isfinite(d->cx)) return fail(RTTDA_E_INVAL, "cx not finite");
  if (need_ptrs) {
    const void *ptrs[] = {d->e_occ, d->e_virt, d->mu, d->workspace};
    const char *names[] = {"e_occ", "e_virt", "mu", "workspace"};
    for (int k = 0; k < 4; ++k) {
      if (!ptrs[k]) return fail(RTTDA_E_INVAL, "%s is NULL", names[k]);
      if (!aligned16(ptrs[k])) return fail(RTTDA_E_INVAL, "%s not 16-byte aligned", names[k]);
    }
    if ((reinterpret_cast<uintptr_t>(d->workspace) & (ALIGN - 1)) != 0)
      return fail(RTTDA_E_INVAL, "workspace not 256-byte aligned");
    if (d->n_aux > 0) {
      const void *bp[] = {d->b_ov, d->b_oo, d->b_vv};
      const char *bn[] = {"b_ov", "b_oo", "b_vv"};
      for (int k = 0; k < 3; ++k) {
        if (!bp[k]) return fail(RTTDA_E_INVAL, "%s is NULL", bn[k]);
        if (!aligned16(bp[k])) return fail(RTTDA_E_INVAL, "%s not 16-byte aligned", bn[k]);
      }
    }
  }
  return RTTDA_OK;
}

int auto_variant(int prec, int o, int ns, int v, const Layout &L) {
  const int n = variant_count(prec);
  // the large-o GEMM path first whenever the workspace carries its scratch
  for (int k = 0; k < n; ++k) {
    const ExchangeVariant *x = variant_of(prec, k);
    if (x->scratch && usable(x, o, v, L)) return k;
  }
  // else the smallest padded occupied size that holds o; among those prefer the variant whose
  // tile wastes the least of the (slices x columns) space, then the larger tile, then the
  // variant's rank (the pipelined direct-to-LDS kernels over the plain ones over the register ones).
  int best = -1, best_rank = -1;
  double best_score = 1e300;
  int o16_best = 1 << 30;
  for (int k = 0; k < n; ++k) {
    const ExchangeVariant *x = variant_of(prec, k);
    if (!x->scratch && x->applies(o, v) && x->o16 < o16_best) o16_best = x->o16;
  }
  for (int k = 0; k < n; ++k) {
    const ExchangeVariant *x = variant_of(prec, k);
    if (x->scratch || x->o16 != o16_best || !x->applies(o, v)) continue;
    const double rows = (double)((ns + x->ks - 1) / x->ks) * x->ks;
    const double cols = (double)((v + x->nt - 1) / x->nt) * x->nt;
    const double waste = rows * cols / ((double)ns * v);
    const double score = waste * (1.0 + 8.0 / (x->ks * x->nt));  // mild preference for big tiles
    if (score < best_score * (1.0 - 1e-12) || (score <= best_score * (1.0 + 1e-12) && x->rank > best_rank)) {
      best_score = score;
      best_rank = x->rank;
      best = k;
    }
  }
  return best;
}

int auto_splits(const ExchangeVariant *x, int o, int ns, int v, int nq, int cap, const Layout &L) {
  if (x->scratch) {
    // GEMM path: splits of each chunk's Q range for the B_oo product (about two workgroups per
    // CU), at most the chunk length
    const size_t per_q = (size_t)v * ns * o * 4;
    const int qc = (int)std::max<size_t>(1, std::min<size_t>((size_t)nq, L.scratch_bytes / per_q));
    const int tiles_b = ns * ((v + 127) / 128);
    int s = (512 + tiles_b - 1) / tiles_b;
    return std::max(1, std::min({s, std::max(1, qc / 2), cap}));
  }
  const int tiles = ((ns + x->ks - 1) / x->ks) * ((v + x->nt - 1) / x->nt);
  const int cus = 256;
  // aim at about six rounds of one workgroup per CU (tail below ~15 %), at least 4 Q per split
  int s = (6 * cus + tiles - 1) / tiles;
  s = std::min(s, std::max(1, nq / 4));
  s = std::max(1, std::min(s, cap));
  return s;
}

rttda_status upload_pulses(rttda_ctx *ctx, const DevPulse *src, int nrhs) {
  HIP_TRY(hipEventSynchronize(ctx->upload_ev));  // previous upload has left the staging buffer
  memcpy(ctx->h_pulses, src, sizeof(DevPulse) * nrhs);
  HIP_TRY(hipMemcpyAsync(ctx->pulses(), ctx->h_pulses, sizeof(DevPulse) * nrhs, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipEventRecord(ctx->upload_ev, ctx->stream));
  return RTTDA_OK;
}

rttda_status check_dirs(const double *dir, int nrhs) {
  for (int r = 0; r < nrhs; ++r) {
    const double *d = dir + 3 * r;
    if (!std::isfinite(d[0]) || !std::isfinite(d[1]) || !std::isfinite(d[2]))
      return fail(RTTDA_E_INVAL, "direction %d not finite", r);
    const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (std::fabs(n2 - 1.0) > 1e-12) return fail(RTTDA_E_INVAL, "direction %d is not a unit vector", r);
  }
  return RTTDA_OK;
}

// Scratch bytes handed to the exchange: the GEMM path sizes its Q chunk from them.  The chunk
// length is fixed per context (what the scratch holds at the largest RHS count, or the tuned
// chunk), so a batch and a single RHS sum their Q chunks identically.
size_t scratch_for(const rttda_ctx *ctx, int ns) {
  if (ctx->L.scratch_bytes == 0) return 0;
  const size_t per_q_max = (size_t)ctx->v * (2 * (size_t)ctx->R) * ctx->o * 4;
  size_t qc = std::max<size_t>(1, ctx->L.scratch_bytes / per_q_max);
  if (ctx->qchunk > 0) qc = std::min(qc, (size_t)ctx->qchunk);
  return qc * (size_t)ctx->v * ns * ctx->o * 4;
}

// Coulomb + exchange partials for the current stage input (x32 or xhi/xlo), `ns` real slices
// (2 per RHS for the complex RK4 stages, 1 per RHS for the split-operator half steps).
rttda_status enqueue_two_electron(rttda_ctx *ctx, int ns) {
  if (ctx->nq == 0) return RTTDA_OK;
  const int ov = (int)ctx->ov;
  hipStream_t s = ctx->stream;
  const bool pr = ctx->prof.on;
  if (ctx->small) {
    if (pr) HIP_TRY(ctx->prof.begin(PC_EXCHANGE, s));
    HIP_TRY(launch_small_2e(s, ctx->d.b_dtype, ctx->d.b_ov, ctx->d.b_oo, ctx->d.b_vv, ctx->x32(), ctx->o, ctx->v,
                            ctx->nq, ns, ctx->small_splits, (float)ctx->d.cx, ctx->P()));
    if (pr) HIP_TRY(ctx->prof.end(PC_EXCHANGE, s));
    return RTTDA_OK;
  }
  // the Coulomb pair and the exchange read the same stage copy and write disjoint partial slabs
  const bool fork = ctx->aux != nullptr && ctx->overlap == 1;
  hipStream_t sc = fork ? ctx->aux : s;
  if (fork) {
    HIP_TRY(hipEventRecord(ctx->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0));
  }
  if (pr) HIP_TRY(ctx->prof.begin(PC_COULOMB, sc));
  if (ctx->coul_mfma) {
    HIP_TRY(launch_coulomb_mfma(sc, ctx->d.b_dtype, ctx->d.b_ov, ctx->x32(), ctx->nq, ov, ns,
                                coulomb_mfma_chunks(ctx->nq, ov), ctx->sj, ctx->dvec(), ctx->P()));
  } else {
    const int nes = gemv1_chunks(ctx->nq, ov);
    HIP_TRY(launch_gemv1(sc, ctx->d.b_dtype, ctx->d.b_ov, ctx->x32(), ctx->nq, ov, ns, nes, ctx->dvec()));
    HIP_TRY(launch_gemv2(sc, ctx->d.b_dtype, ctx->d.b_ov, ctx->dvec(), ctx->nq, ov, ns, ctx->sj, ctx->P()));
  }
  if (pr) HIP_TRY(ctx->prof.end(PC_COULOMB, sc));
  if (fork) HIP_TRY(hipEventRecord(ctx->ev_join, ctx->aux));
  const ExchangeVariant *x = variant_of(ctx->prec, ctx->xvar);
  float *Pk = ctx->P() + (size_t)ctx->sj * ns * ctx->ov;
  const void *X = ctx->prec == RTTDA_PREC_FP32 ? (const void *)ctx->x32() : (const void *)ctx->xhi();
  const void *Xlo = ctx->prec == RTTDA_PREC_FP32 ? nullptr : (const void *)ctx->xlo();
  if (pr) HIP_TRY(ctx->prof.begin(PC_EXCHANGE, s));
  HIP_TRY(x->launch(s, ctx->d.b_oo, ctx->d.b_vv, X, Xlo, ctx->o, ctx->v, ctx->nq, ns, ctx->sk, (float)(-ctx->d.cx),
                    Pk, ctx->scratch(), scratch_for(ctx, ns)));
  if (pr) HIP_TRY(ctx->prof.end(PC_EXCHANGE, s));
  if (fork) HIP_TRY(hipStreamWaitEvent(s, ctx->ev_join, 0));  // join before any reader of the slabs
  return RTTDA_OK;
}

int nslab(const rttda_ctx *ctx) { return ctx->nq > 0 ? (ctx->small ? ctx->small_splits : ctx->sj + ctx->sk) : 0; }

// the small path applies to the shape (o v and the RHS count within its single-workgroup limits)
bool small_fits(int o, int v, int R) { return small_shape_ok(o, v) && R <= SMALL_R_MAX; }

// One RK4 step (4 stages) on the context's stream.
rttda_status enqueue_step(rttda_ctx *ctx, int nrhs, double dt, bool has_field, bool corr, bool pops, bool energy,
                          double *c0, double *c) {
  hipStream_t s = ctx->stream;
  const int o = ctx->o, v = ctx->v;
  if (ctx->small) {  // two launches per stage
    for (int stage = 0; stage < 4; ++stage) {
      double *Xin = stage == 0 ? c : ctx->xs64();
      rttda_status st = enqueue_two_electron(ctx, 2 * nrhs);
      if (st != RTTDA_OK) return st;
      const bool pr = ctx->prof.on;
      if (pr) HIP_TRY(ctx->prof.begin(PC_EPILOGUE, s));
      if (corr && stage == 0) HIP_TRY(launch_corr(s, nrhs, ctx->ov, c, c0, ctx->xref(), ctx->xref0(), ctx->state()));
      if (pops && stage == 0) HIP_TRY(launch_pop(s, nrhs, ctx->ov, c, ctx->state()));
      HIP_TRY(launch_small_epi(s, ctx->prec, nrhs, o, v, nslab(ctx), stage, has_field ? 1 : 0, stage == 0 ? 1 : 0, dt,
                               ctx->pulses(), ctx->state(), ctx->D(), ctx->P(), ctx->moo(), ctx->mov(), ctx->mvv(), Xin,
                               c, c0, ctx->acc(), ctx->acc0(), ctx->xs64(), ctx->xs0(), ctx->x32(), ctx->xhi(),
                               ctx->xlo(), ctx->normref()));
      if (pr) HIP_TRY(ctx->prof.end(PC_EPILOGUE, s));
    }
    (void)energy;  // the small epilogue writes the energy sample itself (stage 0)
    return RTTDA_OK;
  }
  for (int stage = 0; stage < 4; ++stage) {
    double *Xin = stage == 0 ? c : ctx->xs64();
    double *X0 = stage == 0 ? c0 : ctx->xs0();
    rttda_status st = enqueue_two_electron(ctx, 2 * nrhs);
    if (st != RTTDA_OK) return st;
    const bool need_field = stage == 0 || has_field;
    const bool pr = ctx->prof.on;
    if (need_field) {
      if (pr) HIP_TRY(ctx->prof.begin(PC_FIELD, s));
      HIP_TRY(launch_field(s, Xin, X0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
      if (pr) HIP_TRY(ctx->prof.end(PC_FIELD, s));
    }
    if (pr) HIP_TRY(ctx->prof.begin(PC_EPILOGUE, s));
    int mode = 0;
    if (stage == 0) mode |= SM_TRACE;
    if (has_field) mode |= SM_C0 | SM_EFIELD;
    if (stage == 3) mode |= SM_INC;
    if (stage == 1 && energy) mode |= SM_ENERGY;  // the sample of this step, from stage 0's partials
    HIP_TRY(launch_scalar(s, nrhs, ctx->L.nbf, stage, mode, dt, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(),
                          c0, ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
    if (corr && stage == 0) HIP_TRY(launch_corr(s, nrhs, ctx->ov, c, c0, ctx->xref(), ctx->xref0(), ctx->state()));
    if (pops && stage == 0) HIP_TRY(launch_pop(s, nrhs, ctx->ov, c, ctx->state()));
    HIP_TRY(launch_epilogue(s, ctx->prec, nrhs, o, v, nslab(ctx), stage, EP_RK4, has_field ? 1 : 0, dt, ctx->D(),
                            ctx->P(), ctx->F(), ctx->sc(), Xin, c, ctx->acc(), ctx->xs64(), ctx->x32(), ctx->xhi(),
                            ctx->xlo(), nullptr, energy && stage == 0 ? ctx->epart() : nullptr));
    if (pr) HIP_TRY(ctx->prof.end(PC_EPILOGUE, s));
  }
  return RTTDA_OK;
}

// One symplectic split-operator step (k_sso_update): trace sample at the step start, drift with
// H(t_n + dt/2) p_h, kick with H(t_n + dt) q_{n+1}.  Field products only when a pulse is on.
rttda_status enqueue_sso_step(rttda_ctx *ctx, int nrhs, double dt, bool has_field, bool corr, bool pops, double *c0,
                              double *c) {
  hipStream_t s = ctx->stream;
  const int o = ctx->o, v = ctx->v;
  const bool pr = ctx->prof.on;
  double *W = ctx->xs64(), *W0 = ctx->xs0();
  rttda_status st;
  if (pr) HIP_TRY(ctx->prof.begin(PC_FIELD, s));
  HIP_TRY(launch_field(s, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
  HIP_TRY(launch_scalar(s, nrhs, ctx->L.nbf, 0, SM_TRACE, dt, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(), c0,
                        ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
  if (corr) HIP_TRY(launch_corr(s, nrhs, ctx->ov, c, c0, ctx->xref(), ctx->xref0(), ctx->state()));
  if (pops) HIP_TRY(launch_pop(s, nrhs, ctx->ov, c, ctx->state()));
  if (pr) HIP_TRY(ctx->prof.end(PC_FIELD, s));
  for (int half = 0; half < 2; ++half) {  // 0: drift (stage node 1/2), 1: kick (node 1)
    if ((st = enqueue_two_electron(ctx, nrhs)) != RTTDA_OK) return st;
    if (pr) HIP_TRY(ctx->prof.begin(PC_EPILOGUE, s));
    if (has_field)
      HIP_TRY(launch_field(s, W, W0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
    if (has_field || half == 1)
      HIP_TRY(launch_scalar(s, nrhs, ctx->L.nbf, half == 0 ? 1 : 3,
                            (has_field ? SM_EFIELD : 0) | (half == 1 ? SM_INC : 0), dt, ctx->pulses(), ctx->state(),
                            ctx->part(), ctx->sc(), c0, ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
    HIP_TRY(launch_sso_update(s, ctx->prec, nrhs, o, v, nslab(ctx), half == 0 ? SSO_DRIFT : SSO_KICK,
                              has_field ? 1 : 0, dt, ctx->D(), ctx->P(), ctx->F(), ctx->sc(), c, c0, W, W0, ctx->x32(),
                              ctx->xhi(), ctx->xlo()));
    if (pr) HIP_TRY(ctx->prof.end(PC_EPILOGUE, s));
  }
  return RTTDA_OK;
}

// First half kick of a split-operator call: W = (q, p - dt/2 H(t_step0) q), x32 = FP32(p_h).
rttda_status enqueue_sso_start(rttda_ctx *ctx, int nrhs, double dt, bool has_field, double *c0, double *c) {
  hipStream_t s = ctx->stream;
  HIP_TRY(launch_plane_copy(s, ctx->prec, nrhs, ctx->ov, 0, c, ctx->x32(), ctx->xhi(), ctx->xlo()));
  rttda_status st = enqueue_two_electron(ctx, nrhs);
  if (st != RTTDA_OK) return st;
  if (has_field)
    HIP_TRY(launch_field(s, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), ctx->o, ctx->v, nrhs, ctx->F(), ctx->part()));
  HIP_TRY(launch_scalar(s, nrhs, ctx->L.nbf, 0, has_field ? SM_EFIELD : 0, dt, ctx->pulses(), ctx->state(),
                        ctx->part(), ctx->sc(), c0, ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
  HIP_TRY(launch_sso_update(s, ctx->prec, nrhs, ctx->o, ctx->v, nslab(ctx), SSO_KICK_FIRST, has_field ? 1 : 0, dt,
                            ctx->D(), ctx->P(), ctx->F(), ctx->sc(), c, c0, ctx->xs64(), ctx->xs0(), ctx->x32(),
                            ctx->xhi(), ctx->xlo()));
  return RTTDA_OK;
}

// FP32 (and BF16 hi/lo) stage copies of cnt FP64 values, cnt at most the 2R slices the buffers hold
rttda_status to_stage_copy_n(rttda_ctx *ctx, const double *c, long long cnt) {
  if (ctx->prec == RTTDA_PREC_FP32)
    HIP_TRY(launch_to_f32(ctx->stream, c, cnt, ctx->x32()));
  else
    HIP_TRY(launch_to_bf16x2(ctx->stream, c, cnt, ctx->x32(), ctx->xhi(), ctx->xlo()));
  return RTTDA_OK;
}

rttda_status to_stage_copy(rttda_ctx *ctx, const double *c, int nrhs) {
  const long long n = 2LL * nrhs * (long long)ctx->ov;
  if (ctx->prec == RTTDA_PREC_FP32)
    HIP_TRY(launch_to_f32(ctx->stream, c, n, ctx->x32()));
  else
    HIP_TRY(launch_to_bf16x2(ctx->stream, c, n, ctx->x32(), ctx->xhi(), ctx->xlo()));
  return RTTDA_OK;
}

void drop_graph(rttda_ctx *ctx) {
  if (ctx->graph.valid && ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
  ctx->graph = GraphEntry{};
}

// Symmetric tridiagonal T (diagonal a[0..k-1], off-diagonal b[0..k-2]): number of eigenvalues
// below x by the Sturm sequence of the LDL^T pivots.
int sturm_below(const std::vector<double> &a, const std::vector<double> &b, double x) {
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// The m-th smallest eigenvalue of T (m = 0..k-1) by bisection inside the Gershgorin interval.
double tridiag_eig(const std::vector<double> &a, const std::vector<double> &b, int m) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi) + std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, mid) > m) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for eigenvalue theta (inverse iteration with the
// tridiagonal solve of (T - mu I) y = x, mu = theta slightly shifted).
// Eigen-decomposition of a symmetric m x m matrix (row-major, overwritten) by cyclic Jacobi
// rotations: w ascending, z the matching eigenvectors as columns (row-major m x m).
void jacobi_eig(int m, std::vector<double> &a, std::vector<double> &w, std::vector<double> &z) {
  z.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) z[(size_t)i * m + i] = 1.0;
  double scale = 0.0;
  for (double x : a) scale += x * x;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += a[(size_t)p * m + q] * a[(size_t)p * m + q];
    if (!(off > 1e-30 * scale)) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = a[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double th = (a[(size_t)q * m + q] - a[(size_t)p * m + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < m; ++k) {  // A J
          const double akp = a[(size_t)k * m + p], akq = a[(size_t)k * m + q];
          a[(size_t)k * m + p] = c * akp - sn * akq;
          a[(size_t)k * m + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {  // J^T (A J)
          const double apk = a[(size_t)p * m + k], aqk = a[(size_t)q * m + k];
          a[(size_t)p * m + k] = c * apk - sn * aqk;
          a[(size_t)q * m + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {  // Z J
          const double zkp = z[(size_t)k * m + p], zkq = z[(size_t)k * m + q];
          z[(size_t)k * m + p] = c * zkp - sn * zkq;
          z[(size_t)k * m + q] = sn * zkp + c * zkq;
        }
      }
  }
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return a[(size_t)x * m + x] < a[(size_t)y * m + y]; });
  std::vector<double> zs((size_t)m * m);
  w.resize(m);
  for (int j = 0; j < m; ++j) {
    w[j] = a[(size_t)ord[j] * m + ord[j]];
    for (int k = 0; k < m; ++k) zs[(size_t)k * m + j] = z[(size_t)k * m + ord[j]];
  }
  z.swap(zs);
}

// Layout of the eigen-solver workspace: V, W (search space and its image, m_max vectors each),
// Z (2k Ritz vectors, their images, k residuals / corrections), the diagonal of A, small arrays.
struct EigLayout {
  size_t V, W, Z, diag, C, theta, dots, part, total;
};
EigLayout eig_layout(size_t n, int k, int m_max) {
  EigLayout e{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += up(bytes > 0 ? bytes : 1);
    return at;
  };
  e.V = take((size_t)m_max * n * 8);
  e.W = take((size_t)m_max * n * 8);
  e.Z = take((size_t)5 * k * n * 8);
  e.diag = take(n * 8);
  e.C = take((size_t)m_max * m_max * 8);
  e.theta = take((size_t)m_max * 8);
  e.dots = take((size_t)m_max * m_max * 8);
  e.part = take((size_t)std::max(m_max, 3 * k) * DV_BLOCKS_MAX * 8);
  e.total = off;
  return e;
}

double tridiag_last_component(const std::vector<double> &a, const std::vector<double> &b, double theta) {
  const size_t k = a.size();
  const double mu = theta + 1e-10 * std::max(1.0, std::fabs(theta));
  std::vector<double> x(k, 1.0), c(k), d(k);
  for (int it = 0; it < 4; ++it) {
    // Thomas algorithm on the shifted matrix
    std::vector<double> y(k);
    double den = a[0] - mu;
    if (den == 0.0) den = 1e-300;
    c[0] = k > 1 ? b[0] / den : 0.0;
    d[0] = x[0] / den;
    for (size_t i = 1; i < k; ++i) {
      den = (a[i] - mu) - b[i - 1] * c[i - 1];
      if (den == 0.0) den = 1e-300;
      c[i] = i + 1 < k ? b[i] / den : 0.0;
      d[i] = (x[i] - b[i - 1] * d[i - 1]) / den;
    }
    y[k - 1] = d[k - 1];
    for (size_t i = k - 1; i-- > 0;) y[i] = d[i] - c[i] * y[i + 1];
    double nrm = 0.0;
    for (double t : y) nrm += t * t;
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
    for (size_t i = 0; i < k; ++i) x[i] = y[i] / nrm;
  }
  return std::fabs(x[k - 1]);
}

rttda_status check_nrhs(const rttda_ctx *ctx, int nrhs) {
  if (nrhs < 1 || nrhs > ctx->R) return fail(RTTDA_E_INVAL, "nrhs=%d outside 1..max_rhs=%d", nrhs, ctx->R);
  return RTTDA_OK;
}

// sigma's device work once the directions (pulse table) and the E slots are on the device:
// dipole blocks, stage copy, Coulomb pair and exchange, field product, s0 and the sigma epilogue
rttda_status sigma_enqueue(rttda_ctx *ctx, int nrhs, const double *c0, const double *c, double *s0, double *s) {
  hipStream_t hs = ctx->stream;
  rttda_status st;
  HIP_TRY(launch_mu_blocks(hs, ctx->d.mu, ctx->pulses(), ctx->o, ctx->v, nrhs, ctx->moo(), ctx->mov(), ctx->mvv()));
  if ((st = to_stage_copy(ctx, c, nrhs)) != RTTDA_OK) return st;
  if ((st = enqueue_two_electron(ctx, 2 * nrhs)) != RTTDA_OK) return st;
  HIP_TRY(launch_field(hs, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), ctx->o, ctx->v, nrhs, ctx->F(), ctx->part()));
  HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, SM_SIGMA0 | SM_KEEP_E, 0.0, ctx->pulses(), ctx->state(),
                        ctx->part(), ctx->sc(), const_cast<double *>(c0), ctx->acc0(), ctx->xs0(), nullptr,
                        ctx->normref(), s0));
  HIP_TRY(launch_epilogue(hs, ctx->prec, nrhs, ctx->o, ctx->v, nslab(ctx), 0, EP_SIGMA, 1, 0.0, ctx->D(), ctx->P(),
                          ctx->F(), ctx->sc(), c, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s));
  return RTTDA_OK;
}

}  // namespace

extern "C" {

const char *rttda_last_error(void) { return g_last_error.c_str(); }
const char *rttda_version(void) { return "rttda-gfx950 0.1"; }

int32_t rttda_exchange_variants(int32_t precision) {
  if (precision != RTTDA_PREC_FP32 && precision != RTTDA_PREC_MIXED_BF16) return 0;
  return variant_count(precision);
}

const char *rttda_exchange_variant_name(int32_t precision, int32_t k) {
  if (precision != RTTDA_PREC_FP32 && precision != RTTDA_PREC_MIXED_BF16) return "";
  const ExchangeVariant *x = variant_of(precision, k - 1);
  return x ? x->name : "";
}

rttda_status rttda_workspace_bytes(const rttda_desc *desc, size_t *bytes) {
  rttda_status st = validate_desc(desc, false);
  if (st != RTTDA_OK) return st;
  if (!bytes) return fail(RTTDA_E_INVAL, "bytes is NULL");
  *bytes = make_layout(desc->n_occ, desc->n_virt, desc->n_aux, desc->max_rhs, desc->precision).total;
  return RTTDA_OK;
}

rttda_status rttda_create(const rttda_desc *desc, rttda_ctx **out) {
  if (!out) return fail(RTTDA_E_INVAL, "out is NULL");
  *out = nullptr;
  rttda_status st = validate_desc(desc, true);
  if (st != RTTDA_OK) return st;
  Layout L = make_layout(desc->n_occ, desc->n_virt, desc->n_aux, desc->max_rhs, desc->precision);
  if (desc->workspace_bytes < L.total)
    return fail(RTTDA_E_NOMEM, "workspace has %zu bytes, needs %zu", desc->workspace_bytes, L.total);
  const int ns_max = 2 * desc->max_rhs;
  int xv = -1;
  if (desc->n_aux > 0) {
    xv = auto_variant(desc->precision, desc->n_occ, ns_max, desc->n_virt, L);
    if (xv < 0)
      return fail(RTTDA_E_UNSUPPORTED, "no exchange kernel for o=%d in precision %d", desc->n_occ, desc->precision);
  }
  if (xv >= 0) HIP_TRY(variant_of(desc->precision, xv)->prepare());
  HIP_TRY(prepare_small());
  rttda_ctx *ctx = new rttda_ctx();
  ctx->d = *desc;
  ctx->stream = static_cast<hipStream_t>(desc->stream);
  ctx->o = desc->n_occ;
  ctx->v = desc->n_virt;
  ctx->nq = desc->n_aux;
  ctx->R = desc->max_rhs;
  ctx->prec = desc->precision;
  ctx->ov = (size_t)ctx->o * ctx->v;
  ctx->L = L;
  ctx->ws = static_cast<char *>(desc->workspace);
  ctx->xvar = xv;
  if (desc->n_aux > 0) {
    ctx->sk = auto_splits(variant_of(ctx->prec, xv), ctx->o, ns_max, ctx->v, ctx->nq, L.sk_max, L);
    ctx->sj = L.sj_max;
    // the Coulomb pair runs alongside the exchange only where the exchange is long enough to
    // cover the cost of the fork and join (small problems and many concurrent contexts lose)
    ctx->overlap = 4.0 * ctx->nq * (double)ctx->ov * (ctx->o + ctx->v) * ctx->R >= OVERLAP_MIN_FLOPS ? 1 : 2;
    // the small path: at most 2e9 exchange flops per stage (a few tens of microseconds of FP32 FMA);
    // up to SMALL_SPLITS Q ranges (the epilogue adds one slab per range)
    ctx->small_splits = std::max(1, std::min({SMALL_SPLITS, ctx->nq, L.sj_max + L.sk_max}));
    ctx->coul_mfma = 2 * ctx->R >= COUL_MFMA_MIN_SLICES ? 1 : 0;
    // the default only for the smallest problems (8 launches per RK4 step instead of 21; each of
    // its launches takes longer, so from about 2e7 exchange flops per stage it loses)
    ctx->small = small_fits(ctx->o, ctx->v, ctx->R) &&
                         4.0 * ctx->nq * (double)ctx->ov * (ctx->o + ctx->v) * ctx->R <= SMALL_DEFAULT_FLOPS
                     ? 1
                     : 0;
  }
  hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&ctx->h_pulses), sizeof(DevPulse) * ctx->R);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->upload_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ctx->upload_ev, ctx->stream);
  if (e == hipSuccess) e = launch_gaps(ctx->stream, desc->e_occ, desc->e_virt, ctx->o, ctx->v, ctx->D());
  if (e == hipSuccess) e = launch_set_state(ctx->stream, ctx->state(), 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (ctx->h_pulses) (void)hipHostFree(ctx->h_pulses);
    if (ctx->upload_ev) (void)hipEventDestroy(ctx->upload_ev);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    delete ctx;
    return fail(RTTDA_E_DEVICE, "create: %s", hipGetErrorString(e));
  }
  *out = ctx;
  return RTTDA_OK;
}

rttda_status rttda_destroy(rttda_ctx *ctx) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  drop_graph(ctx);
  ctx->prof.destroy();
  if (ctx->upload_ev) (void)hipEventDestroy(ctx->upload_ev);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  if (ctx->h_pulses) (void)hipHostFree(ctx->h_pulses);
  delete ctx;
  return RTTDA_OK;
}

rttda_status rttda_set_profiling(rttda_ctx *ctx, int32_t on) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->prof.reset();
  ctx->prof.on = on != 0;
  drop_graph(ctx);
  return RTTDA_OK;
}

rttda_status rttda_get_profile(rttda_ctx *ctx, rttda_profile *out) {
  if (!ctx || !out) return fail(RTTDA_E_INVAL, "NULL argument");
  for (int k = 0; k < Profiler::CLASSES; ++k) {
    HIP_TRY(ctx->prof.fold(k));
    out->launches[k] = ctx->prof.launches[k];
    out->ms[k] = ctx->prof.ms[k];
  }
  return RTTDA_OK;
}

rttda_status rttda_set_stream(rttda_ctx *ctx, void *stream) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(stream);
  drop_graph(ctx);
  return RTTDA_OK;
}

rttda_status rttda_set_tuning(rttda_ctx *ctx, const rttda_tuning *t) {
  if (!ctx || !t) return fail(RTTDA_E_INVAL, "NULL argument");
  int xv = ctx->xvar, sk = ctx->sk, sj = ctx->sj;
  if (t->exchange_variant) {
    const ExchangeVariant *x = variant_of(ctx->prec, t->exchange_variant - 1);
    if (!x) return fail(RTTDA_E_UNSUPPORTED, "exchange variant %d does not exist", t->exchange_variant);
    if (!usable(x, ctx->o, ctx->v, ctx->L))
      return fail(RTTDA_E_UNSUPPORTED, "variant %s does not apply to o=%d v=%d", x->name, ctx->o, ctx->v);
    HIP_TRY(x->prepare());
    xv = t->exchange_variant - 1;
  }
  if (t->exchange_splits) {
    if (t->exchange_splits < 1 || t->exchange_splits > ctx->L.sk_max)
      return fail(RTTDA_E_NOMEM, "exchange_splits %d outside 1..%d", t->exchange_splits, ctx->L.sk_max);
    sk = t->exchange_splits;
  }
  if (t->coulomb_splits) {
    if (t->coulomb_splits < 1 || t->coulomb_splits > ctx->L.sj_max)
      return fail(RTTDA_E_NOMEM, "coulomb_splits %d outside 1..%d", t->coulomb_splits, ctx->L.sj_max);
    sj = t->coulomb_splits;
  }
  if (t->use_graph && t->use_graph != 1 && t->use_graph != 2) return fail(RTTDA_E_INVAL, "use_graph must be 0, 1 or 2");
  if (t->steps_per_graph < 0 || t->steps_per_graph > 1024) return fail(RTTDA_E_INVAL, "steps_per_graph outside 0..1024");
  if (t->exchange_chunk < -1) return fail(RTTDA_E_INVAL, "exchange_chunk must be -1, 0 or positive");
  if (ctx->nq > 0) {
    ctx->xvar = xv;
    ctx->sk = sk;
    ctx->sj = sj;
  }
  if (t->exchange_chunk) ctx->qchunk = t->exchange_chunk < 0 ? 0 : t->exchange_chunk;
  if (t->use_graph) ctx->use_graph = t->use_graph;
  if (t->overlap) {
    if (t->overlap != 1 && t->overlap != 2) return fail(RTTDA_E_INVAL, "overlap must be 0, 1 or 2");
    ctx->overlap = t->overlap;
  }
  // an explicit exchange tile or split count asks for the general kernels
  if ((t->exchange_variant || t->exchange_splits) && !t->small_path) ctx->small = 0;
  if (t->coulomb_path) {
    if (t->coulomb_path != 1 && t->coulomb_path != 2) return fail(RTTDA_E_INVAL, "coulomb_path must be 0, 1 or 2");
    ctx->coul_mfma = t->coulomb_path == 2 ? 1 : 0;
  }
  if (t->small_path) {
    if (t->small_path != 1 && t->small_path != 2) return fail(RTTDA_E_INVAL, "small_path must be 0, 1 or 2");
    if (t->small_path == 1 && (!small_fits(ctx->o, ctx->v, ctx->R) || ctx->nq == 0))
      return fail(RTTDA_E_UNSUPPORTED, "the small path takes o*v <= %d, max_rhs <= %d and n_aux > 0", SMALL_OV_MAX,
                  SMALL_R_MAX);
    ctx->small = t->small_path == 1 ? 1 : 0;
  }
  if (t->steps_per_graph) ctx->steps_per_graph = t->steps_per_graph;
  drop_graph(ctx);
  return RTTDA_OK;
}

rttda_status rttda_get_tuning(const rttda_ctx *ctx, rttda_tuning *t) {
  if (!ctx || !t) return fail(RTTDA_E_INVAL, "NULL argument");
  t->exchange_variant = ctx->xvar + 1;
  t->exchange_splits = ctx->sk;
  t->coulomb_splits = ctx->sj;
  t->use_graph = ctx->use_graph;
  t->steps_per_graph = ctx->steps_per_graph;
  t->exchange_chunk = ctx->qchunk;
  t->overlap = ctx->overlap;
  t->small_path = ctx->small ? 1 : 2;
  t->coulomb_path = ctx->coul_mfma ? 2 : 1;
  return RTTDA_OK;
}

rttda_status rttda_exchange_splits_max(const rttda_ctx *ctx, int32_t *out) {
  if (!ctx || !out) return fail(RTTDA_E_INVAL, "NULL argument");
  *out = ctx->L.sk_max;
  return RTTDA_OK;
}

rttda_status rttda_sigma(rttda_ctx *ctx, int32_t nrhs, const double *field, const double *dir, const double *c0,
                         const double *c, double *s0, double *s) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  rttda_status st = check_nrhs(ctx, nrhs);
  if (st != RTTDA_OK) return st;
  if (!field || !dir || !c0 || !c || !s0 || !s) return fail(RTTDA_E_INVAL, "NULL array argument");
  if (!aligned16(c0) || !aligned16(c) || !aligned16(s0) || !aligned16(s))
    return fail(RTTDA_E_INVAL, "device arrays must be 16-byte aligned");
  if ((st = check_dirs(dir, nrhs)) != RTTDA_OK) return st;
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(field[r])) return fail(RTTDA_E_INVAL, "field %d not finite", r);
  std::vector<DevPulse> p(nrhs);
  std::vector<double> sc((size_t)nrhs * SC_STRIDE, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    memset(&p[r], 0, sizeof(DevPulse));
    p[r].kind = RTTDA_PULSE_NONE;
    memcpy(p[r].dir, dir + 3 * r, 3 * sizeof(double));
    sc[(size_t)r * SC_STRIDE + SC_E] = field[r];
  }
  if ((st = upload_pulses(ctx, p.data(), nrhs)) != RTTDA_OK) return st;
  hipStream_t hs = ctx->stream;
  // the E slots: host values, synchronous copy (tiny) keeps the vector's lifetime simple
  HIP_TRY(hipMemcpyAsync(ctx->sc(), sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  drop_graph(ctx);
  return sigma_enqueue(ctx, nrhs, c0, c, s0, s);
}

rttda_status rttda_dipole_trace(rttda_ctx *ctx, int32_t nrhs, const double *dir, const double *c0, const double *c,
                                double *out) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  rttda_status st = check_nrhs(ctx, nrhs);
  if (st != RTTDA_OK) return st;
  if (!dir || !c0 || !c || !out) return fail(RTTDA_E_INVAL, "NULL array argument");
  if (!aligned16(c0) || !aligned16(c) || !aligned16(out))
    return fail(RTTDA_E_INVAL, "device arrays must be 16-byte aligned");
  if ((st = check_dirs(dir, nrhs)) != RTTDA_OK) return st;
  std::vector<DevPulse> p(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    memset(&p[r], 0, sizeof(DevPulse));
    memcpy(p[r].dir, dir + 3 * r, 3 * sizeof(double));
  }
  if ((st = upload_pulses(ctx, p.data(), nrhs)) != RTTDA_OK) return st;
  drop_graph(ctx);
  hipStream_t hs = ctx->stream;
  HIP_TRY(launch_mu_blocks(hs, ctx->d.mu, ctx->pulses(), ctx->o, ctx->v, nrhs, ctx->moo(), ctx->mov(), ctx->mvv()));
  HIP_TRY(launch_field(hs, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), ctx->o, ctx->v, nrhs, ctx->F(), ctx->part()));
  HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, SM_OUT, 0.0, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(),
                        const_cast<double *>(c0), ctx->acc0(), ctx->xs0(), out, ctx->normref(), nullptr));
  return RTTDA_OK;
}

}  // extern "C"

namespace {

enum : int { INTEG_RK4 = 0, INTEG_SSO = 1 };

// Unitary kick exp(i kappa M) X for the RHS with PULSE_DELTA_EXACT, as the Taylor series
// sum_j (i kappa M)^j X / j!.  |M X| <= (|mu_oo|_F + |mu_vv|_F + 2 sqrt2 |mu_ov|_F) |X| = b |X|,
// so J terms leave at most x^(J+1)/(J+1)! e^x of |X| with x = kappa b; J is the smallest with
// that below 1e-17.  exact_kick_terms finds J from the dipole blocks of this call (it reads them
// back, so it synchronises) and refuses before anything touches the state; exact_kick_apply runs
// the series, with the terms in the stage buffers (xs64, xs0).
rttda_status exact_kick_terms(rttda_ctx *ctx, int nrhs, const rttda_pulse *pulses, int *terms) {
  hipStream_t hs = ctx->stream;
  const int o = ctx->o, v = ctx->v;
  const long long ov = (long long)ctx->ov;
  double x = 0.0;
  std::vector<double> hp;
  for (int r = 0; r < nrhs; ++r) {
    if (pulses[r].kind != RTTDA_PULSE_DELTA_EXACT) continue;
    const double *blk[3] = {ctx->moo() + (size_t)r * o * o, ctx->mov() + (size_t)r * ov, ctx->mvv() + (size_t)r * v * v};
    const long long len[3] = {(long long)o * o, ov, (long long)v * v};
    double fro[3];
    for (int b = 0; b < 3; ++b) {
      HIP_TRY(launch_dv_norm2(hs, len[b], blk[b], ctx->lzp()));
      const int nb = dv_blocks(len[b]);
      hp.resize(nb);
      HIP_TRY(hipMemcpyAsync(hp.data(), ctx->lzp(), nb * sizeof(double), hipMemcpyDeviceToHost, hs));
      HIP_TRY(hipStreamSynchronize(hs));
      double t = 0.0;
      for (double y : hp) t += y;
      fro[b] = std::sqrt(t);
    }
    x = std::max(x, std::fabs(pulses[r].e0) * (fro[0] + fro[2] + 2.0 * std::sqrt(2.0) * fro[1]));
  }
  int J = 0;
  double term = std::exp(x);  // x^(J+1)/(J+1)! e^x, updated as J grows
  for (J = 0; J < 200; ++J) {
    term *= x / (J + 1);
    if (term <= 1e-17) break;
  }
  if (J > 120)
    return fail(RTTDA_E_UNSUPPORTED, "exact kick: kappa |M| bound %.3g too large for the series (use a smaller kick)",
                x);
  *terms = J;
  return RTTDA_OK;
}

rttda_status exact_kick_apply(rttda_ctx *ctx, int nrhs, int J, double *c0, double *c) {
  hipStream_t hs = ctx->stream;
  const int o = ctx->o, v = ctx->v;
  const long long ov = (long long)ctx->ov;
  double *T = ctx->xs64(), *T0 = ctx->xs0();
  HIP_TRY(hipMemcpyAsync(T, c, (size_t)2 * nrhs * ov * sizeof(double), hipMemcpyDeviceToDevice, hs));
  HIP_TRY(hipMemcpyAsync(T0, c0, (size_t)2 * nrhs * sizeof(double), hipMemcpyDeviceToDevice, hs));
  for (int j = 1; j <= J; ++j) {
    HIP_TRY(launch_field(hs, T, T0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
    HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, 0, 0.0, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(), T0,
                          ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
    HIP_TRY(launch_kick_term(hs, nrhs, (int)ov, ctx->pulses(), ctx->F(), ctx->sc(), 1.0 / j, T, T0, c, c0));
  }
  return RTTDA_OK;
}

inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Host-side checks of a propagation request (pulses, dt, step range, state and output pointers);
// nothing is enqueued.
rttda_status check_request(int32_t nrhs, const rttda_pulse *pulses, double dt, int64_t step0, int64_t n_steps,
                           const double *c0, const double *c, const double *trace, const double *norms,
                           bool *has_field, bool *has_kick, bool *has_exact) {
  if (!pulses || !c0 || !c) return fail(RTTDA_E_INVAL, "NULL argument (pulses, c0 and c are required)");
  if (!aligned16(c0) || !aligned16(c)) return fail(RTTDA_E_INVAL, "c0 and c must be 16-byte aligned");
  // outputs are written one double at a time
  if ((trace && !aligned8(trace)) || (norms && !aligned8(norms)))
    return fail(RTTDA_E_INVAL, "trace and norms must be 8-byte aligned");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RTTDA_E_INVAL, "dt must be finite and > 0 (got %g)", dt);
  if (step0 < 0 || n_steps < 0) return fail(RTTDA_E_INVAL, "step0 and n_steps must be >= 0");
  bool f = false, k = false, e = false;
  for (int r = 0; r < nrhs; ++r) {
    const rttda_pulse &p = pulses[r];
    if (p.kind < RTTDA_PULSE_NONE || p.kind > RTTDA_PULSE_DELTA_EXACT) return fail(RTTDA_E_INVAL, "pulse %d: bad kind", r);
    if (p.reserved != 0) return fail(RTTDA_E_INVAL, "pulse %d: reserved field must be 0", r);
    const double vals[] = {p.e0, p.omega, p.t0, p.fwhm, p.beta, p.phase};
    for (double x : vals)
      if (!std::isfinite(x)) return fail(RTTDA_E_INVAL, "pulse %d: non-finite parameter", r);
    if ((p.kind == RTTDA_PULSE_GAUSS || p.kind == RTTDA_PULSE_CHIRP) && !(p.fwhm > 0))
      return fail(RTTDA_E_INVAL, "pulse %d: fwhm must be > 0", r);
    if (check_dirs(p.dir, 1) != RTTDA_OK) return fail(RTTDA_E_INVAL, "pulse %d: dir is not a unit vector", r);
    f |= (p.kind == RTTDA_PULSE_CW || p.kind == RTTDA_PULSE_GAUSS || p.kind == RTTDA_PULSE_CHIRP);
    k |= (p.kind == RTTDA_PULSE_DELTA && p.e0 != 0.0);
    e |= (p.kind == RTTDA_PULSE_DELTA_EXACT && p.e0 != 0.0);
  }
  if (has_field) *has_field = f;
  if (has_kick) *has_kick = k;
  if (has_exact) *has_exact = e;
  return RTTDA_OK;
}

// resume: the call continues a run of earlier calls on this context (the serving pool's chunks):
// the norm guard keeps its reference norm and first bad step across the calls.
rttda_status propagate_impl(rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses, double dt, int64_t step0,
                            int64_t n_steps, double *c0, double *c, double *trace, double *norms, int integ,
                            bool resume = false) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  double *corr = ctx->corr_next;  // the pending outputs apply to this call only
  ctx->corr_next = nullptr;
  double *pops = ctx->pops_next;
  const double *popU = ctx->popU_next;
  const int popk = ctx->popk_next;
  ctx->pops_next = nullptr;
  ctx->popU_next = nullptr;
  ctx->popk_next = 0;
  double *energy = ctx->energy_next;
  ctx->energy_next = nullptr;
  rttda_status st = check_nrhs(ctx, nrhs);
  if (st != RTTDA_OK) return st;
  bool has_field = false, has_kick = false, has_exact = false;
  if ((st = check_request(nrhs, pulses, dt, step0, n_steps, c0, c, trace, norms, &has_field, &has_kick,
                          &has_exact)) != RTTDA_OK)
    return st;
  if ((corr && !aligned8(corr)) || (pops && !aligned8(pops)) || (energy && !aligned8(energy)))
    return fail(RTTDA_E_INVAL, "correlation, population and energy outputs must be 8-byte aligned");
  if (energy && integ != INTEG_RK4)
    return fail(RTTDA_E_UNSUPPORTED, "the energy output is produced by the RK4 integrator only");
  if ((st = upload_pulses(ctx, reinterpret_cast<const DevPulse *>(pulses), nrhs)) != RTTDA_OK) return st;
  hipStream_t hs = ctx->stream;
  const int o = ctx->o, v = ctx->v;
  HIP_TRY(launch_mu_blocks(hs, ctx->d.mu, ctx->pulses(), o, v, nrhs, ctx->moo(), ctx->mov(), ctx->mvv()));
  int kick_terms = 0;
  if (has_exact && step0 == 0 && (st = exact_kick_terms(ctx, nrhs, pulses, &kick_terms)) != RTTDA_OK) return st;
  // from here on the call changes the state
  HIP_TRY(launch_set_state(hs, ctx->state(), step0, trace, norms, corr, pops, popU, popk, energy, ctx->epart(),
                           epilogue_blocks((long long)ctx->ov), resume ? 1 : 0));
  if (has_kick && step0 == 0) {
    HIP_TRY(launch_field(hs, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
    HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, 0, dt, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(), c0,
                          ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
    HIP_TRY(launch_kick(hs, nrhs, (int)ctx->ov, ctx->pulses(), ctx->F(), ctx->sc(), c, c0));
  }
  if (has_exact && step0 == 0 && (st = exact_kick_apply(ctx, nrhs, kick_terms, c0, c)) != RTTDA_OK) return st;
  if (corr) {  // reference state of the time-correlation function: the state after the kicks
    HIP_TRY(hipMemcpyAsync(ctx->xref(), c, (size_t)2 * nrhs * ctx->ov * sizeof(double), hipMemcpyDeviceToDevice, hs));
    HIP_TRY(hipMemcpyAsync(ctx->xref0(), c0, (size_t)2 * nrhs * sizeof(double), hipMemcpyDeviceToDevice, hs));
  }
  if (integ == INTEG_SSO)
    st = enqueue_sso_start(ctx, nrhs, dt, has_field, c0, c);
  else
    st = to_stage_copy(ctx, c, nrhs);
  if (st != RTTDA_OK) return st;
  auto step = [&]() {
    return integ == INTEG_SSO ? enqueue_sso_step(ctx, nrhs, dt, has_field, corr != nullptr, pops != nullptr, c0, c)
                              : enqueue_step(ctx, nrhs, dt, has_field, corr != nullptr, pops != nullptr,
                                             energy != nullptr, c0, c);
  };

  const int spg = ctx->steps_per_graph;
  const bool graph_ok = ctx->use_graph == 1 && !ctx->prof.on && hs != nullptr && n_steps >= 2LL * spg;
  int64_t done = 0;
  if (graph_ok) {
    const int mode = has_field ? 1 : 0;
    GraphEntry &G = ctx->graph;
    const bool hit = G.valid && G.nrhs == nrhs && G.steps == spg && G.mode == mode && G.integ == integ &&
                     G.dt == dt && G.c0 == c0 && G.c == c && G.trace == (trace != nullptr) &&
                     G.norms == (norms != nullptr) && G.corr == (corr != nullptr) && G.pops == (pops != nullptr) &&
                     G.energy == (energy != nullptr);
    if (!hit) {
      drop_graph(ctx);
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
      rttda_status cst = RTTDA_OK;
      for (int k = 0; k < spg && cst == RTTDA_OK; ++k) cst = step();
      hipError_t ee = hipStreamEndCapture(hs, &graph);
      if (cst != RTTDA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return cst;
      }
      if (ee != hipSuccess) return fail(RTTDA_E_DEVICE, "graph capture: %s", hipGetErrorString(ee));
      hipGraphExec_t exec = nullptr;
      ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ee != hipSuccess) return fail(RTTDA_E_DEVICE, "graph instantiate: %s", hipGetErrorString(ee));
      G.valid = true;
      G.exec = exec;
      G.nrhs = nrhs;
      G.steps = spg;
      G.mode = mode;
      G.integ = integ;
      G.dt = dt;
      G.c0 = c0;
      G.c = c;
      G.trace = trace != nullptr;
      G.norms = norms != nullptr;
      G.corr = corr != nullptr;
      G.pops = pops != nullptr;
      G.energy = energy != nullptr;
    }
    const int64_t reps = n_steps / spg;
    for (int64_t k = 0; k < reps; ++k) HIP_TRY(hipGraphLaunch(G.exec, hs));
    done = reps * spg;
  }
  for (int64_t k = done; k < n_steps; ++k)
    if ((st = step()) != RTTDA_OK) return st;
  // final samples at step0 + n_steps
  if (corr) HIP_TRY(launch_corr(hs, nrhs, ctx->ov, c, c0, ctx->xref(), ctx->xref0(), ctx->state()));
  if (pops) HIP_TRY(launch_pop(hs, nrhs, ctx->ov, c, ctx->state()));
  if (ctx->small && integ == INTEG_RK4) {  // the small epilogue's own sums, as at every step
    if (energy) {  // the energy sample needs one more product A c
      if ((st = to_stage_copy(ctx, c, nrhs)) != RTTDA_OK) return st;
      if ((st = enqueue_two_electron(ctx, 2 * nrhs)) != RTTDA_OK) return st;
    }
    HIP_TRY(launch_small_epi(hs, ctx->prec, nrhs, o, v, energy ? nslab(ctx) : 0, -1, 0, 1, dt, ctx->pulses(),
                             ctx->state(), ctx->D(), ctx->P(), ctx->moo(), ctx->mov(), ctx->mvv(), c, c, c0, ctx->acc(),
                             ctx->acc0(), ctx->xs64(), ctx->xs0(), ctx->x32(), ctx->xhi(), ctx->xlo(), ctx->normref()));
    return RTTDA_OK;
  }
  HIP_TRY(launch_field(hs, c, c0, ctx->moo(), ctx->mov(), ctx->mvv(), o, v, nrhs, ctx->F(), ctx->part()));
  HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, SM_TRACE, dt, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(),
                        c0, ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
  if (energy) {  // the final energy sample needs one more product A c
    if ((st = to_stage_copy(ctx, c, nrhs)) != RTTDA_OK) return st;
    if ((st = enqueue_two_electron(ctx, 2 * nrhs)) != RTTDA_OK) return st;
    HIP_TRY(launch_epilogue(hs, ctx->prec, nrhs, o, v, nslab(ctx), 0, EP_ENERGY, 0, dt, ctx->D(), ctx->P(), ctx->F(),
                            ctx->sc(), c, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            ctx->epart()));
    HIP_TRY(launch_scalar(hs, nrhs, ctx->L.nbf, 0, SM_ENERGY, dt, ctx->pulses(), ctx->state(), ctx->part(), ctx->sc(),
                          c0, ctx->acc0(), ctx->xs0(), nullptr, ctx->normref(), nullptr));
  }
  return RTTDA_OK;
}

}  // namespace

extern "C" {

rttda_status rttda_propagate(rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses, double dt, int64_t step0,
                             int64_t n_steps, double *c0, double *c, double *trace, double *norms) {
  return propagate_impl(ctx, nrhs, pulses, dt, step0, n_steps, c0, c, trace, norms, INTEG_RK4);
}

rttda_status rttda_set_correlation(rttda_ctx *ctx, double *corr) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  ctx->corr_next = corr;
  return RTTDA_OK;
}

rttda_status rttda_set_energy(rttda_ctx *ctx, double *energy) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  ctx->energy_next = energy;
  return RTTDA_OK;
}

rttda_status rttda_spectrum(void *stream, int32_t kind, const double *signal, int32_t n_t, int32_t nsig, double dt,
                            double kappa, int32_t n_omega, double omega0, double domega, int32_t average,
                            double *out) {
  if (!signal || !out) return fail(RTTDA_E_INVAL, "NULL argument");
  if (kind != 0 && kind != 1) return fail(RTTDA_E_INVAL, "kind %d: 0 (dipole trace) or 1 (time correlation)", kind);
  if (n_t < 1 || nsig < 1 || n_omega < 1) return fail(RTTDA_E_INVAL, "need n_t, nsig, n_omega >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(omega0) || !std::isfinite(domega) ||
      (kind == 0 && (!(kappa != 0.0) || !std::isfinite(kappa))))
    return fail(RTTDA_E_INVAL, "dt > 0, finite frequencies and a nonzero kappa (dipole trace) are required");
  HIP_TRY(launch_spectrum(static_cast<hipStream_t>(stream), kind, signal, n_t, nsig, dt, kappa, n_omega, omega0, domega,
                          average ? 1 : 0, out));
  return RTTDA_OK;
}

rttda_status rttda_set_populations(rttda_ctx *ctx, int32_t k, const double *evecs, double *pops) {
  if (!ctx) return fail(RTTDA_E_INVAL, "ctx is NULL");
  if (pops && (k < 1 || k > POP_MAX || !evecs))
    return fail(RTTDA_E_INVAL, "populations need 1 <= k <= %d and the vectors (k=%d)", POP_MAX, k);
  ctx->pops_next = pops;
  ctx->popU_next = pops ? evecs : nullptr;
  ctx->popk_next = pops ? k : 0;
  return RTTDA_OK;
}

rttda_status rttda_propagate_sso(rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses, double dt, int64_t step0,
                                 int64_t n_steps, double *c0, double *c, double *trace, double *norms) {
  return propagate_impl(ctx, nrhs, pulses, dt, step0, n_steps, c0, c, trace, norms, INTEG_SSO);
}

rttda_status rttda_spectral_radius(rttda_ctx *ctx, int32_t n_iter, double *rho, double *rho_bound) {
  if (!ctx || !rho || !rho_bound) return fail(RTTDA_E_INVAL, "NULL argument");
  if (n_iter < 2 || n_iter > 500) return fail(RTTDA_E_INVAL, "n_iter %d outside 2..500", n_iter);
  hipStream_t hs = ctx->stream;
  const long long n = (long long)ctx->ov;
  double *v = ctx->lz(), *vprev = v + n, *w = v + 2 * n, *part = ctx->lzp();
  const int nb = lz_blocks(n);
  std::vector<double> hp(nb);
  auto host_sum = [&](double &out) -> rttda_status {
    HIP_TRY(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    out = 0.0;
    for (double t : hp) out += t;
    return RTTDA_OK;
  };
  rttda_status st;
  double n0 = 0.0;
  HIP_TRY(launch_lz_init(hs, n, w, part));
  if ((st = host_sum(n0)) != RTTDA_OK) return st;
  HIP_TRY(hipMemsetAsync(vprev, 0, n * sizeof(double), hs));
  HIP_TRY(launch_lz_next(hs, ctx->prec, n, 1.0 / std::sqrt(n0), w, v, vprev, ctx->x32(), ctx->xhi(), ctx->xlo(), 0));
  std::vector<double> alpha, beta;
  double bj = 0.0, blast = 0.0;
  const int kmax = (int)std::min<long long>(n_iter, n);
  for (int j = 0; j < kmax; ++j) {
    if (ctx->nq > 0 && (st = enqueue_two_electron(ctx, 1)) != RTTDA_OK) return st;
    double aj = 0.0, b2 = 0.0;
    HIP_TRY(launch_lz_apply(hs, n, nslab(ctx), ctx->D(), ctx->P(), v, vprev, bj, w, part));
    if ((st = host_sum(aj)) != RTTDA_OK) return st;
    HIP_TRY(launch_lz_orth(hs, n, v, aj, w, part));
    if ((st = host_sum(b2)) != RTTDA_OK) return st;
    alpha.push_back(aj);
    const double b = std::sqrt(std::max(b2, 0.0));
    blast = b;
    if (j + 1 == kmax || !(b > 1e-13 * std::max(1.0, std::fabs(aj)))) break;  // done, or invariant subspace
    beta.push_back(b);
    HIP_TRY(launch_lz_next(hs, ctx->prec, n, 1.0 / b, w, v, vprev, ctx->x32(), ctx->xhi(), ctx->xlo(), 1));
    bj = b;
  }
  const int k = (int)alpha.size();
  const double tmin = tridiag_eig(alpha, beta, 0), tmax = tridiag_eig(alpha, beta, k - 1);
  const double emin = blast * tridiag_last_component(alpha, beta, tmin);
  const double emax = blast * tridiag_last_component(alpha, beta, tmax);
  *rho = std::max(std::fabs(tmin), std::fabs(tmax));
  *rho_bound = std::max(std::fabs(tmin) + emin, std::fabs(tmax) + emax);
  return RTTDA_OK;
}

rttda_status rttda_eigen_workspace_bytes(const rttda_ctx *ctx, int32_t k, int32_t m_max, size_t *bytes) {
  if (!ctx || !bytes) return fail(RTTDA_E_INVAL, "NULL argument");
  if (k < 1 || m_max < 3 * k || m_max > DV_SPACE_MAX || (size_t)m_max > ctx->ov)
    return fail(RTTDA_E_INVAL, "need 1 <= k, 3k <= m_max <= min(%d, o*v) (k=%d m_max=%d)", DV_SPACE_MAX, k, m_max);
  *bytes = eig_layout(ctx->ov, k, m_max).total;
  return RTTDA_OK;
}

rttda_status rttda_eigen_lowest(rttda_ctx *ctx, int32_t k, int32_t m_max, int32_t max_iter, double tol, void *work,
                                size_t work_bytes, double *evals, double *resid, double *evecs, int32_t *iters) {
  if (!ctx || !work || !evals || !resid) return fail(RTTDA_E_INVAL, "NULL argument");
  size_t need = 0;
  rttda_status st = rttda_eigen_workspace_bytes(ctx, k, m_max, &need);
  if (st != RTTDA_OK) return st;
  if (work_bytes < need) return fail(RTTDA_E_NOMEM, "eigen workspace %zu bytes < %zu needed", work_bytes, need);
  if ((reinterpret_cast<uintptr_t>(work) & (ALIGN - 1)) != 0) return fail(RTTDA_E_INVAL, "work not 256-byte aligned");
  if (max_iter < 1 || !(tol > 0.0)) return fail(RTTDA_E_INVAL, "need max_iter >= 1 and tol > 0");
  hipStream_t hs = ctx->stream;
  const long long n = (long long)ctx->ov;
  const EigLayout E = eig_layout(ctx->ov, k, m_max);
  char *wb = static_cast<char *>(work);
  double *V = reinterpret_cast<double *>(wb + E.V), *W = reinterpret_cast<double *>(wb + E.W);
  double *Xr = reinterpret_cast<double *>(wb + E.Z), *AXr = Xr + (size_t)2 * k * n, *Rr = Xr + (size_t)4 * k * n;
  double *diag = reinterpret_cast<double *>(wb + E.diag);
  double *Cd = reinterpret_cast<double *>(wb + E.C), *thd = reinterpret_cast<double *>(wb + E.theta);
  double *dotd = reinterpret_cast<double *>(wb + E.dots), *partd = reinterpret_cast<double *>(wb + E.part);
  const int nblk = dv_blocks(n);
  const int batch = 2 * ctx->R;  // real vectors per sigma launch (the stage buffers hold 2R slices)

  // diagonal of A (preconditioner and start vectors), with a host copy
  if (ctx->nq > 0)
    HIP_TRY(launch_dv_diag(hs, ctx->d.b_dtype, ctx->o, ctx->v, ctx->nq, ctx->d.b_ov, ctx->d.b_oo, ctx->d.b_vv,
                           ctx->d.cx, ctx->D(), diag));
  else
    HIP_TRY(hipMemcpyAsync(diag, ctx->D(), n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  std::vector<double> Dh(n);
  HIP_TRY(hipMemcpyAsync(Dh.data(), diag, n * sizeof(double), hipMemcpyDeviceToHost, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  auto upload = [&](double *dst, const std::vector<double> &src) -> rttda_status {
    HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    return RTTDA_OK;
  };
  auto download = [&](std::vector<double> &dst, const double *src, size_t cnt) -> rttda_status {
    dst.resize(cnt);
    HIP_TRY(hipMemcpyAsync(dst.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    return RTTDA_OK;
  };
  // W[j0..j1) = A V[j0..j1), in launches of at most `batch` vectors
  auto apply = [&](int j0, int j1) -> rttda_status {
    for (int b0 = j0; b0 < j1; b0 += batch) {
      const int nb = std::min(batch, j1 - b0);
      rttda_status s2 = to_stage_copy_n(ctx, V + (size_t)b0 * n, (long long)nb * n);
      if (s2 != RTTDA_OK) return s2;
      if (ctx->nq > 0 && (s2 = enqueue_two_electron(ctx, nb)) != RTTDA_OK) return s2;
      HIP_TRY(launch_dv_apply(hs, n, nb, nslab(ctx), ctx->D(), ctx->P(), V + (size_t)b0 * n, W + (size_t)b0 * n));
    }
    return RTTDA_OK;
  };
  std::vector<double> hbuf;
  // <V_i, T_j> for i < m, j < nt, on the host as [m][nt]
  auto dots = [&](int m, const double *T, int nt, std::vector<double> &out) -> rttda_status {
    HIP_TRY(launch_dv_dots(hs, n, m, V, nt, T, dotd));
    return download(out, dotd, (size_t)m * nt);
  };
  auto norm2 = [&](const double *T, double &out) -> rttda_status {
    HIP_TRY(launch_dv_norm2(hs, n, T, partd));
    rttda_status s2 = download(hbuf, partd, nblk);
    if (s2 != RTTDA_OK) return s2;
    out = 0.0;
    for (double t : hbuf) out += t;
    return RTTDA_OK;
  };

  // start: unit vectors at the smallest diagonal entries
  std::vector<long long> idx(n);
  for (long long e = 0; e < n; ++e) idx[e] = e;
  const int m0 = std::min(m_max / 2, std::max(k, std::min(2 * k, m_max / 2)));
  std::partial_sort(idx.begin(), idx.begin() + m0, idx.end(), [&](long long x, long long y) {
    return Dh[x] < Dh[y] || (Dh[x] == Dh[y] && x < y);
  });
  for (int j = 0; j < m0; ++j) HIP_TRY(launch_dv_unit(hs, n, idx[j], V + (size_t)j * n));
  int m = m0;
  if ((st = apply(0, m)) != RTTDA_OK) return st;
  std::vector<double> H((size_t)m_max * m_max, 0.0), d;
  if ((st = dots(m, W, m, d)) != RTTDA_OK) return st;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) H[(size_t)i * m_max + j] = 0.5 * (d[(size_t)i * m + j] + d[(size_t)j * m + i]);

  std::vector<double> theta, Y, a, rn(k, 0.0);
  int it = 0;
  for (;; ++it) {
    a.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) a[(size_t)i * m + j] = H[(size_t)i * m_max + j];
    jacobi_eig(m, a, theta, Y);
    // the nr lowest Ritz vectors X = V Y, their images A X = W Y (the first k are the answer, all
    // nr are kept at a restart), residuals R = A X - theta X of the first k
    const int nr = std::min(2 * k, m);
    std::vector<double> Ck((size_t)m * nr), thk(theta.begin(), theta.begin() + k);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < nr; ++j) Ck[(size_t)i * nr + j] = Y[(size_t)i * m + j];
    if ((st = upload(Cd, Ck)) != RTTDA_OK) return st;
    if ((st = upload(thd, thk)) != RTTDA_OK) return st;
    for (int j0 = 0; j0 < nr; j0 += 16) {
      const int nc = std::min(16, nr - j0);
      HIP_TRY(launch_dv_combine(hs, n, m, V, nc, Cd + j0, nr, 0, Xr + (size_t)j0 * n));
      HIP_TRY(launch_dv_combine(hs, n, m, W, nc, Cd + j0, nr, 0, AXr + (size_t)j0 * n));
    }
    HIP_TRY(launch_dv_resid(hs, n, k, Xr, AXr, thd, Rr, partd));
    if ((st = download(hbuf, partd, (size_t)k * nblk)) != RTTDA_OK) return st;
    std::vector<int> open;
    for (int j = 0; j < k; ++j) {
      double r2 = 0.0;
      for (int b = 0; b < nblk; ++b) r2 += hbuf[(size_t)j * nblk + b];
      rn[j] = std::sqrt(std::max(r2, 0.0));
      if (!(rn[j] <= tol)) open.push_back(j);
    }
    if (open.empty() || it + 1 >= max_iter) break;
    // corrections from the diagonal preconditioner (in place of the residuals)
    HIP_TRY(launch_dv_precond(hs, n, k, Rr, thd, diag, Rr));
    if (m + (int)open.size() > m_max) {  // restart from the nr lowest Ritz vectors and their images
      HIP_TRY(hipMemcpyAsync(V, Xr, (size_t)nr * n * sizeof(double), hipMemcpyDeviceToDevice, hs));
      HIP_TRY(hipMemcpyAsync(W, AXr, (size_t)nr * n * sizeof(double), hipMemcpyDeviceToDevice, hs));
      std::fill(H.begin(), H.end(), 0.0);
      for (int j = 0; j < nr; ++j) H[(size_t)j * m_max + j] = theta[j];
      m = nr;
    }
    const int m_old = m;
    for (int j : open) {
      double *t = Rr + (size_t)j * n;
      double n0 = 0.0, n1 = 0.0;
      if ((st = norm2(t, n0)) != RTTDA_OK) return st;
      for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt against the space, twice
        std::vector<double> c;
        if ((st = dots(m, t, 1, c)) != RTTDA_OK) return st;
        if ((st = upload(Cd, c)) != RTTDA_OK) return st;
        HIP_TRY(launch_dv_combine(hs, n, m, V, 1, Cd, 1, 1, t));
      }
      if ((st = norm2(t, n1)) != RTTDA_OK) return st;
      if (!(n1 > 1e-10 * n0) || !(n1 > 0.0)) continue;  // nothing new in this direction
      HIP_TRY(launch_dv_scale(hs, n, 1.0 / std::sqrt(n1), t, V + (size_t)m * n));
      ++m;
    }
    if (m == m_old) break;  // the space stopped growing
    if ((st = apply(m_old, m)) != RTTDA_OK) return st;
    const int nn = m - m_old;
    if ((st = dots(m, W + (size_t)m_old * n, nn, d)) != RTTDA_OK) return st;
    for (int i = 0; i < m; ++i)
      for (int jj = 0; jj < nn; ++jj) {
        const int j = m_old + jj;
        const double x = d[(size_t)i * nn + jj];
        if (i < m_old) {
          H[(size_t)i * m_max + j] = H[(size_t)j * m_max + i] = x;
        } else if (i <= j) {
          const double y = d[(size_t)j * nn + (i - m_old)];
          H[(size_t)i * m_max + j] = H[(size_t)j * m_max + i] = 0.5 * (x + y);
        }
      }
  }
  for (int j = 0; j < k; ++j) {
    evals[j] = theta[j];
    resid[j] = rn[j];
  }
  if (evecs) HIP_TRY(hipMemcpyAsync(evecs, Xr, (size_t)k * n * sizeof(double), hipMemcpyDeviceToDevice, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  if (iters) *iters = it + 1;
  return RTTDA_OK;
}

rttda_status rttda_populations(rttda_ctx *ctx, int32_t k, const double *evecs, int32_t nrhs, const double *c,
                               void *work, size_t work_bytes, double *out) {
  if (!ctx || !evecs || !c || !work || !out) return fail(RTTDA_E_INVAL, "NULL argument");
  if (k < 1 || k > DV_SPACE_MAX) return fail(RTTDA_E_INVAL, "k=%d outside 1..%d", k, DV_SPACE_MAX);
  if (nrhs < 1 || nrhs > DV_SPACE_MAX / 2) return fail(RTTDA_E_INVAL, "nrhs=%d outside 1..%d", nrhs, DV_SPACE_MAX / 2);
  const size_t need = (size_t)k * 2 * nrhs * sizeof(double);
  if (work_bytes < need) return fail(RTTDA_E_NOMEM, "populations workspace %zu bytes < %zu needed", work_bytes, need);
  hipStream_t hs = ctx->stream;
  const long long n = (long long)ctx->ov;
  double *dd = static_cast<double *>(work);
  HIP_TRY(launch_dv_dots(hs, n, k, evecs, 2 * nrhs, c, dd));
  std::vector<double> h((size_t)k * 2 * nrhs);
  HIP_TRY(hipMemcpyAsync(h.data(), dd, h.size() * sizeof(double), hipMemcpyDeviceToHost, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  for (int r = 0; r < nrhs; ++r)
    for (int i = 0; i < k; ++i) {
      const double re = h[(size_t)i * 2 * nrhs + 2 * r], im = h[(size_t)i * 2 * nrhs + 2 * r + 1];
      out[(size_t)r * k + i] = re * re + im * im;
    }
  return RTTDA_OK;
}

}  // extern "C"

struct rttda_pool {
  struct Slot {
    rttda_ctx *ctx = nullptr;
    int nrhs = 0, integ = 0;
    std::vector<rttda_pulse> pulses;
    double dt = 0.0;
    int64_t n_steps = 0, done = 0;
    double *c0 = nullptr, *c = nullptr, *trace = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool live = false, pending = false;
    rttda_status err = RTTDA_OK;  // status of the chunk that failed (the slot then stops stepping)
    std::string msg;
  };
  size_t budget = 0, used = 0;
  std::vector<Slot> slots;
};

extern "C" {

rttda_status rttda_pool_create(size_t budget_bytes, rttda_pool **out) {
  if (!out) return fail(RTTDA_E_INVAL, "out is NULL");
  *out = new rttda_pool();
  (*out)->budget = budget_bytes;
  return RTTDA_OK;
}

rttda_status rttda_pool_destroy(rttda_pool *pool) {
  if (!pool) return fail(RTTDA_E_INVAL, "pool is NULL");
  for (auto &sl : pool->slots)
    if (sl.ev) {
      (void)hipEventSynchronize(sl.ev);
      (void)hipEventDestroy(sl.ev);
    }
  delete pool;
  return RTTDA_OK;
}

rttda_status rttda_pool_admit(rttda_pool *pool, rttda_ctx *ctx, int32_t nrhs, const rttda_pulse *pulses,
                              double dt, int64_t n_steps, int32_t integrator, double *c0, double *c,
                              double *trace, size_t footprint_bytes, int32_t *slot) {
  if (!pool || !ctx || !pulses || !c0 || !c || !slot) return fail(RTTDA_E_INVAL, "NULL argument");
  rttda_status st = check_nrhs(ctx, nrhs);
  if (st != RTTDA_OK) return st;
  if (integrator != RTTDA_INTEG_RK4 && integrator != RTTDA_INTEG_SSO)
    return fail(RTTDA_E_INVAL, "integrator must be RTTDA_INTEG_RK4 or RTTDA_INTEG_SSO");
  // the request's own checks (pulses, dt, pointers) at admission, so that a bad request is refused
  // here instead of failing inside a later pool step
  if ((st = check_request(nrhs, pulses, dt, 0, n_steps, c0, c, trace, nullptr, nullptr, nullptr, nullptr)) !=
      RTTDA_OK)
    return st;
  for (const auto &sl : pool->slots)
    if (sl.live && sl.ctx == ctx) return fail(RTTDA_E_STATE, "context already admitted");
  if (footprint_bytes > pool->budget - std::min(pool->used, pool->budget))
    return fail(RTTDA_E_NOMEM, "footprint %zu bytes exceeds the %zu bytes left of the budget", footprint_bytes,
                pool->budget - std::min(pool->used, pool->budget));
  size_t k = 0;
  while (k < pool->slots.size() && pool->slots[k].live) ++k;
  if (k == pool->slots.size()) pool->slots.emplace_back();
  rttda_pool::Slot &sl = pool->slots[k];
  if (!sl.ev) HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  sl.ctx = ctx;
  sl.nrhs = nrhs;
  sl.integ = integrator;
  sl.pulses.assign(pulses, pulses + nrhs);
  sl.dt = dt;
  sl.n_steps = n_steps;
  sl.done = 0;
  sl.c0 = c0;
  sl.c = c;
  sl.trace = trace;
  sl.bytes = footprint_bytes;
  sl.live = true;
  sl.pending = false;
  sl.err = RTTDA_OK;
  sl.msg.clear();
  pool->used += footprint_bytes;
  *slot = (int32_t)k;
  return RTTDA_OK;
}

rttda_status rttda_pool_step(rttda_pool *pool, int64_t chunk_steps, int32_t *issued) {
  if (!pool || chunk_steps < 1) return fail(RTTDA_E_INVAL, "pool is NULL or chunk_steps < 1");
  int32_t n = 0;
  for (auto &sl : pool->slots) {
    if (!sl.live || sl.done >= sl.n_steps) continue;
    if (sl.pending) {
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;  // previous chunk still running
      if (q != hipSuccess) return fail(RTTDA_E_DEVICE, "pool: %s", hipGetErrorString(q));
    }
    const int64_t k = std::min(chunk_steps, sl.n_steps - sl.done);
    double *tr = sl.trace ? sl.trace + (size_t)sl.done * sl.nrhs : nullptr;
    rttda_status st = propagate_impl(sl.ctx, sl.nrhs, sl.pulses.data(), sl.dt, sl.done, k, sl.c0, sl.c, tr,
                                     nullptr, sl.integ == RTTDA_INTEG_SSO ? INTEG_SSO : INTEG_RK4, sl.done > 0);
    if (st != RTTDA_OK) {  // this request stops here; the others carry on
      sl.err = st;
      sl.msg = g_last_error;
      sl.done = sl.n_steps;
      continue;
    }
    HIP_TRY(hipEventRecord(sl.ev, sl.ctx->stream));
    sl.pending = true;
    sl.done += k;
    ++n;
  }
  if (issued) *issued = n;
  return RTTDA_OK;
}

rttda_status rttda_pool_poll(rttda_pool *pool, int32_t slot, int64_t *steps_enqueued, int32_t *finished) {
  if (!pool || slot < 0 || slot >= (int32_t)pool->slots.size() || !pool->slots[slot].live)
    return fail(RTTDA_E_INVAL, "no such slot");
  rttda_pool::Slot &sl = pool->slots[slot];
  int32_t fin = 0;
  if (sl.done >= sl.n_steps) {
    if (!sl.pending) {
      fin = 1;
    } else {
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipSuccess) fin = 1;
      else if (q != hipErrorNotReady) return fail(RTTDA_E_DEVICE, "pool: %s", hipGetErrorString(q));
    }
  }
  if (steps_enqueued) *steps_enqueued = sl.done;
  if (finished) *finished = fin;
  if (sl.err != RTTDA_OK) return fail(sl.err, "slot %d stopped: %s", slot, sl.msg.c_str());
  return RTTDA_OK;
}

rttda_status rttda_pool_result(rttda_pool *pool, int32_t slot, int64_t *first_bad_step) {
  if (!pool || slot < 0 || slot >= (int32_t)pool->slots.size() || !pool->slots[slot].live)
    return fail(RTTDA_E_INVAL, "no such slot");
  rttda_pool::Slot &sl = pool->slots[slot];
  if (first_bad_step) *first_bad_step = -1;
  if (sl.pending) HIP_TRY(hipEventSynchronize(sl.ev));
  sl.pending = false;
  if (sl.err != RTTDA_OK) return fail(sl.err, "slot %d stopped: %s", slot, sl.msg.c_str());
  int64_t bad = -1;
  rttda_status st = rttda_guard(sl.ctx, &bad);
  if (first_bad_step) *first_bad_step = bad;
  return st;
}

rttda_status rttda_pool_release(rttda_pool *pool, int32_t slot) {
  if (!pool || slot < 0 || slot >= (int32_t)pool->slots.size() || !pool->slots[slot].live)
    return fail(RTTDA_E_INVAL, "no such slot");
  rttda_pool::Slot &sl = pool->slots[slot];
  if (sl.pending) HIP_TRY(hipEventSynchronize(sl.ev));
  sl.pending = false;
  sl.live = false;
  sl.ctx = nullptr;
  pool->used -= std::min(pool->used, sl.bytes);
  return RTTDA_OK;
}

rttda_status rttda_pool_usage(const rttda_pool *pool, size_t *used_bytes, int32_t *active) {
  if (!pool) return fail(RTTDA_E_INVAL, "pool is NULL");
  int32_t a = 0;
  for (const auto &sl : pool->slots) a += sl.live ? 1 : 0;
  if (used_bytes) *used_bytes = pool->used;
  if (active) *active = a;
  return RTTDA_OK;
}

rttda_status rttda_guard(rttda_ctx *ctx, int64_t *first_bad_step) {
  if (!ctx || !first_bad_step) return fail(RTTDA_E_INVAL, "NULL argument");
  DevState h{};
  HIP_TRY(hipMemcpyAsync(&h, ctx->state(), sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  *first_bad_step = h.bad_step;
  if (h.bad_step >= 0) return fail(RTTDA_E_UNSTABLE, "norm guard tripped at step %lld", (long long)h.bad_step);
  return RTTDA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// sigma for callers that cannot allocate device memory: the workspace is a static device array
// ---------------------------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;       // the static scratch of each device
constexpr size_t NOALLOC_SLAB_BYTES = (size_t)16 << 20;  // of it, for the exchange's partial slabs
constexpr int NOALLOC_MAX_RHS = 64;
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

// Every device the library runs this entry point on holds its own copy until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns for the current
// device (the name itself is a host-side stand-in).
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up on the first call on that device.
rttda_status scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(RTTDA_E_UNSUPPORTED, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(RTTDA_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RTTDA_OK;
}
}  // namespace

extern "C" rttda_status rttda_sigma_noalloc(const rttda_desc *desc, int32_t nrhs, const double *field,
                                            const double *dir, const double *c0, const double *c, double *s0,
                                            double *s) {
  rttda_status st = validate_desc(desc, false);
  if (st != RTTDA_OK) return st;
  {
    const void *ptrs[] = {desc->e_occ, desc->e_virt, desc->mu};
    for (const void *p : ptrs)
      if (!p || !aligned16(p)) return fail(RTTDA_E_INVAL, "e_occ, e_virt and mu must be non-NULL and 16-byte aligned");
    if (desc->n_aux > 0)
      for (const void *p : {desc->b_ov, desc->b_oo, desc->b_vv})
        if (!p || !aligned16(p)) return fail(RTTDA_E_INVAL, "factors must be non-NULL and 16-byte aligned");
  }
  if (nrhs < 1 || nrhs > NOALLOC_MAX_RHS) return fail(RTTDA_E_INVAL, "nrhs=%d outside 1..%d", nrhs, NOALLOC_MAX_RHS);
  if (!field || !dir || !c0 || !c || !s0 || !s) return fail(RTTDA_E_INVAL, "NULL array argument");
  if (!aligned16(c0) || !aligned16(c) || !aligned16(s0) || !aligned16(s))
    return fail(RTTDA_E_INVAL, "device arrays must be 16-byte aligned");
  if ((st = check_dirs(dir, nrhs)) != RTTDA_OK) return st;
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(field[r])) return fail(RTTDA_E_INVAL, "field %d not finite", r);
  const int o = desc->n_occ, v = desc->n_virt, nq = desc->n_aux, prec = desc->precision;
  const Layout L = make_layout(o, v, nq, nrhs, prec, NOALLOC_SLAB_BYTES, false);
  if (L.total > NOALLOC_BYTES)
    return fail(RTTDA_E_NOMEM, "o=%d v=%d n_aux=%d nrhs=%d needs %zu bytes of scratch; the static scratch holds %zu",
                o, v, nq, nrhs, L.total, NOALLOC_BYTES);
  int xv = -1;
  if (nq > 0) {
    xv = auto_variant(prec, o, 2 * nrhs, v, L);  // no W scratch here, so never the large-o GEMM path
    if (xv < 0) return fail(RTTDA_E_UNSUPPORTED, "no exchange kernel for o=%d in precision %d", o, prec);
  }
  void *base = nullptr;
  if ((st = scratch_address(&base)) != RTTDA_OK) return st;
  if (xv >= 0) HIP_TRY(variant_of(prec, xv)->prepare());

  // a context over the static scratch: no pinned staging, events or second stream
  rttda_ctx ctx;
  ctx.d = *desc;
  ctx.stream = static_cast<hipStream_t>(desc->stream);
  ctx.o = o;
  ctx.v = v;
  ctx.nq = nq;
  ctx.R = nrhs;
  ctx.prec = prec;
  ctx.ov = (size_t)o * v;
  ctx.L = L;
  ctx.ws = static_cast<char *>(base);
  ctx.xvar = xv;
  ctx.overlap = 2;
  if (nq > 0) {
    ctx.sk = auto_splits(variant_of(prec, xv), o, 2 * nrhs, v, nq, L.sk_max, L);
    ctx.sj = L.sj_max;
  }
  // directions and field strengths: host arrays copied into the scratch, waited for before they
  // leave scope
  DevPulse hp[NOALLOC_MAX_RHS];
  double hsc[NOALLOC_MAX_RHS * SC_STRIDE];
  for (int r = 0; r < nrhs; ++r) {
    memset(&hp[r], 0, sizeof(DevPulse));
    hp[r].kind = RTTDA_PULSE_NONE;
    memcpy(hp[r].dir, dir + 3 * r, 3 * sizeof(double));
    for (int k = 0; k < SC_STRIDE; ++k) hsc[r * SC_STRIDE + k] = 0.0;
    hsc[r * SC_STRIDE + SC_E] = field[r];
  }
  hipStream_t hs = ctx.stream;
  HIP_TRY(hipMemcpyAsync(ctx.pulses(), hp, sizeof(DevPulse) * nrhs, hipMemcpyHostToDevice, hs));
  HIP_TRY(hipMemcpyAsync(ctx.sc(), hsc, sizeof(double) * SC_STRIDE * nrhs, hipMemcpyHostToDevice, hs));
  HIP_TRY(launch_gaps(hs, desc->e_occ, desc->e_virt, o, v, ctx.D()));
  HIP_TRY(launch_set_state(hs, ctx.state(), 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0));
  HIP_TRY(hipStreamSynchronize(hs));
  return sigma_enqueue(&ctx, nrhs, c0, c, s0, s);
}
