// Internal declarations of the RT-TDA gfx950 library (kernels + runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>

#include "rttda.h"

namespace rttda {

// Device copy of rttda_pulse (identical layout, checked by static_assert in the runtime).
struct DevPulse {
  int32_t kind;
  int32_t reserved;
  double e0, omega, t0, fwhm, beta, phase;
  double dir[3];
};

// Device-resident propagation scalars.
struct DevState {
  long long step;      // absolute step index of the current state c
  long long step0;     // step index at the start of the current propagate call
  long long bad_step;  // first step at which the norm guard tripped, -1 if none
  long long keep_ref;  // 1: the call resumes a run (the guard's reference norm and first bad step
                       // carry over from the previous call), 0: both restart with the call
  double *trace;       // trace row of step0 ([n_steps+1][nrhs]) or NULL; set per call, so a
  double *norms;       // captured step graph stays valid across calls with new output arrays
  double *corr;        // time-correlation output ([n_steps+1][nrhs][2]) or NULL, likewise
  double *pops;        // eigenstate populations output ([n_steps+1][nrhs][popk]) or NULL, likewise
  const double *popU;  // the popk unit vectors ([popk][o][v]) the states are projected on
  long long popk;
  double *energy;      // energy output <X|diag(0,A)|X> ([n_steps+1][nrhs]) or NULL, likewise
  const double *epart; // the epilogue's per-block energy partial sums [nrhs][nbe]
  long long nbe;
};
constexpr int POP_MAX = 64;  // eigenstates per populations output

constexpr double SQRT2 = 1.4142135623730951;
constexpr double FWHM_TO_SIGMA = 2.35482;

// Field of one pulse at time t (eqs. continuous wave, transform_limited, chirped_pulse).
// Delta pulses act as a kick at t = 0 and contribute no continuous field.
__device__ inline double pulse_field(const DevPulse &p, double t) {
  if (p.kind == RTTDA_PULSE_CW) return p.e0 * sin(p.omega * t + p.phase);
  if (p.kind == RTTDA_PULSE_GAUSS || p.kind == RTTDA_PULSE_CHIRP) {
    const double s = p.fwhm / FWHM_TO_SIGMA;
    const double tau = t - p.t0;
    const double env = exp(-tau * tau / (2.0 * s * s));
    const double arg = (p.kind == RTTDA_PULSE_GAUSS) ? p.omega * tau + p.phase
                                                      : (p.omega + 0.5 * p.beta * tau) * tau + p.phase;
    return p.e0 * env * sin(arg);
  }
  return 0.0;
}


// Per-RHS scalar slots (f64): g_re, g_im, E(t_stage), spare.
constexpr int SC_STRIDE = 4;
constexpr int SC_GRE = 0, SC_GIM = 1, SC_E = 2;
// Per-block partial sums of the field kernel (f64): g_re, g_im, <X|F>, |X|^2.
constexpr int PART_STRIDE = 4;

// Field-kernel tile (i x a) and its grid per RHS.
constexpr int FT_I = 16, FT_A = 16;
inline int field_blocks_a(int v) { return (v + FT_A - 1) / FT_A; }
inline int field_blocks_i(int o) { return (o + FT_I - 1) / FT_I; }

// k_scalar modes (bit mask).
enum : int {
  SM_TRACE = 1,     // write trace/norm samples at index step - step0, update the guard
  SM_C0 = 2,        // RK4 stage update of c0 with k0 = i E g
  SM_INC = 4,       // step += 1 once the stage is done
  SM_EFIELD = 8,    // E = pulse field at (step + node) dt (else E = 0 unless SM_KEEP_E)
  SM_SIGMA0 = 16,   // s0 = -E g with E preset by the host
  SM_OUT = 32,      // out[r] = <X|M|X>  (dipole_trace entry point)
  SM_KEEP_E = 64,   // keep the E slots written by the host
  SM_ENERGY = 128,  // energy sample at index step - step0 from the epilogue's partial sums
};

// Epilogue modes.
enum : int { EP_RK4 = 0, EP_SIGMA = 1, EP_ENERGY = 2 };
// Small problems (o v <= SMALL_OV_MAX, at most SMALL_R_MAX RHS): one launch for the Coulomb and
// exchange partial slabs of a stage, one single-workgroup launch for the whole stage epilogue.
constexpr int SMALL_OV_MAX = 2048;
constexpr int SMALL_R_MAX = 64;
// the small path is the default up to this many exchange flops per stage at max_rhs (measured: at
// o10 v40 N_Q120 with one or two RHS it is 10-25 % faster than the general kernels; at o12 v48
// N_Q160 with one RHS, 2.2e7 flops, it is slower)
constexpr double SMALL_DEFAULT_FLOPS = 2e7;
// LDS of the two small-path kernels: the epilogue stages one RHS's X (two planes), mu_vv and mu_oo
// in FP64, the partial-sum kernel a slice's X and W and one Q's B_vv and B_oo in FP32
constexpr int SMALL_LDS_DOUBLES = 12288;
inline bool small_shape_ok(int o, int v) {
  return (long long)o * v <= SMALL_OV_MAX && 2LL * o * v + (long long)v * v + (long long)o * o <= SMALL_LDS_DOUBLES;
}
hipError_t prepare_small();  // one-time kernel attributes (dynamic LDS); call outside graph capture
hipError_t launch_small_2e(hipStream_t s, int b_dtype, const void *Bov, const void *Boo, const void *Bvv,
                           const float *X, int o, int v, int nq, int ns, int nsplit, float cx, float *P);
hipError_t launch_small_epi(hipStream_t s, int prec, int R, int o, int v, int nslab, int stage, int use_field,
                            int want_trace, double dt, const DevPulse *pulses, DevState *st, const double *D,
                            const float *P, const double *moo, const double *mov, const double *mvv,
                            const double *Xin, double *c, double *c0, double *acc, double *acc0, double *xs64,
                            double *xs0, float *x32, __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, double *normref);
// Epilogue grid: blocks per RHS along ia (the energy partial sums come one per block)
constexpr int EP_BX_MAX = 2048;
int epilogue_blocks(long long ov);
// symplectic split-operator update modes (k_sso_update)
enum : int { SSO_KICK_FIRST = 0, SSO_KICK = 1, SSO_DRIFT = 2 };

// ---------------------------------------------------------------------------------------------
// Kernel launchers (all enqueue on `s`, return hipError_t of the launch)
// ---------------------------------------------------------------------------------------------
hipError_t launch_mu_blocks(hipStream_t s, const double *mu, const DevPulse *pulses, int o, int v, int R,
                            double *moo, double *mov, double *mvv);
hipError_t launch_gaps(hipStream_t s, const double *e_occ, const double *e_virt, int o, int v, double *D);
hipError_t launch_to_f32(hipStream_t s, const double *c, long long n, float *x32);
hipError_t launch_to_bf16x2(hipStream_t s, const double *c, long long n, float *x32, __hip_bfloat16 *hi,
                            __hip_bfloat16 *lo);
// Coulomb first product in `nes` ia chunks (partials dpart[nes][nq][ns], summed into slot 0 when
// nes > 1, which is d for the second product); gemv1_chunks picks nes (at most GEMV1_CHUNKS_MAX).
constexpr int GEMV1_CHUNKS_MAX = 16;
int gemv1_chunks(int nq, int ov);
hipError_t launch_gemv1(hipStream_t s, int b_dtype, const void *B, const float *X, int nq, int ov, int ns, int nes,
                        float *dpart);
hipError_t launch_gemv2(hipStream_t s, int b_dtype, const void *B, const float *dvec, int nq, int ov, int ns,
                        int nsplit, float *P);
// The same pair on the FP32 matrix cores for batches of many slices (the context's 2 max_rhs >= 32):
// d in nes ia chunks (coulomb_mfma_chunks, at most GEMV1_CHUNKS_MAX) summed into chunk slot 0 of
// dpart, then the partial slabs P[split][s][ia] of J.
int coulomb_mfma_chunks(int nq, int ov);
hipError_t launch_coulomb_mfma(hipStream_t s, int b_dtype, const void *B, const float *X, int nq, int ov, int ns,
                               int nes, int nsplit, float *dpart, float *P);
hipError_t launch_field(hipStream_t s, const double *X, const double *X0, const double *moo, const double *mov,
                        const double *mvv, int o, int v, int R, double *F, double *part);
hipError_t launch_scalar(hipStream_t s, int R, int nbf, int stage, int mode, double dt, const DevPulse *pulses,
                         DevState *st, const double *part, double *sc, double *c0, double *acc0, double *xs0,
                         double *out, double *normref, double *s0);
// epart != NULL: also the per-block partial sums of <X, A X> per RHS ([R][epilogue_blocks(ov)])
hipError_t launch_epilogue(hipStream_t s, int prec, int R, int o, int v, int nslab, int stage, int mode,
                           int use_field, double dt, const double *D, const float *P, const double *F,
                           const double *sc, const double *Xin, double *c, double *acc, double *xs64, float *x32,
                           __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, double *s_out, double *epart = nullptr);
hipError_t launch_sso_update(hipStream_t s, int prec, int R, int o, int v, int nslab, int mode, int use_field,
                             double dt, const double *D, const float *P, const double *F, const double *sc, double *c,
                             double *c0, double *W, double *W0, float *x32, __hip_bfloat16 *xhi,
                             __hip_bfloat16 *xlo);
hipError_t launch_plane_copy(hipStream_t s, int prec, int R, size_t ov, int plane, const double *c, float *x32,
                             __hip_bfloat16 *xhi, __hip_bfloat16 *xlo);
// Lanczos guard: block partial sums (at most LZ_BLOCKS_MAX) are written to part[] and added on the host
constexpr int LZ_BLOCKS_MAX = 1024;
int lz_blocks(long long n);
hipError_t launch_lz_init(hipStream_t s, long long n, double *v, double *part);
hipError_t launch_lz_apply(hipStream_t s, long long n, int nslab, const double *D, const float *P, const double *v,
                           const double *vprev, double beta, double *w, double *part);
hipError_t launch_lz_orth(hipStream_t s, long long n, const double *v, double alpha, double *w, double *part);
hipError_t launch_lz_next(hipStream_t s, int prec, long long n, double scale, const double *w, double *v,
                          double *vprev, float *x32, __hip_bfloat16 *xhi, __hip_bfloat16 *xlo, int shift);
// Block Davidson (lowest eigenpairs of A) and populations: FP64 vectors of n = o*v stored one after
// another; per-block partial sums (at most DV_BLOCKS_MAX per vector) are added on the host.
constexpr int DV_BLOCKS_MAX = 1024;
constexpr int DV_SPACE_MAX = 64;  // largest search space (vectors)
int dv_blocks(long long n);
hipError_t launch_dv_apply(hipStream_t s, long long n, int nb, int nslab, const double *D, const float *P,
                           const double *V, double *W);
hipError_t launch_dv_dots(hipStream_t s, long long n, int m, const double *V, int nt, const double *T, double *out);
hipError_t launch_dv_combine(hipStream_t s, long long n, int m, const double *V, int nc, const double *C, int ldc,
                             int mode, double *out);
hipError_t launch_dv_resid(hipStream_t s, long long n, int nc, const double *X, const double *AX, const double *theta,
                           double *R, double *part);
hipError_t launch_dv_precond(hipStream_t s, long long n, int nc, const double *R, const double *theta,
                             const double *D, double *T);
hipError_t launch_dv_norm2(hipStream_t s, long long n, const double *T, double *part);
hipError_t launch_dv_scale(hipStream_t s, long long n, double scale, const double *T, double *out);
hipError_t launch_dv_unit(hipStream_t s, long long n, long long idx, double *V);
hipError_t launch_dv_diag(hipStream_t s, int b_dtype, int o, int v, int nq, const void *Bov, const void *Boo,
                          const void *Bvv, double cx, const double *D, double *diag);
hipError_t launch_kick(hipStream_t s, int R, int ov, const DevPulse *pulses, const double *F, const double *sc,
                       double *c, double *c0);
hipError_t launch_kick_term(hipStream_t s, int R, int ov, const DevPulse *pulses, const double *F, const double *sc,
                            double inv_j, double *T, double *T0, double *c, double *c0);
hipError_t launch_set_state(hipStream_t s, DevState *st, long long step0, double *trace, double *norms,
                            double *corr, double *pops, const double *popU, int popk, double *energy = nullptr,
                            const double *epart = nullptr, long long nbe = 0, int resume = 0);
// eigenstate populations |<U_I | X_r>|^2 at the current step (no-op unless st->pops is set)
hipError_t launch_pop(hipStream_t s, int R, size_t ov, const double *X, const DevState *st);
hipError_t launch_spectrum(hipStream_t s, int kind, const double *sig, int n_t, int nsig, double dt, double kappa,
                           int n_w, double w0, double dw, int average, double *out);
// time-correlation sample <Xref_r | X_r> (both planes and the ground amplitude) at the current step
hipError_t launch_corr(hipStream_t s, int R, size_t ov, const double *X, const double *X0, const double *xref,
                       const double *xref0, const DevState *st);

// Exchange: K partials P[split][slice][o][v] = scale * sum_{Q in split} B_oo^Q X_slice B_vv^Q.
// Large-o split-BF16 path (two batched GEMMs per chunk of Q through a W scratch buffer): used
// for o >= XGEMM_O_MIN with o % 8 == 0 and v % 8 == 0; the scratch holds W hi/lo for up to
// XGEMM_SCRATCH_MAX bytes' worth of Q values.
constexpr int XGEMM_O_MIN = 128;
constexpr size_t XGEMM_SCRATCH_MAX = size_t(2048) << 20;

struct ExchangeVariant {
  int precision;  // RTTDA_PREC_*
  int o16;        // padded occupied count handled (o <= o16)
  int ks;         // slices per workgroup
  int nt;         // virtual columns per workgroup
  const char *name;
  hipError_t (*launch)(hipStream_t s, const void *Boo, const void *Bvv, const void *X, const void *Xlo, int o,
                       int v, int nq, int ns, int nsplit, float scale, float *P, void *scratch,
                       size_t scratch_bytes);
  size_t lds_bytes;
  hipError_t (*prepare)();  // one-time kernel attributes (dynamic LDS size); call outside graph capture
  int v_min = 1;            // applicability: v >= v_min, v % v_mod == 0, o % o_mod == 0, o >= o_min
  int v_mod = 1;
  int o_mod = 1;
  int o_min = 1;
  bool scratch = false;  // needs the W scratch region of the workspace
  int rank = 0;          // preference among variants of equal tile waste (higher first)
  bool applies(int o, int v) const {
    return o <= o16 && o >= o_min && v >= v_min && v % v_mod == 0 && o % o_mod == 0;
  }
};

}  // namespace rttda
