/*
 * komahip: MI355X (gfx950) Bloch-simulation hot path of the KomaMRI method
 * (Castillo-Passi et al., arXiv 2301.02702).
 *
 * The library integrates the Bloch equation in the rotating frame
 * (section "Physical and Mathematical Background", Eq. Bloch with the
 * effective field of Eq. B-def) for every spin of a phantom over a
 * discretised sequence, with the paper's first-order operator splitting
 * (rotation, then relaxation, per interval), the spinor rotation of
 * Eq. Rot_exc in the excitation regime, the integral (trapezoidal) phase of
 * precession blocks (section "Simulation blocks, Regime Switching, and
 * Sequence-Aware Time Stepping") and the relaxation update, and returns the
 * acquired signal: at every ADC sample, the sum of the transverse
 * magnetisation Mxy = Mx + i My over the spins of each signal group
 * (Figure 3, the simulation pipeline).
 *
 * Conventions
 *   - SI units: m, s, T/m, T, rad/s, rad/(s T).
 *   - A spin starts at thermal equilibrium (Mxy = 0, Mz = M0) at t[0].
 *   - B1 is constant on each interval (piecewise constant), G is linear
 *     between grid points (piecewise linear), x and dw are constant.
 *   - Interval n is in the excitation regime iff b1_re[n] != 0 or
 *     b1_im[n] != 0 (exact test); otherwise it is in the precession regime.
 *   - An ADC index k samples the state at t[k]; k = 0 samples the initial
 *     state.
 *   - The signal is the plain sum of Mxy over a group's spins (no
 *     normalisation, no coil weighting, no noise).
 *
 * Threading: a context is used by one host thread at a time. Requests are
 * independent objects but share their context's device and allocator.
 * Every entry point returns a koma_status; no C++ exception crosses the ABI.
 * On error, outputs are left untouched and koma_last_error() describes the
 * failure. A device (HIP) failure poisons the context: every later call on
 * it returns KOMA_E_DEVICE.
 */
#ifndef KOMAHIP_H
#define KOMAHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KOMA_OK = 0,
    KOMA_E_ARG = -1,       /* NULL pointer, bad size, bad configuration value */
    KOMA_E_PHANTOM = -2,   /* non-finite value, PD < 0, T1/T2 <= 0 or NaN, bad group offsets */
    KOMA_E_SEQUENCE = -3,  /* n_t < 2, non-finite value, t not strictly increasing,
                              ADC indices out of [0, n_t) or not strictly increasing */
    KOMA_E_NOMEM = -4,     /* device (or, in koma_discretize, host) allocation failed */
    KOMA_E_BUDGET = -5,    /* the request's device footprint exceeds hbm_budget */
    KOMA_E_DEVICE = -6,    /* a HIP call failed; the context is poisoned */
    KOMA_E_CANCELLED = -7, /* the request was cancelled */
    KOMA_E_STATE = -8      /* call not valid in the object's current state */
} koma_status;

/* Arithmetic of the kernels. KOMA_FP64: everything in FP64.
 * KOMA_MIXED: rotations, precession factors and relaxation in FP32; the
 * cumulative gradient/off-resonance phase of precession blocks in FP64
 * (reduced to [0, 1) turns before the FP32 sine/cosine); the sum over the
 * lanes of a wavefront in FP32 and every sum beyond the wavefront in FP64. */
typedef enum { KOMA_FP64 = 0, KOMA_MIXED = 1 } koma_precision;

/* Where the caller's phantom, signal and m_final pointers live. Sequence
 * arrays are always host memory (they are packed on the host). */
typedef enum { KOMA_HOST = 0, KOMA_DEVICE = 1 } koma_mem;

typedef struct {
    double b0;    /* T, > 0; validated, no role in rotating-frame dynamics */
    double gamma; /* rad/(s T), > 0 (proton: 2.6752218744e8) */
} koma_scanner;

/* Phantom: structure of arrays, n spins, float32 (canonical precision of the
 * inputs: every path reads exactly these values). */
typedef struct {
    int64_t n;                /* spins, >= 1 */
    const float *x, *y, *z;   /* m, finite */
    const float *pd;          /* M0, >= 0, finite */
    const float *t1, *t2;     /* s, > 0; +INFINITY means no relaxation */
    const float *dw;          /* off-resonance, rad/s, finite */
    int64_t n_groups;         /* >= 1 */
    const int64_t *group_off; /* host memory always: n_groups + 1 non-decreasing offsets
                                 from 0 to n; NULL means one group */
    /* Motion (section "Overview": the phantom's displacement field): NULL
     * for static spins, or all three velocities (m/s, finite), with the
     * spin at (x, y, z) + v t at sequence time t. The field of an interval is
     * the mean of its end-point fields with the position updated to each end
     * point (the trapezoidal rule of the precession phase); ADC samples are
     * then evaluated one by one, never by a linear recurrence. */
    const float *vx, *vy, *vz;
    /* Receive coils (section "Overview": coil sensitivities; section
     * "Limitations": multiple coils): n_coils = 0 for the plain sum, or
     * n_coils >= 1 complex sensitivities per spin, sens_re/sens_im laid out
     * [n_coils][n] (finite; where `where` says). Coil c's signal is the sum
     * over a group's spins of sens_c * Mxy (unconjugated); a spin's
     * sensitivity is fixed (it does not follow the motion). At most 1024. */
    int64_t n_coils;
    const float *sens_re, *sens_im;
} koma_phantom;

/* Discretised sequence (host memory). */
typedef struct {
    int64_t n_t;                  /* time points, >= 2 */
    const double *t;              /* s, strictly increasing, finite */
    const double *gx, *gy, *gz;   /* T/m at the time points */
    const double *b1_re, *b1_im;  /* T, per interval [n_t - 1] */
    int64_t n_adc;                /* >= 0 */
    const int64_t *adc_idx;       /* strictly increasing indices in [0, n_t) */
} koma_sequence;

typedef struct {
    koma_precision precision;
    int spins_per_lane;    /* spins summed per lane in the sample-parallel kernel: 0 = the planner's
                              choice, or 1 .. 16 (the vector-ALU kernels round down to 1, 2, 4 or 8) */
    int wg_size;           /* 256 (reserved: other values are rejected) */
    int64_t chunk_events;  /* events per launch of the spin-sequential kernel for requests; >= 1 */
    size_t hbm_budget;     /* device bytes: the footprint one call may need, and the total that the
                              open requests of the context hold together with the blocks it keeps
                              cached for reuse (koma_req_open fails with KOMA_E_BUDGET rather
                              than exceed it); 0 = no limit */
    size_t partial_budget; /* bytes for cross-workgroup signal partials per launch; >= 1 MiB */
    int defer_min_adc;     /* precession blocks with at least this many ADC samples are
                              summed by the sample-parallel kernel; < 0 disables it */
    int stretch_max;       /* longest run of evenly spaced samples evaluated by recurrence
                              after one exact FP64 anchor; 1..128 */
    int sample_engine;     /* sums of deferred samples: 0 = matrix cores (the sum over
                              spins of c w^j as a product of an [8 x spins] and a
                              [spins x 16] matrix per 128 samples; FP32 MFMA for
                              KOMA_MIXED, FP64 MFMA for KOMA_FP64), 1 = vector ALU
                              (complex recurrence and a register transpose). Moving
                              spins always use the vector ALU. */
    int tile_packing;      /* 1: when no sample is deferred and every non-empty signal group has
                              >= 64 spins, wavefronts take 64 consecutive spins across group
                              boundaries (a wavefront then holds at most two groups, whose
                              samples it sums apart); 0: every wavefront within one group */
    int lanes_per_spin;    /* lanes per spin of the spin-sequential kernel: 0 = the planner's
                              choice (several when the spins fill few wavefronts), 1, 2, 4, 8 or
                              16 (the events between two observations of the state are affine
                              maps; each lane composes a share of them, the lanes' products are
                              combined, the same operators associated differently) */
    int stretches_per_wg;  /* readout stretches per workgroup of the FP32 matrix-core sample sums:
                              0 = the planner's choice, 4 or 6 (6 shares each staged operand among
                              more sums; 4 gives a finer grid). Other engines and KOMA_FP64 ignore
                              it. */
} koma_config;

typedef struct koma_ctx koma_ctx;
typedef struct koma_req koma_req;

/* Defaults: KOMA_MIXED, auto spins per lane, 256, 4096 events, no budget,
 * 1 GiB partials, defer_min_adc 32, stretch_max 128, sample_engine 0,
 * tile_packing 1, and the planner's lanes per spin and stretches per workgroup. */
void koma_config_default(koma_config *cfg);

/* Create a context on HIP device `device` (sets it current). The context
 * owns a HIP stream used when callers pass a NULL stream. */
koma_status koma_ctx_create(int device, const koma_config *cfg, koma_ctx **out);
void koma_ctx_destroy(koma_ctx *ctx);

/* Message of the last error on this context (empty string if none). The
 * pointer stays valid until the next call on the context. ctx may be NULL
 * (message of the last failed koma_ctx_create or koma_discretize on this
 * thread). */
const char *koma_last_error(const koma_ctx *ctx);

/* Replace the context configuration (validated as in koma_ctx_create). */
koma_status koma_ctx_set_config(koma_ctx *ctx, const koma_config *cfg);

/* Device bytes a request for this phantom and sequence would hold (inputs
 * copied to the device, spin state, snapshots, partials, packed sequence).
 * Validates the sequence (host) and the phantom sizes. */
koma_status koma_footprint(const koma_phantom *ph, const koma_sequence *seq,
                           const koma_config *cfg, size_t *bytes);

/* One whole simulation, synchronous on `hip_stream` (NULL: the context's
 * stream). Phantom arrays, sig and m_final live where `where` says (device
 * pointers must be on the context's device and stay valid until return).
 *   sig:     [n_sig][n_groups][n_adc][2] doubles (re, im), n_sig = max(n_coils, 1),
 *            caller-owned, overwritten.
 *   m_final: NULL or [n][3] doubles (Mx, My, Mz) after the last interval.
 * Nothing is kept after return. */
koma_status koma_simulate(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                          const koma_sequence *seq, koma_mem where, void *hip_stream,
                          double *sig, double *m_final);

/* The same simulation (section "Overview": scanner, phantom and sequence in,
 * raw signal out) enqueued on `hip_stream` (NULL: the context's stream)
 * without waiting for it. The phantom arrays, sig and m_final are device
 * pointers on the context's device and must stay valid until the stream has
 * run the work; the host arrays of the sequence are read before return.
 * Every host-side check and the packing of the sequence happen before return,
 * with the errors of koma_simulate. The phantom's values are checked on the
 * device: status (a device int32, or NULL) receives 0 if they are valid, else
 * the validation bits (1 non-finite position, velocity, dw or PD; 2 PD < 0;
 * 4 T1 or T2 <= 0 or NaN; 8 non-finite coil sensitivity), and then sig and
 * m_final are left untouched. Later calls on the context that use its
 * scratch (koma_simulate, koma_simulate_async) are ordered after the queued
 * work on any stream, so consecutive calls pipeline: the host packs the next
 * simulation while the device runs the previous one. */
koma_status koma_simulate_async(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                                const koma_sequence *seq, void *hip_stream, double *sig,
                                double *m_final, int32_t *status);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * simulation as koma_simulate_async, with the same arguments, semantics and
 * results, but every buffer beyond the caller's inputs and outputs (packed
 * event program, validation word, snapshots, signal partials, spin state)
 * lives in one static device array of koma_noalloc_capacity() bytes
 * (64 MiB), of which each GPU holds its own copy until the process ends. The
 * call makes no device or pinned-host allocation: the packed tables go to the
 * array by hipMemcpyAsync from the context's host plan, which returns once
 * the host buffer has been read. Inputs and outputs are device-resident
 * (KOMA_DEVICE); `status` (device int32, or NULL) receives the phantom's
 * validation bits as for koma_simulate_async. A simulation whose buffers do
 * not fit (the cross-workgroup partials of one launch are held to half the
 * array) fails with KOMA_E_BUDGET before any device work, outputs untouched.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * there: calls that overlap on one GPU (other streams, other contexts, other
 * host threads) race, so the caller orders them, e.g. on one stream. The
 * context's own scratch is not touched, so other calls on the context need
 * not wait for this one. */
koma_status koma_simulate_noalloc(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                                  const koma_sequence *seq, void *hip_stream, double *sig,
                                  double *m_final, int32_t *status);
/* Bytes of the static array koma_simulate_noalloc works in. */
size_t koma_noalloc_capacity(void);

/* ---- chunked execution with device-resident state (serving) ------------
 * koma_req_open copies the phantom (host or device memory per `where`) and
 * the packed sequence into request-owned device buffers and initialises the
 * spin state; nothing of the caller's is kept. koma_req_advance enqueues the
 * next chunk of at most `max_events` events (<= 0: the configured
 * chunk_events; with several lanes per spin the chunk ends at a segment
 * end, so it may exceed `max_events` by up to one segment of 8 x lanes map
 * events plus its observation) on `hip_stream` without waiting; the signal of every
 * precession block finished so far is summed at the same time. koma_req_done
 * reports whether all events have been enqueued. koma_req_result enqueues
 * the final cross-workgroup sums and copies the signal ([n_sig][n_groups]
 * [n_adc][2] doubles, host memory) back, synchronising `hip_stream`. Requests are
 * independent: one request's result does not depend on which other requests
 * run at the same time. All calls on one request use one stream (or the caller
 * orders them); koma_req_close waits for that stream only, and the request's
 * device blocks go back to the context's cache for later requests. */
koma_status koma_req_open(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                          const koma_sequence *seq, koma_mem where, koma_req **out);
koma_status koma_req_advance(koma_req *req, int64_t max_events, void *hip_stream);
koma_status koma_req_done(const koma_req *req, int *done);
koma_status koma_req_result(koma_req *req, double *sig, void *hip_stream);
/* Checkpoint: the spin state, the signal accumulated so far and the event
 * cursor, as an opaque host byte string. Call with host_buf NULL to get the
 * size. The request must be idle (its last advance synchronised). */
koma_status koma_req_save(const koma_req *req, void *host_buf, size_t *bytes);
/* Restore a checkpoint taken from a request opened with the same inputs. */
koma_status koma_req_load(koma_req *req, const void *host_buf, size_t bytes);
void koma_req_close(koma_req *req);

typedef struct {
    int64_t n_spins, n_tiles, n_groups, n_adc;
    int64_t n_events, n_rf, n_rf_events, n_runs, n_inline_adc, n_deferred_adc, n_stretches, n_families,
        n_snapshots;
    int64_t n_blocks, spins_per_lane, n_chunks;
    int64_t events_done;
    size_t footprint;
    int64_t n_ends;        /* precession-block ends every spin evaluates */
    int64_t n_rf_in_runs;  /* excitation intervals inside runs of identical ones */
    int64_t n_rows;        /* rows of inline sample partials: one per tile (a tile holding two
                              groups has two; in FP64 at 16 lanes per spin, one per half tile) */
    int64_t lanes_per_spin; /* lanes per spin of the spin-sequential kernel */
    int64_t max_single_run; /* longest run of single excitation intervals with equal relaxation
                               keys (the one-lane kernel takes such a run in one loop) */
    int64_t stretches_per_wg; /* readout stretches one sample-parallel workgroup takes (4 or 6 on the
                                 FP32 matrix cores, whichever fills the chip's rounds better) */
} koma_req_info;
koma_status koma_req_info_get(const koma_req *req, koma_req_info *info);
/* The same figures for a plan built on the host only (no device work);
 * footprint is what koma_req_open would hold. */
koma_status koma_plan_info(const koma_scanner *sc, const koma_phantom *ph, const koma_sequence *seq,
                           const koma_config *cfg, koma_req_info *info);

/* Device memory of the context's requests: bytes held by open requests,
 * bytes of closed requests' blocks cached for reuse, and the largest
 * held + cached total since the context was created. Any pointer may be
 * NULL. */
koma_status koma_ctx_mem(const koma_ctx *ctx, size_t *held, size_t *cached, size_t *peak);

/* ---- measurement ---------------------------------------------------------
 * With profiling on, every kernel launch of the context is bracketed by HIP
 * events recorded on the stream it is launched on; koma_ctx_kernel_stats
 * synchronises those streams and returns per-kernel totals:
 *   kind 0: spin-sequential kernel (excitation, block ends, inline samples)
 *   kind 1: sample-parallel kernel (samples of long precession blocks)
 *   kind 2: cross-workgroup reduction into the signal
 *   kind 3: state initialisation / export, MRF operand packing and final argmax
 *   kind 4: MRF matching contraction (koma_mrf_match)
 * Totals are reset by koma_ctx_profile(ctx, 1). */
koma_status koma_ctx_profile(koma_ctx *ctx, int on);
koma_status koma_ctx_kernel_stats(koma_ctx *ctx, int kind, double *total_ms, int64_t *launches,
                                  int64_t *work_units);

/* ---- MRF dictionary matching ----------------------------------------------
 * The paper's MR-fingerprinting experiment (Full-Dict reconstruction): each
 * pixel's fingerprint x (n_t complex values, one per TR) is assigned the
 * dictionary entry with the maximum dot product against the normalised
 * entries, best = argmax_e |<d_e, x>|^2 / ||d_e||^2, <d, x> = sum_t conj(d_t) x_t.
 * Precision: the decision is taken on binary16 operands. Every row (entry or
 * fingerprint) is first scaled by an exact power of two so that its largest
 * |Re| or |Im| lies in [0.5, 1), then each part is rounded to binary16 (ties
 * to even); ||d_e||^2 is that of the rounded entry; the dot products
 * accumulate in FP32 on the matrix cores. Ties go to the lower index.
 *   dict:  [n_entries][n_t][2] floats (re, im); fp: [n_pix][n_t][2] floats.
 *   best:  [n_pix] entry index (-1 if every entry is zero).
 *   proj:  [n_pix][2] doubles, <d_best, x> / ||d_best|| in the caller's units
 *          (the pixel's complex scale relative to the unit-norm entry).
 * All four arrays live where `where` says; synchronous on `hip_stream`. */
koma_status koma_mrf_match(koma_ctx *ctx, const float *dict, int64_t n_entries, const float *fp, int64_t n_pix,
                           int64_t n_t, koma_mem where, void *hip_stream, int32_t *best, double *proj);

/* Low-rank dictionary compression (the paper's LRTV reconstruction matches
 * against a dictionary of reduced rank 5): the `rank` leading right singular
 * vectors of the dictionary D ([n_entries][n_t][2] floats) and its singular
 * values, by subspace iteration on D^H D with rank + oversample vectors
 * (<= 32, <= n_t) from a fixed pseudo-random start, `iters` iterations, then a
 * Rayleigh-Ritz step (complex Jacobi); FP64 throughout, deterministic.
 *   basis: [n_t][rank][2] doubles, orthonormal columns, descending singular
 *          values (each column's complex phase is arbitrary);
 *   sv:    [rank] doubles.
 * Arrays live where `where` says; synchronous on `hip_stream`. */
koma_status koma_mrf_svd(koma_ctx *ctx, const float *dict, int64_t n_entries, int64_t n_t, int rank, int oversample,
                         int iters, koma_mem where, void *hip_stream, double *basis, double *sv);
/* Coefficients of rows ([n_rows][n_t][2] floats) in a basis ([n_t][rank][2]
 * doubles): out[r][j] = sum_t x_r[t] basis[t][j] ([n_rows][rank][2] floats,
 * accumulated in FP64). With an orthonormal basis, inner products of rows in
 * its span are preserved, so koma_mrf_match on the coefficients matches in
 * the compressed domain. */
koma_status koma_mrf_project(koma_ctx *ctx, const float *rows, int64_t n_rows, int64_t n_t, const double *basis,
                             int rank, koma_mem where, void *hip_stream, float *out);

/* ---- sequence-aware time stepping ----------------------------------------
 * Section "Simulation blocks, Regime Switching, and Sequence-Aware Time
 * Stepping": with G piecewise linear the trapezoidal phase of a precession
 * interval is exact when only the vertices of G are sampled, and with B1
 * piecewise constant the spinor rotation of Eq. Rot_exc is exact per RF
 * sample; extra points are needed only for the ADC (and for motion). The
 * paper's user knobs are the longest step between intermediate gradient
 * samples (Delta t, here dt_max) and between RF samples (Delta t_rf, here
 * dt_rf_max).
 *
 * A sequence is a list of blocks played back to back from t = 0. Times
 * inside a block are relative to its start; every event must end within the
 * block's duration. */
typedef enum { KOMA_GRAD_NONE = 0, KOMA_GRAD_TRAP = 1, KOMA_GRAD_PWL = 2 } koma_grad_kind;

/* Trapezoid: zero until delay, linear ramp to amp over rise, flat for flat,
 * linear ramp back to zero over fall (rise, fall > 0; delay, flat >= 0). */
typedef struct {
    double amp; /* T/m, finite */
    double delay, rise, flat, fall; /* s */
} koma_trap;

/* One gradient axis of a block. KOMA_GRAD_PWL: a piecewise-linear waveform
 * through pwl_n >= 2 vertices (pwl_t[i] s, block-local, strictly increasing,
 * in [0, duration]; pwl_amp[i] T/m), zero outside them (an arbitrary
 * gradient sampled on a raster is the case pwl_t[i] = delay + i dt). G must
 * stay continuous: the first amplitude is 0 unless the waveform starts at the
 * block start, the last is 0 unless it ends at the block end, and where a
 * waveform meets a block boundary its value equals the neighbouring block's
 * value there (relative tolerance 1e-9). The caller's arrays are read during
 * the call only. */
typedef struct {
    int kind; /* koma_grad_kind */
    koma_trap trap;
    int64_t pwl_n;
    const double *pwl_t, *pwl_amp;
} koma_grad;

/* RF: n piecewise-constant samples (re[i], im[i]) in T, sample i held on
 * [delay + i dt, delay + (i + 1) dt). n = 0: no RF. */
typedef struct {
    double delay, dt;
    int64_t n;
    const double *re, *im;
} koma_rf;

/* ADC: n samples at delay + i * dwell (dwell > 0 when n > 1). */
typedef struct {
    double delay, dwell;
    int64_t n;
} koma_adc;

typedef struct {
    double duration; /* s, > 0 */
    koma_grad g[3];  /* x, y, z */
    koma_rf rf;
    koma_adc adc;
} koma_block;

/* Discretise `n_blocks` blocks into a koma_sequence grid (host memory only).
 * Time points: every block boundary, every gradient vertex, every RF sample
 * boundary (a sample longer than dt_rf_max split into equal parts), every ADC
 * sample, and, on intervals outside RF samples, equally spaced points so that
 * no interval exceeds dt_max; points within 1 ps of each other are one point.
 * dt_max, dt_rf_max > 0; +INFINITY means no such subdivision (the minimal
 * grid). Outputs: t[n_t], gx/gy/gz[n_t] (G at each point), b1_re/b1_im
 * [n_t - 1] (the RF sample in force on each interval, else 0), adc_idx[n_adc]
 * (the point of each ADC sample, in time order).
 * Two calls: with t == NULL, *n_t and *n_adc receive the sizes; then call
 * again with arrays of at least those sizes (*n_t, *n_adc give their
 * capacities and receive the sizes written). Errors: KOMA_E_ARG (NULL or
 * small outputs, dt <= 0, unknown gradient kind), KOMA_E_SEQUENCE (a block
 * or event out of its bounds, a non-finite value, vertex times not
 * increasing, G not continuous, two ADC samples at one instant),
 * KOMA_E_NOMEM; the message is in koma_last_error(NULL). */
koma_status koma_discretize(const koma_block *blocks, int64_t n_blocks, double dt_max, double dt_rf_max,
                            int64_t *n_t, int64_t *n_adc, double *t, double *gx, double *gy, double *gz,
                            double *b1_re, double *b1_im, int64_t *adc_idx);

#ifdef __cplusplus
}
#endif
#endif /* KOMAHIP_H */
