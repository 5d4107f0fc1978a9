// Host side of the komahip C-ABI: validation, sequence packing into the
// event program, spin tiling, launch planning, contexts and requests.
//
// Sequence packing (paper: section "Simulation blocks, Regime Switching, and
// Sequence-Aware Time Stepping"): intervals with B1 != 0 are excitation
// intervals (one EV_RF each); every maximal run of B1 = 0 intervals is one
// precession block. For a block the spin-independent integral of the gradient
// K(t) = gamma_bar * sum((G_n + G_{n+1})/2 dt_n) (cycles/m, trapezoidal, exact
// for piecewise-linear G) and the elapsed time tau(t) are accumulated in FP64
// from the block start; a spin's block phase at t is -2 pi (x.K(t) + f tau(t))
// with f = dw / 2 pi, and its relaxation over the block is the relaxation
// update over tau.
#include <hip/hip_runtime.h>

#include <immintrin.h>

#include <algorithm>
#include <cfloat>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "komahip.h"
#include "komahip_internal.h"
#include "komahip_lowrank.h"
#include "komahip_mrf.h"
#include "komahip_scratch.h"

using namespace koma;

namespace {

thread_local std::string g_create_error;

constexpr double kTwoPi = 6.28318530717958647692;
// Samples are merged into one evenly spaced stretch only when every sample of
// it lies within these bounds of the straight line through the stretch: the
// induced phase error is below 2e-9 turns per metre of |x| and 1e-12 s times
// |f| (about the rounding of the time grid itself, ~1e-16 relative).
constexpr double kStretchTolK = 2e-9;   // cycles/m
constexpr double kStretchTolT = 1e-12;  // s
// moving spins: first moments within this of their quadratic model (phase
// error below 2e-9 turns per m/s of |v|)
constexpr double kStretchTolK1 = 2e-9;  // cycles s/m

struct Chunk {
    int64_t s0, s1;   // stretch range
    int64_t c0, c1;   // deferred sample range (columns)
    int64_t ready;    // event index after which all of its snapshots exist
};

struct Plan {
    // sequence program
    std::vector<Event> ev;
    std::vector<Stretch> st;
    std::vector<std::array<double, 4>> fam_dk;  // increments of each stretch family
    std::vector<int32_t> inl_k, def_k;  // inline / deferred column -> ADC index
    int64_t n_slots = 0, n_rf = 0, n_rf_events = 0, n_runs = 0;
    std::vector<int64_t> snap_event;  // slot -> event index of its EV_SNAP
    // spin layout
    int64_t n_spins = 0, n_groups = 1, n_tiles = 0, n_adc = 0;
    int64_t n_rows = 0;  // rows of inline partials (tiles, plus one per tile holding two groups)
    bool packed = false; // tiles cross group boundaries (no deferred samples)
    int lanes = 1;       // lanes per spin of the spin-sequential kernel
    bool half_tiles = false;  // FP64 at 16 lanes: half a tile per workgroup, two inline rows per tile
    std::vector<SegEv> segs;  // segments of the event program (lanes > 1)
    std::vector<Tile> tiles;
    std::vector<int32_t> tile_off;  // [n_groups + 1]
    std::vector<int32_t> row_off;   // [n_groups + 1]: group g owns inline rows [row_off[g], row_off[g + 1])
    std::vector<Block> blocks;
    std::vector<int32_t> blk_off;   // [n_groups + 1]
    int spl = 1;
    int64_t per_wg = 1;
    std::vector<Chunk> chunks;
    int64_t max_cols = 0;
    double gamma = 0;
    bool moving = false;  // spins carry velocities
    int64_t n_coils = 0;  // receive coils (0: plain sums)
    int64_t n_sig = 1;    // signal planes: max(n_coils, 1)
};

// Phantom arrays: x, y, z, pd, t1, t2, dw ([n] each), then vx, vy, vz ([n],
// moving spins only), then sens_re, sens_im ([n_coils][n], coils only).
constexpr int kPhArrays = 12;
constexpr int64_t kMaxCoils = 1024;

static inline bool ph_used(const koma_phantom *p, int i) {
    return i < 7 || (i < 10 ? p->vx != nullptr : p->n_coils > 0);
}
static inline size_t ph_bytes(const koma_phantom *p, int i) {
    return (size_t)p->n * (i < 10 ? 1 : (size_t)p->n_coils) * sizeof(float);
}

static inline void ph_sources(const koma_phantom *p, const float *src[kPhArrays]) {
    const float *all[kPhArrays] = {p->x,  p->y,  p->z,  p->pd, p->t1,      p->t2,
                                   p->dw, p->vx, p->vy, p->vz, p->sens_re, p->sens_im};
    for (int i = 0; i < kPhArrays; ++i) src[i] = all[i];
}

static inline PhantomDev ph_dev(const float *const d[kPhArrays], bool moving, int64_t n, int64_t n_coils) {
    return PhantomDev{d[0],
                      d[1],
                      d[2],
                      d[3],
                      d[4],
                      d[5],
                      d[6],
                      moving ? d[7] : nullptr,
                      moving ? d[8] : nullptr,
                      moving ? d[9] : nullptr,
                      n,
                      n_coils,
                      n_coils > 0 ? d[10] : nullptr,
                      n_coils > 0 ? d[11] : nullptr};
}

struct DevMem {  // request-owned or context-scratch device allocation
    void *p = nullptr;
    size_t cap = 0;
};

enum { K_SEQ = 0, K_PAR = 1, K_RED = 2, K_AUX = 3, K_MRF = 4, K_KINDS = 5 };

struct ProfRec {
    hipEvent_t a, b;
    int kind;
    int64_t work;
};

}  // namespace

struct koma_ctx {
    int device = 0;
    int n_cu = 256;  // compute units of the device (the planner sizes grids by it)
    // this device's static scratch (koma_simulate_noalloc), looked up once
    // per device when the context is created
    void *nz_scratch = nullptr;
    hipError_t nz_err = hipSuccess;
    koma_config cfg{};
    hipStream_t stream = nullptr;
    std::string err;
    bool poisoned = false;
    bool prof = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> ev_free;
    double tot_ms[K_KINDS] = {};
    int64_t n_launch[K_KINDS] = {};
    int64_t work[K_KINDS] = {};
    Plan plan;  // reused by koma_simulate (capacity kept across calls)
    // The packed tables of a call: a ring of pinned host staging buffers and
    // their device copies, so that a call packs while the uploads and kernels
    // of earlier calls are still queued. The upload goes on the call's stream
    // (ordered after the kernels of the previous call on that stream; a
    // cross-stream wait costs more host time than the copy saves); a slot's
    // host buffer is reused kStageRing calls later, once its upload is done.
    struct StageSlot {
        void *h = nullptr;
        size_t cap = 0;
        DevMem d;
        hipEvent_t copied = nullptr;  // recorded after the upload
        bool pending = false;
    };
    static constexpr int kStageRing = 4;
    StageSlot ring[kStageRing];
    int ring_next = 0;
    int32_t *h_flag = nullptr;
    // work of koma_simulate_async still queued on async_stream, which later
    // calls on the context's scratch order themselves after
    bool async_pending = false;
    hipEvent_t async_done = nullptr;
    // device blocks released by closed requests, reused by later ones (by size)
    std::multimap<size_t, void *> pool;
    size_t pool_bytes = 0;
    // device bytes held by open requests (block capacities), and the largest
    // held + pooled total seen since the context was created
    size_t held_bytes = 0;
    size_t mem_peak = 0;
    // bytes the request being opened has still to take (koma_req_open sets
    // its footprint, every block taken counts down): a reused cached block
    // may be larger than asked for, and must still leave room for the rest
    size_t pool_reserve = 0;
    // scratch reused by koma_simulate (grow-only)
    DevMem s_ev, s_st, s_tiles, s_blocks, s_toff, s_boff, s_inl, s_def, s_snap, s_pa, s_pb, s_sig,
        s_mxy, s_mz, s_flags, s_vcount, s_mf, s_ph[kPhArrays];
    // MRF matching scratch (grow-only)
    DevMem m_src_d, m_src_x, m_dh, m_xh, m_dexp, m_xexp, m_inv, m_ps, m_pi, m_best, m_proj;
    DevMem l_v, l_y, l_zp, l_z, l_basis, l_sv, l_out;  // dictionary compression scratch
};

struct koma_req {
    koma_ctx *ctx = nullptr;
    Plan plan;
    bool fp64 = false;
    // request-owned device memory
    DevMem ph[kPhArrays], ev, st, tiles, blocks, toff, boff, inl, def, snap, pa, pb, sig, mxy, mz, segs;
    hipStream_t last_stream = nullptr;  // stream of the last enqueued work
    int64_t cursor = 0;
    size_t next_chunk = 0;
    bool finished = false;   // all events enqueued and all sums launched
    bool cancelled = false;
    size_t footprint = 0;
};

// ---------------------------------------------------------------- helpers

static koma_status fail(koma_ctx *ctx, koma_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) {
        ctx->err = buf;
        if (st == KOMA_E_DEVICE) ctx->poisoned = true;
    } else {
        g_create_error = buf;
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), e_ == hipErrorOutOfMemory ? KOMA_E_NOMEM : KOMA_E_DEVICE,      \
                        "%s failed: %s", #call, hipGetErrorString(e_));                       \
    } while (0)

static koma_status dev_reserve(koma_ctx *ctx, DevMem &m, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (m.cap >= bytes) return KOMA_OK;
    if (m.p) {
        // queued asynchronous work may still use the block
        if (ctx->async_pending && hipEventSynchronize(ctx->async_done) != hipSuccess)
            return fail(ctx, KOMA_E_DEVICE, "waiting for queued work failed");
        hipError_t e = hipFree(m.p);
        m.p = nullptr;
        m.cap = 0;
        if (e != hipSuccess) return fail(ctx, KOMA_E_DEVICE, "hipFree failed: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&m.p, bytes);
    if (e != hipSuccess) {
        m.p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, KOMA_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    m.cap = bytes;
    return KOMA_OK;
}

static void dev_free(DevMem &m) {
    if (m.p) (void)hipFree(m.p);
    m.p = nullptr;
    m.cap = 0;
}

// Caching allocator for request buffers: hipFree can synchronise the whole
// device, which would stall every other request in flight, so blocks of
// closed requests are kept and reused (smallest fit within 2x). With an HBM
// budget, the blocks held by open requests plus the cached ones never exceed
// it: a reused block must fit beside the held ones and the rest of the
// request being opened, and cached blocks are released (largest first)
// before an allocation that would not fit. Every block is a multiple of 256
// bytes; plan_footprint counts the same sizes, so a request whose footprint
// fits beside the held bytes always gets its memory.
static size_t pool_round(size_t bytes) { return (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255; }

static void pool_trim(koma_ctx *ctx) {
    for (auto &kv : ctx->pool) (void)hipFree(kv.second);
    ctx->pool.clear();
    ctx->pool_bytes = 0;
}

static koma_status pool_get(koma_ctx *ctx, DevMem &m, size_t bytes) {
    bytes = pool_round(bytes);
    const size_t budget = ctx->cfg.hbm_budget;
    const size_t rest = ctx->pool_reserve > bytes ? ctx->pool_reserve - bytes : 0;  // after this block
    auto it = ctx->pool.lower_bound(bytes);
    if (it != ctx->pool.end() && it->first <= 2 * bytes &&
        (!budget || ctx->held_bytes + it->first + rest <= budget)) {
        m.p = it->second;
        m.cap = it->first;
        ctx->pool_bytes -= it->first;
        ctx->pool.erase(it);
        ctx->held_bytes += m.cap;
        ctx->pool_reserve = rest;
        return KOMA_OK;
    }
    if (budget) {
        if (ctx->held_bytes + bytes + rest > budget)
            return fail(ctx, KOMA_E_BUDGET, "device memory of open requests would exceed hbm_budget (%zu + %zu > %zu)",
                        ctx->held_bytes, bytes + rest, budget);
        while (!ctx->pool.empty() && ctx->held_bytes + ctx->pool_bytes + bytes > budget) {
            auto last = std::prev(ctx->pool.end());
            (void)hipFree(last->second);
            ctx->pool_bytes -= last->first;
            ctx->pool.erase(last);
        }
    }
    hipError_t e = hipMalloc(&m.p, bytes);
    if (e == hipErrorOutOfMemory && !ctx->pool.empty()) {
        (void)hipGetLastError();
        pool_trim(ctx);
        e = hipMalloc(&m.p, bytes);
    }
    if (e != hipSuccess) {
        m.p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, KOMA_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    m.cap = bytes;
    ctx->held_bytes += bytes;
    ctx->pool_reserve = rest;
    ctx->mem_peak = std::max(ctx->mem_peak, ctx->held_bytes + ctx->pool_bytes);
    return KOMA_OK;
}

static void pool_put(koma_ctx *ctx, DevMem &m) {
    if (m.p) {
        ctx->pool.insert({m.cap, m.p});
        ctx->pool_bytes += m.cap;
        ctx->held_bytes -= m.cap;
    }
    m.p = nullptr;
    m.cap = 0;
}

template <class T>
static koma_status pool_upload(koma_ctx *ctx, DevMem &m, const std::vector<T> &v, hipStream_t s) {
    koma_status st = pool_get(ctx, m, v.size() * sizeof(T));
    if (st != KOMA_OK) return st;
    if (!v.empty()) HIPCHK(ctx, hipMemcpyAsync(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return KOMA_OK;
}

template <class T>
static koma_status upload(koma_ctx *ctx, DevMem &m, const std::vector<T> &v, hipStream_t s) {
    koma_status st = dev_reserve(ctx, m, v.size() * sizeof(T));
    if (st != KOMA_OK) return st;
    if (!v.empty()) HIPCHK(ctx, hipMemcpyAsync(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return KOMA_OK;
}

static bool finite_d(double v) { return std::isfinite(v); }

// ---------------------------------------------------------------- validation

static koma_status check_config(koma_ctx *ctx, const koma_config *c) {
    if (!c) return fail(ctx, KOMA_E_ARG, "config is NULL");
    if (c->precision != KOMA_FP64 && c->precision != KOMA_MIXED)
        return fail(ctx, KOMA_E_ARG, "precision must be KOMA_FP64 or KOMA_MIXED");
    if (c->spins_per_lane < 0 || c->spins_per_lane > 16)
        return fail(ctx, KOMA_E_ARG, "spins_per_lane must be 0 (planner's choice) or 1 .. 16");
    if (c->wg_size != 256) return fail(ctx, KOMA_E_ARG, "wg_size must be 256");
    if (c->chunk_events < 1) return fail(ctx, KOMA_E_ARG, "chunk_events must be >= 1");
    if (c->partial_budget < ((size_t)1 << 20)) return fail(ctx, KOMA_E_ARG, "partial_budget must be >= 1 MiB");
    if (c->stretch_max < 1 || c->stretch_max > kStretchMax)
        return fail(ctx, KOMA_E_ARG, "stretch_max must be in [1, %d]", kStretchMax);
    if (c->sample_engine != 0 && c->sample_engine != 1)
        return fail(ctx, KOMA_E_ARG, "sample_engine must be 0 (matrix cores) or 1 (vector ALU)");
    if (c->tile_packing != 0 && c->tile_packing != 1) return fail(ctx, KOMA_E_ARG, "tile_packing must be 0 or 1");
    if (c->lanes_per_spin != 0 && c->lanes_per_spin != 1 && c->lanes_per_spin != 2 && c->lanes_per_spin != 4 &&
        c->lanes_per_spin != 8 && c->lanes_per_spin != 16)
        return fail(ctx, KOMA_E_ARG, "lanes_per_spin must be 0 (planner's choice), 1, 2, 4, 8 or 16");
    if (c->stretches_per_wg != 0 && c->stretches_per_wg != kMMStretchesSmall && c->stretches_per_wg != kMMStretches)
        return fail(ctx, KOMA_E_ARG, "stretches_per_wg must be 0 (planner's choice), %d or %d", kMMStretchesSmall,
                    kMMStretches);
    return KOMA_OK;
}

static koma_status check_scanner(koma_ctx *ctx, const koma_scanner *sc) {
    if (!sc) return fail(ctx, KOMA_E_ARG, "scanner is NULL");
    if (!(finite_d(sc->gamma) && sc->gamma > 0)) return fail(ctx, KOMA_E_ARG, "gamma must be finite and > 0");
    if (!(finite_d(sc->b0) && sc->b0 > 0)) return fail(ctx, KOMA_E_ARG, "b0 must be finite and > 0");
    return KOMA_OK;
}

// Structure of the sequence: sizes, pointers, ADC indices.
static koma_status check_sequence(koma_ctx *ctx, const koma_sequence *q) {
    if (!q) return fail(ctx, KOMA_E_ARG, "sequence is NULL");
    if (q->n_t < 2) return fail(ctx, KOMA_E_SEQUENCE, "n_t must be >= 2 (got %lld)", (long long)q->n_t);
    if (q->n_t > ((int64_t)1 << 31) - 2) return fail(ctx, KOMA_E_SEQUENCE, "n_t too large");
    if (!q->t || !q->gx || !q->gy || !q->gz || !q->b1_re || !q->b1_im)
        return fail(ctx, KOMA_E_ARG, "sequence array is NULL");
    if (q->n_adc < 0) return fail(ctx, KOMA_E_SEQUENCE, "n_adc must be >= 0");
    if (q->n_adc > 0 && !q->adc_idx) return fail(ctx, KOMA_E_ARG, "adc_idx is NULL");
    // branch-free pass (vectorised); the slow one below only names the index
    const int64_t *__restrict ai = q->adc_idx;
    int bad = 0;
    if (q->n_adc > 0) bad = (ai[0] < 0) | (ai[q->n_adc - 1] >= q->n_t);
    for (int64_t k = 1; k < q->n_adc; ++k) bad |= ai[k] <= ai[k - 1];
    if (!bad) return KOMA_OK;
    for (int64_t k = 0; k < q->n_adc; ++k) {
        if (q->adc_idx[k] < 0 || q->adc_idx[k] >= q->n_t)
            return fail(ctx, KOMA_E_SEQUENCE, "adc_idx[%lld] = %lld out of [0, n_t)", (long long)k,
                        (long long)q->adc_idx[k]);
        if (k > 0 && q->adc_idx[k] <= q->adc_idx[k - 1])
            return fail(ctx, KOMA_E_SEQUENCE, "adc_idx not strictly increasing at %lld", (long long)k);
    }
    return KOMA_OK;
}

// Values of the sequence: finite, t strictly increasing. The packer tests the
// same conditions branch-free while it reads the arrays (one pass over them)
// and calls this only to name the offending index.
static koma_status check_sequence_values(koma_ctx *ctx, const koma_sequence *q) {
    for (int64_t i = 0; i < q->n_t; ++i) {
        if (!finite_d(q->t[i]) || !finite_d(q->gx[i]) || !finite_d(q->gy[i]) || !finite_d(q->gz[i]))
            return fail(ctx, KOMA_E_SEQUENCE, "non-finite time or gradient at point %lld", (long long)i);
        if (i > 0 && !(q->t[i] > q->t[i - 1]))
            return fail(ctx, KOMA_E_SEQUENCE, "t not strictly increasing at point %lld", (long long)i);
    }
    for (int64_t i = 0; i + 1 < q->n_t; ++i)
        if (!finite_d(q->b1_re[i]) || !finite_d(q->b1_im[i]))
            return fail(ctx, KOMA_E_SEQUENCE, "non-finite B1 on interval %lld", (long long)i);
    return fail(ctx, KOMA_E_SEQUENCE, "invalid sequence value");
}

// Bit 63 of the result is set iff x is infinite or NaN (exponent all ones).
static inline uint64_t nonfinite_bit(double x) {
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return (u & 0x7ff0000000000000ull) + (1ull << 52);
}

static koma_status check_phantom_shape(koma_ctx *ctx, const koma_phantom *p) {
    if (!p) return fail(ctx, KOMA_E_ARG, "phantom is NULL");
    if (p->n < 1) return fail(ctx, KOMA_E_PHANTOM, "phantom needs n >= 1 spins");
    if (!p->x || !p->y || !p->z || !p->pd || !p->t1 || !p->t2 || !p->dw)
        return fail(ctx, KOMA_E_ARG, "phantom array is NULL");
    if ((p->vx || p->vy || p->vz) && !(p->vx && p->vy && p->vz))
        return fail(ctx, KOMA_E_ARG, "give all three velocity arrays or none");
    if (p->n_coils < 0 || p->n_coils > kMaxCoils)
        return fail(ctx, KOMA_E_ARG, "n_coils must be in [0, %lld]", (long long)kMaxCoils);
    if (p->n_coils > 0 && (!p->sens_re || !p->sens_im))
        return fail(ctx, KOMA_E_ARG, "coil sensitivity array is NULL");
    if (p->n_groups < 1) return fail(ctx, KOMA_E_PHANTOM, "n_groups must be >= 1");
    if (!p->group_off) {
        if (p->n_groups != 1) return fail(ctx, KOMA_E_PHANTOM, "group_off is NULL but n_groups != 1");
    } else {
        if (p->group_off[0] != 0 || p->group_off[p->n_groups] != p->n)
            return fail(ctx, KOMA_E_PHANTOM, "group_off must run from 0 to n");
        for (int64_t g = 0; g < p->n_groups; ++g)
            if (p->group_off[g + 1] < p->group_off[g])
                return fail(ctx, KOMA_E_PHANTOM, "group_off decreases at group %lld", (long long)g);
    }
    return KOMA_OK;
}

static koma_status check_phantom_values_host(koma_ctx *ctx, const koma_phantom *p) {
    for (int64_t i = 0; i < p->n; ++i) {
        if (!std::isfinite(p->x[i]) || !std::isfinite(p->y[i]) || !std::isfinite(p->z[i]) ||
            !std::isfinite(p->dw[i]) || !std::isfinite(p->pd[i]))
            return fail(ctx, KOMA_E_PHANTOM, "non-finite position, dw or PD at spin %lld", (long long)i);
        if (p->pd[i] < 0) return fail(ctx, KOMA_E_PHANTOM, "PD < 0 at spin %lld", (long long)i);
        if (!(p->t1[i] > 0) || !(p->t2[i] > 0))
            return fail(ctx, KOMA_E_PHANTOM, "T1/T2 must be > 0 (or +inf) at spin %lld", (long long)i);
    }
    if (p->vx)
        for (int64_t i = 0; i < p->n; ++i)
            if (!std::isfinite(p->vx[i]) || !std::isfinite(p->vy[i]) || !std::isfinite(p->vz[i]))
                return fail(ctx, KOMA_E_PHANTOM, "non-finite velocity at spin %lld", (long long)i);
    for (int64_t i = 0; i < p->n * p->n_coils; ++i)
        if (!std::isfinite(p->sens_re[i]) || !std::isfinite(p->sens_im[i]))
            return fail(ctx, KOMA_E_PHANTOM, "non-finite coil sensitivity at element %lld", (long long)i);
    return KOMA_OK;
}

// ---------------------------------------------------------------- planning

namespace {

// ADC samples of one precession block (structure of arrays): ADC index,
// moments kx, ky, kz (cycles/m) and elapsed time tau (s) from the block start.
struct Samples {
    const int32_t *k;
    const double *v[4];
    size_t n;
    size_t size() const { return n; }
};

// Largest |v[q] - (v0 + q d)| over q = 1 .. n - 1 (NaN if any term is NaN).
inline double line_dev(const double *__restrict v, int n, double v0, double d) {
    double e = 0.0;
    int q = 1;
#if defined(__AVX2__) && defined(__FMA__)
    {
        // eight samples per step in two independent maxima; the sample index
        // kept as exact doubles
        const __m256d a = _mm256_set1_pd(v0), b = _mm256_set1_pd(d), step = _mm256_set1_pd(8.0);
        const __m256d absm = _mm256_castsi256_pd(_mm256_set1_epi64x(0x7fffffffffffffffLL));
        __m256d q0 = _mm256_setr_pd(1.0, 2.0, 3.0, 4.0), q1 = _mm256_setr_pd(5.0, 6.0, 7.0, 8.0);
        __m256d e0 = _mm256_setzero_pd(), e1 = _mm256_setzero_pd(), nan = _mm256_setzero_pd();
        for (; q + 8 <= n; q += 8) {
            const __m256d x0 = _mm256_sub_pd(_mm256_loadu_pd(v + q), _mm256_fmadd_pd(q0, b, a));
            const __m256d x1 = _mm256_sub_pd(_mm256_loadu_pd(v + q + 4), _mm256_fmadd_pd(q1, b, a));
            e0 = _mm256_max_pd(e0, _mm256_and_pd(x0, absm));
            e1 = _mm256_max_pd(e1, _mm256_and_pd(x1, absm));
            nan = _mm256_or_pd(nan, _mm256_cmp_pd(x0, x1, _CMP_UNORD_Q));
            q0 = _mm256_add_pd(q0, step);
            q1 = _mm256_add_pd(q1, step);
        }
        double t[4];
        _mm256_storeu_pd(t, _mm256_max_pd(e0, e1));
        e = std::max(std::max(t[0], t[1]), std::max(t[2], t[3]));
        if (_mm256_movemask_pd(nan)) return std::numeric_limits<double>::quiet_NaN();
    }
#endif
    for (; q < n; ++q) {
        const double x = std::fabs(v[q] - std::fma((double)q, d, v0));
        if (!(x <= e)) e = x;  // a NaN term makes e NaN
    }
    return e;
}

// True when samples i..i+len-1 all lie within the tolerances of the straight
// line through the first and the last of them; the line's increments go to
// inc, and half[c] tells whether component c even lies within half its
// tolerance (the margin a stretch needs to share the increments of another,
// see stretch_family).
inline bool on_line(const Samples &s, size_t i, size_t len, double *inc, bool *half) {
    for (int c = 0; c < 4; ++c) {
        const double *__restrict v = s.v[c] + i;
        const double v0 = v[0];
        const double d = (v[len - 1] - v0) / (double)(len - 1);
        const double tol = c < 3 ? kStretchTolK : kStretchTolT;
        // the last sample lies on the line by construction
        const double e = line_dev(v, (int)len - 1, v0, d);
        if (!(e <= tol)) return false;
        inc[c] = d;
        half[c] = e <= 0.5 * tol;
    }
    return true;
}

// Split the samples of one block into evenly spaced stretches of at most
// max_len samples: every sample of a stretch lies within the tolerances of
// the straight line through its first and last sample.
template <class Emit>
void make_stretches(const Samples &s, int max_len, Emit emit) {
    const size_t m = s.size();
    size_t i = 0;
    while (i < m) {
        double inc[4] = {0, 0, 0, 0};
        bool half[4] = {true, true, true, true};
        size_t len = std::min<size_t>((size_t)max_len, m - i);
        if (len > 1 && !on_line(s, i, len, inc, half)) {
            // greedy: extend while the next sample stays near the line of the first step
            size_t j = i + 1;
            while (j < m && (j - i + 1) <= (size_t)max_len) {
                bool ok = true;
                const double n = (double)(j - i);
                for (int c = 0; c < 4 && ok; ++c) {
                    const double d0 = s.v[c][i + 1] - s.v[c][i];
                    const double tol = (c < 3 ? kStretchTolK : kStretchTolT) * (1.0 + n);
                    ok = std::fabs(s.v[c][j] - (s.v[c][i] + n * d0)) <= tol;
                }
                if (!ok) break;
                ++j;
            }
            len = j - i;
            while (len > 1 && !on_line(s, i, len, inc, half)) len /= 2;
        }
        if (len <= 1) {
            len = 1;
            inc[0] = inc[1] = inc[2] = inc[3] = 0;
            half[0] = half[1] = half[2] = half[3] = true;
        }
        emit(i, len, inc, half);
        i += len;
    }
}

// True when the first moments m[c][i..i+len-1] of a moving spin's samples lie
// within kStretchTolK1 of the quadratic y0 + j d1 + j (j - 1) / 2 d2 through
// the first, middle and last of them (exact for a constant gradient and evenly
// spaced samples: the trapezoidal first moment of G t is quadratic in t).
inline bool on_quadratic(const double *const m[3], size_t i, size_t len, double *d1, double *d2) {
    const int n = (int)len - 1;
    for (int c = 0; c < 3; ++c) {
        const double *__restrict y = m[c] + i;
        if (n == 1) {
            d1[c] = y[1] - y[0];
            d2[c] = 0.0;
            continue;
        }
        const int mid = n / 2;
        const double a1 = mid, b1 = 0.5 * mid * (mid - 1.0), a2 = n, b2 = 0.5 * n * (n - 1.0);
        const double r1 = y[mid] - y[0], r2 = y[n] - y[0];
        const double det = a1 * b2 - a2 * b1;
        const double q2 = (a1 * r2 - a2 * r1) / det;
        const double q1 = (r1 - b1 * q2) / a1;
        double e = 0.0;
        for (int q = 1; q <= n; ++q)
            e = std::max(e, std::fabs(y[q] - (y[0] + q * q1 + 0.5 * q * (q - 1.0) * q2)));
        if (!(e <= kStretchTolK1)) return false;
        d1[c] = q1;
        d2[c] = q2;
    }
    return true;
}

// make_stretches for moving spins: moments linear, first moments quadratic
// in the sample index (halving a stretch until both hold).
template <class Emit>
void make_stretches_moving(const Samples &s, const double *const m[3], int max_len, Emit emit) {
    const size_t n = s.size();
    size_t i = 0;
    while (i < n) {
        double inc[4] = {0, 0, 0, 0}, d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
        bool half[4] = {true, true, true, true};
        size_t len = std::min<size_t>((size_t)max_len, n - i);
        while (len > 1 && !(on_line(s, i, len, inc, half) && on_quadratic(m, i, len, d1, d2))) len = (len + 1) / 2;
        if (len <= 1) {
            len = 1;
            for (int c = 0; c < 4; ++c) {
                inc[c] = 0.0;
                half[c] = true;
            }
            for (int c = 0; c < 3; ++c) d1[c] = d2[c] = 0.0;
        }
        emit(i, len, inc, half, d1, d2);
        i += len;
    }
}

// Family of a deferred stretch with increments inc: the first of the most
// recent families whose increments F keep every sample within the stretch
// tolerances, else a new family with increments inc. A component c qualifies
// if inc[c] == F[c], or if its samples lie within half the tolerance of their
// own line (half[c]) and (len - 1) |inc[c] - F[c]| is within the other half
// (so the stretch may use F instead of inc under the same error bound). The
// stretch takes its family's increments bitwise, so that the sample-parallel
// kernel can share the per-sample powers among the stretches of a family.
int32_t stretch_family(std::vector<std::array<double, 4>> &fams, size_t len, const double *inc, const bool *half) {
    const double n = (double)(len - 1);
    const int64_t nf = (int64_t)fams.size();
    for (int64_t f = nf - 1; f >= 0 && f >= nf - 16; --f) {
        bool ok = true;
        for (int c = 0; c < 4 && ok; ++c)
            ok = inc[c] == fams[f][c] ||
                 (half[c] && n * std::fabs(inc[c] - fams[f][c]) <= 0.5 * (c < 3 ? kStretchTolK : kStretchTolT));
        if (ok) return (int32_t)f;
    }
    fams.push_back({inc[0], inc[1], inc[2], inc[3]});
    return (int32_t)nf;
}

}  // namespace

// Moments of one precession block (points [a, b]): K = gamma_bar sum of
// (G_n + G_{n+1}) dt_n / 2 from the block start, and at every ADC point of
// the block (cursor into the increasing ADC indices) the sample's ADC index, K
// and elapsed time into the sample arrays. Returns the number of samples
// written; k receives K at point b. A function of its own so that the running
// sums stay in registers.
static size_t block_moments(const double *__restrict T, const double *__restrict GX, const double *__restrict GY,
                            const double *__restrict GZ, int64_t a, int64_t b, double gbar,
                            const int64_t *__restrict AI, int64_t n_adc, int64_t &cursor, int32_t *__restrict sk,
                            double *__restrict s0, double *__restrict s1, double *__restrict s2,
                            double *__restrict s3, double k[3]) {
    const double ta = T[a];
    int64_t cur = cursor;
    int64_t next = cur < n_adc ? AI[cur] : -1;
    double kx = 0, ky = 0, kz = 0;
    size_t ns = 0;
    for (int64_t p = a;; ++p) {
        if (next == p) {
            sk[ns] = (int32_t)cur;
            s0[ns] = kx;
            s1[ns] = ky;
            s2[ns] = kz;
            s3[ns] = T[p] - ta;
            ++ns;
            ++cur;
            next = cur < n_adc ? AI[cur] : -1;
        }
        if (p == b) break;
        const double hdt = 0.5 * gbar * (T[p + 1] - T[p]);
        kx += (GX[p] + GX[p + 1]) * hdt;
        ky += (GY[p] + GY[p + 1]) * hdt;
        kz += (GZ[p] + GZ[p + 1]) * hdt;
    }
    cursor = cur;
    k[0] = kx;
    k[1] = ky;
    k[2] = kz;
    return ns;
}

// First interval i >= a with B1 != 0 (n_int if none): 8 intervals at a time
// by OR-ing the bit patterns without their sign bits (-0.0 counts as zero).
static int64_t next_excitation(const double *__restrict br, const double *__restrict bi, int64_t a,
                               int64_t n_int) {
    int64_t b = a;
    for (; b + 8 <= n_int; b += 8) {
        uint64_t m = 0;
        for (int j = 0; j < 8; ++j) {
            uint64_t ur, ui;
            memcpy(&ur, br + b + j, 8);
            memcpy(&ui, bi + b + j, 8);
            m |= (ur | ui) << 1;
        }
        if (m) break;
    }
    while (b < n_int && br[b] == 0.0 && bi[b] == 0.0) ++b;
    return b;
}

static koma_status build_plan(koma_ctx *ctx, const koma_config &cfg, double gamma, const koma_phantom *ph,
                              const koma_sequence *q, Plan &P) {
    // reset, keeping the vectors' capacity (plans are rebuilt every call)
    P.ev.clear();
    P.st.clear();
    P.fam_dk.clear();
    P.inl_k.clear();
    P.def_k.clear();
    P.snap_event.clear();
    P.tiles.clear();
    P.tile_off.clear();
    P.blocks.clear();
    P.blk_off.clear();
    P.chunks.clear();
    P.n_slots = P.n_rf = P.n_rf_events = P.n_runs = 0;
    P.packed = false;
    P.lanes = 1;
    P.half_tiles = false;
    P.segs.clear();
    P.spl = 1;
    P.per_wg = 1;
    P.max_cols = 0;
    P.gamma = gamma;
    P.moving = ph->vx != nullptr;
    P.n_coils = ph->n_coils;
    P.n_sig = std::max<int64_t>(1, ph->n_coils);
    P.n_spins = ph->n;
    P.n_groups = ph->n_groups;
    P.n_adc = q->n_adc;
    const double gbar = gamma / kTwoPi;
    const int64_t n_t = q->n_t, n_int = n_t - 1;

    // ---- spin tiles: 64-spin slots that never straddle a signal group
    P.tile_off.assign(P.n_groups + 1, 0);
    P.tiles.reserve((size_t)(ph->n / kWave + P.n_groups + 1));
    for (int64_t g = 0; g < P.n_groups; ++g) {
        const int64_t a = ph->group_off ? ph->group_off[g] : 0;
        const int64_t b = ph->group_off ? ph->group_off[g + 1] : ph->n;
        P.tile_off[g] = (int32_t)P.tiles.size();
        for (int64_t s = a; s < b; s += kWave) {
            Tile t{};
            t.spin0 = s;
            t.count = (int32_t)std::min<int64_t>(kWave, b - s);
            t.group = (int32_t)g;
            t.split = t.count;
            t.seg = (int32_t)P.tiles.size();
            P.tiles.push_back(t);
            if (P.tiles.size() >= (size_t)1 << 30) return fail(ctx, KOMA_E_PHANTOM, "too many spins");
        }
    }
    P.tile_off[P.n_groups] = (int32_t)P.tiles.size();
    P.n_tiles = (int64_t)P.tiles.size();
    P.n_rows = P.n_tiles;

    // ---- event program
    // values first: one branch-free pass (vectorised) over every array; the
    // slow path only names the offending index
    {
        const double *__restrict T = q->t;
        uint64_t nonfinite = 0;  // bit 63: some value is infinite or NaN
        int disorder = 0;        // some interval has t[n+1] <= t[n]
        for (int64_t i = 0; i < n_t; ++i)
            nonfinite |= nonfinite_bit(T[i]) | nonfinite_bit(q->gx[i]) | nonfinite_bit(q->gy[i]) |
                         nonfinite_bit(q->gz[i]);
        for (int64_t i = 0; i < n_int; ++i) {
            nonfinite |= nonfinite_bit(q->b1_re[i]) | nonfinite_bit(q->b1_im[i]);
            disorder |= !(T[i + 1] > T[i]);
        }
        if ((nonfinite >> 63) || disorder) return check_sequence_values(ctx, q);
    }
    // planner scratch lives per thread and only grows: large per-call
    // allocations would be fresh pages (page faults) on every call
    thread_local std::vector<int32_t> smp_k;
    thread_local std::vector<double> smp_v[4], smp_m[3];
    const bool moving = P.moving;
    if (smp_k.size() < (size_t)q->n_adc + 1) {
        smp_k.resize((size_t)q->n_adc + 1);
        for (auto &v : smp_v) v.resize((size_t)q->n_adc + 1);
    }
    if (moving && smp_m[0].size() < (size_t)q->n_adc + 1)
        for (auto &v : smp_m) v.resize((size_t)q->n_adc + 1);
    const double *const smp_m_ptr[3] = {smp_m[0].data(), smp_m[1].data(), smp_m[2].data()};
    const int defer_min = cfg.defer_min_adc;
    // the current run of identical excitation intervals: the point it ends
    // at, its start time and its G t means (moving spins)
    int64_t rf_run_end = -1;
    double rf_run_t0 = 0.0, rf_run_gt[3] = {0, 0, 0};
    double rf_dt_ref = -1.0;  // reference interval length of the excitation events (Event::dt_ref)

    P.def_k.reserve((size_t)q->n_adc);
    const double *__restrict T = q->t;
    const double *__restrict GX = q->gx;
    const double *__restrict GY = q->gy;
    const double *__restrict GZ = q->gz;
    const double *__restrict BR = q->b1_re;
    const double *__restrict BI = q->b1_im;
    const int64_t *__restrict AI = q->adc_idx;
    const int64_t n_adc = q->n_adc;
    int64_t cursor = 0;  // next ADC sample (indices are strictly increasing)
    int64_t a = 0;
    Samples samples{smp_k.data(), {smp_v[0].data(), smp_v[1].data(), smp_v[2].data(), smp_v[3].data()}, 0};
    for (;;) {
        // precession block: points [a, b], intervals [a, b)
        const int64_t b = next_excitation(BR, BI, a, n_int);
        size_t ns = 0;
        const double ta = T[a];
        int64_t next = cursor < n_adc ? AI[cursor] : -1;
        // running moments in locals (registers); a sample at point p sees the
        // moments accumulated up to p
        double kx = 0, ky = 0, kz = 0;
        double k1x = 0, k1y = 0, k1z = 0;  // first moments gamma_bar sum(mean(G t) dt), moving spins only
        int32_t *__restrict sk = smp_k.data();
        double *__restrict s0 = smp_v[0].data(), *__restrict s1 = smp_v[1].data();
        double *__restrict s2 = smp_v[2].data(), *__restrict s3 = smp_v[3].data();
        if (!moving) {
            double k[3];
            ns = block_moments(T, GX, GY, GZ, a, b, gbar, AI, n_adc, cursor, sk, s0, s1, s2, s3, k);
            kx = k[0];
            ky = k[1];
            kz = k[2];
        } else {
            // moving spins: the samples' first moments beside their moments
            double *__restrict m0 = smp_m[0].data(), *__restrict m1 = smp_m[1].data(), *__restrict m2 = smp_m[2].data();
            int64_t p = a;
            for (;;) {
                if (next == p) {
                    sk[ns] = (int32_t)cursor;
                    s0[ns] = kx;
                    s1[ns] = ky;
                    s2[ns] = kz;
                    s3[ns] = T[p] - ta;
                    m0[ns] = k1x;
                    m1[ns] = k1y;
                    m2[ns] = k1z;
                    ++ns;
                    ++cursor;
                    next = cursor < n_adc ? AI[cursor] : -1;
                }
                if (p == b) break;
                const double t0 = T[p], t1 = T[p + 1];
                const double hdt = 0.5 * gbar * (t1 - t0);
                kx += (GX[p] + GX[p + 1]) * hdt;
                ky += (GY[p] + GY[p + 1]) * hdt;
                kz += (GZ[p] + GZ[p + 1]) * hdt;
                k1x += (GX[p] * t0 + GX[p + 1] * t1) * hdt;
                k1y += (GY[p] * t0 + GY[p + 1] * t1) * hdt;
                k1z += (GZ[p] * t0 + GZ[p + 1] * t1) * hdt;
                ++p;
            }
        }
        const double K[3] = {kx, ky, kz};
        const double K1[3] = {k1x, k1y, k1z};
        samples.n = ns;
        const bool defer = defer_min >= 0 && b > a && (int64_t)samples.size() >= std::max(1, defer_min);
        if (samples.size() > 0 && moving) {
            if (defer) {
                // sample-parallel from a snapshot: moments linear and first
                // moments quadratic in the sample index over every stretch
                const int32_t slot = (int32_t)P.n_slots++;
                Event e{};
                e.kind = EV_SNAP;
                e.a0 = slot;
                P.snap_event.push_back((int64_t)P.ev.size());
                P.ev.push_back(e);
                make_stretches_moving(samples, smp_m_ptr, cfg.stretch_max,
                                      [&](size_t i, size_t len, const double *inc, const bool *half,
                                          const double *d1, const double *d2) {
                    Stretch s{};
                    s.slot = slot;
                    s.d0 = (int32_t)P.def_k.size();
                    s.count = (int32_t)len;
                    s.fam = stretch_family(P.fam_dk, len, inc, half);
                    for (int c = 0; c < 4; ++c) {
                        s.k0[c] = samples.v[c][i];
                        s.dk[c] = P.fam_dk[s.fam][c];
                    }
                    for (int c = 0; c < 3; ++c) {
                        s.k1[c] = smp_m_ptr[c][i];
                        s.dk1[c] = d1[c];
                        s.d2k1[c] = d2[c];
                    }
                    P.def_k.insert(P.def_k.end(), samples.k + i, samples.k + i + len);
                    P.st.push_back(s);
                });
            } else {
                // one event per sample, its moments and first moments exact
                for (size_t i = 0; i < samples.size(); ++i) {
                    Event e{};
                    e.kind = EV_ADC;
                    e.a0 = (int32_t)P.inl_k.size();
                    e.count = 1;
                    for (int c = 0; c < 4; ++c) e.d[c] = samples.v[c][i];
                    for (int c = 0; c < 3; ++c) e.c64[c] = smp_m_ptr[c][i];
                    P.inl_k.push_back(samples.k[i]);
                    P.ev.push_back(e);
                }
            }
        } else if (samples.size() > 0) {
            if (defer) {
                const int32_t slot = (int32_t)P.n_slots++;
                Event e{};
                e.kind = EV_SNAP;
                e.a0 = slot;
                P.snap_event.push_back((int64_t)P.ev.size());
                P.ev.push_back(e);
                make_stretches(samples, cfg.stretch_max, [&](size_t i, size_t len, const double *inc,
                                                             const bool *half) {
                    Stretch s{};
                    s.slot = slot;
                    s.d0 = (int32_t)P.def_k.size();
                    s.count = (int32_t)len;
                    s.fam = stretch_family(P.fam_dk, len, inc, half);
                    for (int c = 0; c < 4; ++c) {
                        s.k0[c] = samples.v[c][i];
                        s.dk[c] = P.fam_dk[s.fam][c];
                    }
                    P.def_k.insert(P.def_k.end(), samples.k + i, samples.k + i + len);
                    P.st.push_back(s);
                });
            } else {
                make_stretches(samples, cfg.stretch_max, [&](size_t i, size_t len, const double *inc,
                                                             const bool *) {
                    Event e{};
                    e.kind = EV_ADC;
                    e.a0 = (int32_t)P.inl_k.size();
                    e.count = (int32_t)len;
                    for (int c = 0; c < 4; ++c) {
                        e.d[c] = samples.v[c][i];
                        e.d[4 + c] = inc[c];
                    }
                    P.inl_k.insert(P.inl_k.end(), samples.k + i, samples.k + i + len);
                    P.ev.push_back(e);
                });
            }
        }
        if (b > a) {
            Event e{};
            e.kind = EV_END;
            e.d[0] = K[0];
            e.d[1] = K[1];
            e.d[2] = K[2];
            e.d[3] = q->t[b] - q->t[a];
            e.d[4] = K1[0];
            e.d[5] = K1[1];
            e.d[6] = K1[2];
            P.ev.push_back(e);
            ++P.n_runs;
        }
        if (b == n_int) break;
        // excitation interval b
        {
            const double dt = q->t[b + 1] - q->t[b];
            const double gb[3] = {0.5 * (q->gx[b] + q->gx[b + 1]), 0.5 * (q->gy[b] + q->gy[b + 1]),
                                  0.5 * (q->gz[b] + q->gz[b + 1])};
            // moving spins: the interval mean of G(t) t, the velocity's share of Bz
            double gt[3] = {0, 0, 0};
            if (moving) {
                const double t0 = q->t[b], t1 = q->t[b + 1];
                gt[0] = 0.5 * (q->gx[b] * t0 + q->gx[b + 1] * t1);
                gt[1] = 0.5 * (q->gy[b] * t0 + q->gy[b + 1] * t1);
                gt[2] = 0.5 * (q->gz[b] * t0 + q->gz[b + 1] * t1);
            }
            // A run of excitation intervals with the same field (bitwise) and
            // lengths equal up to the rounding of the time grid (a hard pulse,
            // say), with no other event in between, is one event with a count
            // and the run's mean interval length.
            Event *prev = nullptr;
            if (!P.ev.empty() && P.ev.back().kind == EV_RF && b == rf_run_end) prev = &P.ev.back();
            bool merge = false;
            if (prev) {
                const double tol = 8.0 * std::numeric_limits<double>::epsilon() * std::fabs(q->t[b + 1]);
                merge = prev->count < (1 << 30) && std::fabs(dt - prev->d[7]) <= tol &&
                        std::memcmp(prev->d, gb, sizeof gb) == 0 && prev->d[3] == q->b1_re[b] &&
                        prev->d[4] == q->b1_im[b] && std::memcmp(rf_run_gt, gt, sizeof gt) == 0;
            }
            int32_t count = 1;
            double dtr = dt;
            if (merge) {
                count = prev->count + 1;
                dtr = (q->t[b + 1] - rf_run_t0) / (double)count;
            } else {
                rf_run_t0 = q->t[b];
                std::memcpy(rf_run_gt, gt, sizeof gt);
            }
            rf_run_end = b + 1;
            const double v[8] = {gb[0], gb[1], gb[2], q->b1_re[b], q->b1_im[b],
                                 q->b1_re[b] * q->b1_re[b] + q->b1_im[b] * q->b1_im[b],
                                 -gamma * dtr / (2.0 * kTwoPi), dtr};
            Event e{};
            e.kind = EV_RF;
            e.count = count;
            for (int c = 0; c < 8; ++c) {
                e.d[c] = v[c];
                e.f[c] = (float)v[c];
            }
            // |b1|^2 at least the smallest normal number of each precision, so
            // that |B|^2 = Bz^2 + |b1|^2 > 0 and the kernels' 1/|B| is finite
            // (a zero field then rotates by a zero angle); no non-zero field
            // of an MRI pulse comes near these values
            e.d[5] = std::max(e.d[5], DBL_MIN);
            e.f[5] = std::max(e.f[5], FLT_MIN);
            e.b1sq_f32 = (double)e.f[3] * (double)e.f[3] + (double)e.f[4] * (double)e.f[4];
            if (!(rf_dt_ref > 0.0 && std::fabs(dtr - rf_dt_ref) <= dtr * 0x1p-30)) rf_dt_ref = dtr;
            e.dt_ref = rf_dt_ref;
            e.rot = -1;
            if (moving) {
                for (int c = 0; c < 3; ++c) {
                    e.c64[c] = gt[c];
                    e.c32[c] = (float)gt[c];
                }
            }
            if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0 && gt[0] == 0.0 && gt[1] == 0.0 && gt[2] == 0.0) {
                // zero gradient: for Bz = 0 the field is (b1, 0) for every spin;
                // alpha = cos(phi/2), beta = -i (b1/|b1|) sin(phi/2), phi = -gamma |b1| dt
                const double nb = std::sqrt(v[5]);
                const double h = -0.5 * gamma * nb * dtr;
                const double ar = std::cos(h), ai = 0.0;
                const double sn = std::sin(h) / nb;
                const double br = q->b1_im[b] * sn, bi = -q->b1_re[b] * sn;
                const double ur = ar * ar - ai * ai, ui = -2.0 * ar * ai;
                const double vr = br * br - bi * bi, vi = 2.0 * br * bi;
                const double wr = ar * br + ai * bi, wi = ar * bi - ai * br;
                const double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
                const double c[9] = {2.0 * wr, ur - vr, -(ui + vi), 2.0 * wi, ur + vr, ui - vi,
                                     (ar * ar + ai * ai) - (br * br + bi * bi), -2.0 * pr, -2.0 * pi};
                for (int k = 0; k < 9; ++k) {
                    e.c64[k] = c[k];
                    e.c32[k] = (float)c[k];
                }
                e.rot = 1;
            }
            if (merge) {
                *prev = e;
            } else {
                P.ev.push_back(e);
                ++P.n_rf_events;
            }
            ++P.n_rf;
        }
        a = b + 1;
        if ((int64_t)P.ev.size() >= ((int64_t)1 << 31) - 4) return fail(ctx, KOMA_E_SEQUENCE, "sequence too long");
    }
    if ((int64_t)P.inl_k.size() + (int64_t)P.def_k.size() != q->n_adc)
        return fail(ctx, KOMA_E_SEQUENCE, "internal: ADC samples lost in packing");
    // Runs of single excitation intervals: a0 of an EV_RF event is the number
    // of events from it on that the one-lane kernel takes in one loop, the
    // event itself and the single intervals (count 1, no precomputed
    // rotation) right after it whose relaxation keys are the same in both
    // forms (the FP32 length's bits, the reference length), so that the
    // factors cached for the first hold for all of them.
    for (int64_t i = (int64_t)P.ev.size() - 1; i >= 0; --i) {
        Event &e = P.ev[(size_t)i];
        if (e.kind != EV_RF) continue;
        e.a0 = 1;
        if (i + 1 < (int64_t)P.ev.size()) {
            const Event &x = P.ev[(size_t)i + 1];
            if (x.kind == EV_RF && x.count == 1 && x.rot < 0 &&
                std::memcmp(&x.f[7], &e.f[7], sizeof(float)) == 0 && x.dt_ref == e.dt_ref && x.a0 < (1 << 30))
                e.a0 = 1 + x.a0;
        }
    }

    // ---- packed tiles: with no deferred samples the only per-tile sums are
    // the inline ones, so wavefronts may take 64 consecutive spins across
    // group boundaries. With every non-empty group >= 64 spins a tile holds
    // at most two groups: lanes [0, split) and [split, count), summed into
    // partial rows seg and seg + 1; group g then owns rows tile_off[g] ..
    // tile_off[g + 1] (the rows are in spin order). Saves the partly empty
    // last wavefront of every group (400-spin groups: 7 -> 6.25 per group).
    if (cfg.tile_packing && P.def_k.empty() && P.n_groups > 1 && ph->group_off) {
        const int64_t *go = ph->group_off;
        const int64_t n = ph->n;
        bool ok = n > 0;
        for (int64_t g = 0; ok && g < P.n_groups; ++g) {
            const int64_t sz = go[g + 1] - go[g];
            if (sz != 0 && sz < kWave) ok = false;
        }
        const int64_t n_packed = (n + kWave - 1) / kWave;
        if (ok && n_packed < P.n_tiles) {
            P.tiles.clear();
            int64_t g = 0;     // group of the tile's first spin
            int64_t row = 0;
            for (int64_t s0 = 0; s0 < n; s0 += kWave) {
                while (go[g + 1] <= s0) ++g;  // skips empty groups
                Tile t{};
                t.spin0 = s0;
                t.count = (int32_t)std::min<int64_t>(kWave, n - s0);
                t.group = (int32_t)g;
                t.split = t.count;
                if (go[g + 1] < s0 + t.count) t.split = (int32_t)(go[g + 1] - s0);  // next group starts inside
                t.seg = (int32_t)row;
                row += t.split < t.count ? 2 : 1;
                P.tiles.push_back(t);
            }
            P.n_tiles = (int64_t)P.tiles.size();
            P.n_rows = row;
            P.packed = true;
            // first row of every group: its first spin's tile, second row if it starts mid-tile
            P.tile_off[P.n_groups] = (int32_t)row;
            for (int64_t gg = P.n_groups - 1; gg >= 0; --gg) {
                if (go[gg + 1] == go[gg]) {
                    P.tile_off[gg] = P.tile_off[gg + 1];  // empty: no rows
                } else {
                    const Tile &t = P.tiles[(size_t)(go[gg] / kWave)];
                    P.tile_off[gg] = t.seg + (go[gg] % kWave != 0 ? 1 : 0);
                }
            }
        }
    }

    // ---- lanes per spin of the spin-sequential kernel. With few tiles one
    // lane per spin leaves most SIMDs idle and each wavefront walks the whole
    // program as one dependent chain; G lanes per spin share every segment of
    // map events (composition of affine maps, then a butterfly over the
    // lanes). The planner takes the largest G in {16, 8, 4, 2} that keeps the
    // grid within two wavefronts per SIMD (kSeqgWaves); packed tiles keep
    // one. FP64 maps need twice the registers: at 16 lanes its workgroups take
    // half a tile (512 lanes), each half summing its inline samples into a
    // row of its own.
    {
        int G = cfg.lanes_per_spin;
        if (G == 0) {
            G = 1;
            if (!P.packed)
                for (int cand : {16, 8, 4, 2})
                    if (P.n_tiles * cand <= kSeqgWaves) {
                        G = cand;
                        break;
                    }
        }
        if (P.packed) G = 1;
        P.lanes = G;
        P.half_tiles = cfg.precision == KOMA_FP64 && G == 16;
        if (G > 1) {
            // map events per segment: kSegPerLane per lane (half that for
            // half tiles, as the kernel stages them)
            const int64_t cap = (int64_t)kSegPerLane * G / (P.half_tiles ? 2 : 1);
            const int64_t ne = (int64_t)P.ev.size();
            int64_t e = 0;
            while (e < ne) {
                SegEv g{};
                g.e0 = (int32_t)e;
                while (e < ne && (P.ev[e].kind == EV_RF || P.ev[e].kind == EV_END) && e - g.e0 < cap) ++e;
                g.e1 = (int32_t)e;
                if (e < ne && (P.ev[e].kind == EV_SNAP || P.ev[e].kind == EV_ADC)) {
                    g.obs = 1;
                    ++e;
                }
                P.segs.push_back(g);
            }
        }
    }

    // inline rows of each group: its tiles (or packed rows), two per tile for half tiles
    P.row_off = P.tile_off;
    if (P.half_tiles) {
        for (int32_t &r : P.row_off) r *= 2;
        P.n_rows = 2 * P.n_tiles;
    }

    // ---- sample-parallel layout: blocks of 4*S tiles of one group
    const int64_t n_st = (int64_t)P.st.size();
    // the matrix-core kernels take kMMStretches or kMMStretchesSmall (FP32:
    // requested, or chosen below) or kMMStretches64 (FP64) stretches per
    // workgroup
    const bool mm = cfg.sample_engine == 0;
    const bool mm32 = mm && !P.moving && cfg.precision != KOMA_FP64;
    int64_t mm_batch = cfg.precision == KOMA_FP64 ? kMMStretches64 : kMMStretchesSmall;
    if (mm32 && cfg.stretches_per_wg != 0) mm_batch = cfg.stretches_per_wg;
    const int64_t st_per_wg = mm ? mm_batch : 1;
    auto n_blocks_for = [&](int cand) {
        int64_t nb = 0;
        for (int64_t g = 0; g < P.n_groups; ++g) {
            const int64_t nt = P.tile_off[g + 1] - P.tile_off[g];
            nb += (nt + 4 * cand - 1) / (4 * cand);
        }
        return nb;
    };
    int spl = cfg.spins_per_lane;
    // the vector-ALU kernels take 1, 2, 4 or 8 tiles per wavefront (the
    // largest of those not above a requested value); the matrix-core one any
    if (spl > 0 && !(mm && !P.moving)) spl = spl >= 8 ? 8 : spl >= 4 ? 4 : spl >= 2 ? 2 : 1;
    if (spl == 0 && mm && !P.moving && n_st > 0) {
        // The matrix-core kernels take any number of tiles per wavefront:
        // size the grid to whole rounds of resident workgroups (kMMResident
        // per CU in FP32, kMMResident64 in FP64), so that the last round does not run a few workgroups on an
        // otherwise idle chip: the S whose rounds are fullest, and among those
        // within 2 % of it the largest (fewest partial rows).
        const int64_t slots =
            (int64_t)(cfg.precision == KOMA_FP64 ? kMMResident64 : kMMResident) * std::max(1, ctx->n_cu);
        // for a batch size: the S, and the rounds of resident workgroups it
        // takes. S is searched up to 16 and, where that picks 16 for a grid
        // of at least 32 rounds (there each workgroup's epilogue and partials
        // weigh more than the last round's tail), up to 32.
        auto choose = [&](int64_t nb_st, int &s_out, int64_t &rounds_out) {
            const int64_t batches = (n_st + nb_st - 1) / nb_st * std::max<int64_t>(1, P.n_coils);
            double eff[33] = {};
            int64_t rounds[33] = {};
            double best_eff = 0.0;
            int smax = 16;
            for (int cand = 1; cand <= smax; ++cand) {
                const int64_t w = n_blocks_for(cand) * batches;
                rounds[cand] = (w + slots - 1) / slots;
                eff[cand] = (double)w / (double)(rounds[cand] * slots);
                best_eff = std::max(best_eff, eff[cand]);
            }
            s_out = 1;
            for (int cand = smax; cand >= 1; --cand)
                if (eff[cand] >= best_eff - 0.02) {
                    s_out = cand;
                    break;
                }
            if (s_out == 16 && rounds[16] >= 32) {
                smax = 32;
                best_eff = 0.0;
                for (int cand = 1; cand <= smax; ++cand) {
                    const int64_t w = n_blocks_for(cand) * batches;
                    rounds[cand] = (w + slots - 1) / slots;
                    eff[cand] = (double)w / (double)(rounds[cand] * slots);
                    best_eff = std::max(best_eff, eff[cand]);
                }
                for (int cand = smax; cand >= 16; --cand)
                    if (eff[cand] >= best_eff - 0.02) {
                        s_out = cand;
                        break;
                    }
            }
            rounds_out = rounds[s_out];
        };
        int64_t rounds = 0;
        choose(mm_batch, spl, rounds);
        if (mm32 && cfg.stretches_per_wg == 0) {
            // FP32: 6 stretches per workgroup do the same work in about 3.5 %
            // less time than 4 (fewer LDS round trips for the shared
            // operands), unless their coarser grid takes more rounds: compare
            // rounds x tiles per wavefront x stretches per workgroup. The
            // partial sums (device footprint, and the reduction's reads) grow
            // with the number of spin blocks, which that count leaves out:
            // 6 only where it does not take more blocks.
            int s6;
            int64_t r6;
            choose(kMMStretches, s6, r6);
            if ((double)r6 * s6 * kMMStretches * 0.965 < (double)rounds * spl * mm_batch &&
                n_blocks_for(s6) <= n_blocks_for(spl)) {
                mm_batch = kMMStretches;
                spl = s6;
            }
        }
    } else if (spl == 0) {
        spl = 1;
        for (int cand : {8, 4, 2}) {  // largest S that still gives >= 8 workgroups per CU
            if (n_blocks_for(cand) * std::max<int64_t>((n_st + st_per_wg - 1) / st_per_wg, 1) >= (mm ? 1024 : 2048)) {
                spl = cand;
                break;
            }
        }
    }
    P.spl = spl;
    P.blk_off.assign(P.n_groups + 1, 0);
    for (int64_t g = 0; g < P.n_groups && !P.packed; ++g) {
        P.blk_off[g] = (int32_t)P.blocks.size();
        for (int32_t t = P.tile_off[g]; t < P.tile_off[g + 1]; t += 4 * spl) {
            Block bl{};
            bl.tile0 = t;
            bl.ntiles = std::min<int32_t>(4 * spl, P.tile_off[g + 1] - t);
            bl.group = (int32_t)g;
            P.blocks.push_back(bl);
        }
    }
    P.blk_off[P.n_groups] = (int32_t)P.blocks.size();
    const int64_t n_blocks = (int64_t)P.blocks.size();
    // stretches per workgroup: keep >= ~16 workgroups per CU, share spin loads beyond that
    P.per_wg = 1;
    if (mm) {
        P.per_wg = mm_batch;
    } else if (n_st > 0) {
        const int64_t target = 4096;
        const int64_t wgs = n_blocks * n_st;
        P.per_wg = std::max<int64_t>(1, std::min<int64_t>(16, wgs / target));
    }

    // ---- deferred sample chunks, sized by the partial budget
    if (n_st > 0) {
        const int64_t cap_cols = std::max<int64_t>(
            kStretchMax,
            (int64_t)(cfg.partial_budget / (size_t)(std::max<int64_t>(n_blocks, 1) * 16 * P.n_sig)));
        int64_t s = 0;
        while (s < n_st) {
            Chunk c;
            c.s0 = s;
            c.c0 = P.st[s].d0;
            int64_t cols = 0;
            while (s < n_st && (cols + P.st[s].count <= cap_cols || cols == 0)) {
                cols += P.st[s].count;
                ++s;
            }
            c.s1 = s;
            c.c1 = c.c0 + cols;
            // families together (each stretch keeps its own columns), so that
            // the stretches of one workgroup mostly share their increments
            std::stable_sort(P.st.begin() + c.s0, P.st.begin() + c.s1,
                             [](const Stretch &x, const Stretch &y) { return x.fam < y.fam; });
            int32_t last = 0;
            for (int64_t i = c.s0; i < c.s1; ++i) last = std::max(last, P.st[i].slot);
            c.ready = P.snap_event[last] + 1;
            P.chunks.push_back(c);
            P.max_cols = std::max(P.max_cols, cols);
        }
    }
    return KOMA_OK;
}

// Device bytes of a simulation of plan P: every buffer rounded up as the
// request allocator rounds it (koma_req_open allocates exactly this list).
static size_t plan_footprint(const Plan &P, bool fp64, bool with_state, bool with_phantom) {
    const size_t r = fp64 ? 8 : 4;
    const size_t n_pad = (size_t)P.n_tiles * kWave;
    const size_t ns = (size_t)P.n_sig;
    size_t b = 0;
    b += pool_round(P.ev.size() * sizeof(Event)) + pool_round(P.st.size() * sizeof(Stretch));
    b += pool_round(P.tiles.size() * sizeof(Tile)) + pool_round(P.blocks.size() * sizeof(Block));
    b += pool_round(P.row_off.size() * 4) + pool_round(P.blk_off.size() * 4);
    b += pool_round(P.inl_k.size() * 4) + pool_round(P.def_k.size() * 4);
    b += pool_round(P.segs.size() * sizeof(SegEv));
    b += pool_round((size_t)P.n_slots * n_pad * 2 * r);                         // snapshots
    b += pool_round(ns * (size_t)P.n_rows * P.inl_k.size() * 2 * r);             // inline partials
    b += pool_round(ns * (size_t)P.blocks.size() * (size_t)P.max_cols * 16);     // cross-workgroup partials
    b += pool_round(ns * (size_t)P.n_groups * (size_t)P.n_adc * 16);             // signal
    if (with_state) b += pool_round(n_pad * 2 * r) + pool_round(n_pad * r);
    if (with_phantom) {
        const size_t arr = pool_round((size_t)P.n_spins * 4);
        b += arr * (7 + (P.moving ? 3 : 0)) + 2 * pool_round((size_t)P.n_spins * (size_t)P.n_coils * 4) *
                                                   (P.n_coils > 0 ? 1 : 0);
    }
    return b;
}

// ---------------------------------------------------------------- profiling

static koma_status prof_begin(koma_ctx *ctx, hipStream_t s, hipEvent_t *out) {
    *out = nullptr;
    if (!ctx->prof) return KOMA_OK;
    hipEvent_t e;
    if (!ctx->ev_free.empty()) {
        e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
    } else {
        HIPCHK(ctx, hipEventCreate(&e));
    }
    HIPCHK(ctx, hipEventRecord(e, s));
    *out = e;
    return KOMA_OK;
}

static koma_status prof_end(koma_ctx *ctx, hipStream_t s, hipEvent_t a, int kind, int64_t work) {
    if (!ctx->prof || !a) return KOMA_OK;
    hipEvent_t e;
    if (!ctx->ev_free.empty()) {
        e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
    } else {
        HIPCHK(ctx, hipEventCreate(&e));
    }
    HIPCHK(ctx, hipEventRecord(e, s));
    ctx->recs.push_back({a, e, kind, work});
    return KOMA_OK;
}

// ---------------------------------------------------------------- execution

namespace {

struct Bufs {  // device views used by the launch sequence
    PhantomDev ph;
    const Event *ev;
    const Stretch *st;
    const Tile *tiles;
    const Block *blocks;
    const int32_t *toff, *boff, *inl, *def;
    void *snap, *pa;
    double *pb;
    double *sig;
    void *mxy, *mz;
    const int32_t *gate = nullptr;  // the sums are written only if *gate == 0 (device-checked phantoms)
    const SegEv *segs = nullptr;
};

}  // namespace

#define LAUNCH(ctx, kind, work, s, expr)                                                  \
    do {                                                                                  \
        hipEvent_t pa_;                                                                   \
        koma_status st_ = prof_begin((ctx), (s), &pa_);                                   \
        if (st_ != KOMA_OK) return st_;                                                   \
        if ((expr) != 0) return fail((ctx), KOMA_E_DEVICE, "kernel launch failed: %s", \
                                     hipGetErrorString(hipGetLastError()));               \
        st_ = prof_end((ctx), (s), pa_, (kind), (work));                                  \
        if (st_ != KOMA_OK) return st_;                                                   \
    } while (0)

static koma_status run_seq(koma_ctx *ctx, const Plan &P, bool fp64, const Bufs &B, int64_t e0, int64_t e1,
                           bool init, bool store, hipStream_t s, int32_t *vbits = nullptr) {
    if (e1 <= e0) return KOMA_OK;
    SeqArgs a{};
    a.vbits = vbits;
    a.ph = B.ph;
    a.tiles = B.tiles;
    a.n_tiles = P.n_tiles;
    a.ev = B.ev;
    a.e0 = e0;
    a.e1 = e1;
    a.inv_gamma = 1.0 / P.gamma;
    a.init = init ? 1 : 0;
    a.store = store ? 1 : 0;
    a.mxy = B.mxy;
    a.mz = B.mz;
    a.snap = B.snap;
    a.pa = B.pa;
    a.n_rows = P.n_rows;
    a.n_inline = (int64_t)P.inl_k.size();
    a.lanes = P.lanes;
    a.half_tiles = P.half_tiles ? 1 : 0;
    if (P.lanes > 1) {
        // segments that reach into [e0, e1): the first whose events end
        // after e0, up to the first that starts at or after e1
        const auto &S = P.segs;
        auto first = std::partition_point(S.begin(), S.end(), [&](const SegEv &g) { return g.e1 + g.obs <= e0; });
        auto last = std::partition_point(S.begin(), S.end(), [&](const SegEv &g) { return g.e0 < e1; });
        a.segs = B.segs;
        a.s0 = first - S.begin();
        a.s1 = last - S.begin();
    }
    LAUNCH(ctx, K_SEQ, P.n_tiles * kWave * (e1 - e0), s, launch_seq(fp64, P.moving, a, s));
    return KOMA_OK;
}

static koma_status run_chunk(koma_ctx *ctx, const Plan &P, bool fp64, const Bufs &B, const Chunk &c,
                             hipStream_t s) {
    ParArgs a{};
    a.ph = B.ph;
    a.tiles = B.tiles;
    a.n_tiles = P.n_tiles;
    a.blocks = B.blocks;
    a.n_blocks = (int64_t)P.blocks.size();
    a.st = B.st;
    a.per_wg = P.per_wg;
    a.snap = B.snap;
    a.pb = B.pb;
    a.col0 = c.c0;
    a.cols = c.c1 - c.c0;
    a.engine = ctx->cfg.sample_engine;
    // a plan laid out for the matrix-core kernel (any tiles per wavefront) run
    // with a vector-ALU kernel (1, 2, 4 or 8) after a configuration change
    if ((a.engine != 0 || P.moving) && !(P.spl == 1 || P.spl == 2 || P.spl == 4 || P.spl == 8))
        return fail(ctx, KOMA_E_STATE, "the plan was laid out for the matrix-core sample sums; "
                                       "set sample_engine back to 0 or open the request again");
    const int64_t max_st = 65535 * P.per_wg;  // grid.y limit
    for (int64_t s0 = c.s0; s0 < c.s1; s0 += max_st) {
        a.s0 = s0;
        a.s1 = std::min(c.s1, s0 + max_st);
        int64_t cols = 0;
        for (int64_t i = a.s0; i < a.s1; ++i) cols += P.st[i].count;
        LAUNCH(ctx, K_PAR, P.n_tiles * kWave * cols, s, launch_par(fp64, P.spl, a, s));
    }
    ReduceArgs r{};
    r.n_sig = P.n_sig;
    r.part_stride = (int64_t)P.blocks.size() * (c.c1 - c.c0);
    r.part = B.pb;
    r.cols = c.c1 - c.c0;
    r.row_off = B.boff;
    r.n_groups = P.n_groups;
    r.col_to_adc = B.def + c.c0;
    r.sig = B.sig;
    r.gate = B.gate;
    r.n_adc = P.n_adc;
    LAUNCH(ctx, K_RED, P.n_sig * (int64_t)P.blocks.size() * (c.c1 - c.c0) * 16, s, launch_reduce(true, r, s));
    return KOMA_OK;
}

static koma_status run_inline_reduce(koma_ctx *ctx, const Plan &P, bool fp64, const Bufs &B, hipStream_t s) {
    if (P.inl_k.empty()) return KOMA_OK;
    ReduceArgs r{};
    r.n_sig = P.n_sig;
    r.part_stride = P.n_rows * (int64_t)P.inl_k.size();
    r.part = B.pa;
    r.cols = (int64_t)P.inl_k.size();
    r.row_off = B.toff;
    r.n_groups = P.n_groups;
    r.col_to_adc = B.inl;
    r.sig = B.sig;
    r.gate = B.gate;
    r.n_adc = P.n_adc;
    LAUNCH(ctx, K_RED, P.n_sig * P.n_rows * r.cols * (fp64 ? 16 : 8), s, launch_reduce(fp64, r, s));
    return KOMA_OK;
}

static koma_status validate_device_phantom(koma_ctx *ctx, const PhantomDev &ph, int64_t n, DevMem &flags,
                                           hipStream_t s) {
    const int64_t nwg = (n + kWG - 1) / kWG;
    koma_status st = dev_reserve(ctx, flags, (size_t)nwg * 4);
    if (st != KOMA_OK) return st;
    LAUNCH(ctx, K_AUX, n, s, launch_validate(ph, n, (int32_t *)flags.p, s));
    std::vector<int32_t> h((size_t)nwg);
    HIPCHK(ctx, hipMemcpyAsync(h.data(), flags.p, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    int32_t bad = 0;
    for (int32_t v : h) bad |= v;
    if (bad & 1) return fail(ctx, KOMA_E_PHANTOM, "non-finite position, velocity, dw or PD in the phantom");
    if (bad & 2) return fail(ctx, KOMA_E_PHANTOM, "PD < 0 in the phantom");
    if (bad & 4) return fail(ctx, KOMA_E_PHANTOM, "T1/T2 must be > 0 (or +inf)");
    if (bad & 8) return fail(ctx, KOMA_E_PHANTOM, "non-finite coil sensitivity in the phantom");
    return KOMA_OK;
}

// ---------------------------------------------------------------- C ABI

namespace koma {
// Errors of calls that have no context (koma_ctx_create, koma_discretize).
void set_thread_error(const std::string &msg) { g_create_error = msg; }
}  // namespace koma

extern "C" {

void koma_config_default(koma_config *cfg) {
    if (!cfg) return;
    cfg->precision = KOMA_MIXED;
    cfg->spins_per_lane = 0;
    cfg->wg_size = 256;
    cfg->chunk_events = 4096;
    cfg->hbm_budget = 0;
    cfg->partial_budget = (size_t)1 << 30;
    cfg->defer_min_adc = 32;
    cfg->stretch_max = 128;
    cfg->sample_engine = 0;
    cfg->tile_packing = 1;
    cfg->lanes_per_spin = 0;
    cfg->stretches_per_wg = 0;
}

koma_status koma_ctx_create(int device, const koma_config *cfg, koma_ctx **out) {
    if (!out) return fail(nullptr, KOMA_E_ARG, "out is NULL");
    *out = nullptr;
    koma_config c;
    if (cfg)
        c = *cfg;
    else
        koma_config_default(&c);
    if (check_config(nullptr, &c) != KOMA_OK) return KOMA_E_ARG;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(nullptr, KOMA_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, KOMA_E_ARG, "device %d out of range", device);
    if ((e = hipSetDevice(device)) != hipSuccess)
        return fail(nullptr, KOMA_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    koma_ctx *ctx = new (std::nothrow) koma_ctx();
    if (!ctx) return fail(nullptr, KOMA_E_NOMEM, "out of host memory");
    ctx->device = device;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            ctx->n_cu = cus;
    }
    ctx->cfg = c;
    ctx->nz_err = noalloc_scratch_attach(device, &ctx->nz_scratch);
    if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete ctx;
        return fail(nullptr, KOMA_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return KOMA_OK;
}

void koma_ctx_destroy(koma_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->async_pending) (void)hipEventSynchronize(ctx->async_done);
    DevMem *all[] = {&ctx->s_ev, &ctx->s_st, &ctx->s_tiles, &ctx->s_blocks, &ctx->s_toff, &ctx->s_boff,
                     &ctx->s_inl, &ctx->s_def, &ctx->s_snap, &ctx->s_pa, &ctx->s_pb, &ctx->s_sig,
                     &ctx->s_mxy, &ctx->s_mz, &ctx->s_flags, &ctx->s_vcount, &ctx->s_mf};
    for (DevMem *m : all) dev_free(*m);
    for (DevMem &m : ctx->s_ph) dev_free(m);
    DevMem *mrf[] = {&ctx->m_src_d, &ctx->m_src_x, &ctx->m_dh, &ctx->m_xh, &ctx->m_dexp, &ctx->m_xexp,
                     &ctx->m_inv, &ctx->m_ps, &ctx->m_pi, &ctx->m_best, &ctx->m_proj,
                     &ctx->l_v, &ctx->l_y, &ctx->l_zp, &ctx->l_z, &ctx->l_basis, &ctx->l_sv, &ctx->l_out};
    for (DevMem *m : mrf) dev_free(*m);
    for (auto &sl : ctx->ring) {
        if (sl.copied) (void)hipEventSynchronize(sl.copied);
        dev_free(sl.d);
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.copied) (void)hipEventDestroy(sl.copied);
    }
    if (ctx->async_done) (void)hipEventDestroy(ctx->async_done);
    if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
    pool_trim(ctx);
    for (auto &r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *koma_last_error(const koma_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

koma_status koma_ctx_set_config(koma_ctx *ctx, const koma_config *cfg) {
    if (!ctx) return KOMA_E_ARG;
    koma_status st = check_config(ctx, cfg);
    if (st != KOMA_OK) return st;
    ctx->cfg = *cfg;
    return KOMA_OK;
}

koma_status koma_footprint(const koma_phantom *ph, const koma_sequence *seq, const koma_config *cfg,
                           size_t *bytes) {
    koma_ctx tmp;
    if (!bytes) return KOMA_E_ARG;
    koma_config c;
    if (cfg)
        c = *cfg;
    else
        koma_config_default(&c);
    koma_status st;
    if ((st = check_config(&tmp, &c)) != KOMA_OK) return st;
    if ((st = check_phantom_shape(&tmp, ph)) != KOMA_OK) return st;
    if ((st = check_sequence(&tmp, seq)) != KOMA_OK) return st;
    Plan P;
    if ((st = build_plan(&tmp, c, 2.6752218744e8, ph, seq, P)) != KOMA_OK) return st;
    *bytes = plan_footprint(P, c.precision == KOMA_FP64, true, true);
    return KOMA_OK;
}

koma_status koma_ctx_mem(const koma_ctx *ctx, size_t *held, size_t *cached, size_t *peak) {
    if (!ctx) return KOMA_E_ARG;
    if (held) *held = ctx->held_bytes;
    if (cached) *cached = ctx->pool_bytes;
    if (peak) *peak = ctx->mem_peak;
    return KOMA_OK;
}

koma_status koma_ctx_profile(koma_ctx *ctx, int on) {
    if (!ctx) return KOMA_E_ARG;
    for (auto &r : ctx->recs) {
        ctx->ev_free.push_back(r.a);
        ctx->ev_free.push_back(r.b);
    }
    ctx->recs.clear();
    for (int k = 0; k < K_KINDS; ++k) {
        ctx->tot_ms[k] = 0;
        ctx->n_launch[k] = 0;
        ctx->work[k] = 0;
    }
    ctx->prof = on != 0;
    return KOMA_OK;
}

koma_status koma_ctx_kernel_stats(koma_ctx *ctx, int kind, double *total_ms, int64_t *launches,
                                  int64_t *work_units) {
    if (!ctx || kind < 0 || kind >= K_KINDS) return KOMA_E_ARG;
    if (ctx->poisoned) return KOMA_E_DEVICE;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    for (auto &r : ctx->recs) {
        HIPCHK(ctx, hipEventSynchronize(r.b));
        float ms = 0;
        HIPCHK(ctx, hipEventElapsedTime(&ms, r.a, r.b));
        ctx->tot_ms[r.kind] += ms;
        ctx->n_launch[r.kind] += 1;
        ctx->work[r.kind] += r.work;
        ctx->ev_free.push_back(r.a);
        ctx->ev_free.push_back(r.b);
    }
    ctx->recs.clear();
    if (total_ms) *total_ms = ctx->tot_ms[kind];
    if (launches) *launches = ctx->n_launch[kind];
    if (work_units) *work_units = ctx->work[kind];
    return KOMA_OK;
}

// Everything of one simulation up to the outputs, enqueued on the stream:
// validation, packing, upload, kernels, and (device-resident phantoms) the
// commit of the results if the device-side validation found them clean. With
// async, the validation bits go to `status` (device) and nothing is waited for.
static koma_status simulate_enqueue(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                                    const koma_sequence *seq, koma_mem where, void *hip_stream, double *sig,
                                    double *m_final, bool async, int32_t *status, bool noalloc = false) {
    if (!ctx) return KOMA_E_ARG;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    ctx->err.clear();
    koma_status st;
    if (where != KOMA_HOST && where != KOMA_DEVICE) return fail(ctx, KOMA_E_ARG, "bad koma_mem");
    if (async && where != KOMA_DEVICE)
        return fail(ctx, KOMA_E_ARG, "koma_simulate_async takes device-resident inputs and outputs");
    if (noalloc && where != KOMA_DEVICE)
        return fail(ctx, KOMA_E_ARG, "koma_simulate_noalloc takes device-resident inputs and outputs");
    if (noalloc && !ctx->nz_scratch)
        return fail(ctx, KOMA_E_DEVICE, "static scratch of device %d unavailable: %s", ctx->device,
                    hipGetErrorString(ctx->nz_err));
    if ((st = check_scanner(ctx, sc)) != KOMA_OK) return st;
    if ((st = check_phantom_shape(ctx, ph)) != KOMA_OK) return st;
    if ((st = check_sequence(ctx, seq)) != KOMA_OK) return st;
    if (seq->n_adc > 0 && !sig) return fail(ctx, KOMA_E_ARG, "sig is NULL");
    if (where == KOMA_HOST && (st = check_phantom_values_host(ctx, ph)) != KOMA_OK) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const bool fp64 = ctx->cfg.precision == KOMA_FP64;
    const size_t r = fp64 ? 8 : 4;
    // the context's scratch is reused: order this call after queued work
    if (ctx->async_pending) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->async_done, 0));

    Plan &P = ctx->plan;
    koma_config pcfg = ctx->cfg;
    // without allocation the cross-workgroup partials of a launch share the
    // static scratch with the rest: at most half of it
    if (noalloc) pcfg.partial_budget = std::min(pcfg.partial_budget, kNoallocScratchBytes / 2);
    if ((st = build_plan(ctx, pcfg, sc->gamma, ph, seq, P)) != KOMA_OK) return st;
    if (ctx->cfg.hbm_budget && plan_footprint(P, fp64, m_final != nullptr, where == KOMA_HOST) > ctx->cfg.hbm_budget)
        return fail(ctx, KOMA_E_BUDGET, "footprint exceeds hbm_budget");

    Bufs B{};
    // phantom
    const float *src[kPhArrays];
    ph_sources(ph, src);
    const float *dptr[kPhArrays] = {};
    for (int i = 0; i < kPhArrays; ++i) {
        if (!ph_used(ph, i)) continue;
        if (where == KOMA_HOST) {
            if ((st = dev_reserve(ctx, ctx->s_ph[i], ph_bytes(ph, i))) != KOMA_OK) return st;
            HIPCHK(ctx, hipMemcpyAsync(ctx->s_ph[i].p, src[i], ph_bytes(ph, i), hipMemcpyHostToDevice, s));
            dptr[i] = (const float *)ctx->s_ph[i].p;
        } else {
            dptr[i] = src[i];
        }
    }
    B.ph = ph_dev(dptr, P.moving, ph->n, P.n_coils);

    // device-resident phantom: the spin-sequential kernel validates the
    // values it reads (their bits ORed into one word, which the upload
    // zeroes first); the final sums are written to the caller's buffers only
    // if they are clean, and the host reads the word after the one
    // synchronisation at the end
    const bool dev_check = where == KOMA_DEVICE;
    const bool store = m_final != nullptr;
    const size_t n_pad = (size_t)P.n_tiles * kWave;
    const size_t nsig = (size_t)P.n_sig;
    const size_t snap_b = (size_t)P.n_slots * n_pad * 2 * r;
    const size_t pa_b = nsig * (size_t)P.n_rows * P.inl_k.size() * 2 * r;
    const size_t pb_b = nsig * P.blocks.size() * (size_t)P.max_cols * 16;

    // packed tables: one pinned staging buffer, one upload
    struct Part {
        const void *src;
        size_t bytes, off;
    } parts[9] = {{P.ev.data(), P.ev.size() * sizeof(Event), 0},
                  {P.st.data(), P.st.size() * sizeof(Stretch), 0},
                  {P.tiles.data(), P.tiles.size() * sizeof(Tile), 0},
                  {P.blocks.data(), P.blocks.size() * sizeof(Block), 0},
                  {P.row_off.data(), P.row_off.size() * 4, 0},
                  {P.blk_off.data(), P.blk_off.size() * 4, 0},
                  {P.inl_k.data(), P.inl_k.size() * 4, 0},
                  {P.def_k.data(), P.def_k.size() * 4, 0},
                  {P.segs.data(), P.segs.size() * sizeof(SegEv), 0}};
    size_t total = 0;
    for (auto &pt : parts) {
        pt.off = total;
        total += (pt.bytes + 255) & ~(size_t)255;
    }
    auto a256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *tb = nullptr;
    int32_t *flag_total = nullptr;
    char *nz = nullptr;  // next free byte of the static scratch
    if (noalloc) {
        // layout: validation word, packed tables, snapshots, partials, state
        const size_t need = 256 + total + a256(snap_b) + a256(pa_b) + a256(pb_b) +
                            (store ? a256(n_pad * 2 * r) + a256(n_pad * r) : 0);
        if (need > kNoallocScratchBytes)
            return fail(ctx, KOMA_E_BUDGET, "the simulation needs %zu bytes of scratch; the static scratch holds %zu",
                        need, kNoallocScratchBytes);
        nz = (char *)ctx->nz_scratch;
        flag_total = (int32_t *)nz;
        tb = nz + 256;
        nz = tb + total;
        for (auto &pt : parts)
            if (pt.bytes) HIPCHK(ctx, hipMemcpyAsync(tb + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice, s));
        // the validation word starts at zero (a kernel, not a memset node)
        LAUNCH(ctx, K_AUX, 1, s, launch_upload(nullptr, nullptr, 0, flag_total, s));
    } else {
        if (dev_check) {
            if ((st = dev_reserve(ctx, ctx->s_vcount, 256)) != KOMA_OK) return st;
            flag_total = (int32_t *)ctx->s_vcount.p;
        }
        koma_ctx::StageSlot &sl = ctx->ring[ctx->ring_next];
        ctx->ring_next = (ctx->ring_next + 1) % koma_ctx::kStageRing;
        // the host only learns from it that the upload kernel has read the
        // staging: no memory fence when it is reached (a system-scope fence
        // writes back and invalidates the caches ahead of the following kernels)
        if (!sl.copied)
            HIPCHK(ctx, hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming | hipEventDisableSystemFence));
        if (sl.pending) HIPCHK(ctx, hipEventSynchronize(sl.copied));  // the host staging is free again
        if (sl.h && sl.cap < total) {
            HIPCHK(ctx, hipHostFree(sl.h));
            sl.h = nullptr;
            sl.cap = 0;
        }
        if (!sl.h) {
            HIPCHK(ctx, hipHostMalloc(&sl.h, total, hipHostMallocDefault));
            sl.cap = total;
        }
        if (!ctx->h_flag) HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_flag, 64, hipHostMallocDefault));
        for (auto &pt : parts)
            if (pt.bytes) memcpy((char *)sl.h + pt.off, pt.src, pt.bytes);
        if ((st = dev_reserve(ctx, sl.d, total)) != KOMA_OK) return st;
        // copied by a kernel that reads the pinned staging directly (no DMA copy)
        void *hdev = nullptr;
        HIPCHK(ctx, hipHostGetDevicePointer(&hdev, sl.h, 0));
        LAUNCH(ctx, K_AUX, (int64_t)(total / 16), s, launch_upload(hdev, sl.d.p, total, flag_total, s));
        HIPCHK(ctx, hipEventRecord(sl.copied, s));
        sl.pending = true;
        tb = (char *)sl.d.p;
    }
    B.ev = (const Event *)(tb + parts[0].off);
    B.st = (const Stretch *)(tb + parts[1].off);
    B.tiles = (const Tile *)(tb + parts[2].off);
    B.blocks = (const Block *)(tb + parts[3].off);
    B.toff = (const int32_t *)(tb + parts[4].off);
    B.boff = (const int32_t *)(tb + parts[5].off);
    B.inl = (const int32_t *)(tb + parts[6].off);
    B.def = (const int32_t *)(tb + parts[7].off);
    B.segs = (const SegEv *)(tb + parts[8].off);

    if (noalloc) {
        B.snap = nz;
        nz += a256(snap_b);
        B.pa = nz;
        nz += a256(pa_b);
        B.pb = (double *)nz;
        nz += a256(pb_b);
        if (store) {
            B.mxy = nz;
            nz += a256(n_pad * 2 * r);
            B.mz = nz;
        }
    } else {
        if ((st = dev_reserve(ctx, ctx->s_snap, snap_b)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->s_pa, pa_b)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->s_pb, pb_b)) != KOMA_OK) return st;
        if (store) {
            if ((st = dev_reserve(ctx, ctx->s_mxy, n_pad * 2 * r)) != KOMA_OK) return st;
            if ((st = dev_reserve(ctx, ctx->s_mz, n_pad * r)) != KOMA_OK) return st;
            if (!dev_check && (st = dev_reserve(ctx, ctx->s_mf, (size_t)ph->n * 24)) != KOMA_OK) return st;
        }
        B.snap = ctx->s_snap.p;
        B.pa = ctx->s_pa.p;
        B.pb = (double *)ctx->s_pb.p;
        B.mxy = ctx->s_mxy.p;
        B.mz = ctx->s_mz.p;
    }
    const size_t sig_n = nsig * (size_t)P.n_groups * P.n_adc * 2;  // doubles
    if (dev_check) {
        // every sample of every signal plane is written by the final sums,
        // straight into the caller's buffer, gated by the validation flag
        B.sig = sig;
        B.gate = flag_total;
    } else {
        if ((st = dev_reserve(ctx, ctx->s_sig, sig_n * 8)) != KOMA_OK) return st;
        B.sig = (double *)ctx->s_sig.p;
    }

    if ((st = run_seq(ctx, P, fp64, B, 0, (int64_t)P.ev.size(), true, store, s, flag_total)) !=
        KOMA_OK)
        return st;
    if (P.n_adc > 0) {
        for (const Chunk &c : P.chunks)
            if ((st = run_chunk(ctx, P, fp64, B, c, s)) != KOMA_OK) return st;
        if ((st = run_inline_reduce(ctx, P, fp64, B, s)) != KOMA_OK) return st;
    }
    double *mf = store ? (dev_check ? m_final : (double *)ctx->s_mf.p) : nullptr;
    if (store)
        LAUNCH(ctx, K_AUX, (int64_t)n_pad, s, launch_export(fp64, B.tiles, P.n_tiles, B.mxy, B.mz, mf, B.gate, s));
    if (dev_check) {
        if (noalloc) {
            // the context's own scratch is untouched: later calls need not wait for this one
            if (status) HIPCHK(ctx, hipMemcpyAsync(status, flag_total, 4, hipMemcpyDeviceToDevice, s));
            return KOMA_OK;
        }
        if (async) {
            if (status) HIPCHK(ctx, hipMemcpyAsync(status, flag_total, 4, hipMemcpyDeviceToDevice, s));
            // waited for by later calls on other streams (device-side
            // consumers: a device-scope release suffices) and by the host
            // before it frees or reuses scratch (completion only)
            if (!ctx->async_done)
                HIPCHK(ctx, hipEventCreateWithFlags(&ctx->async_done, hipEventDisableTiming | hipEventReleaseToDevice));
            HIPCHK(ctx, hipEventRecord(ctx->async_done, s));
            ctx->async_pending = true;
            return KOMA_OK;
        }
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_flag, flag_total, 4, hipMemcpyDeviceToHost, s));
    } else {
        if (sig_n) HIPCHK(ctx, hipMemcpyAsync(sig, B.sig, sig_n * 8, hipMemcpyDeviceToHost, s));
        if (store) HIPCHK(ctx, hipMemcpyAsync(m_final, mf, (size_t)ph->n * 24, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->async_pending = false;  // this stream waited for it
    if (dev_check && *ctx->h_flag) {
        const int32_t bad = *ctx->h_flag;
        if (bad & 1) return fail(ctx, KOMA_E_PHANTOM, "non-finite position, velocity, dw or PD in the phantom");
        if (bad & 2) return fail(ctx, KOMA_E_PHANTOM, "PD < 0 in the phantom");
        if (bad & 4) return fail(ctx, KOMA_E_PHANTOM, "T1/T2 must be > 0 (or +inf)");
        return fail(ctx, KOMA_E_PHANTOM, "non-finite coil sensitivity in the phantom");
    }
    return KOMA_OK;
}

koma_status koma_simulate(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                          const koma_sequence *seq, koma_mem where, void *hip_stream, double *sig,
                          double *m_final) {
    return simulate_enqueue(ctx, sc, ph, seq, where, hip_stream, sig, m_final, false, nullptr);
}

koma_status koma_simulate_async(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                                const koma_sequence *seq, void *hip_stream, double *sig, double *m_final,
                                int32_t *status) {
    return simulate_enqueue(ctx, sc, ph, seq, KOMA_DEVICE, hip_stream, sig, m_final, true, status);
}

koma_status koma_simulate_noalloc(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                                  const koma_sequence *seq, void *hip_stream, double *sig, double *m_final,
                                  int32_t *status) {
    return simulate_enqueue(ctx, sc, ph, seq, KOMA_DEVICE, hip_stream, sig, m_final, false, status, true);
}

size_t koma_noalloc_capacity(void) { return kNoallocScratchBytes; }

// ---------------------------------------------------------------- requests

static Bufs req_bufs(koma_req *q) {
    Bufs B{};
    const float *d[kPhArrays];
    for (int i = 0; i < kPhArrays; ++i) d[i] = (const float *)q->ph[i].p;
    B.ph = ph_dev(d, q->plan.moving, q->plan.n_spins, q->plan.n_coils);
    B.ev = (const Event *)q->ev.p;
    B.segs = (const SegEv *)q->segs.p;
    B.st = (const Stretch *)q->st.p;
    B.tiles = (const Tile *)q->tiles.p;
    B.blocks = (const Block *)q->blocks.p;
    B.toff = (const int32_t *)q->toff.p;
    B.boff = (const int32_t *)q->boff.p;
    B.inl = (const int32_t *)q->inl.p;
    B.def = (const int32_t *)q->def.p;
    B.snap = q->snap.p;
    B.pa = q->pa.p;
    B.pb = (double *)q->pb.p;
    B.sig = (double *)q->sig.p;
    B.mxy = q->mxy.p;
    B.mz = q->mz.p;
    return B;
}

static void req_free(koma_req *q) {
    for (DevMem &m : q->ph) pool_put(q->ctx, m);
    DevMem *all[] = {&q->ev, &q->st, &q->tiles, &q->blocks, &q->toff, &q->boff, &q->inl, &q->def,
                     &q->snap, &q->pa, &q->pb, &q->sig, &q->mxy, &q->mz, &q->segs};
    for (DevMem *m : all) pool_put(q->ctx, *m);
}

koma_status koma_req_open(koma_ctx *ctx, const koma_scanner *sc, const koma_phantom *ph,
                          const koma_sequence *seq, koma_mem where, koma_req **out) {
    if (!ctx || !out) return KOMA_E_ARG;
    *out = nullptr;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    ctx->err.clear();
    koma_status st;
    if (where != KOMA_HOST && where != KOMA_DEVICE) return fail(ctx, KOMA_E_ARG, "bad koma_mem");
    if ((st = check_scanner(ctx, sc)) != KOMA_OK) return st;
    if ((st = check_phantom_shape(ctx, ph)) != KOMA_OK) return st;
    if ((st = check_sequence(ctx, seq)) != KOMA_OK) return st;
    if (where == KOMA_HOST && (st = check_phantom_values_host(ctx, ph)) != KOMA_OK) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    koma_req *q = new (std::nothrow) koma_req();
    if (!q) return fail(ctx, KOMA_E_NOMEM, "out of host memory");
    q->ctx = ctx;
    q->fp64 = ctx->cfg.precision == KOMA_FP64;
    if ((st = build_plan(ctx, ctx->cfg, sc->gamma, ph, seq, q->plan)) != KOMA_OK) {
        delete q;
        return st;
    }
    const Plan &P = q->plan;
    q->footprint = plan_footprint(P, q->fp64, true, true);
    if (ctx->cfg.hbm_budget && q->footprint > ctx->cfg.hbm_budget) {
        delete q;
        return fail(ctx, KOMA_E_BUDGET, "request footprint %zu exceeds hbm_budget %zu", q->footprint,
                    ctx->cfg.hbm_budget);
    }
    if (ctx->cfg.hbm_budget && ctx->held_bytes + q->footprint > ctx->cfg.hbm_budget) {
        const size_t held = ctx->held_bytes, need = q->footprint;
        delete q;
        return fail(ctx, KOMA_E_BUDGET, "open requests hold %zu bytes; %zu more would exceed hbm_budget %zu", held,
                    need, ctx->cfg.hbm_budget);
    }
    hipStream_t s = ctx->stream;
    const size_t r = q->fp64 ? 8 : 4;
    const size_t n_pad = (size_t)P.n_tiles * kWave;
    ctx->pool_reserve = q->footprint;  // counted down by every block taken below
    auto bail = [&](koma_status e) {
        ctx->pool_reserve = 0;
        (void)hipStreamSynchronize(s);
        req_free(q);
        delete q;
        return e;
    };
    const float *src[kPhArrays];
    ph_sources(ph, src);
    for (int i = 0; i < kPhArrays; ++i) {
        if (!ph_used(ph, i)) continue;
        if ((st = pool_get(ctx, q->ph[i], ph_bytes(ph, i))) != KOMA_OK) return bail(st);
        hipError_t e = hipMemcpyAsync(q->ph[i].p, src[i], ph_bytes(ph, i),
                                      where == KOMA_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return bail(fail(ctx, KOMA_E_DEVICE, "phantom copy: %s", hipGetErrorString(e)));
    }
    if ((st = pool_upload(ctx, q->ev, P.ev, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->st, P.st, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->tiles, P.tiles, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->blocks, P.blocks, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->toff, P.row_off, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->boff, P.blk_off, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->inl, P.inl_k, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->def, P.def_k, s)) != KOMA_OK) return bail(st);
    if ((st = pool_upload(ctx, q->segs, P.segs, s)) != KOMA_OK) return bail(st);
    if ((st = pool_get(ctx, q->snap, (size_t)P.n_slots * n_pad * 2 * r)) != KOMA_OK) return bail(st);
    const size_t nsig = (size_t)P.n_sig;
    if ((st = pool_get(ctx, q->pa, nsig * (size_t)P.n_rows * P.inl_k.size() * 2 * r)) != KOMA_OK) return bail(st);
    if ((st = pool_get(ctx, q->pb, nsig * P.blocks.size() * (size_t)P.max_cols * 16)) != KOMA_OK) return bail(st);
    if ((st = pool_get(ctx, q->sig, nsig * (size_t)P.n_groups * P.n_adc * 16)) != KOMA_OK) return bail(st);
    if ((st = pool_get(ctx, q->mxy, n_pad * 2 * r)) != KOMA_OK) return bail(st);
    if ((st = pool_get(ctx, q->mz, n_pad * r)) != KOMA_OK) return bail(st);
    if (where == KOMA_DEVICE) {
        Bufs B = req_bufs(q);
        if ((st = validate_device_phantom(ctx, B.ph, ph->n, ctx->s_flags, s)) != KOMA_OK) return bail(st);
    }
    ctx->pool_reserve = 0;
    hipError_t e = hipStreamSynchronize(s);  // inputs are copied before the caller's buffers may change
    if (e != hipSuccess) return bail(fail(ctx, KOMA_E_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e)));
    *out = q;
    return KOMA_OK;
}

koma_status koma_req_advance(koma_req *q, int64_t max_events, void *hip_stream) {
    if (!q) return KOMA_E_ARG;
    koma_ctx *ctx = q->ctx;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    if (q->cancelled) return fail(ctx, KOMA_E_CANCELLED, "request cancelled");
    if (q->finished) return KOMA_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    q->last_stream = s;
    const Plan &P = q->plan;
    const int64_t n_ev = (int64_t)P.ev.size();
    const int64_t step = max_events > 0 ? max_events : ctx->cfg.chunk_events;
    int64_t e1 = std::min(n_ev, q->cursor + step);
    if (P.lanes > 1 && e1 < n_ev) {
        // whole segments only (the cursor is always at a segment end), so a
        // chunked request composes exactly the maps of one whole run: the
        // last segment end within the step, or one segment beyond it
        const auto &S = P.segs;
        auto it = std::partition_point(S.begin(), S.end(), [&](const SegEv &g) { return g.e1 + g.obs <= e1; });
        int64_t end = it == S.begin() ? -1 : (int64_t)(it - 1)->e1 + (it - 1)->obs;
        if (end <= q->cursor) end = (int64_t)it->e1 + it->obs;
        e1 = end;
    }
    Bufs B = req_bufs(q);
    koma_status st;
    if (e1 > q->cursor || q->cursor == 0) {
        if ((st = run_seq(ctx, P, q->fp64, B, q->cursor, e1, q->cursor == 0, true, s)) != KOMA_OK) return st;
        if (n_ev == 0 && q->cursor == 0) {
            // no events: the state is thermal equilibrium; nothing else to do
        }
        q->cursor = e1;
    }
    while (q->next_chunk < P.chunks.size() && P.chunks[q->next_chunk].ready <= q->cursor) {
        if ((st = run_chunk(ctx, P, q->fp64, B, P.chunks[q->next_chunk], s)) != KOMA_OK) return st;
        ++q->next_chunk;
    }
    if (q->cursor >= n_ev && q->next_chunk >= P.chunks.size()) {
        if ((st = run_inline_reduce(ctx, P, q->fp64, B, s)) != KOMA_OK) return st;
        q->finished = true;
    }
    return KOMA_OK;
}

koma_status koma_req_done(const koma_req *q, int *done) {
    if (!q || !done) return KOMA_E_ARG;
    *done = q->finished ? 1 : 0;
    return KOMA_OK;
}

koma_status koma_req_result(koma_req *q, double *sig, void *hip_stream) {
    if (!q) return KOMA_E_ARG;
    koma_ctx *ctx = q->ctx;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    if (q->cancelled) return fail(ctx, KOMA_E_CANCELLED, "request cancelled");
    if (!q->finished) return fail(ctx, KOMA_E_STATE, "request not finished: advance until done");
    const Plan &P = q->plan;
    if (P.n_adc > 0 && !sig) return fail(ctx, KOMA_E_ARG, "sig is NULL");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    q->last_stream = s;
    if (P.n_adc > 0)
        HIPCHK(ctx, hipMemcpyAsync(sig, q->sig.p, (size_t)P.n_sig * P.n_groups * P.n_adc * 16,
                                   hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return KOMA_OK;
}

// Checkpoint layout: header, then the device buffers that carry progress.
struct CkptHeader {
    uint64_t magic;
    int64_t cursor, next_chunk, finished;
    uint64_t n_ev, n_tiles, n_inl, n_slots, n_adc, n_groups, fp64, n_sig;
    uint64_t bytes_mxy, bytes_mz, bytes_snap, bytes_pa, bytes_sig;
};
static constexpr uint64_t kCkptMagic = 0x314b504b414d4f4bull;

static void ckpt_sizes(const koma_req *q, CkptHeader &h) {
    const Plan &P = q->plan;
    const size_t r = q->fp64 ? 8 : 4;
    const size_t n_pad = (size_t)P.n_tiles * kWave;
    h.magic = kCkptMagic;
    h.cursor = q->cursor;
    h.next_chunk = (int64_t)q->next_chunk;
    h.finished = q->finished ? 1 : 0;
    h.n_ev = P.ev.size();
    h.n_tiles = (uint64_t)P.n_tiles;
    h.n_inl = P.inl_k.size();
    h.n_slots = (uint64_t)P.n_slots;
    h.n_adc = (uint64_t)P.n_adc;
    h.n_groups = (uint64_t)P.n_groups;
    h.fp64 = q->fp64 ? 1 : 0;
    h.n_sig = (uint64_t)P.n_sig;
    h.bytes_mxy = n_pad * 2 * r;
    h.bytes_mz = n_pad * r;
    h.bytes_snap = (size_t)P.n_slots * n_pad * 2 * r;
    h.bytes_pa = (size_t)P.n_sig * P.n_rows * P.inl_k.size() * 2 * r;
    h.bytes_sig = (size_t)P.n_sig * P.n_groups * P.n_adc * 16;
}

koma_status koma_req_save(const koma_req *q, void *host_buf, size_t *bytes) {
    if (!q || !bytes) return KOMA_E_ARG;
    koma_ctx *ctx = q->ctx;
    CkptHeader h;
    ckpt_sizes(q, h);
    const size_t total = sizeof h + h.bytes_mxy + h.bytes_mz + h.bytes_snap + h.bytes_pa + h.bytes_sig;
    if (!host_buf) {
        *bytes = total;
        return KOMA_OK;
    }
    if (*bytes < total) return fail(ctx, KOMA_E_ARG, "checkpoint buffer too small (%zu < %zu)", *bytes, total);
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // wait for this request's own work only (other requests keep running)
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (q->last_stream) HIPCHK(ctx, hipStreamSynchronize(q->last_stream));
    char *p = (char *)host_buf;
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    const std::pair<const DevMem *, uint64_t> parts[] = {
        {&q->mxy, h.bytes_mxy}, {&q->mz, h.bytes_mz}, {&q->snap, h.bytes_snap}, {&q->pa, h.bytes_pa}, {&q->sig, h.bytes_sig}};
    for (auto &pr : parts) {
        if (pr.second) HIPCHK(ctx, hipMemcpy(p, pr.first->p, pr.second, hipMemcpyDeviceToHost));
        p += pr.second;
    }
    *bytes = total;
    return KOMA_OK;
}

koma_status koma_req_load(koma_req *q, const void *host_buf, size_t bytes) {
    if (!q || !host_buf) return KOMA_E_ARG;
    koma_ctx *ctx = q->ctx;
    CkptHeader want, got;
    ckpt_sizes(q, want);
    if (bytes < sizeof got) return fail(ctx, KOMA_E_ARG, "checkpoint too short");
    memcpy(&got, host_buf, sizeof got);
    if (got.magic != kCkptMagic || got.n_ev != want.n_ev || got.n_tiles != want.n_tiles || got.n_inl != want.n_inl ||
        got.n_slots != want.n_slots || got.n_adc != want.n_adc || got.n_groups != want.n_groups ||
        got.fp64 != want.fp64 || got.n_sig != want.n_sig || got.bytes_mxy != want.bytes_mxy || got.bytes_snap != want.bytes_snap ||
        got.bytes_pa != want.bytes_pa || got.bytes_sig != want.bytes_sig)
        return fail(ctx, KOMA_E_STATE, "checkpoint does not match this request");
    const size_t total = sizeof got + got.bytes_mxy + got.bytes_mz + got.bytes_snap + got.bytes_pa + got.bytes_sig;
    if (bytes < total) return fail(ctx, KOMA_E_ARG, "checkpoint truncated");
    if (got.cursor < 0 || (uint64_t)got.cursor > got.n_ev || got.next_chunk < 0 ||
        (size_t)got.next_chunk > q->plan.chunks.size())
        return fail(ctx, KOMA_E_STATE, "checkpoint cursor out of range");
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (q->last_stream) HIPCHK(ctx, hipStreamSynchronize(q->last_stream));
    const char *p = (const char *)host_buf + sizeof got;
    const std::pair<DevMem *, uint64_t> parts[] = {
        {&q->mxy, got.bytes_mxy}, {&q->mz, got.bytes_mz}, {&q->snap, got.bytes_snap}, {&q->pa, got.bytes_pa}, {&q->sig, got.bytes_sig}};
    for (auto &pr : parts) {
        if (pr.second) HIPCHK(ctx, hipMemcpy(pr.first->p, p, pr.second, hipMemcpyHostToDevice));
        p += pr.second;
    }
    q->cursor = got.cursor;
    q->next_chunk = (size_t)got.next_chunk;
    q->finished = got.finished != 0;
    return KOMA_OK;
}

void koma_req_close(koma_req *q) {
    if (!q) return;
    (void)hipSetDevice(q->ctx->device);
    // wait only for this request's own work; other requests keep running
    (void)hipStreamSynchronize(q->ctx->stream);
    if (q->last_stream) (void)hipStreamSynchronize(q->last_stream);
    req_free(q);
    delete q;
}

static void fill_info(const Plan &P, koma_req_info *info) {
    info->n_spins = P.n_spins;
    info->n_tiles = P.n_tiles;
    info->n_groups = P.n_groups;
    info->n_adc = P.n_adc;
    info->n_events = (int64_t)P.ev.size();
    info->n_rf = P.n_rf;
    info->n_rf_events = P.n_rf_events;
    info->n_runs = P.n_runs;
    info->n_inline_adc = (int64_t)P.inl_k.size();
    info->n_deferred_adc = (int64_t)P.def_k.size();
    info->n_stretches = (int64_t)P.st.size();
    info->n_families = (int64_t)P.fam_dk.size();
    info->n_snapshots = P.n_slots;
    info->n_blocks = (int64_t)P.blocks.size();
    info->spins_per_lane = P.spl;
    info->stretches_per_wg = P.per_wg;
    info->n_chunks = (int64_t)P.chunks.size();
    info->events_done = 0;
    info->footprint = 0;
    info->n_ends = 0;
    info->n_rf_in_runs = 0;
    info->n_rows = P.n_rows;
    info->lanes_per_spin = P.lanes;
    info->max_single_run = 0;
    for (const Event &e : P.ev) {
        if (e.kind == EV_END) ++info->n_ends;
        if (e.kind == EV_RF && e.count > 1) info->n_rf_in_runs += e.count;
        if (e.kind == EV_RF && e.count == 1) info->max_single_run = std::max<int64_t>(info->max_single_run, e.a0);
    }
}

koma_status koma_req_info_get(const koma_req *q, koma_req_info *info) {
    if (!q || !info) return KOMA_E_ARG;
    fill_info(q->plan, info);
    info->events_done = q->cursor;
    info->footprint = q->footprint;
    return KOMA_OK;
}

koma_status koma_plan_info(const koma_scanner *sc, const koma_phantom *ph, const koma_sequence *seq,
                           const koma_config *cfg, koma_req_info *info) {
    koma_ctx tmp;
    if (!info) return KOMA_E_ARG;
    koma_config c;
    if (cfg)
        c = *cfg;
    else
        koma_config_default(&c);
    koma_status st;
    if ((st = check_config(&tmp, &c)) != KOMA_OK) return st;
    if ((st = check_scanner(&tmp, sc)) != KOMA_OK) return st;
    if ((st = check_phantom_shape(&tmp, ph)) != KOMA_OK) return st;
    if ((st = check_sequence(&tmp, seq)) != KOMA_OK) return st;
    Plan P;
    if ((st = build_plan(&tmp, c, sc->gamma, ph, seq, P)) != KOMA_OK) return st;
    fill_info(P, info);
    info->footprint = plan_footprint(P, c.precision == KOMA_FP64, true, true);
    return KOMA_OK;
}

// ---------------------------------------------------------------- MRF matching

koma_status koma_mrf_match(koma_ctx *ctx, const float *dict, int64_t n_entries, const float *fp, int64_t n_pix,
                           int64_t n_t, koma_mem where, void *hip_stream, int32_t *best, double *proj) {
    if (!ctx) return KOMA_E_ARG;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    ctx->err.clear();
    if (where != KOMA_HOST && where != KOMA_DEVICE) return fail(ctx, KOMA_E_ARG, "bad koma_mem");
    if (n_entries < 1 || n_pix < 1 || n_t < 1) return fail(ctx, KOMA_E_ARG, "n_entries, n_pix and n_t must be >= 1");
    if (!dict || !fp || !best || !proj) return fail(ctx, KOMA_E_ARG, "NULL array");
    if (n_entries > ((int64_t)1 << 30) || n_pix > ((int64_t)1 << 30) || n_t > ((int64_t)1 << 24))
        return fail(ctx, KOMA_E_ARG, "sizes too large");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    koma_status st;
    const int64_t kp = (2 * n_t + 127) / 128 * 128;  // a multiple of every slice width the kernel may use
    const int64_t pt = mrf_pix_tile(), et = mrf_ent_tile();
    const int64_t n_ent_tiles = (n_entries + et - 1) / et;
    const int64_t n_ent_pad = n_ent_tiles * et;
    const int64_t n_pix_pad = (n_pix + pt - 1) / pt * pt;
    const int64_t pix_tiles = n_pix_pad / pt;
    // entry splits: enough workgroups to fill the chip several times over
    const int64_t n_split = std::max<int64_t>(1, std::min<int64_t>(n_ent_tiles, (2048 + pix_tiles - 1) / pix_tiles));
    const int64_t tiles_per_split = (n_ent_tiles + n_split - 1) / n_split;
    const float2 *src_d = (const float2 *)dict, *src_x = (const float2 *)fp;
    if (where == KOMA_HOST) {
        const size_t bd = (size_t)n_entries * n_t * 8, bx = (size_t)n_pix * n_t * 8;
        if ((st = dev_reserve(ctx, ctx->m_src_d, bd)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->m_src_x, bx)) != KOMA_OK) return st;
        HIPCHK(ctx, hipMemcpyAsync(ctx->m_src_d.p, dict, bd, hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyAsync(ctx->m_src_x.p, fp, bx, hipMemcpyHostToDevice, s));
        src_d = (const float2 *)ctx->m_src_d.p;
        src_x = (const float2 *)ctx->m_src_x.p;
    }
    if ((st = dev_reserve(ctx, ctx->m_dh, (size_t)n_ent_pad * kp * 2)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->m_xh, (size_t)n_pix_pad * kp * 2)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->m_dexp, (size_t)n_ent_pad * 4)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->m_xexp, (size_t)n_pix_pad * 4)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->m_inv, (size_t)n_ent_pad * 4)) != KOMA_OK) return st;
    const int64_t n_planes = et / 64 * n_split;
    if ((st = dev_reserve(ctx, ctx->m_ps, (size_t)n_planes * n_pix_pad * 4)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->m_pi, (size_t)n_planes * n_pix_pad * 4)) != KOMA_OK) return st;
    int32_t *d_best = best;
    double *d_proj = proj;
    if (where == KOMA_HOST) {
        if ((st = dev_reserve(ctx, ctx->m_best, (size_t)n_pix * 4)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->m_proj, (size_t)n_pix * 16)) != KOMA_OK) return st;
        d_best = (int32_t *)ctx->m_best.p;
        d_proj = (double *)ctx->m_proj.p;
    }
    uint16_t *dh = (uint16_t *)ctx->m_dh.p, *xh = (uint16_t *)ctx->m_xh.p;
    LAUNCH(ctx, K_AUX, n_ent_pad * n_t, s,
           launch_mrf_pack(src_d, n_entries, n_ent_pad, n_t, kp, dh, (int32_t *)ctx->m_dexp.p, (float *)ctx->m_inv.p, s));
    LAUNCH(ctx, K_AUX, n_pix_pad * n_t, s,
           launch_mrf_pack(src_x, n_pix, n_pix_pad, n_t, kp, xh, (int32_t *)ctx->m_xexp.p, nullptr, s));
    MrfArgs a{};
    a.xh = xh;
    a.dh = dh;
    a.inv_norm2 = (const float *)ctx->m_inv.p;
    a.x_exp = (const int32_t *)ctx->m_xexp.p;
    a.kp = kp;
    a.n_pix = n_pix;
    a.n_pix_pad = n_pix_pad;
    a.n_ent_tiles = n_ent_tiles;
    a.n_split = n_split;
    a.tiles_per_split = tiles_per_split;
    a.n_planes = n_planes;
    a.part_score = (float *)ctx->m_ps.p;
    a.part_idx = (int32_t *)ctx->m_pi.p;
    // work units: complex multiply-adds of the contraction (8 real FLOP each)
    LAUNCH(ctx, K_MRF, n_pix_pad * n_ent_pad * (kp / 2), s, launch_mrf_match(a, s));
    LAUNCH(ctx, K_AUX, n_pix, s, launch_mrf_final(a, d_best, d_proj, s));
    if (where == KOMA_HOST) {
        HIPCHK(ctx, hipMemcpyAsync(best, d_best, (size_t)n_pix * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipMemcpyAsync(proj, d_proj, (size_t)n_pix * 16, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return KOMA_OK;
}

// ---------------------------------------------------------------- dictionary compression

koma_status koma_mrf_svd(koma_ctx *ctx, const float *dict, int64_t n_entries, int64_t n_t, int rank, int oversample,
                         int iters, koma_mem where, void *hip_stream, double *basis, double *sv) {
    if (!ctx) return KOMA_E_ARG;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    ctx->err.clear();
    if (where != KOMA_HOST && where != KOMA_DEVICE) return fail(ctx, KOMA_E_ARG, "bad koma_mem");
    if (!dict || !basis || !sv) return fail(ctx, KOMA_E_ARG, "NULL array");
    if (n_entries < 1 || n_t < 1 || n_entries > ((int64_t)1 << 30) || n_t > ((int64_t)1 << 24))
        return fail(ctx, KOMA_E_ARG, "bad dictionary size");
    const int p = rank + oversample;
    if (rank < 1 || oversample < 0 || p > 32 || p > n_t || iters < 1 || iters > 10000)
        return fail(ctx, KOMA_E_ARG, "need 1 <= rank, 0 <= oversample, rank + oversample <= min(32, n_t), iters >= 1");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    koma_status st;
    const float2 *d = (const float2 *)dict;
    if (where == KOMA_HOST) {
        const size_t bd = (size_t)n_entries * n_t * 8;
        if ((st = dev_reserve(ctx, ctx->m_src_d, bd)) != KOMA_OK) return st;
        HIPCHK(ctx, hipMemcpyAsync(ctx->m_src_d.p, dict, bd, hipMemcpyHostToDevice, s));
        d = (const float2 *)ctx->m_src_d.p;
    }
    const int64_t n_chunks = std::max<int64_t>(1, std::min<int64_t>(64, n_entries / 64));
    if ((st = dev_reserve(ctx, ctx->l_v, (size_t)n_t * p * 16)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->l_z, (size_t)n_t * p * 16)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->l_zp, (size_t)n_chunks * n_t * p * 16)) != KOMA_OK) return st;
    if ((st = dev_reserve(ctx, ctx->l_y, (size_t)n_entries * p * 16)) != KOMA_OK) return st;
    double2 *dbasis = (double2 *)basis;
    double *dsv = sv;
    if (where == KOMA_HOST) {
        if ((st = dev_reserve(ctx, ctx->l_basis, (size_t)n_t * rank * 16)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->l_sv, (size_t)rank * 8)) != KOMA_OK) return st;
        dbasis = (double2 *)ctx->l_basis.p;
        dsv = (double *)ctx->l_sv.p;
    }
    double2 *v = (double2 *)ctx->l_v.p, *y = (double2 *)ctx->l_y.p;
    LAUNCH(ctx, K_AUX, (int64_t)iters * n_entries * n_t * p * 2, s,
           launch_lr_iter(d, n_entries, n_t, p, iters, v, y, (double2 *)ctx->l_zp.p, n_chunks, (double2 *)ctx->l_z.p, s));
    LAUNCH(ctx, K_AUX, n_entries * p * p, s, launch_lr_ritz(y, n_entries, v, n_t, p, rank, dbasis, dsv, s));
    if (where == KOMA_HOST) {
        HIPCHK(ctx, hipMemcpyAsync(basis, dbasis, (size_t)n_t * rank * 16, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipMemcpyAsync(sv, dsv, (size_t)rank * 8, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    return KOMA_OK;
}

koma_status koma_mrf_project(koma_ctx *ctx, const float *rows, int64_t n_rows, int64_t n_t, const double *basis,
                             int rank, koma_mem where, void *hip_stream, float *out) {
    if (!ctx) return KOMA_E_ARG;
    if (ctx->poisoned) return fail(ctx, KOMA_E_DEVICE, "context poisoned by an earlier device error");
    ctx->err.clear();
    if (where != KOMA_HOST && where != KOMA_DEVICE) return fail(ctx, KOMA_E_ARG, "bad koma_mem");
    if (!rows || !basis || !out) return fail(ctx, KOMA_E_ARG, "NULL array");
    if (n_rows < 1 || n_t < 1 || rank < 1 || rank > 32 || n_rows > ((int64_t)1 << 30) || n_t > ((int64_t)1 << 24))
        return fail(ctx, KOMA_E_ARG, "bad sizes (1 <= rank <= 32)");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    koma_status st;
    const float2 *x = (const float2 *)rows;
    const double2 *b = (const double2 *)basis;
    float2 *o = (float2 *)out;
    if (where == KOMA_HOST) {
        const size_t bx = (size_t)n_rows * n_t * 8, bb = (size_t)n_t * rank * 16, bo = (size_t)n_rows * rank * 8;
        if ((st = dev_reserve(ctx, ctx->m_src_x, bx)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->l_basis, bb)) != KOMA_OK) return st;
        if ((st = dev_reserve(ctx, ctx->l_out, bo)) != KOMA_OK) return st;
        HIPCHK(ctx, hipMemcpyAsync(ctx->m_src_x.p, rows, bx, hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyAsync(ctx->l_basis.p, basis, bb, hipMemcpyHostToDevice, s));
        x = (const float2 *)ctx->m_src_x.p;
        b = (const double2 *)ctx->l_basis.p;
        o = (float2 *)ctx->l_out.p;
    }
    LAUNCH(ctx, K_AUX, n_rows * n_t * rank, s, launch_lr_xv(x, n_rows, n_t, b, rank, nullptr, o, s));
    if (where == KOMA_HOST)
        HIPCHK(ctx, hipMemcpyAsync(out, o, (size_t)n_rows * rank * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return KOMA_OK;
}

}  // extern "C"
