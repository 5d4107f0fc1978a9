// Internal layout shared by the host planner (komahip_host.cpp) and the
// kernels (komahip_kernels.hip). Not part of the public ABI.
//
// The packed sequence is an "event program" that every spin runs in the
// same order (so every branch on an event is uniform across a wavefront):
//
//   EV_RF    one excitation-regime interval: spinor rotation about
//            B = (B1, x.G + dw/gamma) by -gamma|B|dt, then relaxation
//            (Eq. Rot_exc and the relaxation update).
//   EV_END   end of a precession block: rotate Mxy by the block's integral
//            phase -2 pi (x.K + f tau) and relax over the elapsed time tau,
//            where K = gamma_bar * sum(G_mean dt) (cycles/m) and f = dw/2pi
//            are accumulated from the block start (section on precession
//            blocks: exact for piecewise-linear G).
//   EV_ADC   `count` evenly spaced ADC samples inside the current precession
//            block, evaluated from the block-start state; the first at the
//            anchor (K0, tau0), the next ones by the constant increment
//            (dK, dtau). The per-wavefront sums go to inline partials.
//   EV_SNAP  store the block-start Mxy in snapshot `a0`: the block's samples
//            are then summed by the sample-parallel kernel from that snapshot
//            (described by Stretch records).
#pragma once
#include <stdint.h>

namespace koma {

enum : int32_t { EV_RF = 0, EV_END = 1, EV_ADC = 2, EV_SNAP = 3 };

struct alignas(16) Event {
    int32_t kind;
    int32_t a0;     // EV_ADC: first inline sample slot; EV_SNAP: snapshot slot;
                    // EV_RF: events from this one on that form a run of single
                    // intervals with the same relaxation keys (>= 1)
    int32_t count;  // EV_ADC: number of samples; EV_RF: identical consecutive intervals (>= 1)
    int32_t rot;    // EV_RF: 1 if the rotation for Bz = 0 is precomputed (zero gradient), else -1
    // EV_RF: gx, gy, gz (T/m, interval mean), b1_re, b1_im (T), |b1|^2,
    //        hs = -gamma dt / (4 pi) (half rotation angle per tesla, in turns), dt (s)
    float f[8];
    // EV_RF: the same eight values in FP64.
    // EV_END: kx, ky, kz (cycles/m), tau (s) of the block end; for moving
    //         spins then the first moments k1x, k1y, k1z (cycles s/m).
    // EV_ADC: kx, ky, kz, tau of the first sample, then dkx, dky, dkz, dtau
    //         (for moving spins count = 1 and the first moments are in c64).
    double d[8];
    // EV_RF: exact |b1|^2 of the FP32-rounded b1 (f[3], f[4]) for the FP32 kernel.
    double b1sq_f32;
    // EV_RF: a reference interval length within 2^-30 (relative) of d[7], the
    // same for every such run of lengths (time points' rounding makes
    // nominally equal lengths differ in their last bits); the FP64 kernel
    // forms the relaxation factors at it and moves them to d[7] exactly:
    // 1 - e^-(t + h) r = eps(t) + (1 - eps(t)) (1 - e^-h r), with 1 - e^-h r =
    // h r to within (h r)^2 / 2
    double dt_ref;
    // EV_RF with zero gradient (rot >= 0): the interval's rotation for spins
    // without off-resonance (Bz = 0, the same field for all of them), the
    // spinor update of Eq. Rot_exc computed once on the host in FP64:
    //   Mxy_re' = c[0] Mz + c[1] Mxy_re + c[2] Mxy_im
    //   Mxy_im' = c[3] Mz + c[4] Mxy_im + c[5] Mxy_re
    //   Mz'     = c[6] Mz + c[7] Mxy_re + c[8] Mxy_im
    // Moving spins, EV_RF with rot < 0: c32/c64[0..2] = interval mean of
    // G(t) t (T s/m); EV_ADC: c64[0..2] = first moments k1 of the sample.
    float c32[12];   // 9 used (rounded for the FP32 kernel)
    double c64[10];  // 9 used
};
static_assert(sizeof(Event) == 256, "Event layout");

// Evenly spaced samples of one deferred precession block, summed by the
// sample-parallel kernel from snapshot `slot`.
struct alignas(16) Stretch {
    int32_t slot;
    int32_t d0;     // deferred sample index of the first sample
    int32_t count;  // samples (<= 128)
    int32_t fam;    // family: stretches of one family have bitwise-equal dk
    double k0[4];   // kx, ky, kz, tau of the first sample
    double dk[4];   // increments between consecutive samples
    // moving spins: first moments of sample j, k1 + j dk1 + j (j - 1) / 2 d2k1
    // (cycles s/m; quadratic in j on a constant gradient)
    double k1[3], dk1[3], d2k1[3];
    double pad;
};
static_assert(sizeof(Stretch) == 160, "Stretch layout");

// 64 consecutive spin slots (one wavefront): of one signal group, or with
// packed tiles of two, lanes [0, split) in one and [split, count) in the next
// non-empty one. Inline sample sums go to partial row `seg` (lanes below
// split) and `seg + 1` (the others).
struct alignas(16) Tile {
    int64_t spin0;
    int32_t count;  // valid lanes (1..64)
    int32_t group;  // group of lane 0
    int32_t split;  // count: one group
    int32_t seg;    // first partial row
    int32_t pad[2];
};
static_assert(sizeof(Tile) == 32, "Tile layout");

// Consecutive tiles of one group summed into one cross-workgroup partial.
struct alignas(16) Block {
    int32_t tile0;
    int32_t ntiles;
    int32_t group;
    int32_t pad;
};

struct PhantomDev {
    const float *x, *y, *z, *pd, *t1, *t2, *dw;
    const float *vx, *vy, *vz;  // nullptr: static spins
    int64_t n;                  // spins (stride of the sensitivity planes)
    int64_t n_coils;            // 0: plain sums
    const float *sre, *sim;     // [n_coils][n] receive sensitivities
};

constexpr int kWave = 64;
constexpr int kWG = 256;            // 4 wavefronts
constexpr int kWavesPerWG = kWG / kWave;
constexpr int kBatch = 16;          // samples reduced together by the register transpose
constexpr int kStretchMax = 128;
// stretches whose sums one FP32 matrix-core workgroup keeps in registers:
// 6, or 4 where the larger batches would leave the last round of
// workgroups short (the planner chooses; the kernel is built for both)
constexpr int kMMStretches = 6;
constexpr int kMMStretchesSmall = 4;
constexpr int kMMStretches64 = 4;   // the same in FP64
#ifndef KOMA_MM_RESIDENT
#define KOMA_MM_RESIDENT 3
#endif
constexpr int kMMResident = KOMA_MM_RESIDENT;  // FP32 matrix-core workgroups resident per CU (registers; LDS 32 KB each)
constexpr int kMMResident64 = 2;    // the same in FP64 (LDS 64 KB each)

// A segment of the event program for the several-lanes-per-spin kernel:
// map events (EV_RF, EV_END) [e0, e1), then, if obs, the observation event
// at e1 (EV_SNAP or EV_ADC), which needs the state itself. At most
// kSegPerLane * lanes map events per segment.
struct alignas(16) SegEv {
    int32_t e0, e1, obs, pad;
};
constexpr int kSegPerLane = 8;
constexpr int64_t kSeqgWaves = 2048;  // several lanes per spin while tiles x lanes stays within this

struct SeqArgs {  // spin-sequential kernel
    PhantomDev ph;
    const Tile *tiles;
    int64_t n_tiles;
    const Event *ev;
    int64_t e0, e1;
    double inv_gamma;
    int init;         // start from thermal equilibrium instead of the stored state
    int store;        // store the state at the end
    void *mxy;        // state: [n_tiles*64] complex (R2)
    void *mz;         // [n_tiles*64] R
    void *snap;       // [n_slots][n_tiles*64] complex (R2)
    void *pa;         // inline partials [n_sig][n_rows][n_inline] complex (R2)
    int64_t n_rows;
    int64_t n_inline;
    int32_t *vbits;   // nullptr, or a word (zero at the launch) that receives the OR of the
                      // validation bits (as k_validate) of every spin's phantom values
    // several lanes per spin (k_seqg): lanes > 1 splits each segment's map
    // events over `lanes` lanes of a spin; segments [s0, s1) cover [e0, e1)
    int lanes;
    int half_tiles;  // 1: FP64 at 16 lanes, half a tile per workgroup, inline rows 2 tile + half
    const SegEv *segs;
    int64_t s0, s1;
};


struct ParArgs {  // sample-parallel kernel
    PhantomDev ph;
    const Tile *tiles;
    int64_t n_tiles;
    const Block *blocks;
    int64_t n_blocks;
    const Stretch *st;
    int64_t s0, s1;        // stretches of this launch
    int64_t per_wg;        // stretches per workgroup (grid.y = ceil((s1-s0)/per_wg))
    const void *snap;
    double *pb;            // [n_sig][n_blocks][cols] double2 (grid.z = coil)
    int64_t col0, cols;    // deferred sample index of column 0, columns
    int engine;            // mixed precision: 0 matrix cores (k_par_mm), 1 vector ALU (k_par)
    int spl;               // tiles per wavefront (set by the launcher)
};

struct ReduceArgs {  // cross-workgroup sums into the signal (grid.z = coil)
    int64_t n_sig;         // signal planes (coils, or 1)
    int64_t part_stride;   // complex elements between the partial planes of two coils
    const void *part;      // [n_sig][n_rows][cols] complex
    int64_t cols;
    const int32_t *row_off;  // group g owns rows [row_off[g], row_off[g+1])
    int64_t n_groups;
    const int32_t *col_to_adc;  // column c -> ADC index
    double *sig;           // [n_sig][n_groups][n_adc] double2
    const int32_t *gate;   // nullptr, or a flag: the sums are written only if *gate == 0
    int64_t n_adc;
};

}  // namespace koma

// Launchers (komahip_kernels.hip). All asynchronous on `stream`.
namespace koma {
int launch_seq(bool fp64, bool moving, const SeqArgs &a, void *stream);
int launch_par(bool fp64, int spins_per_lane, const ParArgs &a, void *stream);
int launch_reduce(bool part_fp64, const ReduceArgs &a, void *stream);
int launch_upload(const void *src, void *dst, size_t bytes, int32_t *zero, void *stream);  // *zero = 0 first (if set)
int launch_validate(const PhantomDev &ph, int64_t n, int32_t *flags, void *stream);
int launch_export(bool fp64, const Tile *tiles, int64_t n_tiles, const void *mxy, const void *mz,
                  double *m_final, const int32_t *gate, void *stream);
}  // namespace koma
