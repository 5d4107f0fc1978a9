// HIP kernels for gfx950 (CDNA4, wave64) of the Bloch-simulation hot path.
//
// Arithmetic of one spin follows the paper's first-order splitting
// (section "Physical and Mathematical Background"):
//   excitation interval: spinor rotation of Eq. Rot_exc with
//     alpha = cos(phi/2) - i n_z sin(phi/2), beta = -i n_xy sin(phi/2),
//     n = B/|B|, phi = -gamma |B| dt (Eq. angle_precession), B from Eq. B-def,
//     then the relaxation update;
//   precession block: Mxy * exp(i phi) with the integral phase of the block
//     (section "Simulation blocks, Regime Switching, and Sequence-Aware Time
//     Stepping"), then relaxation over the elapsed block time;
//   ADC: sum of Mxy over the spins of a group (Figure 3).
//
// Kernels:
//   k_seq   spin-sequential: one lane per spin, every wavefront walks the
//           shared event program (uniform branches; the program is staged
//           through LDS in chunks). Excitation intervals, block ends, short
//           sample runs (summed per wavefront), snapshots of block-start
//           states.
//   k_par_mm sample-parallel, mixed precision, on the matrix cores: a
//           workgroup owns up to 4*S tiles of one group and a few stretches
//           of evenly spaced samples; per spin one exact anchor phasor (FP64
//           phase) and the per-sample factor give the two factors of
//           S[16 q + r] = sum_s (c w^(16 q)) (w^r), which FP32 MFMA
//           instructions contract over the spins. The four wavefronts are
//           added in FP64 through LDS.
//   k_par   the same sums on the vector ALU (the FP64 form, and the mixed
//           form on request): each lane walks S spins, rotates by the
//           per-sample increment (complex recurrence), and 16 samples at a
//           time are summed over the 64 lanes by a register transpose
//           (permlane32/16 swaps, DPP row rotations and quad permutes).
//   k_reduce fixed-order FP64 sum of per-wavefront / per-workgroup partials.
//   k_export state to the caller's (Mx, My, Mz) layout.
//
// No atomics in any sum: every sum has a fixed order, so results are bitwise
// reproducible for a fixed launch configuration. (The one atomic is the OR of
// a device-resident phantom's validation bits into a status word.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "komahip_internal.h"

namespace koma {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr float kLog2e = 1.44269504088896340736f;

// ---------------------------------------------------------------- precision

// FP32 for rotations and relaxation; FP64 only where a phase accumulates.
struct Mixed {
    using R = float;
    using R2 = float2;
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    // sin/cos of 2*pi*h for h in turns (hardware sine/cosine take turns)
    static __device__ __forceinline__ void sincos_turns(float h, float &s, float &c) {
        float r = __builtin_amdgcn_fractf(h);
        s = __builtin_amdgcn_sinf(r);
        c = __builtin_amdgcn_cosf(r);
    }
    // same for a phase held in FP64: the FP64 reduction to [0, 1) is exact
    static __device__ __forceinline__ void sincos_turns(double h, float &s, float &c) {
        float r = (float)__builtin_amdgcn_fract(h);
        s = __builtin_amdgcn_sinf(r);
        c = __builtin_amdgcn_cosf(r);
    }
    static __device__ __forceinline__ float exp_neg(float x) {  // exp(-x)
        return __builtin_amdgcn_exp2f(-x * kLog2e);
    }
    // 1 - exp(-x), accurate to a few ulp also for tiny x (dt / T ~ 1e-6)
    static __device__ __forceinline__ float one_minus_exp_neg(float x) { return -expm1f(-x); }
};

struct FP64 {
    using R = double;
    using R2 = double2;
    static __device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
    static __device__ __forceinline__ void sincos_turns(double h, double &s, double &c) {
        double r = h - rint(h);
        sincospi(2.0 * r, &s, &c);
    }
    static __device__ __forceinline__ double exp_neg(double x) { return exp(-x); }
    static __device__ __forceinline__ double one_minus_exp_neg(double x) { return -expm1(-x); }
};

template <class R>
struct C2 {
    R re, im;
};

template <class R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Unit phasor (c, s) renormalised by one Newton step towards |.| = 1, so
// repeated products of hardware sines/cosines do not drift in magnitude. In
// FP32 the defect c^2 + s^2 - 1 is formed to within a few ulp of itself with
// FP32 operations only: with a = max(|c|, |s|) (a^2 >= 1/2) and b the other,
// a^2 = p + e exactly (e by an fma), p - 1 is exact (Sterbenz), and
// fma(b, b, p - 1) rounds a value of the size of the defect once. The
// correction is applied as c + c h (one fma): a factor 1 + h rounded to FP32
// near 1.0 would be quantised unevenly and bias every step.
__device__ __forceinline__ void renorm(float &c, float &s) {
    const float a = fmaxf(fabsf(c), fabsf(s)), b = fminf(fabsf(c), fabsf(s));
    const float p = a * a;
    const float e = fmaf(a, a, -p);
    const float d = fmaf(b, b, p - 1.0f) + e;
    const float h = -0.5f * d;
    c = fmaf(c, h, c);
    s = fmaf(s, h, s);
}
__device__ __forceinline__ void renorm(double &c, double &s) {
    const double h = -0.5 * fma(c, c, fma(s, s, -1.0));
    c = fma(c, h, c);
    s = fma(s, h, s);
}

// ---------------------------------------------------------------- spin data

template <class R>
struct SpinP {
    R x, y, z, pd, r1, r2, bz0;  // bz0 = dw / gamma (T)
    double xd, yd, zd, f;        // FP64 copies for block phases, f = dw / 2 pi (Hz)
    R vx, vy, vz;                // velocity (moving spins; 0 otherwise)
    double vxd, vyd, vzd;
};

template <class R, bool MOV>
__device__ __forceinline__ SpinP<R> load_spin(const PhantomDev &ph, const Tile &t, int lane,
                                              double inv_gamma) {
    SpinP<R> s;
    float x = 0.f, y = 0.f, z = 0.f, pd = 0.f, t1 = __builtin_inff(), t2 = __builtin_inff(), dw = 0.f;
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (lane < t.count) {
        const int64_t i = t.spin0 + lane;
        x = ph.x[i];
        y = ph.y[i];
        z = ph.z[i];
        pd = ph.pd[i];
        t1 = ph.t1[i];
        t2 = ph.t2[i];
        dw = ph.dw[i];
        if (MOV) {
            vx = ph.vx[i];
            vy = ph.vy[i];
            vz = ph.vz[i];
        }
    }
    s.vx = vx;
    s.vy = vy;
    s.vz = vz;
    s.vxd = vx;
    s.vyd = vy;
    s.vzd = vz;
    s.x = x;
    s.y = y;
    s.z = z;
    s.pd = pd;
    s.r1 = R(1) / R(t1);  // T = +inf gives exactly 0: no relaxation
    s.r2 = R(1) / R(t2);
    s.bz0 = R((double)dw * inv_gamma);
    s.xd = x;
    s.yd = y;
    s.zd = z;
    s.f = (double)dw * kInv2Pi;
    return s;
}

// ---------------------------------------------------------------- wave sums

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

constexpr int DPP_ROR8 = 0x128;
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_QUAD_1032 = 0xB1;  // quad_perm [1,0,3,2]: lane ^ 1
constexpr int DPP_QUAD_2301 = 0x4E;  // quad_perm [2,3,0,1]: lane ^ 2
constexpr int DPP_QUAD_3210 = 0x1B;  // quad_perm [3,2,1,0]: lane ^ 3

// The value of lane ^ D (D = 1, 2, 4 or 8) by data-parallel moves within
// rows of 16 lanes: ^4 is the half-row mirror (lane ^ 7) then ^3 within quads;
// ^8 is a rotation of the row by 8.
template <int D, class R>
__device__ __forceinline__ R lane_xor(R v) {
    static_assert(D == 1 || D == 2 || D == 4 || D == 8, "xor distance");
    if constexpr (D == 1) return dpp<DPP_QUAD_1032>(v);
    else if constexpr (D == 2) return dpp<DPP_QUAD_2301>(v);
    else if constexpr (D == 4) return dpp<DPP_QUAD_3210>(dpp<DPP_HALF_MIRROR>(v));
    else return dpp<DPP_ROR8>(v);
}

// After the call: a = [a lanes 0-31, b lanes 0-31], b = [a lanes 32-63, b lanes 32-63].
__device__ __forceinline__ void swap32(float &a, float &b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
// Within each half wave: a = [a 0-15, b 0-15], b = [a 16-31, b 16-31] (and the same for 32-63).
__device__ __forceinline__ void swap16(float &a, float &b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void split(double v, uint32_t &lo, uint32_t &hi) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    lo = (uint32_t)u;
    hi = (uint32_t)(u >> 32);
}
__device__ __forceinline__ double join(uint32_t lo, uint32_t hi) {
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ void swap32(double &a, double &b) {
    uint32_t al, ah, bl, bh;
    split(a, al, ah);
    split(b, bl, bh);
    auto lo = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    a = join(lo[0], hi[0]);
    b = join(lo[1], hi[1]);
}
__device__ __forceinline__ void swap16(double &a, double &b) {
    uint32_t al, ah, bl, bh;
    split(a, al, ah);
    split(b, bl, bh);
    auto lo = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
    a = join(lo[0], hi[0]);
    b = join(lo[1], hi[1]);
}

// Sum over the 64 lanes; every lane receives the total. Fixed pairing order.
template <class R>
__device__ __forceinline__ R wave_allsum(R v) {
    R a = v, b = v;
    swap32(a, b);  // a + b = v[l] + v[l ^ 32]
    v = a + b;
    a = v;
    b = v;
    swap16(a, b);  // + v[l ^ 16]
    v = a + b;
    v = v + dpp<DPP_ROR8>(v);         // + lane l ^ 8 within the row
    v = v + dpp<DPP_HALF_MIRROR>(v);  // + lane 7 - l within the half row
    v = v + dpp<DPP_QUAD_1032>(v);
    v = v + dpp<DPP_QUAD_2301>(v);
    return v;
}

// Register transpose-sum of 16 samples held by every lane: on return lane l
// holds in v[0] the sum over all 64 lanes of sample (l >> 2) (the four lanes
// of a quad hold the same value).
template <class R>
__device__ __forceinline__ void transpose_sum16(R (&v)[16]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 8; ++i) {  // lanes 0-31 keep samples 0-7, lanes 32-63 samples 8-15
        swap32(v[i], v[i + 8]);
        v[i] = v[i] + v[i + 8];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // sample i + 4*bit4 + 8*bit5
        swap16(v[i], v[i + 4]);
        v[i] = v[i] + v[i + 4];
    }
    const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {  // sample i + 2*bit3 + 4*bit4 + 8*bit5
        R keep = b3 ? v[i + 2] : v[i];
        R send = b3 ? v[i] : v[i + 2];
        v[i] = keep + dpp<DPP_ROR8>(send);
    }
    {  // sample bit2 + 2*bit3 + 4*bit4 + 8*bit5 = lane >> 2
        R keep = b2 ? v[1] : v[0];
        R send = b2 ? v[0] : v[1];
        v[0] = keep + dpp<DPP_HALF_MIRROR>(send);
    }
    v[0] = v[0] + dpp<DPP_QUAD_1032>(v[0]);
    v[0] = v[0] + dpp<DPP_QUAD_2301>(v[0]);
}

// ---------------------------------------------------------------- the steps

// Block phase (turns) at moment K (cycles/m) and elapsed tau: -(x.K + f tau).
template <class R>
__device__ __forceinline__ double block_phase(const SpinP<R> &s, const double *k) {
    return -fma(s.xd, k[0], fma(s.yd, k[1], fma(s.zd, k[2], s.f * k[3])));
}
// The same for a moving spin, x(t) = x + v t: -(x.K + v.K1 + f tau), with K1
// the first moment (cycles s/m) accumulated by the same trapezoidal rule.
template <class R>
__device__ __forceinline__ double block_phase(const SpinP<R> &s, const double *k, const double *k1) {
    return -fma(s.xd, k[0], fma(s.yd, k[1], fma(s.zd, k[2],
                fma(s.vxd, k1[0], fma(s.vyd, k1[1], fma(s.vzd, k1[2], s.f * k[3]))))));
}

// exp(i*2*pi*theta) * exp(-tau * r2) as a complex factor
template <class P>
__device__ __forceinline__ C2<typename P::R> block_factor(const SpinP<typename P::R> &s, double theta,
                                                          double tau) {
    using R = typename P::R;
    R sn, cs;
    P::sincos_turns(theta, sn, cs);
    renorm(cs, sn);
    R e2 = P::exp_neg(R(tau) * s.r2);
    return {cs * e2, sn * e2};
}

// One Newton step of the spinor towards |alpha|^2 + |beta|^2 = cs^2 + sk^2
// |B|^2 = 1 (sk = sin(phi/2) / |B|), which keeps the rotation orthogonal
// whatever the errors of the hardware sine, cosine and reciprocal square
// root. FP32: the defect from the FP32 |B|^2 (nb2), formed as
// fma(sk^2, nb2, fma(cs, cs, -1)): fma(cs, cs, -1) ~ -sin^2(phi/2) is rounded
// once at its own size, so the defect is good to ~3 ulp of sin^2(phi/2)
// (tiny for the small angles of an excitation interval) and its rounding is
// unbiased; FP64: from the exact |B|^2 of the interval's FP64 values.
__device__ __forceinline__ void spinor_normalise(float &cs, float &sk, float bz, float nb2, double) {
    const float d = fmaf(sk * sk, nb2, fmaf(cs, cs, -1.0f));
    const float h = -0.5f * d;
    cs = fmaf(cs, h, cs);
    sk = fmaf(sk, h, sk);
}
__device__ __forceinline__ void spinor_normalise(double &cs, double &sk, double bz, double, double b1sq) {
    const double B2 = fma(bz, bz, b1sq);
    const double h = -0.5 * fma(sk * sk, B2, fma(cs, cs, -1.0));
    cs = fma(cs, h, cs);
    sk = fma(sk, h, sk);
}

// One excitation interval (Eq. Rot_exc) followed by relaxation with the
// cached eps = 1 - exp(-dt/T) (applied as M - eps*M, exact in the factor).
// For moving spins gt holds the interval mean of G(t) t: Bz gains v . gt.
//
// The spinor of Eq. Rot_exc, alpha = cos(phi/2) - i n_z sin(phi/2), beta =
// -i n_xy sin(phi/2), rotates M about n = B/|B| by phi. Its product is
// applied in the equivalent Rodrigues form (the same matrix, fewer
// operations): M' = cos(phi) M + sin(phi)/|B| (B x M) + (1 - cos phi)/|B|^2
// B (B . M), with sin(phi)/|B| = 2 cs sk, (1 - cos phi)/|B|^2 = 2 sk^2 and
// cos(phi) = 1 - 2 sk^2 |B|^2 from the normalised half-angle spinor
// (cs = cos(phi/2), sk = sin(phi/2)/|B|), so the matrix stays orthogonal to
// rounding whatever the errors of the hardware sine and square root.
template <class P, bool MOV>
__device__ __forceinline__ void excite_relax(const SpinP<typename P::R> &s, const typename P::R *q,
                                             const typename P::R *gt, double b1sq_exact,
                                             typename P::R eps1, typename P::R eps2,
                                             typename P::R &mr, typename P::R &mi,
                                             typename P::R &mz) {
    using R = typename P::R;
    const R gx = q[0], gy = q[1], gz = q[2], b1r = q[3], b1i = q[4], b1sq = q[5], hs = q[6];
    R bz0 = s.bz0;
    if (MOV) bz0 = fma(s.vx, gt[0], fma(s.vy, gt[1], fma(s.vz, gt[2], bz0)));
    const R bz = fma(s.x, gx, fma(s.y, gy, fma(s.z, gz, bz0)));
    // |B|^2 >= |b1|^2, which the host makes at least the smallest normal
    // number: a zero field (b1 = 0, Bz = 0) gives 1/|B| finite and a zero
    // angle, the spin unrotated
    const R nb2 = fma(bz, bz, b1sq);
    const R inv = P::rsq(nb2);
    const R nb = nb2 * inv;
    R sn, cs;
    P::sincos_turns(hs * nb, sn, cs);  // sin, cos of phi/2
    R sk = sn * inv;                   // sin(phi/2) / |B|
    // normalise the spinor, |alpha|^2 + |beta|^2 = cs^2 + sk^2 |B|^2 -> 1
    spinor_normalise(cs, sk, bz, nb2, b1sq_exact);
    const R sk2x = sk + sk;
    const R sg = cs * sk2x;         // sin(phi) / |B| = 2 cs sk
    const R t = sk * sk2x;          // (1 - cos phi) / |B|^2 = 2 sk^2
    const R c = fma(-t, nb2, R(1));  // cos(phi) = 1 - 2 sk^2 |B|^2
    const R u = t * fma(b1r, mr, fma(b1i, mi, bz * mz));  // (1 - cos phi)/|B|^2 (B . M)
    // B x M
    const R xr = fma(b1i, mz, -bz * mi);
    const R xi = fma(bz, mr, -b1r * mz);
    const R xz = fma(b1r, mi, -b1i * mr);
    const R nr = fma(c, mr, fma(sg, xr, u * b1r));
    const R ni = fma(c, mi, fma(sg, xi, u * b1i));
    const R nz = fma(c, mz, fma(sg, xz, u * bz));
    // relaxation: Mxy (1 - eps2), Mz - eps1 (Mz - M0)
    mr = fma(-eps2, nr, nr);
    mi = fma(-eps2, ni, ni);
    mz = fma(-eps1, nz - s.pd, nz);
}

// The rotation of one excitation interval (Eq. Rot_exc, in the Rodrigues
// form of excite_relax) as a real 3 x 3 matrix on (Mx, My, Mz), row-major:
// cos(phi) I + sin(phi)/|B| [B]x + (1 - cos phi)/|B|^2 B B^T.
template <class P, bool MOV>
__device__ __forceinline__ void rot_matrix(const SpinP<typename P::R> &s, const typename P::R *q,
                                           const typename P::R *gt, double b1sq_exact, typename P::R *m) {
    using R = typename P::R;
    const R gx = q[0], gy = q[1], gz = q[2], b1r = q[3], b1i = q[4], b1sq = q[5], hs = q[6];
    R bz0 = s.bz0;
    if (MOV) bz0 = fma(s.vx, gt[0], fma(s.vy, gt[1], fma(s.vz, gt[2], bz0)));
    const R bz = fma(s.x, gx, fma(s.y, gy, fma(s.z, gz, bz0)));
    const R nb2 = fma(bz, bz, b1sq);  // >= the smallest normal number (see excite_relax)
    const R inv = P::rsq(nb2);
    const R nb = nb2 * inv;
    R sn, cs;
    P::sincos_turns(hs * nb, sn, cs);
    R sk = sn * inv;
    spinor_normalise(cs, sk, bz, nb2, b1sq_exact);
    const R sk2x = sk + sk;
    const R sg = cs * sk2x;
    const R t = sk * sk2x;
    const R c = fma(-t, nb2, R(1));
    const R tr = t * b1r, ti = t * b1i, tz = t * bz;
    const R sr = sg * b1r, si = sg * b1i, sz = sg * bz;
    m[0] = fma(tr, b1r, c);
    m[1] = fma(tr, b1i, -sz);
    m[2] = fma(tr, bz, si);
    m[3] = fma(ti, b1r, sz);
    m[4] = fma(ti, b1i, c);
    m[5] = fma(ti, bz, -sr);
    m[6] = fma(tz, b1r, -si);
    m[7] = fma(tz, b1i, sr);
    m[8] = fma(tz, bz, c);
}

// k identical excitation intervals (uniform k >= 1): one interval is the
// affine map M -> A M + b with A the rotation followed by the relaxation
// factors (rows scaled by 1 - eps2, 1 - eps2, 1 - eps1) and b = (0, 0,
// eps1 M0); its k-th power is applied by binary powering, the same product
// of per-interval operators associated differently (log2 k squarings instead
// of k steps). Up to kDirectSteps intervals the map is applied k times
// instead: 9 FMA per step against ~40 per squaring.
constexpr int kDirectSteps = 16;
template <class R>
__device__ __forceinline__ void affine_power(R *p, R b2, int k, R &mr, R &mi, R &mz) {
    if (k <= kDirectSteps) {  // uniform
        for (int i = 0; i < k; ++i) {
            const R nr = fma(p[0], mr, fma(p[1], mi, p[2] * mz));
            const R ni = fma(p[3], mr, fma(p[4], mi, p[5] * mz));
            const R nz = fma(p[6], mr, fma(p[7], mi, fma(p[8], mz, b2)));
            mr = nr;
            mi = ni;
            mz = nz;
        }
        return;
    }
    R q[3] = {R(0), R(0), b2};
    for (;;) {
        if (k & 1) {
            const R nr = fma(p[0], mr, fma(p[1], mi, fma(p[2], mz, q[0])));
            const R ni = fma(p[3], mr, fma(p[4], mi, fma(p[5], mz, q[1])));
            const R nz = fma(p[6], mr, fma(p[7], mi, fma(p[8], mz, q[2])));
            mr = nr;
            mi = ni;
            mz = nz;
        }
        k >>= 1;
        if (k == 0) break;
        R p2[9], q2[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) p2[3 * r + c] = fma(p[3 * r], p[c], fma(p[3 * r + 1], p[3 + c], p[3 * r + 2] * p[6 + c]));
            q2[r] = fma(p[3 * r], q[0], fma(p[3 * r + 1], q[1], fma(p[3 * r + 2], q[2], q[r])));
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) p[i] = p2[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) q[i] = q2[i];
    }
}

// Validation bits of spin i's phantom values (device-resident phantoms):
// bit 0 non-finite x, y, z, dw, PD or velocity; bit 1 PD < 0; bit 2 T1 or T2
// <= 0 or NaN; bit 3 non-finite coil sensitivity.
__device__ __forceinline__ int32_t spin_flags(const PhantomDev &ph, int64_t i) {
    int32_t bad = 0;
    const float x = ph.x[i], y = ph.y[i], z = ph.z[i], dw = ph.dw[i], pd = ph.pd[i];
    const float t1 = ph.t1[i], t2 = ph.t2[i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(dw) || !isfinite(pd)) bad |= 1;
    if (pd < 0.f) bad |= 2;
    if (!(t1 > 0.f) || !(t2 > 0.f)) bad |= 4;
    if (ph.vx && (!isfinite(ph.vx[i]) || !isfinite(ph.vy[i]) || !isfinite(ph.vz[i]))) bad |= 1;
    for (int64_t k = 0; k < ph.n_coils; ++k)
        if (!isfinite(ph.sre[k * ph.n + i]) || !isfinite(ph.sim[k * ph.n + i])) bad |= 8;
    return bad;
}

// ---------------------------------------------------------------- k_seq

// The event program and stretch tables are read-only for a whole launch and
// read at the same address by every lane: reading them through the constant
// address space lets the compiler use scalar loads (scalar cache, SGPRs)
// instead of one vector load per lane.
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ ConstPtr<T> as_const(const T *p) {
    return (ConstPtr<T>)p;
}

// Events are staged through LDS in chunks: the workgroup copies kChunk
// events with coalesced 16-byte loads (one round trip to memory for the
// chunk, however few wavefronts share a SIMD), and every lane then reads the
// fields of the current event at one LDS address (a broadcast).
constexpr int kChunk = 64;
constexpr int kEvWords = (int)(sizeof(Event) / 4);  // 64 dwords
static_assert(sizeof(Event) % 16 == 0, "Event is copied as 16-byte words");

struct EvL {  // view of one staged event
    const uint32_t *u;
    __device__ __forceinline__ uint32_t word(int i) const { return u[i]; }
    // a word every lane of the wavefront reads at the same address, as a
    // scalar (so that branches and compares on it are scalar)
    __device__ __forceinline__ uint32_t uword(int i) const { return __builtin_amdgcn_readfirstlane(u[i]); }
    __device__ __forceinline__ int kind() const { return (int)u[0]; }
    __device__ __forceinline__ int a0() const { return (int)u[1]; }
    __device__ __forceinline__ int count() const { return (int)u[2]; }
    __device__ __forceinline__ int rot() const { return (int)u[3]; }
    __device__ __forceinline__ float f(int i) const { return __uint_as_float(u[4 + i]); }
    __device__ __forceinline__ double d(int i) const {
        return __builtin_bit_cast(double, ((uint64_t)u[12 + 2 * i + 1] << 32) | u[12 + 2 * i]);
    }
    __device__ __forceinline__ double b1sq() const {
        return __builtin_bit_cast(double, ((uint64_t)u[29] << 32) | u[28]);
    }
    __device__ __forceinline__ double dt_ref() const {
        return __builtin_bit_cast(double, ((uint64_t)u[31] << 32) | u[30]);
    }
    __device__ __forceinline__ float c32(int i) const { return __uint_as_float(u[32 + i]); }
    __device__ __forceinline__ double c64(int i) const {
        return __builtin_bit_cast(double, ((uint64_t)u[44 + 2 * i + 1] << 32) | u[44 + 2 * i]);
    }
};

// The wavefront's sum of v into inline partial row `row` of signal plane k;
// a tile holding two groups sums lanes [0, split) into its first row and
// the others into the next one.
template <class R, class R2>
__device__ __forceinline__ void inline_rows(const SeqArgs &a, const Tile &T, int lane, int64_t k, int col,
                                            C2<R> v) {
    R2 *pa = reinterpret_cast<R2 *>(a.pa);
    if (T.split >= T.count) {  // uniform: one group
        const R sr = wave_allsum(v.re);
        const R si = wave_allsum(v.im);
        if (lane == 0) pa[(k * a.n_rows + T.seg) * a.n_inline + col] = R2{sr, si};
        return;
    }
    const bool lo = lane < T.split;
    const R ar = wave_allsum(lo ? v.re : R(0)), ai = wave_allsum(lo ? v.im : R(0));
    const R br = wave_allsum(lo ? R(0) : v.re), bi = wave_allsum(lo ? R(0) : v.im);
    if (lane == 0) {
        pa[(k * a.n_rows + T.seg) * a.n_inline + col] = R2{ar, ai};
        pa[(k * a.n_rows + T.seg + 1) * a.n_inline + col] = R2{br, bi};
    }
}

// One inline ADC sample: the wavefront's sum of Mxy (c), or of sens_k * Mxy
// for every receive coil k, into the per-wavefront partials.
template <class R, class R2>
__device__ __forceinline__ void inline_sample(const SeqArgs &a, const Tile &T, int lane, int col, C2<R> c) {
    const int64_t n_coils = a.ph.n_coils;  // uniform
    if (n_coils == 0) {
        inline_rows<R, R2>(a, T, lane, 0, col, c);
        return;
    }
    const bool valid = lane < T.count;
    const int64_t i = T.spin0 + lane;
    for (int64_t k = 0; k < n_coils; ++k) {
        C2<R> sk{R(0), R(0)};
        if (valid) sk = C2<R>{R(a.ph.sre[k * a.ph.n + i]), R(a.ph.sim[k * a.ph.n + i])};
        inline_rows<R, R2>(a, T, lane, k, col, cmul(sk, c));
    }
}

// Relaxation factors eps = 1 - exp(-dt/T) of an excitation event from the
// factors cached for a key length (eps1c, eps2c). Mixed form: the key is the
// FP32 length itself, so the cached factors are the event's. FP64 form: the
// key is the event's reference length (Event::dt_ref, within 2^-30 of dt),
// and the factors are moved to the event's own length h = dt - dt_ref away:
// 1 - e^-(t + h) r = eps(t) + (1 - eps(t)) h r, exact to within
// (1 - eps) (h r)^2 / 2, far below an ulp of eps.
template <class P, class Ev>
__device__ __forceinline__ void event_eps(const Ev &ev, const SpinP<typename P::R> &s, typename P::R eps1c,
                                          typename P::R eps2c, typename P::R &eps1, typename P::R &eps2) {
    using R = typename P::R;
    if constexpr (sizeof(R) == 4) {
        eps1 = eps1c;
        eps2 = eps2c;
    } else {
        const double h = ev.d(7) - ev.dt_ref();  // exact: the two are within 2^-30 of each other
        eps1 = fma(h * s.r1, 1.0 - eps1c, eps1c);
        eps2 = fma(h * s.r2, 1.0 - eps2c, eps2c);
    }
}

template <class P, bool MOV>
__global__ __launch_bounds__(kWG) void k_seq(SeqArgs a) {
    using R = typename P::R;
    using R2 = typename P::R2;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerWG + wave;
    __shared__ uint4 lds_ev[kChunk * kEvWords / 4];
    // wavefronts past the last tile still help staging and reach every barrier
    const bool active = tile < a.n_tiles;
    Tile T;
    if (active) {
        T = a.tiles[tile];
    } else {
        T.spin0 = 0;
        T.count = 0;
        T.group = 0;
        T.split = 0;
        T.seg = 0;
    }
    const SpinP<R> s = load_spin<R, MOV>(a.ph, T, lane, a.inv_gamma);
    const int64_t n_pad = a.n_tiles * kWave;
    const int64_t pidx = tile * kWave + lane;
    // validate the phantom values of this lane's spin: its bits (as
    // k_validate) are ORed into one word, zeroed by the upload before this
    // launch; only lanes with an invalid spin touch it
    if (a.vbits && lane < T.count) {
        const int32_t bad = spin_flags(a.ph, T.spin0 + lane);
        if (bad) atomicOr(a.vbits, bad);
    }

    R mr = R(0), mi = R(0), mz = s.pd;
    if (active && !a.init) {
        R2 m = reinterpret_cast<const R2 *>(a.mxy)[pidx];
        mr = m.x;
        mi = m.y;
        mz = reinterpret_cast<const R *>(a.mz)[pidx];
    }
    R eps1c = R(0), eps2c = R(0);
    // bits of the key length the cached relaxation factors were formed for:
    // the FP32 length (the FP64 one rounded) in the mixed form, so that
    // lengths which differ only below FP32 resolution (the rounding of
    // time-point differences) reuse the factors; the event's reference length
    // in the FP64 form (see event_eps); uniform
    uint32_t dt_lo = ~0u, dt_hi = ~0u;
    // no spin of this wavefront has off-resonance: zero-gradient excitation
    // intervals are then the same rotation for all of them (precomputed)
    const bool no_offres = __ballot(s.bz0 != R(0)) == 0;
    const uint4 *gev = reinterpret_cast<const uint4 *>(a.ev);
    const uint32_t *base = reinterpret_cast<const uint32_t *>(lds_ev);
    constexpr bool f32 = sizeof(R) == 4;

    for (int64_t c0 = a.e0; c0 < a.e1; c0 += kChunk) {
        const int n = (int)min<int64_t>(kChunk, a.e1 - c0);
        __syncthreads();  // the previous chunk is no longer read
        for (int i = threadIdx.x; i < n * (kEvWords / 4); i += kWG) lds_ev[i] = gev[c0 * (kEvWords / 4) + i];
        __syncthreads();
        if (!active) continue;
        for (int e = 0; e < n; ++e) {
            const EvL ev{base + e * kEvWords};
            const int kind = (int)ev.uword(0);
            if (kind == EV_RF) {
                const uint32_t lo = ev.uword(f32 ? 11 : 30), hi = f32 ? 0u : ev.uword(31);
                if (lo != dt_lo || hi != dt_hi) {  // uniform: same key length for every spin
                    dt_lo = lo;
                    dt_hi = hi;
                    const R dt = f32 ? R(ev.f(7)) : R(ev.dt_ref());  // (the FP32 length is the FP64 one rounded)
                    eps1c = P::one_minus_exp_neg(dt * s.r1);
                    eps2c = P::one_minus_exp_neg(dt * s.r2);
                }
                R eps1, eps2;
                event_eps<P>(ev, s, eps1c, eps2c, eps1, eps2);
                const int reps = (int)ev.uword(2);  // identical consecutive intervals (uniform)
                const int rot = (int)ev.uword(3);
                if (reps > 1) {
                    R m[9];
                    if (rot >= 0 && no_offres) {
                        // the host's coefficients: Mxy_re' = c0 Mz + c1 Mxy_re + c2 Mxy_im, ...
                        const int perm[9] = {1, 2, 0, 5, 4, 3, 7, 8, 6};
#pragma unroll
                        for (int i = 0; i < 9; ++i) m[i] = sizeof(R) == 4 ? R(ev.c32(perm[i])) : R(ev.c64(perm[i]));
                    } else {
                        R q[7];
#pragma unroll
                        for (int i = 0; i < 7; ++i) q[i] = sizeof(R) == 4 ? R(ev.f(i)) : R(ev.d(i));
                        R gt[3] = {R(0), R(0), R(0)};
                        if (MOV && rot < 0) {
#pragma unroll
                            for (int i = 0; i < 3; ++i) gt[i] = sizeof(R) == 4 ? R(ev.c32(i)) : R(ev.c64(i));
                        }
                        const double b1sq = sizeof(R) == 4 ? ev.b1sq() : ev.d(5);
                        rot_matrix<P, MOV>(s, q, gt, b1sq, m);
                    }
                    // the interval's affine map: rotation rows scaled by the
                    // relaxation factors (m - eps m, never a rounded 1 - eps)
#pragma unroll
                    for (int i = 0; i < 6; ++i) m[i] = fma(-eps2, m[i], m[i]);
#pragma unroll
                    for (int i = 6; i < 9; ++i) m[i] = fma(-eps1, m[i], m[i]);
                    affine_power(m, eps1 * s.pd, reps, mr, mi, mz);
                } else if (rot >= 0 && no_offres) {
                    R c[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) c[i] = sizeof(R) == 4 ? R(ev.c32(i)) : R(ev.c64(i));
                    const R nr = fma(c[0], mz, fma(c[1], mr, c[2] * mi));
                    const R ni = fma(c[3], mz, fma(c[4], mi, c[5] * mr));
                    const R nz = fma(c[6], mz, fma(c[7], mr, c[8] * mi));
                    mr = fma(-eps2, nr, nr);
                    mi = fma(-eps2, ni, ni);
                    mz = fma(-eps1, nz - s.pd, nz);
                } else {
                    // A run of single intervals with the same key length (the
                    // intervals of a shaped pulse) goes round a loop of its own,
                    // whose state stays in its registers from one interval to
                    // the next; the event that ends the run is taken up again
                    // by the outer loop.
                    // The run of single intervals that starts here (its length
                    // from the host: the same relaxation keys throughout; cut at
                    // the end of the chunk) goes round a loop of its own, which
                    // keeps the state in its registers and reads each next
                    // interval's values from LDS during the current one's
                    // arithmetic.
                    const int run = min((int)ev.uword(1), n - e);
                    // two sets of interval values in turn (no copies between
                    // passes): the values of interval j + 1 are read into one
                    // while interval j's arithmetic uses the other
                    struct Iv {
                        R q[7], gt[3];
                        double b1sq;
                        R eps1, eps2;
                    };
                    auto read_iv = [&](const EvL &v, Iv &iv, bool first) {
#pragma unroll
                        for (int i = 0; i < 7; ++i) iv.q[i] = f32 ? R(v.f(i)) : R(v.d(i));
#pragma unroll
                        for (int i = 0; i < 3; ++i) iv.gt[i] = R(0);
                        // (rot >= 0: G and G t are zero on the interval; the
                        // run's later intervals have rot < 0)
                        if (MOV && (!first || rot < 0)) {
#pragma unroll
                            for (int i = 0; i < 3; ++i) iv.gt[i] = f32 ? R(v.c32(i)) : R(v.c64(i));
                        }
                        // |b1|^2 of exactly the b1 values the precision uses
                        iv.b1sq = f32 ? v.b1sq() : v.d(5);
                        event_eps<P>(v, s, eps1c, eps2c, iv.eps1, iv.eps2);
                    };
                    auto step = [&](const Iv &iv) {
                        excite_relax<P, MOV>(s, iv.q, iv.gt, iv.b1sq, iv.eps1, iv.eps2, mr, mi, mz);
                    };
                    Iv ia, ib;
                    // the scheduler is told to issue the LDS reads of the
                    // next interval first, then the arithmetic of this one
                    // (left alone it moves each read next to its first use)
                    auto reads_first = [] {
                        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);  // LDS reads
                        __builtin_amdgcn_sched_group_barrier(0x002, 200, 0);  // vector ALU
                    };
                    read_iv(ev, ia, true);
                    for (int j = 1;; j += 2) {
                        read_iv(EvL{base + (e + min(j, run - 1)) * kEvWords}, ib, false);
                        step(ia);
                        reads_first();
                        if (j >= run) break;
                        read_iv(EvL{base + (e + min(j + 1, run - 1)) * kEvWords}, ia, false);
                        step(ib);
                        reads_first();
                        if (j + 1 >= run) break;
                    }
                    e += run - 1;
                }
            } else if (kind == EV_END) {
                const double k4[4] = {ev.d(0), ev.d(1), ev.d(2), ev.d(3)};
                const double tau = k4[3];
                double th;
                if (MOV) {
                    const double k1[3] = {ev.d(4), ev.d(5), ev.d(6)};
                    th = block_phase(s, k4, k1);
                } else {
                    th = block_phase(s, k4);
                }
                C2<R> f = block_factor<P>(s, th, tau);
                C2<R> m = cmul(C2<R>{mr, mi}, f);
                mr = m.re;
                mi = m.im;
                mz = s.pd + (mz - s.pd) * P::exp_neg(R(tau) * s.r1);
            } else if (MOV && kind == EV_ADC) {  // one sample, first moments in c64
                const double k0[4] = {ev.d(0), ev.d(1), ev.d(2), ev.d(3)};
                const double k1[3] = {ev.c64(0), ev.c64(1), ev.c64(2)};
                const C2<R> c = cmul(C2<R>{mr, mi}, block_factor<P>(s, block_phase(s, k0, k1), k0[3]));
                inline_sample<R, R2>(a, T, lane, ev.a0(), c);
            } else if (kind == EV_ADC) {
                const double k0[4] = {ev.d(0), ev.d(1), ev.d(2), ev.d(3)};
                const double dk[4] = {ev.d(4), ev.d(5), ev.d(6), ev.d(7)};
                C2<R> c = cmul(C2<R>{mr, mi}, block_factor<P>(s, block_phase(s, k0), k0[3]));
                const int cnt = (int)ev.uword(2);
                C2<R> w{R(1), R(0)};
                if (cnt > 1) w = block_factor<P>(s, block_phase(s, dk), dk[3]);
                for (int i = 0; i < cnt; ++i) {
                    inline_sample<R, R2>(a, T, lane, ev.a0() + i, c);
                    c = cmul(c, w);
                }
            } else {  // EV_SNAP
                reinterpret_cast<R2 *>(a.snap)[(int64_t)ev.a0() * n_pad + pidx] = R2{mr, mi};
            }
        }
    }
    if (active && a.store) {
        reinterpret_cast<R2 *>(a.mxy)[pidx] = R2{mr, mi};
        reinterpret_cast<R *>(a.mz)[pidx] = mz;
    }
}

// ---------------------------------------------------------------- k_seqg

// Several lanes per spin. With few spins, one lane per spin leaves most of
// the chip idle and every wavefront walks the whole event program as one
// dependent chain. Every event between two observations of the state (a
// snapshot or an inline sample) is an affine map of (Mx, My, Mz): an
// excitation interval is its rotation (Eq. Rot_exc) followed by the
// relaxation update, a run of k identical ones the k-th power of that map,
// a precession-block end the rotation by the block phase with the decay
// over the block. The G lanes of a spin each compose the maps of a
// contiguous share of a segment's events; the G products are combined by a
// tree over the lanes (the later product after the earlier one), which
// leaves the segment's composite on the spin's first lane, and that lane
// applies it to the state it carries. The same operators as the one-lane
// kernel, associated differently.
template <class R>
struct Aff {
    R a[9];  // row-major, on (Mx, My, Mz)
    R b[3];
};

template <class R>
__device__ __forceinline__ Aff<R> aff_identity() {
    Aff<R> m;
#pragma unroll
    for (int i = 0; i < 9; ++i) m.a[i] = (i % 4 == 0) ? R(1) : R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) m.b[i] = R(0);
    return m;
}

// the map of `second` after `first`
template <class R>
__device__ __forceinline__ Aff<R> aff_then(const Aff<R> &second, const Aff<R> &first) {
    Aff<R> c;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const R x = second.a[3 * r], y = second.a[3 * r + 1], z = second.a[3 * r + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k) c.a[3 * r + k] = fma(x, first.a[k], fma(y, first.a[3 + k], z * first.a[6 + k]));
        c.b[r] = fma(x, first.b[0], fma(y, first.b[1], fma(z, first.b[2], second.b[r])));
    }
    return c;
}

template <class R>
__device__ __forceinline__ void aff_apply(const Aff<R> &m, R &mr, R &mi, R &mz) {
    const R nr = fma(m.a[0], mr, fma(m.a[1], mi, fma(m.a[2], mz, m.b[0])));
    const R ni = fma(m.a[3], mr, fma(m.a[4], mi, fma(m.a[5], mz, m.b[1])));
    const R nz = fma(m.a[6], mr, fma(m.a[7], mi, fma(m.a[8], mz, m.b[2])));
    mr = nr;
    mi = ni;
    mz = nz;
}

// k-th power (k >= 1) by binary powering (powers of one map commute)
template <class R>
__device__ __forceinline__ Aff<R> aff_power(Aff<R> p, int k) {
    Aff<R> r = p;
    bool have = false;
    for (;;) {
        if (k & 1) {
            r = have ? aff_then(p, r) : p;
            have = true;
        }
        k >>= 1;
        if (k == 0) break;
        p = aff_then(p, p);
    }
    return r;
}

template <int D, class R>
__device__ __forceinline__ Aff<R> aff_lane_xor(const Aff<R> &m) {
    Aff<R> o;
#pragma unroll
    for (int i = 0; i < 9; ++i) o.a[i] = lane_xor<D>(m.a[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) o.b[i] = lane_xor<D>(m.b[i]);
    return o;
}

// The map of one EV_RF or EV_END event for spin s. eps1c/eps2c and dt_cached
// are the lane's relaxation cache (1 - exp(-dt/T) for the last key length
// seen, see event_eps).
template <class P, bool MOV>
__device__ __forceinline__ Aff<typename P::R> event_map(const EvL &ev, const SpinP<typename P::R> &s,
                                                        bool no_offres, double &dt_cached,
                                                        typename P::R &eps1c, typename P::R &eps2c) {
    using R = typename P::R;
    Aff<R> m;
    if (ev.kind() == EV_END) {
        const double k4[4] = {ev.d(0), ev.d(1), ev.d(2), ev.d(3)};
        double th;
        if (MOV) {
            const double k1[3] = {ev.d(4), ev.d(5), ev.d(6)};
            th = block_phase(s, k4, k1);
        } else {
            th = block_phase(s, k4);
        }
        const C2<R> f = block_factor<P>(s, th, k4[3]);
        const R e1 = P::exp_neg(R(k4[3]) * s.r1);
        m.a[0] = f.re;
        m.a[1] = -f.im;
        m.a[2] = R(0);
        m.a[3] = f.im;
        m.a[4] = f.re;
        m.a[5] = R(0);
        m.a[6] = R(0);
        m.a[7] = R(0);
        m.a[8] = e1;
        m.b[0] = R(0);
        m.b[1] = R(0);
        m.b[2] = fma(-e1, s.pd, s.pd);
        return m;
    }
    // the cache key: the FP32 length (the FP64 one rounded) in the mixed
    // form, the reference length in the FP64 form (see event_eps)
    const double key = sizeof(R) == 4 ? (double)ev.f(7) : ev.dt_ref();
    if (key != dt_cached) {
        dt_cached = key;
        eps1c = P::one_minus_exp_neg(R(key) * s.r1);
        eps2c = P::one_minus_exp_neg(R(key) * s.r2);
    }
    R eps1, eps2;
    event_eps<P>(ev, s, eps1c, eps2c, eps1, eps2);
    if (ev.rot() >= 0 && no_offres) {
        // the host's coefficients: Mxy_re' = c0 Mz + c1 Mxy_re + c2 Mxy_im, ...
        const int perm[9] = {1, 2, 0, 5, 4, 3, 7, 8, 6};
#pragma unroll
        for (int i = 0; i < 9; ++i) m.a[i] = sizeof(R) == 4 ? R(ev.c32(perm[i])) : R(ev.c64(perm[i]));
    } else {
        R q[7];
#pragma unroll
        for (int i = 0; i < 7; ++i) q[i] = sizeof(R) == 4 ? R(ev.f(i)) : R(ev.d(i));
        R gt[3] = {R(0), R(0), R(0)};
        if (MOV && ev.rot() < 0) {
#pragma unroll
            for (int i = 0; i < 3; ++i) gt[i] = sizeof(R) == 4 ? R(ev.c32(i)) : R(ev.c64(i));
        }
        const double b1sq = sizeof(R) == 4 ? ev.b1sq() : ev.d(5);
        rot_matrix<P, MOV>(s, q, gt, b1sq, m.a);
    }
    // relaxation after the rotation: rows scaled by 1 - eps (as m - eps m)
#pragma unroll
    for (int i = 0; i < 6; ++i) m.a[i] = fma(-eps2, m.a[i], m.a[i]);
#pragma unroll
    for (int i = 6; i < 9; ++i) m.a[i] = fma(-eps1, m.a[i], m.a[i]);
    m.b[0] = R(0);
    m.b[1] = R(0);
    m.b[2] = eps1 * s.pd;
    const int reps = ev.count();
    return reps > 1 ? aff_power(m, reps) : m;
}

// Staged events: kSegStride dwords apart (odd, so that lanes reading
// different events of one segment hit different LDS banks).
constexpr int kSegStride = kEvWords + 1;

// SP spins of a tile (all 64, or one half: the FP64 form at 16 lanes, whose
// registers allow 512-lane workgroups) per workgroup of SP G lanes: lane t
// holds spin t / G of the workgroup's spins, share t % G of every segment.
// Segments are staged through LDS, the next one read from memory into
// registers while the current one is composed. A half tile writes its
// inline samples to a row of its own (2 tile + half).
template <class P, bool MOV, int G, int SP>
__global__ __launch_bounds__(SP * G) void k_seqg(SeqArgs a) {
    using R = typename P::R;
    using R2 = typename P::R2;
    static_assert(SP == kWave || SP == kWave / 2, "a whole tile or one half per workgroup");
    constexpr int NT = SP * G;
    constexpr int NW = NT / kWave;  // wavefronts
    // events staged per segment at most: kSegPerLane per lane, half that for
    // half tiles (their event prefetch then fits the registers unspilled)
    constexpr int C = kSegPerLane * G / (kWave / SP) + 1;
    constexpr int kPre = (C * kEvWords + NT - 1) / NT;  // dwords per thread in flight
    __shared__ uint32_t lds[2][C * kSegStride];
    __shared__ double red[NW][2];
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    const int half = SP == kWave ? 0 : (int)(blockIdx.x & 1);
    const int sl = half * SP + tid / G;  // spin slot of the tile
    const int j = tid % G;               // share of each segment
    const int64_t tile = SP == kWave ? (int64_t)blockIdx.x : (int64_t)(blockIdx.x >> 1);
    const Tile T = a.tiles[tile];
    const SpinP<R> s = load_spin<R, MOV>(a.ph, T, sl, a.inv_gamma);
    const int64_t pidx = tile * kWave + sl;
    if (a.vbits && j == 0 && sl < T.count) {
        const int32_t bad = spin_flags(a.ph, T.spin0 + sl);
        if (bad) atomicOr(a.vbits, bad);
    }
    R mr = R(0), mi = R(0), mz = s.pd;
    if (!a.init) {
        R2 m = reinterpret_cast<const R2 *>(a.mxy)[pidx];
        mr = m.x;
        mi = m.y;
        mz = reinterpret_cast<const R *>(a.mz)[pidx];
    }
    R eps1c = R(0), eps2c = R(0);  // relaxation cache (see event_eps)
    double dt_cached = -1.0;
    const bool no_offres = __ballot(s.bz0 != R(0)) == 0;  // per wavefront, as in k_seq
    const uint32_t *gev = reinterpret_cast<const uint32_t *>(a.ev);

    // events [first, last) of segment si within this launch's range, and
    // whether its observation event is in the range
    auto clip = [&](int64_t si, int64_t &first, int64_t &mid, bool &obs) {
        const SegEv g = a.segs[si];
        first = g.e0 > a.e0 ? (int64_t)g.e0 : a.e0;
        mid = g.e1 < a.e1 ? (int64_t)g.e1 : a.e1;
        if (mid < first) mid = first;
        obs = g.obs && g.e1 >= a.e0 && g.e1 < a.e1;
    };
    uint32_t pre[kPre];
    auto fetch = [&](int64_t si) {
        int64_t f, m;
        bool o;
        clip(si, f, m, o);
        const int n = (int)(m - f) + (o ? 1 : 0);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            const int w = tid + r * NT;
            pre[r] = w < n * kEvWords ? gev[f * kEvWords + w] : 0u;
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            const int w = tid + r * NT;
            if (w < C * kEvWords) lds[buf][(w / kEvWords) * kSegStride + w % kEvWords] = pre[r];
        }
    };
    if (a.s0 < a.s1) {
        fetch(a.s0);
        stage(0);
    }
    __syncthreads();
    for (int64_t si = a.s0; si < a.s1; ++si) {
        const int buf = (int)((si - a.s0) & 1);
        if (si + 1 < a.s1) fetch(si + 1);  // in flight while this segment is composed
        int64_t first, mid;
        bool obs;
        clip(si, first, mid, obs);
        const int L = (int)(mid - first);
        const uint32_t *base = lds[buf];
        if (L > 0) {  // uniform
            const int lo = (j * L) / G, hi = ((j + 1) * L) / G;
            Aff<R> m = aff_identity<R>();
            if (lo < hi) {
                m = event_map<P, MOV>(EvL{base + lo * kSegStride}, s, no_offres, dt_cached, eps1c, eps2c);
                for (int k = lo + 1; k < hi; ++k) {
                    const EvL ev{base + k * kSegStride};
                    m = aff_then(event_map<P, MOV>(ev, s, no_offres, dt_cached, eps1c, eps2c), m);
                }
            }
            // tree over the shares: at step d, share j (a multiple of 2d) takes
            // share j + d's product after its own, so share 0 ends with the
            // composite of the segment (the other shares' products are not
            // used, and share 0 alone carries the spin's state)
            if constexpr (G > 1) m = aff_then(aff_lane_xor<1>(m), m);
            if constexpr (G > 2) m = aff_then(aff_lane_xor<2>(m), m);
            if constexpr (G > 4) m = aff_then(aff_lane_xor<4>(m), m);
            if constexpr (G > 8) m = aff_then(aff_lane_xor<8>(m), m);
            static_assert(G <= 16, "at most 16 lanes per spin");
            aff_apply(m, mr, mi, mz);
        }
        if (obs) {  // uniform
            const EvL ev{base + L * kSegStride};
            const int kind = ev.kind();
            if (kind == EV_SNAP) {
                if (j == 0) reinterpret_cast<R2 *>(a.snap)[(int64_t)ev.a0() * (a.n_tiles * kWave) + pidx] = R2{mr, mi};
            } else {  // EV_ADC: inline samples, the workgroup's spins summed once each
                const double k0[4] = {ev.d(0), ev.d(1), ev.d(2), ev.d(3)};
                C2<R> c, w{R(1), R(0)};
                int cnt = 1;
                if (MOV) {
                    const double k1[3] = {ev.c64(0), ev.c64(1), ev.c64(2)};
                    c = cmul(C2<R>{mr, mi}, block_factor<P>(s, block_phase(s, k0, k1), k0[3]));
                } else {
                    const double dk[4] = {ev.d(4), ev.d(5), ev.d(6), ev.d(7)};
                    c = cmul(C2<R>{mr, mi}, block_factor<P>(s, block_phase(s, k0), k0[3]));
                    cnt = ev.count();
                    if (cnt > 1) w = block_factor<P>(s, block_phase(s, dk), dk[3]);
                }
                const int64_t n_planes = a.ph.n_coils > 0 ? a.ph.n_coils : 1;
                for (int i = 0; i < cnt; ++i) {
                    for (int64_t k = 0; k < n_planes; ++k) {
                        C2<R> v = c;
                        if (a.ph.n_coils > 0) {
                            C2<R> sk{R(0), R(0)};
                            if (sl < T.count)
                                sk = C2<R>{R(a.ph.sre[k * a.ph.n + T.spin0 + sl]), R(a.ph.sim[k * a.ph.n + T.spin0 + sl])};
                            v = cmul(sk, c);
                        }
                        if (j != 0) v = C2<R>{R(0), R(0)};
                        const R sr = wave_allsum(v.re);
                        const R sim = wave_allsum(v.im);
                        if (lane == 0) {
                            red[wave][0] = (double)sr;
                            red[wave][1] = (double)sim;
                        }
                        __syncthreads();
                        if (tid == 0) {
                            double tr = 0.0, ti = 0.0;
                            for (int q = 0; q < NW; ++q) {
                                tr += red[q][0];
                                ti += red[q][1];
                            }
                            const int64_t row = SP == kWave ? (int64_t)T.seg : 2 * (int64_t)T.seg + half;
                            reinterpret_cast<R2 *>(a.pa)[(k * a.n_rows + row) * a.n_inline + ev.a0() + i] = R2{R(tr), R(ti)};
                        }
                        __syncthreads();
                    }
                    c = cmul(c, w);
                }
            }
        }
        if (si + 1 < a.s1) stage(buf ^ 1);
        __syncthreads();
    }
    if (a.store && j == 0) {
        reinterpret_cast<R2 *>(a.mxy)[pidx] = R2{mr, mi};
        reinterpret_cast<R *>(a.mz)[pidx] = mz;
    }
}

// ---------------------------------------------------------------- k_par

// Spin parameters the sample-parallel kernel needs, kept in FP32 registers
// (the inputs are FP32); the FP64 block phase is formed at each anchor.
struct ParSpin {
    float x, y, z, dw, t2;  // t2 = +inf: no decay (also for empty lanes)
};

template <class R>
__device__ __forceinline__ double par_phase(const ParSpin &s, const double *k) {
    return -fma((double)s.x, k[0], fma((double)s.y, k[1], fma((double)s.z, k[2], (double)s.dw * kInv2Pi * k[3])));
}

template <class P>
__device__ __forceinline__ C2<typename P::R> par_factor(const ParSpin &s, const double *k) {
    using R = typename P::R;
    R sn, cs;
    P::sincos_turns(par_phase<R>(s, k), sn, cs);
    renorm(cs, sn);
    const R e2 = P::exp_neg(R(k[3]) / R(s.t2));
    return {cs * e2, sn * e2};
}

template <class P, int S>
__global__ __launch_bounds__(kWG) void k_par(ParArgs a) {
    using R = typename P::R;
    using R2 = typename P::R2;
    __shared__ double2 red[kWavesPerWG][kStretchMax];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const Block B = a.blocks[blockIdx.x];
    const int64_t n_pad = a.n_tiles * kWave;
    const int64_t coil = blockIdx.z;  // 0 without receive coils
    const bool coils = a.ph.n_coils > 0;

    const int64_t st0 = a.s0 + (int64_t)blockIdx.y * a.per_wg;
    const int64_t st1 = min(st0 + a.per_wg, a.s1);
    for (int64_t st = st0; st < st1; ++st) {
        const auto &S_ = as_const(a.st)[st];
        const int cnt = S_.count;
        const int slot = S_.slot;
        const int d0 = S_.d0;
        const double k0[4] = {S_.k0[0], S_.k0[1], S_.k0[2], S_.k0[3]};
        const double dk[4] = {S_.dk[0], S_.dk[1], S_.dk[2], S_.dk[3]};
        // exact anchor and per-sample factor of each of this lane's S spins
        // (tiles wave, wave + 4, ... of the block; FP64 phase). Spin data are
        // re-read per stretch (L2-resident) so that only the S recurrences and
        // the 16 sample sums stay in registers across the sample loop.
        C2<R> c[S], w[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int tl = wave + kWavesPerWG * j;
            ParSpin sp{0.f, 0.f, 0.f, 0.f, __builtin_inff()};
            C2<R> m{R(0), R(0)};
            if (tl < B.ntiles) {
                const Tile T = a.tiles[B.tile0 + tl];
                if (lane < T.count) {
                    const int64_t i = T.spin0 + lane;
                    sp = ParSpin{a.ph.x[i], a.ph.y[i], a.ph.z[i], a.ph.dw[i], a.ph.t2[i]};
                    const R2 v = reinterpret_cast<const R2 *>(a.snap)[(int64_t)slot * n_pad +
                                                                      (int64_t)(B.tile0 + tl) * kWave + lane];
                    m = C2<R>{v.x, v.y};
                    if (coils)  // coil `coil` sees sens * Mxy: fold it into the anchor
                        m = cmul(m, C2<R>{R(a.ph.sre[coil * a.ph.n + i]), R(a.ph.sim[coil * a.ph.n + i])});
                }
            }
            c[j] = cmul(m, par_factor<P>(sp, k0));
            w[j] = par_factor<P>(sp, dk);
        }
        for (int b0 = 0; b0 < cnt; b0 += kBatch) {
            R are[kBatch], aim[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                are[i] = R(0);
                aim[i] = R(0);
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
#pragma unroll
                for (int i = 0; i < kBatch; ++i) {
                    are[i] += c[j].re;
                    aim[i] += c[j].im;
                    c[j] = cmul(c[j], w[j]);
                }
            }
            transpose_sum16(are);
            transpose_sum16(aim);
            const int smp = b0 + (lane >> 2);
            if ((lane & 3) == 0 && smp < cnt) red[wave][smp] = make_double2((double)are[0], (double)aim[0]);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kWG) {
            double2 t = red[0][i];
#pragma unroll
            for (int wv = 1; wv < kWavesPerWG; ++wv) {
                t.x += red[wv][i].x;
                t.y += red[wv][i].y;
            }
            reinterpret_cast<double2 *>(a.pb)[(coil * a.n_blocks + (int64_t)blockIdx.x) * a.cols + (d0 - a.col0) + i] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- k_par_mov
//
// The sample-parallel kernel for moving spins, x(t) = x + v t. Over a stretch
// of evenly spaced samples on a constant gradient the moments K are linear
// and the first moments K1 quadratic in the sample index j, so the phase
// -(x.K(j) + v.K1(j) + f tau(j)) is quadratic in j: the per-sample factor
// changes by a constant factor U = exp(-i 2 pi v.d2k1) from one sample to the
// next. Each spin is re-anchored exactly (FP64 phase) at the start of every
// batch of 16 samples, then c <- c w, w <- w U. Same block and stretch layout
// as k_par; spin data are re-read per batch (cache-resident).
template <class P, int S>
__global__ __launch_bounds__(kWG) void k_par_mov(ParArgs a) {
    using R = typename P::R;
    using R2 = typename P::R2;
    __shared__ double2 red[kWavesPerWG][kStretchMax];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const Block B = a.blocks[blockIdx.x];
    const int64_t n_pad = a.n_tiles * kWave;
    const int64_t coil = blockIdx.z;  // 0 without receive coils
    const bool coils = a.ph.n_coils > 0;

    const int64_t st0 = a.s0 + (int64_t)blockIdx.y * a.per_wg;
    const int64_t st1 = min(st0 + a.per_wg, a.s1);
    for (int64_t st = st0; st < st1; ++st) {
        const auto &S_ = as_const(a.st)[st];
        const int cnt = S_.count;
        const int slot = S_.slot;
        const int d0 = S_.d0;
        for (int b0 = 0; b0 < cnt; b0 += kBatch) {
            // moments of sample b0 and the increments at b0 (FP64)
            const double jb = (double)b0;
            const double kb[4] = {fma(jb, S_.dk[0], S_.k0[0]), fma(jb, S_.dk[1], S_.k0[1]),
                                  fma(jb, S_.dk[2], S_.k0[2]), fma(jb, S_.dk[3], S_.k0[3])};
            const double hb = 0.5 * jb * (jb - 1.0);
            const double k1b[3] = {fma(hb, S_.d2k1[0], fma(jb, S_.dk1[0], S_.k1[0])),
                                   fma(hb, S_.d2k1[1], fma(jb, S_.dk1[1], S_.k1[1])),
                                   fma(hb, S_.d2k1[2], fma(jb, S_.dk1[2], S_.k1[2]))};
            const double d1b[3] = {fma(jb, S_.d2k1[0], S_.dk1[0]), fma(jb, S_.d2k1[1], S_.dk1[1]),
                                   fma(jb, S_.d2k1[2], S_.dk1[2])};
            R are[kBatch], aim[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                are[i] = R(0);
                aim[i] = R(0);
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int tl = wave + kWavesPerWG * j;
                float x = 0.f, y = 0.f, z = 0.f, dw = 0.f, t2 = __builtin_inff(), vx = 0.f, vy = 0.f, vz = 0.f;
                C2<R> m{R(0), R(0)};
                if (tl < B.ntiles) {
                    const Tile T = a.tiles[B.tile0 + tl];
                    if (lane < T.count) {
                        const int64_t i = T.spin0 + lane;
                        x = a.ph.x[i];
                        y = a.ph.y[i];
                        z = a.ph.z[i];
                        dw = a.ph.dw[i];
                        t2 = a.ph.t2[i];
                        vx = a.ph.vx[i];
                        vy = a.ph.vy[i];
                        vz = a.ph.vz[i];
                        const R2 v = reinterpret_cast<const R2 *>(a.snap)[(int64_t)slot * n_pad +
                                                                          (int64_t)(B.tile0 + tl) * kWave + lane];
                        m = C2<R>{v.x, v.y};
                        if (coils) m = cmul(m, C2<R>{R(a.ph.sre[coil * a.ph.n + i]), R(a.ph.sim[coil * a.ph.n + i])});
                    }
                }
                const double f = (double)dw * kInv2Pi;
                // phase at b0, its increment to b0 + 1, and the increment's change (turns)
                const double ph0 = -fma((double)x, kb[0], fma((double)y, kb[1], fma((double)z, kb[2],
                                   fma((double)vx, k1b[0], fma((double)vy, k1b[1], fma((double)vz, k1b[2], f * kb[3]))))));
                const double ph1 = -fma((double)x, S_.dk[0], fma((double)y, S_.dk[1], fma((double)z, S_.dk[2],
                                   fma((double)vx, d1b[0], fma((double)vy, d1b[1], fma((double)vz, d1b[2], f * S_.dk[3]))))));
                const double ph2 = -fma((double)vx, S_.d2k1[0], fma((double)vy, S_.d2k1[1], (double)vz * S_.d2k1[2]));
                const R r2 = R(1) / R(t2);  // +inf -> 0: no decay
                R sn, cs;
                P::sincos_turns(ph0, sn, cs);
                renorm(cs, sn);
                const R e0 = P::exp_neg(R(kb[3]) * r2);
                C2<R> c = cmul(m, C2<R>{cs * e0, sn * e0});
                P::sincos_turns(ph1, sn, cs);
                renorm(cs, sn);
                const R e1 = P::exp_neg(R(S_.dk[3]) * r2);
                C2<R> w{cs * e1, sn * e1};
                P::sincos_turns(ph2, sn, cs);
                renorm(cs, sn);
                const C2<R> u{cs, sn};
#pragma unroll
                for (int i = 0; i < kBatch; ++i) {
                    are[i] += c.re;
                    aim[i] += c.im;
                    c = cmul(c, w);
                    w = cmul(w, u);
                }
            }
            transpose_sum16(are);
            transpose_sum16(aim);
            const int smp = b0 + (lane >> 2);
            if ((lane & 3) == 0 && smp < cnt) red[wave][smp] = make_double2((double)are[0], (double)aim[0]);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kWG) {
            double2 t = red[0][i];
#pragma unroll
            for (int wv = 1; wv < kWavesPerWG; ++wv) {
                t.x += red[wv][i].x;
                t.y += red[wv][i].y;
            }
            reinterpret_cast<double2 *>(a.pb)[(coil * a.n_blocks + (int64_t)blockIdx.x) * a.cols + (d0 - a.col0) + i] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- work order
//
// The matrix-core sample kernels run a grid of (spin block) x (stretch
// batch) workgroups. Launched in the order x fastest, the batches of one
// spin block would be a whole row of spin blocks apart, and every batch
// would fetch the block's spin data again from memory. Workgroups are
// dispatched to the eight XCDs in turn (workgroup L to XCD L % 8), each with
// its own L2, so XCD x takes a contiguous range of the order (spin block,
// then batch): the workgroups resident on one XCD at a time are the batches
// of a few spin blocks, and share those blocks' data in its L2.
struct ParWG {
    int64_t blk, batch;
};
__device__ __forceinline__ ParWG par_work_item() {
    const int64_t nx = gridDim.x, ny = gridDim.y;
    const int64_t L = (int64_t)blockIdx.x + nx * (int64_t)blockIdx.y;  // dispatch order within a z plane
    const int64_t per = nx * ny / 8;
    const int64_t w = L < 8 * per ? (L % 8) * per + L / 8 : L;
    return {w / ny, w % ny};
}

// ---------------------------------------------------------------- k_par_mm
//
// The mixed-precision sample-parallel kernel on the matrix cores. For one
// stretch, spin s contributes c_s w_s^j to sample j (c_s its anchor, w_s its
// per-sample factor). Writing j = 16 q + r (q < 8, r < 16),
//   S[16 q + r] = sum_s (c_s w_s^(16 q)) (w_s^r) = sum_s A[q][s] B[s][r],
// a complex product of an 8 x n_spins and an n_spins x 16 matrix: the sum
// over spins is the contraction. Two stretches whose B is the same (see
// below) stack their A into the 16 rows of v_mfma_f32_16x16x4f32 (FP32
// products and sums, four spins per instruction), and the complex product
// takes three real ones (Gauss):
//   P1 = (Re A + Im A) Re B,  P2 = Re A (Im B - Re B),  P3 = Im A (Re B + Im B),
//   Re S = P1 - P3,  Im S = P1 + P2,
// so 24 instructions per 64 spins and stretch instead of 32. Lane l of an
// instruction holds A[l % 16][l / 16] and B[l / 16][l % 16], and accumulates
// rows 4 (l / 16) + i of column l % 16: lanes l < 32 the first stretch of
// the pair, lanes l >= 32 the second, each with Re S and Im S of the same
// samples in its own registers.
//
// B depends on the stretch only through its increments, which the host makes
// bitwise equal within a family of stretches (all lines of one readout
// polarity, say). A workgroup takes up to NS stretches (6, or 4 for grids
// that 6 would leave short: a planner's choice) and loops
// over its tiles outside them: per tile and family, each lane forms its
// spin's w^r (r < 16) and w^(16 q) once, and the wavefront turns the B
// operands round through LDS into registers; per stretch only the anchor c
// and its 8 products c w^(16 q) are formed and staged, as their Re and Im
// planes (Re A + Im A is formed as the operands are read: a third less LDS
// traffic for one addition per operand, measured 5 % faster). The sums of
// all the batch's stretches stay in registers until the workgroup's tiles
// are done, then the four wavefronts are added in FP64 through LDS.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kStageFloats = 32;  // per spin: 2 A planes of 16 (per pair), or the B operands (32)

// par_factor with the decay rate 1/T2 given.
__device__ __forceinline__ C2<float> mm_factor(const ParSpin &s, float r2, const double *k) {
    float sn, cs;
    Mixed::sincos_turns(par_phase<float>(s, k), sn, cs);
    renorm(cs, sn);
    const float e2 = Mixed::exp_neg(float(k[3]) * r2);
    return {cs * e2, sn * e2};
}

// The anchor factor of a stretch start: as mm_factor but without the
// renormalisation (a single factor, not raised to powers).
__device__ __forceinline__ C2<float> mm_anchor(const ParSpin &s, float r2, const double *k) {
    float sn, cs;
    Mixed::sincos_turns(par_phase<float>(s, k), sn, cs);
    const float e2 = Mixed::exp_neg(float(k[3]) * r2);
    return {cs * e2, sn * e2};
}

// Tiles per wavefront: a.spl (a block is 4 a.spl tiles), a run-time value so
// that the planner can size the grid to whole rounds of resident workgroups.
template <int NS>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(kMMResident))) void k_par_mm(ParArgs a) {
    const int S = a.spl;
    // per-wavefront stage (8 KB): B operands at a family's start, the two
    // A planes per stretch pair; after the tiles, the FP64 sums
    // [wave][stretch of the pair][sample] (16 KB of the workgroup's 32)
    __shared__ __attribute__((aligned(16))) float stage[kWavesPerWG][kWave * kStageFloats];
    static_assert(sizeof(double2) * kWavesPerWG * 2 * kStretchMax <= sizeof(stage), "sums fit in the stage");
    static_assert(NS % 2 == 0, "whole stretch pairs per batch");
    constexpr int NP = NS / 2;  // stretch pairs per batch
    double2(*red)[2][kStretchMax] = reinterpret_cast<double2(*)[2][kStretchMax]>(&stage[0][0]);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const ParWG wg = par_work_item();
    const Block B = a.blocks[wg.blk];
    const int64_t n_pad = a.n_tiles * kWave;
    const int64_t coil = blockIdx.z;  // 0 without receive coils
    const bool coils = a.ph.n_coils > 0;
    float *my = stage[wave];
    // Stage layouts (floats), with XOR-permuted 16-byte chunks so that the
    // 16-byte writes of 8 consecutive lanes and the operand reads of a
    // wavefront fall in distinct banks:
    //   B: spin s, chunk c (w^(2c), w^(2c+1) as re, im, re, im) at 32 s + 4 (c ^ (s & 7));
    //   A plane p (Re A, Im A) at 1024 p: spin s, chunk c (rows 4c .. 4c + 3;
    //   row 8 h + q is A[q] of stretch h of the pair) at 16 s + 4 (c ^ ((s >> 1) & 3)).
    const int m = lane & 15, g = lane >> 4;  // row (A) / column (B) m; spin 4u + g of group u
    // operand read positions for even and odd u (spin 4u + g), plus 64 u (A) or 128 u (B)
    const int a_rd0 = 16 * g + 4 * ((m >> 2) ^ (g >> 1)) + (m & 3);
    const int a_rd1 = 16 * g + 4 * ((m >> 2) ^ (2 + (g >> 1))) + (m & 3);
    const int b_rd0 = 32 * g + 4 * ((m >> 1) ^ g) + 2 * (m & 1);
    const int b_rd1 = 32 * g + 4 * ((m >> 1) ^ (4 + g)) + 2 * (m & 1);

    const int64_t st0 = a.s0 + wg.batch * a.per_wg;
    const int64_t st1 = min(st0 + a.per_wg, a.s1);
    for (int64_t sb = st0; sb < st1; sb += NS) {
        const int nb = (int)min<int64_t>(NS, st1 - sb);  // uniform
        f32x4 acc[NP][3];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p][0] = acc[p][1] = acc[p][2] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < S; ++j) {
            // the wavefront's tile (uniform: read through the scalar cache)
            const int tl = __builtin_amdgcn_readfirstlane(wave) + kWavesPerWG * j;
            if (tl >= B.ntiles) break;  // uniform; later slots are empty too
            const auto &T = as_const(a.tiles)[B.tile0 + tl];
            const bool valid = lane < T.count;
            const int64_t pidx = (int64_t)(B.tile0 + tl) * kWave + lane;  // padded spin slot of this lane
            // every load of the tile issued at once: spin data, sensitivity,
            // and the snapshots of the batch's stretches
            ParSpin spn{0.f, 0.f, 0.f, 0.f, __builtin_inff()};
            C2<float> sens{1.f, 0.f};
            float2 snap[NS];
            // snapshots of stretch i2 of the batch (zero for empty lanes)
            auto load_snap = [&](int i2) {
                snap[i2] = make_float2(0.f, 0.f);
                if (valid)
                    snap[i2] = reinterpret_cast<const float2 *>(a.snap)[(int64_t)as_const(a.st)[sb + min(i2, nb - 1)].slot * n_pad + pidx];
            };
            if (valid) {
                const int64_t i = T.spin0 + lane;
                spn = ParSpin{a.ph.x[i], a.ph.y[i], a.ph.z[i], a.ph.dw[i], a.ph.t2[i]};
                if (coils) sens = C2<float>{a.ph.sre[coil * a.ph.n + i], a.ph.sim[coil * a.ph.n + i]};
            }
            load_snap(0);
            load_snap(1);
            const float r2 = __builtin_amdgcn_rcpf(spn.t2);  // +inf -> 0: no decay
            int32_t fam = -1;                                   // family of the operands in registers
            C2<float> wq[8];                                    // w^(16 q)
            float b1[16], b2[16], b3[16];                       // Re B, Im B - Re B, Re B + Im B (spin 4u + g, column m)
            // anchor of stretch i2 of the batch: snapshot x coil sensitivity x
            // exact FP64-phase factor
            auto anchor = [&](const auto &T_, int i2) -> C2<float> {
                C2<float> mm{snap[i2].x, snap[i2].y};
                if (coils) mm = cmul(mm, sens);
                const double k0[4] = {T_.k0[0], T_.k0[1], T_.k0[2], T_.k0[3]};
                return cmul(mm, mm_anchor(spn, r2, k0));
            };
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                // a short batch repeats its last stretch (no branch around the
                // products, so the sums keep their registers); the repeats are
                // not stored
                const auto &Sa = as_const(a.st)[sb + min(2 * p, nb - 1)];
                const auto &Sb = as_const(a.st)[sb + min(2 * p + 1, nb - 1)];
                // two families in one pair: one pass per stretch, the other half zero
                const int passes = Sa.fam == Sb.fam ? 1 : 2;  // uniform
                for (int pass = 0; pass < passes; ++pass) {
                    const auto &Sf = pass == 0 ? Sa : Sb;
                    if (Sf.fam != fam) {  // uniform: the first stretch, or a new family
                        fam = Sf.fam;
                        const double dk[4] = {Sf.dk[0], Sf.dk[1], Sf.dk[2], Sf.dk[3]};
                        const C2<float> w = mm_factor(spn, r2, dk);
                        // powers by a shallow product tree
                        C2<float> pw[16];
                        pw[0] = C2<float>{1.f, 0.f};
                        pw[1] = w;
                        pw[2] = cmul(w, w);
                        pw[3] = cmul(pw[2], w);
                        pw[4] = cmul(pw[2], pw[2]);
#pragma unroll
                        for (int r = 5; r < 8; ++r) pw[r] = cmul(pw[4], pw[r - 4]);
                        pw[8] = cmul(pw[4], pw[4]);
#pragma unroll
                        for (int r = 9; r < 16; ++r) pw[r] = cmul(pw[8], pw[r - 8]);
                        wq[0] = C2<float>{1.f, 0.f};
                        wq[1] = cmul(pw[8], pw[8]);
                        wq[2] = cmul(wq[1], wq[1]);
                        wq[3] = cmul(wq[2], wq[1]);
                        wq[4] = cmul(wq[2], wq[2]);
#pragma unroll
                        for (int q = 5; q < 8; ++q) wq[q] = cmul(wq[4], wq[q - 4]);
                        // write positions formed here from an opaque copy of
                        // the lane, not hoisted out of the loops into registers
                        int ln_b;
                        asm volatile("v_mov_b32 %0, %1" : "=v"(ln_b) : "v"(lane));
                        float *bw = my + 32 * ln_b;
                        const int bsw = ln_b & 7;
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            *reinterpret_cast<float4 *>(bw + 4 * (c ^ bsw)) =
                                make_float4(pw[2 * c].re, pw[2 * c].im, pw[2 * c + 1].re, pw[2 * c + 1].im);
                        // the stage is private to this wavefront, and its LDS
                        // operations complete in program order: only the
                        // compiler must not move LDS accesses across these points
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int u = 0; u < 16; ++u) {
                            const float2 v = *reinterpret_cast<const float2 *>(my + 128 * u + ((u & 1) ? b_rd1 : b_rd0));
                            b1[u] = v.x;
                            b2[u] = v.y - v.x;
                            b3[u] = v.x + v.y;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                    const C2<float> zero{0.f, 0.f};
                    const C2<float> ca = (passes == 1 || pass == 0) ? anchor(Sa, 2 * p) : zero;
                    const C2<float> cb = (passes == 1 || pass == 1) ? anchor(Sb, 2 * p + 1) : zero;
                    C2<float> aa[8], ab[8];
                    aa[0] = ca;
                    ab[0] = cb;
#pragma unroll
                    for (int q = 1; q < 8; ++q) {
                        aa[q] = cmul(ca, wq[q]);
                        ab[q] = cmul(cb, wq[q]);
                    }
                    int ln_a;
                    asm volatile("v_mov_b32 %0, %1" : "=v"(ln_a) : "v"(lane));
                    float *pl = my + 16 * ln_a;
                    const int a_sw = (ln_a >> 1) & 3;
#define KOMA_A4(arr, q0, f) make_float4(f(arr[q0]), f(arr[q0 + 1]), f(arr[q0 + 2]), f(arr[q0 + 3]))
#define KOMA_RE(z) ((z).re)
#define KOMA_IM(z) ((z).im)
                    *reinterpret_cast<float4 *>(pl + 4 * (0 ^ a_sw)) = KOMA_A4(aa, 0, KOMA_RE);
                    *reinterpret_cast<float4 *>(pl + 4 * (1 ^ a_sw)) = KOMA_A4(aa, 4, KOMA_RE);
                    *reinterpret_cast<float4 *>(pl + 4 * (2 ^ a_sw)) = KOMA_A4(ab, 0, KOMA_RE);
                    *reinterpret_cast<float4 *>(pl + 4 * (3 ^ a_sw)) = KOMA_A4(ab, 4, KOMA_RE);
                    *reinterpret_cast<float4 *>(pl + 1024 + 4 * (0 ^ a_sw)) = KOMA_A4(aa, 0, KOMA_IM);
                    *reinterpret_cast<float4 *>(pl + 1024 + 4 * (1 ^ a_sw)) = KOMA_A4(aa, 4, KOMA_IM);
                    *reinterpret_cast<float4 *>(pl + 1024 + 4 * (2 ^ a_sw)) = KOMA_A4(ab, 0, KOMA_IM);
                    *reinterpret_cast<float4 *>(pl + 1024 + 4 * (3 ^ a_sw)) = KOMA_A4(ab, 4, KOMA_IM);
#undef KOMA_A4
#undef KOMA_RE
#undef KOMA_IM
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // the next pair's snapshots arrive during these products
                    if (p + 1 < NP && pass == passes - 1) {
                        load_snap(2 * p + 2);
                        load_snap(2 * p + 3);
                    }
                    // the planes in two halves of 8 spin groups: reads first
                    // (one wait), then Re A + Im A, then the products
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        float av[3][8];
#pragma unroll
                        for (int pl_ = 1; pl_ < 3; ++pl_)  // av[1] = Re A, av[2] = Im A
#pragma unroll
                            for (int uu = 0; uu < 8; ++uu) {
                                const int u = 8 * h + uu;
                                av[pl_][uu] = my[1024 * (pl_ - 1) + 64 * u + ((u & 1) ? a_rd1 : a_rd0)];
                            }
#pragma unroll
                        for (int uu = 0; uu < 8; ++uu) av[0][uu] = av[1][uu] + av[2][uu];
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int uu = 0; uu < 8; ++uu) {
                            const int u = 8 * h + uu;
                            acc[p][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][uu], b1[u], acc[p][0], 0, 0, 0);
                            acc[p][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][uu], b2[u], acc[p][1], 0, 0, 0);
                            acc[p][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2][uu], b3[u], acc[p][2], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        __syncthreads();  // every wavefront is done with its stage
        // The thread's indices formed afresh (an opaque copy of the thread id),
        // so that nothing derived from them stays live across the tile loop.
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
        const int e_wave = tid >> 6, e_lane = tid & 63, e_m = e_lane & 15, e_g = e_lane >> 4;
        // lane l holds rows 4 (l / 16) + v: stretch h = l / 32 of the pair,
        // q = 4 ((l / 16) % 2) + v; column m
        const int half = e_lane >> 5;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (2 * p >= nb) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int smp = 16 * (4 * (e_g & 1) + v) + e_m;
                const double p1 = (double)acc[p][0][v];
                red[e_wave][half][smp] = make_double2(p1 - (double)acc[p][2][v], p1 + (double)acc[p][1][v]);
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (2 * p + h >= nb) break;
                const auto &S_ = as_const(a.st)[sb + 2 * p + h];
                const int cnt = S_.count, d0 = S_.d0;
                for (int k = tid; k < cnt; k += kWG) {
                    double2 t = red[0][h][k];
#pragma unroll
                    for (int wv = 1; wv < kWavesPerWG; ++wv) {
                        t.x += red[wv][h][k].x;
                        t.y += red[wv][h][k].y;
                    }
                    reinterpret_cast<double2 *>(a.pb)[(coil * a.n_blocks + wg.blk) * a.cols + (d0 - a.col0) + k] = t;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- k_par_mm64
//
// The FP64 form of k_par_mm: the same factorisation S[16 q + r] =
// sum_s (c_s w_s^(16 q)) (w_s^r), two stretches of a family stacked in the 16
// rows, Gauss's three real products, now on v_mfma_f64_16x16x4f64 (FP64
// products and sums). That instruction takes its operands as the FP32 one
// (lane l: A[l % 16][l / 16], B[l / 16][l % 16]) but returns row 4 v + l / 16
// of column l % 16 in its element v. Every factor is formed in FP64 (exact
// FP64 phase, FP64 sincos and exp), the powers by the same shallow product
// trees. The family's B operands (Re B, Im B of spin 4 u + l / 16, column
// l % 16) are turned round through LDS into 64 registers once per tile and
// family, Im B - Re B and Re B + Im B formed at each use; the A rows of each
// stretch pair are staged in LDS as a Re and an Im plane, their sum formed
// as it is read.
// 16 KB of stage per wavefront: two workgroups per CU, two wavefronts per
// SIMD, so that one wavefront's LDS round trips and factors overlap the
// other's products.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kStage64 = 32;  // doubles per spin: B (16 complex), then A (16 rows, Re and Im planes)

// sin and cos of 2 pi h (h in turns) and exp(-x) for x >= 0 in FP64, shorter
// than the library routines (which cover every argument with branches):
// Taylor polynomials on exactly reduced arguments. sin, cos: y = 4 (h -
// rint(h)) and f = y - rint(y) are exact, |f| <= 1/2; sin(pi f / 2) to degree
// 17 and cos(pi f / 2) to degree 18 (truncation below 1e-19), then the
// quadrant rint(y) mod 4. exp: n = rint(-x log2 e), r = -x - n ln 2 with ln 2
// in two parts, |r| <= ln 2 / 2, exp(r) to degree 13 (truncation 4e-18),
// times 2^n. Against 80-bit references on the CPU: 1.5e-16 absolute (sin,
// cos), 1.4e-16 relative (exp).
constexpr double kSinPi2[9] = {  // (-1)^k (pi/2)^(2k+1) / (2k+1)!
    1.5707963267948966, -0.6459640975062463, 0.07969262624616705, -0.004681754135318688,
    0.00016044118478735983, -3.598843235212085e-06, 5.692172921967927e-08, -6.688035109811468e-10,
    6.0669357311061955e-12};
constexpr double kCosPi2[10] = {  // (-1)^k (pi/2)^(2k) / (2k)!
    1.0, -1.2337005501361697, 0.25366950790104803, -0.02086348076335296, 0.0009192602748394266,
    -2.5202042373060607e-05, 4.710874778818172e-07, -6.386603083791852e-09, 6.565963114979473e-11,
    -5.294400200734623e-13};
constexpr double kExpTaylor[14] = {  // 1 / k!
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333, 0.001388888888888889,
    0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06, 2.755731922398589e-07,
    2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10};

__device__ __forceinline__ void mm64_sincos_turns(double h, double &s, double &c) {
    const double y = 4.0 * (h - rint(h));
    const double q = rint(y);
    const double f = y - q, f2 = f * f;
    double ps = kSinPi2[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) ps = fma(ps, f2, kSinPi2[k]);
    const double sa = f * ps;
    double cb = kCosPi2[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) cb = fma(cb, f2, kCosPi2[k]);
    // sin(pi/2 (q + f)) = sa, cb, -sa, -cb and cos = cb, -sa, -cb, sa for q mod 4 = 0 .. 3
    const int iq = (int)q & 3;
    s = (iq & 1) ? cb : sa;
    c = (iq & 1) ? sa : cb;
    if (iq & 2) s = -s;
    if ((iq + 1) & 2) c = -c;
}

__device__ __forceinline__ double mm64_exp_neg(double x) {  // exp(-x), x >= 0 (NaN stays NaN)
    if (x > 746.0) return 0.0;
    const double y = -x;
    const double n = rint(y * 1.4426950408889634);
    double r = fma(-n, 0.6931467056274414, y);   // ln 2 to 21 bits: n ln2_hi exact
    r = fma(-n, 4.7493250390316726e-07, r);      // ln 2 - ln2_hi
    double p = kExpTaylor[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) p = fma(p, r, kExpTaylor[k]);
    return ldexp(p, (int)n);
}

// par_factor in FP64 with the decay rate 1/T2 given.
__device__ __forceinline__ C2<double> mm64_factor(const ParSpin &s, double r2, const double *k) {
    double sn, cs;
    mm64_sincos_turns(par_phase<double>(s, k), sn, cs);
    renorm(cs, sn);
    const double e2 = mm64_exp_neg(k[3] * r2);
    return {cs * e2, sn * e2};
}

__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(kMMResident64))) void k_par_mm64(ParArgs a) {
    const int S = a.spl;
    // per-wavefront stage (16 KB): B operands at a family's start, then the
    // A rows of the current stretch pair in a Re and an Im plane (1024
    // doubles each); after the tiles, the FP64 sums
    // [wave][stretch of the pair][sample]
    __shared__ __attribute__((aligned(16))) double stage[kWavesPerWG][kWave * kStage64];
    static_assert(sizeof(double2) * kWavesPerWG * 2 * kStretchMax <= sizeof(stage), "sums fit in the stage");
    static_assert(kMMStretches64 == 4, "two stretch pairs per batch");
    double2(*red)[2][kStretchMax] = reinterpret_cast<double2(*)[2][kStretchMax]>(&stage[0][0]);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const ParWG wg = par_work_item();
    const Block B = a.blocks[wg.blk];
    const int64_t n_pad = a.n_tiles * kWave;
    const int64_t coil = blockIdx.z;  // 0 without receive coils
    const bool coils = a.ph.n_coils > 0;
    double *my = stage[wave];
    // Stage layouts (doubles), 16-byte chunks XOR-permuted by the spin so
    // that the chunk writes of consecutive lanes fall in distinct banks:
    //   B: spin s, complex r at 32 s + 2 (r ^ (s & 15));
    //   A plane p (Re A, Im A) at 1024 p: spin s, rows 2c, 2c + 1 (row
    //   8 h + q is A[q] of stretch h of the pair) at 16 s + 2 (c ^ (s & 7)).
    const int m = lane & 15, g = lane >> 4;  // row (A) / column (B) m; spin 4u + g of group u
    // operand read positions: B of spin 4u + g at 128 u + b_rd[u % 4], A of
    // spin 4u + g at 64 u + a_rd[u % 2] (and 1024 further in the Im plane)
    int b_rd[4], a_rd[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) b_rd[k] = 32 * g + 2 * (m ^ (4 * k + g));
#pragma unroll
    for (int k = 0; k < 2; ++k) a_rd[k] = 16 * g + 2 * ((m >> 1) ^ (4 * k + g)) + (m & 1);

    const int64_t st0 = a.s0 + wg.batch * a.per_wg;
    const int64_t st1 = min(st0 + a.per_wg, a.s1);
    for (int64_t sb = st0; sb < st1; sb += kMMStretches64) {
        const int nb = (int)min<int64_t>(kMMStretches64, st1 - sb);  // uniform
        f64x4 acc[2][3];
#pragma unroll
        for (int p = 0; p < 2; ++p) acc[p][0] = acc[p][1] = acc[p][2] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < S; ++j) {
            const int tl = __builtin_amdgcn_readfirstlane(wave) + kWavesPerWG * j;
            if (tl >= B.ntiles) break;  // uniform; later slots are empty too
            const auto &T = as_const(a.tiles)[B.tile0 + tl];
            const bool valid = lane < T.count;
            const int64_t pidx = (int64_t)(B.tile0 + tl) * kWave + lane;  // padded spin slot of this lane
            // the tile's inputs (zero for empty lanes); the second pair's
            // snapshots arrive during the first pair's products
            ParSpin spn{0.f, 0.f, 0.f, 0.f, __builtin_inff()};
            C2<double> sens{1.0, 0.0};
            double2 snap[kMMStretches64];
            auto load_snap = [&](int i2) {
                snap[i2] = make_double2(0.0, 0.0);
                if (valid)
                    snap[i2] = reinterpret_cast<const double2 *>(a.snap)[(int64_t)as_const(a.st)[sb + min(i2, nb - 1)].slot * n_pad + pidx];
            };
            if (valid) {
                const int64_t i = T.spin0 + lane;
                spn = ParSpin{a.ph.x[i], a.ph.y[i], a.ph.z[i], a.ph.dw[i], a.ph.t2[i]};
                if (coils) sens = C2<double>{(double)a.ph.sre[coil * a.ph.n + i], (double)a.ph.sim[coil * a.ph.n + i]};
            }
            load_snap(0);
            load_snap(1);
            const double r2 = 1.0 / (double)spn.t2;  // +inf -> 0: no decay
            int32_t fam = -1;                         // family of the operands in registers
            C2<double> w16;                           // w^16
            double bre[16], bim[16];                  // Re B, Im B (spin 4u + g, column m)
            auto anchor = [&](const auto &T_, int i2) -> C2<double> {
                C2<double> mm{snap[i2].x, snap[i2].y};
                if (coils) mm = cmul(mm, sens);
                const double k0[4] = {T_.k0[0], T_.k0[1], T_.k0[2], T_.k0[3]};
                return cmul(mm, mm64_factor(spn, r2, k0));
            };
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                // a short batch repeats its last stretch; the repeats are not stored
                const auto &Sa = as_const(a.st)[sb + min(2 * p, nb - 1)];
                const auto &Sb = as_const(a.st)[sb + min(2 * p + 1, nb - 1)];
                const int passes = Sa.fam == Sb.fam ? 1 : 2;  // uniform
                for (int pass = 0; pass < passes; ++pass) {
                    const auto &Sf = pass == 0 ? Sa : Sb;
                    if (Sf.fam != fam) {  // uniform: the first stretch, or a new family
                        fam = Sf.fam;
                        const double dk[4] = {Sf.dk[0], Sf.dk[1], Sf.dk[2], Sf.dk[3]};
                        __builtin_amdgcn_sched_barrier(0);
                        const C2<double> w = mm64_factor(spn, r2, dk);
                        __builtin_amdgcn_sched_barrier(0);
                        C2<double> pw[16];
                        pw[0] = C2<double>{1.0, 0.0};
                        pw[1] = w;
                        pw[2] = cmul(w, w);
                        pw[3] = cmul(pw[2], w);
                        pw[4] = cmul(pw[2], pw[2]);
#pragma unroll
                        for (int r = 5; r < 8; ++r) pw[r] = cmul(pw[4], pw[r - 4]);
                        pw[8] = cmul(pw[4], pw[4]);
#pragma unroll
                        for (int r = 9; r < 16; ++r) pw[r] = cmul(pw[8], pw[r - 8]);
                        w16 = cmul(pw[8], pw[8]);
                        // the stage is private to this wavefront, and its LDS
                        // operations complete in program order: only the
                        // compiler must not move LDS accesses across these points
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        // write positions formed here from an opaque copy of
                        // the lane (not hoisted out of the loops, where they
                        // would hold 16 registers)
                        int ln;
                        asm volatile("v_mov_b32 %0, %1" : "=v"(ln) : "v"(lane));
                        double *bw = my + 32 * ln;
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            *reinterpret_cast<double2 *>(bw + 2 * (r ^ (ln & 15))) = make_double2(pw[r].re, pw[r].im);
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int u = 0; u < 16; ++u) {
                            const double2 v = *reinterpret_cast<const double2 *>(my + 128 * u + b_rd[u & 3]);
                            bre[u] = v.x;
                            bim[u] = v.y;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    const C2<double> zero{0.0, 0.0};
                    const C2<double> ca = (passes == 1 || pass == 0) ? anchor(Sa, 2 * p) : zero;
                    __builtin_amdgcn_sched_barrier(0);
                    const C2<double> cb = (passes == 1 || pass == 1) ? anchor(Sb, 2 * p + 1) : zero;
                    __builtin_amdgcn_sched_barrier(0);
                    if (p == 0 && pass == passes - 1) {
                        load_snap(2);
                        load_snap(3);
                    }
                    int ln;
                    asm volatile("v_mov_b32 %0, %1" : "=v"(ln) : "v"(lane));
                    double *pl = my + 16 * ln;
                    const int sw = ln & 7;
                    // rows 2c, 2c + 1: stretch a (c < 4) or b, q = 2c % 8 and
                    // 2c % 8 + 1; A[q] = c w^(16 q) by successive products
                    // with w^16 (the two stretches' chains interleaved; 7
                    // FP64 roundings at most, far inside the FP64 form's
                    // error)
                    C2<double> xa = ca, xb = cb;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const C2<double> ya = cmul(xa, w16), yb = cmul(xb, w16);
                        *reinterpret_cast<double2 *>(pl + 2 * (c ^ sw)) = make_double2(xa.re, ya.re);
                        *reinterpret_cast<double2 *>(pl + 1024 + 2 * (c ^ sw)) = make_double2(xa.im, ya.im);
                        *reinterpret_cast<double2 *>(pl + 2 * ((c + 4) ^ sw)) = make_double2(xb.re, yb.re);
                        *reinterpret_cast<double2 *>(pl + 1024 + 2 * ((c + 4) ^ sw)) = make_double2(xb.im, yb.im);
                        if (c < 3) {
                            xa = cmul(ya, w16);
                            xb = cmul(yb, w16);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    // four quarters of 4 spin groups: reads first (one wait),
                    // then Re A + Im A and the products
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        double are[4], aim[4];
#pragma unroll
                        for (int uu = 0; uu < 4; ++uu) {
                            const int ai = 64 * (4 * h + uu) + a_rd[uu & 1];
                            are[uu] = my[ai];
                            aim[uu] = my[ai + 1024];
                        }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int uu = 0; uu < 4; ++uu) {
                            const int u = 4 * h + uu;
                            acc[p][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[uu] + aim[uu], bre[u], acc[p][0], 0, 0, 0);
                            acc[p][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[uu], bim[u] - bre[u], acc[p][1], 0, 0, 0);
                            acc[p][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[uu], bre[u] + bim[u], acc[p][2], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        __syncthreads();  // every wavefront is done with its stage
        // element v of lane l: row 4 v + l / 16 = 8 h + q of column l % 16, so
        // stretch h = v / 2 of the pair and q = 4 (v % 2) + l / 16
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            if (2 * p >= nb) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int smp = 16 * (4 * (v & 1) + g) + m;
                const double p1 = acc[p][0][v];
                red[wave][v >> 1][smp] = make_double2(p1 - acc[p][2][v], p1 + acc[p][1][v]);
            }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (2 * p + h >= nb) break;
                const auto &S_ = as_const(a.st)[sb + 2 * p + h];
                const int cnt = S_.count, d0 = S_.d0;
                for (int k = threadIdx.x; k < cnt; k += kWG) {
                    double2 t = red[0][h][k];
#pragma unroll
                    for (int wv = 1; wv < kWavesPerWG; ++wv) {
                        t.x += red[wv][h][k].x;
                        t.y += red[wv][h][k].y;
                    }
                    reinterpret_cast<double2 *>(a.pb)[(coil * a.n_blocks + wg.blk) * a.cols + (d0 - a.col0) + k] = t;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- k_reduce

// sig[k][g][adc(c)] = sum over rows r of group g (in order) of part[k][r][c],
// k = blockIdx.z the coil. A workgroup covers 64 columns; its 4 wavefronts
// take rows r = r0 + w (mod 4) and the four partial sums are added in wave
// order.
template <class T2>
__global__ __launch_bounds__(kWG) void k_reduce(ReduceArgs a) {
    __shared__ double2 red[kWavesPerWG][kWave];
    if (a.gate && *as_const(a.gate) != 0) return;  // uniform: invalid inputs leave the output untouched
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * kWave + lane;
    const int64_t k = blockIdx.z;
    const T2 *part = reinterpret_cast<const T2 *>(a.part) + k * a.part_stride;
    double2 *sig = reinterpret_cast<double2 *>(a.sig) + k * a.n_groups * a.n_adc;
    for (int64_t g = blockIdx.y; g < a.n_groups; g += gridDim.y) {  // uniform per workgroup
        const int32_t r0 = a.row_off[g], r1 = a.row_off[g + 1];
        double sx = 0.0, sy = 0.0;
        if (col < a.cols) {
            for (int32_t r = r0 + wave; r < r1; r += kWavesPerWG) {
                T2 v = part[(int64_t)r * a.cols + col];
                sx += (double)v.x;
                sy += (double)v.y;
            }
        }
        red[wave][lane] = make_double2(sx, sy);
        __syncthreads();
        if (wave == 0 && col < a.cols) {
            double2 t = red[0][lane];
#pragma unroll
            for (int wv = 1; wv < kWavesPerWG; ++wv) {
                t.x += red[wv][lane].x;
                t.y += red[wv][lane].y;
            }
            sig[g * a.n_adc + a.col_to_adc[col]] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- k_export

// gate: nullptr, or a flag that must be 0 for anything to be written.
template <class R, class R2>
__global__ __launch_bounds__(kWG) void k_export(const Tile *tiles, int64_t n_tiles, const R2 *mxy,
                                                const R *mz, double *out, const int32_t *gate) {
    if (gate && *as_const(gate) != 0) return;
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int64_t tile = p / kWave;
    const int lane = (int)(p % kWave);
    if (tile >= n_tiles) return;
    const Tile T = tiles[tile];
    if (lane >= T.count) return;
    const int64_t i = T.spin0 + lane;
    out[3 * i + 0] = (double)mxy[p].x;
    out[3 * i + 1] = (double)mxy[p].y;
    out[3 * i + 2] = (double)mz[p];
}

// ---------------------------------------------------------------- k_validate

// Per-workgroup flags of invalid phantom values (device-resident phantoms):
// bit 0 non-finite x, y, z, dw, PD or velocity; bit 1 PD < 0; bit 2 T1 or T2
// <= 0 or NaN; bit 3 non-finite coil sensitivity.
__global__ __launch_bounds__(kWG) void k_validate(PhantomDev ph, int64_t n, int32_t *flags) {
    __shared__ int32_t f[kWG];
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int32_t bad = i < n ? spin_flags(ph, i) : 0;
    f[threadIdx.x] = bad;
    __syncthreads();
    for (int s = kWG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) f[threadIdx.x] |= f[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[blockIdx.x] = f[0];
}

// ---------------------------------------------------------------- k_upload

// Copy n 16-byte words from pinned host memory (mapped into the device's
// address space) to device memory, on the compute queue: the packed tables
// of a call reach the device without a DMA-engine copy, whose ordering with
// the kernels around it costs tens of microseconds per call.
__global__ __launch_bounds__(kWG) void k_upload(const uint4 *src, uint4 *dst, int64_t n, int32_t *zero) {
    if (zero && blockIdx.x == 0 && threadIdx.x == 0) *zero = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        dst[i] = src[i];
}

// ---------------------------------------------------------------- launchers

static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

// FP32 maps: up to 16 lanes per spin (1024-lane workgroups, 128 registers);
// FP64 maps: up to 8 (their registers do not fit beside 1024 lanes).
template <class P, bool MOV>
static int launch_seqg(const SeqArgs &a, hipStream_t st) {
    constexpr bool f32 = sizeof(typename P::R) == 4;
    const dim3 grid((unsigned)a.n_tiles);
    // 16 lanes: whole tiles in FP32 (1,024-lane workgroups); half tiles in
    // FP64 (512 lanes: two of its wavefronts per SIMD), two rows per tile
    if (a.half_tiles != (!f32 && a.lanes == 16)) return -1;
    switch (a.lanes) {
        case 2: hipLaunchKernelGGL((k_seqg<P, MOV, 2, kWave>), grid, dim3(kWave * 2), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_seqg<P, MOV, 4, kWave>), grid, dim3(kWave * 4), 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_seqg<P, MOV, 8, kWave>), grid, dim3(kWave * 8), 0, st, a); break;
        case 16:
            if constexpr (f32)
                hipLaunchKernelGGL((k_seqg<P, MOV, 16, kWave>), grid, dim3(kWave * 16), 0, st, a);
            else
                hipLaunchKernelGGL((k_seqg<P, MOV, 16, kWave / 2>), dim3(2 * (unsigned)a.n_tiles),
                                   dim3(kWave / 2 * 16), 0, st, a);
            break;
        default: return -1;
    }
    return 0;
}

int launch_seq(bool fp64, bool moving, const SeqArgs &a, void *stream) {
    if (a.n_tiles <= 0 || a.e1 <= a.e0) return 0;
    // moving spins need all three velocity arrays (checked on the host)
    if (moving && (!a.ph.vx || !a.ph.vy || !a.ph.vz)) return -1;
    if (a.ph.n_coils < 0 || (a.ph.n_coils > 0 && (!a.ph.sre || !a.ph.sim))) return -1;
    hipStream_t st = (hipStream_t)stream;
    if (a.lanes > 1) {
        if (!a.segs || a.s1 < a.s0) return -1;
        if (a.s1 == a.s0) return 0;
        int r;
        if (fp64)
            r = moving ? launch_seqg<FP64, true>(a, st) : launch_seqg<FP64, false>(a, st);
        else
            r = moving ? launch_seqg<Mixed, true>(a, st) : launch_seqg<Mixed, false>(a, st);
        return r != 0 ? r : check_launch();
    }
    dim3 grid((unsigned)((a.n_tiles + kWavesPerWG - 1) / kWavesPerWG));
    if (fp64) {
        if (moving)
            hipLaunchKernelGGL((k_seq<FP64, true>), grid, dim3(kWG), 0, st, a);
        else
            hipLaunchKernelGGL((k_seq<FP64, false>), grid, dim3(kWG), 0, st, a);
    } else {
        if (moving)
            hipLaunchKernelGGL((k_seq<Mixed, true>), grid, dim3(kWG), 0, st, a);
        else
            hipLaunchKernelGGL((k_seq<Mixed, false>), grid, dim3(kWG), 0, st, a);
    }
    return check_launch();
}

static void par_dispatch_mm(int spl, dim3 grid, const ParArgs &a, hipStream_t st) {
    ParArgs b = a;
    b.spl = spl;
    if (a.per_wg == kMMStretches)
        hipLaunchKernelGGL(k_par_mm<kMMStretches>, grid, dim3(kWG), 0, st, b);
    else
        hipLaunchKernelGGL(k_par_mm<kMMStretchesSmall>, grid, dim3(kWG), 0, st, b);
}

static void par_dispatch_mm64(int spl, dim3 grid, const ParArgs &a, hipStream_t st) {
    ParArgs b = a;
    b.spl = spl;
    hipLaunchKernelGGL(k_par_mm64, grid, dim3(kWG), 0, st, b);
}

template <class P>
static void par_dispatch(int spl, dim3 grid, const ParArgs &a, hipStream_t st) {
    switch (spl) {
        case 1: hipLaunchKernelGGL((k_par<P, 1>), grid, dim3(kWG), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_par<P, 2>), grid, dim3(kWG), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_par<P, 4>), grid, dim3(kWG), 0, st, a); break;
        default: hipLaunchKernelGGL((k_par<P, 8>), grid, dim3(kWG), 0, st, a); break;
    }
}

template <class P>
static void par_dispatch_mov(int spl, dim3 grid, const ParArgs &a, hipStream_t st) {
    switch (spl) {
        case 1: hipLaunchKernelGGL((k_par_mov<P, 1>), grid, dim3(kWG), 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_par_mov<P, 2>), grid, dim3(kWG), 0, st, a); break;
        case 4: hipLaunchKernelGGL((k_par_mov<P, 4>), grid, dim3(kWG), 0, st, a); break;
        default: hipLaunchKernelGGL((k_par_mov<P, 8>), grid, dim3(kWG), 0, st, a); break;
    }
}

int launch_par(bool fp64, int spl, const ParArgs &a, void *stream) {
    if (a.n_blocks <= 0 || a.s1 <= a.s0) return 0;
    if (a.ph.n_coils < 0 || a.ph.n_coils > 65535 || (a.ph.n_coils > 0 && (!a.ph.sre || !a.ph.sim))) return -1;
    dim3 grid((unsigned)a.n_blocks, (unsigned)((a.s1 - a.s0 + a.per_wg - 1) / a.per_wg),
              (unsigned)(a.ph.n_coils > 0 ? a.ph.n_coils : 1));
    // the vector-ALU kernels are instantiated for 1, 2, 4 and 8 tiles per
    // wavefront; the matrix-core ones take any number
    const bool pow2 = spl == 1 || spl == 2 || spl == 4 || spl == 8;
    if ((a.engine != 0 || a.ph.vx) && !pow2) return -1;
    if (spl < 1 || spl > 64) return -1;
    if (a.ph.vx) {  // moving spins (all three velocity arrays, checked on the host)
        if (!a.ph.vy || !a.ph.vz) return -1;
        if (fp64)
            par_dispatch_mov<FP64>(spl, grid, a, (hipStream_t)stream);
        else
            par_dispatch_mov<Mixed>(spl, grid, a, (hipStream_t)stream);
        return check_launch();
    }
    if (a.engine == 0) {
        if (fp64)
            par_dispatch_mm64(spl, grid, a, (hipStream_t)stream);
        else
            par_dispatch_mm(spl, grid, a, (hipStream_t)stream);
    } else if (fp64) {
        par_dispatch<FP64>(spl, grid, a, (hipStream_t)stream);
    } else {
        par_dispatch<Mixed>(spl, grid, a, (hipStream_t)stream);
    }
    return check_launch();
}

int launch_reduce(bool part_fp64, const ReduceArgs &a, void *stream) {
    if (a.cols <= 0 || a.n_groups <= 0) return 0;
    if (a.n_sig < 1 || a.n_sig > 65535) return -1;
    dim3 grid((unsigned)((a.cols + kWave - 1) / kWave), (unsigned)(a.n_groups < 65535 ? a.n_groups : 65535),
              (unsigned)a.n_sig);
    if (part_fp64)
        hipLaunchKernelGGL(k_reduce<double2>, grid, dim3(kWG), 0, (hipStream_t)stream, a);
    else
        hipLaunchKernelGGL(k_reduce<float2>, grid, dim3(kWG), 0, (hipStream_t)stream, a);
    return check_launch();
}

int launch_upload(const void *src, void *dst, size_t bytes, int32_t *zero, void *stream) {
    if (bytes == 0 && !zero) return 0;
    if ((bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return -1;
    const int64_t n = (int64_t)(bytes / 16);
    int64_t g = (n + kWG - 1) / kWG;
    if (g > 256) g = 256;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_upload, dim3((unsigned)g), dim3(kWG), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, n, zero);
    return check_launch();
}

int launch_validate(const PhantomDev &ph, int64_t n, int32_t *flags, void *stream) {
    if (n <= 0) return 0;
    dim3 grid((unsigned)((n + kWG - 1) / kWG));
    hipLaunchKernelGGL(k_validate, grid, dim3(kWG), 0, (hipStream_t)stream, ph, n, flags);
    return check_launch();
}

int launch_export(bool fp64, const Tile *tiles, int64_t n_tiles, const void *mxy, const void *mz,
                  double *m_final, const int32_t *gate, void *stream) {
    if (n_tiles <= 0) return 0;
    const int64_t n = n_tiles * kWave;
    dim3 grid((unsigned)((n + kWG - 1) / kWG));
    if (fp64)
        hipLaunchKernelGGL((k_export<double, double2>), grid, dim3(kWG), 0, (hipStream_t)stream, tiles,
                           n_tiles, (const double2 *)mxy, (const double *)mz, m_final, gate);
    else
        hipLaunchKernelGGL((k_export<float, float2>), grid, dim3(kWG), 0, (hipStream_t)stream, tiles,
                           n_tiles, (const float2 *)mxy, (const float *)mz, m_final, gate);
    return check_launch();
}

}  // namespace koma
