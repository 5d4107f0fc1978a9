// Sequence-aware time stepping (section "Simulation blocks, Regime Switching,
// and Sequence-Aware Time Stepping"): a block-structured sequence is turned
// into the discretised sequence the simulator integrates over, keeping only
// the time points the method needs:
//   - every vertex of every gradient waveform: with G piecewise linear, the
//     trapezoidal phase integral over an interval between vertices is exact;
//   - every boundary of every RF sample: with B1 piecewise constant, the
//     spinor rotation of each interval is exact (Eq. Rot_exc); a sample
//     longer than dt_rf_max is split evenly (the paper's Delta t_rf);
//   - every ADC sample time;
//   - every block boundary;
//   - outside RF samples, extra points so that no interval is longer than
//     dt_max (the paper's Delta t).
// Host code only; nothing here touches the device.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "komahip.h"

namespace koma {
void set_thread_error(const std::string &msg);
}

namespace {

// Points closer than this (seconds) are one point of the grid.
constexpr double kMergeTol = 1e-12;

struct Pt {
    double t;
    int adc;  // an ADC sample falls on this point
};

// Value of one gradient axis at block-local time u (piecewise linear).
double grad_at(const koma_grad &g, double u) {
    if (g.kind == KOMA_GRAD_TRAP) {
        const koma_trap &p = g.trap;
        double v = u - p.delay;
        if (v <= 0.0) return 0.0;
        if (v < p.rise) return p.amp * (v / p.rise);
        v -= p.rise;
        if (v <= p.flat) return p.amp;
        v -= p.flat;
        if (v < p.fall) return p.amp * (1.0 - v / p.fall);
        return 0.0;
    }
    if (g.kind == KOMA_GRAD_PWL) {
        const int64_t n = g.pwl_n;
        const double *tv = g.pwl_t, *av = g.pwl_amp;
        if (u < tv[0] - kMergeTol || u > tv[n - 1] + kMergeTol) return 0.0;
        int64_t i = (int64_t)(std::upper_bound(tv, tv + n, u) - tv) - 1;
        i = std::min<int64_t>(std::max<int64_t>(i, 0), n - 2);
        const double f = std::min(1.0, std::max(0.0, (u - tv[i]) / (tv[i + 1] - tv[i])));
        return av[i] + f * (av[i + 1] - av[i]);
    }
    return 0.0;
}

double grad_end(const koma_grad &g) {
    if (g.kind == KOMA_GRAD_TRAP) return g.trap.delay + g.trap.rise + g.trap.flat + g.trap.fall;
    if (g.kind == KOMA_GRAD_PWL) return g.pwl_t[g.pwl_n - 1];
    return 0.0;
}

// Value of a gradient axis at the start and at the end of its block.
double grad_first(const koma_grad &g) {
    return (g.kind == KOMA_GRAD_PWL && g.pwl_t[0] <= kMergeTol) ? g.pwl_amp[0] : 0.0;
}
double grad_last(const koma_grad &g, double duration) {
    return (g.kind == KOMA_GRAD_PWL && g.pwl_t[g.pwl_n - 1] >= duration - kMergeTol) ? g.pwl_amp[g.pwl_n - 1]
                                                                                     : 0.0;
}

bool pos(double x) { return std::isfinite(x) && x > 0.0; }
bool nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

koma_status fail(koma_status st, const std::string &msg) {
    koma::set_thread_error("koma_discretize: " + msg);
    return st;
}

koma_status check_block(const koma_block &B, int64_t b) {
    const std::string at = "block " + std::to_string(b) + ": ";
    const double end = B.duration * (1.0 + 1e-12);
    if (!pos(B.duration)) return fail(KOMA_E_SEQUENCE, at + "duration must be finite and > 0");
    for (int a = 0; a < 3; ++a) {
        const koma_grad &g = B.g[a];
        const std::string ax = at + "gradient " + "xyz"[a] + ": ";
        if (g.kind == KOMA_GRAD_TRAP) {
            const koma_trap &p = g.trap;
            if (!std::isfinite(p.amp) || !nonneg(p.delay) || !pos(p.rise) || !nonneg(p.flat) || !pos(p.fall))
                return fail(KOMA_E_SEQUENCE, ax + "trapezoid needs finite amp, delay >= 0, rise > 0, "
                                                  "flat >= 0, fall > 0");
        } else if (g.kind == KOMA_GRAD_PWL) {
            if (g.pwl_n < 2 || !g.pwl_t || !g.pwl_amp)
                return fail(KOMA_E_SEQUENCE, ax + "waveform needs at least 2 vertices");
            for (int64_t i = 0; i < g.pwl_n; ++i) {
                if (!std::isfinite(g.pwl_t[i]) || !std::isfinite(g.pwl_amp[i]))
                    return fail(KOMA_E_SEQUENCE, ax + "non-finite vertex");
                if (i > 0 && !(g.pwl_t[i] > g.pwl_t[i - 1]))
                    return fail(KOMA_E_SEQUENCE, ax + "vertex times must be strictly increasing");
            }
            if (g.pwl_t[0] < 0.0) return fail(KOMA_E_SEQUENCE, ax + "waveform starts before the block");
            if (g.pwl_t[0] > kMergeTol && g.pwl_amp[0] != 0.0)
                return fail(KOMA_E_SEQUENCE, ax + "a waveform that starts inside the block must start at 0");
            if (g.pwl_t[g.pwl_n - 1] < B.duration - kMergeTol && g.pwl_amp[g.pwl_n - 1] != 0.0)
                return fail(KOMA_E_SEQUENCE, ax + "a waveform that ends inside the block must end at 0");
        } else if (g.kind != KOMA_GRAD_NONE) {
            return fail(KOMA_E_ARG, ax + "unknown gradient kind");
        }
        if (grad_end(g) > end) return fail(KOMA_E_SEQUENCE, ax + "extends past the end of the block");
    }
    if (B.rf.n < 0) return fail(KOMA_E_SEQUENCE, at + "RF n < 0");
    if (B.rf.n > 0) {
        if (!B.rf.re || !B.rf.im || !pos(B.rf.dt) || !nonneg(B.rf.delay))
            return fail(KOMA_E_SEQUENCE, at + "RF needs re/im arrays, dt > 0, delay >= 0");
        for (int64_t i = 0; i < B.rf.n; ++i)
            if (!std::isfinite(B.rf.re[i]) || !std::isfinite(B.rf.im[i]))
                return fail(KOMA_E_SEQUENCE, at + "non-finite RF sample");
        if (B.rf.delay + B.rf.dt * (double)B.rf.n > end)
            return fail(KOMA_E_SEQUENCE, at + "RF extends past the end of the block");
    }
    if (B.adc.n < 0) return fail(KOMA_E_SEQUENCE, at + "ADC n < 0");
    if (B.adc.n > 0) {
        if (!nonneg(B.adc.delay) || !(B.adc.n == 1 ? nonneg(B.adc.dwell) : pos(B.adc.dwell)))
            return fail(KOMA_E_SEQUENCE, at + "ADC needs delay >= 0 and dwell > 0");
        if (B.adc.delay + B.adc.dwell * (double)(B.adc.n - 1) > end)
            return fail(KOMA_E_SEQUENCE, at + "ADC extends past the end of the block");
    }
    return KOMA_OK;
}

// Index of the block holding absolute time tm (a boundary belongs to the
// block that starts there; the end of the sequence to the last block).
int64_t block_of(const std::vector<double> &t0, double tm) {
    const int64_t nb = (int64_t)t0.size() - 1;
    const int64_t b = (int64_t)(std::upper_bound(t0.begin(), t0.end(), tm) - t0.begin()) - 1;
    return std::min<int64_t>(std::max<int64_t>(b, 0), nb - 1);
}

// RF sample in force at absolute time tm, if any.
bool rf_sample(const koma_block *blocks, const std::vector<double> &t0, double tm, double *re, double *im) {
    const int64_t b = block_of(t0, tm);
    const koma_rf &rf = blocks[b].rf;
    if (rf.n <= 0) return false;
    const double v = (tm - t0[b] - rf.delay) / rf.dt;
    if (!(v >= 0.0) || !(v < (double)rf.n)) return false;
    const int64_t i = std::min<int64_t>((int64_t)v, rf.n - 1);
    *re = rf.re[i];
    *im = rf.im[i];
    return true;
}

}  // namespace

extern "C" koma_status koma_discretize(const koma_block *blocks, int64_t n_blocks, double dt_max,
                                       double dt_rf_max, int64_t *n_t, int64_t *n_adc, double *t,
                                       double *gx, double *gy, double *gz, double *b1_re, double *b1_im,
                                       int64_t *adc_idx) {
    try {
        if (!blocks || n_blocks < 1 || !n_t || !n_adc) return fail(KOMA_E_ARG, "blocks, n_t and n_adc are required");
        if (!(dt_max > 0.0) || !(dt_rf_max > 0.0))
            return fail(KOMA_E_ARG, "dt_max and dt_rf_max must be > 0 (+inf: no subdivision)");
        for (int64_t b = 0; b < n_blocks; ++b) {
            const koma_status st = check_block(blocks[b], b);
            if (st != KOMA_OK) return st;
        }
        for (int64_t b = 0; b + 1 < n_blocks; ++b)
            for (int a = 0; a < 3; ++a) {
                const double e = grad_last(blocks[b].g[a], blocks[b].duration), f = grad_first(blocks[b + 1].g[a]);
                if (std::fabs(e - f) > 1e-9 * std::max(std::fabs(e), std::fabs(f)))
                    return fail(KOMA_E_SEQUENCE, "gradient " + std::string(1, "xyz"[a]) +
                                                     " is not continuous between blocks " + std::to_string(b) +
                                                     " and " + std::to_string(b + 1));
            }
        // block start times, accumulated in FP64
        std::vector<double> t0((size_t)n_blocks + 1, 0.0);
        for (int64_t b = 0; b < n_blocks; ++b) t0[b + 1] = t0[b] + blocks[b].duration;

        // ---- required points
        std::vector<Pt> pts;
        for (int64_t b = 0; b < n_blocks; ++b) {
            const koma_block &B = blocks[b];
            const double T = t0[b];
            pts.push_back({T, 0});
            for (int a = 0; a < 3; ++a) {
                const koma_grad &g = B.g[a];
                if (g.kind == KOMA_GRAD_TRAP) {
                    const koma_trap &p = g.trap;
                    const double v0 = T + p.delay, v1 = v0 + p.rise, v2 = v1 + p.flat, v3 = v2 + p.fall;
                    pts.insert(pts.end(), {{v0, 0}, {v1, 0}, {v2, 0}, {v3, 0}});
                } else if (g.kind == KOMA_GRAD_PWL) {
                    for (int64_t i = 0; i < g.pwl_n; ++i) pts.push_back({T + g.pwl_t[i], 0});
                }
            }
            if (B.rf.n > 0) {
                const int64_t sub = std::isfinite(dt_rf_max)
                                        ? std::max<int64_t>(1, (int64_t)std::ceil((B.rf.dt - kMergeTol) / dt_rf_max))
                                        : 1;
                for (int64_t i = 0; i < B.rf.n; ++i)
                    for (int64_t k = 0; k < sub; ++k)
                        pts.push_back({T + B.rf.delay + B.rf.dt * ((double)i + (double)k / (double)sub), 0});
                pts.push_back({T + B.rf.delay + B.rf.dt * (double)B.rf.n, 0});
            }
            for (int64_t i = 0; i < B.adc.n; ++i) pts.push_back({T + B.adc.delay + B.adc.dwell * (double)i, 1});
        }
        pts.push_back({t0[n_blocks], 0});
        std::stable_sort(pts.begin(), pts.end(), [](const Pt &x, const Pt &y) { return x.t < y.t; });
        std::vector<Pt> u;
        u.reserve(pts.size());
        for (const Pt &p : pts) {
            if (!u.empty() && p.t - u.back().t <= kMergeTol) {
                if (p.adc && u.back().adc)
                    return fail(KOMA_E_SEQUENCE, "two ADC samples within 1 ps of each other");
                u.back().adc |= p.adc;
            } else {
                u.push_back(p);
            }
        }
        // ---- optional intermediate points outside RF samples
        std::vector<Pt> w;
        w.reserve(u.size());
        for (size_t i = 0; i < u.size(); ++i) {
            w.push_back(u[i]);
            if (i + 1 == u.size() || !std::isfinite(dt_max)) continue;
            const double a = u[i].t, b = u[i + 1].t;
            double re, im;
            if (b - a > dt_max && !rf_sample(blocks, t0, 0.5 * (a + b), &re, &im)) {
                // an interval within the grid's time resolution of dt_max is not split
                const int64_t k = (int64_t)std::ceil((b - a - kMergeTol) / dt_max);
                for (int64_t j = 1; j < k; ++j) w.push_back({a + (b - a) * ((double)j / (double)k), 0});
            }
        }
        int64_t na = 0;
        for (const Pt &p : w) na += p.adc;
        const int64_t nt = (int64_t)w.size();
        if (!t) {  // size query
            *n_t = nt;
            *n_adc = na;
            return KOMA_OK;
        }
        if (*n_t < nt || *n_adc < na) return fail(KOMA_E_ARG, "output arrays are too small");
        if (!gx || !gy || !gz || !b1_re || !b1_im || (na > 0 && !adc_idx))
            return fail(KOMA_E_ARG, "output arrays are required");
        // ---- values: G at every point, B1 of the RF sample holding each interval's midpoint
        int64_t k = 0;
        for (int64_t i = 0; i < nt; ++i) {
            const double tm = w[i].t;
            const int64_t b = block_of(t0, tm);
            const double loc = tm - t0[b];
            t[i] = tm;
            gx[i] = grad_at(blocks[b].g[0], loc);
            gy[i] = grad_at(blocks[b].g[1], loc);
            gz[i] = grad_at(blocks[b].g[2], loc);
            if (w[i].adc) adc_idx[k++] = i;
            if (i + 1 < nt) {
                double re = 0.0, im = 0.0;
                if (!rf_sample(blocks, t0, 0.5 * (tm + w[i + 1].t), &re, &im)) re = im = 0.0;
                b1_re[i] = re;
                b1_im[i] = im;
            }
        }
        *n_t = nt;
        *n_adc = na;
        return KOMA_OK;
    } catch (const std::bad_alloc &) {
        return fail(KOMA_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(KOMA_E_ARG, "unexpected failure");
    }
}
