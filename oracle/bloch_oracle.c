/*
 * Plain FP64 CPU oracle of the KomaMRI Bloch simulation (arXiv 2301.02702).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or helper with the GPU library, and neither uses the other.
 *
 * What it computes (section "Physical and Mathematical Background"):
 *   For every spin (spins are independent; same section, statement after the
 *   effective-field equation), start from thermal equilibrium
 *   M = (Mxy = 0, Mz = M0) and, for every interval [t_n, t_{n+1}] of the
 *   discretised sequence, apply the first-order operator splitting:
 *     1. rotation about the effective field
 *          B = (B1x, B1y, G.x + dw/gamma)                       (Eq. B-def)
 *        - excitation regime (B1 != 0): spinor (Cayley-Klein) rotation with
 *          n = B/|B|, phi = -gamma |B| dt                     (Eq. angle_precession)
 *          alpha = cos(phi/2) - i n_z sin(phi/2), beta = -i n_xy sin(phi/2),
 *          Mxy+ = 2 conj(alpha) beta Mz + conj(alpha)^2 Mxy - beta^2 conj(Mxy)
 *          Mz+  = (|alpha|^2 - |beta|^2) Mz - 2 Re(alpha beta conj(Mxy))   (Eq. Rot_exc)
 *        - precession regime (B1 = 0): Mxy+ = Mxy exp(i phi) with the
 *          trapezoidal phase phi = -gamma (x . (G_n + G_{n+1})/2 + dw/gamma) dt
 *          (Eq. Rotation_precession; section "Simulation blocks, Regime
 *          Switching, and Sequence-Aware Time Stepping": exact for a
 *          piecewise-linear G)
 *     2. relaxation: Mxy+ = exp(-dt/T2) Mxy,
 *        Mz+ = Mz exp(-dt/T1) + M0 (1 - exp(-dt/T1))            (relaxation update)
 *   and whenever t_{n+1} is an ADC point add Mxy to that sample of the spin's
 *   signal group (Figure 3, the simulation pipeline: the signal contributions are
 *   added into sig[t]). An ADC point at index 0 samples the initial state.
 *
 * Two modes, both from the paper:
 *   mode 0 (per interval): the splitting above on every interval.
 *   mode 1 (precession blocks): a maximal run of consecutive B1 = 0 intervals
 *     is one precession block; its phase is the integral of Bz over the block
 *     (the sum of the per-interval trapezoid phases) and its relaxation is the
 *     relaxation update over the elapsed block time. ADC points inside a block
 *     are evaluated from the block's start state with the phase and elapsed
 *     time accumulated so far. Excitation intervals are as in mode 0.
 *
 * Motion (section "Overview": the phantom's displacement field u(x, t); the
 * section on sequence-aware time stepping: with motion, intermediate points
 * are needed): a spin with velocity v sits at x(t) = x + v t, t the
 * sequence's own time. Its field is taken at the grid points with the
 * position updated to each point, Bz(t_n) = G_n . x(t_n) + dw/gamma, and an
 * interval's field is the mean of its two end values (the trapezoidal rule
 * the precession phase uses; for v = 0 the static formula above).
 *
 * Receive coils (section "Overview": coil sensitivities as scanner
 * properties; section "Limitations": multiple coils): with n_coils >= 1 every
 * spin carries one complex sensitivity per coil, and coil c's signal is the
 * sum over a group's spins of sens_c * Mxy. n_coils = 0 is the plain sum.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   initial state (0, 0, M0); B1 per interval and G as the interval mean;
 *   regime chosen per interval by B1 != 0 exactly; rotation then relaxation
 *   (no symmetrisation); the signal is the plain sum of Mxy over a group's
 *   spins; T = +inf means no relaxation; a moving spin's field per interval
 *   is the mean of its end-point values; a coil sensitivity is fixed per
 *   spin (it does not follow the motion) and multiplies Mxy unconjugated.
 *
 * Parallelism is the paper's CPU scheme: static contiguous spin ranges per
 * thread, one signal matrix per thread, added in thread order at the end.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ---- single-step operators (also exported for unit tests) -------------- */

/* Excitation-regime rotation about B = (Re b1, Im b1, bz) over dt. */
static void excite(double gamma, cplx b1, double bz, double dt, cplx *mxy, double *mz)
{
    double nrm = sqrt(creal(b1) * creal(b1) + cimag(b1) * cimag(b1) + bz * bz);
    if (nrm == 0.0)
        return; /* no field: identity rotation */
    double phi = -gamma * nrm * dt;
    cplx nxy = b1 / nrm;
    double nz = bz / nrm;
    cplx alpha = cos(phi / 2) - I * nz * sin(phi / 2);
    cplx beta = -I * nxy * sin(phi / 2);
    cplx m = *mxy;
    double z = *mz;
    cplx mxy_new = 2.0 * conj(alpha) * beta * z + conj(alpha) * conj(alpha) * m - beta * beta * conj(m);
    double mz_new = (creal(alpha * conj(alpha)) - creal(beta * conj(beta))) * z
                    - 2.0 * creal(alpha * beta * conj(m));
    *mxy = mxy_new;
    *mz = mz_new;
}

/* Relaxation over dt. */
static void relax(double dt, double t1, double t2, double m0, cplx *mxy, double *mz)
{
    double e1 = exp(-dt / t1);
    double e2 = exp(-dt / t2);
    *mxy = e2 * (*mxy);
    *mz = (*mz) * e1 + m0 * (1.0 - e1);
}

void oracle_excite_step(double gamma, const double m_in[3], double b1_re, double b1_im,
                        double bz, double dt, double m_out[3])
{
    cplx mxy = m_in[0] + I * m_in[1];
    double mz = m_in[2];
    excite(gamma, b1_re + I * b1_im, bz, dt, &mxy, &mz);
    m_out[0] = creal(mxy);
    m_out[1] = cimag(mxy);
    m_out[2] = mz;
}

void oracle_relax_step(double dt, double t1, double t2, double m0, const double m_in[3],
                       double m_out[3])
{
    cplx mxy = m_in[0] + I * m_in[1];
    double mz = m_in[2];
    relax(dt, t1, t2, m0, &mxy, &mz);
    m_out[0] = creal(mxy);
    m_out[1] = cimag(mxy);
    m_out[2] = mz;
}

/* ---- whole simulation ---------------------------------------------------- */

typedef struct {
    double gamma;
    int64_t n_t;
    const double *t, *gx, *gy, *gz, *b1re, *b1im;
    int64_t n_adc;
    const int64_t *adc_idx;
    int mode;
    /* spins */
    const float *x, *y, *z, *pd, *t1, *t2, *dw;
    const float *vx, *vy, *vz; /* NULL: static spins */
    int64_t n_coils;           /* 0: plain sum */
    const float *sens_re, *sens_im; /* [n_coils][n] */
    int64_t n_spins;
    const int64_t *group_off; /* n_groups + 1 */
    int64_t n_groups;
    double *m_final;
} problem;

typedef struct {
    const problem *p;
    int64_t s0, s1;   /* spin range */
    int64_t g0, g1;   /* groups touched: [g0, g1] */
    cplx *part;       /* [max(n_coils, 1)][g1 - g0 + 1][n_adc] */
    cplx *row;        /* one spin's signal, [n_adc] */
} job;

static int64_t group_of(const problem *p, int64_t s)
{
    /* largest g with group_off[g] <= s */
    int64_t lo = 0, hi = p->n_groups - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (p->group_off[mid] <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/* z field of spin s over interval n (T): the interval-mean gradient times the
 * position for a static spin; for a moving spin the mean of the end-point
 * fields with the position updated to each end point. */
static double interval_bz(const problem *p, int64_t s, int64_t n)
{
    const double x = p->x[s], y = p->y[s], z = p->z[s];
    const double dw = p->dw[s];
    if (!p->vx) {
        double gbx = 0.5 * (p->gx[n] + p->gx[n + 1]);
        double gby = 0.5 * (p->gy[n] + p->gy[n + 1]);
        double gbz = 0.5 * (p->gz[n] + p->gz[n + 1]);
        return x * gbx + y * gby + z * gbz + dw / p->gamma;
    }
    const double vx = p->vx[s], vy = p->vy[s], vz = p->vz[s];
    const double ta = p->t[n], tb = p->t[n + 1];
    double bza = p->gx[n] * (x + vx * ta) + p->gy[n] * (y + vy * ta) + p->gz[n] * (z + vz * ta);
    double bzb = p->gx[n + 1] * (x + vx * tb) + p->gy[n + 1] * (y + vy * tb) + p->gz[n + 1] * (z + vz * tb);
    return 0.5 * (bza + bzb) + dw / p->gamma;
}

static void simulate_spin(const problem *p, int64_t s, cplx *row)
{
    const double gamma = p->gamma;
    const double m0 = p->pd[s], t1 = p->t1[s], t2 = p->t2[s];
    const int64_t n_int = p->n_t - 1;
    cplx mxy = 0.0;
    double mz = m0;
    int64_t k = 0; /* next ADC sample */

    if (k < p->n_adc && p->adc_idx[k] == 0)
        row[k++] += mxy;

    int64_t n = 0;
    while (n < n_int) {
        double dt = p->t[n + 1] - p->t[n];
        double bz = interval_bz(p, s, n);
        cplx b1 = p->b1re[n] + I * p->b1im[n];
        if (b1 != 0.0) {
            excite(gamma, b1, bz, dt, &mxy, &mz);
            relax(dt, t1, t2, m0, &mxy, &mz);
            n++;
            if (k < p->n_adc && p->adc_idx[k] == n)
                row[k++] += mxy;
        } else if (p->mode == 0) {
            double phi = -gamma * bz * dt;
            mxy = mxy * cexp(I * phi);
            relax(dt, t1, t2, m0, &mxy, &mz);
            n++;
            if (k < p->n_adc && p->adc_idx[k] == n)
                row[k++] += mxy;
        } else {
            /* precession block: integral phase and elapsed time from its start */
            cplx mxy_a = mxy;
            double mz_a = mz;
            double phi = 0.0, tau = 0.0;
            while (n < n_int && p->b1re[n] == 0.0 && p->b1im[n] == 0.0) {
                double dtn = p->t[n + 1] - p->t[n];
                double bzn = interval_bz(p, s, n);
                phi += -gamma * bzn * dtn;
                tau += dtn;
                n++;
                if (k < p->n_adc && p->adc_idx[k] == n) {
                    cplx m = mxy_a * cexp(I * phi);
                    double mzt = mz_a;
                    relax(tau, t1, t2, m0, &m, &mzt);
                    row[k++] += m;
                }
            }
            mxy = mxy_a * cexp(I * phi);
            mz = mz_a;
            relax(tau, t1, t2, m0, &mxy, &mz);
        }
    }
    if (p->m_final) {
        p->m_final[3 * s + 0] = creal(mxy);
        p->m_final[3 * s + 1] = cimag(mxy);
        p->m_final[3 * s + 2] = mz;
    }
}

static void *run_job(void *arg)
{
    job *j = (job *)arg;
    const problem *p = j->p;
    const int64_t ng = j->g1 - j->g0 + 1;
    for (int64_t s = j->s0; s < j->s1; s++) {
        int64_t g = group_of(p, s);
        if (p->n_coils == 0) {
            simulate_spin(p, s, j->part + (g - j->g0) * p->n_adc);
            continue;
        }
        /* one spin's Mxy at every sample, then weighted into every coil */
        memset(j->row, 0, sizeof(cplx) * (size_t)p->n_adc);
        simulate_spin(p, s, j->row);
        for (int64_t c = 0; c < p->n_coils; c++) {
            cplx sens = p->sens_re[c * p->n_spins + s] + I * p->sens_im[c * p->n_spins + s];
            cplx *dst = j->part + (c * ng + (g - j->g0)) * p->n_adc;
            for (int64_t k = 0; k < p->n_adc; k++)
                dst[k] += sens * j->row[k];
        }
    }
    return NULL;
}

/*
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * vx, vy, vz: NULL (static spins) or velocities in m/s.
 * n_coils: 0 (plain sum) or the number of coils; sens_re, sens_im: [n_coils][n].
 * sig: [max(n_coils, 1)][n_groups][n_adc] complex as interleaved (re, im)
 *      doubles, overwritten.
 * m_final: NULL or [n][3] (Mx, My, Mz).
 * group_off: NULL for one group, else n_groups + 1 ascending offsets from 0 to n.
 */
int oracle_simulate(double gamma, int64_t n, const float *x, const float *y, const float *z,
                    const float *pd, const float *t1, const float *t2, const float *dw,
                    const float *vx, const float *vy, const float *vz, int64_t n_coils,
                    const float *sens_re, const float *sens_im,
                    int64_t n_groups, const int64_t *group_off, int64_t n_t, const double *t,
                    const double *gx, const double *gy, const double *gz, const double *b1_re,
                    const double *b1_im, int64_t n_adc, const int64_t *adc_idx, int mode,
                    int n_threads, double *sig, double *m_final)
{
    if (n < 0 || n_t < 2 || n_adc < 0 || n_groups < 1 || (mode != 0 && mode != 1))
        return -1;
    if ((vx || vy || vz) && !(vx && vy && vz))
        return -1;
    if (n_coils < 0 || (n_coils > 0 && (!sens_re || !sens_im)))
        return -1;
    const int64_t n_sig = n_coils > 0 ? n_coils : 1;
    int64_t one_group[2] = {0, n};
    if (!group_off) {
        if (n_groups != 1)
            return -1;
        group_off = one_group;
    }
    if (group_off[0] != 0 || group_off[n_groups] != n)
        return -1;
    problem p = {gamma, n_t, t, gx, gy, gz, b1_re, b1_im, n_adc, adc_idx, mode,
                 x, y, z, pd, t1, t2, dw, vx, vy, vz, n_coils, sens_re, sens_im, n,
                 group_off, n_groups, m_final};
    memset(sig, 0, sizeof(double) * 2 * (size_t)n_sig * (size_t)n_groups * (size_t)n_adc);
    if (n == 0)
        return 0;
    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > n)
        n_threads = (int)n;

    job *jobs = calloc((size_t)n_threads, sizeof(job));
    pthread_t *th = calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    int rc = 0;
    for (int i = 0; i < n_threads; i++) {
        jobs[i].p = &p;
        jobs[i].s0 = n * i / n_threads;
        jobs[i].s1 = n * (i + 1) / n_threads;
        jobs[i].g0 = group_of(&p, jobs[i].s0);
        jobs[i].g1 = group_of(&p, jobs[i].s1 - 1);
        size_t len = (size_t)n_sig * (size_t)(jobs[i].g1 - jobs[i].g0 + 1) * (size_t)(n_adc > 0 ? n_adc : 1);
        jobs[i].part = calloc(len, sizeof(cplx));
        jobs[i].row = calloc((size_t)(n_adc > 0 ? n_adc : 1), sizeof(cplx));
        if (!jobs[i].part || !jobs[i].row)
            rc = -2;
    }
    if (rc == 0) {
        for (int i = 0; i < n_threads; i++)
            pthread_create(&th[i], NULL, run_job, &jobs[i]);
        for (int i = 0; i < n_threads; i++)
            pthread_join(th[i], NULL);
        /* per-thread signals added in thread order */
        for (int i = 0; i < n_threads; i++) {
            const int64_t ng = jobs[i].g1 - jobs[i].g0 + 1;
            for (int64_t c = 0; c < n_sig; c++) {
                for (int64_t g = jobs[i].g0; g <= jobs[i].g1; g++) {
                    const cplx *src = jobs[i].part + (c * ng + (g - jobs[i].g0)) * n_adc;
                    double *dst = sig + 2 * (c * n_groups + g) * n_adc;
                    for (int64_t k = 0; k < n_adc; k++) {
                        dst[2 * k] += creal(src[k]);
                        dst[2 * k + 1] += cimag(src[k]);
                    }
                }
            }
        }
    }
    for (int i = 0; i < n_threads; i++) {
        free(jobs[i].part);
        free(jobs[i].row);
    }
    free(jobs);
    free(th);
    return rc;
}
