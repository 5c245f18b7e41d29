/*
 * oracle.c -- plain, slow FP64 reference of the spiking-network hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file.  It exists so that tests, the smoke check and the
 * CPU-baseline leg of the benchmark can compare the HIP implementation with
 * an implementation that follows the paper step by step.  It shares no code,
 * header, table or constant with the HIP library.
 *
 * Paper: Pastorelli et al., "Gaussian and exponential lateral connectivity on
 * distributed spiking neural network simulation" (PDP 2018).
 *
 * What is computed, and where it comes from:
 *   - a 2-D grid of cortical modules of excitatory and inhibitory point
 *     neurons (Sec. III.B);
 *   - distance-dependent connection probabilities from the Gaussian law
 *     B*exp(-r^2/2 sigma^2) and the exponential law A*exp(-r/lambda), where
 *     the prefactor fixes the total number of connections (Sec. I, Sec. III.B);
 *   - per-neuron synapse projections with individual target, delay and weight
 *     (Sec. II.B), weights Gaussian for excitatory sources, delays uniform;
 *   - external (thalamo-cortical) drive as a Poisson process (Sec. III.A);
 *   - leaky integrate-and-fire neurons with spike-frequency adaptation,
 *     Eq. (1) and Eq. (2), threshold, reset and absolute refractory period
 *     (Sec. III.A), instantaneous (delta) synapses;
 *   - the 1 ms time-driven step: find spikers, send spikes, queue them by
 *     delay, inject charge at arrival, integrate (Sec. II.A);
 *   - counting of recurrent and external synaptic events (Sec. III.D);
 *   - optionally, the exact-time event-driven solver (Sec. II.A, Sec. II.C):
 *     spikes carry their emission time inside the step, each neuron takes its
 *     queued and external inputs in time order and integrates Eq. (1)-(2)
 *     exactly between them.
 *
 * Readings of points where the paper is silent or ambiguous are listed in the
 * design document; the ones that change arithmetic are repeated next to the
 * code below.  Floating point is FP64 throughout; integer work (connectivity,
 * fixed-point charge, delivery) is exact.
 *
 * Parity pins: Philox4x32-10 is checked against an independent library
 * implementation; tables against closed forms and library distributions;
 * the neuron map against closed-form interspike intervals; connectivity
 * against its expected in-degree and distance statistics; delivery against
 * a dense brute-force simulation and exact charge conservation.  The
 * exact-time solver against the step solver (to which it reduces when every
 * input arrives at offset 0), closed-form superposition of sub-threshold
 * inputs, closed-form spike times of isolated neurons, and causality of
 * every spike of a recurrent network.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_NOMEM (-2)
#define OR_E_OVERFLOW (-5)

#define OR_GAUSS 0
#define OR_EXP 1
#define OR_REC_F32 0
#define OR_REC_CODE8 1
#define OR_EXT_POISSON 0
#define OR_EXT_CONST 1
#define OR_PRESET_LATERAL 0
#define OR_PRESET_PAPER 1

#define RING 32            /* delay ring slots: must exceed the largest delay */
#define POIS_MAX 64        /* longest Poisson CDF threshold table            */

/* Philox stream identifiers (third counter word). */
#define ST_CONN 1u
#define ST_ATTR 2u
#define ST_EXT 3u
#define ST_INIT 4u
#define ST_COUNT 5u        /* binomial generator: synapse count per (source, module) */
#define ST_PICK 6u         /* binomial generator: Floyd's draws                     */

#define OR_GEN_PAIRWISE 0
#define OR_GEN_BINOMIAL 1
#define BINOM_MAX_M 4096   /* binomial generator: largest module               */
#define OR_DELAY_UNIFORM 0
#define OR_DELAY_EXP 1
#define OR_SOLVER_STEP 0   /* charge summed per 1 ms step, one jump per step   */
#define OR_SOLVER_EXACT 1  /* exact-time event-driven integration              */
#define ST_EXT_TIME 7u     /* exact solver: arrival times of external events    */
#define STDP_WIN_MAX 256   /* longest plasticity window, steps                  */

/* Flat description of one network.  Times in ms, potentials in mV. */
typedef struct {
    uint32_t gx, gy, n_exc, n_inh;
    uint32_t periodic;
    double tau_m, v_th, v_reset, e_rest, t_ref, alpha_w, tau_w;
    uint32_t sfa_on_inh;
    uint64_t seed;
    uint32_t kernel;          /* OR_GAUSS / OR_EXP                            */
    double range;             /* sigma or lambda, in module spacings          */
    double k_in;              /* expected number of recurrent synapses/neuron */
    uint32_t d_min, d_max;    /* integer delays in ms                         */
    double w_exc, w_exc_sd, w_inh;
    uint32_t record;          /* OR_REC_F32 / OR_REC_CODE8                    */
    uint32_t ext_mode;        /* OR_EXT_POISSON / OR_EXT_CONST                */
    double ext_n, ext_rate_hz, ext_w;
    int32_t ext_const_q;      /* charge per step in const mode (2^-16 mV)    */
    uint32_t pad_;
    uint32_t preset;          /* OR_PRESET_LATERAL / OR_PRESET_PAPER          */
    uint32_t pad2_;
    double p_local;           /* paper preset: probability inside a module    */
    double amp;               /* paper preset: remote law amplitude A         */
    double p_cut;             /* paper preset: stencil cut-off probability    */
    uint32_t gen;             /* OR_GEN_PAIRWISE / OR_GEN_BINOMIAL            */
    uint32_t delay_dist;      /* OR_DELAY_UNIFORM / OR_DELAY_EXP              */
    double delay_tau;         /* exponential delays: scale (ms)               */
    uint32_t solver;          /* OR_SOLVER_STEP / OR_SOLVER_EXACT             */
    uint32_t pad3_;
    uint32_t stdp;            /* 1: spike-timing plasticity of excitatory synapses */
    uint32_t ltp_period;      /* steps between long-term applications (1000 = 1 s) */
    double a_plus, a_minus;   /* pair amplitudes at zero lag (mV)             */
    double tau_plus, tau_minus; /* window time constants (ms)                 */
    double w_max;             /* upper bound of a plastic weight (mV)         */
} or_cfg;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and   */
/* Shaw (SC'11): ten rounds of two 32x32->64 multiplications, with the      */
/* key advanced by the Weyl constants between rounds.                       */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_draw(uint64_t seed, uint32_t a, uint32_t b, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {a, b, stream, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Standard normal helpers (used only to build the weight tables).          */
/* ------------------------------------------------------------------------ */
static double norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }
/* 2.5066282746310002 is sqrt(2 pi) rounded to double */
static double norm_pdf(double x) { return exp(-0.5 * x * x) / 2.5066282746310002; }

/* Inverse normal CDF by plain bisection on norm_cdf. */
static double norm_quantile(double u)
{
    if (u <= 0.0) return -INFINITY;
    if (u >= 1.0) return INFINITY;
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 400; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (norm_cdf(mid) < u) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Mean of Z ~ N(0,1) restricted to the quantile interval [ua, ub):
 * (phi(a) - phi(b)) / (ub - ua). */
static double norm_bin_mean(double ua, double ub)
{
    double a = norm_quantile(ua), b = norm_quantile(ub);
    double pa = isinf(a) ? 0.0 : norm_pdf(a);
    double pb = isinf(b) ? 0.0 : norm_pdf(b);
    return (pa - pb) / (ub - ua);
}

static int32_t fixq(double mv) { return (int32_t)nearbyint(mv * 65536.0); }

/* ------------------------------------------------------------------------ */
/* Tables                                                                   */
/* ------------------------------------------------------------------------ */
/* Binomial count table of one (source type, offset): thresholds of counts
 * k0 .. k0 + len - 1 at thr[at ..]; counts below k0 have threshold 0. */
typedef struct {
    uint32_t k0, len;
    size_t at;
} or_binom;

typedef struct {
    uint32_t *T;            /* [2][gy*gx] connection thresholds per torus offset,
                               for excitatory (0) and inhibitory (1) sources    */
    uint32_t dthr[RING];    /* exponential delays: CDF thresholds of the bucket */
    or_binom *bt;           /* binomial generator: [2][gy*gx] count tables      */
    uint32_t *bthr;         /* their thresholds                                 */
    int32_t wtab[65536];    /* excitatory weight by top 16 bits of the draw   */
    int32_t cb[256];        /* 8-bit weight codebook                          */
    uint32_t poisc[POIS_MAX];
    uint32_t npois;
    double dm, dw, kappa;   /* one-step propagator constants                  */
    uint32_t nref;          /* refractory steps                               */
    int32_t jext_q, winh_q;
    /* plasticity: weight change of one pair at lag k steps, 2^-16 mV */
    int32_t kp[STDP_WIN_MAX];   /* potentiation, post k >= 0 steps after the arrival */
    int32_t km[STDP_WIN_MAX];   /* depression, arrival k >= 1 steps after the post spike */
    uint32_t win;               /* lags below win count                              */
    int32_t wmax_q;
} or_tables;

static uint32_t module_size(const or_cfg *c) { return c->n_exc + c->n_inh; }

/* Signed torus offset of a raw difference in [0, g): mapped to (-g/2, g/2]. */
static int torus_off(int raw, int g) { return (2 * raw <= g) ? raw : raw - g; }

/* Distance law, Sec. I and Sec. III.B: Gaussian exp(-r^2 / 2 sigma^2) or
 * exponential exp(-r / lambda), r in module spacings. */
static double law(const or_cfg *c, int r2)
{
    if (c->kernel == OR_GAUSS) return exp(-(double)r2 / (2.0 * c->range * c->range));
    return exp(-sqrt((double)r2) / c->range);
}

/* Connection thresholds, stored as round(p * 2^32) per torus offset and
 * source type.
 *
 * Lateral preset (one law for every pair): the prefactor B fixes the expected
 * number of recurrent synapses per neuron to k_in (Sec. I: "fixes the
 * total"): B = k_in / sum_off n(off) f(r_off), with n = module size for a
 * remote offset and module size - 1 for the own module (no self-connection);
 * p = B f(r) for both source types.
 *
 * Paper preset (Sec. III.B, the two lateral rules and the Fig. 2 caption):
 * every neuron connects inside its own module with probability p_local;
 * excitatory neurons also project to other modules with probability
 * amp * f(r); inhibitory neurons project only locally.  Remote projection is
 * cut off where the probability falls to p_cut, which the paper states as
 * square stencils centred on the source (7x7 Gaussian, 21x21 exponential):
 * read as the square of half-width ceil(r_c), r_c the distance at which
 * amp * f(r_c) = p_cut. */
static int stencil_half_width(const or_cfg *c)
{
    if (!(c->amp > c->p_cut)) return 0;
    double rc = (c->kernel == OR_GAUSS) ? c->range * sqrt(2.0 * log(c->amp / c->p_cut))
                                        : c->range * log(c->amp / c->p_cut);
    return (int)ceil(rc);
}

static int put_threshold(double p, uint32_t *dst)
{
    double q = nearbyint(p * 4294967296.0);
    if (!(q >= 0.0 && q < 4294967296.0)) return OR_E_INVAL;
    *dst = (uint32_t)q;
    return OR_OK;
}

static int make_thresholds(const or_cfg *c, uint32_t *T)
{
    int gx = (int)c->gx, gy = (int)c->gy;
    size_t S = (size_t)gx * gy;
    if (c->preset == OR_PRESET_PAPER) {
        int h = stencil_half_width(c);
        for (int dyr = 0; dyr < gy; dyr++)
            for (int dxr = 0; dxr < gx; dxr++) {
                int dx = torus_off(dxr, gx), dy = torus_off(dyr, gy);
                double pe = 0.0, pi = 0.0;
                if (dxr == 0 && dyr == 0) {
                    pe = pi = c->p_local;
                } else if (abs(dx) <= h && abs(dy) <= h) {
                    pe = c->amp * law(c, dx * dx + dy * dy);
                }
                if (put_threshold(pe, &T[dyr * gx + dxr]) || put_threshold(pi, &T[S + dyr * gx + dxr]))
                    return OR_E_INVAL;
            }
        return OR_OK;
    }
    double M = (double)module_size(c);
    double s = 0.0;
    for (int dyr = 0; dyr < gy; dyr++)
        for (int dxr = 0; dxr < gx; dxr++) {
            int dx = torus_off(dxr, gx), dy = torus_off(dyr, gy);
            double n = (dxr == 0 && dyr == 0) ? M - 1.0 : M;
            s += n * law(c, dx * dx + dy * dy);
        }
    double B = (c->k_in > 0.0) ? c->k_in / s : 0.0;
    for (int dyr = 0; dyr < gy; dyr++)
        for (int dxr = 0; dxr < gx; dxr++) {
            int dx = torus_off(dxr, gx), dy = torus_off(dyr, gy);
            if (put_threshold(B * law(c, dx * dx + dy * dy), &T[dyr * gx + dxr])) return OR_E_INVAL;
            T[S + dyr * gx + dxr] = T[dyr * gx + dxr];
        }
    return OR_OK;
}

/* Excitatory weights: Gaussian efficacies (Sec. II.B), realised as the
 * conditional mean of each of 65536 equiprobable bins of N(mu, sd^2),
 * in fixed point with 2^-16 mV resolution. */
static void make_wtab(const or_cfg *c, int32_t *wtab)
{
    for (int k = 0; k < 65536; k++) {
        double e = norm_bin_mean((double)k / 65536.0, (double)(k + 1) / 65536.0);
        wtab[k] = fixq(c->w_exc + c->w_exc_sd * e);
    }
}

/* 8-bit codebook: codes 0..254 are the conditional means of the bins
 * selected by floor(u * 255 / 2^32) of the same draw; code 255 is the
 * inhibitory weight. */
static void make_codebook(const or_cfg *c, int32_t *cb)
{
    for (int k = 0; k < 255; k++) {
        /* smallest u with floor(u*255/2^32) == k is ceil(k * 2^32 / 255) */
        uint64_t e0 = ((uint64_t)k * 4294967296ull + 254u) / 255u;
        uint64_t e1 = ((uint64_t)(k + 1) * 4294967296ull + 254u) / 255u;
        double e = norm_bin_mean((double)e0 / 4294967296.0, (double)e1 / 4294967296.0);
        cb[k] = fixq(c->w_exc + c->w_exc_sd * e);
    }
    cb[255] = fixq(c->w_inh);
}

/* External Poisson drive (Sec. III.A): mean count per 1 ms step is
 * ext_n * rate * 1e-3.  CDF thresholds round(2^32 F(k)) are kept while
 * below 2^32; the count is the number of thresholds not above the draw. */
static int make_poisson(const or_cfg *c, uint32_t *poisc, uint32_t *npois)
{
    double m = c->ext_n * c->ext_rate_hz * 1e-3;
    double term = exp(-m), F = term;
    uint32_t n = 0;
    for (int k = 0; k < POIS_MAX; k++) {
        if (k > 0) { term *= m / (double)k; F += term; }
        double q = nearbyint(F * 4294967296.0);
        if (!(q < 4294967296.0)) { *npois = n; return OR_OK; }
        poisc[n++] = (uint32_t)q;
    }
    return OR_E_INVAL; /* distribution not exhausted within the table */
}

/* Binomial generator (the exact-distribution alternative to one trial per
 * pair): for a source and a target module with n candidates and pair
 * probability p = T / 2^32, the number of synapses is Binomial(n, p), drawn
 * by integer CDF thresholds round(2^32 F(k)), F summed in increasing k from
 * pmf(k) = exp(lgamma(n+1) - lgamma(k+1) - lgamma(n-k+1) + k log p +
 * (n-k) log1p(-p)); counts whose threshold rounds to 2^32 are never drawn. */
static int make_binomial(const or_cfg *c, or_tables *tb)
{
    size_t S = (size_t)c->gx * c->gy, cap = 4096, used = 0;
    uint32_t M = module_size(c);
    tb->bt = (or_binom *)calloc(2 * S, sizeof(or_binom));
    tb->bthr = (uint32_t *)malloc(cap * sizeof(uint32_t));
    if (!tb->bt || !tb->bthr) return OR_E_NOMEM;
    for (size_t e = 0; e < 2 * S; e++) {
        uint32_t T = tb->T[e];
        tb->bt[e].at = used;
        if (T == 0) continue;
        uint32_t n = (e % S == 0) ? M - 1 : M;
        double p = (double)T / 4294967296.0;
        double lp = log(p), lq = log1p(-p), ln = lgamma((double)n + 1.0), F = 0.0;
        uint32_t k0 = 0, len = 0;   /* k0: leading counts whose threshold rounds to 0 */
        for (uint32_t k = 0; k <= n; k++) {
            F += exp(ln - lgamma((double)k + 1.0) - lgamma((double)(n - k) + 1.0) + (double)k * lp +
                     (double)(n - k) * lq);
            double q = nearbyint(F * 4294967296.0);
            if (q >= 4294967296.0) break;
            if (q <= 0.0) {
                k0++;
                continue;
            }
            if (used == cap) {
                cap *= 2;
                uint32_t *nb = (uint32_t *)realloc(tb->bthr, cap * sizeof(uint32_t));
                if (!nb) return OR_E_NOMEM;
                tb->bthr = nb;
            }
            tb->bthr[used++] = (uint32_t)q;
            len++;
        }
        tb->bt[e].k0 = k0;
        tb->bt[e].len = len;
    }
    return OR_OK;
}

static void free_tables(or_tables *tb)
{
    free(tb->T);
    free(tb->bt);
    free(tb->bthr);
}

static int make_tables(const or_cfg *c, or_tables *tb)
{
    if (c->gx == 0 || c->gy == 0 || module_size(c) == 0) return OR_E_INVAL;
    if (!c->periodic) return OR_E_INVAL;
    if (c->d_min < 1 || c->d_max < c->d_min || c->d_max >= RING) return OR_E_INVAL;
    if (!(c->range > 0.0) || c->k_in < 0.0) return OR_E_INVAL;
    if (c->preset > OR_PRESET_PAPER) return OR_E_INVAL;
    if (c->preset == OR_PRESET_PAPER &&
        !(c->p_local >= 0.0 && c->p_local < 1.0 && c->amp >= 0.0 && c->amp < 1.0 && c->p_cut > 0.0))
        return OR_E_INVAL;
    if (!(c->tau_m > 0.0) || !(c->tau_w > 0.0) || c->t_ref < 0.0) return OR_E_INVAL;
    if (c->solver > OR_SOLVER_EXACT) return OR_E_INVAL;
    /* exact solver: a refractory period of at least one step keeps spikes to
     * one per neuron and step, and bounds it below 2^32 steps */
    if (c->solver == OR_SOLVER_EXACT && !(c->t_ref >= 1.0 && c->t_ref < 1e6)) return OR_E_INVAL;
    tb->T = (uint32_t *)calloc(2 * (size_t)c->gx * c->gy, sizeof(uint32_t));
    if (!tb->T) return OR_E_NOMEM;
    int st = make_thresholds(c, tb->T);
    if (st) return st;
    if (c->gen > OR_GEN_BINOMIAL) return OR_E_INVAL;
    /* Delays (Sec. II.B: uniform or exponential).  Exponential: bucket k of
     * the D integer delays has probability exp(-k/tau) / sum_i exp(-i/tau);
     * the bucket is the number of thresholds round(2^32 F(k)), k < D - 1,
     * not above the pair's first ATTR word. */
    if (c->delay_dist > OR_DELAY_EXP) return OR_E_INVAL;
    if (c->delay_dist == OR_DELAY_EXP) {
        uint32_t D = c->d_max - c->d_min + 1;
        if (!(c->delay_tau > 0.0)) return OR_E_INVAL;
        double total = 0.0, acc = 0.0;
        for (uint32_t k = 0; k < D; k++) total += exp(-(double)k / c->delay_tau);
        for (uint32_t k = 0; k + 1 < D; k++) {
            acc += exp(-(double)k / c->delay_tau);
            double q = nearbyint(acc / total * 4294967296.0);
            tb->dthr[k] = (q >= 4294967296.0) ? 0xFFFFFFFFu : (uint32_t)q;
        }
    }
    if (c->gen == OR_GEN_BINOMIAL) {
        if (module_size(c) > BINOM_MAX_M) return OR_E_INVAL;
        st = make_binomial(c, tb);
        if (st) return st;
    }
    make_wtab(c, tb->wtab);
    make_codebook(c, tb->cb);
    tb->npois = 0;
    if (c->ext_mode == OR_EXT_POISSON) {
        st = make_poisson(c, tb->poisc, &tb->npois);
        if (st) return st;
    }
    /* Exact one-step solution of du/dt = -(u + w)/tau_m, dw/dt = -w/tau_w
     * (Eq. (1)-(2) with the leak restoring towards E and the fatigue term
     * g_c c / C_m read as w / tau_m, w in mV), step 1 ms. */
    const double h = 1.0;
    tb->dm = -expm1(-h / c->tau_m);
    tb->dw = -expm1(-h / c->tau_w);
    if (c->tau_w != c->tau_m)
        tb->kappa = c->tau_w / (c->tau_w - c->tau_m) * (exp(-h / c->tau_w) - exp(-h / c->tau_m));
    else
        tb->kappa = (h / c->tau_m) * exp(-h / c->tau_m);
    tb->nref = (uint32_t)llround(c->t_ref / h);
    tb->jext_q = fixq(c->ext_w);
    tb->winh_q = fixq(c->w_inh);
    /* Spike-timing plasticity (Sec. II, Sec. II.A steps 1 and 4; pair-based
     * with exponential windows, the family of the rules the paper cites).
     * One pair of a presynaptic arrival and a postsynaptic spike k steps
     * apart changes the weight by kp[k] = round(A+ e^{-k/tau+} 2^16) when
     * the spike is not before the arrival, and by -km[k] = -round(A-
     * e^{-k/tau-} 2^16) when the arrival is k >= 1 steps after it; the
     * window ends at the first lag where both round to zero. */
    tb->win = 0;
    tb->wmax_q = 0;
    if (c->stdp > 1) return OR_E_INVAL;
    if (c->stdp) {
        if (c->solver != OR_SOLVER_STEP || c->record != OR_REC_F32) return OR_E_INVAL;
        if (!(c->a_plus >= 0.0) || !(c->a_minus >= 0.0) || !(c->tau_plus > 0.0) || !(c->tau_minus > 0.0) ||
            !(c->w_max > 0.0) || c->ltp_period == 0)
            return OR_E_INVAL;
        uint32_t win = 0;
        for (uint32_t k = 0; k < STDP_WIN_MAX; k++) {
            tb->kp[k] = (int32_t)nearbyint(c->a_plus * exp(-(double)k / c->tau_plus) * 65536.0);
            tb->km[k] = k ? (int32_t)nearbyint(c->a_minus * exp(-(double)k / c->tau_minus) * 65536.0) : 0;
            if (tb->kp[k] || tb->km[k]) win = k + 1;
        }
        if (win == STDP_WIN_MAX) return OR_E_INVAL;   /* window longer than the table */
        tb->win = win;
        tb->wmax_q = fixq(c->w_max);
    }
    return OR_OK;
}

/* Host threads the oracle's step uses (1 unless built with OpenMP). */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Exported for the table pins. */
int or_make_tables(const or_cfg *c, uint32_t *T, int32_t *wtab, int32_t *cb,
                   uint32_t *poisc, uint32_t *npois, double *consts, int32_t *iconsts)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    if (st == OR_OK) {
        if (T) memcpy(T, tb->T, 2 * sizeof(uint32_t) * c->gx * c->gy);
        if (wtab) memcpy(wtab, tb->wtab, sizeof(tb->wtab));
        if (cb) memcpy(cb, tb->cb, sizeof(tb->cb));
        if (poisc) memcpy(poisc, tb->poisc, sizeof(uint32_t) * tb->npois);
        if (npois) *npois = tb->npois;
        if (consts) { consts[0] = tb->dm; consts[1] = tb->dw; consts[2] = tb->kappa; }
        if (iconsts) { iconsts[0] = (int32_t)tb->nref; iconsts[1] = tb->jext_q; iconsts[2] = tb->winh_q; }
    }
    free_tables(tb);
    free(tb);
    return st;
}

/* Plasticity tables: kp[win], km[win] (km[0] unused, 0), the window and the
 * weight bound in 2^-16 mV.  Exported for the table pins. */
int or_stdp_tables(const or_cfg *c, int32_t *kp, int32_t *km, uint32_t *win, int32_t *wmax_q)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    if (st == OR_OK) {
        if (kp) memcpy(kp, tb->kp, sizeof(int32_t) * tb->win);
        if (km) memcpy(km, tb->km, sizeof(int32_t) * tb->win);
        if (win) *win = tb->win;
        if (wmax_q) *wmax_q = tb->wmax_q;
    }
    free_tables(tb);
    free(tb);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Connectivity (Sec. II.B, Sec. III.B)                                     */
/* ------------------------------------------------------------------------ */

/* Threshold of the ordered pair (i -> j): the source's type selects the
 * table, the torus offset of the two modules the entry. */
static uint32_t pair_threshold(const or_cfg *c, const or_tables *tb, uint32_t i, uint32_t j)
{
    uint32_t M = module_size(c);
    uint32_t mi = i / M, mj = j / M;
    uint32_t xi = mi % c->gx, yi = mi / c->gx, xj = mj % c->gx, yj = mj / c->gx;
    uint32_t dxr = (xj + c->gx - xi) % c->gx, dyr = (yj + c->gy - yi) % c->gy;
    size_t type = (i % M) < c->n_exc ? 0 : 1;
    return tb->T[type * c->gx * c->gy + dyr * c->gx + dxr];
}

/* Does neuron i project a synapse onto neuron j?  One Bernoulli trial per
 * ordered pair, no self-connections, at most one synapse per pair. */
static uint32_t module_subset(const or_cfg *c, const or_tables *tb, uint32_t i, uint32_t mj, uint8_t *in);

static int connects(const or_cfg *c, const or_tables *tb, uint32_t i, uint32_t j)
{
    if (i == j) return 0;
    if (c->gen == OR_GEN_BINOMIAL) {
        uint8_t in[BINOM_MAX_M];
        uint32_t M = module_size(c), mj = j / M, l = j % M;
        module_subset(c, tb, i, mj, in);
        if (mj == i / M && l > i % M) l--;
        return in[l];
    }
    uint32_t r[4];
    philox_draw(c->seed, i, j >> 2, ST_CONN, r);
    return r[j & 3u] < pair_threshold(c, tb, i, j);
}

/* Delay and fixed-point weight of the synapse i -> j (Sec. II.B: individual
 * delay, uniform; individual weight, Gaussian for excitatory sources). */
static void attributes(const or_cfg *c, const or_tables *tb, uint32_t i, uint32_t j,
                       uint32_t *delay, int32_t *wq, uint32_t *code)
{
    uint32_t a[4];
    philox_draw(c->seed, i, j, ST_ATTR, a);
    uint32_t span = c->d_max - c->d_min + 1;
    if (c->delay_dist == OR_DELAY_EXP) {
        uint32_t b = 0;
        for (uint32_t k = 0; k + 1 < span; k++)
            if (tb->dthr[k] <= a[0]) b++;
        *delay = c->d_min + b;
    } else {
        *delay = c->d_min + (uint32_t)(((uint64_t)a[0] * span) >> 32);
    }
    int exc = (i % module_size(c)) < c->n_exc;
    if (c->record == OR_REC_CODE8) {
        uint32_t k = exc ? (uint32_t)(((uint64_t)a[1] * 255u) >> 32) : 255u;
        *code = k;
        *wq = tb->cb[k];
    } else {
        *code = 0;
        *wq = exc ? tb->wtab[a[1] >> 16] : tb->winh_q;
    }
}

/* Uncompressed FP64 weight of the same draw, for precision statements. */
static double attributes_fp64_weight(const or_cfg *c, uint32_t i, uint32_t j)
{
    uint32_t a[4];
    philox_draw(c->seed, i, j, ST_ATTR, a);
    int exc = (i % module_size(c)) < c->n_exc;
    if (!exc) return c->w_inh;
    return c->w_exc + c->w_exc_sd * norm_quantile(((double)a[1] + 0.5) / 4294967296.0);
}

/* One synapse as stored: target, delay, weight (fixed point and FP64). */
typedef struct {
    uint32_t tgt, delay, code;
    int32_t wq;
    double wf;
} or_syn;

/* The projection of neuron i: every j with connects(i, j), ordered by
 * (delay, target).  Returns the count; *out is malloc'ed. */
/* Binomial generator, one (source i, target module mj): the count is the
 * number of the table's thresholds not above the draw Philox(i, mj, COUNT)[0];
 * the targets are a uniform random c-subset of the n candidates by Floyd's
 * algorithm (for j = n - c .. n - 1: t uniform in [0, j] from Philox(i, mj,
 * PICK, j / 4)[j % 4] as mulhi(draw, j + 1); take t, or j if t is already
 * taken).  Candidate l is neuron l of module mj, skipping the source itself
 * in its own module.  in[] (n flags) receives the subset; returns c. */
static uint32_t module_subset(const or_cfg *c, const or_tables *tb, uint32_t i, uint32_t mj, uint8_t *in)
{
    uint32_t M = module_size(c), mi = i / M;
    uint32_t xi = mi % c->gx, yi = mi / c->gx, xj = mj % c->gx, yj = mj / c->gx;
    size_t S = (size_t)c->gx * c->gy;
    size_t off = ((yj + c->gy - yi) % c->gy) * c->gx + (xj + c->gx - xi) % c->gx;
    size_t e = ((i % M) < c->n_exc ? 0 : S) + off;
    uint32_t n = (mj == mi) ? M - 1 : M;
    memset(in, 0, n);
    if (tb->T[e] == 0) return 0;
    uint32_t r[4];
    philox_draw(c->seed, i, mj, ST_COUNT, r);
    const or_binom *b = &tb->bt[e];
    uint32_t cnt = b->k0;
    for (uint32_t k = 0; k < b->len; k++)
        if (tb->bthr[b->at + k] <= r[0]) cnt++;
    for (uint32_t j = n - cnt; j < n; j++) {
        uint32_t w[4];
        uint32_t ctr[4] = {i, mj, ST_PICK, j >> 2};
        uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
        or_philox(ctr, key, w);
        uint32_t t = (uint32_t)(((uint64_t)w[j & 3u] * (uint64_t)(j + 1u)) >> 32);
        if (in[t]) in[j] = 1;
        else in[t] = 1;
    }
    return cnt;
}

static int64_t build_row(const or_cfg *c, const or_tables *tb, uint32_t i, or_syn **out, int want_fp64)
{
    uint32_t N = c->gx * c->gy * module_size(c);
    uint32_t D = c->d_max - c->d_min + 1;
    size_t cap = 1024, n = 0;
    or_syn *hits = (or_syn *)malloc(cap * sizeof(or_syn));
    if (!hits) return OR_E_NOMEM;
    uint8_t *in = NULL;
    if (c->gen == OR_GEN_BINOMIAL) {
        in = (uint8_t *)malloc(module_size(c));
        if (!in) { free(hits); return OR_E_NOMEM; }
    }
    for (uint32_t j = 0; j < N; j++) {
        if (c->gen == OR_GEN_BINOMIAL) {
            /* module by module: the module's subset, targets ascending */
            uint32_t M = module_size(c), mj = j / M;
            if (j % M == 0) module_subset(c, tb, i, mj, in);
            uint32_t l = j % M, self = (mj == i / M) ? i % M : M;
            if (l == self) continue;
            if (!in[l < self ? l : l - 1]) continue;
        } else if (!connects(c, tb, i, j)) {
            continue;
        }
        if (n == cap) {
            cap *= 2;
            or_syn *nh = (or_syn *)realloc(hits, cap * sizeof(or_syn));
            if (!nh) { free(hits); return OR_E_NOMEM; }
            hits = nh;
        }
        or_syn s;
        s.tgt = j;
        attributes(c, tb, i, j, &s.delay, &s.wq, &s.code);
        s.wf = want_fp64 ? attributes_fp64_weight(c, i, j) : 0.0;
        hits[n++] = s;
    }
    free(in);
    /* stable counting sort by delay: targets stay ascending within a delay */
    or_syn *sorted = (or_syn *)malloc((n ? n : 1) * sizeof(or_syn));
    if (!sorted) { free(hits); return OR_E_NOMEM; }
    size_t k = 0;
    for (uint32_t d = 0; d < D; d++)
        for (size_t h = 0; h < n; h++)
            if (hits[h].delay == c->d_min + d) sorted[k++] = hits[h];
    free(hits);
    *out = sorted;
    return (int64_t)n;
}

/* ------------------------------------------------------------------------ */
/* Network                                                                  */
/* ------------------------------------------------------------------------ */
/* Exact solver: one queued input, arriving at (slot step, offset f). */
typedef struct or_ev {
    uint32_t tgt;           /* target neuron                     */
    uint32_t f;             /* offset in the step, 2^-32 ms      */
    int32_t wq;             /* charge, 2^-16 mV                  */
} or_ev;

typedef struct {
    or_cfg c;
    or_tables tb;
    uint32_t N, D;
    /* CSR of outgoing synapses, rows ordered by (delay, target) */
    uint64_t *row_ptr;      /* [N+1] */
    uint16_t *bend;         /* [N][D] end of each delay bucket, row-relative */
    or_syn *syn;            /* [nnz] */
    uint64_t nnz;
    int built;
    int fp64_weights;       /* deliver FP64 weights instead of fixed point  */
    /* state */
    double *V, *w;
    int32_t *ref;
    int32_t *ring;          /* [RING][N] fixed-point charge, int32 wrap-add */
    int64_t *ring64;        /* [RING][N] exact shadow                        */
    double *ringf;          /* [RING][N] FP64 charge when fp64_weights       */
    uint8_t *flag;
    uint32_t t;
    /* spike history (AER: time step, neuron id), Sec. II.C */
    uint32_t *hist;
    size_t hist_n, hist_cap;
    uint64_t n_spikes, rec_events, ext_events;
    int overflow;
    /* exact-time solver */
    uint64_t *rend;         /* [N] end of the refractory period, ms in 32.32 fixed point */
    uint32_t *fs;           /* [N] emission offset of this step's spike (2^-32 ms)       */
    struct or_ev *q[RING];  /* per arrival slot: queued events, unsorted                 */
    size_t qn[RING], qcap[RING];
    uint32_t *hist_f;       /* emission offset of each history entry                     */
    /* spike-timing plasticity */
    int64_t *acc;           /* [nnz] weight change of the running period, 2^-16 mV */
    uint64_t *in_ptr;       /* [N+1] incoming synapses grouped by target            */
    uint64_t *in_syn;       /* [nnz] index in syn[] of each incoming synapse         */
    uint32_t *in_pre;       /* [nnz] its presynaptic neuron                          */
    uint32_t **spk;         /* [N] spike steps of each neuron, ascending            */
    uint32_t *spk_n, *spk_cap;
} or_net;

void or_net_free(void *h)
{
    or_net *n = (or_net *)h;
    if (!n) return;
    free(n->tb.T); free(n->row_ptr); free(n->bend); free(n->syn);
    free(n->V); free(n->w); free(n->ref); free(n->ring); free(n->ring64); free(n->ringf);
    free(n->flag); free(n->hist);
    free(n->rend); free(n->fs); free(n->hist_f);
    for (int k = 0; k < RING; k++) free(n->q[k]);
    free(n->acc); free(n->in_ptr); free(n->in_syn); free(n->in_pre);
    if (n->spk)
        for (uint32_t i = 0; i < n->N; i++) free(n->spk[i]);
    free(n->spk); free(n->spk_n); free(n->spk_cap);
    free(n);
}

/* Initial state: V uniform in [E, V_th) from the INIT stream, no fatigue,
 * not refractory, empty delay queues. */
void *or_net_create(const or_cfg *c, int fp64_weights)
{
    or_net *n = (or_net *)calloc(1, sizeof(or_net));
    if (!n) return NULL;
    n->c = *c;
    if (make_tables(c, &n->tb) != OR_OK) { or_net_free(n); return NULL; }
    n->N = c->gx * c->gy * module_size(c);
    n->D = c->d_max - c->d_min + 1;
    n->fp64_weights = fp64_weights;
    n->V = (double *)calloc(n->N, sizeof(double));
    n->w = (double *)calloc(n->N, sizeof(double));
    n->ref = (int32_t *)calloc(n->N, sizeof(int32_t));
    n->ring = (int32_t *)calloc((size_t)RING * n->N, sizeof(int32_t));
    n->ring64 = (int64_t *)calloc((size_t)RING * n->N, sizeof(int64_t));
    n->ringf = (double *)calloc((size_t)RING * n->N, sizeof(double));
    n->flag = (uint8_t *)calloc(n->N, 1);
    n->hist_cap = 1024;
    n->hist = (uint32_t *)malloc(2 * n->hist_cap * sizeof(uint32_t));
    n->rend = (uint64_t *)calloc(n->N, sizeof(uint64_t));
    n->fs = (uint32_t *)calloc(n->N, sizeof(uint32_t));
    n->hist_f = (uint32_t *)malloc(n->hist_cap * sizeof(uint32_t));
    if (!n->V || !n->w || !n->ref || !n->ring || !n->ring64 || !n->ringf || !n->flag || !n->hist ||
        !n->rend || !n->fs || !n->hist_f) {
        or_net_free(n);
        return NULL;
    }
    for (uint32_t g = 0; g < n->N; g++) {
        uint32_t r[4];
        philox_draw(c->seed, g >> 2, 0u, ST_INIT, r);
        double u = (double)(r[g & 3u] >> 8) * (1.0 / 16777216.0);
        n->V[g] = c->e_rest + (c->v_th - c->e_rest) * u;
    }
    return n;
}

/* Build every projection (Sec. II.B). */
int or_net_build(void *h)
{
    or_net *n = (or_net *)h;
    n->row_ptr = (uint64_t *)calloc((size_t)n->N + 1, sizeof(uint64_t));
    n->bend = (uint16_t *)calloc((size_t)n->N * n->D, sizeof(uint16_t));
    if (!n->row_ptr || !n->bend) return OR_E_NOMEM;
    size_t cap = 1024;
    n->syn = (or_syn *)malloc(cap * sizeof(or_syn));
    if (!n->syn) return OR_E_NOMEM;
    uint64_t nnz = 0;
    for (uint32_t i = 0; i < n->N; i++) {
        or_syn *row = NULL;
        int64_t len = build_row(&n->c, &n->tb, i, &row, n->fp64_weights);
        if (len < 0) return (int)len;
        if (len > 65535) { free(row); return OR_E_OVERFLOW; }
        while (nnz + (uint64_t)len > cap) {
            cap *= 2;
            or_syn *ns = (or_syn *)realloc(n->syn, cap * sizeof(or_syn));
            if (!ns) { free(row); return OR_E_NOMEM; }
            n->syn = ns;
        }
        memcpy(n->syn + nnz, row, (size_t)len * sizeof(or_syn));
        n->row_ptr[i] = nnz;
        for (uint32_t d = 0; d < n->D; d++) {
            uint32_t e = 0;
            for (int64_t k = 0; k < len; k++)
                if (row[k].delay <= n->c.d_min + d) e = (uint32_t)(k + 1);
            n->bend[(size_t)i * n->D + d] = (uint16_t)e;
        }
        nnz += (uint64_t)len;
        free(row);
    }
    n->row_ptr[n->N] = nnz;
    n->nnz = nnz;
    n->built = 1;
    return OR_OK;
}

/* Serialise projections in the library's record layout: for F32 records
 * 8 bytes {u32 target, f32 weight in mV}; for CODE8 records one u32
 * (target << 8 | code).  Buckets end offsets are row-relative u16. */
static void put_record(const or_cfg *c, const or_syn *s, uint8_t *dst)
{
    if (c->record == OR_REC_CODE8) {
        uint32_t v = (s->tgt << 8) | s->code;
        memcpy(dst, &v, 4);
    } else {
        float wf = (float)((double)s->wq / 65536.0);
        memcpy(dst, &s->tgt, 4);
        memcpy(dst + 4, &wf, 4);
    }
}

static size_t record_bytes(const or_cfg *c) { return c->record == OR_REC_CODE8 ? 4 : 8; }

/* Rows pre0 .. pre0+cnt-1 of the projection table, built one by one. */
int or_build_rows(const or_cfg *c, uint32_t pre0, uint32_t cnt, uint64_t *row_len,
                  uint16_t *bend, void *recs, uint64_t rec_cap, uint64_t *n_out)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    uint32_t D = c->d_max - c->d_min + 1;
    uint64_t total = 0;
    size_t rb = record_bytes(c);
    for (uint32_t r = 0; st == OR_OK && r < cnt; r++) {
        or_syn *row = NULL;
        int64_t len = build_row(c, tb, pre0 + r, &row, 0);
        if (len < 0) { st = (int)len; break; }
        row_len[r] = (uint64_t)len;
        for (uint32_t d = 0; d < D; d++) {
            uint32_t e = 0;
            for (int64_t k = 0; k < len; k++)
                if (row[k].delay <= c->d_min + d) e = (uint32_t)(k + 1);
            bend[(size_t)r * D + d] = (uint16_t)e;
        }
        for (int64_t k = 0; k < len; k++)
            if (total + (uint64_t)k < rec_cap)
                put_record(c, &row[k], (uint8_t *)recs + (size_t)(total + (uint64_t)k) * rb);
        total += (uint64_t)len;
        free(row);
    }
    *n_out = total;
    free_tables(tb);
    free(tb);
    if (st == OR_OK && total > rec_cap) return OR_E_OVERFLOW;
    return st;
}

/* Charge that the presynaptic neurons pres[0..np) deliver to neuron j, by
 * delay bucket: sum of fixed-point weights of the synapses pres -> j. */
int or_col_input(const or_cfg *c, uint32_t j, const uint32_t *pres, uint64_t np, int64_t *per_delay)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    uint32_t D = c->d_max - c->d_min + 1;
    for (uint32_t d = 0; d < D; d++) per_delay[d] = 0;
    for (uint64_t k = 0; st == OR_OK && k < np; k++) {
        uint32_t i = pres[k];
        if (!connects(c, tb, i, j)) continue;
        uint32_t delay, code;
        int32_t wq;
        attributes(c, tb, i, j, &delay, &wq, &code);
        per_delay[delay - c->d_min] += wq;
    }
    free_tables(tb);
    free(tb);
    return st;
}

/* Charge queued for target j after steps 0 .. T-1 (delay ring in flight):
 * out[a], a < d_max, is the fixed-point charge arriving at step T + a from
 * the spikes (steps[k], pres[k]), each reaching j at its step plus the
 * synapse's delay (Sec. II.A steps 2-4). */
int or_col_pending(const or_cfg *c, uint32_t j, const uint32_t *steps, const uint32_t *pres, uint64_t np,
                   uint32_t T, int64_t *out)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    for (uint32_t a = 0; a < c->d_max; a++) out[a] = 0;
    for (uint64_t k = 0; st == OR_OK && k < np; k++) {
        uint32_t i = pres[k];
        if (!connects(c, tb, i, j)) continue;
        uint32_t delay, code;
        int32_t wq;
        attributes(c, tb, i, j, &delay, &wq, &code);
        uint64_t arr = (uint64_t)steps[k] + delay;
        if (arr >= T && arr < (uint64_t)T + c->d_max) out[arr - T] += wq;
    }
    free_tables(tb);
    free(tb);
    return st;
}

int or_net_csr(void *h, uint64_t *row_ptr, uint16_t *bend, void *recs, uint64_t rec_cap)
{
    or_net *n = (or_net *)h;
    if (!n->built) return OR_E_INVAL;
    if (row_ptr) memcpy(row_ptr, n->row_ptr, ((size_t)n->N + 1) * sizeof(uint64_t));
    if (bend) memcpy(bend, n->bend, (size_t)n->N * n->D * sizeof(uint16_t));
    if (recs) {
        if (rec_cap < n->nnz) return OR_E_OVERFLOW;
        size_t rb = record_bytes(&n->c);
        for (uint64_t k = 0; k < n->nnz; k++) put_record(&n->c, &n->syn[k], (uint8_t *)recs + k * rb);
    }
    return OR_OK;
}

uint64_t or_net_nnz(void *h) { return ((or_net *)h)->nnz; }

/* Use a caller-supplied projection table (rows in the library's record
 * layout, F32 records only): lets a brute-force or hand-made network be
 * simulated by the same step code. */
int or_net_set_csr(void *h, const uint64_t *row_ptr, const uint16_t *bend, const uint32_t *tgt,
                   const uint32_t *delay, const int32_t *wq)
{
    or_net *n = (or_net *)h;
    uint64_t nnz = row_ptr[n->N];
    free(n->row_ptr); free(n->bend); free(n->syn);
    n->row_ptr = (uint64_t *)malloc(((size_t)n->N + 1) * sizeof(uint64_t));
    n->bend = (uint16_t *)malloc((size_t)n->N * n->D * sizeof(uint16_t));
    n->syn = (or_syn *)malloc((nnz ? nnz : 1) * sizeof(or_syn));
    if (!n->row_ptr || !n->bend || !n->syn) return OR_E_NOMEM;
    memcpy(n->row_ptr, row_ptr, ((size_t)n->N + 1) * sizeof(uint64_t));
    memcpy(n->bend, bend, (size_t)n->N * n->D * sizeof(uint16_t));
    for (uint64_t k = 0; k < nnz; k++) {
        n->syn[k].tgt = tgt[k];
        n->syn[k].delay = delay[k];
        n->syn[k].wq = wq[k];
        n->syn[k].code = 0;
        n->syn[k].wf = (double)wq[k] / 65536.0;
    }
    n->nnz = nnz;
    n->built = 1;
    free(n->in_ptr); free(n->in_syn); free(n->in_pre); free(n->acc);
    n->in_ptr = NULL; n->in_syn = NULL; n->in_pre = NULL; n->acc = NULL;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Simulation (Sec. II.A, Sec. III.A)                                       */
/* ------------------------------------------------------------------------ */

/* External Poisson count of neuron g in step t. */
static uint32_t ext_count(const or_net *n, uint32_t g, uint32_t t)
{
    uint32_t r[4];
    philox_draw(n->c.seed, g >> 2, t, ST_EXT, r);
    uint32_t u = r[g & 3u], k = 0;
    for (uint32_t q = 0; q < n->tb.npois; q++)
        if (n->tb.poisc[q] <= u) k++;
    return k;
}

/* External Poisson counts of every neuron for steps t0 .. t1-1, out[(t - t0)
 * N + g] (saturated at 255); the same draw the simulation takes. */
int or_net_ext_counts(void *h, uint32_t t0, uint32_t t1, uint8_t *out)
{
    or_net *n = (or_net *)h;
    if (t1 < t0) return OR_E_INVAL;
    for (uint32_t t = t0; t < t1; t++)
        for (uint32_t g = 0; g < n->N; g++) {
            uint32_t k = ext_count(n, g, t);
            out[(size_t)(t - t0) * n->N + g] = (uint8_t)(k > 255u ? 255u : k);
        }
    return OR_OK;
}

static void hist_push(or_net *n, uint32_t t, uint32_t g, uint32_t f)
{
    if (n->hist_n == n->hist_cap) {
        size_t nc = n->hist_cap * 2;
        uint32_t *nh = (uint32_t *)realloc(n->hist, 2 * nc * sizeof(uint32_t));
        if (!nh) { n->overflow = 1; return; }
        n->hist = nh;
        uint32_t *nf = (uint32_t *)realloc(n->hist_f, nc * sizeof(uint32_t));
        if (!nf) { n->overflow = 1; return; }
        n->hist_f = nf;
        n->hist_cap = nc;
    }
    n->hist[2 * n->hist_n] = t;
    n->hist[2 * n->hist_n + 1] = g;
    n->hist_f[n->hist_n] = f;
    n->hist_n++;
}

/* ------------------------------------------------------------------------ */
/* Spike-timing plasticity (Sec. II, Sec. II.A steps 1 and 4, long-term    */
/* application every period)                                                */
/* ------------------------------------------------------------------------ */
/* A synapse i -> j of delay d sees a presynaptic event at every arrival
 * a = s + d of a spike of i at step s, and a postsynaptic event at every
 * spike of j at step p.  Each pair of the two within the window contributes
 * once, when its later event happens: at a postsynaptic spike (step 1 of the
 * step loop: the step's spikers are identified) every arrival a <= p adds
 * kp[p - a]; at an arrival (step 4: the synapse injects its current) every
 * earlier postsynaptic spike p < a adds -km[a - p].  An arrival and a spike
 * in the same step form a potentiating pair (the input is applied before the
 * threshold test).  Only synapses of excitatory sources are plastic.  At the
 * end of every period of ltp_period steps a synapse whose accumulated change
 * is not zero gets its weight plus the change, clipped to [0, w_max] (the
 * others keep theirs), and the accumulator is cleared; spikes use the weight
 * in force when they are emitted. */
static int stdp_prepare(or_net *n)
{
    const uint32_t N = n->N;
    if (!n->spk) {
        n->spk = (uint32_t **)calloc(N, sizeof(uint32_t *));
        n->spk_n = (uint32_t *)calloc(N, sizeof(uint32_t));
        n->spk_cap = (uint32_t *)calloc(N, sizeof(uint32_t));
        if (!n->spk || !n->spk_n || !n->spk_cap) return OR_E_NOMEM;
    }
    if (n->in_ptr || !n->built) return OR_OK;
    const uint64_t nnz = n->nnz;
    n->in_ptr = (uint64_t *)calloc((size_t)N + 1, sizeof(uint64_t));
    n->in_syn = (uint64_t *)malloc((nnz ? nnz : 1) * sizeof(uint64_t));
    n->in_pre = (uint32_t *)malloc((nnz ? nnz : 1) * sizeof(uint32_t));
    n->acc = (int64_t *)calloc(nnz ? nnz : 1, sizeof(int64_t));
    if (!n->in_ptr || !n->in_syn || !n->in_pre || !n->acc) return OR_E_NOMEM;
    for (uint64_t k = 0; k < nnz; k++) n->in_ptr[n->syn[k].tgt + 1]++;
    for (uint32_t j = 0; j < N; j++) n->in_ptr[j + 1] += n->in_ptr[j];
    uint64_t *fill = (uint64_t *)malloc(((size_t)N + 1) * sizeof(uint64_t));
    if (!fill) return OR_E_NOMEM;
    memcpy(fill, n->in_ptr, ((size_t)N + 1) * sizeof(uint64_t));
    for (uint32_t i = 0; i < N; i++)
        for (uint64_t k = n->row_ptr[i]; k < n->row_ptr[i + 1]; k++) {
            uint64_t e = fill[n->syn[k].tgt]++;
            n->in_syn[e] = k;
            n->in_pre[e] = i;
        }
    free(fill);
    return OR_OK;
}

static int spike_log(or_net *n, uint32_t i, uint32_t t)
{
    if (n->spk_n[i] == n->spk_cap[i]) {
        uint32_t nc = n->spk_cap[i] ? 2 * n->spk_cap[i] : 16;
        uint32_t *p = (uint32_t *)realloc(n->spk[i], nc * sizeof(uint32_t));
        if (!p) return OR_E_NOMEM;
        n->spk[i] = p;
        n->spk_cap[i] = nc;
    }
    n->spk[i][n->spk_n[i]++] = t;
    return OR_OK;
}

/* First history entry of step s (the history is ordered by step). */
static size_t hist_lower(const or_net *n, uint32_t s)
{
    size_t lo = 0, hi = n->hist_n;
    while (lo < hi) {
        size_t mid = (lo + hi) / 2;
        if (n->hist[2 * mid] < s) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* Contributions of the pairs whose later event falls in step t. */
static void stdp_events(or_net *n, uint32_t t)
{
    const or_cfg *c = &n->c;
    const or_tables *tb = &n->tb;
    const uint32_t M = module_size(c), win = tb->win;
    /* postsynaptic spikes of step t: potentiation against arrivals a <= t */
    for (uint32_t j = 0; j < n->N; j++) {
        if (!n->flag[j]) continue;
        for (uint64_t e = n->in_ptr[j]; e < n->in_ptr[j + 1]; e++) {
            uint32_t i = n->in_pre[e];
            if (i % M >= c->n_exc) continue;
            uint64_t k = n->in_syn[e];
            uint32_t d = n->syn[k].delay;
            for (uint32_t q = 0; q < n->spk_n[i]; q++) {
                uint32_t a = n->spk[i][q] + d;
                if (a > t) break;
                if (t - a < win) n->acc[k] += tb->kp[t - a];
            }
        }
    }
    /* arrivals at step t (spikes of step t - d through delay-d synapses):
     * depression against postsynaptic spikes p < t */
    for (uint32_t d = c->d_min; d <= c->d_max && d <= t; d++) {
        uint32_t s = t - d;
        for (size_t h = hist_lower(n, s); h < n->hist_n && n->hist[2 * h] == s; h++) {
            uint32_t i = n->hist[2 * h + 1];
            if (i % M >= c->n_exc) continue;
            uint64_t r0 = n->row_ptr[i];
            uint64_t b0 = r0 + (d > c->d_min ? n->bend[(size_t)i * n->D + (d - c->d_min - 1)] : 0);
            uint64_t b1 = r0 + n->bend[(size_t)i * n->D + (d - c->d_min)];
            for (uint64_t k = b0; k < b1; k++) {
                uint32_t j = n->syn[k].tgt;
                for (uint32_t q = n->spk_n[j]; q-- > 0;) {
                    uint32_t p = n->spk[j][q];
                    if (p >= t) continue;
                    if (t - p >= win) break;
                    n->acc[k] -= tb->km[t - p];
                }
            }
        }
    }
}

/* The change of a period for given synapses, straight from the definition:
 * for synapse k (pre[k] -> tgt[k], delay[k]) the sum over every pair of a
 * spike s of the source and a spike p of the target in the raster, with
 * arrival a = s + delay, max(a, p) in [T0, T1) and |p - a| < win, of
 * kp[p - a] (p >= a) or -km[a - p] (p < a).  Unclipped; 0 for inhibitory
 * sources.  The raster is (step, gid) pairs in any order. */
int or_stdp_totals(const or_cfg *c, const uint32_t *r_step, const uint32_t *r_gid, uint64_t nr,
                   const uint32_t *pre, const uint32_t *tgt, const uint32_t *delay, uint64_t ns,
                   uint32_t T0, uint32_t T1, int64_t *out)
{
    or_tables *tb = (or_tables *)calloc(1, sizeof(or_tables));
    if (!tb) return OR_E_NOMEM;
    int st = make_tables(c, tb);
    const uint32_t M = module_size(c);
    for (uint64_t k = 0; st == OR_OK && k < ns; k++) {
        int64_t acc = 0;
        if (c->stdp && pre[k] % M < c->n_exc) {
            for (uint64_t x = 0; x < nr; x++) {
                if (r_gid[x] != pre[k]) continue;
                int64_t a = (int64_t)r_step[x] + delay[k];
                for (uint64_t y = 0; y < nr; y++) {
                    if (r_gid[y] != tgt[k]) continue;
                    int64_t p = r_step[y], later = p > a ? p : a, lag = p - a;
                    if (later < T0 || later >= T1) continue;
                    if (lag >= 0 && lag < (int64_t)tb->win) acc += tb->kp[lag];
                    if (lag < 0 && -lag < (int64_t)tb->win) acc -= tb->km[-lag];
                }
            }
        }
        out[k] = acc;
    }
    free_tables(tb);
    free(tb);
    return st;
}

/* Long-term application at the end of a period. */
static void stdp_apply(or_net *n)
{
    const uint32_t M = module_size(&n->c);
    for (uint32_t i = 0; i < n->N; i++) {
        if (i % M >= n->c.n_exc) continue;
        for (uint64_t k = n->row_ptr[i]; k < n->row_ptr[i + 1]; k++) {
            if (n->acc[k] == 0) continue;   /* no net change: the weight is kept as it is */
            int64_t w = (int64_t)n->syn[k].wq + n->acc[k];
            if (w < 0) w = 0;
            if (w > n->tb.wmax_q) w = n->tb.wmax_q;
            n->syn[k].wq = (int32_t)w;
            n->syn[k].wf = (double)w / 65536.0;
            n->acc[k] = 0;
        }
    }
}

/* One 1 ms step.  Every neuron first takes the charge queued for this step
 * (recurrent, from the delay queue, plus external), then integrates
 * Eq. (1)-(2); the spikers, in ascending id, are recorded and their
 * projections enqueue charge at step t + delay.
 * When forced is non-NULL the spike set is forced[] instead of the
 * threshold test (lock-step mode): forced neurons that are not refractory
 * are reset as spikers, every other neuron integrates. */
static int step_once(or_net *n, const uint8_t *forced)
{
    const or_cfg *c = &n->c;
    uint32_t t = n->t, slot = t % RING, N = n->N;
    uint64_t ext_ev = 0, rec_ev = 0;
    /* each neuron's update reads and writes only its own state (the OpenMP
     * build of the CPU baseline splits this loop over the host cores) */
#pragma omp parallel for schedule(static) reduction(+ : ext_ev)
    for (uint32_t j = 0; j < N; j++) {
        size_t s = (size_t)slot * N + j;
        int64_t in64 = n->ring64[s];
        double inf = n->ringf[s];
        if (in64 > INT32_MAX || in64 < INT32_MIN) n->overflow = 1;
        int32_t iq = n->ring[s];
        n->ring[s] = 0;
        n->ring64[s] = 0;
        n->ringf[s] = 0.0;
        int32_t eq;
        if (c->ext_mode == OR_EXT_CONST) {
            eq = c->ext_const_q;
        } else {
            uint32_t k = ext_count(n, j, t);
            ext_ev += k;
            eq = (int32_t)k * n->tb.jext_q;
        }
        double J = n->fp64_weights ? inf + (double)eq / 65536.0 : (double)(iq + eq) / 65536.0;
        int exc = (j % module_size(c)) < c->n_exc;
        n->flag[j] = 0;
        if (n->ref[j] > 0) {
            /* absolute refractory period: held at reset, input ignored */
            n->ref[j] -= 1;
            n->V[j] = c->v_reset;
        } else {
            double V = n->V[j] + J;
            int spike = forced ? (forced[j] != 0) : (V > c->v_th);
            if (spike) {
                n->flag[j] = 1;
                V = c->v_reset;
                n->ref[j] = (int32_t)n->tb.nref;
                if (exc || c->sfa_on_inh) n->w[j] += c->alpha_w;
            } else {
                double u = V - c->e_rest;
                u = u - u * n->tb.dm - n->tb.kappa * n->w[j];
                V = c->e_rest + u;
            }
            n->V[j] = V;
        }
        n->w[j] = n->w[j] - n->w[j] * n->tb.dw;
    }
    n->ext_events += ext_ev;
    if (c->stdp) {
        int st = stdp_prepare(n);
        if (st) return st;
    }
    /* the step's spikers, in ascending id, into the AER history */
    for (uint32_t i = 0; i < N; i++) {
        if (!n->flag[i]) continue;
        hist_push(n, t, i, 0u);
        n->n_spikes++;
        if (c->stdp && spike_log(n, i, t)) return OR_E_NOMEM;
    }
    /* each spiker's projection into the delay ring at step t + delay (integer
     * sums commute: the OpenMP build adds from several cores at once) */
    if (n->built) {
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : rec_ev)
        for (uint32_t i = 0; i < N; i++) {
            if (!n->flag[i]) continue;
            for (uint64_t k = n->row_ptr[i]; k < n->row_ptr[i + 1]; k++) {
                const or_syn *s = &n->syn[k];
                size_t a = (size_t)((t + s->delay) % RING) * N + s->tgt;
#pragma omp atomic
                ((uint32_t *)n->ring)[a] += (uint32_t)s->wq;
#pragma omp atomic
                n->ring64[a] += s->wq;
#pragma omp atomic
                n->ringf[a] += s->wf;
                rec_ev++;
            }
        }
        n->rec_events += rec_ev;
    }
    if (c->stdp && n->built) {
        stdp_events(n, t);
        if ((t + 1) % c->ltp_period == 0) stdp_apply(n);
    }
    n->t = t + 1;
    return n->overflow ? OR_E_OVERFLOW : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact-time event-driven solver (Sec. II.A, Sec. II.C)                    */
/* ------------------------------------------------------------------------ */
/* Times are absolute, in ms, in 32.32 fixed point: step t, offset f, is
 * (t << 32) | f.  A spike is emitted at the time of the input that takes V
 * above threshold (with delta synapses and E below V_th the potential only
 * falls between inputs, so threshold is crossed only at an input); it
 * reaches each target at emission time + the synapse's integer delay, so it
 * keeps its offset inside the step.  External inputs of a step: the same
 * Poisson count as the step solver, arriving at offsets drawn uniformly from
 * the EXT_TIME stream; the constant drive arrives at offset 0.  Inputs that
 * arrive at the same instant are summed before the threshold test.  A spike
 * at time s holds V at V_r over [s, s + t_ref), inputs inside it are
 * discarded, and w keeps decaying.  With every offset 0 and t_ref one step
 * longer this is exactly the step solver. */

static void ev_push(or_net *n, uint32_t slot, uint32_t tgt, uint32_t f, int32_t wq)
{
    if (n->qn[slot] == n->qcap[slot]) {
        size_t nc = n->qcap[slot] ? 2 * n->qcap[slot] : 1024;
        or_ev *nq = (or_ev *)realloc(n->q[slot], nc * sizeof(or_ev));
        if (!nq) { n->overflow = 1; return; }
        n->q[slot] = nq;
        n->qcap[slot] = nc;
    }
    or_ev *e = &n->q[slot][n->qn[slot]++];
    e->tgt = tgt;
    e->f = f;
    e->wq = wq;
}

static int ev_cmp(const void *a, const void *b)
{
    const or_ev *x = (const or_ev *)a, *y = (const or_ev *)b;
    if (x->tgt != y->tgt) return x->tgt < y->tgt ? -1 : 1;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    if (x->wq != y->wq) return x->wq < y->wq ? -1 : 1;
    return 0;
}

/* Exact solution of du/dt = -(u + w)/tau_m, dw/dt = -w/tau_w over h ms. */
static void propagate(const or_cfg *c, double h, double *V, double *w)
{
    double em = exp(-h / c->tau_m), ew = exp(-h / c->tau_w);
    double kap = (c->tau_w != c->tau_m) ? c->tau_w / (c->tau_w - c->tau_m) * (ew - em) : (h / c->tau_m) * em;
    double u = *V - c->e_rest;
    u = u * em - kap * *w;
    *V = c->e_rest + u;
    *w = *w * ew;
}

/* Advance one neuron from absolute time a to b (a <= b), holding V at V_r
 * while refractory (before re). */
static void advance(const or_cfg *c, uint64_t a, uint64_t b, uint64_t re, double *V, double *w)
{
    const double q = 1.0 / 4294967296.0;
    if (a < re) {
        uint64_t e = re < b ? re : b;
        *w = *w * exp(-(double)(e - a) * q / c->tau_w);
        *V = c->v_reset;
        a = e;
    }
    if (a < b) propagate(c, (double)(b - a) * q, V, w);
}

/* External input times of neuron g in step t: offsets of the k-th event. */
static uint32_t ext_offset(const or_net *n, uint32_t g, uint32_t t, uint32_t k)
{
    uint32_t ctr[4] = {g, t, ST_EXT_TIME, k >> 2}, key[2], r[4];
    key[0] = (uint32_t)n->c.seed;
    key[1] = (uint32_t)(n->c.seed >> 32);
    or_philox(ctr, key, r);
    return r[k & 3u];
}

typedef struct {
    uint32_t f;
    int32_t wq;
} or_in;

static int in_cmp(const void *a, const void *b)
{
    const or_in *x = (const or_in *)a, *y = (const or_in *)b;
    if (x->f != y->f) return x->f < y->f ? -1 : 1;
    return (x->wq > y->wq) - (x->wq < y->wq);
}

/* One 1 ms step of the exact solver.  forced != NULL: lock-step mode, neuron
 * j spikes exactly at offset ff[j] when forced[j] is set (and it is not
 * refractory and an input arrives then), never otherwise. */
static int step_exact(or_net *n, const uint8_t *forced, const uint32_t *ff)
{
    const or_cfg *c = &n->c;
    const uint32_t t = n->t, slot = t % RING, N = n->N;
    const uint64_t t0 = (uint64_t)t << 32, t1 = t0 + (1ull << 32);
    const uint64_t tref = (uint64_t)llround(c->t_ref * 4294967296.0);
    or_ev *q = n->q[slot];
    const size_t nq = n->qn[slot];
    if (nq) qsort(q, nq, sizeof(or_ev), ev_cmp);
    size_t k = 0;
    size_t cap = 64;
    or_in *in = (or_in *)malloc(cap * sizeof(or_in));
    if (!in) return OR_E_NOMEM;
    for (uint32_t j = 0; j < N; j++) {
        /* this step's inputs: queued recurrent ones, then external ones */
        size_t m = 0, k1 = k;
        while (k1 < nq && q[k1].tgt == j) k1++;
        uint32_t next = 0;
        if (c->ext_mode == OR_EXT_CONST) {
            next = 1;
        } else {
            next = ext_count(n, j, t);
            n->ext_events += next;
        }
        size_t need = (k1 - k) + next;
        if (need > cap) {
            while (cap < need) cap *= 2;
            or_in *ni = (or_in *)realloc(in, cap * sizeof(or_in));
            if (!ni) { free(in); return OR_E_NOMEM; }
            in = ni;
        }
        for (size_t e = k; e < k1; e++) { in[m].f = q[e].f; in[m].wq = q[e].wq; m++; }
        k = k1;
        if (c->ext_mode == OR_EXT_CONST) {
            in[m].f = 0; in[m].wq = c->ext_const_q; m++;
        } else {
            for (uint32_t e = 0; e < next; e++) { in[m].f = ext_offset(n, j, t, e); in[m].wq = n->tb.jext_q; m++; }
        }
        qsort(in, m, sizeof(or_in), in_cmp);
        double V = n->V[j], w = n->w[j];
        uint64_t now = t0, re = n->rend[j];
        const int exc = (j % module_size(c)) < c->n_exc;
        n->flag[j] = 0;
        for (size_t e = 0; e < m;) {
            const uint32_t f = in[e].f;
            int64_t J = 0;
            while (e < m && in[e].f == f) J += in[e++].wq;
            const uint64_t T = t0 | f;
            advance(c, now, T, re, &V, &w);
            now = T;
            if (T < re) continue;   /* refractory: input discarded */
            V += (double)J / 65536.0;
            int spike = forced ? (forced[j] && ff[j] == f) : (V > c->v_th);
            if (spike) {
                n->flag[j] = 1;
                n->fs[j] = f;
                V = c->v_reset;
                re = T + tref;
                if (exc || c->sfa_on_inh) w += c->alpha_w;
            }
        }
        advance(c, now, t1, re, &V, &w);
        n->V[j] = V;
        n->w[j] = w;
        n->rend[j] = re;
        /* whole steps of refractoriness left at the end of the step */
        n->ref[j] = re > t1 ? (int32_t)((re - t1 + 0xFFFFFFFFull) >> 32) : 0;
    }
    free(in);
    n->qn[slot] = 0;
    for (uint32_t i = 0; i < N; i++) {
        if (!n->flag[i]) continue;
        hist_push(n, t, i, n->fs[i]);
        n->n_spikes++;
        if (!n->built) continue;
        for (uint64_t s = n->row_ptr[i]; s < n->row_ptr[i + 1]; s++) {
            const or_syn *y = &n->syn[s];
            ev_push(n, (t + y->delay) % RING, y->tgt, n->fs[i], y->wq);
            n->rec_events++;
        }
    }
    n->t = t + 1;
    return n->overflow ? OR_E_OVERFLOW : OR_OK;
}

int or_net_step(void *h, uint32_t steps)
{
    or_net *n = (or_net *)h;
    for (uint32_t s = 0; s < steps; s++) {
        int st = n->c.solver == OR_SOLVER_EXACT ? step_exact(n, NULL, NULL) : step_once(n, NULL);
        if (st) return st;
    }
    return OR_OK;
}

/* Exact solver, lock-step mode: spikes (gids[k], at offset fr[k]) this step. */
int or_net_step_forced_exact(void *h, const uint32_t *gids, const uint32_t *fr, uint64_t cnt)
{
    or_net *n = (or_net *)h;
    if (n->c.solver != OR_SOLVER_EXACT) return OR_E_INVAL;
    uint8_t *forced = (uint8_t *)calloc(n->N, 1);
    uint32_t *ff = (uint32_t *)calloc(n->N, sizeof(uint32_t));
    if (!forced || !ff) { free(forced); free(ff); return OR_E_NOMEM; }
    int st = OR_OK;
    for (uint64_t k = 0; k < cnt; k++) {
        if (gids[k] >= n->N) { st = OR_E_INVAL; break; }
        forced[gids[k]] = 1;
        ff[gids[k]] = fr[k];
    }
    if (st == OR_OK) st = step_exact(n, forced, ff);
    free(forced);
    free(ff);
    return st;
}

/* Emission offsets of the history entries, in history order. */
uint64_t or_net_hist_frac(void *h, uint32_t *fr, uint64_t cap)
{
    or_net *n = (or_net *)h;
    uint64_t m = n->hist_n < cap ? n->hist_n : cap;
    if (fr) memcpy(fr, n->hist_f, (size_t)m * sizeof(uint32_t));
    return n->hist_n;
}

/* Queued inputs of arrival slot `slot`, ordered by (target, offset, charge):
 * returns their number; copies at most cap. */
uint64_t or_net_queue(void *h, uint32_t slot, uint32_t *tgt, uint32_t *fr, int32_t *wq, uint64_t cap)
{
    or_net *n = (or_net *)h;
    if (slot >= RING) return 0;
    const size_t m = n->qn[slot];
    if (m) qsort(n->q[slot], m, sizeof(or_ev), ev_cmp);
    for (size_t e = 0; e < m && e < cap; e++) {
        tgt[e] = n->q[slot][e].tgt;
        fr[e] = n->q[slot][e].f;
        wq[e] = n->q[slot][e].wq;
    }
    return m;
}

/* Exact solver: refractory ends, 32.32 fixed-point ms. */
int or_net_rend(void *h, uint64_t *re)
{
    or_net *n = (or_net *)h;
    memcpy(re, n->rend, n->N * sizeof(uint64_t));
    return OR_OK;
}

/* One step with a given spike set (ids need not be sorted). */
int or_net_step_forced(void *h, const uint32_t *gids, uint64_t cnt)
{
    or_net *n = (or_net *)h;
    uint8_t *forced = (uint8_t *)calloc(n->N, 1);
    if (!forced) return OR_E_NOMEM;
    for (uint64_t k = 0; k < cnt; k++) {
        if (gids[k] >= n->N) { free(forced); return OR_E_INVAL; }
        forced[gids[k]] = 1;
    }
    if (n->c.solver == OR_SOLVER_EXACT) { free(forced); return OR_E_INVAL; }
    int st = step_once(n, forced);
    free(forced);
    return st;
}

int or_net_state(void *h, double *V, double *w, int32_t *ref)
{
    or_net *n = (or_net *)h;
    if (V) memcpy(V, n->V, n->N * sizeof(double));
    if (w) memcpy(w, n->w, n->N * sizeof(double));
    if (ref) memcpy(ref, n->ref, n->N * sizeof(int32_t));
    return OR_OK;
}

int or_net_ring(void *h, int32_t *ring)
{
    or_net *n = (or_net *)h;
    memcpy(ring, n->ring, (size_t)RING * n->N * sizeof(int32_t));
    return OR_OK;
}

uint64_t or_net_hist(void *h, uint32_t *pairs, uint64_t cap)
{
    or_net *n = (or_net *)h;
    uint64_t m = n->hist_n < cap ? n->hist_n : cap;
    if (pairs) memcpy(pairs, n->hist, (size_t)m * 2 * sizeof(uint32_t));
    return n->hist_n;
}

void or_net_stats(void *h, uint64_t *out)
{
    or_net *n = (or_net *)h;
    out[0] = n->t;
    out[1] = n->n_spikes;
    out[2] = n->rec_events;
    out[3] = n->ext_events;
    out[4] = n->nnz;
    out[5] = (uint64_t)n->overflow;
}
