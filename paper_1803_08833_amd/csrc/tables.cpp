// tables.cpp -- FP64 host tables that turn the model's real-valued laws into the
// integer tables the kernels use.
//
//   * connection thresholds, per source type: p(offset) = B f(r) with f the
//     Gaussian exp(-r^2/2 sigma^2) or exponential exp(-r/lambda) lateral law
//     (Sec. I, Sec. III.B), B making the expected recurrent in-degree equal
//     to k_in ("fixes the total"); or the paper's own rules (Sec. III.B, Fig. 2
//     caption): p_local inside the module, amp f(r) elsewhere for excitatory
//     sources only, within the square stencil the 1/1000 cut-off gives;
//     stored as round(p * 2^32);
//   * excitatory weights: Gaussian efficacies (Sec. II.B) as the conditional
//     means of 65536 equiprobable bins (and of 255 bins for the 8-bit codebook);
//   * external drive: Poisson count per 1 ms step (Sec. III.A) by integer CDF
//     thresholds;
//   * neuron propagator: exact one-step solution of Eq. (1)-(2).
//
// Rounding is round-half-even everywhere; sums are taken in a fixed order
// (offset rows outer, columns inner; Poisson terms in increasing k) so that the
// integer tables are a deterministic function of the description.
#include "tables.h"

#include <cmath>

namespace snn {

namespace {

constexpr double kTwo32 = 4294967296.0;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;

double phi(double x) { return kInvSqrt2Pi * std::exp(-0.5 * x * x); }
double Phi(double x) { return 0.5 * std::erfc(-x * kInvSqrt2); }

// Lower-tail quantile (0 < u <= 0.5): the rational start of Abramowitz and
// Stegun 26.2.23 (|error| < 4.5e-4), then Newton steps on Phi.
double inv_lower(double u)
{
    const double t = std::sqrt(-2.0 * std::log(u));
    double x = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                         (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    for (int it = 0; it < 60; ++it) {
        const double dx = (Phi(x) - u) / phi(x);
        x -= dx;
        if (std::fabs(dx) <= 1e-17 * std::fmax(1.0, std::fabs(x))) break;
    }
    return x;
}

int32_t to_fixed(double mv) { return (int32_t)std::nearbyint(mv * 65536.0); }

// Mean of a standard normal restricted to the probability interval [u0, u1).
double bin_mean(double u0, double u1)
{
    const double a = inv_norm_cdf(u0), b = inv_norm_cdf(u1);
    const double pa = std::isinf(a) ? 0.0 : phi(a);
    const double pb = std::isinf(b) ? 0.0 : phi(b);
    return (pa - pb) / (u1 - u0);
}

int signed_offset(int raw, int g) { return 2 * raw <= g ? raw : raw - g; }

double lateral_law(uint32_t kernel, double range, int r2)
{
    if (kernel == 0) return std::exp(-(double)r2 / (2.0 * range * range));
    return std::exp(-std::sqrt((double)r2) / range);
}

}  // namespace

double inv_norm_cdf(double u)
{
    if (u <= 0.0) return -INFINITY;
    if (u >= 1.0) return INFINITY;
    if (u == 0.5) return 0.0;
    if (u > 0.5) return -inv_lower(1.0 - u);
    return inv_lower(u);
}

namespace {

// Half-width of the paper preset's square stencil: the first whole number of
// module spacings at or past the distance where amp f(r) falls to p_cut.
int stencil_half_width(const TableParams& p)
{
    if (!(p.amp > p.p_cut)) return 0;
    const double ratio = std::log(p.amp / p.p_cut);
    const double rc = p.kernel == 0 ? p.range * std::sqrt(2.0 * ratio) : p.range * ratio;
    return (int)std::ceil(rc);
}

std::string threshold(double prob, uint32_t& out)
{
    const double thr = std::nearbyint(prob * kTwo32);
    if (!(thr >= 0.0 && thr < kTwo32)) return "connection probability outside [0, 1)";
    out = (uint32_t)thr;
    return std::string();
}

}  // namespace

std::string connection_tables(const TableParams& p, std::vector<uint32_t>& T, double& mean_out, double& max_out)
{
    const int gx = (int)p.gx, gy = (int)p.gy;
    const size_t S = (size_t)gx * gy;
    T.assign(2 * S, 0u);
    std::string why;
    if (p.preset == 1) {
        if (!(p.p_local >= 0.0 && p.p_local < 1.0) || !(p.amp >= 0.0 && p.amp < 1.0) || !(p.p_cut > 0.0))
            return "paper preset needs 0 <= p_local < 1, 0 <= amp < 1 and p_cut > 0";
        const int h = stencil_half_width(p);
        for (int ry = 0; ry < gy; ++ry) {
            for (int rx = 0; rx < gx; ++rx) {
                const int dx = signed_offset(rx, gx), dy = signed_offset(ry, gy);
                double pe = 0.0, pi = 0.0;
                if (rx == 0 && ry == 0) pe = pi = p.p_local;
                else if (std::abs(dx) <= h && std::abs(dy) <= h) pe = p.amp * lateral_law(p.kernel, p.range, dx * dx + dy * dy);
                why = threshold(pe, T[(size_t)ry * gx + rx]);
                if (why.empty()) why = threshold(pi, T[S + (size_t)ry * gx + rx]);
                if (!why.empty()) return why;
            }
        }
    } else {
        double total = 0.0;
        for (int ry = 0; ry < gy; ++ry) {
            for (int rx = 0; rx < gx; ++rx) {
                const int dx = signed_offset(rx, gx), dy = signed_offset(ry, gy);
                const double cand = (rx == 0 && ry == 0) ? (double)p.M - 1.0 : (double)p.M;
                total += cand * lateral_law(p.kernel, p.range, dx * dx + dy * dy);
            }
        }
        const double B = p.k_in > 0.0 ? p.k_in / total : 0.0;
        for (int ry = 0; ry < gy; ++ry) {
            for (int rx = 0; rx < gx; ++rx) {
                const int dx = signed_offset(rx, gx), dy = signed_offset(ry, gy);
                why = threshold(B * lateral_law(p.kernel, p.range, dx * dx + dy * dy), T[(size_t)ry * gx + rx]);
                if (!why.empty()) return "connection probability reaches 1: k_in too large for this grid";
                T[S + (size_t)ry * gx + rx] = T[(size_t)ry * gx + rx];
            }
        }
    }
    // expected out-degree per source type: sum over offsets of candidates x p
    double out_deg[2] = {0.0, 0.0};
    for (int type = 0; type < 2; ++type)
        for (size_t o = 0; o < S; ++o)
            out_deg[type] += ((o == 0) ? (double)p.M - 1.0 : (double)p.M) * (double)T[type * S + o] / kTwo32;
    const double fe = p.M ? (double)p.n_exc / (double)p.M : 1.0;
    mean_out = fe * out_deg[0] + (1.0 - fe) * out_deg[1];
    max_out = std::max(p.n_exc ? out_deg[0] : 0.0, p.n_exc < p.M ? out_deg[1] : 0.0);
    return std::string();
}

// Binomial generator: for a (source type, offset) with threshold T > 0 and n
// candidates, the count thresholds round(2^32 F(k)) of Binomial(n, T / 2^32),
// F summed in increasing k from pmf(k) = exp(lgamma(n+1) - lgamma(k+1) -
// lgamma(n-k+1) + k log p + (n-k) log1p(-p)); leading counts whose threshold
// rounds to 0 are folded into k0, and the table ends before the first
// threshold that rounds to 2^32.
static void binomial_tables(const TableParams& p, HostTables& out)
{
    const size_t S = (size_t)p.gx * p.gy;
    out.btab.assign(4 * 2 * S, 0u);
    out.bthr.clear();
    for (size_t e = 0; e < 2 * S; ++e) {
        const uint64_t at = out.bthr.size();
        out.btab[4 * e + 2] = (uint32_t)at;
        out.btab[4 * e + 3] = (uint32_t)(at >> 32);
        const uint32_t T = out.T[e];
        if (T == 0) continue;
        const uint32_t n = (e % S == 0) ? p.M - 1 : p.M;
        const double pr = (double)T / 4294967296.0;
        const double lp = std::log(pr), lq = std::log1p(-pr), ln = std::lgamma((double)n + 1.0);
        double F = 0.0;
        uint32_t k0 = 0, len = 0;
        for (uint32_t k = 0; k <= n; ++k) {
            F += std::exp(ln - std::lgamma((double)k + 1.0) - std::lgamma((double)(n - k) + 1.0) + (double)k * lp +
                          (double)(n - k) * lq);
            const double q = std::nearbyint(F * kTwo32);
            if (q >= kTwo32) break;
            if (q <= 0.0) {
                ++k0;
                continue;
            }
            out.bthr.push_back((uint32_t)q);
            ++len;
        }
        out.btab[4 * e] = k0;
        out.btab[4 * e + 1] = len;
    }
}

std::string build_tables(const TableParams& p, HostTables& out)
{
    // --- connection thresholds -------------------------------------------
    std::string why = connection_tables(p, out.T, out.mean_out, out.max_out);
    if (!why.empty()) return why;
    if (p.gen > 1) return "unknown synapse generator";
    // --- exponential delays: P(bucket k) ~ exp(-k / tau), k < D, by CDF thresholds
    out.dthr.clear();
    if (p.delay_exp > 1) return "unknown delay distribution";
    if (p.delay_exp == 1) {
        if (!(p.delay_tau > 0.0)) return "exponential delays need delay_tau > 0";
        double total = 0.0;
        for (uint32_t k = 0; k < p.D; ++k) total += std::exp(-(double)k / p.delay_tau);
        double acc = 0.0;
        for (uint32_t k = 0; k + 1 < p.D; ++k) {
            acc += std::exp(-(double)k / p.delay_tau);
            const double q = std::nearbyint(acc / total * kTwo32);
            out.dthr.push_back(q >= kTwo32 ? 0xFFFFFFFFu : (uint32_t)q);
        }
    }
    if (p.gen == 1) {
        if (p.M > 4096) return "the binomial generator needs modules of at most 4096 neurons";
        binomial_tables(p, out);
    }
    // --- weights -----------------------------------------------------------
    out.wtab.resize(65536);
    for (int k = 0; k < 65536; ++k)
        out.wtab[k] = to_fixed(p.w_exc + p.w_exc_sd * bin_mean(k / 65536.0, (k + 1) / 65536.0));
    out.cb.resize(256);
    for (int k = 0; k < 255; ++k) {
        // draws u with floor(u * 255 / 2^32) == k start at ceil(k 2^32 / 255)
        const uint64_t lo = ((uint64_t)k << 32) / 255u + ((((uint64_t)k << 32) % 255u) ? 1u : 0u);
        const uint64_t hi = ((uint64_t)(k + 1) << 32) / 255u + ((((uint64_t)(k + 1) << 32) % 255u) ? 1u : 0u);
        out.cb[k] = to_fixed(p.w_exc + p.w_exc_sd * bin_mean((double)lo / kTwo32, (double)hi / kTwo32));
    }
    out.winh_q = to_fixed(p.w_inh);
    out.cb[255] = out.winh_q;
    // --- external drive ----------------------------------------------------
    out.poisc.clear();
    if (p.ext_poisson) {
        const double mean = p.ext_n * p.ext_rate_hz * 1e-3;
        double term = std::exp(-mean), cdf = term;
        bool done = false;
        for (int k = 0; k < 64; ++k) {
            if (k > 0) {
                term *= mean / (double)k;
                cdf += term;
            }
            const double thr = std::nearbyint(cdf * kTwo32);
            if (!(thr < kTwo32)) {
                done = true;
                break;
            }
            out.poisc.push_back((uint32_t)thr);
        }
        if (!done) return "external Poisson mean too large for a 64-entry CDF table";
    }
    out.jext_q = to_fixed(p.ext_w);
    // --- propagator (step h = 1 ms) ---------------------------------------
    const double h = 1.0;
    out.dm = -std::expm1(-h / p.tau_m);
    out.dw = -std::expm1(-h / p.tau_w);
    if (p.tau_w != p.tau_m)
        out.kappa = p.tau_w / (p.tau_w - p.tau_m) * (out.dm - out.dw);
    else
        out.kappa = (h / p.tau_m) * std::exp(-h / p.tau_m);
    out.nref = (uint32_t)std::llround(p.t_ref / h);
    // --- plasticity: one pair k steps apart, potentiating (spike not before
    // the arrival) or depressing (arrival after the spike), rounded to 2^-16 mV
    out.kp.clear();
    out.km.clear();
    out.stdp_win = 0;
    out.wmax_q = 0;
    if (p.stdp > 1) return "unknown plasticity mode";
    if (p.stdp) {
        if (!(p.a_plus >= 0.0 && p.a_minus >= 0.0)) return "plasticity amplitudes must be >= 0";
        if (!(p.tau_plus > 0.0 && p.tau_minus > 0.0)) return "plasticity time constants must be > 0";
        std::vector<int32_t> kp(256), km(256);
        uint32_t win = 0;
        for (uint32_t k = 0; k < 256; ++k) {
            kp[k] = to_fixed(p.a_plus * std::exp(-(double)k / p.tau_plus));
            km[k] = k == 0 ? 0 : to_fixed(p.a_minus * std::exp(-(double)k / p.tau_minus));
            if (kp[k] != 0 || km[k] != 0) win = k + 1;
        }
        if (win >= 256) return "plasticity window longer than 255 steps";
        out.kp.assign(kp.begin(), kp.begin() + win);
        out.km.assign(km.begin(), km.begin() + win);
        out.stdp_win = win;
        out.wmax_q = to_fixed(p.w_max);
    }
    return std::string();
}

}  // namespace snn
