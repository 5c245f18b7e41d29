// tables.h -- host-side FP64 construction of a network's integer tables.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace snn {

struct HostTables {
    std::vector<uint32_t> T;     // [2][gy][gx] 32-bit connection thresholds per torus offset,
                                 // excitatory sources first, then inhibitory
    std::vector<int32_t> wtab;   // [65536] excitatory weights, 2^-16 mV
    std::vector<int32_t> cb;     // [256] 8-bit weight codebook, 2^-16 mV
    std::vector<uint32_t> poisc; // Poisson CDF thresholds of the external drive
    std::vector<uint32_t> dthr;  // exponential delays: D - 1 CDF thresholds of the delay bucket
    std::vector<uint32_t> btab;  // binomial generator: [2][gy][gx] x {k0, len, at lo, at hi}
    std::vector<uint32_t> bthr;  //   count thresholds of counts k0 .. k0 + len - 1 at bthr[at ..]
    double mean_out = 0.0;       // expected synapses per source, averaged over neurons
    double max_out = 0.0;        // the same for the busiest source type
    double dm = 0.0, dw = 0.0, kappa = 0.0;  // one-step propagator constants
    uint32_t nref = 0;           // refractory steps
    int32_t jext_q = 0, winh_q = 0;
    // spike-timing plasticity: change per pair at lag k (2^-16 mV), window, bound
    std::vector<int32_t> kp, km; // [win]; km[0] = 0
    uint32_t stdp_win = 0;
    int32_t wmax_q = 0;
};

struct TableParams {
    uint32_t gx, gy, M;          // grid and module size
    uint32_t kernel;             // 0 Gaussian, 1 exponential
    double range, k_in;
    uint32_t n_exc;              // excitatory neurons per module
    uint32_t preset;             // 0 one normalised law, 1 the paper's local + remote rules
    double p_local, amp, p_cut;  // paper preset parameters
    uint32_t gen;                // 0 one trial per pair, 1 binomial count + uniform subset
    uint32_t D;                  // delay buckets
    uint32_t delay_exp;          // 0 uniform delays, 1 exponential with scale delay_tau
    double delay_tau;
    double w_exc, w_exc_sd, w_inh;
    uint32_t ext_poisson;
    double ext_n, ext_rate_hz, ext_w;
    double tau_m, tau_w, t_ref;
    uint32_t stdp;               // 1: pair-based plasticity of excitatory synapses
    double a_plus, a_minus, tau_plus, tau_minus, w_max;
};

// Returns an empty string on success, else the reason the description is invalid.
std::string build_tables(const TableParams& p, HostTables& out);

// Connection thresholds only (T of HostTables), and the expected number of
// synapses a source projects, averaged over neurons and for the busiest
// source type.  Returns the reason on failure, like build_tables.
std::string connection_tables(const TableParams& p, std::vector<uint32_t>& T, double& mean_out,
                              double& max_out);

// Exposed for tests of the library's own normal quantile.
double inv_norm_cdf(double u);

}  // namespace snn
