// tables.h -- host-side FP64 construction of a network's integer tables.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace snn {

struct HostTables {
    std::vector<uint32_t> T;     // [gy][gx] 32-bit connection thresholds per torus offset
    std::vector<int32_t> wtab;   // [65536] excitatory weights, 2^-16 mV
    std::vector<int32_t> cb;     // [256] 8-bit weight codebook, 2^-16 mV
    std::vector<uint32_t> poisc; // Poisson CDF thresholds of the external drive
    double B = 0.0;              // probability prefactor
    double dm = 0.0, dw = 0.0, kappa = 0.0;  // one-step propagator constants
    uint32_t nref = 0;           // refractory steps
    int32_t jext_q = 0, winh_q = 0;
};

struct TableParams {
    uint32_t gx, gy, M;          // grid and module size
    uint32_t kernel;             // 0 Gaussian, 1 exponential
    double range, k_in;
    double w_exc, w_exc_sd, w_inh;
    uint32_t ext_poisson;
    double ext_n, ext_rate_hz, ext_w;
    double tau_m, tau_w, t_ref;
};

// Returns an empty string on success, else the reason the description is invalid.
std::string build_tables(const TableParams& p, HostTables& out);

// Exposed for tests of the library's own normal quantile.
double inv_norm_cdf(double u);

}  // namespace snn
