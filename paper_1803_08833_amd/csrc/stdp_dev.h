// stdp_dev.h -- device side of spike-timing plasticity (Sec. II; Sec. II.A
// steps 1 and 4; the long-term application every period): arguments and
// launcher of the kernels in stdp.hip.
#pragma once
#include "snn_dev.h"

namespace snn {

constexpr uint32_t kStdpWinMax = 256;   // longest plasticity window, steps

// Everything one long-term application reads and writes.  The period covers
// steps [T0, T1); every pair of a presynaptic arrival a (spike of the source
// at s, a = s + delay) and a postsynaptic spike p with max(a, p) in the
// period and |p - a| < win changes the synapse's weight by kp[p - a] (p >= a)
// or -km[a - p] (p < a); a synapse whose total is not zero gets
// clamp(w + total, 0, wmax_q).  Spikes come from the AER history: those of
// steps [W0, T1), W0 = T0 - win + 1 - d_max (or 0), can take part.
struct StdpArgs {
    uint32_t N, M, n_exc, D, d_min;
    uint32_t win;
    int32_t wmax_q;
    uint32_t T0, T1, W0;
    uint32_t smax;              // 256-record segments of the longest row
    const uint2* hist;          // AER history (step, gid), ordered by step
    uint64_t hist_cap;
    Ctrl* ctrl;                 // hist_n read; err bit 3 set when the history overflowed
    uint64_t* range;            // [2] the window's history range (device scratch)
    uint32_t* cnt;              // [N] window spikes per neuron
    uint32_t* fill;             // [N] placement cursors
    uint64_t* off;              // [N + 1] each neuron's list start (scan of cnt)
    uint32_t* times;            // [times_cap] spike steps per neuron, ascending after the sort
    uint64_t times_cap;
    uint32_t* act;              // [N] excitatory neurons with window spikes
    uint32_t* nact;             // their number
    const uint64_t* row_ptr;    // [N + 1]
    const uint16_t* bend;       // [N][D]
    Rec8* recs;                 // F32 records: weights updated in place
    const int32_t* kp;          // [win]
    const int32_t* km;          // [win] (km[0] unused)
};

// Enqueue one long-term application on stream s.  tile_sums: the scan's
// scratch (scan_tiles(N) + 1 entries).
hipError_t launch_stdp_period(const StdpArgs& a, uint64_t* tile_sums, hipStream_t s);

}  // namespace snn
