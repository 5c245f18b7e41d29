// stdp.hip -- gfx950 kernels of spike-timing plasticity (Sec. II: STDP with
// long-term potentiation and depression; Sec. II.A steps 1 and 4 give each
// pair's contribution at the later of its two events; the contributions of a
// period are integrated and applied to every synapse at its end).
//
// The contributions are integers (2^-16 mV per pair, from the kp / km lag
// tables), so summing them when the period ends gives exactly what summing
// them event by event would.  One application:
//   k_stdp_clear   per-neuron counters and cursors cleared
//   k_stdp_window  the AER history range of the steps whose spikes can pair
//                  in the period (binary search on the step-ordered history)
//   k_stdp_count   window spikes per neuron;   scan -> list offsets
//   k_stdp_place   each spike step into its neuron's list; excitatory
//                  neurons with spikes listed as the rows to visit
//   k_stdp_sort    each neuron's list in ascending step (insertion sort: a
//                  neuron has at most one spike per refractory period)
//   k_stdp_apply   one wave per (listed source, 256-record row segment): each
//                  lane takes a synapse, walks the source's arrivals against
//                  the target's spikes inside the window, and writes the
//                  clipped weight back when the total is not zero
// Bound by the gathers of the targets' spike lists and the record read and
// write: no MFMA.
#include "stdp_dev.h"

namespace snn {
namespace {

constexpr uint32_t kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_stdp_clear(StdpArgs a)
{
    const uint32_t i0 = blockIdx.x * kThreads + threadIdx.x;
    for (uint32_t i = i0; i < a.N; i += gridDim.x * kThreads) {
        a.cnt[i] = 0u;
        a.fill[i] = 0u;
    }
    if (i0 == 0) {
        *a.nact = 0u;
        a.off[0] = 0u;
    }
}

__global__ void k_stdp_window(StdpArgs a)
{
    if (threadIdx.x != 0) return;
    const uint64_t n = a.ctrl->hist_n;
    const uint64_t kept = n < a.hist_cap ? n : a.hist_cap;
    if (n > a.hist_cap) atomicOr(&a.ctrl->err, 8u);   // spikes were dropped: pairs would be missed
    uint64_t lo = 0, hi = kept;                        // first entry of step >= W0
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (a.hist[mid].x < a.W0) lo = mid + 1;
        else hi = mid;
    }
    a.range[0] = lo;
    a.range[1] = kept;
}

__global__ __launch_bounds__(kThreads) void k_stdp_count(StdpArgs a)
{
    const uint64_t h0 = a.range[0], h1 = a.range[1];
    for (uint64_t k = h0 + (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < h1; k += (uint64_t)gridDim.x * kThreads)
        atomicAdd(&a.cnt[a.hist[k].y], 1u);
}

__global__ __launch_bounds__(kThreads) void k_stdp_place(StdpArgs a)
{
    const uint64_t h0 = a.range[0], h1 = a.range[1];
    for (uint64_t k = h0 + (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < h1; k += (uint64_t)gridDim.x * kThreads) {
        const uint2 e = a.hist[k];
        const uint32_t p = atomicAdd(&a.fill[e.y], 1u);
        const uint64_t at = a.off[e.y] + p;
        if (at < a.times_cap) a.times[at] = e.x;
        else atomicOr(&a.ctrl->err, 8u);
        if (p == 0 && e.y % a.M < a.n_exc) a.act[atomicAdd(a.nact, 1u)] = e.y;
    }
}

__global__ __launch_bounds__(kThreads) void k_stdp_sort(StdpArgs a)
{
    for (uint32_t g = blockIdx.x * kThreads + threadIdx.x; g < a.N; g += gridDim.x * kThreads) {
        const uint64_t b = a.off[g];
        uint64_t e = a.off[g + 1];
        e = e < a.times_cap ? e : a.times_cap;
        for (uint64_t x = b + 1; x < e; ++x) {
            const uint32_t v = a.times[x];
            uint64_t y = x;
            while (y > b && a.times[y - 1] > v) {
                a.times[y] = a.times[y - 1];
                --y;
            }
            a.times[y] = v;
        }
    }
}

// Total change of one synapse of delay d from the source's spike list
// [s0, s1) (wave-uniform) and its target's list [q0, q1).
__device__ __forceinline__ int32_t pair_total(const StdpArgs& a, uint64_t s0, uint64_t s1, uint64_t q0, uint64_t q1,
                                              uint32_t d)
{
    int32_t acc = 0;
    uint64_t q = q0;   // first target spike with p + win > a (advances with a)
    for (uint64_t x = s0; x < s1; ++x) {
        const uint32_t arr = a.times[x] + d;
        if (arr >= a.T1) break;            // later arrivals belong to later periods
        while (q < q1 && a.times[q] + a.win <= arr) ++q;
        for (uint64_t y = q; y < q1; ++y) {
            const uint32_t p = a.times[y];
            if (p >= arr + a.win) break;
            if ((p > arr ? p : arr) < a.T0) continue;   // counted in an earlier period
            acc += p >= arr ? a.kp[p - arr] : -a.km[arr - p];
        }
    }
    return acc;
}

__global__ __launch_bounds__(kThreads) void k_stdp_apply(StdpArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const uint32_t nw = (gridDim.x * kThreads) >> 6;
    const uint64_t items = (uint64_t)(*a.nact) * a.smax;
    for (uint64_t it = wave; it < items; it += nw) {
        const uint32_t pre = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.act[it / a.smax]);
        const uint32_t seg = (uint32_t)(it % a.smax);
        const uint64_t rb = a.row_ptr[pre];
        const uint32_t len = (uint32_t)(a.row_ptr[pre + 1] - rb);
        const uint32_t c0 = seg * 256u;
        if (c0 >= len) continue;
        const uint64_t s0 = a.off[pre];
        uint64_t s1 = a.off[pre + 1];
        s1 = s1 < a.times_cap ? s1 : a.times_cap;
        const uint32_t be = lane < a.D ? (uint32_t)a.bend[(size_t)pre * a.D + lane] : 0xFFFFFFFFu;
        for (uint32_t u = 0; u < 4u; ++u) {
            const uint32_t c = c0 + 64u * u;
            if (c >= len) break;
            const uint32_t kk = c + lane;
            // delay bucket of record kk: the bucket ends not above it
            uint32_t bl = __popcll(__ballot(be <= c));
            uint64_t inm = __ballot(be > c && be < c + 64u);
            while (inm) {
                const uint32_t l = (uint32_t)__builtin_ctzll(inm);
                inm &= inm - 1u;
                bl += (kk >= (uint32_t)__builtin_amdgcn_readlane((int)be, (int)l)) ? 1u : 0u;
            }
            if (kk < len) {
                Rec8& r = a.recs[rb + kk];
                const uint32_t j = r.tgt & kTgtMask;   // (bl comes from the bucket ends)
                const uint64_t q0 = a.off[j];
                uint64_t q1 = a.off[j + 1];
                q1 = q1 < a.times_cap ? q1 : a.times_cap;
                const int32_t tot = q1 > q0 ? pair_total(a, s0, s1, q0, q1, a.d_min + bl) : 0;
                if (tot != 0) {
                    int64_t w = (int64_t)__float2int_rn(r.w * 65536.0f) + tot;
                    w = w < 0 ? 0 : (w > a.wmax_q ? a.wmax_q : w);
                    r.w = (float)w * 0x1p-16f;   // exact: |w| < 2^24
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_stdp_period(const StdpArgs& a, uint64_t* tile_sums, hipStream_t s)
{
    const uint32_t nb = (a.N + kThreads - 1) / kThreads;
    const uint32_t grid = nb < 4096 ? nb : 4096;
    hipLaunchKernelGGL(k_stdp_clear, dim3(grid), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_stdp_window, dim3(1), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_stdp_count, dim3(2048), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_rows(a.cnt, a.off, tile_sums, a.N, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stdp_place, dim3(2048), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_stdp_sort, dim3(grid), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_stdp_apply, dim3(4096), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace snn
