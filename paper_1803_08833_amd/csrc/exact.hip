// exact.hip -- gfx950 kernels of the exact-time event-driven solver
// (Sec. II.A, Sec. II.C).
//
//   k_xs_count, k_xs_scan, k_xs_scatter, k_xs_group
//                the arriving slot's queued inputs, counting-sorted by target
//                (per target group in chunk histograms, then per neuron inside
//                each group), which also gives every neuron's offset
//   k_x_update   one thread per neuron: this step's inputs (queued and
//                external) in time order, Eq. (1)-(2) solved exactly between
//                them, a spike at the input that crosses threshold; ordered
//                spiker list per 256-neuron workgroup
//   k_x_update_busy
//                workgroups with many inputs: one wave per neuron in turn,
//                the inputs sorted in registers and every instant evaluated
//                at once in closed form
//   k_x_list     dense spike list of the step (each workgroup's place from the
//                counts of those before it), its AER history entries
//                (step, id, offset) and each spike's row bucket lengths
//   k_x_offsets  each spike's place in each delay bucket's arrival list (a
//                scan of the bucket lengths over the step's spikes)
//   k_x_deliver  one wave per (spike, 256-record row segment): fan-out into
//                the arrival slots' lists at those places, no atomics
//   k_x_finish   step counters (external events totalled over the workgroups)
//
// Like the step kernels this is bound by memory traffic and latency, not by
// arithmetic: no MFMA.
#include "exact_dev.h"

#include <hip/hip_ext.h>

namespace snn {
namespace {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the generator of the
// step kernels: ten rounds of two 32x32->64-bit products, key advanced by
// the Weyl increments.
__device__ __forceinline__ uint4 x_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t word(const uint4& r, uint32_t i)
{
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}

__device__ __forceinline__ uint32_t x_mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T x_wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One neuron's state while its inputs are taken in time order.
struct XNeuron {
    float V, W;
    uint64_t re;     // end of the refractory period
    uint64_t now;    // time the state refers to
    uint32_t spiked, fsp, dis;
};

// Advance from `now` to `to`: V held at V_r (w decaying) until the
// refractory period ends, then the exact solution of du/dt = -(u + w)/tau_m,
// dw/dt = -w/tau_w.  expm1 keeps the short intervals between inputs accurate.
__device__ __forceinline__ void x_advance(const XArgs& a, XNeuron& s, uint64_t to)
{
    uint64_t from = s.now;
    if (from < s.re) {
        const uint64_t e = s.re < to ? s.re : to;
        const float h = (float)(e - from) * 0x1p-32f;
        s.W = s.W + s.W * expm1f(-h * a.inv_tau_w);
        s.V = a.v_reset;
        from = e;
    }
    if (from < to) {
        const float h = (float)(to - from) * 0x1p-32f;
        const float xm = expm1f(-h * a.inv_tau_m), xw = expm1f(-h * a.inv_tau_w);
        const float kap = a.tau_equal ? h * a.inv_tau_m * (1.0f + xm) : a.ck * (xw - xm);
        float u = s.V - a.e_rest;
        u = u + u * xm - kap * s.W;
        s.V = a.e_rest + u;
        s.W = s.W + s.W * xw;
    }
    s.now = to;
}

// The inputs of one instant (offset f, summed charge J): discarded while
// refractory, else added and tested (lock-step: the forced decision).
__device__ __forceinline__ void x_input(const XArgs& a, XNeuron& s, uint64_t t0, uint32_t f, int32_t J, bool exc,
                                        bool forced, uint32_t ff)
{
    const uint64_t T = t0 | f;
    x_advance(a, s, T);
    if (T < s.re) return;
    s.V += (float)J * 0x1p-16f;
    const bool own = s.V > a.v_th;
    const bool spike = a.forced ? (forced && ff == f) : own;
    if (a.forced && own != spike) s.dis++;
    if (spike) {
        s.spiked = 1u;
        s.fsp = f;
        s.V = a.v_reset;
        s.re = T + a.tref_q;
        if (exc || a.sfa_on_inh) s.W += a.alpha;
    }
}

// In-place heap sort of one neuron's placed inputs by offset (the segment
// belongs to that neuron alone).  Every sift moves strictly down the heap, so
// each loop ends.
__device__ __forceinline__ void x_sift(uint2* v, uint32_t root, uint32_t n)
{
    const uint2 x = v[root];
    for (;;) {
        uint32_t c = 2u * root + 1u;
        if (c >= n) break;
        uint2 y = v[c];
        if (c + 1u < n) {
            const uint2 z = v[c + 1u];
            if (z.x > y.x) {
                ++c;
                y = z;
            }
        }
        if (y.x <= x.x) break;
        v[root] = y;
        root = c;
    }
    v[root] = x;
}

__device__ void x_heap_sort(uint2* v, uint32_t n)
{
    for (uint32_t r = n / 2u; r-- > 0u;) x_sift(v, r, n);
    for (uint32_t end = n; end-- > 1u;) {
        const uint2 top = v[0];
        v[0] = v[end];
        v[end] = top;
        x_sift(v, 0u, end);
    }
}

// Compare-exchange at distance JJ * 64 (pairs within a lane) of the bitonic
// merge of size k.
template <uint32_t K, uint32_t JJ>
__device__ __forceinline__ void x_cx_in_lane(uint64_t* v, uint32_t k)
{
    if constexpr (JJ < K) {
#pragma unroll
        for (uint32_t r = 0; r < K; ++r) {
            if (r & JJ) continue;
            const bool asc = ((r * 64u) & k) == 0u;
            const uint64_t x = v[r], y = v[r | JJ];
            const bool swap = (y < x) == asc;
            v[r] = swap ? y : x;
            v[r | JJ] = swap ? x : y;
        }
    }
}

// Bitonic sort (ascending) of 64 K 64-bit keys held by one wave, element
// r * 64 + lane in the lane's register r.  Distances below 64 exchange across
// lanes, larger ones within a lane.  The stages are loops, not unrolled, so
// that the code stays small enough for the instruction cache.
template <uint32_t K>
__device__ __forceinline__ void x_bitonic(uint64_t* v, uint32_t lane)
{
#pragma unroll 1
    for (uint32_t k = 2; k <= 64u * K; k <<= 1) {
#pragma unroll 1
        for (uint32_t jj = k >> 7; jj > 0; jj >>= 1) {
            if (jj == 1u) x_cx_in_lane<K, 1>(v, k);
            else if (jj == 2u) x_cx_in_lane<K, 2>(v, k);
            else if (jj == 4u) x_cx_in_lane<K, 4>(v, k);
            else x_cx_in_lane<K, 8>(v, k);
        }
#pragma unroll 1
        for (uint32_t j = (k >> 1) < 32u ? (k >> 1) : 32u; j > 0; j >>= 1) {
            // every partner is fetched before any is used, so the exchanges'
            // LDS round trips overlap instead of following one another
            const uint32_t src = (lane ^ j) << 2;
            uint32_t ylo[K], yhi[K];
#pragma unroll
            for (uint32_t r = 0; r < K; ++r) {
                ylo[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)src, (int)(uint32_t)v[r]);
                yhi[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)src, (int)(uint32_t)(v[r] >> 32));
            }
            const bool low = (lane & j) == 0u;
#pragma unroll
            for (uint32_t r = 0; r < K; ++r) {
                const uint64_t x = v[r], y = ((uint64_t)yhi[r] << 32) | ylo[r];
                const bool asc = ((r * 64u + lane) & k) == 0u;
                // keep the smaller of the two where this lane's element is the
                // lower one of an ascending pair or the upper one of a descending pair
                v[r] = ((x < y) == (asc == low)) ? x : y;
            }
        }
    }
}

// Arrival sort of the step's slot (its inputs in delivery order) by target,
// in three passes and no device atomic per input.  1: each workgroup counts
// its contiguous chunk of the list per target group in LDS and adds the
// nonzero counts to the group totals.  2: one workgroup scans the totals.
// 3: each workgroup counts its chunk again, reserves each group's share at
// the group's cursor and writes every input there (its place among the
// chunk's inputs of the group from an LDS counter).  4: one workgroup per
// group counts the group's inputs per neuron in LDS, writes the neurons'
// offsets and places the {offset, charge} pairs by neuron.  Within one
// target the order is arbitrary: the update sorts by offset.
__device__ __forceinline__ void x_chunk(const XArgs& a, uint64_t& c0, uint64_t& c1, const uint4*& L)
{
    const uint32_t slot = a.ctrl->t0 % a.R;   // the step in flight (k_x_finish advances it)
    const uint64_t n0 = a.qn[slot];
    const uint64_t n = n0 < a.qcap ? n0 : a.qcap;
    // chunks of at least kXChunkMin inputs: a short list leaves most
    // workgroups idle instead of each sweeping its LDS histogram
    uint64_t per = (n + gridDim.x - 1u) / gridDim.x;
    per = per < kXChunkMin ? kXChunkMin : per;
    c0 = (uint64_t)blockIdx.x * per;
    c0 = c0 < n ? c0 : n;
    c1 = c0 + per < n ? c0 + per : n;
    L = a.qlist + (size_t)slot * a.qcap;
}

__global__ __launch_bounds__(256) void k_xs_count(XArgs a)
{
    __shared__ uint32_t h[kXGroups];
    uint64_t c0, c1;
    const uint4* L;
    x_chunk(a, c0, c1, L);
    if (c0 >= c1) return;   // (uniform) an empty chunk
    for (uint32_t i = threadIdx.x; i < a.ngroups; i += 256u) h[i] = 0u;
    __syncthreads();
    for (uint64_t e0 = c0 + threadIdx.x; e0 < c1; e0 += 4u * 256u) {
        uint32_t x[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {   // every load in flight before any count
            const uint64_t e = e0 + 256u * u;
            x[u] = e < c1 ? L[e].x : ~0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
            if (x[u] < a.N) atomicAdd(&h[x[u] >> a.gbits], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < a.ngroups; i += 256u)
        if (h[i]) atomicAdd(a.gcnt + i, h[i]);
}

__global__ __launch_bounds__(1024) void k_xs_scan(XArgs a)
{
    __shared__ uint64_t wsum[16];
    // thread i holds groups 4i .. 4i + 3 (ngroups <= kXGroups = 4 x 1024)
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint32_t c[4];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t g = 4u * tid + u;
        c[u] = g < a.ngroups ? a.gcnt[g] : 0u;
        sum += c[u];
    }
    uint64_t inc = sum;
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63u) wsum[wv] = inc;
    __syncthreads();
    uint64_t off = inc - sum;
    for (uint32_t w = 0; w < wv; ++w) off += wsum[w];
#pragma unroll
    for (uint32_t u = 0; u < 4; ++u) {
        const uint32_t g = 4u * tid + u;
        if (g < a.ngroups) {
            a.goff[g] = off;
            a.gcur[g] = off;
            a.gcnt[g] = 0u;   // zero for the next step
        }
        if (g == a.ngroups) a.goff[g] = off;
        off += c[u];
    }
    if (tid == 1023u && a.ngroups == kXGroups) a.goff[kXGroups] = off;
}

__global__ __launch_bounds__(256) void k_xs_scatter(XArgs a)
{
    __shared__ uint32_t h[kXGroups];
    __shared__ unsigned long long base[kXGroups];
    uint64_t c0, c1;
    const uint4* L;
    x_chunk(a, c0, c1, L);
    if (c0 >= c1) return;   // (uniform) an empty chunk
    for (uint32_t i = threadIdx.x; i < a.ngroups; i += 256u) h[i] = 0u;
    __syncthreads();
    for (uint64_t e0 = c0 + threadIdx.x; e0 < c1; e0 += 4u * 256u) {
        uint32_t x[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t e = e0 + 256u * u;
            x[u] = e < c1 ? L[e].x : ~0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
            if (x[u] < a.N) atomicAdd(&h[x[u] >> a.gbits], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < a.ngroups; i += 256u) {
        base[i] = h[i] ? atomicAdd(a.gcur + i, (unsigned long long)h[i]) : 0ull;
        h[i] = 0u;
    }
    __syncthreads();
    unsigned long long bad = 0;
    for (uint64_t e0 = c0 + threadIdx.x; e0 < c1; e0 += 4u * 256u) {
        uint4 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t e = e0 + 256u * u;
            v[u] = e < c1 ? L[e] : make_uint4(~0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            if (e0 + 256u * u >= c1) continue;
            if (v[u].x >= a.N) {   // cannot happen: delivery writes only targets < N
                ++bad;
                continue;
            }
            const uint32_t g = v[u].x >> a.gbits;
            a.qtmp[base[g] + atomicAdd(&h[g], 1u)] = v[u];
        }
    }
    if (bad) atomicAdd(a.dropped, bad);
}

__global__ __launch_bounds__(256) void k_xs_group(XArgs a)
{
    __shared__ uint32_t c[1u << kXGroupBitsMax];
    __shared__ uint32_t wsum[4];
    const uint32_t g = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t j0 = g << a.gbits;
    const uint32_t gs = 1u << a.gbits;
    const uint32_t nj = a.N - j0 < gs ? a.N - j0 : gs;
    const uint64_t lo = a.goff[g], hi = a.goff[g + 1];
    for (uint32_t i = tid; i < nj; i += 256u) c[i] = 0u;
    __syncthreads();
    for (uint64_t e0 = lo + tid; e0 < hi; e0 += 4u * 256u) {
        uint32_t x[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t e = e0 + 256u * u;
            x[u] = e < hi ? a.qtmp[e].x - j0 : ~0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
            if (x[u] < nj) atomicAdd(&c[x[u]], 1u);
    }
    __syncthreads();
    // exclusive scan of the nj <= 4096 counts: thread i holds 16 in a row
    const uint32_t per = (nj + 255u) / 256u;
    const uint32_t b0 = tid * per;
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per; ++i)
        if (b0 + i < nj) sum += c[b0 + i];
    uint32_t inc = sum;
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63u) wsum[wv] = inc;
    __syncthreads();
    uint32_t off = inc - sum;
    for (uint32_t w = 0; w < wv; ++w) off += wsum[w];
    for (uint32_t i = 0; i < per; ++i) {
        if (b0 + i >= nj) break;
        const uint32_t k = c[b0 + i];
        a.qoff[j0 + b0 + i] = lo + off;
        c[b0 + i] = off;   // the neuron's fill cursor
        off += k;
    }
    if (j0 + nj == a.N && tid == 255u) a.qoff[a.N] = hi;
    __syncthreads();
    for (uint64_t e0 = lo + tid; e0 < hi; e0 += 4u * 256u) {
        uint4 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint64_t e = e0 + 256u * u;
            v[u] = e < hi ? a.qtmp[e] : make_uint4(~0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t x = v[u].x - j0;
            if (e0 + 256u * u < hi && x < nj) a.qsorted[lo + atomicAdd(&c[x], 1u)] = make_uint2(v[u].y, v[u].z);
        }
    }
}

// What one neuron's step takes besides its queued inputs.
struct XIn {
    uint32_t j, t, next;    // neuron, step, external inputs this step
    int32_t jext;           // charge of one external input
    bool exc, forced;       // excitatory; lock-step flag
    uint32_t ff;            // lock-step offset
    uint64_t t0;            // the step's start, 32.32 fixed point
};

// The external inputs of the step in the lane's LDS slots e[i * kXBlock],
// i < next <= kXLocal, sorted by offset.
__device__ __forceinline__ void x_ext_sorted(const XArgs& a, const XIn& in, uint2* e)
{
    for (uint32_t i = 0; i < in.next; i += 4) {
        const uint4 r = a.ext_const ? make_uint4(0u, 0u, 0u, 0u)
                                    : x_philox(in.j, in.t, kStreamExtTime, i >> 2, a.key0, a.key1);
        for (uint32_t q = 0; q < 4 && i + q < in.next; ++q)
            e[(i + q) * kXBlock] = make_uint2(word(r, q), (uint32_t)in.jext);
    }
    for (uint32_t i = 1; i < in.next; ++i) {
        const uint2 x = e[i * kXBlock];
        uint32_t p = i;
        while (p > 0 && e[(p - 1) * kXBlock].x > x.x) {
            e[p * kXBlock] = e[(p - 1) * kXBlock];
            --p;
        }
        e[p * kXBlock] = x;
    }
}

// Many queued inputs: heap-sort the neuron's own slice seg[0 .. nrec) in
// place (unless a wave has sorted it already), hold its external inputs
// sorted in its LDS slots, and take the two in time order, inputs of one
// instant together.
__device__ __forceinline__ void x_take_merged(const XArgs& a, XNeuron& s, const XIn& in, uint2* seg,
                                              uint32_t nrec, uint2* e, bool sorted)
{
    if (!sorted) x_heap_sort(seg, nrec);
    x_ext_sorted(a, in, e);
    uint32_t ir = 0, ie = 0;
    while (ir < nrec || ie < in.next) {
        const uint64_t fr = ir < nrec ? (uint64_t)seg[ir].x : (1ull << 32);
        const uint64_t fe = ie < in.next ? (uint64_t)e[ie * kXBlock].x : (1ull << 32);
        const uint32_t f = (uint32_t)(fr < fe ? fr : fe);
        int32_t J = 0;
        while (ir < nrec && seg[ir].x == f) J += (int32_t)seg[ir++].y;
        while (ie < in.next && e[ie * kXBlock].x == f) J += (int32_t)e[ie++ * kXBlock].y;
        x_input(a, s, in.t0, f, J, in.exc, in.forced, in.ff);
    }
}

// More external inputs than the LDS slots (a drive far above any workload's):
// the earliest remaining instant each time.
__device__ __forceinline__ void x_take_selected(const XArgs& a, XNeuron& s, const XIn& in, const uint2* seg,
                                                uint32_t nrec)
{
    uint64_t lo = 0;
    while (lo <= 0xFFFFFFFFull) {
        uint64_t best = 1ull << 32;
        int32_t J = 0;
        for (uint32_t i = 0; i < nrec; ++i) {
            const uint2 x = seg[i];
            if (x.x < lo) continue;
            if (x.x < best) {
                best = x.x;
                J = (int32_t)x.y;
            } else if (x.x == best) {
                J += (int32_t)x.y;
            }
        }
        for (uint32_t i = 0; i < in.next; i += 4) {
            const uint4 r = a.ext_const ? make_uint4(0u, 0u, 0u, 0u)
                                        : x_philox(in.j, in.t, kStreamExtTime, i >> 2, a.key0, a.key1);
            for (uint32_t q = 0; q < 4 && i + q < in.next; ++q) {
                const uint32_t f = word(r, q);
                if (f < lo) continue;
                if (f < best) {
                    best = f;
                    J = in.jext;
                } else if (f == best) {
                    J += in.jext;
                }
            }
        }
        if (best > 0xFFFFFFFFull) break;
        x_input(a, s, in.t0, (uint32_t)best, J, in.exc, in.forced, in.ff);
        lo = best + 1;
    }
}

// What a wave's update of one neuron hands back (the same in every lane).
struct XWaveOut {
    float V, W;
    uint64_t re;
    uint32_t spiked, fsp, dis;
};

// One neuron's step by a whole wave, in closed form (Eq. (1)-(2)).  Its n
// queued inputs (seg) and its external inputs are sorted together
// by offset (a bitonic network over {offset, charge} packed as 64-bit keys;
// padding sorts last and is never taken).  From the start Ts (the step's
// start, or the end of a refractory period inside the step; earlier inputs
// are discarded) until the neuron spikes, w decays freely and u = V - E is
// linear in the inputs: after the inputs up to instant T_k,
//   u_k = e^{-h_k/tau_m} (u_s + sum_{i<=k} J_i e^{(T_i - Ts)/tau_m}) - kappa(h_k) w_s,
// h_k = T_k - Ts, kappa(h) = ck (e^{-h/tau_w} - e^{-h/tau_m}) (h/tau_m e^{-h/tau_m}
// when tau_w = tau_m), so every instant is evaluated at once from a prefix sum
// over the sorted inputs (summed in double; the per-input decay factors in
// single precision, the end-of-step state in double).  Inputs of one instant
// are summed before the threshold test, which takes place at the last input
// of each instant.
// The spike is the first instant above threshold (lock-step: the forced
// instant; disagreements are counted up to it); the refractory period (at
// least 1 ms) then covers the rest of the step.
template <uint32_t K>
__device__ __forceinline__ void x_wave_neuron(const XArgs& a, const uint2* seg, uint32_t n, const XIn& in,
                                              float V0, float W0, uint64_t re0, uint32_t lane, XWaveOut& o)
{
    const uint32_t nall = n + in.next;
    uint64_t v[K];
#pragma unroll
    for (uint32_t r = 0; r < K; ++r) {
        const uint32_t i = r * 64u + lane;
        uint2 x = make_uint2(~0u, ~0u);
        if (i < n) {
            x = seg[i];
        } else if (i < nall) {
            const uint32_t e = i - n;
            const uint32_t f =
                a.ext_const ? 0u : word(x_philox(in.j, in.t, kStreamExtTime, e >> 2, a.key0, a.key1), e & 3u);
            x = make_uint2(f, (uint32_t)in.jext);
        }
        v[r] = ((uint64_t)x.x << 32) | x.y;
    }
    x_bitonic<K>(v, lane);

    const uint64_t t0 = in.t0, t1 = t0 + (1ull << 32);
    const double dt = 0x1p-32;   // ms per unit of the 32.32 times
    const bool held = re0 > t0;
    const uint64_t Ts = held ? (re0 < t1 ? re0 : t1) : t0;
    const double us = held ? a.dv_reset - a.de_rest : (double)V0 - a.de_rest;
    const double ws = held ? (double)W0 * exp(-(double)(Ts - t0) * dt * a.dinv_tau_w) : (double)W0;
    o.re = re0;
    o.spiked = 0u;
    o.fsp = 0u;
    o.dis = 0u;
    if (Ts >= t1) {   // (uniform) refractory for the whole step: every input is discarded
        o.V = a.v_reset;
        o.W = (float)ws;
        return;
    }
    // the decay factors of one input or instant (h in ms, at most 1) in
    // single precision: each multiplies a term that is then summed in double
    const float fm = a.inv_tau_m, fw = a.inv_tau_w, fck = a.ck;
    auto kappa = [&](float h, float em) {
        return a.tau_equal ? h * fm * em : fck * (expf(-h * fw) - em);
    };
    // prefix sums of the decay-weighted charges, in sorted order: a wave scan
    // of every register at once (their shuffles overlap), then the carries
    double P[K];
    uint32_t F[K];
#pragma unroll
    for (uint32_t r = 0; r < K; ++r) {
        const uint32_t i = r * 64u + lane;
        F[r] = (uint32_t)(v[r] >> 32);
        const uint64_t T = t0 | F[r];
        const bool valid = i < nall && T >= Ts;
        const float g = expf((float)(T - Ts) * 0x1p-32f * fm);
        P[r] = valid ? (double)(int32_t)(uint32_t)v[r] * 0x1p-16 * (double)g : 0.0;
    }
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        double y[K];
#pragma unroll
        for (uint32_t r = 0; r < K; ++r) y[r] = __shfl_up(P[r], d);
#pragma unroll
        for (uint32_t r = 0; r < K; ++r)
            if (lane >= d) P[r] += y[r];
    }
    double carry = 0.0;
#pragma unroll
    for (uint32_t r = 0; r < K; ++r) {
        P[r] += carry;
        carry = __shfl(P[r], 63);
    }
    // threshold tests at the last input of each instant
    bool found = false, ffound = false;
    uint32_t fstar = 0u, fidx = ~0u;
    bool own[K], test[K];
#pragma unroll
    for (uint32_t r = 0; r < K; ++r) {
        const uint32_t i = r * 64u + lane;
        const uint64_t T = t0 | F[r];
        uint32_t fn = __shfl_down(F[r], 1u);
        const uint32_t f0 = r + 1u < K ? (uint32_t)__builtin_amdgcn_readlane((int)F[r + 1u < K ? r + 1u : r], 0) : 0u;
        if (lane == 63u) fn = f0;
        test[r] = i < nall && T >= Ts && (i + 1u >= nall || fn != F[r]);
        const float h = (float)(T - Ts) * 0x1p-32f;
        const float em = expf(-h * fm);
        const double u = (double)em * (us + P[r]) - (double)kappa(h, em) * ws;
        own[r] = test[r] && a.de_rest + u > a.dv_th;
        const uint64_t m = __ballot(own[r]);
        if (!found && m) {
            found = true;
            const int l = __builtin_ctzll(m);
            fstar = (uint32_t)__builtin_amdgcn_readlane((int)F[r], l);
        }
        if (a.forced) {
            const uint64_t mf = __ballot(test[r] && in.forced && F[r] == in.ff);
            if (!ffound && mf) {
                ffound = true;
                fidx = r * 64u + (uint32_t)__builtin_ctzll(mf);
            }
        }
    }
    if (a.forced) {
        // lock-step: the spike is the forced instant; an instant up to it
        // whose own decision differs from the forced one is a disagreement
        uint32_t dis = 0;
#pragma unroll
        for (uint32_t r = 0; r < K; ++r) {
            const uint32_t i = r * 64u + lane;
            dis += (uint32_t)__popcll(__ballot(test[r] && i <= fidx && own[r] != (i == fidx)));
        }
        o.dis = dis;
        found = ffound;
        fstar = in.ff;
    }
    if (found) {
        const uint64_t Tsp = t0 | fstar;
        double w = ws * exp(-(double)(Tsp - Ts) * dt * a.dinv_tau_w);
        if (in.exc || a.sfa_on_inh) w += a.dalpha;
        o.spiked = 1u;
        o.fsp = fstar;
        o.re = Tsp + a.tref_q;   // >= t1: held to the end of the step
        o.V = a.v_reset;
        o.W = (float)(w * exp(-(double)(t1 - Tsp) * dt * a.dinv_tau_w));
    } else {
        const double h = (double)(t1 - Ts) * dt;
        const double em = exp(-h * a.dinv_tau_m), ew = exp(-h * a.dinv_tau_w);
        const double kap = a.tau_equal ? h * a.dinv_tau_m * em : a.dck * (ew - em);
        o.V = (float)(a.de_rest + em * (us + carry) - kap * ws);
        o.W = (float)(ws * ew);
    }
}

// (n + next wave-uniform, at most kXWaveSort)
__device__ __forceinline__ void x_wave_neuron_any(const XArgs& a, const uint2* seg, uint32_t n, const XIn& in,
                                                  float V0, float W0, uint64_t re0, uint32_t lane, XWaveOut& o)
{
    const uint32_t nall = n + in.next;
    if (nall <= 64u) x_wave_neuron<1>(a, seg, n, in, V0, W0, re0, lane, o);
    else if (nall <= 128u) x_wave_neuron<2>(a, seg, n, in, V0, W0, re0, lane, o);
    else if (nall <= 256u) x_wave_neuron<4>(a, seg, n, in, V0, W0, re0, lane, o);
    else if (nall <= 512u) x_wave_neuron<8>(a, seg, n, in, V0, W0, re0, lane, o);
    else x_wave_neuron<16>(a, seg, n, in, V0, W0, re0, lane, o);
}

// A workgroup whose queued inputs average more than kXBusyPer per neuron is
// updated by k_x_update_busy (its inputs are contiguous in qsorted); both
// kernels take the same decision from the same two offsets.
__device__ __forceinline__ uint64_t x_block_inputs(const XArgs& a)
{
    const uint32_t first = blockIdx.x * kXBlock;
    const uint32_t last = first + kXBlock < a.N ? first + kXBlock : a.N;
    uint64_t lo = a.qoff[first], hi = a.qoff[last];
    hi = hi < a.qcap ? hi : a.qcap;
    lo = lo < hi ? lo : hi;
    return hi - lo;
}

__device__ __forceinline__ bool x_block_busy(const XArgs& a)
{
    return x_block_inputs(a) > (uint64_t)kXBusyPer * kXBlock;
}

// The end of an update workgroup: its spikers in ascending id, its spike and
// external-event totals (added up later: no shared counter here).
__device__ __forceinline__ void x_close_block(const XArgs& a, uint32_t j, uint32_t spiked, uint32_t next,
                                              uint32_t dis, uint32_t* wcnt, unsigned long long* wext,
                                              unsigned long long* wdis)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    // spikers of the workgroup in ascending id
    const uint64_t m = __ballot(spiked != 0u);
    // external events count Poisson inputs only (the constant drive is no event)
    const unsigned long long we = x_wave_sum<unsigned long long>(a.ext_const ? 0u : next);
    const unsigned long long wd = x_wave_sum<unsigned long long>(dis);
    if (lane == 0) {
        wcnt[wv] = (uint32_t)__popcll(m);
        wext[wv] = we;
        wdis[wv] = wd;
    }
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t w = 0; w < kXBlock / 64; ++w) {
        if (w < wv) off += wcnt[w];
        tot += wcnt[w];
    }
    if (spiked) a.blk_list[(size_t)blockIdx.x * kXBlock + off + x_mbcnt(m)] = j;
    if (tid == 0) {
        // per-workgroup totals, added up by k_x_list and k_x_finish (no shared counter here)
        a.blk_cnt[blockIdx.x] = tot;
        unsigned long long ex = 0, ds = 0;
        for (uint32_t w = 0; w < kXBlock / 64; ++w) {
            ex += wext[w];
            ds += wdis[w];
        }
        a.blk_ext[blockIdx.x] = (uint32_t)ex;
        if (ds) atomicAdd((unsigned long long*)&a.ctrl->disagree, ds);   // lock-step only
    }
}

__global__ __launch_bounds__(kXBlock) void k_x_update(XArgs a)
{
    const uint32_t t = a.ctrl->t0;
    __shared__ uint2 ev_s[kXLocal * kXBlock];   // [input][thread]
    __shared__ uint32_t pois_s[kMaxPois];
    __shared__ uint32_t wcnt[kXBlock / 64];
    __shared__ unsigned long long wext[kXBlock / 64], wdis[kXBlock / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t j = blockIdx.x * kXBlock + tid;
    const bool live = j < a.N;
    if (blockIdx.x == 0 && tid == 0) {
        a.qn[t % a.R] = 0;   // the slot's list has been placed
        for (uint32_t s = 0; s < a.R; ++s) a.qn_prev[s] = a.qn[s];   // before this step's delivery
    }
    if (x_block_busy(a)) return;   // (uniform) the workgroup is k_x_update_busy's
    // the neuron's loads go out before the barrier, which then waits for them
    // and for the table load together
    uint64_t k0 = 0, k1 = 0, re0 = 0;
    float V0 = 0.f, W0 = 0.f;
    if (live) {
        k0 = a.qoff[j];
        k1 = a.qoff[j + 1];
        V0 = a.V[j];
        W0 = a.W[j];
        re0 = a.rend[j];
    }
    if (tid < a.npois) pois_s[tid] = a.poisc[tid];
    __syncthreads();
    const uint64_t t0 = (uint64_t)t << 32, t1 = t0 + (1ull << 32);
    uint32_t spiked = 0, next = 0, dis = 0;
    if (live) {
        k1 = k1 < a.qcap ? k1 : a.qcap;
        k0 = k0 < k1 ? k0 : k1;
        const uint32_t nrec = (uint32_t)(k1 - k0);
        if (a.ext_const) {
            next = 1;
        } else {
            const uint32_t u = word(x_philox(j >> 2, t, kStreamExt, 0u, a.key0, a.key1), j & 3u);
            for (uint32_t i = 0; i < a.npois; ++i) next += pois_s[i] <= u ? 1u : 0u;
        }
        const int32_t jext = a.ext_const ? a.ext_const_q : a.jext_q;
        XNeuron s{V0, W0, re0, t0, 0u, 0u, 0u};
        const bool exc = (j % a.M) < a.n_exc;
        const bool fj = a.forced ? a.forced[j] != 0 : false;
        const uint32_t ff = a.forced ? a.forced_f[j] : 0u;
        const XIn in{j, t, next, jext, exc, fj, ff, t0};
        const uint32_t n = nrec + next;
        if (n <= kXLocal) {
            uint2* e = ev_s + tid;   // input i at e[i * kXBlock]
            for (uint32_t i = 0; i < nrec; ++i) e[i * kXBlock] = a.qsorted[k0 + i];
            for (uint32_t i = 0; i < next; i += 4) {
                const uint4 r = a.ext_const ? make_uint4(0u, 0u, 0u, 0u)
                                            : x_philox(j, t, kStreamExtTime, i >> 2, a.key0, a.key1);
                for (uint32_t q = 0; q < 4 && i + q < next; ++q)
                    e[(nrec + i + q) * kXBlock] = make_uint2(word(r, q), (uint32_t)jext);
            }
            for (uint32_t i = 1; i < n; ++i) {   // insertion sort by offset
                const uint2 x = e[i * kXBlock];
                uint32_t p = i;
                while (p > 0 && e[(p - 1) * kXBlock].x > x.x) {
                    e[p * kXBlock] = e[(p - 1) * kXBlock];
                    --p;
                }
                e[p * kXBlock] = x;
            }
            for (uint32_t i = 0; i < n;) {
                const uint32_t f = e[i * kXBlock].x;
                int32_t J = 0;
                while (i < n && e[i * kXBlock].x == f) {
                    J += (int32_t)e[i * kXBlock].y;
                    ++i;
                }
                x_input(a, s, t0, f, J, exc, fj, ff);
            }
        } else if (next <= kXLocal) {
            x_take_merged(a, s, in, a.qsorted + k0, nrec, ev_s + tid, false);
        } else {
            x_take_selected(a, s, in, a.qsorted + k0, nrec);
        }
        x_advance(a, s, t1);
        a.V[j] = s.V;
        a.W[j] = s.W;
        a.rend[j] = s.re;
        if (s.spiked) a.fs[j] = s.fsp;
        spiked = s.spiked;
        dis = s.dis;
    }
    x_close_block(a, j, spiked, next, dis, wcnt, wext, wdis);
}

// Busy workgroups: each wave updates its own 64 neurons one at a time with
// all its lanes, in closed form (x_wave_neuron, the slice read coalesced
// straight from qsorted into registers; at most kXWaveSort inputs with the
// external ones).  No LDS window, so two workgroups share a CU and one's
// loads overlap the other's shuffles.  A neuron with more inputs is updated
// by its own lane, which heap-sorts its slice where it lies, holds its
// external inputs sorted in its LDS slots, merges the two and integrates
// input by input.
__global__ __launch_bounds__(kXBlock) void k_x_update_busy(XArgs a)
{
    __shared__ uint2 ev_s[kXLocal * kXBlock];    // external inputs [input][thread]
    __shared__ uint32_t pois_s[kMaxPois];
    __shared__ uint32_t wcnt[kXBlock / 64];
    __shared__ unsigned long long wext[kXBlock / 64], wdis[kXBlock / 64];
    if (!x_block_busy(a)) return;   // (uniform) the workgroup is k_x_update's
    const uint32_t t = a.ctrl->t0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t j = blockIdx.x * kXBlock + tid;
    const bool live = j < a.N;
    uint64_t k0 = 0, k1 = 0, re0 = 0;
    float V0 = 0.f, W0 = 0.f;
    if (live) {
        k0 = a.qoff[j];
        k1 = a.qoff[j + 1];
        V0 = a.V[j];
        W0 = a.W[j];
        re0 = a.rend[j];
    }
    if (tid < a.npois) pois_s[tid] = a.poisc[tid];
    __syncthreads();
    const uint64_t t0 = (uint64_t)t << 32, t1 = t0 + (1ull << 32);
    uint32_t spiked = 0, next = 0, dis = 0;
    k1 = k1 < a.qcap ? k1 : a.qcap;
    k0 = k0 < k1 ? k0 : k1;
    const uint32_t nrec = (uint32_t)(k1 - k0);
    if (live) {
        if (a.ext_const) {
            next = 1;
        } else {
            const uint32_t u = word(x_philox(j >> 2, t, kStreamExt, 0u, a.key0, a.key1), j & 3u);
            for (uint32_t i = 0; i < a.npois; ++i) next += pois_s[i] <= u ? 1u : 0u;
        }
    }
    const int32_t jext = a.ext_const ? a.ext_const_q : a.jext_q;
    const bool exc = (j % a.M) < a.n_exc;
    const bool fj = (live && a.forced) ? a.forced[j] != 0 : false;
    const uint32_t ff = (live && a.forced) ? a.forced_f[j] : 0u;
    const bool coop = live && nrec + next <= kXWaveSort;
    // (uniform) this wave's neurons, one at a time with every lane
    for (uint64_t m = __ballot(coop); m; m &= m - 1ull) {
        const int l = __builtin_ctzll(m);
        const uint64_t k0_l = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(k0 >> 32), l) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k0, l);
        const uint64_t re_l = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(re0 >> 32), l) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)re0, l);
        const XIn in_l{(uint32_t)__builtin_amdgcn_readlane((int)j, l), t,
                       (uint32_t)__builtin_amdgcn_readlane((int)next, l), jext,
                       __builtin_amdgcn_readlane((int)exc, l) != 0, __builtin_amdgcn_readlane((int)fj, l) != 0,
                       (uint32_t)__builtin_amdgcn_readlane((int)ff, l), t0};
        XWaveOut o;
        x_wave_neuron_any(a, a.qsorted + k0_l, (uint32_t)__builtin_amdgcn_readlane((int)nrec, l), in_l,
                          __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, V0), l)),
                          __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, W0), l)),
                          re_l, lane, o);
        if (lane == (uint32_t)l) {
            a.V[j] = o.V;
            a.W[j] = o.W;
            a.rend[j] = o.re;
            if (o.spiked) a.fs[j] = o.fsp;
            spiked = o.spiked;
            dis = o.dis;
        }
    }
    if (live && !coop) {
        XNeuron s{V0, W0, re0, t0, 0u, 0u, 0u};
        const XIn in{j, t, next, jext, exc, fj, ff, t0};
        if (next <= kXLocal) x_take_merged(a, s, in, a.qsorted + k0, nrec, ev_s + tid, false);
        else x_take_selected(a, s, in, a.qsorted + k0, nrec);
        x_advance(a, s, t1);
        a.V[j] = s.V;
        a.W[j] = s.W;
        a.rend[j] = s.re;
        if (s.spiked) a.fs[j] = s.fsp;
        spiked = s.spiked;
        dis = s.dis;
    }
    x_close_block(a, j, spiked, next, dis, wcnt, wext, wdis);
}

__global__ __launch_bounds__(kXBlock) void k_x_list(XArgs a)
{
    __shared__ unsigned long long part[kXBlock / 64];
    const uint32_t b = blockIdx.x, i = threadIdx.x, lane = i & 63u;
    // this workgroup's first spike: the spike counts of the workgroups before it
    // (a few thousand L2-resident words; no separate scan launch)
    unsigned long long before = 0;
    for (uint32_t k = i; k < b; k += kXBlock) before += a.blk_cnt[k];
    before = x_wave_sum<unsigned long long>(before);
    if (lane == 0) part[i >> 6] = before;
    __syncthreads();
    unsigned long long off = 0;
    for (uint32_t w = 0; w < kXBlock / 64; ++w) off += part[w];
    const uint32_t cnt = a.blk_cnt[b];
    if (i == 0) {
        a.blk_off[b] = off;
        if (b + 1 == a.nblk) a.blk_off[a.nblk] = off + cnt;   // the step's spike total
    }
    if (i >= cnt) return;
    const uint32_t t = a.ctrl->t0;
    const uint64_t p = off + i;
    const uint32_t gid = a.blk_list[(size_t)b * kXBlock + i];
    const uint32_t f = a.fs[gid];
    const uint64_t hb = a.ctrl->hist_n;
    if (hb + p < a.hist_cap) {
        a.hist[hb + p] = make_uint2(t, gid);
        a.hist_f[hb + p] = f;
    }
    const uint64_t rb = a.row_ptr[gid];
    a.spk[p] = make_uint4(gid, f, (uint32_t)rb, (uint32_t)(rb >> 32));
    // the row's bucket lengths, which k_x_offsets turns into the spike's places
    uint32_t prev = 0;
    for (uint32_t d = 0; d < a.D; ++d) {
        const uint32_t e = a.bend[(size_t)gid * a.D + d];
        a.xpref[p * a.D + d] = e - prev;
        prev = e;
    }
}

// Where each spike's inputs go in the arrival lists, with no atomics: for
// delay bucket d (one workgroup each, d < D), an exclusive scan over the
// step's spikes of their rows' bucket-d lengths (k_x_list left them in
// xpref) gives each spike's place in the list of slot (t + d_min + d) mod R,
// after what earlier steps appended; the slot's count grows by the total.
// Each thread scans a contiguous run of spikes, eight loads in flight.
__global__ __launch_bounds__(1024) void k_x_offsets(XArgs a)
{
    __shared__ unsigned long long wsum[16];
    const uint32_t d = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t D = a.D;
    const uint32_t slot = (a.ctrl->t0 + a.d_min + d) % a.R;
    const uint64_t n = a.blk_off[a.nblk];   // the step's spikes
    const uint64_t per = (n + 1023u) / 1024u;
    const uint64_t p0 = (uint64_t)tid * per < n ? (uint64_t)tid * per : n;
    const uint64_t p1 = p0 + per < n ? p0 + per : n;
    uint32_t* const x = a.xpref + d;        // x[p * D]: spike p's bucket-d length, then place
    unsigned long long sum = 0;
    for (uint64_t p = p0; p < p1; p += 8u) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) v[u] = p + u < p1 ? x[(p + u) * D] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) sum += v[u];
    }
    unsigned long long inc = sum;
#pragma unroll
    for (uint32_t o = 1; o < 64u; o <<= 1) {
        const unsigned long long y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63u) wsum[wv] = inc;
    __syncthreads();
    unsigned long long off = inc - sum, tot = 0;
    for (uint32_t w = 0; w < 16u; ++w) {
        if (w < wv) off += wsum[w];
        tot += wsum[w];
    }
    for (uint64_t p = p0; p < p1; p += 8u) {
        uint32_t v[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) v[u] = p + u < p1 ? x[(p + u) * D] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
            // (a place past 2^32 - 1 is past any list's capacity: the inputs are dropped, counted)
            if (p + u < p1) x[(p + u) * D] = off < 0xFFFFFFFFull ? (uint32_t)off : 0xFFFFFFFFu;
            off += v[u];
        }
    }
    if (tid == 0) a.qn[slot] = a.qn_prev[slot] + tot;
}

__global__ __launch_bounds__(256) void k_x_deliver(XArgs a)
{
    __shared__ int32_t cb_s[256];
    cb_s[threadIdx.x] = a.record ? a.cb[threadIdx.x] : 0;
    __syncthreads();
    const uint32_t t = a.ctrl->t0;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * 4u;
    const uint64_t items = a.blk_off[a.nblk] * a.smax;
    unsigned long long drop = 0;
    for (uint64_t it = wave; it < items; it += nw) {
        const uint64_t p = it / a.smax;
        const uint32_t s0 = (uint32_t)(it % a.smax) * 256u;
        const uint4 sp = a.spk[p];
        const uint32_t gid = sp.x, f = sp.y;
        const uint64_t rb = (uint64_t)sp.z | ((uint64_t)sp.w << 32);
        // lane d < D: delay bucket d of the row, [start, end); the last end is the row length
        const uint32_t endv = lane < a.D ? (uint32_t)a.bend[(size_t)gid * a.D + lane] : 0u;
        const uint32_t len = (uint32_t)__builtin_amdgcn_readlane((int)endv, (int)(a.D - 1u));
        if (s0 >= len) continue;
        const uint32_t s1 = len - s0 < 256u ? len : s0 + 256u;
        const uint32_t end = lane < a.D ? endv : len;
        const uint32_t prev = __shfl_up(end, 1u);
        const uint32_t start = lane == 0 ? 0u : prev;
        // bucket `lane`: its slot and where this spike's inputs of it start in
        // the slot's list (the place k_x_offsets gave the spike there)
        const uint32_t slot = (t + a.d_min + lane) % a.R;
        const unsigned long long base =
            lane < a.D ? a.qn_prev[slot] + a.xpref[p * a.D + lane] : 0ull;
        // this lane's records k = s0 + 64 u + lane, u < 4: every load issued before any use
        uint32_t tg[4], bk[4];
        int32_t wq[4];
        if (a.record) {   // (uniform)
            uint32_t v[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t k = s0 + 64u * u + lane;
                v[u] = reinterpret_cast<const uint32_t*>(a.recs)[rb + (k < s1 ? k : s1 - 1u)];
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                tg[u] = v[u] >> 8;
                wq[u] = (int32_t)(v[u] & 255u);
                bk[u] = 0u;
            }
        } else {
            Rec8 r[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t k = s0 + 64u * u + lane;
                r[u] = reinterpret_cast<const Rec8*>(a.recs)[rb + (k < s1 ? k : s1 - 1u)];
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                tg[u] = r[u].tgt & kTgtMask;
                bk[u] = r[u].tgt >> kTgtBits;   // 8-byte records carry their delay bucket
                wq[u] = __float2int_rn(r[u].w * 65536.0f);
            }
        }
        // each record's bucket and its place in that bucket's slot list
        unsigned long long pos[4];
        uint32_t sl[4];
        bool ok[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t k = s0 + 64u * u + lane;
            const uint32_t kk = k < s1 ? k : s1 - 1u;
            uint32_t d = bk[u];
            if (a.record) {   // (uniform) 8-bit codes: the bucket from the row's bucket ends
                d = 0;
                for (uint32_t l = 0; l < a.D; ++l)
                    d += kk >= (uint32_t)__builtin_amdgcn_readlane((int)end, (int)l) ? 1u : 0u;
            }
            const uint32_t bs = __shfl(start, (int)d);
            sl[u] = __shfl(slot, (int)d);
            pos[u] = __shfl(base, (int)d) + (kk - bs);
            ok[u] = k < s1 && pos[u] < a.qcap && tg[u] < a.N;
            if (k < s1 && !ok[u]) ++drop;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u)
            if (ok[u])
                a.qlist[(size_t)sl[u] * a.qcap + pos[u]] =
                    make_uint4(tg[u], f, (uint32_t)(a.record ? cb_s[wq[u]] : wq[u]), 0u);
    }
    drop = x_wave_sum<unsigned long long>(drop);
    if (lane == 0 && drop) atomicAdd(a.dropped, drop);
}

__global__ __launch_bounds__(1024) void k_x_finish(XArgs a)
{
    // the step's external events: the update workgroups' totals
    __shared__ unsigned long long wext[16];
    const uint32_t tid = threadIdx.x;
    unsigned long long ext = 0;
    for (uint32_t k = tid; k < a.nblk; k += 1024u) ext += a.blk_ext[k];
    ext = x_wave_sum<unsigned long long>(ext);
    if ((tid & 63u) == 0) wext[tid >> 6] = ext;
    __syncthreads();
    if (tid != 0) return;
    for (uint32_t w = 0; w < 16; ++w) a.ctrl->ext_events += wext[w];
    const uint64_t n = a.blk_off[a.nblk];
    // the step's recurrent events: what delivery appended to the slots' lists
    unsigned long long ev = 0;
    for (uint32_t s = 0; s < a.R; ++s) ev += a.qn[s] - a.qn_prev[s];
    a.ctrl->rec_events += ev;
    a.ctrl->hist_n += n;
    a.ctrl->spikes += n;
    a.ctrl->t0 += 1u;
}

constexpr uint32_t kXGrid = 1024;   // workgroups of the grid-stride kernels

}  // namespace

#define SNN_X_LAUNCH(ev, kern, grid, block, s, ...)                                                    \
    do {                                                                                               \
        if (ev) hipExtLaunchKernelGGL(kern, grid, block, 0, s, (ev)->start, (ev)->stop, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);                                \
    } while (0)

hipError_t launch_x_place(const XArgs& a, hipStream_t s, const LaunchEv* ev)
{
    // timed from the first kernel's start to the last one's end
    if (ev) hipExtLaunchKernelGGL(k_xs_count, dim3(kXGrid), dim3(256), 0, s, ev->start, nullptr, 0, a);
    else hipLaunchKernelGGL(k_xs_count, dim3(kXGrid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_xs_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_xs_scatter, dim3(kXGrid), dim3(256), 0, s, a);
    if (ev) hipExtLaunchKernelGGL(k_xs_group, dim3(a.ngroups), dim3(256), 0, s, nullptr, ev->stop, 0, a);
    else hipLaunchKernelGGL(k_xs_group, dim3(a.ngroups), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_x_update(const XArgs& a, hipStream_t s, const LaunchEv* ev)
{
    SNN_X_LAUNCH(ev, k_x_update, dim3(a.nblk), dim3(kXBlock), s, a);
    hipLaunchKernelGGL(k_x_update_busy, dim3(a.nblk), dim3(kXBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_x_list(const XArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_x_list, dim3(a.nblk), dim3(kXBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_x_deliver(const XArgs& a, hipStream_t s, const LaunchEv* ev)
{
    hipLaunchKernelGGL(k_x_offsets, dim3(a.D), dim3(1024), 0, s, a);
    SNN_X_LAUNCH(ev, k_x_deliver, dim3(kXGrid), dim3(256), s, a);
    return hipGetLastError();
}

hipError_t launch_x_finish(const XArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_x_finish, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace snn
