// exact.hip -- gfx950 kernels of the exact-time event-driven solver
// (Sec. II.A, Sec. II.C).
//
//   k_x_place    the arriving slot's queued inputs, counting-sorted by target
//                (position: the target's scanned offset plus the input's rank
//                among the target's inputs, taken when it was delivered)
//   k_x_update   one thread per neuron: this step's inputs (queued and
//                external) in time order, Eq. (1)-(2) solved exactly between
//                them, a spike at the input that crosses threshold; ordered
//                spiker list per 256-neuron workgroup
//   k_x_list     dense spike list of the step (each workgroup's place from the
//                counts of those before it) and its AER history entries
//                (step, id, offset)
//   k_x_deliver  one wave per (spike, 256-record row segment): fan-out into
//                the arrival slots' lists, one reservation per delay bucket
//                the segment touches
//   k_x_finish   step counters (external events totalled over the workgroups)
//
// Like the step kernels this is bound by memory traffic and atomics, not by
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

__global__ __launch_bounds__(256) void k_x_place(XArgs a)
{
    const uint32_t t = a.ctrl->t0;   // the step in flight (k_x_finish advances it)
    const uint32_t slot = t % a.R;
    const uint64_t n0 = a.qn[slot];
    const uint64_t n = n0 < a.qcap ? n0 : a.qcap;
    const uint4* L = a.qlist + (size_t)slot * a.qcap;
    unsigned long long bad = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * 256u + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256u) {
        const uint4 v = L[e];   // {target, offset, charge, rank}
        if (v.x >= a.N) {
            ++bad;
            continue;
        }
        const uint64_t pos = a.qoff[v.x] + (uint64_t)v.w;
        if (pos >= a.qoff[v.x + 1] || pos >= a.qcap) {   // cannot happen while counts and lists agree
            ++bad;
            continue;
        }
        a.qsorted[pos] = make_uint2(v.y, v.z);
    }
    if (bad) atomicAdd(a.dropped, bad);
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
// place, hold its external inputs sorted in its LDS slots, and take the two
// in time order, inputs of one instant together.
__device__ __forceinline__ void x_take_merged(const XArgs& a, XNeuron& s, const XIn& in, uint2* seg,
                                              uint32_t nrec, uint2* e)
{
    x_heap_sort(seg, nrec);
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
            x_take_merged(a, s, in, a.qsorted + k0, nrec, ev_s + tid);
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

// Busy workgroups: the workgroup's queued inputs are read into LDS in
// windows of up to kXBusyCap entries, coalesced; a neuron whose whole slice
// lies in the window heap-sorts it there, holds its external inputs sorted in
// its LDS slots, merges the two and integrates.  The next window starts at
// the first neuron not yet done, so every pass finishes at least that neuron;
// only a slice longer than a whole window is sorted where it lies, in global
// memory.
__global__ __launch_bounds__(kXBlock) void k_x_update_busy(XArgs a)
{
    __shared__ uint2 in_s[kXBusyCap];            // one window of the workgroup's inputs, by target
    __shared__ uint2 ev_s[kXLocal * kXBlock];    // external inputs [input][thread]
    __shared__ uint32_t pois_s[kMaxPois];
    __shared__ uint32_t wcnt[kXBlock / 64];
    __shared__ unsigned long long wext[kXBlock / 64], wdis[kXBlock / 64];
    __shared__ unsigned long long wlo[kXBlock / 64];
    if (!x_block_busy(a)) return;   // (uniform) the workgroup is k_x_update's
    const uint32_t t = a.ctrl->t0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t j = blockIdx.x * kXBlock + tid;
    const bool live = j < a.N;
    const uint32_t first = blockIdx.x * kXBlock;
    uint64_t base = a.qoff[first];
    base = base < a.qcap ? base : a.qcap;
    const uint64_t end = base + x_block_inputs(a);
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
    k0 = k0 > base ? k0 : base;
    k1 = k1 > k0 ? k1 : k0;
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
    const XIn in{j, t, next, jext, exc, fj, ff, t0};
    bool done = !live;
    uint64_t lo = base;
    for (;;) {
        const uint64_t hi = (end - lo) < kXBusyCap ? end : lo + kXBusyCap;
        for (uint64_t i = lo + tid; i < hi; i += kXBlock) in_s[i - lo] = a.qsorted[i];
        __syncthreads();
        const bool whole = k0 >= lo && k1 <= hi;          // the slice lies in this window
        const bool huge = nrec > kXBusyCap;                 // no window holds it
        if (!done && (whole || huge)) {
            XNeuron s{V0, W0, re0, t0, 0u, 0u, 0u};
            uint2* seg = whole ? in_s + (k0 - lo) : a.qsorted + k0;
            if (next <= kXLocal) x_take_merged(a, s, in, seg, nrec, ev_s + tid);
            else x_take_selected(a, s, in, seg, nrec);
            x_advance(a, s, t1);
            a.V[j] = s.V;
            a.W[j] = s.W;
            a.rend[j] = s.re;
            if (s.spiked) a.fs[j] = s.fsp;
            spiked = s.spiked;
            dis = s.dis;
            done = true;
        }
        // the next window starts at the slice of the first neuron not done
        unsigned long long m = done ? ~0ull : (unsigned long long)k0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long y = __shfl_xor(m, o);
            m = y < m ? y : m;
        }
        if (lane == 0) wlo[wv] = m;
        __syncthreads();   // also: every lane is done with this window's LDS copy
        unsigned long long nlo = ~0ull;
        for (uint32_t w = 0; w < kXBlock / 64; ++w) nlo = wlo[w] < nlo ? wlo[w] : nlo;
        __syncthreads();   // wlo is rewritten by the next pass
        if (nlo == ~0ull) break;
        lo = nlo;
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
        // the part of bucket `lane` inside this segment, its slot and reservation
        const uint32_t lo = start > s0 ? start : s0;
        const uint32_t hi = end < s1 ? end : s1;
        const uint32_t cnt = (lane < a.D && hi > lo) ? hi - lo : 0u;
        const uint32_t slot = (t + a.d_min + lane) % a.R;
        unsigned long long base = 0;
        if (cnt) base = atomicAdd(a.qn + slot, (unsigned long long)cnt);
        // this lane's records k = s0 + 64 u + lane, u < 4: every load issued before any use
        auto load = [&](uint32_t u, uint32_t& tgt, int32_t& wf) {
            const uint32_t k = s0 + 64u * u + lane;
            const uint32_t kk = k < s1 ? k : s1 - 1u;
            if (a.record) {
                const uint32_t v = reinterpret_cast<const uint32_t*>(a.recs)[rb + kk];
                tgt = v >> 8;
                wf = (int32_t)(v & 255u);
            } else {
                const Rec8 r = reinterpret_cast<const Rec8*>(a.recs)[rb + kk];
                tgt = r.tgt & kTgtMask;
                wf = __float2int_rn(r.w * 65536.0f);
            }
        };
        auto emit = [&](uint32_t u, uint32_t tgt, int32_t wf) {
            if (s0 + 64u * u >= s1) return;   // (uniform) past the segment's end
            const uint32_t k = s0 + 64u * u + lane;
            const uint32_t kk = k < s1 ? k : s1 - 1u;
            uint32_t d = 0;
            for (uint32_t l = 0; l < a.D; ++l)
                d += kk >= (uint32_t)__builtin_amdgcn_readlane((int)end, (int)l) ? 1u : 0u;
            const uint32_t bl = __shfl(lo, (int)d);
            const uint32_t sl = __shfl(slot, (int)d);
            const unsigned long long bb = __shfl(base, (int)d);
            if (k < s1) {
                const unsigned long long pos = bb + (kk - bl);
                const int32_t w = a.record ? cb_s[wf] : wf;
                if (pos < a.qcap && tgt < a.N) {
                    // the input's rank among its target's inputs of the slot
                    const uint32_t r = atomicAdd(a.qcnt + (size_t)sl * a.N + tgt, 1u);
                    a.qlist[(size_t)sl * a.qcap + pos] = make_uint4(tgt, f, (uint32_t)w, r);
                } else {
                    ++drop;
                }
            }
        };
        uint32_t t0r, t1r, t2r, t3r;
        int32_t w0r, w1r, w2r, w3r;
        load(0, t0r, w0r);
        load(1, t1r, w1r);
        load(2, t2r, w2r);
        load(3, t3r, w3r);
        emit(0, t0r, w0r);
        emit(1, t1r, w1r);
        emit(2, t2r, w2r);
        emit(3, t3r, w3r);
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
    SNN_X_LAUNCH(ev, k_x_place, dim3(kXGrid), dim3(256), s, a);
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
    SNN_X_LAUNCH(ev, k_x_deliver, dim3(kXGrid), dim3(256), s, a);
    return hipGetLastError();
}

hipError_t launch_x_finish(const XArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_x_finish, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

}  // namespace snn
