// exact.hip -- gfx950 kernels of the exact-time event-driven solver
// (Sec. II.A, Sec. II.C).
//
//   k_x_place    the arriving slot's queued inputs, counting-sorted by target
//                (positions from the scanned per-target counts, which count
//                back down to zero for the slot's next use)
//   k_x_update   one thread per neuron: this step's inputs (queued and
//                external) in time order, Eq. (1)-(2) solved exactly between
//                them, a spike at the input that crosses threshold; ordered
//                spiker list per 256-neuron workgroup
//   k_x_deliver  one wave per spike: AER history entry (step, id, offset) and
//                fan-out of the row, one reservation per delay bucket in the
//                arrival slot's list
//   k_x_finish   step counters
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

__global__ __launch_bounds__(256) void k_x_place(XArgs a, uint32_t t)
{
    const uint32_t slot = t % a.R;
    const uint64_t n0 = a.qn[slot];
    const uint64_t n = n0 < a.qcap ? n0 : a.qcap;
    const uint4* L = a.qlist + (size_t)slot * a.qcap;
    uint32_t* cnt = a.qcnt + (size_t)slot * a.N;
    unsigned long long bad = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * 256u + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256u) {
        const uint4 v = L[e];
        if (v.x >= a.N) {
            ++bad;
            continue;
        }
        const uint32_t c = atomicSub(cnt + v.x, 1u);
        const uint64_t pos = a.qoff[v.x] + (uint64_t)c - 1u;
        if (c == 0 || pos >= a.qcap) {   // cannot happen while counts and lists agree
            ++bad;
            continue;
        }
        a.qsorted[pos] = make_uint2(v.y, v.z);
    }
    if (bad) atomicAdd(a.dropped, bad);
}

__global__ __launch_bounds__(kXBlock) void k_x_update(XArgs a, uint32_t t)
{
    __shared__ uint2 ev_s[kXLocal * kXBlock];   // [input][thread]
    __shared__ uint32_t pois_s[kMaxPois];
    __shared__ uint32_t wcnt[kXBlock / 64];
    __shared__ unsigned long long wext[kXBlock / 64], wdis[kXBlock / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t j = blockIdx.x * kXBlock + tid;
    if (tid < a.npois) pois_s[tid] = a.poisc[tid];
    if (blockIdx.x == 0 && tid == 0) a.qn[t % a.R] = 0;   // the slot's list has been placed
    __syncthreads();
    const uint64_t t0 = (uint64_t)t << 32, t1 = t0 + (1ull << 32);
    uint32_t spiked = 0, next = 0, dis = 0;
    if (j < a.N) {
        uint64_t k0 = a.qoff[j], k1 = a.qoff[j + 1];
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
        XNeuron s{a.V[j], a.W[j], a.rend[j], t0, 0u, 0u, 0u};
        const bool exc = (j % a.M) < a.n_exc;
        const bool fj = a.forced ? a.forced[j] != 0 : false;
        const uint32_t ff = a.forced ? a.forced_f[j] : 0u;
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
        } else {
            // many inputs: take the earliest remaining instant each time
            uint64_t lo = 0;
            while (lo <= 0xFFFFFFFFull) {
                uint64_t best = 1ull << 32;
                int32_t J = 0;
                for (uint32_t i = 0; i < nrec; ++i) {
                    const uint2 x = a.qsorted[k0 + i];
                    if (x.x < lo) continue;
                    if (x.x < best) {
                        best = x.x;
                        J = (int32_t)x.y;
                    } else if (x.x == best) {
                        J += (int32_t)x.y;
                    }
                }
                for (uint32_t i = 0; i < next; i += 4) {
                    const uint4 r = a.ext_const ? make_uint4(0u, 0u, 0u, 0u)
                                                : x_philox(j, t, kStreamExtTime, i >> 2, a.key0, a.key1);
                    for (uint32_t q = 0; q < 4 && i + q < next; ++q) {
                        const uint32_t f = word(r, q);
                        if (f < lo) continue;
                        if (f < best) {
                            best = f;
                            J = jext;
                        } else if (f == best) {
                            J += jext;
                        }
                    }
                }
                if (best > 0xFFFFFFFFull) break;
                x_input(a, s, t0, (uint32_t)best, J, exc, fj, ff);
                lo = best + 1;
            }
        }
        x_advance(a, s, t1);
        a.V[j] = s.V;
        a.W[j] = s.W;
        a.rend[j] = s.re;
        if (s.spiked) a.fs[j] = s.fsp;
        spiked = s.spiked;
        dis = s.dis;
    }
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
        a.blk_cnt[blockIdx.x] = tot;
        unsigned long long ex = 0, ds = 0;
        for (uint32_t w = 0; w < kXBlock / 64; ++w) {
            ex += wext[w];
            ds += wdis[w];
        }
        if (ex) atomicAdd((unsigned long long*)&a.ctrl->ext_events, ex);
        if (ds) atomicAdd((unsigned long long*)&a.ctrl->disagree, ds);
    }
}

__global__ __launch_bounds__(256) void k_x_deliver(XArgs a, uint32_t t)
{
    __shared__ int32_t cb_s[256];
    cb_s[threadIdx.x] = a.record ? a.cb[threadIdx.x] : 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * 4u;
    const uint64_t nspk = a.blk_off[a.nblk];
    const uint64_t hb = a.ctrl->hist_n;
    unsigned long long ev = 0, drop = 0;
    for (uint64_t p = wave; p < nspk; p += nw) {
        // the workgroup list holding spike p: the last b with blk_off[b] <= p
        uint32_t lo = 0, hi = a.nblk;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.blk_off[mid] <= p) lo = mid;
            else hi = mid;
        }
        const uint32_t gid = a.blk_list[(size_t)lo * kXBlock + (uint32_t)(p - a.blk_off[lo])];
        const uint32_t f = a.fs[gid];
        if (lane == 0 && hb + p < a.hist_cap) {
            a.hist[hb + p] = make_uint2(t, gid);
            a.hist_f[hb + p] = f;
        }
        const uint64_t rb = a.row_ptr[gid];
        const uint32_t len = (uint32_t)(a.row_ptr[gid + 1] - rb);
        // lane d < D: delay bucket d of the row, [start, end), its arrival
        // slot and its reservation in that slot's list
        const uint32_t end = lane < a.D ? (uint32_t)a.bend[(size_t)gid * a.D + lane] : len;
        const uint32_t prev = __shfl_up(end, 1u);
        const uint32_t start = lane == 0 ? 0u : prev;
        const uint32_t size = lane < a.D ? end - start : 0u;
        const uint32_t slot = (t + a.d_min + lane) % a.R;
        unsigned long long base = 0;
        if (size) base = atomicAdd(a.qn + slot, (unsigned long long)size);
        for (uint32_t c0 = 0; c0 < len; c0 += 64u) {
            const uint32_t k = c0 + lane;
            const uint32_t kk = k < len ? k : len - 1u;
            uint32_t tgt;
            int32_t wq;
            if (a.record) {
                const uint32_t v = reinterpret_cast<const uint32_t*>(a.recs)[rb + kk];
                tgt = v >> 8;
                wq = cb_s[v & 255u];
            } else {
                const Rec8 r = reinterpret_cast<const Rec8*>(a.recs)[rb + kk];
                tgt = r.tgt;
                wq = __float2int_rn(r.w * 65536.0f);
            }
            uint32_t d = 0;
            for (uint32_t l = 0; l < a.D; ++l)
                d += kk >= (uint32_t)__builtin_amdgcn_readlane((int)end, (int)l) ? 1u : 0u;
            const uint32_t bs = __shfl(start, (int)d);
            const uint32_t sl = __shfl(slot, (int)d);
            const unsigned long long bb = __shfl(base, (int)d);
            if (k < len) {
                const unsigned long long pos = bb + (kk - bs);
                if (pos < a.qcap && tgt < a.N) {
                    a.qlist[(size_t)sl * a.qcap + pos] = make_uint4(tgt, f, (uint32_t)wq, 0u);
                    atomicAdd(a.qcnt + (size_t)sl * a.N + tgt, 1u);
                } else {
                    ++drop;
                }
            }
        }
        if (lane == 0) ev += len;
    }
    ev = x_wave_sum<unsigned long long>(ev);
    drop = x_wave_sum<unsigned long long>(drop);
    if (lane == 0) {
        if (ev) atomicAdd((unsigned long long*)&a.ctrl->rec_events, ev);
        if (drop) atomicAdd(a.dropped, drop);
    }
}

__global__ void k_x_finish(XArgs a)
{
    if (threadIdx.x != 0) return;
    const uint64_t n = a.blk_off[a.nblk];
    a.ctrl->hist_n += n;
    a.ctrl->spikes += n;
    a.ctrl->t0 += 1u;
}

constexpr uint32_t kXGrid = 2048;   // workgroups of the grid-stride kernels

}  // namespace

#define SNN_X_LAUNCH(ev, kern, grid, block, s, ...)                                                    \
    do {                                                                                               \
        if (ev) hipExtLaunchKernelGGL(kern, grid, block, 0, s, (ev)->start, (ev)->stop, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);                                \
    } while (0)

hipError_t launch_x_place(const XArgs& a, uint32_t t, hipStream_t s, const LaunchEv* ev)
{
    SNN_X_LAUNCH(ev, k_x_place, dim3(kXGrid), dim3(256), s, a, t);
    return hipGetLastError();
}

hipError_t launch_x_update(const XArgs& a, uint32_t t, hipStream_t s, const LaunchEv* ev)
{
    SNN_X_LAUNCH(ev, k_x_update, dim3(a.nblk), dim3(kXBlock), s, a, t);
    return hipGetLastError();
}

hipError_t launch_x_deliver(const XArgs& a, uint32_t t, hipStream_t s, const LaunchEv* ev)
{
    SNN_X_LAUNCH(ev, k_x_deliver, dim3(kXGrid), dim3(256), s, a, t);
    return hipGetLastError();
}

hipError_t launch_x_finish(const XArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_x_finish, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace snn
