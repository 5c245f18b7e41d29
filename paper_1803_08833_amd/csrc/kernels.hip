// kernels.hip -- gfx950 kernels of the spiking-network hot path.
//
//   k_init        initial membrane potentials (INIT stream)
//   k_syn_gen     projection generation: per-pair Bernoulli trials, hits per row
//   k_scan_*      row offsets (exclusive scan of row lengths)
//   k_syn_out     projection write-out: delay buckets, records ordered by (delay, target)
//   k_syn_out_seg the same for two-level networks, records ordered by (super tile,
//                 delay, target), with each row's super-tile segment starts
//   k_update      fused neuron step: ring read+clear, Poisson drive, LIF+SFA, ordered
//                 block-local spike compaction
//   k_compact     ordered global spike list + AER history
//   k_deliver     wave-per-row-segment fan-out into the delay ring (int32 atomics)
//   k_scatter     tile-binned delivery, phase A: events binned by target tile
//   k_tile        tile-binned delivery, phase B: LDS accumulation, ring write-back
//   k_seg_emit    two-level networks: the step's record segments listed per super tile
//   k_seg_bin     two-level networks: each super tile's segments binned by tile
//                 (or delivered directly in a step below the binning threshold)
//
// Nothing here is a dense contraction: the path is bound by HBM/L2 traffic and
// atomics (update, delivery) or by 32-bit integer multiplies (Philox), so no MFMA.
#include "snn_dev.h"

#include <hip/hip_ext.h>

#include <mutex>

namespace snn {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64-bit products of the even counter words with the round
// multipliers, the odd words and key XORed into the high halves; the key is
// advanced by the golden-ratio and sqrt(3)-1 Weyl increments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
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

// ---- wave64 helpers ----
__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// inclusive prefix sum over the 64 lanes
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, uint32_t lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v += u;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Initial state: V uniform in [E, V_th) from the top 24 bits of the INIT draw.
// One thread per quad of neurons (gid = 4q + s).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(StepArgs a)
{
    const uint32_t q = blockIdx.x * 256u + threadIdx.x;
    if (q >= a.nq) return;
    const uint4 r = philox(q, 0u, kStreamInit, 0u, a.key0, a.key1);
    const float span = a.v_th - a.e_rest;
    float4 v;
    v.x = a.e_rest + span * ((float)(r.x >> 8) * 0x1p-24f);
    v.y = a.e_rest + span * ((float)(r.y >> 8) * 0x1p-24f);
    v.z = a.e_rest + span * ((float)(r.z >> 8) * 0x1p-24f);
    v.w = a.e_rest + span * ((float)(r.w >> 8) * 0x1p-24f);
    reinterpret_cast<float4*>(a.V)[q] = v;
    reinterpret_cast<float4*>(a.W)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    reinterpret_cast<uchar4*>(a.ref)[q] = make_uchar4(0, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Projection construction, in slices of rows, each drawing every candidate
// pair once.  Generation: one wave per presynaptic row walks the target
// modules in ascending index (so targets come out ascending) and tests each
// module's candidates 256 at a time: lane l draws Philox CONN at (row, j/4)
// and compares the four words with the module's threshold; hits are appended
// in target order to the row's slot of a slice buffer.  After the slice's row
// offsets are scanned, write-out takes the hits 64 at a time: each lane draws
// the ATTR word of one hit (delay bucket, weight), and per-bucket ballots give
// each hit its rank among the same-delay hits before it, so records land in
// (delay, target) order.  syn_flush counts (lane b: hits of bucket b) or, with
// FILL, writes (lane b: the next free offset of bucket b).
// ---------------------------------------------------------------------------
// Delay bucket and weight draw of the synapse row -> j (ATTR stream).
__device__ __forceinline__ void hit_attr(const BuildArgs& a, uint32_t row, uint32_t j, uint32_t& b, uint32_t& wsel)
{
    const uint4 r = philox(row, j, kStreamAttr, 0u, a.key0, a.key1);
    if (a.delay_exp) {
        b = 0;
        for (uint32_t k = 0; k + 1u < a.D; ++k) b += a.dthr[k] <= r.x ? 1u : 0u;
    } else {
        b = __umulhi(r.x, a.D);
    }
    wsel = r.y;
}

template <bool FILL>
__device__ __forceinline__ void syn_flush(const BuildArgs& a, const uint32_t* q, uint32_t n,
                                          uint32_t row, bool exc, uint32_t lane, uint32_t& pos,
                                          uint64_t rbase)
{
    wave_sync();
    for (uint32_t base = 0; base < n; base += 64u) {
        const uint32_t e = base + lane;
        const bool valid = e < n;
        uint32_t j = 0, b = 0xFFFFFFFFu, wsel = 0;
        if (valid) {
            j = q[e];
            hit_attr(a, row, j, b, wsel);
        }
        for (uint32_t bb = 0; bb < a.D; ++bb) {
            const uint64_t mb = __ballot(b == bb);
            if (mb == 0) continue;
            if (FILL) {
                const uint32_t p0 = readlane(pos, bb);
                if (b == bb) {
                    const uint64_t at = rbase + p0 + mbcnt(mb);
                    if (a.record == 1u) {
                        const uint32_t code = exc ? __umulhi(wsel, 255u) : 255u;
                        reinterpret_cast<uint32_t*>(a.recs)[at] = (j << 8) | code;
                    } else {
                        const int32_t wq = exc ? a.wtab[wsel >> 16] : a.winh_q;
                        Rec8 r8;
                        r8.tgt = j | (b << kTgtBits);
                        r8.w = (float)wq * 0x1p-16f;
                        reinterpret_cast<Rec8*>(a.recs)[at] = r8;
                    }
                }
            }
            if (lane == bb) pos += popc(mb);
        }
    }
    wave_sync();
}

// Binomial generator, one row (one wave): the lanes take 64 target modules at
// a time and draw each module's count (one COUNT draw, binary search of the
// module's CDF thresholds); the modules with a nonzero count then take turns,
// in ascending order: Floyd's algorithm picks the subset into a bitmap held
// two 32-bit words per lane (candidates 0..4095), and the set bits are written
// out ascending.  Candidate l of the source's own module skips the source.
__device__ void syn_gen_binomial(const BuildArgs& a, uint32_t row, uint32_t lane, uint32_t* out, uint32_t& n)
{
    const uint32_t M = a.M, gx = a.gx, gy = a.gy, S = gx * gy;
    const uint32_t mi = row / M, xi = mi % gx, yi = mi / gx, li = row % M;
    const uint32_t tsel = li < a.n_exc ? 0u : S;
    for (uint32_t m0 = 0; m0 < S; m0 += 64u) {
        const uint32_t mj = m0 + lane;
        uint32_t cnt = 0;
        if (mj < S) {
            const uint32_t xj = mj % gx, yj = mj / gx;
            const uint32_t e = tsel + ((yj + gy - yi) % gy) * gx + (xj + gx - xi) % gx;
            if (a.T[e] != 0u) {
                const uint32_t u = philox(row, mj, kStreamCount, 0u, a.key0, a.key1).x;
                const uint4 b = a.btab[e];
                const uint32_t* thr = a.bthr + ((uint64_t)b.w << 32 | b.z);
                uint32_t lo = 0, hi = b.y;   // thresholds not above u: [0, lo)
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (thr[mid] <= u) lo = mid + 1u;
                    else hi = mid;
                }
                cnt = b.x + lo;
            }
        }
        uint64_t has = __ballot(cnt != 0u);
        while (has) {
            const uint32_t l = (uint32_t)__builtin_ctzll(has);
            has &= has - 1u;
            const uint32_t c = readlane(cnt, l), mt = m0 + l;
            const uint32_t nn = mt == mi ? M - 1u : M;
            uint32_t w0 = 0, w1 = 0;   // candidate bits [32 lane, +32) and [2048 + 32 lane, +32)
            uint4 pr = make_uint4(0, 0, 0, 0);
            for (uint32_t j = nn - c; j < nn; ++j) {
                if (j == nn - c || (j & 3u) == 0u) pr = philox(row, mt, kStreamPick, j >> 2, a.key0, a.key1);
                const uint32_t q = j & 3u;
                const uint32_t w = q == 0u ? pr.x : (q == 1u ? pr.y : (q == 2u ? pr.z : pr.w));
                const uint32_t t = __umulhi(w, j + 1u);
                const uint32_t wt = t >> 5;
                const uint32_t word = (wt >> 6) ? readlane(w1, wt & 63u) : readlane(w0, wt & 63u);
                const uint32_t x = ((word >> (t & 31u)) & 1u) ? j : t;
                const uint32_t wx = x >> 5;
                if (lane == (wx & 63u)) {
                    if (wx >> 6) w1 |= 1u << (x & 31u);
                    else w0 |= 1u << (x & 31u);
                }
            }
            for (uint32_t h = 0; h < 2u; ++h) {
                uint32_t bits = h ? w1 : w0;
                const uint32_t pc = popc(bits);
                const uint32_t incl = wave_incl_scan<uint32_t>(pc, lane);
                uint32_t o = n + incl - pc;
                while (bits) {
                    uint32_t cand = 2048u * h + 32u * lane + (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1u;
                    if (mt == mi && cand >= li) ++cand;
                    if (o < a.slab_cap) out[o] = mt * M + cand;
                    ++o;
                }
                n += readlane(incl, 63u);
            }
        }
    }
}

// Generation (one wave per row): the row's hits, targets ascending, go to the
// row's slot of the slice buffer (capacity slab_cap); the row length too.
__global__ __launch_bounds__(256) void k_syn_gen(BuildArgs a)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t rl = blockIdx.x * 4u + wv;
    if (rl >= a.nrows) return;
    const uint32_t row = a.row0 + rl;
    uint32_t* const out = a.slab + (size_t)rl * a.slab_cap;
    if (a.gen) {
        uint32_t n = 0;
        syn_gen_binomial(a, row, lane, out, n);
        if (lane == 0) {
            a.rowlen[row] = n;
            atomicMax(&a.ctrl->max_len, n);
            if (n > 65535u) atomicOr(&a.ctrl->err, 1u);
            if (n > a.slab_cap) atomicOr(&a.ctrl->err, 2u);
        }
        return;
    }
    const uint32_t M = a.M, gx = a.gx, gy = a.gy;
    const uint32_t mi = row / M, xi = mi % gx, yi = mi / gx;
    // the source's type selects its threshold table (excitatory first)
    const uint32_t* const Tsrc = a.T + ((row % M) < a.n_exc ? 0u : gx * gy);
    uint32_t n = 0;   // hits so far (wave-uniform)
    for (uint32_t yj = 0; yj < gy; ++yj) {
        const uint32_t dyr = yj >= yi ? yj - yi : yj + gy - yi;
        const uint32_t* Trow = Tsrc + dyr * gx;
        for (uint32_t xj = 0; xj < gx; ++xj) {
            const uint32_t dxr = xj >= xi ? xj - xi : xj + gx - xi;
            const uint32_t T = Trow[dxr];
            if (T == 0u) continue;
            const uint32_t jb = (yj * gx + xj) * M;
            for (uint32_t c = 0; c < M; c += 256u) {
                const uint32_t jo = c + 4u * lane;
                uint32_t h = 0;
                if (jo < M) {
                    const uint32_t j0 = jb + jo;
                    const uint4 r = philox(row, j0 >> 2, kStreamConn, 0u, a.key0, a.key1);
                    h = (uint32_t)(r.x < T) | ((uint32_t)(r.y < T) << 1) |
                        ((uint32_t)(r.z < T) << 2) | ((uint32_t)(r.w < T) << 3);
                    const uint32_t self = row - j0;      // no self-connection
                    if (self < 4u) h &= ~(1u << self);
                }
                const uint64_t m0 = __ballot(h & 1u), m1 = __ballot(h & 2u);
                const uint64_t m2 = __ballot(h & 4u), m3 = __ballot(h & 8u);
                const uint32_t tot = popc(m0) + popc(m1) + popc(m2) + popc(m3);
                if (tot) {
                    uint32_t o = n + mbcnt(m0) + mbcnt(m1) + mbcnt(m2) + mbcnt(m3);
                    const uint32_t j0 = jb + jo;
                    for (uint32_t s = 0; s < 4u; ++s)
                        if (h & (1u << s)) {
                            if (o < a.slab_cap) out[o] = j0 + s;
                            ++o;
                        }
                    n += tot;
                }
            }
        }
    }
    if (lane == 0) {
        a.rowlen[row] = n;
        atomicMax(&a.ctrl->max_len, n);
        if (n > 65535u) atomicOr(&a.ctrl->err, 1u);
        if (n > a.slab_cap) atomicOr(&a.ctrl->err, 2u);
    }
}

// Write-out (one wave per row): the delay bucket of every hit from its ATTR
// draw gives the bucket ends, then the records are written in (delay, target)
// order at the row's offset.
__global__ __launch_bounds__(256) void k_syn_out(BuildArgs a)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t rl = blockIdx.x * 4u + wv;
    if (rl >= a.nrows) return;
    const uint32_t row = a.row0 + rl;
    const uint32_t* const hits = a.slab + (size_t)rl * a.slab_cap;
    const bool exc = (row % a.M) < a.n_exc;
    uint32_t n = a.rowlen[row];
    n = n < a.slab_cap ? n : a.slab_cap;
    const uint64_t rbase = a.row_ptr[row];
    if (rbase + n > a.rec_cap) {   // the record buffer's bound was too small: report, write nothing
        if (lane == 0) atomicOr(&a.ctrl->err, 4u);
        return;
    }
    uint32_t pos = 0;   // lane b: hits of bucket b
    syn_flush<false>(a, hits, n, row, exc, lane, pos, 0);
    const uint32_t v = wave_incl_scan<uint32_t>(lane < a.D ? pos : 0u, lane);
    if (lane < a.D) a.bend[(size_t)row * a.D + lane] = (uint16_t)(v > 65535u ? 65535u : v);
    pos = v - (lane < a.D ? pos : 0u);   // lane b: start of bucket b
    syn_flush<true>(a, hits, n, row, exc, lane, pos, rbase);
}

// Write-out of a two-level network's row (8-bit codes; one wave per row), laid
// out by super tile of 2^kSegBits targets: every hit's delay bucket from its
// ATTR draw (as above), counts per (super tile, bucket) in the wave's LDS
// table, whose exclusive scan in (super tile, bucket) order gives each super
// tile's segment start and each (super tile, bucket) run's first slot; the
// hits, taken in target order, then go to their run's cursor, so a run keeps
// its targets ascending.  Record: target & (2^kSegBits - 1) | bucket <<
// kSegBits | code << (kSegBits + 5).  The bucket ends of the whole row (the
// (delay, target) order every other layout uses) are written too.
__global__ __launch_bounds__(256) void k_syn_out_seg(BuildArgs a)
{
    constexpr uint32_t KB = 32;   // table entries per super tile (>= kMaxD)
    __shared__ uint32_t tab_s[4][kMaxSuper * KB];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t rl = blockIdx.x * 4u + wv;
    if (rl >= a.nrows) return;   // no workgroup barrier below: each wave works alone
    uint32_t* const tab = tab_s[wv];
    const uint32_t row = a.row0 + rl;
    const uint32_t* const hits = a.slab + (size_t)rl * a.slab_cap;
    const bool exc = (row % a.M) < a.n_exc;
    uint32_t n = a.rowlen[row];
    n = n < a.slab_cap ? n : a.slab_cap;
    const uint64_t rbase = a.row_ptr[row];
    if (rbase + n > a.rec_cap) {
        if (lane == 0) atomicOr(&a.ctrl->err, 4u);
        return;
    }
    const uint32_t ns = a.nsuper;
    for (uint32_t i = lane; i < ns * KB; i += 64u) tab[i] = 0;
    wave_sync();
    for (uint32_t base = 0; base < n; base += 64u) {
        const uint32_t e = base + lane;
        if (e < n) {
            const uint32_t j = hits[e];
            uint32_t b, wsel;
            hit_attr(a, row, j, b, wsel);
            atomicAdd(&tab[(j >> kSegBits) * KB + b], 1u);
        }
    }
    wave_sync();
    // bucket ends of the whole row: lane b totals bucket b over the super tiles
    {
        uint32_t c = 0;
        if (lane < a.D)
            for (uint32_t sp = 0; sp < ns; ++sp) c += tab[sp * KB + lane];
        const uint32_t v = wave_incl_scan<uint32_t>(lane < a.D ? c : 0u, lane);
        if (lane < a.D) a.bend[(size_t)row * a.D + lane] = (uint16_t)(v > 65535u ? 65535u : v);
    }
    // lane s: super tile s's segment length, its start, then its runs' cursors
    uint32_t seg = 0;
    if (lane < ns)
        for (uint32_t b = 0; b < a.D; ++b) seg += tab[lane * KB + b];
    const uint32_t incl = wave_incl_scan<uint32_t>(seg, lane);
    wave_sync();
    if (lane < ns) {
        uint32_t at = incl - seg;
        a.sstart[(size_t)row * ns + lane] = (uint16_t)at;
        for (uint32_t b = 0; b < a.D; ++b) {
            const uint32_t c = tab[lane * KB + b];
            tab[lane * KB + b] = at;
            at += c;
        }
    }
    wave_sync();
    uint32_t* const out = reinterpret_cast<uint32_t*>(a.recs);
    for (uint32_t base = 0; base < n; base += 64u) {
        const uint32_t e = base + lane;
        const bool valid = e < n;
        uint32_t j = 0, b = 0, wsel = 0, key = 0;
        if (valid) {
            j = hits[e];
            hit_attr(a, row, j, b, wsel);
            key = (j >> kSegBits) * KB + b;
        }
        // the chunk's distinct (super tile, bucket) runs in turn; within a run
        // the lanes keep their (target) order
        uint64_t pend = __ballot(valid);
        while (pend) {
            const uint32_t k0 = readlane(key, (uint32_t)__builtin_ctzll(pend));
            const uint64_t m = __ballot(valid && key == k0);
            const uint32_t c0 = tab[k0];
            if (valid && key == k0) {
                const uint32_t code = exc ? __umulhi(wsel, 255u) : 255u;
                out[rbase + c0 + mbcnt(m)] = (j & ((1u << kSegBits) - 1u)) | (b << kSegBits) | (code << (kSegBits + 5u));
            }
            wave_sync();
            if (lane == 0) tab[k0] = c0 + popc(m);
            wave_sync();
            pend &= ~m;
        }
    }
}

// ---------------------------------------------------------------------------
// Row offsets: exclusive scan of u32 row lengths into u64 offsets, 1024 rows
// per tile (256 threads x 4).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* wsum, uint64_t& total)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint64_t inc = wave_incl_scan<uint64_t>(v, lane);
    if (lane == 63u) wsum[wv] = inc;
    __syncthreads();
    uint64_t off = 0;
    total = 0;
    for (uint32_t i = 0; i < 4u; ++i) {
        if (i < wv) off += wsum[i];
        total += wsum[i];
    }
    __syncthreads();
    return off + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* x, uint64_t* tsum, uint32_t N)
{
    __shared__ uint64_t ws[4];
    const uint32_t i0 = blockIdx.x * 1024u + threadIdx.x * 4u;
    uint64_t s = 0;
    for (uint32_t u = 0; u < 4u; ++u)
        if (i0 + u < N) s += x[i0 + u];
    uint64_t tot;
    block_excl_scan(s, ws, tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_tiles(uint64_t* tsum, uint32_t nt)
{
    __shared__ uint64_t ws[4];
    uint64_t carry = 0;
    for (uint32_t b = 0; b < nt; b += 256u) {
        const uint32_t i = b + threadIdx.x;
        const uint64_t v = i < nt ? tsum[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_excl_scan(v, ws, tot);
        if (i < nt) tsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* x, const uint64_t* toff,
                                                    uint64_t* out, uint32_t N, uint32_t* clear)
{
    __shared__ uint64_t ws[4];
    const uint32_t i0 = blockIdx.x * 1024u + threadIdx.x * 4u;
    uint32_t v[4];
    uint64_t s = 0;
    for (uint32_t u = 0; u < 4u; ++u) {
        v[u] = (i0 + u < N) ? x[i0 + u] : 0u;
        s += v[u];
    }
    if (clear)   // the counts are consumed: zero them for their next use
        for (uint32_t u = 0; u < 4u; ++u)
            if (i0 + u < N && v[u]) clear[i0 + u] = 0u;
    uint64_t tot;
    const uint64_t base = out[0];   // offset of the first row (set before; rewritten unchanged)
    uint64_t o = base + toff[blockIdx.x] + block_excl_scan(s, ws, tot);
    for (uint32_t u = 0; u < 4u; ++u) {
        if (i0 + u < N) out[i0 + u] = o;
        o += v[u];
    }
    if (blockIdx.x == gridDim.x - 1u && threadIdx.x == 0) out[N] = base + toff[blockIdx.x] + tot;
}

// ---------------------------------------------------------------------------
// Fused neuron step (one thread per quad of neurons, 1024 neurons per block):
// take the charge queued for step t and clear its ring slot, draw the external
// Poisson count (one Philox EXT call per quad), integrate the LIF+SFA exact
// one-step map in fp32, and compact the block's spikers in ascending id.
// ---------------------------------------------------------------------------

// streaming stores: written once per step and read by the next kernel from
// memory, so they need not stay dirty in this XCD's L2 until the kernel ends
typedef int v4i_nt __attribute__((ext_vector_type(4)));
typedef float v4f_nt __attribute__((ext_vector_type(4)));
typedef unsigned int v4u_nt __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_nt(float4* p, float4 v) { __builtin_nontemporal_store((v4f_nt){v.x, v.y, v.z, v.w}, reinterpret_cast<v4f_nt*>(p)); }
__device__ __forceinline__ void st_nt(int4* p, int4 v) { __builtin_nontemporal_store((v4i_nt){v.x, v.y, v.z, v.w}, reinterpret_cast<v4i_nt*>(p)); }
__device__ __forceinline__ void st_nt(uint4* p, uint4 v) { __builtin_nontemporal_store((v4u_nt){v.x, v.y, v.z, v.w}, reinterpret_cast<v4u_nt*>(p)); }
__device__ __forceinline__ void st_nt(uchar4* p, uchar4 v)
{
    const uint32_t w = (uint32_t)v.x | ((uint32_t)v.y << 8) | ((uint32_t)v.z << 16) | ((uint32_t)v.w << 24);
    __builtin_nontemporal_store(w, reinterpret_cast<uint32_t*>(p));
}

__device__ __forceinline__ bool neuron_step(const StepArgs& a, uint32_t gid, bool exc, int32_t iq,
                                            float& V, float& W, uint8_t& R, uint32_t& dis)
{
    const float J = (float)iq * 0x1p-16f;
    bool spike = false;
    if (R > 0) {
        R = (uint8_t)(R - 1);
        V = a.v_reset;
    } else {
        const float Vn = V + J;
        const bool own = Vn > a.v_th;
        if (a.forced) {
            spike = a.forced[gid] != 0;
            dis += (spike != own) ? 1u : 0u;
        } else {
            spike = own;
        }
        if (spike) {
            V = a.v_reset;
            R = (uint8_t)a.nref;
            if (exc || a.sfa_on_inh) W += a.alpha;
        } else {
            float u = Vn - a.e_rest;
            u = u - u * a.dm - a.kappa * W;
            V = a.e_rest + u;
        }
    }
    W = W - W * a.dw;
    return spike;
}

// One quad of neurons (gid = 4q .. 4q+3, all in one module since M % 4 == 0)
// takes its step-t input `in` (ring slot, already cleared by the caller), draws
// its external Poisson counts (one Philox EXT call) and integrates.  Returns the
// spike flags (bit s for neuron 4q + s); adds to *ext_tot and *dis.
__device__ __forceinline__ uint32_t update_quad(const StepArgs& a, const uint32_t* pois_s, uint32_t q,
                                                uint32_t t, int4 in, uint32_t& ext_tot, uint32_t& dis)
{
    float4 V = reinterpret_cast<const float4*>(a.V)[q];
    float4 W = reinterpret_cast<const float4*>(a.W)[q];
    uchar4 R = reinterpret_cast<const uchar4*>(a.ref)[q];
    int32_t e0, e1, e2, e3;
    if (a.ext_const) {
        e0 = e1 = e2 = e3 = a.ext_const_q;
    } else {
        const uint4 u = philox(q, t, kStreamExt, 0u, a.key0, a.key1);
        uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (uint32_t i = 0; i < a.npois; ++i) {
            const uint32_t th = pois_s[i];
            c0 += (th <= u.x) ? 1u : 0u;
            c1 += (th <= u.y) ? 1u : 0u;
            c2 += (th <= u.z) ? 1u : 0u;
            c3 += (th <= u.w) ? 1u : 0u;
        }
        ext_tot += c0 + c1 + c2 + c3;
        e0 = (int32_t)c0 * a.jext_q;
        e1 = (int32_t)c1 * a.jext_q;
        e2 = (int32_t)c2 * a.jext_q;
        e3 = (int32_t)c3 * a.jext_q;
    }
    const uint32_t g0 = 4u * q;
    const uint32_t loc = g0 % a.M;
    const auto add = [](int32_t x, int32_t y) { return (int32_t)((uint32_t)x + (uint32_t)y); };
    uint32_t flags = 0;
    flags |= neuron_step(a, g0, loc < a.n_exc, add(in.x, e0), V.x, W.x, R.x, dis) ? 1u : 0u;
    flags |= neuron_step(a, g0 + 1u, loc + 1u < a.n_exc, add(in.y, e1), V.y, W.y, R.y, dis) ? 2u : 0u;
    flags |= neuron_step(a, g0 + 2u, loc + 2u < a.n_exc, add(in.z, e2), V.z, W.z, R.z, dis) ? 4u : 0u;
    flags |= neuron_step(a, g0 + 3u, loc + 3u < a.n_exc, add(in.w, e3), V.w, W.w, R.w, dis) ? 8u : 0u;
    st_nt(reinterpret_cast<float4*>(a.V) + q, V);
    st_nt(reinterpret_cast<float4*>(a.W) + q, W);
    st_nt(reinterpret_cast<uchar4*>(a.ref) + q, R);
    return flags;
}

// Ordered block-local compaction of the spikers of update block `blk` (1024
// neurons; thread i < 256 holds the flags of quad 4*blk*256 + i): each spiker
// is written as {gid, row length, row start} in ascending id; the block's
// spike count, recurrent events (the spikers' row lengths) and external
// events are stored per block (the step's consumer totals them: no atomic on
// a shared counter here); the spike count also goes to the group counter of
// parity t & 1 while direct delivery is selected; lock-step disagreements are
// accumulated.
template <uint32_t NW>
//
// The block's NW waves are threads [0, 64 NW) of a thread group (gtid = index
// in the group); several groups of one workgroup may compact their own blocks
// side by side (every thread of the workgroup takes part in the barriers, a
// group that has no block passes live = false).
__device__ __forceinline__ void block_compact(const StepArgs& a, uint32_t blk, uint32_t t, uint32_t q,
                                              uint32_t flags, uint32_t ext_tot, uint32_t dis, uint32_t gtid,
                                              bool live, uint32_t* wtot, unsigned long long* wext, uint32_t* wdis,
                                              unsigned long long* wev)
{
    const uint32_t tid = gtid, lane = tid & 63u, wv = tid >> 6;
    const uint64_t m0 = __ballot(flags & 1u), m1 = __ballot(flags & 2u);
    const uint64_t m2 = __ballot(flags & 4u), m3 = __ballot(flags & 8u);
    const uint32_t pre = mbcnt(m0) + mbcnt(m1) + mbcnt(m2) + mbcnt(m3);
    const uint32_t wt = popc(m0) + popc(m1) + popc(m2) + popc(m3);
    const unsigned long long we = wave_sum<unsigned long long>(ext_tot);
    const uint32_t wd = wave_sum<uint32_t>(dis);
    if (lane == 0) {
        wtot[wv] = wt;
        wext[wv] = we;
        wdis[wv] = wd;
    }
    __syncthreads();
    uint32_t woff = 0, btot = 0;
    for (uint32_t i = 0; i < NW; ++i) {
        if (i < wv) woff += wtot[i];
        btot += wtot[i];
    }
    unsigned long long ev = 0;
    if (flags) {
        uint4* dst = a.blk_list + (size_t)blk * kNeuronsPerBlock + woff + pre;
        for (uint32_t s = 0; s < 4u; ++s) {
            if (flags & (1u << s)) {
                const uint32_t gid = 4u * q + s;
                const uint64_t rb = a.row_ptr[gid];
                const uint32_t len = (uint32_t)(a.row_ptr[gid + 1] - rb);
                st_nt(dst++, make_uint4(gid, len, (uint32_t)rb, (uint32_t)(rb >> 32)));
                ev += len;
            }
        }
    }
    ev = wave_sum<unsigned long long>(ev);
    if (lane == 0) wev[wv] = ev;
    __syncthreads();
    if (tid == 0 && live) {
        unsigned long long be = 0, bv = 0;
        uint32_t bd = 0;
        for (uint32_t i = 0; i < NW; ++i) {
            be += wext[i];
            bd += wdis[i];
            bv += wev[i];
        }
        // events: <= 1024 rows of < 2^16 records; external: <= 1024 x kMaxPois
        st_nt(a.blk_stat + blk, make_uint4(btot, (uint32_t)bv, (uint32_t)be, 0u));
        if (a.grp_atomic && btot) atomicAdd(&a.grp_cnt[(t & 1u) * a.ngrp + blk / kGroup], btot);
        if (bd) atomicAdd((unsigned long long*)&a.ctrl->disagree, (unsigned long long)bd);
    }
}

__global__ __launch_bounds__(256) void k_update(StepArgs a, uint32_t k)
{
    __shared__ uint32_t wtot[4];
    __shared__ unsigned long long wext[4];
    __shared__ uint32_t wdis[4];
    __shared__ unsigned long long wev[4];
    __shared__ uint32_t pois_s[kMaxPois];
    const uint32_t tid = threadIdx.x;
    if (tid < a.npois) pois_s[tid] = a.poisc[tid];
    __syncthreads();
    const uint32_t q = blockIdx.x * 256u + tid;
    const uint32_t t = a.ctrl->t0 + k;
    uint32_t flags = 0, ext_tot = 0, dis = 0;
    if (q < a.nq) {
        int4* rp = reinterpret_cast<int4*>(a.ring + (size_t)(t & (kRing - 1u)) * a.N) + q;
        const int4 in = *rp;
        st_nt(rp, make_int4(0, 0, 0, 0));
        flags = update_quad(a, pois_s, q, t, in, ext_tot, dis);
    }
    block_compact<4>(a, blockIdx.x, t, q, flags, ext_tot, dis, threadIdx.x, true, wtot, wext, wdis, wev);
}

// ---------------------------------------------------------------------------
// Ordered global compaction for direct delivery: block g owns update blocks
// [kGroup g, kGroup g + kGroup); its base offset is the sum of the group
// counts before it (this step's parity buffer).  Each thread places one spike
// (binary search over the group's block offsets), copying its {gid, row
// length, row start} record to the step's spike list and writing the AER
// history entry.  Also clears this group's entry of the other parity buffer
// for the next step and adds its blocks' event counts to the totals (and to
// the step's event total that decides two-level binning).  Single-level binned
// delivery does this compaction inside its scatter kernel instead.
// ---------------------------------------------------------------------------
constexpr uint32_t kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void k_compact(StepArgs a, uint32_t k)
{
    constexpr uint32_t NW = kCompactThreads / 64;
    __shared__ uint32_t red[NW];
    __shared__ uint32_t boff[kGroup + 1];
    const uint32_t g = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint32_t t = a.ctrl->t0 + k, par = t & 1u;
    const uint32_t* gc = a.grp_cnt + par * a.ngrp;
    uint32_t s = 0;
    for (uint32_t i = tid; i < g; i += kCompactThreads) s += gc[i];
    s = wave_sum<uint32_t>(s);
    if (lane == 0) red[wv] = s;
    const uint32_t b0 = g * kGroup;
    const uint32_t nb = (a.nblk - b0) < kGroup ? (a.nblk - b0) : kGroup;
    if (wv == 0) {
        const uint32_t c = lane < nb ? a.blk_stat[b0 + lane].x : 0u;
        const uint32_t v = wave_incl_scan<uint32_t>(c, lane);
        if (lane < kGroup) boff[lane + 1u] = v;
        if (lane == 0) boff[0] = 0;
    }
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t i = 0; i < NW; ++i) base += red[i];
    const uint32_t gtot = boff[nb];
    const uint64_t h0 = a.ctrl->hist_n;
    for (uint32_t i = tid; i < gtot; i += kCompactThreads) {
        uint32_t lo = 0, hi = nb;   // boff[lo] <= i < boff[hi]
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (boff[mid] <= i) lo = mid;
            else hi = mid;
        }
        const uint4 rec = a.blk_list[(size_t)(b0 + lo) * kNeuronsPerBlock + (i - boff[lo])];
        const uint32_t p = base + i;
        a.spk[p] = rec;
        const uint64_t hp = h0 + p;
        if (hp < a.hist_cap) a.hist[hp] = make_uint2(t, rec.x);
    }
    if (tid == 0) {
        a.grp_cnt[(par ^ 1u) * a.ngrp + g] = 0u;
        unsigned long long be = 0, bx = 0;
        for (uint32_t i = 0; i < nb; ++i) {
            const uint4 st = a.blk_stat[b0 + i];
            be += st.y;
            bx += st.z;
        }
        if (be) {
            atomicAdd((unsigned long long*)&a.ctrl->rec_events, be);
            atomicAdd((unsigned long long*)&a.ctrl->step_ev[par], be);   // two-level binning's switch
        }
        if (bx) atomicAdd((unsigned long long*)&a.ctrl->ext_events, bx);
        if (g == 0) a.ctrl->step_ev[par ^ 1u] = 0;
        if (g == a.ngrp - 1u) {
            a.ctrl->nspk = base + gtot;
            a.ctrl->spikes += base + gtot;
        }
    }
}

// ---------------------------------------------------------------------------
// Delivery.  Work item = (spike, segment of 64*U records of its row); one wave
// per item.  Each lane loads U records (coalesced), finds its delay bucket
// from the row's bucket ends (held one per lane: a ballot gives the bucket of
// the first record of each 64-record chunk, and only the few ends falling
// inside the chunk are walked), and adds the fixed-point weight into
// ring[(t + delay) mod 32][target] with a non-returning device-scope atomic.
// ---------------------------------------------------------------------------
// One work item of direct delivery: segment `seg` (64*U records) of the row of
// spike record `info`, one global atomic per event.
template <int U, bool CODE8>
__device__ __forceinline__ void deliver_item(const StepArgs& a, uint32_t t, uint4 info, uint32_t seg,
                                             uint32_t lane, const int32_t* cb)
{
    constexpr uint32_t SEG = 64u * U;
    const uint32_t pre = (uint32_t)__builtin_amdgcn_readfirstlane((int)info.x);
    const uint32_t len = (uint32_t)__builtin_amdgcn_readfirstlane((int)info.y);
    const uint64_t rb = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)info.z) |
                        ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)info.w) << 32);
    const uint32_t c0 = seg * SEG;
    if (c0 >= len) return;
    // 8-bit codes: the row's bucket ends, one per lane (8-byte records carry
    // their bucket)
    const uint32_t be = (CODE8 && lane < a.D) ? (uint32_t)a.bend[(size_t)pre * a.D + lane] : 0xFFFFFFFFu;
    uint32_t tg[U];
    int32_t wq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {   // all loads issued before any use
        uint32_t kk = c0 + 64u * u + lane;
        kk = kk < len ? kk : len - 1u;
        if (CODE8) {
            const uint32_t v = reinterpret_cast<const uint32_t*>(a.recs)[rb + kk];
            tg[u] = v >> 8;
            wq[u] = (int32_t)(v & 255u);
        } else {
            const Rec8 r = reinterpret_cast<const Rec8*>(a.recs)[rb + kk];
            tg[u] = r.tgt;
            wq[u] = __float2int_rn(r.w * 65536.0f);
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t c = c0 + 64u * u;
        if (c >= len) break;
        const uint32_t kk = c + lane;
        uint32_t bl;
        if (CODE8) {
            bl = popc(__ballot(be <= c));
            uint64_t inm = __ballot(be > c && be < c + 64u);
            while (inm) {
                const uint32_t l = (uint32_t)__builtin_ctzll(inm);
                inm &= inm - 1u;
                bl += (kk >= readlane(be, l)) ? 1u : 0u;
            }
        } else {
            bl = tg[u] >> kTgtBits;
            tg[u] &= kTgtMask;
        }
        if (kk < len) {
            const int32_t w = CODE8 ? cb[wq[u]] : wq[u];
            const uint32_t slot = (t + a.d_min + bl) & (kRing - 1u);
            __hip_atomic_fetch_add(a.ring + (size_t)slot * a.N + tg[u], w, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int U, bool CODE8>
__device__ __forceinline__ void deliver_direct(const StepArgs& a, uint32_t t, uint32_t n, uint32_t smax,
                                               uint32_t wave, uint32_t nw, uint32_t lane, const int32_t* cb)
{
    const uint32_t items = n * smax;    // host guarantees N * smax < 2^32
    uint32_t it = wave;
    uint4 nxt = make_uint4(0, 0, 0, 0);
    if (it < items) nxt = a.spk[it / smax];
    while (it < items) {
        const uint4 info = nxt;
        const uint32_t seg = it % smax;
        const uint32_t itn = it + nw;
        if (itn < items) nxt = a.spk[itn / smax];     // prefetch the next item's spike record
        it = itn;
        deliver_item<U, CODE8>(a, t, info, seg, lane, cb);
    }
}

template <int U, bool CODE8>
__global__ __launch_bounds__(256) void k_deliver(StepArgs a, uint32_t k, uint32_t smax)
{
    __shared__ int32_t cb_s[256];
    if (CODE8) {
        cb_s[threadIdx.x] = a.cb[threadIdx.x];
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * 256u + threadIdx.x) >> 6;
    const uint32_t nw = (gridDim.x * 256u) >> 6;
    const uint32_t t = a.ctrl->t0 + k;
    const uint32_t n = a.ctrl->nspk;
    if (wave == 0 && lane == 0) a.ctrl->hist_n += n;
    deliver_direct<U, CODE8>(a, t, n, smax, wave, nw, lane, cb_s);
}

// Binned delivery pays a fixed price per step (every tile's D ring rows are
// read and written), so steps with few events are delivered directly instead.
// The scatter kernel totals the step's events from the update blocks' counts
// and takes the decision; it leaves the total in the control block for the
// step's tile kernel.
__device__ __forceinline__ bool step_binned(const StepArgs& a, uint32_t t)
{
    return a.ctrl->step_ev[t & 1u] >= a.bin_threshold;
}

// ---------------------------------------------------------------------------
// Tile-binned delivery, phase A (scatter).  Scattered global atomics are
// limited to a few tens of G/s on this GPU, so events are first grouped by
// target tile (1024 targets).  A workgroup takes a chunk of row segments and
//   1. counts the chunk's events per tile in LDS,
//   2. reserves room in each tile's bin with one global atomic per tile,
//   3. re-reads the records, encodes each event in 32 bits
//      (target & 1023 | delay bucket << 10 | weight field << 15) and stages
//      it in LDS sorted by tile,
//   4. writes each tile's run contiguously into the tile's bin.
// Events that do not fit in a bin fall back to a direct ring atomic.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t decode_weight(uint32_t field, bool code8, const int32_t* cb, int32_t winh)
{
    if (code8) return cb[field];
    return field == kWInhField ? winh : (int32_t)field - 65536;
}

// One row segment (256 records) of the scatter phase, held in registers from
// the counting pass to the staging pass: this lane's four records (target,
// weight field) and the row's bucket ends (one per lane).
struct SegLoad {
    uint32_t len, s0, be;
    uint32_t tg[4], wf[4];
};

template <bool CODE8>
__device__ __forceinline__ void seg_load(const StepArgs& a, uint4 info, uint32_t seg, uint32_t lane, SegLoad& L)
{
    const uint32_t pre = (uint32_t)__builtin_amdgcn_readfirstlane((int)info.x);
    L.len = (uint32_t)__builtin_amdgcn_readfirstlane((int)info.y);
    const uint64_t rb = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)info.z) |
                        ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)info.w) << 32);
    L.s0 = seg * 256u;
    L.be = 0xFFFFFFFFu;
    if (L.s0 >= L.len) return;
    if (CODE8 && lane < a.D) L.be = (uint32_t)a.bend[(size_t)pre * a.D + lane];   // 8-byte records carry their bucket
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        uint32_t kk = L.s0 + 64u * u + lane;
        kk = kk < L.len ? kk : L.len - 1u;
        if (CODE8) {
            L.tg[u] = reinterpret_cast<const uint32_t*>(a.recs)[rb + kk];   // raw: decoded by seg_decode
        } else {
            const uint2 r = reinterpret_cast<const uint2*>(a.recs)[rb + kk];  // {target, weight bits}
            L.tg[u] = r.x;
            L.wf[u] = r.y;
        }
    }
}

// The loaded records as (target, weight field): kept raw until here so that
// the loads of a chunk can stay in flight while the previous chunk's runs are
// written.
template <bool CODE8>
__device__ __forceinline__ void seg_decode(const StepArgs& a, SegLoad& L)
{
    if (L.s0 >= L.len) return;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (CODE8) {
            const uint32_t v = L.tg[u];
            L.tg[u] = v >> 8;
            L.wf[u] = v & 255u;
        } else {
            // weight field (17 bits) and, above it, the record's bucket
            const int32_t wq = __float2int_rn(__uint_as_float(L.wf[u]) * 65536.0f);
            L.wf[u] = (wq == a.winh_q ? kWInhField : (uint32_t)(wq + 65536)) | ((L.tg[u] >> kTgtBits) << 17);
            L.tg[u] &= kTgtMask;
        }
    }
}

// A bin covers the 2^SHIFT targets of a tile (SHIFT = kTileBits).  The event
// code keeps the target's low SHIFT bits, the delay bucket and the weight
// field: target & (2^SHIFT - 1) | bucket << SHIFT | weight field << (SHIFT + 5).
template <uint32_t SHIFT>
__device__ __forceinline__ void seg_count(const SegLoad& L, uint32_t lane, uint32_t* tcnt)
{
    if (L.s0 >= L.len) return;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (L.s0 + 64u * u + lane < L.len) atomicAdd(&tcnt[L.tg[u] >> SHIFT], 1u);
}

// CODE8: the bucket from the row's bucket ends (L.be); 8-byte records: from
// the weight field's top bits (seg_decode).
template <uint32_t SHIFT, bool CODE8>
__device__ __forceinline__ void seg_stage(const SegLoad& L, uint32_t lane, uint32_t* tcnt, uint32_t* stage)
{
    if (L.s0 >= L.len) return;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t c = L.s0 + 64u * u;
        if (c >= L.len) break;
        const uint32_t kk = c + lane;
        uint32_t bl, wf;
        if (CODE8) {
            bl = popc(__ballot(L.be <= c));
            uint64_t inm = __ballot(L.be > c && L.be < c + 64u);
            while (inm) {
                const uint32_t l = (uint32_t)__builtin_ctzll(inm);
                inm &= inm - 1u;
                bl += (kk >= readlane(L.be, l)) ? 1u : 0u;
            }
            wf = L.wf[u];
        } else {
            bl = L.wf[u] >> 17;
            wf = L.wf[u] & 0x1FFFFu;
        }
        if (kk < L.len) {
            const uint32_t p = atomicAdd(&tcnt[L.tg[u] >> SHIFT], 1u);
            stage[p] = (L.tg[u] & ((1u << SHIFT) - 1u)) | (bl << SHIFT) | (wf << (SHIFT + 5u));
        }
    }
}

constexpr uint32_t kScatterThreads = 1024;
constexpr uint32_t kScatterWaves = kScatterThreads / 64;
constexpr uint32_t kSegPerWave = kChunkItems / kScatterWaves;   // 5 row segments per wave
// Lanes that write one bin's run in the last scatter phase: a chunk puts a few
// dozen events in a typical bin, and the phase is bound by the latency of its
// per-bin steps, so four bins go at once per wave.
constexpr uint32_t kRunLanes = 16;

// Spike s of the step's ascending-id list: its update block is found in the
// exclusive block offsets boff[0 .. nb] (UNIFORM: s is wave-uniform).
template <bool UNIFORM = true>
__device__ __forceinline__ uint4 spike_rec(const StepArgs& a, const uint32_t* boff, uint32_t nb, uint32_t s)
{
    uint32_t lo = 0, hi = nb;   // boff[lo] <= s < boff[hi]
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (boff[mid] <= s) lo = mid;
        else hi = mid;
    }
    uint32_t i = s - boff[lo];
    if (UNIFORM) {
        lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
        i = (uint32_t)__builtin_amdgcn_readfirstlane((int)i);
    }
    return a.blk_list[(size_t)lo * kNeuronsPerBlock + i];
}

// AER history of step t, written once the step's delivery is under way: the
// workgroups share the spikes in ascending order.
__device__ __forceinline__ void write_history(const StepArgs& a, const uint32_t* boff, uint32_t nb, uint32_t n,
                                              uint32_t t)
{
    const uint64_t h0 = a.ctrl->hist_n;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = nb;   // boff[lo] <= s < boff[hi]
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (boff[mid] <= s) lo = mid;
            else hi = mid;
        }
        const uint32_t gid = a.blk_list[(size_t)lo * kNeuronsPerBlock + (s - boff[lo])].x;
        if (h0 + s < a.hist_cap) a.hist[h0 + s] = make_uint2(t, gid);
    }
}

// Step t's delivery through the tile bins, or directly when the step is below
// the switch threshold.  The ordered compaction of the step's spikes (the
// update blocks' ascending lists placed by an exclusive scan of their counts)
// happens here: every workgroup scans the block counts in LDS and addresses
// spike records in the per-block lists; the workgroups write the AER history
// in ascending order; workgroup 0 publishes the spike count and the step's
// event totals.
template <bool CODE8>
__global__ __launch_bounds__(kScatterThreads) void k_scatter(StepArgs a, uint32_t k, uint32_t smax)
{
    constexpr uint32_t SHIFT = kTileBits;
    // row segments per wave and chunk: 8-byte records carry their bucket, so
    // a segment holds no bucket ends and six fit the registers (8-bit codes: five)
    constexpr uint32_t SPW = CODE8 ? kSegPerWave : kSegPerWave + 1u;
    constexpr uint32_t CHUNK = kScatterWaves * SPW;
    __shared__ uint32_t stage[CHUNK * 256u];
    __shared__ uint32_t tcnt2[2][kMaxTiles];   // counts, then fill cursor (by chunk parity)
    __shared__ uint32_t toff[kMaxTiles];   // start of each bin's run in `stage`
    __shared__ uint32_t tres[kMaxTiles];   // reserved offset in the bin
    __shared__ uint32_t boff[kMaxTiles + 1];
    __shared__ uint4 info_s[CHUNK + kScatterWaves];  // spike records of the chunk whose segments load next
    __shared__ int32_t cb_s[256];
    __shared__ uint32_t wsum[kScatterWaves];
    __shared__ unsigned long long red[2 * kScatterWaves + 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));   // uniform: scalar registers
    if (CODE8 && tid < 256u) cb_s[tid] = a.cb[tid];
    const uint32_t t = a.ctrl->t0 + k;
    const uint32_t nb = a.nblk;          // <= kMaxTiles
    bool binned;
    uint32_t n;
    {
        // exclusive scan of the update blocks' spike counts (two blocks per
        // thread) and the step's recurrent and external event totals: the
        // event total decides binned vs direct; workgroup 0 books the totals
        const uint32_t i0 = 2u * tid, i1 = 2u * tid + 1u;
        const uint4 s0 = i0 < nb ? a.blk_stat[i0] : make_uint4(0, 0, 0, 0);
        const uint4 s1 = i1 < nb ? a.blk_stat[i1] : make_uint4(0, 0, 0, 0);
        const uint32_t sum = s0.x + s1.x;
        const uint32_t inc = wave_incl_scan<uint32_t>(sum, lane);
        const unsigned long long e = wave_sum<unsigned long long>((unsigned long long)s0.y + s1.y);
        const unsigned long long x = wave_sum<unsigned long long>((unsigned long long)s0.z + s1.z);
        if (lane == 63u) wsum[wv] = inc;
        if (lane == 0) {
            red[wv] = e;
            red[kScatterWaves + wv] = x;
        }
        __syncthreads();
        uint32_t off = inc - sum;
        for (uint32_t i = 0; i < wv; ++i) off += wsum[i];
        if (i0 <= nb) boff[i0] = off;
        if (i1 <= nb) boff[i1] = off + s0.x;
        if (i1 + 1u == nb) boff[nb] = off + sum;
        if (tid == 0) {
            unsigned long long et = 0, xt = 0;
            for (uint32_t i = 0; i < kScatterWaves; ++i) {
                et += red[i];
                xt += red[kScatterWaves + i];
            }
            red[2 * kScatterWaves] = et;
            if (blockIdx.x == 0) {
                a.ctrl->rec_events += et;
                a.ctrl->ext_events += xt;
                a.ctrl->step_ev[t & 1u] = et;   // the tile kernel's copy of the switch decision
            }
        }
        __syncthreads();
        binned = __builtin_amdgcn_readfirstlane(red[2 * kScatterWaves] >= a.bin_threshold ? 1 : 0) != 0;
        n = (uint32_t)__builtin_amdgcn_readfirstlane((int)boff[nb]);
        if (blockIdx.x == 0 && tid == 0) {
            a.ctrl->nspk = n;
            a.ctrl->spikes += n;
        }
    }
    // spike s of the step (wave-uniform s)
    auto spike = [&](uint32_t s) { return spike_rec(a, boff, nb, s); };
    if (!binned) {
        const uint32_t items = n * smax;    // host guarantees N * smax < 2^32
        const uint32_t nw = gridDim.x * kScatterWaves;
        for (uint32_t it = blockIdx.x * kScatterWaves + wv; it < items; it += nw)
            deliver_item<4, CODE8>(a, t, spike(it / smax), it % smax, lane, cb_s);
        write_history(a, boff, nb, n, t);
        return;
    }
    const uint32_t items = n * smax;
    const uint32_t nt = a.ntiles;
    const uint32_t cap = a.bin_cap_tile;
    uint32_t* const fill = a.bin_fill;
    uint32_t* const bins = a.bins;
    // chunk size: large chunks bin better, but every workgroup should get work
    uint32_t per = (items + gridDim.x - 1u) / gridDim.x;
    per = per < kScatterWaves ? kScatterWaves : (per > CHUNK ? CHUNK : per);
    unsigned long long spill = 0;
    // this wave's row segments of chunk [c0, c1): items c0 + wv + 16 j, all
    // loads issued before use; the next chunk's segments are loaded while the
    // current chunk's runs are written (phase 4)
    //
    // The spike records a chunk's segments start from are fetched one chunk
    // earlier still: lane j of a wave fetches its segment j's record (a
    // register while phase 4 runs), the top of the next chunk parks it in
    // info_s, and the segments' loads read it there.
    SegLoad S[SPW];
    uint4 nxt = make_uint4(0, 0, 0, 0);
    auto fetch_info = [&](uint32_t c0, uint32_t c1) {
        const uint32_t it = c0 + wv + kScatterWaves * lane;
        if (lane < SPW && it < c1)
            nxt = spike_rec<false>(a, boff, nb, it / smax);
        else
            nxt = make_uint4(0, 0, 0, 0);
    };
    auto park_info = [&]() {   // every lane stores (lanes past the segments to a spare slot)
        info_s[lane < SPW ? wv + kScatterWaves * lane : CHUNK + wv] = nxt;
    };
    auto load_chunk = [&](uint32_t c0, uint32_t c1) {
#pragma unroll
        for (uint32_t j = 0; j < SPW; ++j) {
            const uint32_t it = c0 + wv + kScatterWaves * j;
            seg_load<CODE8>(a, info_s[wv + kScatterWaves * j], it < c1 ? it % smax : 0u, lane, S[j]);
        }
    };
    auto chunk_end = [&](uint32_t c0) { return (items - c0) < per ? items : c0 + per; };
    const uint32_t stride = gridDim.x * per;
    // a chunk counts into one of two arrays; the other is cleared while the
    // chunk writes its runs, so no barrier separates clearing from counting
    for (uint32_t i = tid; i < nt; i += kScatterThreads) tcnt2[0][i] = 0;
    uint32_t par = 0;
    if (blockIdx.x * per < items) {
        fetch_info(blockIdx.x * per, chunk_end(blockIdx.x * per));
        park_info();
        __syncthreads();
        load_chunk(blockIdx.x * per, chunk_end(blockIdx.x * per));
        const uint32_t n1 = blockIdx.x * per + stride;
        fetch_info(n1, n1 < items ? chunk_end(n1) : n1);
    }
    for (uint32_t c0 = blockIdx.x * per; c0 < items; c0 += stride, par ^= 1u) {
        uint32_t* const tcnt = tcnt2[par];
        park_info();   // the next chunk's spike records (zeros past the end)
#pragma unroll
        for (uint32_t j = 0; j < SPW; ++j) seg_decode<CODE8>(a, S[j]);
        // 1. histogram of targets by bin
#pragma unroll
        for (uint32_t j = 0; j < SPW; ++j) seg_count<SHIFT>(S[j], lane, tcnt);
        __syncthreads();
        // 2. exclusive scan of the counts (2 bins per thread) and reservation
        // in the bins; the reservations' results are first needed in phase 4,
        // so they stay in registers (in flight) while phase 3 stages
        const uint32_t t0i = 2u * tid, t1i = 2u * tid + 1u;
        uint32_t res0 = 0, res1 = 0;
        {
            const uint32_t v0 = t0i < nt ? tcnt[t0i] : 0u;
            const uint32_t v1 = t1i < nt ? tcnt[t1i] : 0u;
            const uint32_t sum = v0 + v1;
            const uint32_t inc = wave_incl_scan<uint32_t>(sum, lane);
            if (lane == 63u) wsum[wv] = inc;
            __syncthreads();
            uint32_t off = inc - sum;
            for (uint32_t i = 0; i < wv; ++i) off += wsum[i];
            if (t0i < nt) {
                toff[t0i] = off;
                tcnt[t0i] = off;
                if (v0) res0 = atomicAdd(&fill[(size_t)t0i * kFillStride], v0);
            }
            if (t1i < nt) {
                toff[t1i] = off + v0;
                tcnt[t1i] = off + v0;
                if (v1) res1 = atomicAdd(&fill[(size_t)t1i * kFillStride], v1);
            }
        }
        __syncthreads();
        // 3. encode and stage sorted by bin
#pragma unroll
        for (uint32_t j = 0; j < SPW; ++j) seg_stage<SHIFT, CODE8>(S[j], lane, tcnt, stage);
        if (t0i < nt) tres[t0i] = res0;
        if (t1i < nt) tres[t1i] = res1;
        __syncthreads();
        {
            const uint32_t n1 = c0 + stride, n2 = n1 + stride;
            fetch_info(n2, n2 < items ? chunk_end(n2) : n2);
            if (n1 < items) load_chunk(n1, chunk_end(n1));
        }
        for (uint32_t i = tid; i < nt; i += kScatterThreads) tcnt2[par ^ 1u][i] = 0;
        // 4. contiguous runs into the bins: each group of kRunLanes lanes
        // writes one bin's run at a time
        const uint32_t rl = tid % kRunLanes;
        for (uint32_t tt = tid / kRunLanes; tt < nt; tt += kScatterThreads / kRunLanes) {
            const uint32_t o0 = toff[tt];
            const uint32_t cnt = tcnt[tt] - o0;
            const uint32_t r0 = tres[tt];
            uint32_t* dst = bins + (size_t)tt * cap;
            for (uint32_t e = rl; e < cnt; e += kRunLanes) {
                const uint32_t code = stage[o0 + e];
                const uint32_t pos = r0 + e;
                if (pos < cap) {
                    dst[pos] = code;
                } else {
                    const uint32_t tgt = (tt << SHIFT) | (code & ((1u << SHIFT) - 1u));
                    const uint32_t b = (code >> SHIFT) & 31u;
                    const int32_t w = decode_weight(code >> (SHIFT + 5u), CODE8, cb_s, a.winh_q);
                    const uint32_t slot = (t + a.d_min + b) & (kRing - 1u);
                    __hip_atomic_fetch_add(a.ring + (size_t)slot * a.N + tgt, w, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    spill += 1;
                }
            }
        }
        __syncthreads();
    }
    spill = wave_sum<unsigned long long>(spill);
    if (lane == 0 && spill) atomicAdd((unsigned long long*)&a.ctrl->bin_overflow, spill);
    write_history(a, boff, nb, n, t);
}

// ---------------------------------------------------------------------------
// Two-level delivery: 8-bit-code networks with more tiles than one LDS table,
// rows laid out by super tile (k_syn_out_seg).  The step's spike list,
// history and event totals come from k_compact.
//
// k_seg_emit cuts every spike's row at its super tiles' segment starts and
// lists each nonempty segment, in pieces of at most 256 records, in its super
// tile's segment list.  A workgroup takes kEmitPass spikes per pass (each wave
// kEmitPerWave of them; lane s of a wave handles super tile s): the pieces are
// counted per super tile in LDS, one global atomic per super tile reserves the
// pass's room, and the pieces are written.  A piece beyond its list's
// capacity is delivered on the spot by one lane (a fallback, counted as
// overflow like a full bin).
// ---------------------------------------------------------------------------
constexpr uint32_t kEmitThreads = 1024;
constexpr uint32_t kEmitPerWave = 4;
constexpr uint32_t kEmitPass = kEmitThreads / 64 * kEmitPerWave;

// Record v of super tile `sup` (segmented layout) as a ring atomic.
__device__ __forceinline__ void seg_atomic(const StepArgs& a, uint32_t t, uint32_t sup, uint32_t v, const int32_t* cb)
{
    const uint32_t tgt = (sup << kSegBits) | (v & ((1u << kSegBits) - 1u));
    const uint32_t slot = (t + a.d_min + ((v >> kSegBits) & 31u)) & (kRing - 1u);
    __hip_atomic_fetch_add(a.ring + (size_t)slot * a.N + tgt, cb[v >> (kSegBits + 5u)], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kEmitThreads) void k_seg_emit(StepArgs a, uint32_t k)
{
    __shared__ uint32_t cnt[kMaxSuper];   // pieces of the pass per super tile
    __shared__ uint32_t res[kMaxSuper];   // their reserved start in the list
    __shared__ int32_t cb_s[256];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    if (tid < 256u) cb_s[tid] = a.cb[tid];
    const uint32_t t = a.ctrl->t0 + k;
    const uint32_t n = a.ctrl->nspk;
    const uint32_t ns = a.nsuper;
    const uint32_t* const recs = reinterpret_cast<const uint32_t*>(a.recs);
    unsigned long long spill = 0;
    for (uint32_t p0 = blockIdx.x * kEmitPass; p0 < n; p0 += gridDim.x * kEmitPass) {
        if (tid < kMaxSuper) cnt[tid] = 0;
        __syncthreads();
        uint32_t st[kEmitPerWave], len[kEmitPerWave], off[kEmitPerWave];
        uint64_t rb[kEmitPerWave];
#pragma unroll
        for (uint32_t i = 0; i < kEmitPerWave; ++i) {
            const uint32_t sp = p0 + wv * kEmitPerWave + i;   // wave-uniform
            st[i] = 0;
            len[i] = 0;
            off[i] = 0;
            rb[i] = 0;
            if (sp < n) {
                const uint4 r = a.spk[sp];   // {gid, row length, row start lo, hi}
                rb[i] = (uint64_t)r.z | ((uint64_t)r.w << 32);
                const uint32_t s0 = lane < ns ? (uint32_t)a.sstart[(size_t)r.x * ns + lane] : r.y;
                const uint32_t nx = (uint32_t)__shfl_down((int)s0, 1);
                const uint32_t s1 = lane + 1u < ns ? nx : r.y;
                if (lane < ns) {
                    st[i] = s0;
                    len[i] = s1 - s0;
                }
                if (len[i]) off[i] = atomicAdd(&cnt[lane], (len[i] + 255u) >> 8);
            }
        }
        __syncthreads();
        if (tid < ns) {
            const uint32_t c = cnt[tid];
            res[tid] = c ? atomicAdd(&a.dfill[(size_t)tid * kFillStride], c) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (uint32_t i = 0; i < kEmitPerWave; ++i) {
            if (!len[i]) continue;
            uint32_t pos = res[lane] + off[i];
            uint64_t r0 = rb[i] + st[i];
            for (uint32_t q = 0; q < len[i]; q += 256u, ++pos, r0 += 256u) {
                const uint32_t pl = (len[i] - q) < 256u ? len[i] - q : 256u;
                if (pos < a.dcap) {
                    a.dsc[(size_t)lane * a.dcap + pos] = make_uint2((uint32_t)r0, (uint32_t)(r0 >> 32) | (pl << 8));
                } else {
                    for (uint32_t e = 0; e < pl; ++e) seg_atomic(a, t, lane, recs[r0 + e], cb_s);
                    spill += pl;
                }
            }
        }
        __syncthreads();   // cnt and res are reused by the next pass
    }
    spill = wave_sum<unsigned long long>(spill);
    if (lane == 0 && spill) atomicAdd((unsigned long long*)&a.ctrl->bin_overflow, spill);
}

// k_seg_bin: the super tiles' segment lists are cut into chunks of up to
// kBinDesc pieces, all of one super tile.  A workgroup takes a chunk: its
// pieces' descriptors and the exclusive scan of their lengths go to LDS, and
// the chunk's records, read as one concatenated sequence, are binned in rounds
// of up to kSegStage records.  A round is kSegSlots slots of 256 records,
// kSegSlotsPerWave per wave; a wave holds the pieces of a slot in registers
// (lane l: piece f + l) and each record finds its own piece by comparing its
// position with their starts.  The records are counted by tile (kSegTiles
// tiles per super tile; the returned count is the record's rank in its
// tile), one global atomic per tile reserves room in its bin, the tile codes
// (target & 1023 | bucket << 10 | code << 15) are staged in LDS at their
// tile's offset plus their rank, and each tile's run is written into its bin
// while the next round's records are being read (at a chunk's last round the
// next chunk's descriptors go to the other LDS buffer first).  Pieces are short (a row reaches most super tiles with a few
// dozen to a few hundred records), so a wave does not take one piece per
// 256-record slot.  Events beyond a tile bin's capacity take a direct ring
// atomic.  In a step below the binning threshold every piece is delivered
// directly instead, one wave per piece.
constexpr uint32_t kBinDesc = kScatterThreads;   // pieces per chunk
// lanes per tile run in the write phase (16 measured faster than 8 or 4 on the
// 96x96 grid: 512 tiles of ~40 events per round)
constexpr uint32_t kSegRunLanes = 16;
// 256-record slots per wave and round: 28,672 records per round, the most
// the LDS holds next to the tables (147 KB); 5 slots measured 6 % slower
constexpr uint32_t kSegSlotsPerWave = 7;
constexpr uint32_t kSegSlots = kScatterWaves * kSegSlotsPerWave;
constexpr uint32_t kSegStage = kSegSlots * 256u;                 // records per round
constexpr uint32_t kGather = kSegSlotsPerWave * 4u;               // records per lane and round

__global__ __launch_bounds__(kScatterThreads) void k_seg_bin(StepArgs a, uint32_t k)
{
    __shared__ uint32_t stage[kSegStage];
    __shared__ uint32_t tcnt[kSegTiles];       // records of the round per tile
    __shared__ uint32_t toff[kSegTiles];       // start of each tile's run in `stage`
    __shared__ uint32_t tres[kSegTiles];       // reserved offset in the tile's bin
    __shared__ uint32_t cpre[kMaxSuper + 1];   // work units (chunks, or pieces) before each super tile
    __shared__ uint32_t pcnt[kMaxSuper];       // pieces listed per super tile
    __shared__ uint2 dsc_s[2][kBinDesc];       // a chunk's pieces (two buffers: this chunk, the next)
    __shared__ uint32_t pref[2][kBinDesc + 1]; // exclusive scan of their lengths
    __shared__ uint32_t first[kSegSlots];      // piece holding each slot's first record
    __shared__ int32_t cb_s[256];
    __shared__ uint32_t wsum[kScatterWaves];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    if (tid < 256u) cb_s[tid] = a.cb[tid];
    const uint32_t t = a.ctrl->t0 + k;
    const bool binned = step_binned(a, t);
    const uint32_t ns = a.nsuper;
    const uint32_t unit = binned ? kBinDesc : 1u;
    if (wv == 0) {
        uint32_t f = lane < ns ? a.dfill[(size_t)lane * kFillStride] : 0u;
        f = f < a.dcap ? f : a.dcap;
        const uint32_t c = (f + unit - 1u) / unit;
        const uint32_t inc = wave_incl_scan<uint32_t>(c, lane);
        if (lane < ns) {
            pcnt[lane] = f;
            cpre[lane + 1u] = inc;
        }
        if (lane == 0) cpre[0] = 0;
    }
    __syncthreads();
    const uint32_t total = cpre[ns];
    const uint32_t* const recs = reinterpret_cast<const uint32_t*>(a.recs);
    auto super_of = [&](uint32_t u) {   // cpre[s] <= u < cpre[s + 1] (u wave-uniform)
        uint32_t lo = 0, hi = ns;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (cpre[mid] <= u) lo = mid;
            else hi = mid;
        }
        return (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    };
    if (!binned) {
        const uint32_t nw = gridDim.x * kScatterWaves;
        for (uint32_t it = blockIdx.x * kScatterWaves + wv; it < total; it += nw) {
            const uint32_t sup = super_of(it);
            const uint2 d = a.dsc[(size_t)sup * a.dcap + (it - cpre[sup])];
            const uint64_t r0 = (uint64_t)d.x | ((uint64_t)(d.y & 255u) << 32);
            const uint32_t len = d.y >> 8;
            uint32_t v[4];
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u) {
                const uint32_t e = 64u * u + lane;
                v[u] = recs[r0 + (e < len ? e : len - 1u)];
            }
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u)
                if (64u * u + lane < len) seg_atomic(a, t, sup, v[u], cb_s);
        }
        return;
    }
    unsigned long long spill = 0;
    const uint32_t nt = kSegTiles;
    const uint32_t cap = a.bin_cap_tile;
    // Descriptors of chunk c into buffer b (one piece per thread) and the
    // exclusive scan of their lengths; two barriers.
    auto load_chunk = [&](uint32_t c, uint32_t b) {
        const uint32_t sup = super_of(c);
        const uint32_t d0 = (c - cpre[sup]) * kBinDesc;
        const uint32_t nd = (pcnt[sup] - d0) < kBinDesc ? pcnt[sup] - d0 : kBinDesc;
        uint2* const ds = dsc_s[b];
        uint32_t* const pf = pref[b];
        if (tid < kBinDesc) {
            const uint2 d = tid < nd ? a.dsc[(size_t)sup * a.dcap + d0 + tid] : make_uint2(0, 0);
            const uint32_t len = d.y >> 8;
            const uint32_t inc = wave_incl_scan<uint32_t>(len, lane);
            ds[tid] = d;
            pf[tid + 1u] = inc;   // within the wave; waves' totals added below
            if (lane == 63u) wsum[wv] = inc;
        }
        __syncthreads();
        if (tid < kBinDesc) {
            uint32_t add = 0;
            for (uint32_t i = 0; i < wv; ++i) add += wsum[i];
            pf[tid + 1u] += add;
            if (tid == 0) pf[0] = 0;
        }
        __syncthreads();
    };
    // slot j of a round: records q0 + 256 j .. + 255 of the chunk's
    // concatenated pieces, taken by wave j mod 16; the piece holding its
    // first record is found by one thread per slot
    auto find_first = [&](uint32_t q0, uint32_t b) {
        if (tid < kSegSlots) {
            const uint32_t* const pf = pref[b];
            const uint32_t P = q0 + 256u * tid;
            uint32_t lo = 0, hi = kBinDesc;   // pf[lo] <= P < pf[hi]
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (pf[mid] <= P) lo = mid;
                else hi = mid;
            }
            first[tid] = lo;
        }
    };
    // the round's records into v: a slot's pieces (one per lane: start,
    // length prefix) sit in registers, and each record finds its piece by
    // comparing its position with the prefixes
    uint32_t v[kGather], rk[kGather];
    auto gather = [&](uint32_t q0, uint32_t b) {
        const uint2* const ds = dsc_s[b];
        const uint32_t* const pfa = pref[b];
        const uint32_t R = pfa[kBinDesc];
#pragma unroll
        for (uint32_t j = 0; j < kSegSlotsPerWave; ++j) {
            const uint32_t P = q0 + 256u * (wv + kScatterWaves * j);
            const uint32_t f = first[wv + kScatterWaves * j];
            const uint32_t fl = f + lane < kBinDesc ? f + lane : kBinDesc - 1u;
            const uint32_t pf = pfa[fl];
            const uint2 dd = ds[fl];
            // the window: pieces f .. f + 63, ending where piece f + 64 starts
            const uint32_t wend = pfa[f + 64u < kBinDesc ? f + 64u : kBinDesc];
            // window pieces starting inside the slot, besides the first (uniform)
            const uint64_t inside = __ballot(lane >= 1u && f + lane < kBinDesc && pf < P + 256u && pf < R);
            const uint32_t np = 1u + popc(inside);
#pragma unroll
            for (uint32_t u = 0; u < 4u; ++u) {
                const uint32_t p = P + 64u * u + lane;
                uint32_t k = 0;
                for (uint32_t l = 1; l < np; ++l) k += readlane(pf, l) <= p ? 1u : 0u;
                uint32_t lo32 = 0, hi8 = 0, st = 0;
                for (uint32_t l = 0; l < np; ++l)
                    if (k == l) {
                        lo32 = readlane(dd.x, l);
                        hi8 = readlane(dd.y, l) & 255u;
                        st = readlane(pf, l);
                    }
                if (p >= wend && p < R) {
                    // past the window (more than 64 pieces in 256 records):
                    // the piece from the scanned lengths
                    uint32_t lo = f + 64u, hi = kBinDesc;   // pfa[lo] <= p < pfa[hi]
                    while (hi - lo > 1u) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (pfa[mid] <= p) lo = mid;
                        else hi = mid;
                    }
                    lo32 = ds[lo].x;
                    hi8 = ds[lo].y & 255u;
                    st = pfa[lo];
                }
                const uint64_t at = ((uint64_t)hi8 << 32 | lo32) + (p - st);
                v[4u * j + u] = p < R ? recs[at] : 0u;
            }
        }
    };
    if (tid < nt) tcnt[tid] = 0;
    // The workgroup's rounds in turn (chunks c = blockIdx.x, + gridDim.x, ...;
    // rounds q0 = 0, kSegStage, ... of each).  Each pass finishes the current
    // round and reads the next one's records before writing the current runs;
    // the first pass only reads.
    bool cur = false;                 // a current round (records in v)
    uint32_t c = 0, q0 = 0, buf = 0, R = 0, sup = 0;
    for (;;) {
        if (cur) {
            // 1. histogram by tile; the returned count is the record's rank
            //    among the round's records of its tile
#pragma unroll
            for (uint32_t i = 0; i < kGather; ++i) {
                const uint32_t p = q0 + 256u * (wv + kScatterWaves * (i >> 2)) + 64u * (i & 3u) + lane;
                rk[i] = p < R ? atomicAdd(&tcnt[(v[i] >> kTileBits) & (kSegTiles - 1u)], 1u) : 0u;
            }
        }
        __syncthreads();
        // 2. exclusive scan of the counts (one tile per thread) and
        //    reservation in the bins; the reservations' results are first
        //    needed in phase 4, so they stay in flight while phase 3 stages
        uint32_t res = 0;
        if (cur && tid < nt) {
            const uint32_t cnt = tcnt[tid];
            const uint32_t inc = wave_incl_scan<uint32_t>(cnt, lane);
            if (lane == 63u) wsum[wv] = inc;
            toff[tid] = inc - cnt;   // within the wave for now
            if (cnt) res = atomicAdd(&a.bin_fill[(size_t)(sup * kSegTiles + tid) * kFillStride], cnt);
        }
        __syncthreads();
        if (cur) {
            if (tid < nt) {
                uint32_t add = 0;
                for (uint32_t i = 0; i < wv; ++i) add += wsum[i];
                toff[tid] += add;
            }
        }
        __syncthreads();
        if (cur) {
            // 3. tile codes staged sorted by tile, each at its tile's start
            //    plus its rank
#pragma unroll
            for (uint32_t i = 0; i < kGather; ++i) {
                const uint32_t p = q0 + 256u * (wv + kScatterWaves * (i >> 2)) + 64u * (i & 3u) + lane;
                if (p < R) {
                    const uint32_t x = v[i];
                    stage[toff[(x >> kTileBits) & (kSegTiles - 1u)] + rk[i]] =
                        (x & (kTile - 1u)) | (((x >> kSegBits) & 31u) << kTileBits) | ((x >> (kSegBits + 5u)) << 15);
                }
            }
            if (tid < nt) tres[tid] = res;
        }
        __syncthreads();
        // the next round: of this chunk, or the workgroup's next chunk (its
        // descriptors into the other buffer); its records are read while this
        // round's runs are written
        bool nxt = false, load = false;
        uint32_t nc = c, nq = q0 + kSegStage, nb = buf;
        if (cur && nq < R) {
            nxt = true;
        } else {
            nc = cur ? c + gridDim.x : blockIdx.x;
            nq = 0;
            nb = cur ? buf ^ 1u : 0u;
            nxt = load = nc < total;
        }
        if (nxt) {
            if (load) load_chunk(nc, nb);
            find_first(nq, nb);
            __syncthreads();
            gather(nq, nb);
        }
        if (cur) {
            // 4. contiguous runs into the bins: each group of kSegRunLanes
            // lanes writes one tile's run at a time
            const uint32_t rl = tid % kSegRunLanes;
            for (uint32_t tt = tid / kSegRunLanes; tt < nt; tt += kScatterThreads / kSegRunLanes) {
                const uint32_t o0 = toff[tt];
                const uint32_t cnt = tcnt[tt];
                const uint32_t r0 = tres[tt];
                const uint32_t tile = sup * kSegTiles + tt;
                uint32_t* dst = a.bins + (size_t)tile * cap;
                for (uint32_t e = rl; e < cnt; e += kSegRunLanes) {
                    const uint32_t code = stage[o0 + e];
                    const uint32_t pos = r0 + e;
                    if (pos < cap) {
                        dst[pos] = code;
                    } else {
                        const uint32_t tgt = (tile << kTileBits) | (code & (kTile - 1u));
                        const uint32_t b = (code >> kTileBits) & 31u;
                        const uint32_t slot = (t + a.d_min + b) & (kRing - 1u);
                        __hip_atomic_fetch_add(a.ring + (size_t)slot * a.N + tgt, cb_s[code >> 15], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        spill += 1;
                    }
                }
            }
        }
        __syncthreads();
        if (tid < nt) tcnt[tid] = 0;   // the next round's histogram
        if (!nxt) break;
        cur = true;
        c = nc;
        q0 = nq;
        buf = nb;
        R = pref[buf][kBinDesc];
        sup = super_of(c);
    }
    spill = wave_sum<unsigned long long>(spill);
    if (lane == 0 && spill) atomicAdd((unsigned long long*)&a.ctrl->bin_overflow, spill);
}

// ---------------------------------------------------------------------------
// Tile-binned delivery, phase B: one workgroup per tile of 1024 targets.  The
// tile's D future ring rows are loaded into LDS, the tile's binned events are
// added with LDS atomics, and the rows are written back (coalesced 16-byte
// accesses); the bin is emptied for the next step.
// ---------------------------------------------------------------------------
constexpr uint32_t kTileThreads = 1024;

// Spikers of one update block appended, unordered, to the network's spike
// list of step t (batched stepping): one atomic per block reserves room, each
// spiker writes its record {gid, row length, row start} and history entry, and
// the block's spike, external and recurrent event counts are accumulated
// (including the step's event total used by the delivery switch).
template <uint32_t NW>
// The block's NW waves are threads [0, 64 NW) of a thread group (gtid = index
// in the group, as in block_compact); a group without a block passes
// live = false and takes part in the barriers only.
__device__ __forceinline__ void block_append(const StepArgs& a, uint32_t t, uint32_t q, uint32_t flags,
                                             uint32_t ext_tot, uint32_t gtid, bool live, uint32_t* wtot,
                                             unsigned long long* wext, unsigned long long* wev, uint32_t* sbase)
{
    const uint32_t tid = gtid, lane = tid & 63u, wv = tid >> 6;
    const uint64_t m0 = __ballot(flags & 1u), m1 = __ballot(flags & 2u);
    const uint64_t m2 = __ballot(flags & 4u), m3 = __ballot(flags & 8u);
    const uint32_t pre = mbcnt(m0) + mbcnt(m1) + mbcnt(m2) + mbcnt(m3);
    const uint32_t wt = popc(m0) + popc(m1) + popc(m2) + popc(m3);
    const unsigned long long we = wave_sum<unsigned long long>(ext_tot);
    if (lane == 0) {
        wtot[wv] = wt;
        wext[wv] = we;
    }
    __syncthreads();
    uint32_t woff = 0, btot = 0;
    unsigned long long bext = 0;
    for (uint32_t i = 0; i < NW; ++i) {
        if (i < wv) woff += wtot[i];
        btot += wtot[i];
        bext += wext[i];
    }
    if (tid == 0 && live) {
        *sbase = btot ? atomicAdd(&a.ctrl->nspk_par[t & 1u], btot) : 0u;
        if (bext) atomicAdd((unsigned long long*)&a.ctrl->ext_events, bext);
        if (btot) atomicAdd((unsigned long long*)&a.ctrl->spikes, (unsigned long long)btot);
    }
    __syncthreads();
    unsigned long long ev = 0;
    if (flags) {
        uint32_t p = *sbase + woff + pre;
        const uint64_t h0 = a.ctrl->hist_n;
        for (uint32_t s = 0; s < 4u; ++s) {
            if (flags & (1u << s)) {
                const uint32_t gid = 4u * q + s;
                const uint64_t rb = a.row_ptr[gid];
                const uint32_t len = (uint32_t)(a.row_ptr[gid + 1] - rb);
                a.spk[p] = make_uint4(gid, len, (uint32_t)rb, (uint32_t)(rb >> 32));
                if (h0 + p < a.hist_cap) a.hist[h0 + p] = make_uint2(t, gid);
                ev += len;
                ++p;
            }
        }
    }
    ev = wave_sum<unsigned long long>(ev);
    if (lane == 0) wev[wv] = ev;
    __syncthreads();
    if (tid == 0 && live) {
        unsigned long long be = 0;
        for (uint32_t i = 0; i < NW; ++i) be += wev[i];
        if (be) {
            atomicAdd((unsigned long long*)&a.ctrl->rec_events, be);
            atomicAdd((unsigned long long*)&a.ctrl->step_ev[t & 1u], be);
        }
    }
}

// Phase B of binned delivery for tile tt of one network at step t (see
// k_tile), optionally followed (UPD, d_min == 1, upd_live) by the neuron
// update of step t + 1 for the tile's 1024 neurons.  The first LDS row is slot
// t + 1: it is handed to the update and written back as zeros, and its LDS
// space then holds the update's small tables, so no static LDS is needed and
// two workgroups fit a CU.  APPEND selects the batched (unordered) spike
// compaction instead of the ordered per-block one.
template <bool CODE8, bool UPD, bool APPEND>
__device__ __forceinline__ void tile_work(const StepArgs& a, uint32_t tt, uint32_t t, bool binned, bool upd_live,
                                          int32_t* acc)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t g0 = tt << kTileBits;
    const uint32_t nn = (a.N - g0) < kTile ? (a.N - g0) : kTile;
    const uint32_t D = a.D;
    const bool do_upd = UPD && upd_live;
    if (!do_upd && !binned) return;
    if (binned) {
        for (uint32_t idx = tid; idx < D * (kTile / 4u); idx += kTileThreads) {
            const uint32_t b = idx / (kTile / 4u), q = idx % (kTile / 4u);
            int4 v = make_int4(0, 0, 0, 0);
            if (4u * q < nn) {
                const uint32_t slot = (t + a.d_min + b) & (kRing - 1u);
                v = reinterpret_cast<const int4*>(a.ring + (size_t)slot * a.N + g0)[q];
            }
            reinterpret_cast<int4*>(acc)[idx] = v;
        }
        __syncthreads();
        const uint32_t fill = a.bin_fill[(size_t)tt * kFillStride];
        const uint32_t cap = a.bin_cap_tile;
        const uint32_t n = fill < cap ? fill : cap;
        const uint32_t* ev = a.bins + (size_t)tt * cap;
        // U codes per thread and pass; the next pass's codes are read while
        // this pass's are added
        constexpr uint32_t U = 8;
        uint32_t code[U], nxt[U];
        auto fetch = [&](uint32_t e0, uint32_t* c) {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t e = e0 + u * kTileThreads + tid;
                c[u] = e < n ? ev[e] : 0xFFFFFFFFu;
            }
        };
        fetch(0, nxt);
        for (uint32_t e0 = 0; e0 < n; e0 += U * kTileThreads) {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) code[u] = nxt[u];
            if (e0 + U * kTileThreads < n) fetch(e0 + U * kTileThreads, nxt);
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                if (code[u] != 0xFFFFFFFFu) {
                    const uint32_t b = (code[u] >> kTileBits) & 31u;
                    atomicAdd(&acc[b * kTile + (code[u] & (kTile - 1u))],
                              decode_weight(code[u] >> 15, CODE8, a.cb, a.winh_q));
                }
            }
        }
        __syncthreads();
    }
    uint32_t flags = 0, ext_tot = 0, dis = 0;
    const uint32_t q = (g0 >> 2) + tid;
    uint32_t* scratch = reinterpret_cast<uint32_t*>(acc);   // row 0 once consumed
    if (do_upd) {
        int4 in = make_int4(0, 0, 0, 0);
        if (tid < kTile / 4u && 4u * tid < nn) {
            if (binned) {
                in = reinterpret_cast<const int4*>(acc)[tid];
            } else {
                int4* rp = reinterpret_cast<int4*>(a.ring + (size_t)((t + 1u) & (kRing - 1u)) * a.N) + q;
                in = *rp;
                st_nt(rp, make_int4(0, 0, 0, 0));
            }
        }
        __syncthreads();
        if (tid < a.npois) scratch[tid] = a.poisc[tid];
        __syncthreads();
        if (tid < kTile / 4u && 4u * tid < nn) flags = update_quad(a, scratch, q, t + 1u, in, ext_tot, dis);
    }
    if (binned) {
        for (uint32_t idx = tid; idx < D * (kTile / 4u); idx += kTileThreads) {
            const uint32_t b = idx / (kTile / 4u), qq = idx % (kTile / 4u);
            if (4u * qq < nn) {
                const uint32_t slot = (t + a.d_min + b) & (kRing - 1u);
                const int4 v = (do_upd && b == 0u) ? make_int4(0, 0, 0, 0) : reinterpret_cast<const int4*>(acc)[idx];
                st_nt(reinterpret_cast<int4*>(a.ring + (size_t)slot * a.N + g0) + qq, v);
            }
        }
        if (tid == 0) a.bin_fill[(size_t)tt * kFillStride] = 0u;
    }
    if (do_upd) {
        __syncthreads();   // every thread is past its use of the Poisson table
        constexpr uint32_t NW = kTileThreads / 64;
        if (APPEND)
            block_append<NW>(a, t + 1u, q, flags, ext_tot, threadIdx.x, true, scratch + 64,
                             reinterpret_cast<unsigned long long*>(scratch + 96),
                             reinterpret_cast<unsigned long long*>(scratch + 128), scratch + 160);
        else
            block_compact<NW>(a, tt, t + 1u, q, flags, ext_tot, dis, threadIdx.x, true, scratch + 64,
                              reinterpret_cast<unsigned long long*>(scratch + 96), scratch + 80,
                              reinterpret_cast<unsigned long long*>(scratch + 128));
    }
}

// Neuron update of step t for four blocks per pass, one per group of four
// waves (a step without binned delivery needs no LDS rows, so a workgroup
// covers four tiles and the whole grid fits the GPU at once).  The input is
// read from ring slot t and cleared; the LDS at `scr` holds the Poisson table
// and each group's compaction scratch.
__device__ __forceinline__ void update_groups(const StepArgs& a, uint32_t t, uint32_t* scr)
{
    const uint32_t tid = threadIdx.x, g = tid >> 8, gtid = tid & 255u;
    if (tid < a.npois) scr[tid] = a.poisc[tid];
    __syncthreads();
    uint32_t* gs = scr + 64 + 32 * g;   // per group: wtot[4] wdis[4] wext[4] wev[4] (u64)
    for (uint32_t base = 4u * blockIdx.x; base < a.nblk; base += 4u * gridDim.x) {
        const uint32_t blk = base + g;
        const bool live = blk < a.nblk;
        const uint32_t q = blk * 256u + gtid;
        uint32_t flags = 0, ext_tot = 0, dis = 0;
        if (live && q < a.nq) {
            int4* rp = reinterpret_cast<int4*>(a.ring + (size_t)(t & (kRing - 1u)) * a.N) + q;
            const int4 in = *rp;
            st_nt(rp, make_int4(0, 0, 0, 0));
            flags = update_quad(a, scr, q, t, in, ext_tot, dis);
        }
        block_compact<4>(a, blk, t, q, flags, ext_tot, dis, gtid, live, gs, reinterpret_cast<unsigned long long*>(gs + 8),
                         gs + 4, reinterpret_cast<unsigned long long*>(gs + 16));
        __syncthreads();   // the groups' scratch is reused by the next pass
    }
}

// Phase B of step t and, with UPD, the neuron update of step t + 1.  A binned
// step takes the tiles in turn (tile b, b + grid, ...); otherwise the update
// alone runs four blocks per workgroup pass.
template <bool CODE8, bool UPD>
__global__ __launch_bounds__(kTileThreads) void k_tile(StepArgs a, uint32_t k)
{
    extern __shared__ int32_t acc[];      // [D][1024]
    const uint32_t t = a.ctrl->t0 + k;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->hist_n += a.ctrl->nspk;   // step t's history is complete
    if (blockIdx.x == 0 && threadIdx.x < a.nsuper)
        a.dfill[(size_t)threadIdx.x * kFillStride] = 0u;   // two levels: the second pass has consumed the lists
    if (step_binned(a, t)) {
        for (uint32_t tt = blockIdx.x; tt < a.ntiles; tt += gridDim.x) {
            tile_work<CODE8, UPD, false>(a, tt, t, true, true, acc);
            __syncthreads();   // the LDS rows are reloaded for the next tile
        }
    } else if (UPD) {
        update_groups(a, t + 1u, reinterpret_cast<uint32_t*>(acc));
    }
}

// ---------------------------------------------------------------------------
// Batched stepping of many independent networks ("jobs") per launch.  A
// device job table holds each job's step arguments; the update kernel's
// blocks are spread over the jobs (job j owns blocks [blk_base, blk_base +
// nblk)), spikers are appended to their job's spike list (order within a step
// is free: delivery is order-independent and the history is sorted when read),
// and the delivery kernel walks the concatenated work items of all jobs.  Jobs
// stop at their own duration.  The kernels read everything from the table, so
// captured step graphs stay valid while jobs come and go.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int job_of_block(const JobDesc* jobs, uint32_t b)
{
    const uint32_t lane = threadIdx.x & 63u;
    const JobDesc& J = jobs[lane];
    const bool mine = J.active && b >= J.blk_base && b < J.blk_base + J.a.nblk;
    const uint64_t m = __ballot(mine);
    return m ? (int)__builtin_ctzll(m) : -1;
}

__global__ __launch_bounds__(256) void k_batch_update(const JobDesc* __restrict__ jobs, uint32_t k)
{
    __shared__ uint32_t pois_s[kMaxPois];
    __shared__ uint32_t wtot[4], sbase;
    __shared__ unsigned long long wext[4], wev[4];
    const uint32_t tid = threadIdx.x;
    const int j = job_of_block(jobs, blockIdx.x);
    if (j < 0) return;
    const StepArgs& a = jobs[j].a;
    const uint32_t t = a.ctrl->t0 + k;
    if (t >= jobs[j].t_end) return;
    const uint32_t blk = blockIdx.x - jobs[j].blk_base;
    if (tid < a.npois) pois_s[tid] = a.poisc[tid];
    __syncthreads();
    const uint32_t q = blk * 256u + tid;
    uint32_t flags = 0, ext_tot = 0, dis = 0;
    if (q < a.nq) {
        int4* rp = reinterpret_cast<int4*>(a.ring + (size_t)(t & (kRing - 1u)) * a.N) + q;
        const int4 in = *rp;
        st_nt(rp, make_int4(0, 0, 0, 0));
        flags = update_quad(a, pois_s, q, t, in, ext_tot, dis);
    }
    block_append<4>(a, t, q, flags, ext_tot, threadIdx.x, true, wtot, wext, wev, &sbase);
}

// Batched phase A: the concatenated row segments of all jobs are cut into
// chunks; a chunk bins the events of its binned jobs into a window of tiles
// (the chunk's jobs' tiles side by side, at most kMaxTiles), segments of jobs
// delivered directly this step go out as atomics.  Also closes the previous
// step's bookkeeping of each job (history count, cleared parity counters).
__global__ __launch_bounds__(kScatterThreads) void k_bscatter(const JobDesc* __restrict__ jobs, uint32_t k)
{
    __shared__ uint32_t stage[kStage];
    __shared__ uint32_t tcnt[kMaxTiles];
    __shared__ uint32_t toff[kMaxTiles];
    __shared__ uint32_t tres[kMaxTiles];
    __shared__ uint32_t ibase[kMaxJobs + 1];
    __shared__ uint32_t wbase[kMaxJobs + 1];
    __shared__ uint32_t jbin[kMaxJobs];
    __shared__ uint8_t segjob[kChunkItems];   // job of each row segment of the chunk
    __shared__ uint8_t tjob[kMaxTiles];       // job of each window tile
    __shared__ uint32_t wsum[kScatterWaves];
    __shared__ uint32_t wtotal;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    if (wv == 0) {
        const JobDesc& J = jobs[lane];
        uint32_t items = 0, bin = 0;
        if (J.active) {
            Ctrl* c = J.a.ctrl;
            const uint32_t t = c->t0 + k;
            if (t < J.t_end) {
                items = c->nspk_par[t & 1u] * J.smax;
                bin = (J.binned && c->step_ev[t & 1u] >= J.a.bin_threshold) ? 1u : 0u;
                if (blockIdx.x == 0) {
                    c->hist_n += c->nspk_par[t & 1u];
                    c->nspk_par[(t + 1u) & 1u] = 0u;
                    c->step_ev[(t + 1u) & 1u] = 0u;
                }
            }
        }
        const uint32_t v = wave_incl_scan<uint32_t>(items, lane);
        ibase[lane + 1u] = v;
        if (lane == 0) ibase[0] = 0;
        jbin[lane] = bin;
    }
    __syncthreads();
    const uint32_t total = ibase[kMaxJobs];
    uint32_t per = (total + gridDim.x - 1u) / gridDim.x;
    per = per < kScatterWaves ? kScatterWaves : (per > kChunkItems ? kChunkItems : per);
    auto job_of_item = [&](uint32_t it) {
        uint32_t lo = 0, hi = kMaxJobs;   // ibase[lo] <= it < ibase[hi]
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ibase[mid] <= it) lo = mid;
            else hi = mid;
        }
        return (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);   // callers pass wave-uniform items
    };
    for (uint32_t c0 = blockIdx.x * per; c0 < total; c0 += gridDim.x * per) {
        const uint32_t c1 = (total - c0) < per ? total : c0 + per;
        const uint32_t jl = job_of_item(c0), jh = job_of_item(c1 - 1u);
        if (tid == 0) {
            uint32_t w = 0;
            for (uint32_t j = jl; j <= jh; ++j) {
                wbase[j] = w;
                if (jbin[j]) w += jobs[j].a.ntiles;
            }
            wbase[jh + 1u] = w;
            wtotal = w;
        }
        __syncthreads();
        const uint32_t W = wtotal;
        const bool windowed = W <= kMaxTiles;
        for (uint32_t i = tid; i < (windowed ? W : 0u); i += kScatterThreads) tcnt[i] = 0;
        // segments delivered directly go out first, so that no binned segment
        // is held in registers meanwhile: those of jobs not binned this step,
        // and every segment of a chunk whose tile window is too wide
        for (uint32_t jj = 0; jj < kSegPerWave; ++jj) {
            const uint32_t it = c0 + wv + kScatterWaves * jj;
            const uint32_t j = it < c1 ? job_of_item(it) : 0u;
            if (lane == 0) segjob[wv + kScatterWaves * jj] = (uint8_t)j;
            if (it >= c1 || (windowed && jbin[j])) continue;
            const StepArgs& a = jobs[j].a;
            const uint32_t smax = jobs[j].smax;
            const uint32_t local = it - ibase[j];
            const uint4 info = a.spk[local / smax];
            const uint32_t t = a.ctrl->t0 + k;
            if (a.record == 1u) deliver_item<4, true>(a, t, info, local % smax, lane, a.cb);
            else deliver_item<4, false>(a, t, info, local % smax, lane, a.cb);
        }
        if (!windowed) {
            __syncthreads();
            continue;
        }
        SegLoad S[kSegPerWave];
#pragma unroll
        for (uint32_t jj = 0; jj < kSegPerWave; ++jj) {
            const uint32_t it = c0 + wv + kScatterWaves * jj;
            S[jj].s0 = 1u;
            S[jj].len = 0u;
            const uint32_t j = it < c1 ? job_of_item(it) : 0u;
            if (it < c1 && jbin[j]) {
                const StepArgs& a = jobs[j].a;
                const uint32_t local = it - ibase[j];
                seg_load<false>(a, a.spk[local / jobs[j].smax], local % jobs[j].smax, lane, S[jj]);
                seg_decode<false>(a, S[jj]);
            }
        }
        __syncthreads();
        // 1. histogram of targets by window tile
#pragma unroll
        for (uint32_t jj = 0; jj < kSegPerWave; ++jj) {
            if (S[jj].s0 >= S[jj].len) continue;
            const uint32_t wb = wbase[segjob[wv + kScatterWaves * jj]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (S[jj].s0 + 64u * u + lane < S[jj].len) atomicAdd(&tcnt[wb + (S[jj].tg[u] >> kTileBits)], 1u);
        }
        __syncthreads();
        // 2. scan and reservation in each window tile's bin
        uint32_t res0 = 0, res1 = 0;
        {
            const uint32_t t0i = 2u * tid, t1i = 2u * tid + 1u;
            const uint32_t v0 = t0i < W ? tcnt[t0i] : 0u;
            const uint32_t v1 = t1i < W ? tcnt[t1i] : 0u;
            const uint32_t sum = v0 + v1;
            const uint32_t inc = wave_incl_scan<uint32_t>(sum, lane);
            if (lane == 63u) wsum[wv] = inc;
            __syncthreads();
            uint32_t off = inc - sum;
            for (uint32_t i = 0; i < wv; ++i) off += wsum[i];
            for (uint32_t e = 0; e < 2u; ++e) {
                const uint32_t w = 2u * tid + e;
                if (w >= W) break;
                const uint32_t v = e ? v1 : v0;
                toff[w] = off;
                tcnt[w] = off;
                uint32_t lo = jl, hi = jh + 1u;   // wbase[lo] <= w < wbase[hi]
                while (hi - lo > 1u) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (wbase[mid] <= w) lo = mid;
                    else hi = mid;
                }
                tjob[w] = (uint8_t)lo;
                // the reservation's result is first needed in phase 4: it
                // stays in a register while phase 3 stages
                if (v) (e ? res1 : res0) = atomicAdd(&jobs[lo].a.bin_fill[(size_t)(w - wbase[lo]) * kFillStride], v);
                off += v;
            }
        }
        __syncthreads();
        // 3. encode and stage sorted by window tile
#pragma unroll
        for (uint32_t jj = 0; jj < kSegPerWave; ++jj) {
            if (S[jj].s0 >= S[jj].len) continue;
            const uint32_t wb = wbase[segjob[wv + kScatterWaves * jj]];
            const SegLoad& L = S[jj];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t c = L.s0 + 64u * u;
                if (c >= L.len) break;
                const uint32_t kk = c + lane;
                if (kk < L.len) {
                    // 8-byte records: the bucket above the weight field (seg_decode)
                    const uint32_t bl = L.wf[u] >> 17, wf = L.wf[u] & 0x1FFFFu;
                    const uint32_t p = atomicAdd(&tcnt[wb + (L.tg[u] >> kTileBits)], 1u);
                    stage[p] = (L.tg[u] & (kTile - 1u)) | (bl << kTileBits) | (wf << 15);
                }
            }
        }
        if (2u * tid < W) tres[2u * tid] = res0;
        if (2u * tid + 1u < W) tres[2u * tid + 1u] = res1;
        __syncthreads();
        // 4. runs into the bins: each group of kRunLanes lanes writes one
        // window tile's run at a time (the tile's job differs between groups)
        const uint32_t rl = tid % kRunLanes;
        for (uint32_t w = tid / kRunLanes; w < W; w += kScatterThreads / kRunLanes) {
            const uint32_t o0 = toff[w];
            const uint32_t cnt = tcnt[w] - o0;
            if (cnt == 0) continue;
            const uint32_t lo = tjob[w];
            const StepArgs& a = jobs[lo].a;
            const uint32_t tt = w - wbase[lo];
            const uint32_t r0 = tres[w];
            const uint32_t cap = a.bin_cap_tile;
            uint32_t* dst = a.bins + (size_t)tt * cap;
            for (uint32_t e = rl; e < cnt; e += kRunLanes) {
                const uint32_t code = stage[o0 + e];
                const uint32_t pos = r0 + e;
                if (pos < cap) {
                    dst[pos] = code;
                } else {
                    const uint32_t t = a.ctrl->t0 + k;
                    const uint32_t tgt = (tt << kTileBits) | (code & (kTile - 1u));
                    const uint32_t b = (code >> kTileBits) & 31u;
                    const uint32_t slot = (t + a.d_min + b) & (kRing - 1u);
                    __hip_atomic_fetch_add(a.ring + (size_t)slot * a.N + tgt,
                                           decode_weight(code >> 15, false, nullptr, a.winh_q), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    atomicAdd((unsigned long long*)&a.ctrl->bin_overflow, 1ull);
                }
            }
        }
        __syncthreads();
    }
}

// Batched phase B (+ fused update of the next step) over the batch's blocks
// [0, nb_total) (block b belongs to the job whose block range holds it), with
// as many workgroups as are resident at once.  First the tiles of the jobs
// binned this step, one per workgroup pass (accumulation, write-back and the
// next step's update); then the next step's update of every other running
// job, four blocks per pass (one per group of four waves, no LDS rows needed).
template <bool UPD>
__global__ __launch_bounds__(kTileThreads) void k_btile(const JobDesc* __restrict__ jobs, uint32_t k,
                                                         uint32_t nb_total)
{
    extern __shared__ int32_t acc[];
    auto binned_now = [&](const JobDesc& J, uint32_t t) {
        return J.binned && J.a.ctrl->step_ev[t & 1u] >= J.a.bin_threshold;
    };
    for (uint32_t b = blockIdx.x; b < nb_total; b += gridDim.x) {
        const int j = job_of_block(jobs, b);
        if (j < 0) continue;
        const JobDesc& J = jobs[j];
        const uint32_t t = J.a.ctrl->t0 + k;
        if (t >= J.t_end || !binned_now(J, t)) continue;
        tile_work<false, UPD, true>(J.a, b - J.blk_base, t, true, t + 1u < J.t_end, acc);
        __syncthreads();   // the LDS rows are reloaded for the next tile
    }
    if (!UPD) return;
    uint32_t* scr = reinterpret_cast<uint32_t*>(acc);
    const uint32_t tid = threadIdx.x, g = tid >> 8, gtid = tid & 255u;
    uint32_t* pois = scr + 64u * g;          // the group's job's Poisson table
    uint32_t* gs = scr + 256u + 32u * g;     // wtot[4], sbase, wext[4] (u64), wev[4] (u64)
    for (uint32_t base = 4u * blockIdx.x; base < nb_total; base += 4u * gridDim.x) {
        const uint32_t b = base + g;
        const int j = b < nb_total ? job_of_block(jobs, b) : -1;
        bool live = false;
        uint32_t t = 0;
        if (j >= 0) {
            const JobDesc& J = jobs[j];
            t = J.a.ctrl->t0 + k;
            live = t + 1u < J.t_end && !binned_now(J, t);
        }
        const StepArgs& a = jobs[j >= 0 ? j : 0].a;   // read only when live
        if (live && gtid < a.npois) pois[gtid] = a.poisc[gtid];
        __syncthreads();
        uint32_t q = 0, flags = 0, ext_tot = 0, dis = 0;
        if (live) {
            q = (b - jobs[j].blk_base) * 256u + gtid;
            if (q < a.nq) {
                int4* rp = reinterpret_cast<int4*>(a.ring + (size_t)((t + 1u) & (kRing - 1u)) * a.N) + q;
                const int4 in = *rp;
                st_nt(rp, make_int4(0, 0, 0, 0));
                flags = update_quad(a, pois, q, t + 1u, in, ext_tot, dis);
            }
        }
        block_append<4>(a, t + 1u, q, flags, ext_tot, gtid, live, gs, reinterpret_cast<unsigned long long*>(gs + 8),
                        reinterpret_cast<unsigned long long*>(gs + 16), gs + 4);
        __syncthreads();   // scratch reused by the next pass
    }
}

__global__ void k_batch_advance(const JobDesc* __restrict__ jobs, uint32_t n)
{
    const uint32_t j = threadIdx.x;
    if (j < kMaxJobs && jobs[j].active) {
        Ctrl* c = jobs[j].a.ctrl;
        const uint32_t te = jobs[j].t_end;
        c->t0 = (c->t0 + n < te) ? c->t0 + n : te;
    }
}

__global__ void k_advance(Ctrl* c, uint32_t n)
{
    if (threadIdx.x == 0) c->t0 += n;
}

__global__ __launch_bounds__(256) void k_set_flags(uint8_t* flags, const uint32_t* ids, uint32_t n,
                                                   uint8_t v)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) flags[ids[i]] = v;
}

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* p, uint64_t n, uint8_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256u) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_init(const StepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(cdiv(a.nq, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_syn_gen(const BuildArgs& a, hipStream_t s)
{
    if (a.nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_syn_gen, dim3(cdiv(a.nrows, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_syn_out(const BuildArgs& a, hipStream_t s)
{
    if (a.nrows == 0) return hipSuccess;
    if (a.nsuper) hipLaunchKernelGGL(k_syn_out_seg, dim3(cdiv(a.nrows, 4)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_syn_out, dim3(cdiv(a.nrows, 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

uint32_t scan_tiles(uint32_t N) { return cdiv(N, 1024); }

hipError_t launch_scan_rows(const uint32_t* rowlen, uint64_t* row_ptr, uint64_t* tile_sums,
                            uint32_t N, hipStream_t s, bool clear)
{
    const uint32_t nt = scan_tiles(N);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(256), 0, s, rowlen, tile_sums, N);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(256), 0, s, tile_sums, nt);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(256), 0, s, rowlen, tile_sums, row_ptr, N,
                       clear ? const_cast<uint32_t*>(rowlen) : nullptr);
    return hipGetLastError();
}

static uint32_t g_cus = 256;   // compute units of the device (set by setup_kernels)

// Launch on stream s; with timing events, the launch packet itself stamps the
// kernel's start and end into them.
#define SNN_LAUNCH(ev, kern, grid, block, shm, s, ...)                                                    \
    do {                                                                                                 \
        if (ev) hipExtLaunchKernelGGL(kern, grid, block, shm, s, (ev)->start, (ev)->stop, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kern, grid, block, shm, s, __VA_ARGS__);                                  \
    } while (0)

hipError_t launch_update(const StepArgs& a, uint32_t k, hipStream_t s, const LaunchEv* ev)
{
    SNN_LAUNCH(ev, k_update, dim3(a.nblk), dim3(256), 0, s, a, k);
    return hipGetLastError();
}

hipError_t launch_compact(const StepArgs& a, uint32_t k, hipStream_t s, const LaunchEv* ev)
{
    SNN_LAUNCH(ev, k_compact, dim3(a.ngrp), dim3(kCompactThreads), 0, s, a, k);
    return hipGetLastError();
}

hipError_t launch_deliver(const StepArgs& a, uint32_t k, uint32_t waves, uint32_t unroll,
                          uint32_t max_len, hipStream_t s, const LaunchEv* ev)
{
    const uint32_t blocks = cdiv(waves < 4u ? 4u : waves, 4);
    const uint32_t seg = 64u * unroll;
    const uint32_t smax = max_len ? cdiv(max_len, seg) : 1u;
    const bool c8 = a.record == 1u;
#define SNN_DELIVER(U)                                                                          \
    if (c8) SNN_LAUNCH(ev, (k_deliver<U, true>), dim3(blocks), dim3(256), 0, s, a, k, smax); \
    else SNN_LAUNCH(ev, (k_deliver<U, false>), dim3(blocks), dim3(256), 0, s, a, k, smax)
    if (unroll == 1u) {
        SNN_DELIVER(1);
    } else if (unroll == 2u) {
        SNN_DELIVER(2);
    } else {
        SNN_DELIVER(4);
    }
#undef SNN_DELIVER
    return hipGetLastError();
}

hipError_t launch_scatter(const StepArgs& a, uint32_t k, uint32_t max_len, uint32_t blocks,
                          hipStream_t s, const LaunchEv* ev)
{
    const uint32_t smax = max_len ? cdiv(max_len, 256) : 1u;
    if (a.nsuper) SNN_LAUNCH(ev, k_seg_emit, dim3(blocks), dim3(kEmitThreads), 0, s, a, k);
    else if (a.record == 1u) SNN_LAUNCH(ev, (k_scatter<true>), dim3(blocks), dim3(kScatterThreads), 0, s, a, k, smax);
    else SNN_LAUNCH(ev, (k_scatter<false>), dim3(blocks), dim3(kScatterThreads), 0, s, a, k, smax);
    return hipGetLastError();
}

hipError_t launch_sub(const StepArgs& a, uint32_t k, uint32_t blocks, hipStream_t s, const LaunchEv* ev)
{
    SNN_LAUNCH(ev, k_seg_bin, dim3(blocks), dim3(kScatterThreads), 0, s, a, k);
    return hipGetLastError();
}

static hipError_t setup_kernels_once()
{
    int dev = 0, cus = 0;
    hipError_t ce = hipGetDevice(&dev);
    if (ce == hipSuccess) ce = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (ce != hipSuccess) return ce;
    if (cus > 0) g_cus = (uint32_t)cus;
    // phase B keeps D rows of 1024 int32 in LDS (up to 124 KB of the 160 KB per CU)
    const int lds = (int)(kMaxD * kTile * sizeof(int32_t));
    const void* fns[6] = {(const void*)k_tile<true, false>, (const void*)k_tile<false, false>,
                          (const void*)k_tile<true, true>, (const void*)k_tile<false, true>,
                          (const void*)k_btile<true>, (const void*)k_btile<false>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Once per process (several construction threads may ask at the same time).
hipError_t setup_kernels()
{
    static std::once_flag once;
    static hipError_t result = hipSuccess;
    std::call_once(once, [] { result = setup_kernels_once(); });
    return result;
}

hipError_t launch_tile(const StepArgs& a, uint32_t k, bool update_next, hipStream_t s, const LaunchEv* ev)
{
    const size_t lds = (size_t)a.D * kTile * sizeof(int32_t);
    // as many workgroups as are resident at once: two per CU (1024 threads and
    // up to 124 KB of LDS each)
    const uint32_t grid = a.ntiles < 2u * g_cus ? a.ntiles : 2u * g_cus;
    const dim3 g(grid), b(kTileThreads);
    if (a.record == 1u) {
        if (update_next) SNN_LAUNCH(ev, (k_tile<true, true>), g, b, lds, s, a, k);
        else SNN_LAUNCH(ev, (k_tile<true, false>), g, b, lds, s, a, k);
    } else {
        if (update_next) SNN_LAUNCH(ev, (k_tile<false, true>), g, b, lds, s, a, k);
        else SNN_LAUNCH(ev, (k_tile<false, false>), g, b, lds, s, a, k);
    }
    return hipGetLastError();
}

hipError_t launch_batch_update(const JobDesc* jobs, uint32_t blocks, uint32_t k, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_update, dim3(blocks), dim3(256), 0, s, jobs, k);
    return hipGetLastError();
}

hipError_t launch_batch_scatter(const JobDesc* jobs, uint32_t blocks, uint32_t k, hipStream_t s)
{
    hipLaunchKernelGGL(k_bscatter, dim3(blocks), dim3(kScatterThreads), 0, s, jobs, k);
    return hipGetLastError();
}

hipError_t launch_batch_tile(const JobDesc* jobs, uint32_t blocks, uint32_t k, bool update_next, hipStream_t s)
{
    const size_t lds = (size_t)kBatchMaxD * kTile * sizeof(int32_t);
    const uint32_t grid = blocks < 2u * g_cus ? blocks : 2u * g_cus;   // resident workgroups
    if (update_next) hipLaunchKernelGGL((k_btile<true>), dim3(grid), dim3(kTileThreads), lds, s, jobs, k, blocks);
    else hipLaunchKernelGGL((k_btile<false>), dim3(grid), dim3(kTileThreads), lds, s, jobs, k, blocks);
    return hipGetLastError();
}

hipError_t launch_batch_advance(const JobDesc* jobs, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, jobs, n);
    return hipGetLastError();
}

hipError_t launch_advance(Ctrl* c, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, c, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u8, dim3((uint32_t)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_flags(uint8_t* flags, const uint32_t* ids, uint32_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_flags, dim3(cdiv(n, 256)), dim3(256), 0, s, flags, ids, n, v);
    return hipGetLastError();
}

}  // namespace snn
