// api.cpp -- C ABI of the gfx950 spiking-network library (include/snn.h):
// device memory, construction, step orchestration (HIP graphs of step
// sequences), read-back and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "snn.h"
#include "exact_dev.h"
#include "snn_dev.h"
#include "stdp_dev.h"
#include "tables.h"

using snn::Ctrl;
using snn::StepArgs;

// A device allocator: the caller's pair installed by snn_set_allocator, or
// hipMalloc / hipFree when none is.  Networks and batches take a copy when
// they are created and release every buffer through that copy.
struct DevAllocator {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free_)(void*, void*) = nullptr;
    void* ctx = nullptr;
};

struct snn_net {
    snn_grid_desc g{};
    snn_syn_desc s{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool built = false;
    bool poisoned = false;
    std::string err;
    StepArgs a{};
    DevAllocator dev_alloc;
    std::vector<std::pair<void*, size_t>> allocs;
    uint64_t bytes = 0;
    uint32_t N = 0, M = 0, D = 0;
    uint64_t nnz = 0;
    uint32_t max_len = 0;
    double build_ms = 0.0;
    uint32_t* T = nullptr;
    int32_t* wtab = nullptr;
    uint8_t* forced = nullptr;
    uint32_t* forced_ids = nullptr;
    // options
    uint32_t graph_chunk = 64;
    uint32_t deliver_waves = 8192;
    uint32_t unroll = 4;
    uint32_t mode = 0;          // 0 direct atomics, 1 tile-binned, 2 two-level tile-binned
    int mode_pref = -1;         // set before the build: -1 automatic, 0 direct only, 1 / 2 levels
    bool binned_ok = false;     // single-level binning possible
    bool two_level_ok = false;  // two-level binning possible (bins allocated only when selected)
    uint32_t scatter_blocks = 256;
    double bin_frac = 0.5;      // bin capacity as a fraction of the tile's in-synapses
    bool bin_threshold_set = false;
    uint64_t bin_threshold_opt = 0;
    uint64_t bin_threshold_auto = 0;   // the build's default (0.039 D N events)
    std::map<uint32_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    // exact-time solver (SNN_SOLVER_EXACT)
    bool exact = false;
    snn::XArgs x{};
    uint32_t xt = 0;                  // steps taken
    uint64_t qcap_opt = 0;            // SNN_OPT_QUEUE_CAP, set before the build (0: automatic)
    uint8_t* xforced = nullptr;       // lock-step flags and offsets
    uint32_t* xforced_f = nullptr;
    hipGraph_t xgraph = nullptr;      // R captured steps from a step t with t mod R = 0
    hipGraphExec_t xgraph_ex = nullptr;
    // spike-timing plasticity (s.stdp)
    bool stdp = false;
    snn::StdpArgs sa{};
    uint64_t* stdp_tsum = nullptr;    // scan scratch of the long-term application
    uint64_t stdp_t = 0;              // steps taken (the period's position)
};

namespace {

thread_local std::string g_create_err;

snn_status fail(snn_net* n, snn_status st, const std::string& msg)
{
    if (n) n->err = msg;
    else g_create_err = msg;
    return st;
}

snn_status fail_hip(snn_net* n, hipError_t e, const char* what)
{
    std::string m = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    if (n) n->poisoned = true;
    return fail(n, SNN_E_HIP, m);
}

#define HIPCHK(net, x)                                      \
    do {                                                    \
        hipError_t e_ = (x);                                \
        if (e_ != hipSuccess) return fail_hip(net, e_, #x); \
    } while (0)

std::mutex g_alloc_mu;
DevAllocator g_alloc;   // the allocator new networks and batches take

DevAllocator current_allocator()
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

// Every buffer is used with 16-byte vector accesses and the staging layouts
// assume 256-byte alignment, which hipMalloc gives; a caller's allocator must
// give it too.
constexpr uintptr_t kDevAlign = 256;

hipError_t dev_malloc(const DevAllocator& al, void** p, size_t b)
{
    if (!al.alloc) return hipMalloc(p, b);
    void* q = al.alloc(b, al.ctx);
    if (!q) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(q) % kDevAlign) {
        al.free_(q, al.ctx);
        return hipErrorInvalidValue;
    }
    *p = q;
    return hipSuccess;
}

void dev_free(const DevAllocator& al, void* p)
{
    if (!p) return;
    if (al.free_) al.free_(p, al.ctx);
    else (void)hipFree(p);
}

template <typename T>
hipError_t dalloc(snn_net* n, T** p, size_t count)
{
    void* q = nullptr;
    const size_t b = count * sizeof(T) > 0 ? count * sizeof(T) : 16;
    hipError_t e = dev_malloc(n->dev_alloc, &q, b);
    if (e != hipSuccess) return e;
    n->allocs.push_back(std::make_pair(q, b));
    n->bytes += b;
    *p = (T*)q;
    return hipSuccess;
}

void dfree(snn_net* n, void* p)
{
    if (!p) return;
    for (size_t i = 0; i < n->allocs.size(); ++i) {
        if (n->allocs[i].first == p) {
            n->bytes -= n->allocs[i].second;
            n->allocs.erase(n->allocs.begin() + (long)i);
            break;
        }
    }
    dev_free(n->dev_alloc, p);
}

void drop_graphs(snn_net* n)
{
    for (auto& kv : n->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    n->graphs.clear();
    if (n->xgraph_ex) (void)hipGraphExecDestroy(n->xgraph_ex);
    if (n->xgraph) (void)hipGraphDestroy(n->xgraph);
    n->xgraph_ex = nullptr;
    n->xgraph = nullptr;
}

snn_status check_usable(snn_net* n)
{
    if (!n) return fail(nullptr, SNN_E_INVAL, "null network handle");
    if (n->poisoned) return SNN_E_HIP;
    return SNN_OK;
}

// Kernel sequence of a network: one whose rows are laid out by super tile
// always steps through the two-level kernels (its direct delivery, mode 0, is
// their direct branch at every step); otherwise the selected mode's.
uint32_t seq(const snn_net* n) { return n->a.nsuper ? 2u : n->mode; }

// Binning threshold in force: mode 0 of a two-level network delivers every
// step directly.
uint64_t threshold_in_force(const snn_net* n)
{
    if (n->a.nsuper && n->mode == 0) return ~0ull;
    return n->bin_threshold_set ? n->bin_threshold_opt : n->bin_threshold_auto;
}

// Enqueue step k (0-based within the current chunk) of the plain path.
// Binned delivery of step k (tile kernel without the next step's update).
hipError_t enqueue_binned(snn_net* n, const StepArgs& a, uint32_t k, bool update_next)
{
    hipError_t e = snn::launch_scatter(a, k, n->max_len, n->scatter_blocks, n->stream);
    if (e == hipSuccess && seq(n) == 2) e = snn::launch_sub(a, k, n->scatter_blocks, n->stream);
    if (e == hipSuccess) e = snn::launch_tile(a, k, update_next, n->stream);
    return e;
}

hipError_t enqueue_deliver(snn_net* n, const StepArgs& a, uint32_t k)
{
    if (seq(n) != 0) return enqueue_binned(n, a, k, false);
    return snn::launch_deliver(a, k, n->deliver_waves, n->unroll, n->max_len, n->stream);
}

hipError_t check_items(snn_net* n)
{
    const uint64_t seg = 64ull * (seq(n) != 0 ? 4 : n->unroll);
    const uint64_t smax = n->max_len ? (n->max_len + seg - 1) / seg : 1;
    return ((uint64_t)n->N * smax >= (1ull << 32)) ? hipErrorInvalidValue : hipSuccess;
}

// Enqueue step k (0-based within the current chunk) of the plain path.
hipError_t enqueue_step(snn_net* n, const StepArgs& a, uint32_t k)
{
    hipError_t e = check_items(n);
    if (e != hipSuccess) return e;
    e = snn::launch_update(a, k, n->stream);
    if (e != hipSuccess) return e;
    if (seq(n) != 1) {   // single-level binned delivery compacts inside its scatter kernel
        e = snn::launch_compact(a, k, n->stream);
        if (e != hipSuccess) return e;
    }
    return enqueue_deliver(n, a, k);
}

// Enqueue steps k0 .. k0+count-1.  With binned delivery the neuron update of
// step k+1 runs inside step k's tile kernel, so only the first update is a
// launch of its own; the last tile kernel does not update, leaving the state
// at the end of the last step.  Single level: the spike compaction runs inside
// the scatter kernel, so a step is two launches; two levels: compaction,
// scatter, second pass, tiles.
hipError_t enqueue_steps(snn_net* n, uint32_t k0, uint32_t count)
{
    if (count == 0) return hipSuccess;
    if (seq(n) == 0 || n->a.d_min != 1) {
        for (uint32_t k = k0; k < k0 + count; ++k) {
            hipError_t e = enqueue_step(n, n->a, k);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = check_items(n);
    if (e == hipSuccess) e = snn::launch_update(n->a, k0, n->stream);
    for (uint32_t k = k0; k < k0 + count && e == hipSuccess; ++k) {
        if (seq(n) == 2) e = snn::launch_compact(n->a, k, n->stream);
        if (e == hipSuccess) e = enqueue_binned(n, n->a, k, k + 1 < k0 + count);
    }
    return e;
}

hipError_t get_graph(snn_net* n, uint32_t chunk, hipGraphExec_t* out)
{
    auto it = n->graphs.find(chunk);
    if (it != n->graphs.end()) {
        *out = it->second.second;
        return hipSuccess;
    }
    hipGraph_t gr = nullptr;
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipStreamBeginCapture(n->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_steps(n, 0, chunk);
    if (le == hipSuccess) le = snn::launch_advance(n->a.ctrl, chunk, n->stream);
    e = hipStreamEndCapture(n->stream, &gr);
    if (le != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return e;
    }
    n->graphs[chunk] = std::make_pair(gr, ex);
    *out = ex;
    return hipSuccess;
}

snn::TableParams table_params(const snn_grid_desc& g, const snn_syn_desc& s)
{
    snn::TableParams tp{};
    tp.gx = g.gx;
    tp.gy = g.gy;
    tp.M = g.n_exc + g.n_inh;
    tp.kernel = s.kernel;
    tp.range = s.range;
    tp.k_in = s.k_in;
    tp.n_exc = g.n_exc;
    tp.preset = s.preset;
    tp.p_local = s.p_local;
    tp.amp = s.amp;
    tp.p_cut = s.p_cut;
    tp.gen = s.gen;
    tp.D = s.d_max >= s.d_min ? s.d_max - s.d_min + 1 : 0;
    tp.delay_exp = s.delay_dist;
    tp.delay_tau = s.delay_tau;
    tp.w_exc = s.w_exc;
    tp.w_exc_sd = s.w_exc_sd;
    tp.w_inh = s.w_inh;
    tp.ext_poisson = s.ext_mode == SNN_EXT_POISSON;
    tp.ext_n = s.ext_n;
    tp.ext_rate_hz = s.ext_rate_hz;
    tp.ext_w = s.ext_w;
    tp.tau_m = g.tau_m;
    tp.tau_w = g.tau_w;
    tp.t_ref = g.t_ref;
    tp.stdp = s.stdp;
    tp.a_plus = s.a_plus;
    tp.a_minus = s.a_minus;
    tp.tau_plus = s.tau_plus;
    tp.tau_minus = s.tau_minus;
    tp.w_max = s.w_max;
    return tp;
}

bool valid_grid(const snn_grid_desc* g, std::string& why)
{
    const uint64_t M = (uint64_t)g->n_exc + g->n_inh;
    if (g->gx == 0 || g->gy == 0 || M == 0) return why = "empty grid", false;
    if (M % 4 != 0) return why = "module size must be a multiple of 4", false;
    if (!g->periodic) return why = "only torus (periodic) grids are supported", false;
    const uint64_t N = (uint64_t)g->gx * g->gy * M;
    if (N * snn::kRing >= (1ull << 32)) return why = "too many neurons for a 32-slot int32 ring", false;
    if (!(g->tau_m > 0) || !(g->tau_w > 0) || !(g->t_ref >= 0)) return why = "bad time constants", false;
    if (g->t_ref > 250.0) return why = "refractory period too long", false;
    if (!(g->v_th > g->e_rest)) return why = "threshold must exceed the resting potential", false;
    return true;
}

}  // namespace

extern "C" {

const char* snn_last_error(const snn_net* net)
{
    return net ? net->err.c_str() : g_create_err.c_str();
}

snn_status snn_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx)
{
    if ((alloc == nullptr) != (free_ == nullptr))
        return fail(nullptr, SNN_E_INVAL, "snn_set_allocator: give both functions, or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free_ = free_;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return SNN_OK;
}

snn_status snn_build_grid(const snn_grid_desc* g, void* hip_stream, snn_net** out)
{
    if (!g || !out) return fail(nullptr, SNN_E_INVAL, "null argument");
    *out = nullptr;
    std::string why;
    if (!valid_grid(g, why)) return fail(nullptr, SNN_E_INVAL, why);
    snn_net* n = new snn_net();
    n->dev_alloc = current_allocator();
    n->g = *g;
    if (n->g.hist_cap == 0) n->g.hist_cap = 1ull << 24;
    n->M = g->n_exc + g->n_inh;
    n->N = g->gx * g->gy * n->M;
    if (hip_stream) {
        n->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete n;
            return fail_hip(nullptr, e, "hipStreamCreateWithFlags");
        }
        n->own_stream = true;
    }
    StepArgs& a = n->a;
    a.N = n->N;
    a.nq = n->N / 4;
    a.M = n->M;
    a.n_exc = g->n_exc;
    a.sfa_on_inh = g->sfa_on_inh;
    a.nblk = (n->N + snn::kNeuronsPerBlock - 1) / snn::kNeuronsPerBlock;
    a.ngrp = (a.nblk + snn::kGroup - 1) / snn::kGroup;
    a.key0 = (uint32_t)g->seed;
    a.key1 = (uint32_t)(g->seed >> 32);
    a.hist_cap = n->g.hist_cap;
    a.v_th = (float)g->v_th;
    a.v_reset = (float)g->v_reset;
    a.e_rest = (float)g->e_rest;
    a.alpha = (float)g->alpha_w;
    hipError_t e = hipSuccess;
#define ALLOC(p, cnt)                                       \
    if (e == hipSuccess) e = dalloc(n, &(p), (size_t)(cnt))
    ALLOC(a.V, n->N);
    ALLOC(a.W, n->N);
    ALLOC(a.ref, n->N);
    ALLOC(a.ring, (size_t)snn::kRing * n->N);
    ALLOC(a.blk_stat, a.nblk);
    ALLOC(a.blk_list, (size_t)a.nblk * snn::kNeuronsPerBlock);
    ALLOC(a.grp_cnt, 2 * a.ngrp);
    ALLOC(a.spk, n->N);
    ALLOC(a.hist, n->g.hist_cap);
    ALLOC(a.ctrl, 1);
    ALLOC(n->forced, n->N);
    ALLOC(n->forced_ids, n->N);
#undef ALLOC
    if (e != hipSuccess) {
        snn_destroy(n);
        return fail(nullptr, SNN_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    e = hipMemsetAsync(a.ring, 0, sizeof(int32_t) * (size_t)snn::kRing * n->N, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(a.grp_cnt, 0, sizeof(uint32_t) * 2 * a.ngrp, n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(a.ctrl, 0, sizeof(Ctrl), n->stream);
    if (e == hipSuccess) e = hipMemsetAsync(n->forced, 0, n->N, n->stream);
    if (e == hipSuccess) e = snn::launch_init(a, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        snn_status st = fail_hip(nullptr, e, "grid initialisation");
        snn_destroy(n);
        return st;
    }
    *out = n;
    return SNN_OK;
}

// Exact-time solver state (after the projections exist): refractory ends,
// spike offsets, the arrival slots' input lists and counts, scan scratch.
static snn_status setup_exact(snn_net* n, const snn::HostTables& tb)
{
    const StepArgs& a = n->a;
    snn::XArgs& x = n->x;
    const snn_grid_desc& g = n->g;
    x.N = n->N;
    x.M = n->M;
    x.n_exc = g.n_exc;
    x.sfa_on_inh = g.sfa_on_inh;
    x.D = n->D;
    x.d_min = n->s.d_min;
    x.R = n->s.d_max + 1;    // every arrival slot but the current one is ahead
    x.record = n->s.record;
    x.npois = a.npois;
    x.ext_const = a.ext_const;
    x.ext_const_q = a.ext_const_q;
    x.jext_q = a.jext_q;
    x.key0 = a.key0;
    x.key1 = a.key1;
    x.nblk = (n->N + snn::kXBlock - 1) / snn::kXBlock;
    x.smax = (n->max_len + 255u) / 256u;
    x.tau_equal = g.tau_w == g.tau_m;
    x.hist_cap = g.hist_cap;
    x.tref_q = (uint64_t)std::llround(g.t_ref * 4294967296.0);
    x.v_th = a.v_th;
    x.v_reset = a.v_reset;
    x.e_rest = a.e_rest;
    x.alpha = a.alpha;
    x.inv_tau_m = (float)(1.0 / g.tau_m);
    x.inv_tau_w = (float)(1.0 / g.tau_w);
    x.ck = x.tau_equal ? 0.0f : (float)(g.tau_w / (g.tau_w - g.tau_m));
    x.dinv_tau_m = 1.0 / g.tau_m;
    x.dinv_tau_w = 1.0 / g.tau_w;
    x.dck = x.tau_equal ? 0.0 : g.tau_w / (g.tau_w - g.tau_m);
    x.dv_th = g.v_th;
    x.dv_reset = g.v_reset;
    x.de_rest = g.e_rest;
    x.dalpha = g.alpha_w;
    // inputs queued per slot: a step's events at a 150 Hz mean rate, or the option
    const double qc = n->qcap_opt ? (double)n->qcap_opt : (double)n->N * (tb.mean_out + 1.0) * 0.15 + 65536.0;
    x.qcap = (uint64_t)std::min(qc, 4.0e9);
    // arrival sort: targets in at most kXGroups groups of 2^gbits >= 256 neurons
    x.gbits = 8;
    while (((uint64_t)n->N + (1ull << x.gbits) - 1) >> x.gbits > snn::kXGroups) ++x.gbits;
    if (x.gbits > snn::kXGroupBitsMax)
        return fail(n, SNN_E_INVAL, "the exact solver takes at most 2^24 neurons");
    x.ngroups = (uint32_t)(((uint64_t)n->N + (1ull << x.gbits) - 1) >> x.gbits);
    hipError_t e = hipSuccess;
#define XALLOC(p, cnt) \
    if (e == hipSuccess) e = dalloc(n, &(p), (size_t)(cnt))
    XALLOC(x.rend, n->N);
    XALLOC(x.fs, n->N);
    XALLOC(x.qlist, (size_t)x.R * x.qcap);
    XALLOC(x.qn, x.R);
    XALLOC(x.qn_prev, x.R);
    XALLOC(x.blk_ext, x.nblk);
    XALLOC(x.dropped, 1);
    XALLOC(x.qoff, (size_t)n->N + 1);
    XALLOC(x.qsorted, x.qcap);
    XALLOC(x.qtmp, x.qcap);
    XALLOC(x.gcnt, x.ngroups);
    XALLOC(x.goff, (size_t)x.ngroups + 1);
    XALLOC(x.gcur, x.ngroups);
    XALLOC(x.xpref, (size_t)n->N * x.D);
    XALLOC(x.blk_cnt, x.nblk);
    XALLOC(x.blk_list, (size_t)x.nblk * snn::kXBlock);
    XALLOC(x.blk_off, (size_t)x.nblk + 1);
    XALLOC(x.spk, n->N);
    XALLOC(x.hist_f, g.hist_cap);
    XALLOC(n->xforced, n->N);
    XALLOC(n->xforced_f, n->N);
#undef XALLOC
    if (e != hipSuccess) return fail(n, SNN_E_NOMEM, "device allocation failed (exact-solver queues)");
    HIPCHK(n, hipMemsetAsync(x.rend, 0, 8 * (size_t)n->N, n->stream));
    HIPCHK(n, hipMemsetAsync(x.gcnt, 0, 4 * (size_t)x.ngroups, n->stream));
    HIPCHK(n, hipMemsetAsync(x.qn, 0, 8 * (size_t)x.R, n->stream));
    HIPCHK(n, hipMemsetAsync(x.dropped, 0, 8, n->stream));
    HIPCHK(n, hipMemsetAsync(x.qoff, 0, 8, n->stream));      // offset of the first target
    HIPCHK(n, hipMemsetAsync(x.blk_off, 0, 8, n->stream));   // offset of the first workgroup
    HIPCHK(n, hipStreamSynchronize(n->stream));
    x.V = a.V;
    x.W = a.W;
    x.hist = a.hist;
    x.ctrl = a.ctrl;
    x.row_ptr = a.row_ptr;
    x.bend = a.bend;
    x.recs = a.recs;
    x.poisc = a.poisc;
    x.cb = a.cb;
    x.forced = nullptr;
    x.forced_f = nullptr;
    n->xt = 0;
    n->exact = true;
    return SNN_OK;
}

// One step of the exact solver on the network's stream (x: the network's
// arguments, possibly with lock-step flags); ev, if given: timing events of
// the place, update and deliver launches.
static hipError_t enqueue_exact_step(snn_net* n, const snn::XArgs& x, const snn::LaunchEv* ev)
{
    const uint32_t t = n->xt;
    hipError_t e = snn::launch_x_place(x, n->stream, ev ? &ev[0] : nullptr);
    if (e == hipSuccess) e = snn::launch_x_update(x, n->stream, ev ? &ev[1] : nullptr);
    if (e == hipSuccess) e = snn::launch_x_list(x, n->stream);
    if (e == hipSuccess) e = snn::launch_x_deliver(x, n->stream, ev ? &ev[2] : nullptr);
    if (e == hipSuccess) e = snn::launch_x_finish(x, n->stream);
    if (e == hipSuccess) n->xt = t + 1;
    return e;
}

// Exact solver, n_ms steps: whenever the step index is a multiple of R and R
// steps are left, the R steps are replayed from a captured graph (the kernels
// read the step from the device, so one capture serves every such sequence);
// other steps are launched one by one.
static hipError_t step_exact(snn_net* n, uint32_t n_ms)
{
    const uint32_t R = n->x.R;
    uint32_t left = n_ms;
    while (left) {
        if (n->xt % R == 0 && left >= R) {
            if (!n->xgraph_ex) {
                const uint32_t xt0 = n->xt;
                hipError_t e = hipStreamBeginCapture(n->stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return e;
                hipError_t le = hipSuccess;
                for (uint32_t i = 0; i < R && le == hipSuccess; ++i) le = enqueue_exact_step(n, n->x, nullptr);
                n->xt = xt0;
                e = hipStreamEndCapture(n->stream, &n->xgraph);
                if (le == hipSuccess) le = e;
                if (le == hipSuccess) le = hipGraphInstantiate(&n->xgraph_ex, n->xgraph, nullptr, nullptr, 0);
                if (le != hipSuccess) {
                    drop_graphs(n);
                    return le;
                }
            }
            hipError_t e = hipGraphLaunch(n->xgraph_ex, n->stream);
            if (e != hipSuccess) return e;
            n->xt += R;
            left -= R;
        } else {
            hipError_t e = enqueue_exact_step(n, n->x, nullptr);
            if (e != hipSuccess) return e;
            --left;
        }
    }
    return hipSuccess;
}

// Inputs dropped because an arrival slot's list was full (exact solver).
// Buffers of the long-term plasticity application: per-neuron counters,
// list offsets, the window's spike steps (at most one spike per refractory
// period and neuron, and never more than the history holds), the rows to
// visit, and the lag tables.
static snn_status setup_stdp(snn_net* n, const snn::HostTables& tb)
{
    snn::StdpArgs& sa = n->sa;
    const StepArgs& a = n->a;
    sa.N = n->N;
    sa.M = n->M;
    sa.n_exc = n->g.n_exc;
    sa.D = n->D;
    sa.d_min = n->s.d_min;
    sa.win = tb.stdp_win;
    sa.wmax_q = tb.wmax_q;
    sa.smax = n->max_len ? (n->max_len + 255u) / 256u : 1u;
    sa.hist = a.hist;
    sa.hist_cap = a.hist_cap;
    sa.ctrl = a.ctrl;
    sa.row_ptr = a.row_ptr;
    sa.bend = a.bend;
    sa.recs = reinterpret_cast<snn::Rec8*>(const_cast<void*>(a.recs));
    const uint64_t span = (uint64_t)n->s.ltp_period + tb.stdp_win + n->s.d_max;
    const uint64_t per = (span + tb.nref) / (tb.nref + 1u);   // spikes a neuron can have in the span
    sa.times_cap = std::max<uint64_t>(1, std::min<uint64_t>(a.hist_cap, (uint64_t)n->N * per));
    int32_t* kp = nullptr;
    int32_t* km = nullptr;
    hipError_t e = dalloc(n, &sa.range, 2);
    if (e == hipSuccess) e = dalloc(n, &sa.cnt, n->N);
    if (e == hipSuccess) e = dalloc(n, &sa.fill, n->N);
    if (e == hipSuccess) e = dalloc(n, &sa.off, (size_t)n->N + 1);
    if (e == hipSuccess) e = dalloc(n, &sa.times, sa.times_cap);
    if (e == hipSuccess) e = dalloc(n, &sa.act, n->N);
    if (e == hipSuccess) e = dalloc(n, &sa.nact, 1);
    if (e == hipSuccess) e = dalloc(n, &kp, tb.kp.size());
    if (e == hipSuccess) e = dalloc(n, &km, tb.km.size());
    if (e == hipSuccess) e = dalloc(n, &n->stdp_tsum, snn::scan_tiles(n->N) + 1);
    if (e != hipSuccess) return fail(n, SNN_E_NOMEM, "device allocation failed (plasticity)");
    HIPCHK(n, hipMemcpyAsync(kp, tb.kp.data(), tb.kp.size() * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipMemcpyAsync(km, tb.km.data(), tb.km.size() * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    sa.kp = kp;
    sa.km = km;
    n->stdp = true;
    n->stdp_t = 0;
    return SNN_OK;
}

// The long-term application that ends the period just stepped.
static hipError_t enqueue_ltp(snn_net* n)
{
    snn::StdpArgs sa = n->sa;
    const uint64_t P = n->s.ltp_period;
    sa.T1 = (uint32_t)n->stdp_t;
    sa.T0 = (uint32_t)(n->stdp_t - P);
    const uint64_t back = (uint64_t)sa.win + n->s.d_max;
    sa.W0 = (uint64_t)sa.T0 + 1 >= back ? (uint32_t)(sa.T0 + 1 - back) : 0u;
    return snn::launch_stdp_period(sa, n->stdp_tsum, n->stream);
}

// Book `count` steps just enqueued on a plastic network (never past the end
// of a period) and apply the period when they end it.
static hipError_t stdp_after(snn_net* n, uint32_t count)
{
    if (!n->stdp) return hipSuccess;
    n->stdp_t += count;
    return n->stdp_t % n->s.ltp_period == 0 ? enqueue_ltp(n) : hipSuccess;
}

static snn_status check_dropped(snn_net* n)
{
    if (n->stdp) {
        Ctrl hc{};
        HIPCHK(n, hipMemcpy(&hc, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err & 8u)
            return fail(n, SNN_E_OVERFLOW, "plasticity: the spike history overflowed its capacity, so pairs were "
                                           "missed (raise hist_cap)");
    }
    if (!n->exact) return SNN_OK;
    unsigned long long d = 0;
    HIPCHK(n, hipMemcpy(&d, n->x.dropped, 8, hipMemcpyDeviceToHost));
    if (d) return fail(n, SNN_E_OVERFLOW, "exact solver: " + std::to_string(d) +
                                          " inputs found their arrival slot full (raise SNN_OPT_QUEUE_CAP)");
    return SNN_OK;
}

snn_status snn_build_synapses(snn_net* n, const snn_syn_desc* s)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!s) return fail(n, SNN_E_INVAL, "null synapse description");
    if (n->built) return fail(n, SNN_E_STATE, "synapses already built");
    if (s->kernel > 1u) return fail(n, SNN_E_INVAL, "unknown lateral kernel");
    if (s->record > 1u) return fail(n, SNN_E_INVAL, "unknown record format");
    if (s->ext_mode > 1u) return fail(n, SNN_E_INVAL, "unknown external drive mode");
    if (s->preset > 1u) return fail(n, SNN_E_INVAL, "unknown connectivity preset");
    if (s->d_min < 1 || s->d_max < s->d_min || s->d_max > snn::kMaxD)
        return fail(n, SNN_E_INVAL, "delays must satisfy 1 <= d_min <= d_max <= 31");
    if (!(s->range > 0) || !(s->k_in >= 0)) return fail(n, SNN_E_INVAL, "bad range or in-degree");
    if (s->record == SNN_REC_CODE8 && n->N > (1u << 24))
        return fail(n, SNN_E_INVAL, "8-bit code records need fewer than 2^24 neurons");
    if (s->ext_mode == SNN_EXT_POISSON && !(s->ext_n * s->ext_rate_hz >= 0))
        return fail(n, SNN_E_INVAL, "bad external drive");
    if (s->solver > SNN_SOLVER_EXACT) return fail(n, SNN_E_INVAL, "unknown solver");
    if (s->solver == SNN_SOLVER_EXACT && !(n->g.t_ref >= 1.0 && n->g.t_ref < 1.0e6))
        return fail(n, SNN_E_INVAL, "the exact solver needs 1 <= t_ref < 1e6 ms");
    const auto t_start = std::chrono::steady_clock::now();
    snn::TableParams tp = table_params(n->g, *s);
    snn::HostTables tb;
    std::string why = snn::build_tables(tp, tb);
    if (!why.empty()) return fail(n, SNN_E_INVAL, why);
    if (s->stdp) {
        if (s->solver != SNN_SOLVER_STEP) return fail(n, SNN_E_INVAL, "plasticity runs under the step solver only");
        if (s->record != SNN_REC_F32) return fail(n, SNN_E_INVAL, "plasticity needs F32 records");
        if (s->ltp_period == 0) return fail(n, SNN_E_INVAL, "ltp_period must be at least one step");
        // a plastic weight must keep the binned delivery's 17-bit weight field
        if (!(s->w_max > 0.0) || tb.wmax_q > 65534)
            return fail(n, SNN_E_INVAL, "w_max must be in (0, 65534/65536] mV");
    }
    n->s = *s;
    n->D = s->d_max - s->d_min + 1;
    StepArgs& a = n->a;
    a.D = n->D;
    a.d_min = s->d_min;
    a.record = s->record;
    a.npois = (uint32_t)tb.poisc.size();
    a.ext_const = s->ext_mode == SNN_EXT_CONST;
    a.ext_const_q = s->ext_const_q;
    a.jext_q = tb.jext_q;
    a.dm = (float)tb.dm;
    a.dw = (float)tb.dw;
    a.kappa = (float)tb.kappa;
    a.nref = tb.nref;

    uint32_t* poisc = nullptr;
    int32_t* cb = nullptr;
    uint64_t* row_ptr = nullptr;
    uint16_t* bend = nullptr;
    uint32_t* rowlen = nullptr;
    uint64_t* tsum = nullptr;
    hipError_t e = dalloc(n, &n->T, tb.T.size());
    if (e == hipSuccess) e = dalloc(n, &n->wtab, 65536);
    if (e == hipSuccess) e = dalloc(n, &cb, 256);
    if (e == hipSuccess) e = dalloc(n, &poisc, snn::kMaxPois);
    if (e == hipSuccess) e = dalloc(n, &row_ptr, (size_t)n->N + 1);
    if (e == hipSuccess) e = dalloc(n, &bend, (size_t)n->N * n->D);
    if (e == hipSuccess) e = dalloc(n, &rowlen, n->N);
    if (e == hipSuccess) e = dalloc(n, &tsum, snn::scan_tiles(n->N) + 1);
    uint32_t* btab = nullptr;   // binomial generator tables (construction only)
    uint32_t* bthr = nullptr;
    if (e == hipSuccess && s->gen == SNN_GEN_BINOMIAL) {
        e = dalloc(n, &btab, tb.btab.size());
        if (e == hipSuccess) e = dalloc(n, &bthr, tb.bthr.size());
    }
    if (e != hipSuccess) return fail(n, SNN_E_NOMEM, "device allocation failed (tables/offsets)");
    if (btab) HIPCHK(n, hipMemcpyAsync(btab, tb.btab.data(), tb.btab.size() * 4, hipMemcpyHostToDevice, n->stream));
    if (bthr && !tb.bthr.empty())
        HIPCHK(n, hipMemcpyAsync(bthr, tb.bthr.data(), tb.bthr.size() * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipMemcpyAsync(n->T, tb.T.data(), tb.T.size() * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipMemcpyAsync(n->wtab, tb.wtab.data(), 65536 * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipMemcpyAsync(cb, tb.cb.data(), 256 * 4, hipMemcpyHostToDevice, n->stream));
    if (!tb.poisc.empty())
        HIPCHK(n, hipMemcpyAsync(poisc, tb.poisc.data(), tb.poisc.size() * 4, hipMemcpyHostToDevice, n->stream));
    a.poisc = poisc;
    a.cb = cb;
    a.row_ptr = row_ptr;
    a.bend = bend;

    snn::BuildArgs b{};
    b.gen = s->gen;
    b.delay_exp = s->delay_dist;
    for (size_t k = 0; k < tb.dthr.size() && k < snn::kMaxD; ++k) b.dthr[k] = tb.dthr[k];
    b.btab = reinterpret_cast<const uint4*>(btab);
    b.bthr = bthr;
    b.N = n->N;
    b.M = n->M;
    b.n_exc = n->g.n_exc;
    b.gx = n->g.gx;
    b.gy = n->g.gy;
    b.D = n->D;
    b.d_min = s->d_min;
    b.record = s->record;
    b.key0 = a.key0;
    b.key1 = a.key1;
    b.winh_q = tb.winh_q;
    b.T = n->T;
    b.wtab = n->wtab;
    b.bend = bend;
    b.rowlen = rowlen;
    b.row_ptr = row_ptr;
    b.ctrl = a.ctrl;
    // Delivery schedule, chosen before the rows are written (two levels lay
    // the rows out by super tile).  Single level: the tiles fit the scatter
    // kernel's LDS tables and every weight has a 17-bit event field (code, or
    // w_q + 65536 in range).  Two levels (8-bit codes): networks with more
    // tiles than one LDS table.
    a.ntiles = (n->N + snn::kTile - 1) / snn::kTile;
    a.winh_q = tb.winh_q;
    bool ok1 = a.ntiles <= snn::kMaxTiles;
    if (s->record != SNN_REC_CODE8)
        for (int32_t w : tb.wtab)
            if (w != tb.winh_q && (w < -65536 || w > 65534)) ok1 = false;
    const uint32_t nsuper = (uint32_t)(((uint64_t)n->N + (1u << snn::kSegBits) - 1) >> snn::kSegBits);
    const bool ok2 = s->record == SNN_REC_CODE8 && nsuper <= snn::kMaxSuper;
    uint32_t mode = 0;
    if (s->solver == SNN_SOLVER_EXACT) {
        ok1 = false;   // the exact solver has its own queues
    } else if (n->mode_pref == 2) mode = ok2 ? 2 : 0;
    else if (n->mode_pref == 1) mode = ok1 ? 1 : 0;
    else if (n->mode_pref < 0) mode = ok1 ? 1 : (ok2 ? 2 : 0);
    uint16_t* sstart = nullptr;
    if (mode == 2) {
        if (dalloc(n, &sstart, (size_t)n->N * nsuper) != hipSuccess)
            return fail(n, SNN_E_NOMEM, "device allocation failed (segment starts)");
        b.nsuper = nsuper;
        b.sstart = sstart;
    }
    // Rows are built in slices so that no single launch runs for long: the
    // slice's rows are generated into a buffer of slab_cap hits per row
    // (8 standard deviations above the busiest source type's expected row
    // length), their offsets scanned, and the records written out.  The
    // record buffer is sized to a bound on the total (expected total + 10
    // standard deviations).
    const uint32_t slice = 1u << 16;
    const double kmax = tb.max_out + 1.0, kin = tb.mean_out + 1.0;
    b.slab_cap = (uint32_t)std::min(kmax + 8.0 * std::sqrt(kmax) + 256.0, 65536.0);
    const double tot_bound = (double)n->N * kin + 10.0 * std::sqrt((double)n->N * kin) + 65536.0;
    const size_t rb = s->record == SNN_REC_CODE8 ? 4 : 8;
    b.rec_cap = (uint64_t)tot_bound;
    void* recs = nullptr;
    uint32_t* slab = nullptr;
    e = dalloc(n, (uint8_t**)&recs, (size_t)b.rec_cap * rb);
    if (e == hipSuccess) e = dalloc(n, &slab, (size_t)std::min(n->N, slice) * b.slab_cap);
    if (e != hipSuccess) return fail(n, SNN_E_NOMEM, "device allocation failed (synapse records)");
    b.recs = recs;
    b.slab = slab;
    HIPCHK(n, hipMemsetAsync(row_ptr, 0, 8, n->stream));   // offset of row 0
    for (uint32_t r0 = 0; r0 < n->N; r0 += slice) {
        b.row0 = r0;
        b.nrows = (n->N - r0) < slice ? (n->N - r0) : slice;
        HIPCHK(n, snn::launch_syn_gen(b, n->stream));
        HIPCHK(n, snn::launch_scan_rows(rowlen + r0, row_ptr + r0, tsum, b.nrows, n->stream));
        HIPCHK(n, snn::launch_syn_out(b, n->stream));
    }
    Ctrl hc{};
    HIPCHK(n, hipMemcpyAsync(&hc, a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, n->stream));
    uint64_t nnz = 0;
    HIPCHK(n, hipMemcpyAsync(&nnz, row_ptr + n->N, 8, hipMemcpyDeviceToHost, n->stream));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    dfree(n, slab);
    dfree(n, btab);
    dfree(n, bthr);
    if (hc.err & 1u) return fail(n, SNN_E_OVERFLOW, "a projection row exceeds 65535 synapses");
    if (hc.err & 2u) return fail(n, SNN_E_OVERFLOW, "a projection row exceeds the construction buffer");
    if (hc.err & 4u) return fail(n, SNN_E_OVERFLOW, "the synapse total exceeds its bound");
    n->nnz = nnz;
    n->max_len = hc.max_len;
    a.recs = recs;
    dfree(n, rowlen);
    dfree(n, tsum);
    // Tile-binned delivery (mode chosen above).
    n->binned_ok = ok1;
    n->two_level_ok = mode == 2;   // two levels need rows laid out for them
    if (s->solver == SNN_SOLVER_EXACT) {
        n->binned_ok = n->two_level_ok = false;
        st = setup_exact(n, tb);
        if (st) return st;
    }
    if (mode) {
        HIPCHK(n, snn::setup_kernels());
        // the expected in-degree equals the mean row length (every module alike)
        const double kin = tb.mean_out + 6.0 * std::sqrt(tb.mean_out + 1.0);
        // two-level networks are the largest: their bins hold half as much
        // (a quarter of every row firing in one step by default)
        const double frac = mode == 2 ? 0.5 * n->bin_frac : n->bin_frac;
        a.bin_cap_tile = (uint32_t)std::min(frac * (double)snn::kTile * kin + 4096.0, 1.0e9);
        e = dalloc(n, &a.bin_fill, (size_t)a.ntiles * snn::kFillStride);
        if (e == hipSuccess) e = dalloc(n, &a.bins, (size_t)a.ntiles * a.bin_cap_tile);
        if (e == hipSuccess && mode == 2) {
            // segment lists: a row touches a super tile in one segment, cut in
            // pieces of 256 records; capacity for the same fraction of every
            // row firing at once (pieces beyond it are delivered directly)
            a.nsuper = nsuper;
            a.sstart = sstart;
            const double pieces = (double)n->N * (std::min<double>(nsuper, kin) + kin / 256.0) / nsuper;
            a.dcap = (uint32_t)std::min(frac * pieces + 65536.0, 2.0e9);
            e = dalloc(n, &a.dfill, (size_t)nsuper * snn::kFillStride);
            if (e == hipSuccess) e = dalloc(n, &a.dsc, (size_t)nsuper * a.dcap);
        }
        if (e != hipSuccess) return fail(n, SNN_E_NOMEM, "device allocation failed (delivery bins)");
        HIPCHK(n, hipMemset(a.bin_fill, 0, 4 * (size_t)a.ntiles * snn::kFillStride));
        if (mode == 2) HIPCHK(n, hipMemset(a.dfill, 0, 4 * (size_t)nsuper * snn::kFillStride));
        // Per-step switch: binning costs about one read and one write of every
        // future ring row (8 D N bytes at ~5.5 TB/s); direct delivery about one
        // global atomic per event (~27 G/s).  Equal at ~0.039 D N events.
        n->bin_threshold_auto = (uint64_t)(0.039 * n->D * (double)n->N);
        a.bin_threshold = n->bin_threshold_set ? n->bin_threshold_opt : n->bin_threshold_auto;
    }
    n->mode = mode;
    a.grp_atomic = n->mode == 1 ? 0u : 1u;
    if (s->stdp) {
        st = setup_stdp(n, tb);
        if (st) return st;
    }
    n->built = true;
    n->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return SNN_OK;
}

snn_status snn_step(snn_net* n, uint32_t n_ms)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before stepping");
    if (n->exact) {
        if (n->graph_chunk == 0) {
            for (uint32_t i = 0; i < n_ms; ++i) HIPCHK(n, enqueue_exact_step(n, n->x, nullptr));
        } else {
            HIPCHK(n, step_exact(n, n_ms));
        }
        return SNN_OK;
    }
    uint32_t todo = n_ms;
    while (todo) {
        // a plastic network stops at the end of each period for its long-term
        // application
        uint32_t run = todo;
        if (n->stdp) {
            const uint64_t to_end = n->s.ltp_period - n->stdp_t % n->s.ltp_period;
            run = to_end < run ? (uint32_t)to_end : run;
        }
        uint32_t left = run;
        if (n->graph_chunk > 0) {
            while (left >= n->graph_chunk) {
                hipGraphExec_t ex = nullptr;
                HIPCHK(n, get_graph(n, n->graph_chunk, &ex));
                HIPCHK(n, hipGraphLaunch(ex, n->stream));
                left -= n->graph_chunk;
            }
        }
        if (left) {
            HIPCHK(n, enqueue_steps(n, 0, left));
            HIPCHK(n, snn::launch_advance(n->a.ctrl, left, n->stream));
        }
        HIPCHK(n, stdp_after(n, run));
        todo -= run;
    }
    return SNN_OK;
}

snn_status snn_step_forced(snn_net* n, const uint32_t* gids, size_t cnt)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before stepping");
    if (n->exact) return fail(n, SNN_E_STATE, "the exact solver takes spike times: use snn_step_forced_exact");
    if (cnt > n->N || (cnt && !gids)) return fail(n, SNN_E_INVAL, "bad forced spike set");
    for (size_t i = 0; i < cnt; ++i)
        if (gids[i] >= n->N) return fail(n, SNN_E_INVAL, "forced spike id out of range");
    if (cnt) HIPCHK(n, hipMemcpyAsync(n->forced_ids, gids, cnt * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, snn::launch_set_flags(n->forced, n->forced_ids, (uint32_t)cnt, 1, n->stream));
    StepArgs a = n->a;
    a.forced = n->forced;
    HIPCHK(n, enqueue_step(n, a, 0));
    HIPCHK(n, snn::launch_advance(a.ctrl, 1, n->stream));
    HIPCHK(n, snn::launch_set_flags(n->forced, n->forced_ids, (uint32_t)cnt, 0, n->stream));
    HIPCHK(n, stdp_after(n, 1));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    return SNN_OK;
}

}  // extern "C"

// Lock-step without allocation.  snn_step_forced_noalloc stages the forced
// spike ids and the per-neuron forced flags in this file-scope device array
// instead of the network's buffers: the flags of up to kNoAllocMaxNeurons
// neurons (one byte each), then up to kNoAllocMaxIds staged ids.  Each device
// the library runs on holds its own copy until the process ends; every call
// on a device shares it.
constexpr size_t kNoAllocMaxNeurons = size_t(1) << 24;
constexpr size_t kNoAllocMaxIds = size_t(1) << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocMaxNeurons + 4 * kNoAllocMaxIds];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// stand-in: kernels and copies get this address.
hipError_t scratch_for_current_device(uint8_t** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

snn_status snn_step_forced_noalloc(snn_net* n, const uint32_t* gids, size_t cnt)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before stepping");
    if (n->exact) return fail(n, SNN_E_STATE, "the exact solver takes spike times: use snn_step_forced_exact");
    if (cnt > kNoAllocMaxIds)
        return fail(n, SNN_E_INVAL, "forced spike set larger than the allocation-free maximum of 2^20 ids");
    if (n->N > kNoAllocMaxNeurons)
        return fail(n, SNN_E_INVAL, "network larger than the allocation-free maximum of 2^24 neurons");
    if (cnt > n->N || (cnt && !gids)) return fail(n, SNN_E_INVAL, "bad forced spike set");
    for (size_t i = 0; i < cnt; ++i)
        if (gids[i] >= n->N) return fail(n, SNN_E_INVAL, "forced spike id out of range");
    uint8_t* scr = nullptr;
    HIPCHK(n, scratch_for_current_device(&scr));
    uint8_t* flags = scr;
    uint32_t* ids = reinterpret_cast<uint32_t*>(scr + kNoAllocMaxNeurons);
    // the array keeps the last call's flags (any network's): clear this one's range
    HIPCHK(n, snn::launch_fill_u8(flags, n->N, 0, n->stream));
    if (cnt) HIPCHK(n, hipMemcpyAsync(ids, gids, cnt * 4, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, snn::launch_set_flags(flags, ids, (uint32_t)cnt, 1, n->stream));
    StepArgs a = n->a;
    a.forced = flags;
    HIPCHK(n, enqueue_step(n, a, 0));
    HIPCHK(n, snn::launch_advance(a.ctrl, 1, n->stream));
    HIPCHK(n, stdp_after(n, 1));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    return SNN_OK;
}

static snn_status read_history(snn_net* n, uint64_t t0, uint64_t t1, snn_spike* buf, uint32_t* frac, size_t cap,
                        size_t* n_out)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n_out || (cap && (!buf || (frac && !n->exact)))) return fail(n, SNN_E_INVAL, "null output");
    HIPCHK(n, hipStreamSynchronize(n->stream));
    Ctrl hc{};
    HIPCHK(n, hipMemcpy(&hc, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    const uint64_t kept = hc.hist_n < n->g.hist_cap ? hc.hist_n : n->g.hist_cap;
    // history is sorted by time: binary-search the [t0, t1) range
    auto time_at = [&](uint64_t i, uint32_t* t) -> hipError_t {
        uint2 v;
        hipError_t e = hipMemcpy(&v, n->a.hist + i, sizeof(uint2), hipMemcpyDeviceToHost);
        *t = v.x;
        return e;
    };
    auto lower = [&](uint64_t tv, uint64_t* pos) -> hipError_t {
        uint64_t lo = 0, hi = kept;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            uint32_t tm = 0;
            hipError_t e = time_at(mid, &tm);
            if (e != hipSuccess) return e;
            if ((uint64_t)tm < tv) lo = mid + 1;
            else hi = mid;
        }
        *pos = lo;
        return hipSuccess;
    };
    uint64_t p0 = 0, p1 = kept;
    if (t0 > 0) HIPCHK(n, lower(t0, &p0));
    if (t1 <= hc.t0) HIPCHK(n, lower(t1, &p1));
    if (p1 < p0) p1 = p0;
    const uint64_t m = p1 - p0;
    *n_out = (size_t)m;
    if (m > cap) return fail(n, SNN_E_TRUNC, "spike buffer too small");
    if (m) HIPCHK(n, hipMemcpy(buf, n->a.hist + p0, m * sizeof(snn_spike), hipMemcpyDeviceToHost));
    if (m && frac) HIPCHK(n, hipMemcpy(frac, n->x.hist_f + p0, m * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (hc.hist_n > n->g.hist_cap) return fail(n, SNN_E_TRUNC, "spike history overflowed its capacity");
    return check_dropped(n);
}

snn_status snn_read_spikes(snn_net* n, uint64_t t0, uint64_t t1, snn_spike* buf, size_t cap,
                           size_t* n_out)
{
    return read_history(n, t0, t1, buf, nullptr, cap, n_out);
}

snn_status snn_read_spike_times(snn_net* n, uint64_t t0, uint64_t t1, snn_spike* buf, uint32_t* frac,
                                size_t cap, size_t* n_out)
{
    if (n && !n->exact) return fail(n, SNN_E_STATE, "spike offsets exist only under the exact solver");
    if (cap && !frac) return fail(n, SNN_E_INVAL, "null output");
    return read_history(n, t0, t1, buf, frac, cap, n_out);
}

snn_status snn_step_forced_exact(snn_net* n, const uint32_t* gids, const uint32_t* frac, size_t cnt)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before stepping");
    if (!n->exact) return fail(n, SNN_E_STATE, "snn_step_forced_exact needs the exact solver");
    if (cnt > n->N || (cnt && (!gids || !frac))) return fail(n, SNN_E_INVAL, "bad forced spike set");
    std::vector<uint8_t> flags(n->N, 0);
    std::vector<uint32_t> ff(n->N, 0);
    for (size_t i = 0; i < cnt; ++i) {
        if (gids[i] >= n->N) return fail(n, SNN_E_INVAL, "forced spike id out of range");
        if (flags[gids[i]]) return fail(n, SNN_E_INVAL, "a neuron is forced twice in one step");
        flags[gids[i]] = 1;
        ff[gids[i]] = frac[i];
    }
    HIPCHK(n, hipMemcpyAsync(n->xforced, flags.data(), n->N, hipMemcpyHostToDevice, n->stream));
    HIPCHK(n, hipMemcpyAsync(n->xforced_f, ff.data(), 4 * (size_t)n->N, hipMemcpyHostToDevice, n->stream));
    snn::XArgs x = n->x;
    x.forced = n->xforced;
    x.forced_f = n->xforced_f;
    HIPCHK(n, enqueue_exact_step(n, x, nullptr));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    return SNN_OK;
}

snn_status snn_read_queue(snn_net* n, uint32_t k, uint32_t* tgt, uint32_t* frac, int32_t* wq, size_t cap,
                          size_t* n_out)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->exact) return fail(n, SNN_E_STATE, "input queues exist only under the exact solver");
    if (!n_out || (cap && (!tgt || !frac || !wq))) return fail(n, SNN_E_INVAL, "null output");
    if (k >= n->x.R) return fail(n, SNN_E_INVAL, "arrival step beyond the largest delay");
    HIPCHK(n, hipStreamSynchronize(n->stream));
    const uint32_t slot = (n->xt + k) % n->x.R;
    unsigned long long qn = 0;
    HIPCHK(n, hipMemcpy(&qn, n->x.qn + slot, 8, hipMemcpyDeviceToHost));
    const uint64_t m = qn < n->x.qcap ? qn : n->x.qcap;
    *n_out = (size_t)m;
    if (m > cap) return fail(n, SNN_E_TRUNC, "queue buffer too small");
    std::vector<uint4> q(m);
    if (m) HIPCHK(n, hipMemcpy(q.data(), n->x.qlist + (size_t)slot * n->x.qcap, m * sizeof(uint4),
                               hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < m; ++i) {
        tgt[i] = q[i].x;
        frac[i] = q[i].y;
        wq[i] = (int32_t)q[i].z;
    }
    return check_dropped(n);
}

snn_status snn_read_state(snn_net* n, float* v, float* w, uint8_t* ref)
{
    snn_status st = check_usable(n);
    if (st) return st;
    HIPCHK(n, hipStreamSynchronize(n->stream));
    if (v) HIPCHK(n, hipMemcpy(v, n->a.V, (size_t)n->N * 4, hipMemcpyDeviceToHost));
    if (w) HIPCHK(n, hipMemcpy(w, n->a.W, (size_t)n->N * 4, hipMemcpyDeviceToHost));
    if (ref && n->exact) {
        // whole steps of refractoriness left after the last step
        std::vector<uint64_t> re(n->N);
        HIPCHK(n, hipMemcpy(re.data(), n->x.rend, (size_t)n->N * 8, hipMemcpyDeviceToHost));
        const uint64_t now = (uint64_t)n->xt << 32;
        for (uint32_t i = 0; i < n->N; ++i)
            ref[i] = re[i] > now ? (uint8_t)std::min<uint64_t>((re[i] - now + 0xFFFFFFFFull) >> 32, 255) : 0;
    } else if (ref) {
        HIPCHK(n, hipMemcpy(ref, n->a.ref, (size_t)n->N, hipMemcpyDeviceToHost));
    }
    return SNN_OK;
}

snn_status snn_read_ring(snn_net* n, int32_t* host_ring)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!host_ring) return fail(n, SNN_E_INVAL, "null output");
    HIPCHK(n, hipStreamSynchronize(n->stream));
    HIPCHK(n, hipMemcpy(host_ring, n->a.ring, (size_t)snn::kRing * n->N * 4, hipMemcpyDeviceToHost));
    return SNN_OK;
}

snn_status snn_export_rows(snn_net* n, uint32_t pre0, uint32_t cnt, uint64_t* row_len,
                           uint16_t* bend, void* rec_buf, size_t rec_cap, size_t* n_out)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "no synapses built");
    if ((uint64_t)pre0 + cnt > n->N || !n_out) return fail(n, SNN_E_INVAL, "row range out of bounds");
    HIPCHK(n, hipStreamSynchronize(n->stream));
    std::vector<uint64_t> rp((size_t)cnt + 1);
    HIPCHK(n, hipMemcpy(rp.data(), n->a.row_ptr + pre0, ((size_t)cnt + 1) * 8, hipMemcpyDeviceToHost));
    if (row_len)
        for (uint32_t i = 0; i < cnt; ++i) row_len[i] = rp[i + 1] - rp[i];
    if (bend && cnt)
        HIPCHK(n, hipMemcpy(bend, n->a.bend + (size_t)pre0 * n->D, (size_t)cnt * n->D * 2, hipMemcpyDeviceToHost));
    const uint64_t m = rp[cnt] - rp[0];
    *n_out = (size_t)m;
    if (m > rec_cap) return fail(n, SNN_E_TRUNC, "record buffer too small");
    const size_t rb = n->s.record == SNN_REC_CODE8 ? 4 : 8;
    if (m && rec_buf)
        HIPCHK(n, hipMemcpy(rec_buf, (const uint8_t*)n->a.recs + rp[0] * rb, m * rb, hipMemcpyDeviceToHost));
    if (m && rec_buf && n->s.record != SNN_REC_CODE8) {
        // 8-byte records: the target without the delay bucket it carries
        uint32_t* r = static_cast<uint32_t*>(rec_buf);
        for (uint64_t i = 0; i < m; ++i) r[2 * i] &= snn::kTgtMask;
    }
    if (m && rec_buf && n->a.nsuper) {
        // rows laid out by super tile: back to (delay, target) order, records
        // target << 8 | code (within a (super tile, delay) run the targets
        // ascend, and the super tiles come in order)
        const uint32_t ns = n->a.nsuper;
        std::vector<uint16_t> ss((size_t)cnt * ns);
        HIPCHK(n, hipMemcpy(ss.data(), n->a.sstart + (size_t)pre0 * ns, ss.size() * 2, hipMemcpyDeviceToHost));
        uint32_t* r = static_cast<uint32_t*>(rec_buf);
        std::vector<uint32_t> row, out;
        for (uint32_t i = 0; i < cnt; ++i) {
            const uint64_t o = rp[i] - rp[0], len = rp[i + 1] - rp[i];
            row.assign(r + o, r + o + len);
            out.clear();
            for (uint32_t b = 0; b < n->D; ++b)
                for (uint32_t sp = 0; sp < ns; ++sp) {
                    const uint32_t s0 = ss[(size_t)i * ns + sp];
                    const uint32_t s1 = sp + 1 < ns ? ss[(size_t)i * ns + sp + 1] : (uint32_t)len;
                    for (uint32_t k = s0; k < s1; ++k) {
                        const uint32_t v = row[k];
                        if (((v >> snn::kSegBits) & 31u) != b) continue;
                        const uint32_t tgt = (sp << snn::kSegBits) | (v & ((1u << snn::kSegBits) - 1u));
                        out.push_back((tgt << 8) | (v >> (snn::kSegBits + 5)));
                    }
                }
            if (out.size() != len) return fail(n, SNN_E_STATE, "segmented row does not decode");
            std::copy(out.begin(), out.end(), r + o);
        }
    }
    return SNN_OK;
}

}  // extern "C"
void fill_stats(const snn_net* n, const Ctrl& hc, snn_stats_t* out);
extern "C" {

snn_status snn_stats(snn_net* n, snn_stats_t* out)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!out) return fail(n, SNN_E_INVAL, "null output");
    HIPCHK(n, hipStreamSynchronize(n->stream));
    Ctrl hc{};
    HIPCHK(n, hipMemcpy(&hc, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    fill_stats(n, hc, out);
    return check_dropped(n);
}

}  // extern "C"

void fill_stats(const snn_net* n, const Ctrl& hc, snn_stats_t* out)
{
    out->t = hc.t0;
    out->spikes = hc.spikes;
    out->rec_events = hc.rec_events;
    out->ext_events = hc.ext_events;
    out->nnz = n->nnz;
    out->n_neurons = n->N;
    out->bytes_device = n->bytes;
    out->hist_n = hc.hist_n;
    out->disagree = hc.disagree;
    out->bin_overflow = hc.bin_overflow;
    out->deliver_mode = n->mode;
    out->bin_threshold = n->a.bin_threshold;
    out->binned_ok = (n->binned_ok ? 1u : 0u) | (n->two_level_ok ? 2u : 0u);
    out->build_ms = n->build_ms;
}

extern "C" {

// Kernel timing of the exact solver: place, update and deliver launches
// stamped by their own events, and each whole step between two events.
static snn_status time_exact(snn_net* n, uint32_t n_ms, snn_kernel_times* out)
{
    std::memset(out, 0, sizeof(*out));
    constexpr uint32_t kB = 64;   // steps per batch
    std::vector<snn::LaunchEv> ev(kB * 4);
    hipError_t e = hipSuccess;
    for (auto& x : ev) {
        if (e == hipSuccess) e = hipEventCreate(&x.start);
        if (e == hipSuccess) e = hipEventCreate(&x.stop);
    }
    auto destroy = [&]() {
        for (auto& x : ev) {
            if (x.start) (void)hipEventDestroy(x.start);
            if (x.stop) (void)hipEventDestroy(x.stop);
        }
    };
    Ctrl c0{}, c1{};
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e == hipSuccess) e = hipMemcpy(&c0, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    double sum[4] = {0, 0, 0, 0};
    for (uint32_t b0 = 0; b0 < n_ms && e == hipSuccess; b0 += kB) {
        const uint32_t nb = (n_ms - b0) < kB ? (n_ms - b0) : kB;
        for (uint32_t i = 0; i < nb && e == hipSuccess; ++i) {
            snn::LaunchEv* x = &ev[i * 4];
            e = hipEventRecord(x[3].start, n->stream);
            if (e == hipSuccess) e = enqueue_exact_step(n, n->x, x);
            if (e == hipSuccess) e = hipEventRecord(x[3].stop, n->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
        for (uint32_t j = 0; j < nb * 4 && e == hipSuccess; ++j) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, ev[j].start, ev[j].stop);
            sum[j % 4] += ms;
        }
    }
    if (e == hipSuccess) e = hipMemcpy(&c1, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    destroy();
    if (e != hipSuccess) {
        n->poisoned = true;
        return fail_hip(n, e, "kernel timing");
    }
    const double steps = n_ms ? (double)n_ms : 1.0;
    out->scatter_ms = sum[0] / steps;
    out->update_ms = sum[1] / steps;
    out->deliver_ms = sum[2] / steps;
    out->step_ms = sum[3] / steps;
    out->steps = n_ms;
    out->rec_events = c1.rec_events - c0.rec_events;
    out->spikes = c1.spikes - c0.spikes;
    return check_dropped(n);
}

snn_status snn_time_kernels(snn_net* n, uint32_t n_ms, snn_kernel_times* out)
{
    snn_status st = check_usable(n);
    if (st) return st;
    if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before stepping");
    if (!out) return fail(n, SNN_E_INVAL, "null output");
    if (n->exact) return time_exact(n, n_ms, out);
    if (n->stdp) return fail(n, SNN_E_STATE, "per-launch timing is not available for plastic networks");
    if (check_items(n) != hipSuccess) return fail(n, SNN_E_INVAL, "spike items exceed 32 bits");
    std::memset(out, 0, sizeof(*out));
    // The steps are the ones snn_step enqueues (same kernels, same order), each
    // launch stamped with its own start/stop events; steps go out in batches
    // and the events of a batch are read once it has finished.
    constexpr uint32_t kB = 128, kL = 5;   // steps per batch, launches per step (at most)
    std::vector<snn::LaunchEv> ev(kB * kL);
    hipError_t e = hipSuccess;
    for (auto& x : ev) {
        if (e == hipSuccess) e = hipEventCreate(&x.start);
        if (e == hipSuccess) e = hipEventCreate(&x.stop);
    }
    auto destroy = [&]() {
        for (auto& x : ev) {
            if (x.start) (void)hipEventDestroy(x.start);
            if (x.stop) (void)hipEventDestroy(x.stop);
        }
    };
    if (e != hipSuccess) {
        destroy();
        return fail_hip(n, e, "hipEventCreate");
    }
    Ctrl c0{}, c1{};
    e = hipStreamSynchronize(n->stream);
    if (e == hipSuccess) e = hipMemcpy(&c0, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    const bool fused = seq(n) != 0 && n->a.d_min == 1;
    // kind of each launch slot: 0 update, 1 compact, 2 direct deliver, 3 scatter, 4 tile, 5 second pass
    double sum[6] = {0, 0, 0, 0, 0, 0};
    uint32_t cnt[6] = {0, 0, 0, 0, 0, 0};
    std::vector<int> kind(kB * kL, -1);
    for (uint32_t b0 = 0; b0 < n_ms && e == hipSuccess; b0 += kB) {
        const uint32_t nb = (n_ms - b0) < kB ? (n_ms - b0) : kB;
        std::fill(kind.begin(), kind.end(), -1);
        for (uint32_t i = 0; i < nb && e == hipSuccess; ++i) {
            const uint32_t k = b0 + i;
            snn::LaunchEv* x = &ev[i * kL];
            if (!fused || k == 0) {
                e = snn::launch_update(n->a, k, n->stream, &x[0]);
                kind[i * kL] = 0;
            }
            if (e != hipSuccess) break;
            if (seq(n) != 0) {
                if (seq(n) == 2) {
                    e = snn::launch_compact(n->a, k, n->stream, &x[3]);
                    kind[i * kL + 3] = 1;
                }
                if (e == hipSuccess) e = snn::launch_scatter(n->a, k, n->max_len, n->scatter_blocks, n->stream, &x[1]);
                kind[i * kL + 1] = 3;
                if (e == hipSuccess && seq(n) == 2) {
                    e = snn::launch_sub(n->a, k, n->scatter_blocks, n->stream, &x[4]);
                    kind[i * kL + 4] = 5;
                }
                if (e == hipSuccess) e = snn::launch_tile(n->a, k, fused && k + 1 < n_ms, n->stream, &x[2]);
                kind[i * kL + 2] = 4;
            } else {
                e = snn::launch_compact(n->a, k, n->stream, &x[1]);
                kind[i * kL + 1] = 1;
                if (e == hipSuccess)
                    e = snn::launch_deliver(n->a, k, n->deliver_waves, n->unroll, n->max_len, n->stream, &x[2]);
                kind[i * kL + 2] = 2;
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
        for (uint32_t j = 0; j < nb * kL && e == hipSuccess; ++j) {
            if (kind[j] < 0) continue;
            float ms = 0;
            e = hipEventElapsedTime(&ms, ev[j].start, ev[j].stop);
            sum[kind[j]] += ms;
            cnt[kind[j]] += 1;
        }
    }
    if (e == hipSuccess) e = snn::launch_advance(n->a.ctrl, n_ms, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e == hipSuccess) e = hipMemcpy(&c1, n->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    destroy();
    if (e != hipSuccess) {
        n->poisoned = true;
        return fail_hip(n, e, "kernel timing");
    }
    auto avg = [&](int i) { return cnt[i] ? sum[i] / cnt[i] : 0.0; };
    const double steps = n_ms ? (double)n_ms : 1.0;
    out->update_ms = avg(0);
    out->compact_ms = avg(1);
    out->scatter_ms = avg(3);
    out->tile_ms = avg(4);
    out->sub_ms = avg(5);
    out->deliver_ms = seq(n) != 0 ? avg(3) + avg(4) + avg(5) : avg(2);
    out->step_ms = (sum[0] + sum[1] + sum[2] + sum[3] + sum[4] + sum[5]) / steps;
    out->steps = n_ms;
    out->rec_events = c1.rec_events - c0.rec_events;
    out->spikes = c1.spikes - c0.spikes;
    return SNN_OK;
}

snn_status snn_reset(snn_net* n)
{
    snn_status st = check_usable(n);
    if (st) return st;
    StepArgs& a = n->a;
    HIPCHK(n, hipMemsetAsync(a.ring, 0, sizeof(int32_t) * (size_t)snn::kRing * n->N, n->stream));
    HIPCHK(n, hipMemsetAsync(a.grp_cnt, 0, sizeof(uint32_t) * 2 * a.ngrp, n->stream));
    HIPCHK(n, hipMemsetAsync(a.ctrl, 0, sizeof(Ctrl), n->stream));
    if (a.bin_fill) HIPCHK(n, hipMemsetAsync(a.bin_fill, 0, 4 * (size_t)a.ntiles * snn::kFillStride, n->stream));
    if (a.dfill) HIPCHK(n, hipMemsetAsync(a.dfill, 0, 4 * (size_t)a.nsuper * snn::kFillStride, n->stream));
    HIPCHK(n, snn::launch_init(a, n->stream));
    n->stdp_t = 0;   // a plastic network keeps the weights it has learned
    if (n->exact) {
        const snn::XArgs& x = n->x;
        HIPCHK(n, hipMemsetAsync(x.rend, 0, 8 * (size_t)n->N, n->stream));
        HIPCHK(n, hipMemsetAsync(x.gcnt, 0, 4 * (size_t)x.ngroups, n->stream));
        HIPCHK(n, hipMemsetAsync(x.qn, 0, 8 * (size_t)x.R, n->stream));
        HIPCHK(n, hipMemsetAsync(x.dropped, 0, 8, n->stream));
        n->xt = 0;
    }
    if (n->built) {
        // the construction statistics live in the control block too
        snn::Ctrl keep{};
        keep.max_len = n->max_len;
        HIPCHK(n, hipMemcpyAsync(a.ctrl, &keep, sizeof(Ctrl), hipMemcpyHostToDevice, n->stream));
    }
    HIPCHK(n, hipStreamSynchronize(n->stream));
    return SNN_OK;
}

snn_status snn_set_option(snn_net* n, int key, int64_t value)
{
    snn_status st = check_usable(n);
    if (st) return st;
    switch (key) {
    case SNN_OPT_GRAPH_CHUNK:
        if (value < 0 || value > 4096) return fail(n, SNN_E_INVAL, "graph chunk out of range");
        n->graph_chunk = (uint32_t)value;
        break;
    case SNN_OPT_DELIVER_WAVES:
        if (value < 4 || value > (1 << 20)) return fail(n, SNN_E_INVAL, "wave count out of range");
        n->deliver_waves = (uint32_t)value;
        break;
    case SNN_OPT_QUEUE_CAP:
        if (n->built) return fail(n, SNN_E_STATE, "queue capacity is fixed once synapses are built");
        if (value < 0 || value > 4000000000ll) return fail(n, SNN_E_INVAL, "queue capacity out of range");
        n->qcap_opt = (uint64_t)value;
        return SNN_OK;
    case SNN_OPT_DELIVER_MODE:
        if (value < 0 || value > 2) return fail(n, SNN_E_INVAL, "delivery mode must be 0, 1 or 2");
        if (n->exact) return fail(n, SNN_E_STATE, "the exact solver delivers through its own input queues");
        if (!n->built) {
            n->mode_pref = (int)value;    // before the build: selects which bins are allocated
            return SNN_OK;
        }
        {
            // bins exist for the mode chosen at the build (single level, or two levels)
            const bool have1 = n->binned_ok && n->a.bins && !n->a.nsuper;
            const bool have2 = n->a.nsuper != 0;
            if ((value == 1 && !have1) || (value == 2 && !have2))
                return fail(n, SNN_E_INVAL, "this delivery mode was not selected when the synapses were built");
        }
        n->mode = (uint32_t)value;
        n->a.bin_threshold = threshold_in_force(n);
        HIPCHK(n, hipStreamSynchronize(n->stream));
        HIPCHK(n, hipMemset(reinterpret_cast<char*>(n->a.ctrl) + offsetof(Ctrl, step_ev), 0, sizeof(uint64_t) * 2));
        // direct delivery's compaction reads the group counts, which the
        // update maintains only while direct delivery is selected
        n->a.grp_atomic = n->mode == 1 ? 0u : 1u;
        HIPCHK(n, hipStreamSynchronize(n->stream));
        HIPCHK(n, hipMemset(n->a.grp_cnt, 0, sizeof(uint32_t) * 2 * n->a.ngrp));
        break;
    case SNN_OPT_BIN_FRAC_PPM:
        if (n->built) return fail(n, SNN_E_STATE, "bin capacity is fixed once synapses are built");
        if (value < 1 || value > 4000000) return fail(n, SNN_E_INVAL, "bin fraction out of range");
        n->bin_frac = (double)value * 1e-6;
        return SNN_OK;
    case SNN_OPT_BIN_THRESHOLD:
        if (value < 0) return fail(n, SNN_E_INVAL, "threshold must be >= 0");
        n->bin_threshold_set = true;
        n->bin_threshold_opt = (uint64_t)value;
        n->a.bin_threshold = threshold_in_force(n);
        break;
    case SNN_OPT_EXT_RATE_UHZ: {
        if (!n->built) return fail(n, SNN_E_STATE, "build the synapses before changing the drive");
        if (value < 0) return fail(n, SNN_E_INVAL, "rate must be >= 0");
        if (n->s.ext_mode != SNN_EXT_POISSON) return fail(n, SNN_E_INVAL, "network has no Poisson drive");
        snn::TableParams tp = table_params(n->g, n->s);
        tp.ext_rate_hz = (double)value * 1e-6;
        snn::HostTables tb;
        std::string why = snn::build_tables(tp, tb);
        if (!why.empty()) return fail(n, SNN_E_INVAL, why);
        HIPCHK(n, hipStreamSynchronize(n->stream));
        HIPCHK(n, hipMemcpy((void*)n->a.poisc, tb.poisc.data(), tb.poisc.size() * 4, hipMemcpyHostToDevice));
        n->a.npois = (uint32_t)tb.poisc.size();
        n->x.npois = n->a.npois;   // the exact solver reads the same table
        n->s.ext_rate_hz = tp.ext_rate_hz;
        break;
    }
    case SNN_OPT_SCATTER_BLOCKS:
        if (value < 1 || value > 65536) return fail(n, SNN_E_INVAL, "scatter blocks out of range");
        n->scatter_blocks = (uint32_t)value;
        break;
    case SNN_OPT_DELIVER_UNROLL:
        if (value != 1 && value != 2 && value != 4) return fail(n, SNN_E_INVAL, "unroll must be 1, 2 or 4");
        n->unroll = (uint32_t)value;
        break;
    default:
        return fail(n, SNN_E_INVAL, "unknown option");
    }
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    drop_graphs(n);
    return SNN_OK;
}

snn_status snn_host_tables(const snn_grid_desc* g, const snn_syn_desc* s, uint32_t* T, int32_t* wtab,
                           int32_t* cb, uint32_t* poisc, uint32_t* npois, double* consts)
{
    if (!g || !s) return fail(nullptr, SNN_E_INVAL, "null argument");
    std::string why;
    if (!valid_grid(g, why)) return fail(nullptr, SNN_E_INVAL, why);
    snn::TableParams tp = table_params(*g, *s);
    snn::HostTables tb;
    why = snn::build_tables(tp, tb);
    if (!why.empty()) return fail(nullptr, SNN_E_INVAL, why);
    if (T) std::memcpy(T, tb.T.data(), tb.T.size() * 4);
    if (wtab) std::memcpy(wtab, tb.wtab.data(), 65536 * 4);
    if (cb) std::memcpy(cb, tb.cb.data(), 256 * 4);
    if (poisc && !tb.poisc.empty()) std::memcpy(poisc, tb.poisc.data(), tb.poisc.size() * 4);
    if (npois) *npois = (uint32_t)tb.poisc.size();
    if (consts) {
        consts[0] = tb.dm;
        consts[1] = tb.dw;
        consts[2] = tb.kappa;
    }
    return SNN_OK;
}

snn_status snn_host_stdp_tables(const snn_grid_desc* g, const snn_syn_desc* s, int32_t* kp, int32_t* km,
                                uint32_t* win, int32_t* wmax_q)
{
    if (!g || !s) return fail(nullptr, SNN_E_INVAL, "null argument");
    if (s->stdp != 1) return fail(nullptr, SNN_E_INVAL, "the description has no plasticity");
    std::string why;
    if (!valid_grid(g, why)) return fail(nullptr, SNN_E_INVAL, why);
    snn::HostTables tb;
    why = snn::build_tables(table_params(*g, *s), tb);
    if (!why.empty()) return fail(nullptr, SNN_E_INVAL, why);
    if (kp) std::memcpy(kp, tb.kp.data(), tb.kp.size() * 4);
    if (km) std::memcpy(km, tb.km.data(), tb.km.size() * 4);
    if (win) *win = tb.stdp_win;
    if (wmax_q) *wmax_q = tb.wmax_q;
    return SNN_OK;
}

void snn_destroy(snn_net* n)
{
    if (!n) return;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    drop_graphs(n);
    for (auto& p : n->allocs) dev_free(n->dev_alloc, p.first);
    n->allocs.clear();
    if (n->own_stream && n->stream) (void)hipStreamDestroy(n->stream);
    delete n;
}

}  // extern "C"

/* ------------------------------------------------------------------------ */
/* Batched stepping                                                          */
/* ------------------------------------------------------------------------ */
struct snn_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    static constexpr int kBuilders = 2;   // construction threads, each with its own stream
    hipStream_t build_stream[kBuilders] = {};
    uint64_t budget = 0, used = 0;        // used: held or reserved by admitted jobs
    uint32_t blk_cap = 0, blk_used = 0;   // blk_used: blocks of the jobs in the device table
    uint32_t blk_reserved = 0;            // blocks of every admitted job (building included)
    uint32_t scatter_blocks = 256;        // one 1024-thread workgroup per CU (its LDS use allows no more)
    uint32_t deliver_mode = 1;            // 0: every job direct; 1: tile-binned where the job allows it
    uint64_t thr_ppm = 0;                 // binned steps from ppm * N * D events (0: each job's own)
    enum State { kFree, kBuilding, kActive, kFailed };
    struct Job {
        snn_net* net = nullptr;
        uint64_t bytes = 0;
        uint32_t dur = 0, nblk = 0;
        uint32_t t = 0;               // steps enqueued for the job (host-side schedule)
        State state = kFree;
        bool binned = false;          // built with delivery bins for the batched kernels
        snn_status fail_st = SNN_OK;  // kFailed: why
        std::string fail_msg;
    };
    Job jobs[snn::kMaxJobs];
    snn::JobDesc* d_jobs = nullptr;
    DevAllocator dev_alloc;            // the allocator d_jobs came from
    static constexpr int kTables = 8;  // pinned staging copies of the table, used in turn
    snn::JobDesc* h_jobs[kTables] = {};
    hipEvent_t h_done[kTables] = {};
    int h_next = 0;
    // captured chunks by (steps, grid blocks of the update and tile kernels)
    std::map<std::pair<uint32_t, uint32_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    std::string err;
    bool poisoned = false;
    // Construction threads: build admitted jobs, two at a time, each on its
    // own stream, while the caller keeps stepping, and free retired jobs once
    // the stepping stream has passed the table update that removed them.
    struct BuildReq {
        int slot;
        snn_grid_desc g;
        snn_syn_desc s;
    };
    struct Retired {
        snn_net* net;
        hipEvent_t after;
    };
    std::mutex mu;
    std::condition_variable cv;        // worker: work to do; caller: a build finished
    // Graph capture on the stepping stream excludes the construction threads'
    // runtime calls (allocation, frees that synchronise the device, memsets),
    // which would invalidate a capture in progress; builds share the lock.
    std::shared_mutex capture_mu;
    std::deque<BuildReq> todo;
    std::vector<std::pair<int, snn_net*>> built;   // finished builds, activated at the next step
    std::deque<Retired> retired;
    bool stop = false;
    std::thread workers[kBuilders];
};

namespace {

thread_local std::string g_batch_err;

snn_status bfail(snn_batch* b, snn_status st, const std::string& msg)
{
    if (b) b->err = msg;
    else g_batch_err = msg;
    return st;
}

#define BHIPCHK(b, x)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            (b)->poisoned = true;                                                             \
            return bfail(b, SNN_E_HIP, std::string("HIP error in " #x ": ") + hipGetErrorString(e_)); \
        }                                                                                     \
    } while (0)

// A batch job may use binned delivery: F32 records, the fused next-step update
// (d_min == 1) and a tile's delay rows within the batched tile kernel's LDS.
bool batch_binnable(const snn_syn_desc& s)
{
    return s.record != SNN_REC_CODE8 && s.d_min == 1 && s.d_max - s.d_min + 1 <= snn::kBatchMaxD;
}

// Device bytes a network will hold (upper estimate used for admission).
uint64_t estimate_bytes(const snn_grid_desc& g, const snn_syn_desc& s, uint64_t hist_cap)
{
    const uint64_t M = (uint64_t)g.n_exc + g.n_inh, N = (uint64_t)g.gx * g.gy * M;
    const uint64_t D = s.d_max - s.d_min + 1;
    const uint64_t nblk = (N + 1023) / 1024;
    std::vector<uint32_t> T;
    double mean_out = 0.0, max_out = 0.0;
    if (!snn::connection_tables(table_params(g, s), T, mean_out, max_out).empty()) mean_out = s.k_in;
    const double k = mean_out + 6.0 * std::sqrt(mean_out + 1.0);
    const uint64_t rec = s.record == SNN_REC_CODE8 ? 4 : 8;
    uint64_t b = N * (4 + 4 + 1) + 32 * N * 4 + nblk * 16 + nblk * 1024 * 16 + N * 16 + hist_cap * 8 + N * 5;
    b += (uint64_t)g.gx * g.gy * 4 + 65536 * 4 + 1024 + 256 + (N + 1) * 8 + N * D * 2;
    b += (uint64_t)((double)N * k) * rec + N * 4 + (1ull << 20);
    if (batch_binnable(s)) b += nblk * 4 * snn::kFillStride + nblk * (uint64_t)(0.5 * 1024.0 * k + 4096.0) * 4;
    return b;
}

void batch_drop_graphs(snn_batch* b)
{
    for (auto& kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->graphs.clear();
}

// Rewrite the device job table (block ranges are packed in slot order).  The
// copy is ordered on the stepping stream after the steps already enqueued; the
// pinned staging buffers are reused in turn once their previous copy is done.
// Caller holds b->mu.
hipError_t batch_upload(snn_batch* b)
{
    const int i = b->h_next;
    b->h_next = (b->h_next + 1) % snn_batch::kTables;
    hipError_t e = hipEventSynchronize(b->h_done[i]);
    if (e != hipSuccess) return e;
    snn::JobDesc* tab = b->h_jobs[i];
    uint32_t base = 0;
    for (uint32_t j = 0; j < snn::kMaxJobs; ++j) {
        snn::JobDesc& d = tab[j];
        std::memset(&d, 0, sizeof(d));
        const snn_batch::Job& J = b->jobs[j];
        if (J.state != snn_batch::kActive) continue;
        d.a = J.net->a;
        d.t_end = J.dur;
        d.active = 1;
        d.blk_base = base;
        d.smax = J.net->max_len ? (J.net->max_len + 255) / 256 : 1;
        d.binned = (b->deliver_mode == 1 && J.binned && J.net->binned_ok && d.a.bins) ? 1u : 0u;
        if (b->thr_ppm) d.a.bin_threshold = (uint64_t)((double)b->thr_ppm * 1e-6 * J.net->N * J.net->D);
        base += J.nblk;
    }
    b->blk_used = base;
    e = hipMemcpyAsync(b->d_jobs, tab, sizeof(snn::JobDesc) * snn::kMaxJobs, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return e;
    return hipEventRecord(b->h_done[i], b->stream);
}

// Jobs whose construction has finished join the table.  Caller holds b->mu.
hipError_t batch_activate(snn_batch* b)
{
    if (b->built.empty()) return hipSuccess;
    for (auto& kv : b->built) {
        snn_batch::Job& J = b->jobs[kv.first];
        if (!kv.second) continue;   // the worker already marked the job failed
        J.net = kv.second;
        b->used = b->used - J.bytes + J.net->bytes;   // the estimate gives way to the real footprint
        J.bytes = J.net->bytes;
        J.t = 0;
        J.state = snn_batch::kActive;
    }
    b->built.clear();
    return batch_upload(b);
}

void batch_worker(snn_batch* b, int w)
{
    std::unique_lock<std::mutex> lk(b->mu);
    for (;;) {
        b->cv.wait(lk, [b] { return b->stop || !b->todo.empty() || !b->retired.empty(); });
        if (!b->retired.empty()) {
            const snn_batch::Retired r = b->retired.front();
            b->retired.pop_front();
            lk.unlock();
            {
                // the event was recorded on the stepping stream: waiting for it
                // while that stream is being captured would invalidate the
                // capture, so the wait holds the capture lock too (the event
                // completes with work already enqueued: the capture only waits)
                std::shared_lock<std::shared_mutex> cap(b->capture_mu);
                (void)hipEventSynchronize(r.after);   // no kernel still reads the job's descriptor
                (void)hipEventDestroy(r.after);
                snn_destroy(r.net);
            }
            lk.lock();
            continue;
        }
        if (b->stop) break;
        const snn_batch::BuildReq q = b->todo.front();
        b->todo.pop_front();
        lk.unlock();
        snn_net* n = nullptr;
        std::string msg;
        snn_status st;
        {
            std::shared_lock<std::shared_mutex> cap(b->capture_mu);
            st = snn_build_grid(&q.g, b->build_stream[w], &n);
            if (st) {
                msg = snn_last_error(nullptr);
            } else {
                if (!batch_binnable(q.s)) snn_set_option(n, SNN_OPT_DELIVER_MODE, 0);   // no bins to allocate
                st = snn_build_synapses(n, &q.s);
                if (st) {
                    msg = snn_last_error(n);
                    snn_destroy(n);
                    n = nullptr;
                }
            }
        }
        lk.lock();
        if (st) {
            snn_batch::Job& J = b->jobs[q.slot];
            J.state = snn_batch::kFailed;
            J.fail_st = st;
            J.fail_msg = msg;
        }
        b->built.emplace_back(q.slot, n);
        b->cv.notify_all();
    }
}

// Grid of the per-block kernels for the blocks in use: the next power of two
// (at least 64), so that a few captured graphs serve every batch size.
uint32_t batch_grid(const snn_batch* b)
{
    uint32_t g = 64;
    while (g < b->blk_used) g <<= 1;
    return g < b->blk_cap ? g : b->blk_cap;
}

hipError_t batch_graph(snn_batch* b, uint32_t chunk, hipGraphExec_t* out)
{
    const uint32_t grid = batch_grid(b);
    const auto key = std::make_pair(chunk, grid);
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
        *out = it->second.second;
        return hipSuccess;
    }
    hipGraph_t gr = nullptr;
    hipGraphExec_t ex = nullptr;
    std::unique_lock<std::shared_mutex> cap(b->capture_mu);   // no construction call during the capture
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    // step k: delivery of step k's spikes (binned or direct per job), then the
    // tiles, which also update the neurons for step k + 1; the chunk's first
    // update runs on its own and its last tile kernel updates nothing.
    le = snn::launch_batch_update(b->d_jobs, grid, 0, b->stream);
    for (uint32_t k = 0; k < chunk && le == hipSuccess; ++k) {
        le = snn::launch_batch_scatter(b->d_jobs, b->scatter_blocks, k, b->stream);
        if (le == hipSuccess) le = snn::launch_batch_tile(b->d_jobs, grid, k, k + 1 < chunk, b->stream);
    }
    if (le == hipSuccess) le = snn::launch_batch_advance(b->d_jobs, chunk, b->stream);
    e = hipStreamEndCapture(b->stream, &gr);
    if (le != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return e;
    }
    b->graphs[key] = std::make_pair(gr, ex);
    *out = ex;
    return hipSuccess;
}

snn_status batch_check(snn_batch* b)
{
    if (!b) return bfail(nullptr, SNN_E_INVAL, "null batch handle");
    if (b->poisoned) return SNN_E_HIP;
    return SNN_OK;
}

// Release an admitted job's slot and reservation.  Caller holds b->mu.
void batch_release(snn_batch* b, int slot)
{
    snn_batch::Job& J = b->jobs[slot];
    b->used -= J.bytes;
    b->blk_reserved -= J.nblk;
    J = snn_batch::Job();
}

}  // namespace

extern "C" {

snn_status snn_batch_create(uint64_t hbm_budget, uint64_t max_neurons, void* hip_stream, snn_batch** out)
{
    if (!out || hbm_budget == 0 || max_neurons == 0) return bfail(nullptr, SNN_E_INVAL, "bad batch arguments");
    *out = nullptr;
    snn_batch* b = new snn_batch();
    b->budget = hbm_budget;
    b->blk_cap = (uint32_t)((max_neurons + 1023) / 1024);
    hipError_t e = hipSuccess;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
    }
    for (int w = 0; w < snn_batch::kBuilders && e == hipSuccess; ++w)
        e = hipStreamCreateWithFlags(&b->build_stream[w], hipStreamNonBlocking);
    if (e == hipSuccess) e = snn::setup_kernels();
    b->dev_alloc = current_allocator();
    if (e == hipSuccess) e = dev_malloc(b->dev_alloc, (void**)&b->d_jobs, sizeof(snn::JobDesc) * snn::kMaxJobs);
    for (int i = 0; i < snn_batch::kTables && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&b->h_jobs[i], sizeof(snn::JobDesc) * snn::kMaxJobs, 0);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->h_done[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(b->mu);
        e = batch_upload(b);
    }
    if (e != hipSuccess) {
        snn_batch_destroy(b);
        return bfail(nullptr, SNN_E_HIP, std::string("batch creation failed: ") + hipGetErrorString(e));
    }
    for (int w = 0; w < snn_batch::kBuilders; ++w) b->workers[w] = std::thread(batch_worker, b, w);
    *out = b;
    return SNN_OK;
}

snn_status snn_batch_admit(snn_batch* b, const snn_grid_desc* g, const snn_syn_desc* s, uint32_t dur_ms,
                           int32_t* slot)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (!g || !s || !slot || dur_ms == 0) return bfail(b, SNN_E_INVAL, "bad job arguments");
    if (s->solver != SNN_SOLVER_STEP) return bfail(b, SNN_E_INVAL, "batches run the step solver only");
    if (s->stdp) return bfail(b, SNN_E_INVAL, "batches run networks without plasticity");
    *slot = -1;
    std::string why;
    if (!valid_grid(g, why)) return bfail(b, SNN_E_INVAL, why);
    const uint64_t N = (uint64_t)g->gx * g->gy * (g->n_exc + g->n_inh);
    const uint32_t nblk = (uint32_t)((N + 1023) / 1024);
    snn_grid_desc gd = *g;
    gd.hist_cap = (uint64_t)((double)N * dur_ms * 0.15) + 65536;   // room for a 150 Hz mean rate
    const uint64_t est = estimate_bytes(gd, *s, gd.hist_cap);
    std::lock_guard<std::mutex> lk(b->mu);
    // a job that would not fit even in an empty batch is refused for good
    if (nblk > b->blk_cap) return bfail(b, SNN_E_INVAL, "job larger than the batch's neuron capacity");
    if (est > b->budget) return bfail(b, SNN_E_INVAL, "job footprint larger than the batch's HBM budget");
    int free_slot = -1;
    for (uint32_t j = 0; j < snn::kMaxJobs; ++j)
        if (b->jobs[j].state == snn_batch::kFree) {
            free_slot = (int)j;
            break;
        }
    if (free_slot < 0) return bfail(b, SNN_E_NOMEM, "all job slots in use");
    if (b->blk_reserved + nblk > b->blk_cap) return bfail(b, SNN_E_NOMEM, "neuron capacity of the batch in use");
    if (b->used + est > b->budget) return bfail(b, SNN_E_NOMEM, "HBM budget in use");
    snn_batch::Job& J = b->jobs[free_slot];
    J.state = snn_batch::kBuilding;
    J.bytes = est;
    J.dur = dur_ms;
    J.nblk = nblk;
    J.binned = batch_binnable(*s);
    b->used += est;
    b->blk_reserved += nblk;
    b->todo.push_back(snn_batch::BuildReq{free_slot, gd, *s});
    b->cv.notify_all();
    *slot = free_slot;
    return SNN_OK;
}

snn_status snn_batch_set_option(snn_batch* b, int opt, int64_t value)
{
    snn_status st = batch_check(b);
    if (st) return st;
    std::lock_guard<std::mutex> lk(b->mu);
    switch (opt) {
    case SNN_OPT_SCATTER_BLOCKS:
        if (value < 64 || value > 4096) return bfail(b, SNN_E_INVAL, "scatter blocks out of range (64 .. 4096)");
        if ((uint32_t)value != b->scatter_blocks) {
            // the grid is part of the captured chunks: none may still be pending
            BHIPCHK(b, hipStreamSynchronize(b->stream));
            batch_drop_graphs(b);
            b->scatter_blocks = (uint32_t)value;
        }
        return SNN_OK;
    case SNN_OPT_DELIVER_MODE:
        if (value != 0 && value != 1) return bfail(b, SNN_E_INVAL, "batch delivery mode must be 0 or 1");
        b->deliver_mode = (uint32_t)value;
        break;
    case SNN_OPT_BIN_THRESHOLD_PPM:
        if (value < 0 || value > 1000000000) return bfail(b, SNN_E_INVAL, "threshold out of range");
        b->thr_ppm = (uint64_t)value;
        break;
    default:
        return bfail(b, SNN_E_INVAL, "unknown batch option");
    }
    // the running jobs' table entries change from the next chunk on (the
    // copy is ordered after the chunks already enqueued)
    BHIPCHK(b, batch_upload(b));
    return SNN_OK;
}

snn_status snn_batch_step(snn_batch* b, uint32_t chunk_ms)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (chunk_ms == 0) return SNN_OK;
    std::unique_lock<std::mutex> lk(b->mu);
    auto count = [b](snn_batch::State s) {
        uint32_t c = 0;
        for (auto& J : b->jobs) c += J.state == s ? 1u : 0u;
        return c;
    };
    // nothing to step yet but jobs under construction: wait for one of them
    if (count(snn_batch::kActive) == 0 && b->built.empty() && count(snn_batch::kBuilding) > 0)
        b->cv.wait(lk, [b] { return !b->built.empty() || b->stop; });
    BHIPCHK(b, batch_activate(b));
    bool any = false;
    for (auto& J : b->jobs) any = any || (J.state == snn_batch::kActive && J.t < J.dur);
    if (!any) return SNN_OK;
    hipGraphExec_t ex = nullptr;
    BHIPCHK(b, batch_graph(b, chunk_ms, &ex));
    BHIPCHK(b, hipGraphLaunch(ex, b->stream));
    for (auto& J : b->jobs)
        if (J.state == snn_batch::kActive) J.t = (J.t + chunk_ms < J.dur) ? J.t + chunk_ms : J.dur;
    return SNN_OK;
}

snn_status snn_batch_poll(snn_batch* b, int32_t* done, size_t cap, size_t* n_out)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (!n_out || (cap && !done)) return bfail(b, SNN_E_INVAL, "null output");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    std::lock_guard<std::mutex> lk(b->mu);
    BHIPCHK(b, batch_activate(b));
    size_t n = 0;
    for (uint32_t j = 0; j < snn::kMaxJobs; ++j) {
        const snn_batch::Job& J = b->jobs[j];
        const bool fin = (J.state == snn_batch::kActive && J.t >= J.dur) || J.state == snn_batch::kFailed;
        if (!fin) continue;
        if (n < cap) done[n] = (int32_t)j;
        ++n;
    }
    *n_out = n;
    return n > cap ? bfail(b, SNN_E_TRUNC, "slot buffer too small") : SNN_OK;
}

snn_status snn_batch_read_spikes(snn_batch* b, int32_t slot, snn_spike* buf, size_t cap, size_t* n_out)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (slot < 0 || slot >= (int32_t)snn::kMaxJobs || !n_out) return bfail(b, SNN_E_INVAL, "no job in this slot");
    std::unique_lock<std::mutex> lk(b->mu);
    snn_batch::Job& J = b->jobs[slot];
    if (J.state == snn_batch::kFailed) {
        const snn_status fs = J.fail_st;
        const std::string m = J.fail_msg;
        batch_release(b, slot);
        return bfail(b, fs, "job construction failed: " + m);
    }
    if (J.state != snn_batch::kActive) return bfail(b, SNN_E_INVAL, "no job in this slot");
    if (J.t < J.dur) return bfail(b, SNN_E_STATE, "job has not finished");
    BHIPCHK(b, hipStreamSynchronize(b->stream));   // the job's last steps are done
    Ctrl hc{};
    BHIPCHK(b, hipMemcpy(&hc, J.net->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    const bool truncated = hc.hist_n > J.net->g.hist_cap;
    const uint64_t m = truncated ? J.net->g.hist_cap : hc.hist_n;
    *n_out = (size_t)m;
    if (m > cap) return bfail(b, SNN_E_TRUNC, "spike buffer too small");
    if (m) BHIPCHK(b, hipMemcpy(buf, J.net->a.hist, m * sizeof(snn_spike), hipMemcpyDeviceToHost));
    // Entries of one step are contiguous and steps ascend.  Within a step each
    // update block (1024 neurons, gid >> 10) appended its spikers as one
    // ascending run, the blocks in arrival order: put the runs in block order.
    {
        std::vector<std::pair<uint32_t, uint64_t>> runs;   // (block, start)
        std::vector<snn_spike> tmp;
        for (uint64_t i0 = 0; i0 < m;) {
            uint64_t i1 = i0 + 1;
            while (i1 < m && buf[i1].t_ms == buf[i0].t_ms) ++i1;
            runs.clear();
            bool ordered = true;
            for (uint64_t i = i0; i < i1; ++i) {
                const uint32_t blk = buf[i].gid >> 10;
                if (i == i0 || blk != (buf[i - 1].gid >> 10)) {
                    if (!runs.empty() && blk < runs.back().first) ordered = false;
                    runs.emplace_back(blk, i);
                }
            }
            if (!ordered) {
                std::vector<std::pair<uint32_t, uint64_t>> sorted_runs(runs);
                std::sort(sorted_runs.begin(), sorted_runs.end());
                auto end_of = [&](uint64_t start) {
                    uint64_t e = start + 1;
                    while (e < i1 && (buf[e].gid >> 10) == (buf[start].gid >> 10)) ++e;
                    return e;
                };
                tmp.clear();
                for (auto& r : sorted_runs) tmp.insert(tmp.end(), buf + r.second, buf + end_of(r.second));
                std::memcpy(buf + i0, tmp.data(), tmp.size() * sizeof(snn_spike));
            }
            i0 = i1;
        }
    }
    // Leave the table, then hand the network to the worker, which frees it
    // once the stepping stream has passed this table update.
    snn_net* net = J.net;
    J.state = snn_batch::kFree;
    BHIPCHK(b, batch_upload(b));
    hipEvent_t after = nullptr;
    BHIPCHK(b, hipEventCreateWithFlags(&after, hipEventDisableTiming));
    BHIPCHK(b, hipEventRecord(after, b->stream));
    batch_release(b, slot);
    b->retired.push_back(snn_batch::Retired{net, after});
    b->cv.notify_all();
    return truncated ? bfail(b, SNN_E_TRUNC, "job history overflowed its capacity") : SNN_OK;
}

snn_status snn_batch_job_stats(snn_batch* b, int32_t slot, snn_stats_t* out)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (slot < 0 || slot >= (int32_t)snn::kMaxJobs || !out) return bfail(b, SNN_E_INVAL, "no job in this slot");
    std::lock_guard<std::mutex> lk(b->mu);
    const snn_batch::Job& J = b->jobs[slot];
    if (J.state != snn_batch::kActive) return bfail(b, SNN_E_INVAL, "no running or finished job in this slot");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    Ctrl hc{};
    BHIPCHK(b, hipMemcpy(&hc, J.net->a.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    fill_stats(J.net, hc, out);
    return SNN_OK;
}

snn_status snn_batch_read_state(snn_batch* b, int32_t slot, float* v, float* w, uint8_t* ref, int32_t* ring)
{
    snn_status st = batch_check(b);
    if (st) return st;
    if (slot < 0 || slot >= (int32_t)snn::kMaxJobs) return bfail(b, SNN_E_INVAL, "no job in this slot");
    std::lock_guard<std::mutex> lk(b->mu);
    const snn_batch::Job& J = b->jobs[slot];
    if (J.state != snn_batch::kActive) return bfail(b, SNN_E_INVAL, "no running or finished job in this slot");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const size_t N = J.net->N;
    if (v) BHIPCHK(b, hipMemcpy(v, J.net->a.V, N * 4, hipMemcpyDeviceToHost));
    if (w) BHIPCHK(b, hipMemcpy(w, J.net->a.W, N * 4, hipMemcpyDeviceToHost));
    if (ref) BHIPCHK(b, hipMemcpy(ref, J.net->a.ref, N, hipMemcpyDeviceToHost));
    if (ring) BHIPCHK(b, hipMemcpy(ring, J.net->a.ring, (size_t)snn::kRing * N * 4, hipMemcpyDeviceToHost));
    return SNN_OK;
}

snn_status snn_batch_usage(snn_batch* b, uint64_t* bytes, uint32_t* jobs)
{
    snn_status st = batch_check(b);
    if (st) return st;
    std::lock_guard<std::mutex> lk(b->mu);
    uint32_t n = 0;
    for (auto& J : b->jobs) n += J.state != snn_batch::kFree ? 1u : 0u;
    if (bytes) *bytes = b->used;
    if (jobs) *jobs = n;
    return SNN_OK;
}

void snn_batch_destroy(snn_batch* b)
{
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->stop = true;
        b->todo.clear();
    }
    b->cv.notify_all();
    for (auto& w : b->workers)
        if (w.joinable()) w.join();   // each finishes its build in progress; pending frees are drained
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    for (auto& kv : b->built)
        if (kv.second) snn_destroy(kv.second);
    for (auto& J : b->jobs)
        if (J.net) snn_destroy(J.net);
    for (auto& r : b->retired) {
        (void)hipEventDestroy(r.after);
        snn_destroy(r.net);
    }
    dev_free(b->dev_alloc, b->d_jobs);
    for (int i = 0; i < snn_batch::kTables; ++i) {
        if (b->h_jobs[i]) (void)hipHostFree(b->h_jobs[i]);
        if (b->h_done[i]) (void)hipEventDestroy(b->h_done[i]);
    }
    for (auto& bs : b->build_stream)
        if (bs) (void)hipStreamDestroy(bs);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* snn_batch_last_error(const snn_batch* b)
{
    return b ? b->err.c_str() : g_batch_err.c_str();
}

}  // extern "C"
