// snn_dev.h -- device-side data layout, kernel arguments and launchers of the
// gfx950 spiking-network library.  Included by the kernels and by the host
// runtime; contains no host-only code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

constexpr uint32_t kRing = 32;      // delay-ring slots (more than the largest delay)
constexpr uint32_t kQuadsPerBlock = 256;
constexpr uint32_t kNeuronsPerBlock = 4 * kQuadsPerBlock;  // one update block: 1024 neurons
constexpr uint32_t kGroup = 16;     // update blocks per compaction group
constexpr uint32_t kMaxPois = 64;   // Poisson CDF thresholds
constexpr uint32_t kMaxD = 31;      // delay buckets per row
// Tile-binned delivery: targets are grouped in tiles of 1024; each step's
// events are binned per tile, then accumulated in LDS tile by tile.
constexpr uint32_t kTileBits = 10;
constexpr uint32_t kTile = 1u << kTileBits;
static_assert(kTile == kNeuronsPerBlock, "a delivery tile is an update block");
constexpr uint32_t kMaxTiles = 2048;          // binned delivery needs N <= 2M neurons
constexpr uint32_t kChunkItems = 80;        // row segments (256 records) per scatter chunk: 16 waves x 5
constexpr uint32_t kStage = kChunkItems * 256;
constexpr uint32_t kWInhField = 0x1FFFFu;     // weight field that stands for the inhibitory weight
// Bin fill counters sit one per 128-byte line: every scatter workgroup reserves
// in every tile's bin each chunk, and counters sharing a line serialise there.
constexpr uint32_t kFillStride = 32;
// Two-level binning (8-bit-code networks with more tiles than one LDS table):
// the records of every row are laid out by super tile of 2^kSegBits targets
// at construction, a step lists the (spike, super tile) record segments per
// super tile, and a second pass bins each super tile's segments by tile.
constexpr uint32_t kSegBits = 19;
constexpr uint32_t kSegTiles = 1u << (kSegBits - kTileBits);   // tiles per super tile
constexpr uint32_t kMaxSuper = 32;                             // N <= 2^24 neurons

// Philox stream identifiers (third counter word).
constexpr uint32_t kStreamConn = 1u, kStreamAttr = 2u, kStreamExt = 3u, kStreamInit = 4u;
// binomial synapse generator: count per (source, module), then Floyd's draws
constexpr uint32_t kStreamCount = 5u, kStreamPick = 6u;

struct Rec8 {        // 8-byte record: target and weight in mV (an exact multiple of 2^-16)
    uint32_t tgt;    // target | delay bucket << kTgtBits
    float w;
};
// The target word of an 8-byte record also carries the synapse's delay bucket
// in its top bits (a network has fewer than 2^27 neurons: 32 N < 2^32), so a
// kernel reading the record needs no search of the row's bucket ends.
constexpr uint32_t kTgtBits = 27;
constexpr uint32_t kTgtMask = (1u << kTgtBits) - 1u;

// Device-side control block, one per network.
struct Ctrl {
    uint32_t t0;            // first step of the chunk being executed
    uint32_t nspk;          // spikes of the step in flight (written by compaction)
    uint64_t hist_n;        // spikes recorded so far
    uint64_t rec_events;    // recurrent events delivered
    uint64_t ext_events;    // external Poisson events
    uint64_t spikes;        // total spikes
    uint64_t disagree;      // lock-step threshold disagreements
    uint32_t err;           // construction error flags (bit 0: row longer than 65535)
    uint32_t max_len;       // longest projection row
    uint64_t bin_overflow;  // events delivered by the direct fallback (bin full)
    uint64_t step_ev[2];    // recurrent events of the step in flight, by step parity
    uint32_t nspk_par[2];   // batched stepping: spikes appended this step, by parity
};

// Everything the step kernels read, passed by value.
struct StepArgs {
    uint32_t N, nq, M, n_exc, sfa_on_inh;
    uint32_t nblk, ngrp, D, d_min;
    uint32_t npois, ext_const, record;
    int32_t ext_const_q, jext_q;
    uint32_t key0, key1;
    uint64_t hist_cap;
    float v_th, v_reset, e_rest, alpha, dm, dw, kappa;
    uint32_t nref;
    float* V;
    float* W;
    uint8_t* ref;
    int32_t* ring;          // [kRing][N]
    uint4* blk_stat;        // [nblk] per update block, step in flight: {spikers, their recurrent
                            //   events (sum of row lengths), external Poisson events, 0}
    uint4* blk_list;        // [nblk * kNeuronsPerBlock] spikers {gid, row length, row start}
    uint32_t* grp_cnt;      // [2][ngrp] spikers per group of kGroup blocks (direct delivery)
    uint32_t grp_atomic;    // the update maintains grp_cnt (direct delivery selected)
    uint4* spk;             // [N] spikes of the step in flight: {gid, row length, row start lo, hi}
    uint2* hist;            // [hist_cap] (t, gid)
    Ctrl* ctrl;
    const uint64_t* row_ptr;  // [N+1]
    const uint16_t* bend;     // [N][D]
    const void* recs;
    const uint32_t* poisc;    // [npois]
    const int32_t* cb;        // [256] codebook (CODE8 records)
    const uint8_t* forced;    // lock-step flags or nullptr
    // tile-binned delivery
    uint32_t ntiles;
    int32_t winh_q;
    uint32_t bin_cap_tile;    // capacity of every tile's bin (events)
    uint64_t bin_threshold;   // steps with fewer events are delivered directly
    uint32_t* bin_fill;       // [ntiles * kFillStride] events binned this step (one counter per line)
    uint32_t* bins;           // [ntiles][bin_cap_tile] event codes:
                              //   target & 1023 | bucket << 10 | weight field << 15
    // two-level binning (nsuper > 0; 8-bit-code records laid out by super
    // tile: each row's records sorted by (super tile, delay bucket, target),
    // record = target & (2^kSegBits - 1) | bucket << kSegBits | code << (kSegBits + 5))
    uint32_t nsuper;          // super tiles of 2^kSegBits targets (<= kMaxSuper)
    const uint16_t* sstart;   // [N][nsuper] start of each super tile's segment in the row
    uint32_t dcap;            // capacity of every super tile's segment list
    uint32_t* dfill;          // [nsuper * kFillStride] segments listed this step
    uint2* dsc;               // [nsuper][dcap] segments of at most 256 records:
                              //   {record index lo, record index hi | length << 8}
};

// One job of a batch: the job network's step arguments plus its schedule.
constexpr uint32_t kMaxJobs = 64;
constexpr uint32_t kBatchMaxD = 20;   // batched binned delivery: delay buckets per job at most
struct JobDesc {
    StepArgs a;
    uint32_t t_end;      // steps to simulate
    uint32_t active;     // the slot holds a job
    uint32_t blk_base;   // first batch update block (= first tile) of the job
    uint32_t smax;       // 256-record segments per spike row
    uint32_t binned;     // the job may use binned delivery (F32 records, bins, D <= kBatchMaxD)
    uint32_t pad;
};

// Arguments of the projection builder.
struct BuildArgs {
    uint32_t N, M, n_exc, gx, gy, D, d_min, record;
    uint32_t key0, key1;
    int32_t winh_q;
    uint32_t row0, nrows;      // rows built by this launch
    const uint32_t* T;         // [2][gy][gx] thresholds per torus offset (excitatory, inhibitory sources)
    const int32_t* wtab;       // [65536]
    uint16_t* bend;            // [N][D]
    uint32_t* rowlen;          // [N]
    const uint64_t* row_ptr;   // [N+1] (write-out)
    void* recs;
    uint64_t rec_cap;          // records the buffer holds
    uint32_t* slab;            // [nrows][slab_cap] hits of the slice's rows
    uint32_t slab_cap;
    Ctrl* ctrl;
    uint32_t gen;              // 0 one trial per pair, 1 binomial count + Floyd subset
    uint32_t delay_exp;        // 1: delay bucket = thresholds of dthr not above the draw
    uint32_t dthr[kMaxD];      //    (D - 1 of them); 0: mulhi(draw, D)
    const uint4* btab;         // gen 1: [2][gy][gx] {k0, len, at lo, at hi} count tables
    const uint32_t* bthr;      // gen 1: their thresholds
    uint32_t nsuper;           // > 0: write the rows laid out by super tile (8-bit codes)
    uint16_t* sstart;          //      [N][nsuper] segment starts
};

// ---- launchers (kernels.hip) ----
hipError_t launch_init(const StepArgs& a, hipStream_t s);
hipError_t launch_syn_gen(const BuildArgs& a, hipStream_t s);
hipError_t launch_syn_out(const BuildArgs& a, hipStream_t s);
// row_ptr[i] = row_ptr[0] + sum of rowlen[0 .. i) for i <= N (row_ptr[0] is
// the offset of the first row, set before); with clear, rowlen is zeroed as
// it is consumed.
hipError_t launch_scan_rows(const uint32_t* rowlen, uint64_t* row_ptr, uint64_t* tile_sums,
                            uint32_t N, hipStream_t s, bool clear = false);
// Optional per-launch timing: the launch records the kernel's start and end
// in these events (both created with timing enabled).
struct LaunchEv {
    hipEvent_t start, stop;
};
hipError_t launch_update(const StepArgs& a, uint32_t k, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_compact(const StepArgs& a, uint32_t k, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_deliver(const StepArgs& a, uint32_t k, uint32_t waves, uint32_t unroll,
                          uint32_t max_len, hipStream_t s,
                          const LaunchEv* ev = nullptr);
hipError_t launch_scatter(const StepArgs& a, uint32_t k, uint32_t max_len, uint32_t blocks,
                          hipStream_t s,
                          const LaunchEv* ev = nullptr);
// Two-level networks (a.nsuper > 0): launch_scatter lists the step's record
// segments per super tile (k_seg_emit), launch_sub bins them by tile or, in a
// step below the binning threshold, delivers them directly (k_seg_bin).
hipError_t launch_sub(const StepArgs& a, uint32_t k, uint32_t blocks, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_tile(const StepArgs& a, uint32_t k, bool update_next, hipStream_t s,
                       const LaunchEv* ev = nullptr);
hipError_t setup_kernels();
hipError_t launch_batch_update(const JobDesc* jobs, uint32_t blocks, uint32_t k, hipStream_t s);
hipError_t launch_batch_scatter(const JobDesc* jobs, uint32_t blocks, uint32_t k, hipStream_t s);
hipError_t launch_batch_tile(const JobDesc* jobs, uint32_t blocks, uint32_t k, bool update_next, hipStream_t s);
hipError_t launch_batch_advance(const JobDesc* jobs, uint32_t n, hipStream_t s);
hipError_t launch_advance(Ctrl* c, uint32_t n, hipStream_t s);
hipError_t launch_set_flags(uint8_t* flags, const uint32_t* ids, uint32_t n, uint8_t v,
                            hipStream_t s);
// p[0 .. n) = v (a kernel, so that it may be recorded in a captured graph)
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s);
uint32_t scan_tiles(uint32_t N);

}  // namespace snn
