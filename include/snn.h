/*
 * snn.h -- C ABI of the MI355X (gfx950) spiking-network hot path.
 *
 * Method: Pastorelli et al., "Gaussian and exponential lateral connectivity
 * on distributed spiking neural network simulation" (PDP 2018).  A 2-D grid
 * of cortical modules of point neurons (Sec. III.B) is simulated in 1 ms
 * time-driven steps (Sec. II.A): LIF neurons with spike-frequency adaptation
 * (Sec. III.A, Eq. (1)-(2)) are integrated, spikers are identified, and each
 * spike is fanned out through its neuron's projection (target, weight,
 * delay; Sec. II.B) into per-target delay queues.  Projections are drawn from
 * the Gaussian B*exp(-r^2/2 sigma^2) or exponential A*exp(-r/lambda) lateral
 * laws (Sec. I, Sec. III.B).
 *
 * Conventions for every call:
 *   - Status codes: SNN_OK (0) or a negative snn_status; no C++ exception
 *     crosses the ABI.  snn_last_error() gives the text of the last error.
 *   - Ownership: the library owns every device buffer it allocates (with
 *     hipMalloc, or the allocator installed by snn_set_allocator) and frees
 *     it in snn_destroy().  Host buffers passed in are owned by the caller
 *     and only read or written during the call.
 *   - Streams: all device work of a network runs on the HIP stream given to
 *     snn_build_grid (NULL = the default stream).  Calls that return host
 *     data synchronise that stream; the others only enqueue work.
 *   - Truncation: calls that fill a caller buffer of capacity `cap` return
 *     SNN_E_TRUNC when it is too small and set *n_out to the size needed.
 *   - Lifecycle: snn_step* before snn_build_synapses, or snn_build_synapses
 *     twice, returns SNN_E_STATE.  A HIP runtime error returns SNN_E_HIP and
 *     poisons the handle (every later call except destroy returns SNN_E_HIP).
 *   - Threading: one network handle is used by one host thread at a time.
 *
 * Fixed-point charge: synaptic weights and external charge are integers in
 * units of 2^-16 mV and are summed in int32 (two's-complement wrap-add, exact
 * while the per-step total of a neuron fits in int32).
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SNN_OK = 0,
    SNN_E_INVAL = -1,     /* invalid argument or description               */
    SNN_E_NOMEM = -2,     /* device or host allocation failed / over budget */
    SNN_E_HIP = -3,       /* HIP runtime error; handle is poisoned          */
    SNN_E_STATE = -4,     /* call out of order                              */
    SNN_E_OVERFLOW = -5,  /* a row longer than 65535 synapses, or similar   */
    SNN_E_TRUNC = -6      /* caller buffer too small; *n_out = size needed  */
} snn_status;

enum { SNN_GAUSS = 0, SNN_EXP = 1 };
enum { SNN_REC_F32 = 0, SNN_REC_CODE8 = 1 };
enum { SNN_EXT_POISSON = 0, SNN_EXT_CONST = 1 };
enum { SNN_PRESET_LATERAL = 0, SNN_PRESET_PAPER = 1 };
enum { SNN_GEN_PAIRWISE = 0, SNN_GEN_BINOMIAL = 1 };
enum { SNN_DELAY_UNIFORM = 0, SNN_DELAY_EXP = 1 };
enum { SNN_SOLVER_STEP = 0, SNN_SOLVER_EXACT = 1 };

typedef struct snn_net snn_net;

/* AER spike record (Sec. II.C): step index and neuron id.  Under the step
 * solver spike times are quantised to the 1 ms step; under the exact solver
 * snn_read_spike_times gives each spike's offset inside its step as well.
 * History is ordered by (t_ms, gid). */
typedef struct {
    uint32_t t_ms;
    uint32_t gid;
} snn_spike;

/* The grid of modules and its neurons (Sec. III.A-B).
 * Neuron id: gid = module * (n_exc + n_inh) + local, module = y * gx + x;
 * local < n_exc is excitatory.  Potentials in mV, times in ms. */
typedef struct {
    uint32_t gx, gy;          /* grid size in modules                           */
    uint32_t n_exc, n_inh;    /* neurons per module                             */
    uint32_t periodic;        /* must be 1: torus boundaries                    */
    double tau_m;             /* membrane time constant                         */
    double v_th;              /* threshold V_theta; a spike when V exceeds it   */
    double v_reset;           /* reset potential V_r                            */
    double e_rest;            /* resting potential E                            */
    double t_ref;             /* absolute refractory period (whole steps)       */
    double alpha_w;           /* fatigue increment per spike (mV)               */
    double tau_w;             /* fatigue decay time                             */
    uint32_t sfa_on_inh;      /* 0: inhibitory neurons have no adaptation       */
    uint32_t pad0_;
    uint64_t seed;            /* Philox4x32-10 key of every random draw         */
    uint64_t hist_cap;        /* spike-history capacity in records (0 = 1<<24)  */
} snn_grid_desc;

/* Recurrent projections and external drive (Sec. II.B, Sec. III.A-B).
 * Connection probability of a pair at torus distance r (module spacings),
 * f = exp(-r^2 / 2 range^2) (Gaussian) or exp(-r / range) (exponential):
 *   SNN_PRESET_LATERAL: p = B f(r) for every pair, B chosen so that the
 *     expected number of recurrent synapses per neuron is k_in;
 *   SNN_PRESET_PAPER (the paper's own rules, Sec. III.B and the Fig. 2
 *     caption): p = p_local inside the source's module for every source;
 *     p = amp f(r) to other modules for excitatory sources only, inside the
 *     square stencil of half-width ceil(r_c) where amp f(r_c) = p_cut
 *     (7x7 for the Gaussian, 21x21 for the exponential parameters of the
 *     paper); k_in is unused.
 * Delays are integers in [d_min, d_max] ms (Sec. II.B: uniform or
 * exponential): SNN_DELAY_UNIFORM, d = d_min + mulhi(a0, D); SNN_DELAY_EXP,
 * P(d) proportional to exp(-(d - d_min) / delay_tau), drawn as d_min plus the
 * number of CDF thresholds round(2^32 F(k)), k < D - 1, not above a0 (a0 the
 * first word of the pair's ATTR draw).  Excitatory weights Gaussian (w_exc,
 * w_exc_sd), inhibitory weight w_inh.
 * Generator: SNN_GEN_PAIRWISE draws one Bernoulli trial per ordered pair
 * (Philox stream 1); SNN_GEN_BINOMIAL draws, per source and target module,
 * the number of synapses from Binomial(n, p) by integer CDF thresholds
 * (stream 5) and then which n candidates by Floyd's algorithm (stream 6) --
 * the same law with different bits, in work proportional to modules and
 * synapses instead of pairs (modules of at most 4096 neurons).
 * Solver: SNN_SOLVER_STEP sums each neuron's inputs per 1 ms step and
 * applies them as one jump before the threshold test (spike times are whole
 * steps).  SNN_SOLVER_EXACT is the event-driven solver of Sec. II.A / II.C:
 * times are 32.32 fixed-point ms; a spike is emitted at the instant of the
 * input that takes V above V_th and reaches each target the synapse's delay
 * later, keeping its offset inside the step; a step's external inputs (the
 * same Poisson count) arrive at offsets drawn from Philox stream 7, counter
 * (gid, t, 7, k / 4), word k % 4 (the constant drive at offset 0); inputs of
 * one instant are summed before the threshold test; Eq. (1)-(2) are solved
 * exactly between inputs; a spike at s holds V at V_r over [s, s + t_ref),
 * discarding inputs there (t_ref >= 1 ms).  The exact solver delivers through
 * its own per-slot input queues (SNN_OPT_QUEUE_CAP), not the delay ring, is
 * not available to batches and takes at most 2^24 neurons (SNN_E_INVAL from
 * snn_build_synapses above that). */
typedef struct {
    uint32_t kernel;          /* SNN_GAUSS or SNN_EXP                           */
    uint32_t record;          /* SNN_REC_F32 (8 B) or SNN_REC_CODE8 (4 B)       */
    double range;             /* sigma or lambda, in module spacings            */
    double k_in;              /* expected recurrent in-degree (0 = none)        */
    uint32_t d_min, d_max;    /* 1 <= d_min <= d_max <= 31                      */
    double w_exc, w_exc_sd, w_inh;
    uint32_t ext_mode;        /* SNN_EXT_POISSON or SNN_EXT_CONST              */
    int32_t ext_const_q;      /* const mode: charge per neuron and step, 2^-16 mV */
    double ext_n;             /* number of external synapses per neuron          */
    double ext_rate_hz;       /* their Poisson rate                              */
    double ext_w;             /* their weight (mV)                               */
    uint32_t preset;          /* SNN_PRESET_LATERAL or SNN_PRESET_PAPER          */
    uint32_t pad1_;
    double p_local;           /* paper preset: probability inside a module, [0, 1) */
    double amp;               /* paper preset: remote amplitude A, [0, 1)         */
    double p_cut;             /* paper preset: stencil cut-off probability, > 0   */
    uint32_t gen;             /* SNN_GEN_PAIRWISE or SNN_GEN_BINOMIAL            */
    uint32_t delay_dist;      /* SNN_DELAY_UNIFORM or SNN_DELAY_EXP              */
    double delay_tau;         /* exponential delays: scale in ms, > 0            */
    uint32_t solver;          /* SNN_SOLVER_STEP or SNN_SOLVER_EXACT              */
    uint32_t pad2_;
    /* Spike-timing plasticity (stdp = 1; F32 records, step solver, no
     * batches).  Synapses of excitatory sources only.  A synapse of delay d
     * sees a presynaptic event at every arrival a = s + d of a spike of its
     * source at step s, and a postsynaptic event at every spike of its target
     * at step p.  Each pair within the window changes the weight by
     * kp[p - a] = round(a_plus e^{-(p-a)/tau_plus} 2^16) when p >= a, and by
     * -km[a - p] = -round(a_minus e^{-(a-p)/tau_minus} 2^16) when p < a
     * (2^-16 mV; the window ends at the first lag where both round to zero,
     * at most 255 steps).  A pair counts in the period of its later event;
     * at the end of every ltp_period steps a synapse whose total is not
     * zero takes weight + total, clipped to [0, w_max]; spikes use the
     * weight in force when they are emitted.  The spikes come from the AER
     * history, which must hold the period and the window before it
     * (hist_cap): an overflow is reported as SNN_E_OVERFLOW. */
    uint32_t stdp;            /* 0 off, 1 on                                      */
    uint32_t ltp_period;      /* steps between long-term applications (1000 = 1 s) */
    double a_plus, a_minus;   /* pair amplitudes at zero lag (mV), >= 0           */
    double tau_plus, tau_minus; /* window time constants (ms), > 0                */
    double w_max;             /* weight bound (mV), in (0, 65534 / 65536]          */
} snn_syn_desc;

typedef struct {
    uint64_t t;               /* steps simulated so far                          */
    uint64_t spikes;          /* total spikes                                    */
    uint64_t rec_events;      /* recurrent synaptic events delivered             */
    uint64_t ext_events;      /* external (Poisson) events                       */
    uint64_t nnz;             /* recurrent synapses                              */
    uint64_t n_neurons;
    uint64_t bytes_device;    /* device memory held by the network               */
    uint64_t hist_n;          /* spikes recorded (may exceed hist_cap)           */
    uint64_t disagree;        /* lock-step: own threshold test != forced set     */
    uint64_t bin_overflow;    /* binned delivery: events that took the fallback  */
    uint32_t deliver_mode;    /* delivery schedule in use (SNN_OPT_DELIVER_MODE) */
    uint32_t binned_ok;       /* bit 0: single-level binned delivery possible;
                                 bit 1: two-level binned delivery built (rows
                                 laid out by super tile)                       */
    uint64_t bin_threshold;   /* per-step switch to direct delivery (events)     */
    double build_ms;          /* wall time of snn_build_synapses                 */
} snn_stats_t;

/* Per-launch average durations in ms, each launch stamped by its own start
 * and stop events on the network's stream.  With binned delivery the update
 * of the next step runs inside the tile kernel (update_ms is then the first
 * step's own update launch only). */
typedef struct {
    double update_ms;         /* neuron update launch                            */
    double compact_ms;        /* ordered spike compaction launch (direct and
                                 two-level delivery)                             */
    double deliver_ms;        /* projection fan-out into the delay ring (all phases) */
    double scatter_ms;        /* binned delivery: compaction (single level) and
                                 events binned by tile or super tile            */
    double tile_ms;           /* binned delivery: per-tile LDS accumulation and
                                 the next step's update                          */
    double step_ms;           /* sum of all launches per step                    */
    uint64_t steps;
    uint64_t rec_events;      /* recurrent events delivered in the timed steps   */
    uint64_t spikes;
    double sub_ms;            /* two-level binning: super-tile bins split by tile */
} snn_kernel_times;

/* Tuning knobs (snn_set_option). */
enum {
    SNN_OPT_GRAPH_CHUNK = 1,     /* steps per captured HIP graph (0 = no graph)   */
    SNN_OPT_DELIVER_WAVES = 2,   /* waves in the fan-out grid                      */
    SNN_OPT_DELIVER_UNROLL = 3,  /* direct delivery: records in flight per lane: 1, 2, 4 */
    SNN_OPT_DELIVER_MODE = 4,    /* 0: direct ring atomics; 1: tile-binned (default
                                    when the network allows it, see snn_stats);
                                    2: two-level tile-binned (8-bit-code records;
                                    default when the tiles exceed one level; the
                                    rows are then laid out by super tile of 2^19
                                    targets, and mode 0 is the two-level kernels'
                                    direct branch at every step).
                                    Before snn_build_synapses it selects which bins
                                    are allocated; afterwards it switches between
                                    direct delivery and the mode built for.     */
    SNN_OPT_SCATTER_BLOCKS = 5,  /* workgroups of the binned scatter phase          */
    SNN_OPT_BIN_FRAC_PPM = 6,    /* before snn_build_synapses: bin capacity per tile
                                    as a fraction (ppm) of its expected in-synapses;
                                    events beyond it take the direct path           */
    SNN_OPT_BIN_THRESHOLD = 7,   /* binned schedule: steps with fewer recurrent
                                    events than this are delivered directly
                                    (0 = always binned)                             */
    SNN_OPT_EXT_RATE_UHZ = 8,    /* after snn_build_synapses: external Poisson rate
                                    in micro-hertz (rebuilds the CDF thresholds)    */
    SNN_OPT_QUEUE_CAP = 9,       /* before snn_build_synapses, exact solver: inputs
                                    one arrival slot holds (0 = automatic: a step's
                                    events at a 150 Hz mean rate + 65536); inputs
                                    beyond it are dropped and reported as
                                    SNN_E_OVERFLOW by the reads and snn_stats       */
    SNN_OPT_BIN_THRESHOLD_PPM = 10 /* batches only (snn_batch_set_option): a binned
                                    job's steps with fewer recurrent events than
                                    value * 1e-6 * neurons * delay rows are
                                    delivered directly (0 = each job's own
                                    threshold, 0.039 * neurons * delay rows)      */
};

/* Create the grid (Sec. III.B) and the initial neuron state: V uniform in
 * [E, V_th) from the INIT stream, no fatigue, not refractory, empty delay
 * queues, t = 0.  hip_stream: a hipStream_t owned by the caller, or NULL. */
snn_status snn_build_grid(const snn_grid_desc* g, void* hip_stream, snn_net** out);

/* Draw every projection on the device (Sec. II.B): for each ordered pair
 * i != j one Bernoulli trial against the 32-bit threshold of their torus
 * offset, then delay and weight from a second draw.  Rows are stored ordered
 * by (delay, target).  Blocks until construction has finished. */
snn_status snn_build_synapses(snn_net* net, const snn_syn_desc* s);

/* Enqueue n_ms 1 ms steps (Sec. II.A) on the network's stream. */
snn_status snn_step(snn_net* net, uint32_t n_ms);

/* One step in lock-step mode: the spike set of this step is gids[0..n)
 * (host array, any order) instead of each neuron's own threshold test; the
 * threshold test is still evaluated and disagreements are counted.  Step
 * solver only (SNN_E_STATE under the exact solver). */
snn_status snn_step_forced(snn_net* net, const uint32_t* gids, size_t n);

/* snn_step_forced without device allocation, for callers that cannot
 * allocate device memory (code running under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * synchronisation as snn_step_forced; the forced ids and per-neuron forced
 * flags are staged in a library-owned static device array (20 MiB per device,
 * held until the process ends) instead of the network's buffers, so the call
 * allocates nothing.  Limits: at most 2^20 ids per call and networks of at
 * most 2^24 neurons (SNN_E_INVAL beyond them, before any device work).  The
 * array is shared by every call on one device and keeps the last call's
 * contents (each call clears its own range first): calls that overlap on one
 * device, from several threads or streams, race and must not be issued.
 * Call with the network's device current, as every call. */
snn_status snn_step_forced_noalloc(snn_net* net, const uint32_t* gids, size_t n);

/* Exact solver, lock-step mode (Sec. II.C): neuron gids[k] spikes this step
 * at offset frac[k] (2^-32 ms) -- at its input of that instant, if it is not
 * refractory then -- and no other neuron spikes; each neuron's own threshold
 * test is still evaluated and disagreements are counted.  Host arrays of n
 * entries, each id at most once.  Synchronises.  SNN_E_STATE under the step
 * solver. */
snn_status snn_step_forced_exact(snn_net* net, const uint32_t* gids, const uint32_t* frac, size_t n);

/* Copy recorded spikes with t0_ms <= t_ms < t1_ms, ordered by (t_ms, gid),
 * into host_buf.  Synchronises.  SNN_E_TRUNC when more than cap match, or
 * when the history itself overflowed (then *n_out is what was kept). */
snn_status snn_read_spikes(snn_net* net, uint64_t t0_ms, uint64_t t1_ms,
                           snn_spike* host_buf, size_t cap, size_t* n_out);

/* Exact solver: snn_read_spikes plus each spike's emission offset inside
 * its step, frac[i] in 2^-32 ms for host_buf[i] (both cap entries).
 * SNN_E_STATE under the step solver. */
snn_status snn_read_spike_times(snn_net* net, uint64_t t0_ms, uint64_t t1_ms, snn_spike* host_buf,
                                uint32_t* frac, size_t cap, size_t* n_out);

/* Exact solver: the inputs queued to arrive k steps after the last step taken
 * (0 <= k <= d_max), unordered: target, offset (2^-32 ms), charge (2^-16 mV),
 * host arrays of cap entries; *n_out = their number (SNN_E_TRUNC above cap).
 * Synchronises.  SNN_E_STATE under the step solver. */
snn_status snn_read_queue(snn_net* net, uint32_t k, uint32_t* tgt, uint32_t* frac, int32_t* wq,
                          size_t cap, size_t* n_out);

/* Copy the neuron state to host arrays of n_neurons entries each (any may be
 * NULL): membrane potential, fatigue (mV), refractory steps left (exact
 * solver: whole steps until the refractory period ends, rounded up). */
snn_status snn_read_state(snn_net* net, float* v, float* w, uint8_t* ref);

/* Copy the delay ring, int32 [32][n_neurons], slot = arrival step mod 32. */
snn_status snn_read_ring(snn_net* net, int32_t* host_ring);

/* Copy rows pre0 .. pre0+n-1 of the projection table to host memory:
 * row_len[n] (u64), bucket ends bend[n][d_max-d_min+1] (u16, row-relative end
 * of each delay), and the records back to back in rec_buf (8 B
 * {u32 target, f32 weight mV} for SNN_REC_F32; 4 B (target << 8 | code) for
 * SNN_REC_CODE8), each row in (delay, target) order: rows that two-level
 * delivery holds laid out by super tile are converted back on the host.
 * rec_cap is in records; *n_out = records in the range. */
snn_status snn_export_rows(snn_net* net, uint32_t pre0, uint32_t n, uint64_t* row_len,
                           uint16_t* bend, void* rec_buf, size_t rec_cap, size_t* n_out);

/* Counters (synchronises). */
snn_status snn_stats(snn_net* net, snn_stats_t* out);

/* Run n_ms steps launching each kernel separately between HIP events on the
 * network's stream and report average kernel durations.  The steps are real
 * simulation steps (state advances).  Exact solver: update_ms is the neuron
 * update, scatter_ms the ordering of the arriving inputs by target (from the
 * first of its kernels' start to the last one's end), deliver_ms the fan-out
 * into the input queues, step_ms a whole step. */
snn_status snn_time_kernels(snn_net* net, uint32_t n_ms, snn_kernel_times* out);

/* Return the network to its initial state (as after snn_build_grid: V from the
 * INIT stream, no fatigue, not refractory, empty ring, t = 0, empty history,
 * zero counters); projections are kept.  Enqueued on the network's stream. */
snn_status snn_reset(snn_net* net);

/* Set a tuning knob (SNN_OPT_*).  Takes effect on the next step call. */
snn_status snn_set_option(snn_net* net, int key, int64_t value);

/* Host-only (no device work): the integer tables the library derives from a
 * description, for inspection and tests.  T[2][gy*gx] connection thresholds
 * round(p 2^32) for excitatory (first half) and inhibitory sources, indexed
 * by torus offset (dy mod gy) * gx + (dx mod gx);
 * wtab[65536] excitatory weights by the top 16 bits of the weight draw;
 * cb[256] the 8-bit codebook; poisc[64] Poisson CDF thresholds (*npois
 * used); consts[3] = {1 - exp(-1/tau_m), 1 - exp(-1/tau_w), kappa} of the
 * one-step propagator.  Any output may be NULL. */
snn_status snn_host_tables(const snn_grid_desc* g, const snn_syn_desc* s, uint32_t* T, int32_t* wtab,
                           int32_t* cb, uint32_t* poisc, uint32_t* npois, double* consts);

/* Host-only: the plasticity tables of a description with stdp = 1: kp and km
 * (win entries each, km[0] = 0; capacity 256), *win, and w_max in 2^-16 mV.
 * Any output may be NULL. */
snn_status snn_host_stdp_tables(const snn_grid_desc* g, const snn_syn_desc* s, int32_t* kp, int32_t* km,
                                uint32_t* win, int32_t* wmax_q);

/* Measurement aid, not part of the method: the rate of scattered
 * device-scope int32 atomic adds (the unit of direct delivery) on this GPU.
 * n_adds adds go to hashed words of a buffer of n_targets int32 (allocated
 * and freed by the call); one untimed launch, then one timed with HIP events
 * on hip_stream (NULL = default).  *adds_per_s receives the rate.
 * Synchronises.  SNN_E_INVAL for zero sizes, SNN_E_NOMEM when the buffer
 * cannot be allocated, SNN_E_HIP on a runtime error. */
snn_status snn_probe_atomics(uint64_t n_targets, uint64_t n_adds, void* hip_stream, double* adds_per_s);

/* Free every device buffer of the network (synchronises its stream). */
void snn_destroy(snn_net* net);

/* ---- Batched / served stepping of many networks ("jobs") ----------------
 * A batch advances every admitted job by the same number of steps with one
 * launch per phase for all jobs together (multi-job kernels over a device job
 * table, replayed as HIP graphs), so many small networks share the GPU.  Each
 * job is an ordinary network (same definitions, same results as stepping it
 * alone).  Jobs are built by the batch's two construction threads, each on
 * its own stream, so construction overlaps with the steps of the jobs already
 * running; a job joins the table at the first snn_batch_step after its build
 * has finished and stops at its own duration.  Jobs with F32 records,
 * d_min = 1 and at most 20 delay buckets use the binned delivery (per step,
 * above the same event threshold as a single network); the others direct
 * delivery.  The calls are meant for one controlling thread; the batch's own
 * construction threads are synchronised internally. */
typedef struct snn_batch snn_batch;

/* hbm_budget: device bytes the batch may hold for its jobs (admission
 * control); max_neurons: total neurons of jobs admitted at once (sizes the
 * update grid); hip_stream: stepping stream (NULL = own stream).  Starts the
 * construction threads. */
snn_status snn_batch_create(uint64_t hbm_budget, uint64_t max_neurons, void* hip_stream, snn_batch** out);

/* Admit a job of dur_ms steps: checks the footprint estimate (including a
 * spike history with room for a 150 Hz mean rate) against the free budget,
 * reserves a slot, the estimated bytes and the job's update blocks, and queues
 * the build; returns at once with the job's slot in *slot.  SNN_E_NOMEM: not
 * now (budget, neurons or all 64 slots in use by other jobs); SNN_E_INVAL: bad
 * description, or a job that could never be admitted (more neurons than
 * max_neurons, or a footprint estimate above hbm_budget).
 * A build that fails later is reported by snn_batch_poll as a finished slot
 * whose snn_batch_read_spikes returns the build's error and frees the slot. */
snn_status snn_batch_admit(snn_batch* b, const snn_grid_desc* g, const snn_syn_desc* s, uint32_t dur_ms,
                           int32_t* slot);

/* Enqueue chunk_ms steps for every running, unfinished job (jobs whose build
 * has finished join first).  With no running job but builds in progress it
 * waits for a build to finish; with nothing to run it returns at once. */
snn_status snn_batch_step(snn_batch* b, uint32_t chunk_ms);

/* Set a knob of the batched schedule (what the batch autotuner chooses; the
 * results do not depend on it: integer delivery is order-free):
 *   SNN_OPT_SCATTER_BLOCKS     workgroups of the batched scatter kernel,
 *                              64 .. 4096 (waits for the enqueued steps and
 *                              drops the captured chunks);
 *   SNN_OPT_DELIVER_MODE       0: every job by direct ring atomics; 1: tile-
 *                              binned for the jobs that allow it (default);
 *   SNN_OPT_BIN_THRESHOLD_PPM  see the enum above.
 * The running jobs take the change from the next snn_batch_step on.
 * SNN_E_INVAL for an unknown option or a value out of range. */
snn_status snn_batch_set_option(snn_batch* b, int opt, int64_t value);

/* Finished jobs (and failed builds) whose spikes have not been read yet
 * (synchronises the stepping stream). */
snn_status snn_batch_poll(snn_batch* b, int32_t* done_slots, size_t cap, size_t* n_out);

/* Copy a finished job's whole spike history, ordered by (t_ms, gid), then
 * free its slot; its device memory is released by a construction thread
 * once the stepping stream has passed the job's removal from the table.
 * SNN_E_STATE if the job has not finished; SNN_E_TRUNC (slot kept) if cap is
 * too small, *n_out = count needed. */
snn_status snn_batch_read_spikes(snn_batch* b, int32_t slot, snn_spike* host_buf, size_t cap, size_t* n_out);

/* Counters of one running or finished job (synchronises the stepping
 * stream). */
snn_status snn_batch_job_stats(snn_batch* b, int32_t slot, snn_stats_t* out);

/* Parity hook: copy a running or finished job's neuron state and delay ring
 * to host arrays (any may be NULL): v, w (n_neurons floats, mV), ref
 * (n_neurons bytes, refractory steps left), ring (int32 [32][n_neurons],
 * slot = arrival step mod 32), as snn_read_state / snn_read_ring give them
 * for a network stepped alone.  A finished job keeps its state until its
 * spikes are read.  Synchronises the stepping stream. */
snn_status snn_batch_read_state(snn_batch* b, int32_t slot, float* v, float* w, uint8_t* ref, int32_t* ring);

/* Device bytes held or reserved by the batch's jobs; number of admitted jobs
 * (building, running or finished and unread). */
snn_status snn_batch_usage(snn_batch* b, uint64_t* bytes, uint32_t* jobs);

/* Stops the construction threads (pending builds are dropped), waits for the
 * stepping stream and frees every job. */
void snn_batch_destroy(snn_batch* b);
const char* snn_batch_last_error(const snn_batch* b);

/* Text of the last error of this handle (or of the last failed create when
 * net is NULL).  Valid until the next call on the handle. */
const char* snn_last_error(const snn_net* net);

/* Route the library's device allocations through the caller's allocator (for
 * example a framework's caching allocator), so that networks share its pool
 * instead of holding hipMalloc blocks of their own.  Process-wide.
 *   alloc(bytes, ctx): return device memory of the current device, aligned to
 *     256 bytes, or NULL.  A NULL or misaligned result fails the call that
 *     allocated with SNN_E_NOMEM (a misaligned block is handed back first).
 *   free_(ptr, ctx): take back a block alloc returned.  The library calls it
 *     only after the stream that used the block has finished with it.
 *   ctx: passed through untouched; owned by the caller.
 * Both NULL restores hipMalloc / hipFree; exactly one NULL is SNN_E_INVAL.
 * Each network (snn_build_grid) and each batch (snn_batch_create, and the
 * networks it builds for its jobs) takes the allocator in force when it is
 * created and releases its buffers through the same pair, so the pair and ctx
 * must stay valid until every such handle is destroyed.  Either function may
 * be called from the library's construction threads.  Memory from the
 * allocator need not be zeroed: the library clears what it reads before
 * writing it. */
snn_status snn_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SNN_H */
