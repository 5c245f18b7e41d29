// exact_dev.h -- the exact-time event-driven solver (Sec. II.A, Sec. II.C):
// device layout, kernel arguments and launchers.
//
// Times are ms in 32.32 fixed point, (step << 32) | offset.  A spike is
// emitted at the instant of the input that takes V above V_th and reaches each
// target an integer delay later, keeping its offset.  Per arrival slot the
// queued inputs are held twice: as an unsorted list appended by delivery
// (one 16-byte {target, offset, charge} entry per event), and, at the step
// they arrive, counting-sorted by target into {offset, charge} pairs.  The
// update takes each neuron's inputs, with its external ones, in time order
// and integrates Eq. (1)-(2) exactly between them.
#pragma once
#include "snn_dev.h"

namespace snn {

constexpr uint32_t kStreamExtTime = 7u;   // offsets of the external inputs of a step
constexpr uint32_t kXBlock = 256;          // neurons per update workgroup
constexpr uint32_t kXLocal = 16;           // inputs per neuron sorted in LDS (more: slow path)
constexpr uint32_t kXBusyPer = 8;          // a workgroup averaging more inputs per neuron is busy
constexpr uint32_t kXWaveSort = 1024;      // most inputs of a neuron a busy workgroup's wave takes together
constexpr uint32_t kXGroups = 4096;        // most target groups of the arrival sort
constexpr uint32_t kXGroupBitsMax = 12;    // neurons per target group: at most 2^12
constexpr uint64_t kXChunkMin = 1024;      // fewest inputs per workgroup of the arrival sort's chunk passes

struct XArgs {
    uint32_t N, M, n_exc, sfa_on_inh;
    uint32_t D, d_min, R, record;          // R: arrival slots (d_max + 1)
    uint32_t npois, ext_const;
    int32_t ext_const_q, jext_q;
    uint32_t key0, key1;
    uint32_t nblk;                         // update workgroups (kXBlock neurons each)
    uint32_t smax;                         // 256-record segments of the longest row
    uint32_t tau_equal;                    // tau_w == tau_m
    uint64_t hist_cap;
    uint64_t qcap;                         // queued inputs per slot
    uint64_t tref_q;                       // refractory period, 2^-32 ms
    float v_th, v_reset, e_rest, alpha;
    float inv_tau_m, inv_tau_w, ck;        // ck = tau_w / (tau_w - tau_m)
    double dinv_tau_m, dinv_tau_w, dck;    // the same in double (closed-form update of busy workgroups)
    double dv_th, dv_reset, de_rest, dalpha;
    float* V;
    float* W;
    uint64_t* rend;                        // [N] end of the refractory period
    uint32_t* fs;                          // [N] offset of the neuron's last spike
    uint4* qlist;                          // [R][qcap] {target, offset, charge, 0}, in delivery order
    unsigned long long* qn;                // [R] entries appended per slot (may exceed qcap)
    uint32_t* xpref;                       // [N][D] each spike's bucket lengths, then its place in each bucket's slot
    unsigned long long* qn_prev;           // [R] the same before the step's delivery
    unsigned long long* dropped;           // inputs that found their slot full
    uint64_t* qoff;                        // [N + 1] start of each target's inputs of this step in qsorted
    uint2* qsorted;                        // [qcap] {offset, charge} by target
    // arrival sort: targets in groups of 2^gbits neurons (ngroups <= kXGroups)
    uint32_t gbits, ngroups;
    uint32_t* gcnt;                        // [ngroups] inputs per group (zero between steps)
    uint64_t* goff;                        // [ngroups + 1] start of each group's inputs
    unsigned long long* gcur;              // [ngroups] fill cursors
    uint4* qtmp;                           // [qcap] the arriving inputs by group
    uint32_t* blk_cnt;                     // [nblk] spikers per update workgroup
    uint32_t* blk_ext;                     // [nblk] external Poisson events per update workgroup
    uint32_t* blk_list;                    // [nblk * kXBlock] their ids, ascending
    uint64_t* blk_off;                     // [nblk + 1] exclusive scan of blk_cnt
    uint4* spk;                            // [N] spikes of the step: {gid, offset, row start lo, hi}
    uint2* hist;                           // [hist_cap] (t, gid)
    uint32_t* hist_f;                      // [hist_cap] emission offsets
    Ctrl* ctrl;                            // counters shared with the step solver's reads
    const uint64_t* row_ptr;
    const uint16_t* bend;
    const void* recs;
    const uint32_t* poisc;
    const int32_t* cb;
    const uint8_t* forced;                 // lock-step: spike flags, or nullptr
    const uint32_t* forced_f;              //            and their offsets
};

// One step of the solver, the step index t read from ctrl->t0 on the device
// (so that a captured sequence of steps can be replayed): order the arriving
// slot's inputs by target (a counting sort by target group, then by neuron
// within each group, which also gives qoff), update every neuron, list the
// spikes (with their history entries), deliver them, and close the step
// (t0 + 1).
hipError_t launch_x_place(const XArgs& a, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_x_update(const XArgs& a, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_x_list(const XArgs& a, hipStream_t s);
hipError_t launch_x_deliver(const XArgs& a, hipStream_t s, const LaunchEv* ev = nullptr);
hipError_t launch_x_finish(const XArgs& a, hipStream_t s);

}  // namespace snn
