"""Thin ctypes binding of the gfx950 library (include/snn.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libsnn.so.  PyTorch is imported first so that the process uses one HIP runtime
(torch's) and so that callers can hand in a torch stream; the library owns its
device memory, which it takes from hipMalloc or from an allocator installed with
set_allocator (use_torch_allocator: torch's caching allocator).  There is no CPU fallback: if libsnn.so is missing this module
raises on import of the library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsnn.so")

SNN_OK, SNN_E_INVAL, SNN_E_NOMEM, SNN_E_HIP, SNN_E_STATE, SNN_E_OVERFLOW, SNN_E_TRUNC = 0, -1, -2, -3, -4, -5, -6
OPT_GRAPH_CHUNK, OPT_DELIVER_WAVES, OPT_DELIVER_UNROLL, OPT_DELIVER_MODE, OPT_SCATTER_BLOCKS = 1, 2, 3, 4, 5
OPT_BIN_FRAC_PPM = 6
OPT_BIN_THRESHOLD = 7
OPT_EXT_RATE_UHZ = 8
OPT_QUEUE_CAP = 9
OPT_BIN_THRESHOLD_PPM = 10
SOLVER_STEP, SOLVER_EXACT = 0, 1
RING = 32

EXPORTS = [
    "snn_build_grid", "snn_build_synapses", "snn_step", "snn_step_forced", "snn_read_spikes",
    "snn_read_state", "snn_read_ring", "snn_export_rows", "snn_stats", "snn_time_kernels",
    "snn_set_option", "snn_host_tables", "snn_reset", "snn_destroy", "snn_last_error",
    "snn_batch_create", "snn_batch_admit", "snn_batch_step", "snn_batch_poll", "snn_batch_read_spikes",
    "snn_batch_job_stats", "snn_batch_usage", "snn_batch_destroy", "snn_batch_last_error",
    "snn_set_allocator", "snn_step_forced_exact", "snn_read_spike_times", "snn_read_queue",
    "snn_batch_read_state", "snn_step_forced_noalloc", "snn_host_stdp_tables", "snn_probe_atomics",
    "snn_batch_set_option",
]

# snn_set_allocator's function types: alloc(bytes, ctx) -> pointer, free(ptr, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class GridDesc(C.Structure):
    _fields_ = [
        ("gx", C.c_uint32), ("gy", C.c_uint32), ("n_exc", C.c_uint32), ("n_inh", C.c_uint32),
        ("periodic", C.c_uint32),
        ("tau_m", C.c_double), ("v_th", C.c_double), ("v_reset", C.c_double), ("e_rest", C.c_double),
        ("t_ref", C.c_double), ("alpha_w", C.c_double), ("tau_w", C.c_double),
        ("sfa_on_inh", C.c_uint32), ("pad0_", C.c_uint32),
        ("seed", C.c_uint64), ("hist_cap", C.c_uint64),
    ]


class SynDesc(C.Structure):
    _fields_ = [
        ("kernel", C.c_uint32), ("record", C.c_uint32),
        ("range", C.c_double), ("k_in", C.c_double),
        ("d_min", C.c_uint32), ("d_max", C.c_uint32),
        ("w_exc", C.c_double), ("w_exc_sd", C.c_double), ("w_inh", C.c_double),
        ("ext_mode", C.c_uint32), ("ext_const_q", C.c_int32),
        ("ext_n", C.c_double), ("ext_rate_hz", C.c_double), ("ext_w", C.c_double),
        ("preset", C.c_uint32), ("pad1_", C.c_uint32),
        ("p_local", C.c_double), ("amp", C.c_double), ("p_cut", C.c_double),
        ("gen", C.c_uint32), ("delay_dist", C.c_uint32), ("delay_tau", C.c_double),
        ("solver", C.c_uint32), ("pad2_", C.c_uint32),
        ("stdp", C.c_uint32), ("ltp_period", C.c_uint32),
        ("a_plus", C.c_double), ("a_minus", C.c_double),
        ("tau_plus", C.c_double), ("tau_minus", C.c_double), ("w_max", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("t", C.c_uint64), ("spikes", C.c_uint64), ("rec_events", C.c_uint64),
        ("ext_events", C.c_uint64), ("nnz", C.c_uint64), ("n_neurons", C.c_uint64),
        ("bytes_device", C.c_uint64), ("hist_n", C.c_uint64), ("disagree", C.c_uint64),
        ("bin_overflow", C.c_uint64), ("deliver_mode", C.c_uint32), ("binned_ok", C.c_uint32),
        ("bin_threshold", C.c_uint64),
        ("build_ms", C.c_double),
    ]


class KernelTimes(C.Structure):
    _fields_ = [
        ("update_ms", C.c_double), ("compact_ms", C.c_double), ("deliver_ms", C.c_double),
        ("scatter_ms", C.c_double), ("tile_ms", C.c_double), ("step_ms", C.c_double), ("steps", C.c_uint64), ("rec_events", C.c_uint64),
        ("spikes", C.c_uint64), ("sub_ms", C.c_double),
    ]


class SNNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"snn status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libsnn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1803_08833_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, U32, U64, SZ = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
        sig = {
            "snn_build_grid": ([C.POINTER(GridDesc), P, C.POINTER(P)], C.c_int),
            "snn_build_synapses": ([P, C.POINTER(SynDesc)], C.c_int),
            "snn_step": ([P, U32], C.c_int),
            "snn_step_forced": ([P, P, SZ], C.c_int),
            "snn_step_forced_noalloc": ([P, P, SZ], C.c_int),
            "snn_read_spikes": ([P, U64, U64, P, SZ, C.POINTER(SZ)], C.c_int),
            "snn_read_state": ([P, P, P, P], C.c_int),
            "snn_read_ring": ([P, P], C.c_int),
            "snn_export_rows": ([P, U32, U32, P, P, P, SZ, C.POINTER(SZ)], C.c_int),
            "snn_stats": ([P, C.POINTER(Stats)], C.c_int),
            "snn_time_kernels": ([P, U32, C.POINTER(KernelTimes)], C.c_int),
            "snn_set_option": ([P, C.c_int, C.c_int64], C.c_int),
            "snn_host_tables": ([C.POINTER(GridDesc), C.POINTER(SynDesc), P, P, P, P, P, P], C.c_int),
            "snn_reset": ([P], C.c_int),
            "snn_batch_create": ([U64, U64, P, C.POINTER(P)], C.c_int),
            "snn_batch_admit": ([P, C.POINTER(GridDesc), C.POINTER(SynDesc), U32, C.POINTER(C.c_int32)], C.c_int),
            "snn_batch_step": ([P, U32], C.c_int),
            "snn_batch_set_option": ([P, C.c_int, C.c_int64], C.c_int),
            "snn_batch_poll": ([P, P, SZ, C.POINTER(SZ)], C.c_int),
            "snn_batch_read_spikes": ([P, C.c_int32, P, SZ, C.POINTER(SZ)], C.c_int),
            "snn_batch_job_stats": ([P, C.c_int32, C.POINTER(Stats)], C.c_int),
            "snn_batch_usage": ([P, C.POINTER(U64), C.POINTER(U32)], C.c_int),
            "snn_batch_read_state": ([P, C.c_int32, P, P, P, P], C.c_int),
            "snn_host_stdp_tables": ([C.POINTER(GridDesc), C.POINTER(SynDesc), P, P, P, P], C.c_int),
            "snn_probe_atomics": ([U64, U64, P, C.POINTER(C.c_double)], C.c_int),
            "snn_batch_destroy": ([P], None),
            "snn_batch_last_error": ([P], C.c_char_p),
            "snn_destroy": ([P], None),
            "snn_last_error": ([P], C.c_char_p),
            "snn_set_allocator": ([ALLOC_FN, FREE_FN, P], C.c_int),
            "snn_step_forced_exact": ([P, P, P, SZ], C.c_int),
            "snn_read_spike_times": ([P, U64, U64, P, P, SZ, C.POINTER(SZ)], C.c_int),
            "snn_read_queue": ([P, U32, P, P, P, SZ, C.POINTER(SZ)], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def grid_desc(net: dict, hist_cap: int = 0) -> GridDesc:
    g = GridDesc()
    for k in ("gx", "gy", "n_exc", "n_inh", "periodic", "tau_m", "v_th", "v_reset", "e_rest",
              "t_ref", "alpha_w", "tau_w", "sfa_on_inh", "seed"):
        setattr(g, k, net[k])
    g.hist_cap = hist_cap
    return g


def syn_desc(net: dict) -> SynDesc:
    s = SynDesc()
    for k in ("kernel", "record", "range", "k_in", "d_min", "d_max", "w_exc", "w_exc_sd", "w_inh",
              "ext_mode", "ext_const_q", "ext_n", "ext_rate_hz", "ext_w"):
        setattr(s, k, net[k])
    for k in ("preset", "p_local", "amp", "p_cut", "gen", "delay_dist", "delay_tau", "solver",
              "stdp", "ltp_period", "a_plus", "a_minus", "tau_plus", "tau_minus", "w_max"):   # absent: defaults
        setattr(s, k, net.get(k, 0))
    return s


# Every callback pair ever installed stays referenced: networks created under
# a pair release their buffers through it even after another is installed.
_installed_allocators = []


def set_allocator(alloc=None, free=None):
    """Install a process-wide device allocator (snn_set_allocator).

    alloc(nbytes) -> int device address (256-byte aligned) or 0 on failure;
    free(address) takes a block back.  Both None restores hipMalloc / hipFree.
    Networks and batches keep the allocator in force when they were created.
    """
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        st = lib().snn_set_allocator(ALLOC_FN(), FREE_FN(), None)
    else:
        fa = ALLOC_FN(lambda nbytes, ctx: alloc(int(nbytes)) or None)
        ff = FREE_FN(lambda ptr, ctx: free(int(ptr)))
        _installed_allocators.append((fa, ff))
        st = lib().snn_set_allocator(fa, ff, None)
    if st != SNN_OK:
        raise SNNError(st, lib().snn_last_error(None).decode())


def use_torch_allocator(device=None):
    """Route the library's device memory through torch's caching allocator.

    Blocks are taken on the calling thread's current stream of `device` (the
    current device by default); the library returns a block only once the
    stream that used it has finished with it, so the cache may hand it out
    again at once.  Memory shows up in torch.cuda.memory_allocated().
    """
    dev = torch.cuda.current_device() if device is None else int(device)
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev),
                  lambda p: torch.cuda.caching_allocator_delete(p))


def current_stream_handle():
    """The torch current HIP stream as a raw handle (None without a GPU)."""
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


def probe_atomics(n_targets: int, n_adds: int, stream=None) -> float:
    """Scattered int32 device-scope atomic adds per second (snn_probe_atomics)."""
    r = C.c_double(0.0)
    st = lib().snn_probe_atomics(n_targets, n_adds, stream, C.byref(r))
    if st != SNN_OK:
        raise SNNError(st, "snn_probe_atomics failed")
    return r.value


def host_stdp_tables(net: dict) -> dict:
    """The library's plasticity tables for a description with stdp = 1."""
    g, s = grid_desc(net), syn_desc(net)
    kp = np.zeros(256, dtype=np.int32)
    km = np.zeros(256, dtype=np.int32)
    win = C.c_uint32(0)
    wmax = C.c_int32(0)
    st = lib().snn_host_stdp_tables(C.byref(g), C.byref(s), _p(kp), _p(km), C.byref(win), C.byref(wmax))
    if st != SNN_OK:
        raise SNNError(st, lib().snn_last_error(None).decode())
    return dict(kp=kp[: win.value].copy(), km=km[: win.value].copy(), win=win.value, wmax_q=wmax.value)


def host_tables(net: dict) -> dict:
    """The library's own integer tables for a description (host computation)."""
    g, s = grid_desc(net), syn_desc(net)
    T = np.zeros(2 * net["gx"] * net["gy"], dtype=np.uint32)
    wtab = np.zeros(65536, dtype=np.int32)
    cb = np.zeros(256, dtype=np.int32)
    poisc = np.zeros(64, dtype=np.uint32)
    npois = np.zeros(1, dtype=np.uint32)
    consts = np.zeros(3, dtype=np.float64)
    st = lib().snn_host_tables(C.byref(g), C.byref(s), _p(T), _p(wtab), _p(cb), _p(poisc), _p(npois),
                               _p(consts))
    if st != SNN_OK:
        raise SNNError(st, lib().snn_last_error(None).decode())
    T = T.reshape(2, net["gy"], net["gx"])
    return dict(T=T[0].copy(), T_inh=T[1].copy(), wtab=wtab, cb=cb, poisc=poisc[: int(npois[0])].copy(),
                dm=consts[0], dw=consts[1], kappa=consts[2])


class Net:
    """One network on the GPU: build_grid at construction, then
    build_synapses, step, read_spikes ...  (names follow the C ABI)."""

    def __init__(self, net: dict, hist_cap: int = 0, stream=None):
        self.net = dict(net)
        self.N = net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])
        self.D = net["d_max"] - net["d_min"] + 1
        self._g = grid_desc(net, hist_cap)
        h = C.c_void_p()
        st = lib().snn_build_grid(C.byref(self._g), stream, C.byref(h))
        if st != SNN_OK:
            raise SNNError(st, lib().snn_last_error(None).decode())
        self.h = h

    def _check(self, st):
        if st != SNN_OK:
            raise SNNError(st, lib().snn_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.snn_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- the ABI calls ----
    def build_synapses(self):
        self._s = syn_desc(self.net)
        self._check(lib().snn_build_synapses(self.h, C.byref(self._s)))
        return self

    def step(self, n_ms: int):
        self._check(lib().snn_step(self.h, n_ms))

    def step_forced(self, gids):
        g = np.ascontiguousarray(gids, dtype=np.uint32)
        self._check(lib().snn_step_forced(self.h, _p(g), g.size))

    def step_forced_noalloc(self, gids):
        """step_forced staged in the library's static device array (no device allocation)."""
        g = np.ascontiguousarray(gids, dtype=np.uint32)
        self._check(lib().snn_step_forced_noalloc(self.h, _p(g), g.size))

    def read_spikes(self, t0=0, t1=2**63):
        n = C.c_size_t(0)
        st = lib().snn_read_spikes(self.h, t0, t1, None, 0, C.byref(n))
        if st not in (SNN_OK, SNN_E_TRUNC):
            self._check(st)
        out = np.zeros((max(n.value, 1), 2), dtype=np.uint32)
        self._check(lib().snn_read_spikes(self.h, t0, t1, _p(out), n.value, C.byref(n)))
        return out[: n.value]

    def step_forced_exact(self, gids, fracs):
        """Exact solver, lock-step: neuron gids[k] spikes at offset fracs[k] (2^-32 ms)."""
        g = np.ascontiguousarray(gids, dtype=np.uint32)
        f = np.ascontiguousarray(fracs, dtype=np.uint32)
        if g.size != f.size:
            raise ValueError("one offset per forced spike")
        self._check(lib().snn_step_forced_exact(self.h, _p(g), _p(f), g.size))

    def read_spike_times(self, t0=0, t1=2**63):
        """Exact solver: (t_ms, gid) rows and each spike's offset (2^-32 ms)."""
        n = C.c_size_t(0)
        st = lib().snn_read_spike_times(self.h, t0, t1, None, None, 0, C.byref(n))
        if st not in (SNN_OK, SNN_E_TRUNC):
            self._check(st)
        out = np.zeros((max(n.value, 1), 2), dtype=np.uint32)
        fr = np.zeros(max(n.value, 1), dtype=np.uint32)
        self._check(lib().snn_read_spike_times(self.h, t0, t1, _p(out), _p(fr), n.value, C.byref(n)))
        return out[: n.value], fr[: n.value]

    def read_queue(self, k: int):
        """Exact solver: inputs arriving k steps ahead, (target, offset, charge)
        rows ordered by target, offset, charge."""
        n = C.c_size_t(0)
        st = lib().snn_read_queue(self.h, k, None, None, None, 0, C.byref(n))
        if st not in (SNN_OK, SNN_E_TRUNC):
            self._check(st)
        m = max(n.value, 1)
        tgt, fr, wq = np.zeros(m, np.uint32), np.zeros(m, np.uint32), np.zeros(m, np.int32)
        self._check(lib().snn_read_queue(self.h, k, _p(tgt), _p(fr), _p(wq), n.value, C.byref(n)))
        q = np.stack([tgt[: n.value].astype(np.int64), fr[: n.value].astype(np.int64),
                      wq[: n.value].astype(np.int64)], axis=1)
        return q[np.lexsort((q[:, 2], q[:, 1], q[:, 0]))] if len(q) else q

    def read_state(self):
        V = np.zeros(self.N, dtype=np.float32)
        W = np.zeros(self.N, dtype=np.float32)
        R = np.zeros(self.N, dtype=np.uint8)
        self._check(lib().snn_read_state(self.h, _p(V), _p(W), _p(R)))
        return V, W, R

    def read_ring(self):
        r = np.zeros((RING, self.N), dtype=np.int32)
        self._check(lib().snn_read_ring(self.h, _p(r)))
        return r

    def export_rows(self, pre0: int, n: int):
        """(row_len u64[n], bend u16[n, D], record bytes) of rows pre0..pre0+n-1."""
        rb = 4 if self.net["record"] == 1 else 8
        row_len = np.zeros(n, dtype=np.uint64)
        bend = np.zeros((n, self.D), dtype=np.uint16)
        m = C.c_size_t(0)
        st = lib().snn_export_rows(self.h, pre0, n, _p(row_len), _p(bend), None, 0, C.byref(m))
        if st not in (SNN_OK, SNN_E_TRUNC):
            self._check(st)
        recs = np.zeros(max(m.value, 1) * rb, dtype=np.uint8)
        self._check(lib().snn_export_rows(self.h, pre0, n, _p(row_len), _p(bend), _p(recs), m.value,
                                          C.byref(m)))
        return row_len, bend, recs[: m.value * rb]

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().snn_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def time_kernels(self, n_ms: int) -> dict:
        kt = KernelTimes()
        self._check(lib().snn_time_kernels(self.h, n_ms, C.byref(kt)))
        return {k: getattr(kt, k) for k, _ in KernelTimes._fields_}

    def set_option(self, key: int, value: int):
        self._check(lib().snn_set_option(self.h, key, value))

    def reset(self):
        self._check(lib().snn_reset(self.h))

    def set_ext_rate(self, hz: float):
        self.set_option(OPT_EXT_RATE_UHZ, int(round(hz * 1e6)))
        self.net["ext_rate_hz"] = hz


class Batch:
    """Many networks ("jobs") stepped together by the batched multi-job
    kernels (names follow the C ABI: admit, step, poll, read_spikes)."""

    def __init__(self, hbm_budget: int, max_neurons: int, stream=None):
        h = C.c_void_p()
        st = lib().snn_batch_create(hbm_budget, max_neurons, stream, C.byref(h))
        if st != SNN_OK:
            raise SNNError(st, lib().snn_batch_last_error(None).decode())
        self.h = h
        self._descs = {}

    def _check(self, st):
        if st != SNN_OK:
            raise SNNError(st, lib().snn_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.snn_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def admit(self, net: dict, dur_ms: int):
        """Slot of the admitted job, or None when it does not fit now."""
        g, s = grid_desc(net), syn_desc(net)
        slot = C.c_int32(-1)
        st = lib().snn_batch_admit(self.h, C.byref(g), C.byref(s), dur_ms, C.byref(slot))
        if st == SNN_E_NOMEM:
            return None
        self._check(st)
        self._descs[slot.value] = (g, s)
        return slot.value

    def step(self, chunk_ms: int):
        self._check(lib().snn_batch_step(self.h, chunk_ms))

    def set_option(self, opt: int, value: int):
        """A knob of the batched schedule (OPT_SCATTER_BLOCKS,
        OPT_DELIVER_MODE, OPT_BIN_THRESHOLD_PPM)."""
        self._check(lib().snn_batch_set_option(self.h, int(opt), int(value)))

    def poll(self):
        out = np.zeros(64, dtype=np.int32)
        n = C.c_size_t(0)
        self._check(lib().snn_batch_poll(self.h, _p(out), 64, C.byref(n)))
        return [int(x) for x in out[: n.value]]

    def job_stats(self, slot: int) -> dict:
        s = Stats()
        self._check(lib().snn_batch_job_stats(self.h, slot, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def read_spikes(self, slot: int):
        """The finished job's raster ((t_ms, gid) rows); frees the slot."""
        n = C.c_size_t(0)
        st = lib().snn_batch_read_spikes(self.h, slot, None, 0, C.byref(n))
        if st == SNN_OK:   # no spikes: the slot is already free
            self._descs.pop(slot, None)
            return np.zeros((0, 2), dtype=np.uint32)
        if st != SNN_E_TRUNC:
            self._descs.pop(slot, None)
            self._check(st)
        out = np.zeros((max(n.value, 1), 2), dtype=np.uint32)
        self._check(lib().snn_batch_read_spikes(self.h, slot, _p(out), n.value, C.byref(n)))
        self._descs.pop(slot, None)
        return out[: n.value]

    def read_state(self, slot: int, ring: bool = True):
        """A running or finished job's (V, w, refractory steps, ring [32][N])."""
        g, _ = self._descs[slot]
        N = g.gx * g.gy * (g.n_exc + g.n_inh)
        V = np.zeros(N, dtype=np.float32)
        Wf = np.zeros(N, dtype=np.float32)
        R = np.zeros(N, dtype=np.uint8)
        rg = np.zeros((RING, N), dtype=np.int32) if ring else None
        self._check(lib().snn_batch_read_state(self.h, slot, _p(V), _p(Wf), _p(R),
                                               _p(rg) if ring else None))
        return V, Wf, R, rg

    def usage(self):
        b = C.c_uint64(0)
        j = C.c_uint32(0)
        self._check(lib().snn_batch_usage(self.h, C.byref(b), C.byref(j)))
        return b.value, j.value
