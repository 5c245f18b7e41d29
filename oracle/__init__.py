"""Test-only FP64 CPU oracle of the spiking-network hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: importable from tests, the smoke check and the
CPU-baseline leg of the benchmark, never from the product path.  The C source
(`oracle.c`) follows the paper step by step and shares nothing with the HIP
library.  This wrapper only marshals arguments.

Parity pins and their status are listed in `oracle.c`'s header; Philox
against a library implementation, tables against closed forms, neuron map
against closed-form interspike intervals, connectivity against expected
statistics, delivery against brute force and charge conservation.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
RING = 32


LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force=False, openmp=False):
    """Compile oracle.c with gcc (plain -O2, no fast-math).  openmp: the
    multi-threaded build timed as the CPU baseline (same source; its OpenMP
    loops are the neuron update and the delivery's integer adds)."""
    lib_path = LIB_OMP if openmp else LIB
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(SRC):
        tmp = lib_path + ".tmp"
        flags = ["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"]
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", *flags, "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


class Cfg(C.Structure):
    _fields_ = [
        ("gx", C.c_uint32), ("gy", C.c_uint32), ("n_exc", C.c_uint32), ("n_inh", C.c_uint32),
        ("periodic", C.c_uint32),
        ("tau_m", C.c_double), ("v_th", C.c_double), ("v_reset", C.c_double), ("e_rest", C.c_double),
        ("t_ref", C.c_double), ("alpha_w", C.c_double), ("tau_w", C.c_double),
        ("sfa_on_inh", C.c_uint32),
        ("seed", C.c_uint64),
        ("kernel", C.c_uint32), ("range", C.c_double), ("k_in", C.c_double),
        ("d_min", C.c_uint32), ("d_max", C.c_uint32),
        ("w_exc", C.c_double), ("w_exc_sd", C.c_double), ("w_inh", C.c_double),
        ("record", C.c_uint32), ("ext_mode", C.c_uint32),
        ("ext_n", C.c_double), ("ext_rate_hz", C.c_double), ("ext_w", C.c_double),
        ("ext_const_q", C.c_int32), ("pad_", C.c_uint32),
        ("preset", C.c_uint32), ("pad2_", C.c_uint32),
        ("p_local", C.c_double), ("amp", C.c_double), ("p_cut", C.c_double),
        ("gen", C.c_uint32), ("delay_dist", C.c_uint32), ("delay_tau", C.c_double),
        ("solver", C.c_uint32), ("pad3_", C.c_uint32),
        ("stdp", C.c_uint32), ("ltp_period", C.c_uint32),
        ("a_plus", C.c_double), ("a_minus", C.c_double),
        ("tau_plus", C.c_double), ("tau_minus", C.c_double), ("w_max", C.c_double),
    ]

SOLVER_STEP, SOLVER_EXACT = 0, 1
# absent from a description: 0
OPTIONAL = ("solver", "stdp", "ltp_period", "a_plus", "a_minus", "tau_plus", "tau_minus", "w_max")


def cfg(net: dict) -> Cfg:
    c = Cfg()
    for name, _ in Cfg._fields_:
        if not name.startswith("pad"):
            setattr(c, name, net.get(name, 0) if name in OPTIONAL else net[name])
    return c


_lib = None


def _load(path):
    """Open a build of oracle.c and declare its entry points."""
    L = C.CDLL(path)
    P, U32, U64, I32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
    L.or_philox.argtypes = [P, P, P]
    L.or_philox.restype = None
    L.or_make_tables.argtypes = [C.POINTER(Cfg), P, P, P, P, P, P, P]
    L.or_make_tables.restype = C.c_int
    L.or_net_create.argtypes = [C.POINTER(Cfg), C.c_int]
    L.or_net_create.restype = P
    L.or_net_free.argtypes = [P]
    L.or_net_free.restype = None
    L.or_net_build.argtypes = [P]
    L.or_net_build.restype = C.c_int
    L.or_build_rows.argtypes = [C.POINTER(Cfg), U32, U32, P, P, P, U64, C.POINTER(U64)]
    L.or_build_rows.restype = C.c_int
    L.or_col_input.argtypes = [C.POINTER(Cfg), U32, P, U64, P]
    L.or_col_input.restype = C.c_int
    L.or_col_pending.argtypes = [C.POINTER(Cfg), U32, P, P, U64, U32, P]
    L.or_col_pending.restype = C.c_int
    L.or_net_csr.argtypes = [P, P, P, P, U64]
    L.or_net_csr.restype = C.c_int
    L.or_net_nnz.argtypes = [P]
    L.or_net_nnz.restype = U64
    L.or_net_set_csr.argtypes = [P, P, P, P, P, P]
    L.or_net_set_csr.restype = C.c_int
    L.or_net_step.argtypes = [P, U32]
    L.or_net_step.restype = C.c_int
    L.or_net_step_forced.argtypes = [P, P, U64]
    L.or_net_step_forced.restype = C.c_int
    L.or_net_state.argtypes = [P, P, P, P]
    L.or_net_state.restype = C.c_int
    L.or_net_ring.argtypes = [P, P]
    L.or_net_ring.restype = C.c_int
    L.or_net_hist.argtypes = [P, P, U64]
    L.or_net_hist.restype = U64
    L.or_net_stats.argtypes = [P, P]
    L.or_net_step_forced_exact.argtypes = [P, P, P, U64]
    L.or_net_step_forced_exact.restype = C.c_int
    L.or_net_hist_frac.argtypes = [P, P, U64]
    L.or_net_hist_frac.restype = U64
    L.or_net_queue.argtypes = [P, U32, P, P, P, U64]
    L.or_net_queue.restype = U64
    L.or_net_rend.argtypes = [P, P]
    L.or_net_rend.restype = C.c_int
    L.or_net_stats.restype = None
    L.or_threads.argtypes = []
    L.or_threads.restype = C.c_int
    L.or_stdp_totals.argtypes = [C.POINTER(Cfg), P, P, U64, P, P, P, U64, U32, U32, P]
    L.or_stdp_totals.restype = C.c_int
    L.or_stdp_tables.argtypes = [C.POINTER(Cfg), P, P, P, P]
    L.or_stdp_tables.restype = C.c_int
    L.or_net_ext_counts.argtypes = [P, U32, U32, P]
    L.or_net_ext_counts.restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _load(LIB)
    return _lib


@contextlib.contextmanager
def library(path):
    """Route every oracle call inside the block to another build of
    oracle.c (a planted-mistake variant compiled by a test)."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    """Philox4x32-10 of one 128-bit counter under one 64-bit key."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c), _p(k), _p(out))
    return out


def tables(net: dict):
    """Host tables: thresholds T[gy, gx] of excitatory sources and T_inh of
    inhibitory ones, weight table, codebook, Poisson CDF thresholds,
    propagator constants (dm, dw, kappa), (nref, jext_q, winh_q)."""
    c = cfg(net)
    T = np.zeros(2 * net["gx"] * net["gy"], dtype=np.uint32)
    wtab = np.zeros(65536, dtype=np.int32)
    cb = np.zeros(256, dtype=np.int32)
    poisc = np.zeros(64, dtype=np.uint32)
    npois = np.zeros(1, dtype=np.uint32)
    consts = np.zeros(3, dtype=np.float64)
    iconsts = np.zeros(3, dtype=np.int32)
    st = lib().or_make_tables(C.byref(c), _p(T), _p(wtab), _p(cb), _p(poisc), _p(npois),
                              _p(consts), _p(iconsts))
    if st != 0:
        raise ValueError(f"oracle tables: status {st}")
    T = T.reshape(2, net["gy"], net["gx"])
    return dict(T=T[0].copy(), T_inh=T[1].copy(), wtab=wtab, cb=cb,
                poisc=poisc[: int(npois[0])].copy(), dm=consts[0], dw=consts[1], kappa=consts[2],
                nref=int(iconsts[0]), jext_q=int(iconsts[1]), winh_q=int(iconsts[2]))


def stdp_tables(net: dict):
    """Plasticity tables: kp[win], km[win] (2^-16 mV per pair at lag k), the
    window and the weight bound w_max in 2^-16 mV."""
    c = cfg(net)
    kp = np.zeros(256, dtype=np.int32)
    km = np.zeros(256, dtype=np.int32)
    win = np.zeros(1, dtype=np.uint32)
    wmax = np.zeros(1, dtype=np.int32)
    st = lib().or_stdp_tables(C.byref(c), _p(kp), _p(km), _p(win), _p(wmax))
    if st != 0:
        raise ValueError(f"oracle stdp tables: status {st}")
    w = int(win[0])
    return dict(kp=kp[:w].copy(), km=km[:w].copy(), win=w, wmax_q=int(wmax[0]))


def stdp_totals(net: dict, raster, pre, tgt, delay, T0: int, T1: int) -> np.ndarray:
    """Plasticity change of a period [T0, T1) for the synapses (pre, tgt,
    delay), summed pair by pair from the (step, gid) raster (unclipped)."""
    c = cfg(net)
    r = np.asarray(raster, dtype=np.uint32).reshape(-1, 2)
    rs, rg = np.ascontiguousarray(r[:, 0]), np.ascontiguousarray(r[:, 1])
    pre = np.ascontiguousarray(pre, dtype=np.uint32)
    tgt = np.ascontiguousarray(tgt, dtype=np.uint32)
    delay = np.ascontiguousarray(delay, dtype=np.uint32)
    out = np.zeros(pre.size, dtype=np.int64)
    st = lib().or_stdp_totals(C.byref(c), _p(rs), _p(rg), rs.size, _p(pre), _p(tgt), _p(delay), pre.size,
                              T0, T1, _p(out))
    if st != 0:
        raise ValueError(f"oracle stdp_totals: status {st}")
    return out


def n_neurons(net):
    return net["gx"] * net["gy"] * (net["n_exc"] + net["n_inh"])


def n_delays(net):
    return net["d_max"] - net["d_min"] + 1


def rec_bytes(net):
    return 4 if net["record"] == 1 else 8


def build_rows(net: dict, pre0: int, cnt: int, cap: int | None = None):
    """Rows pre0..pre0+cnt-1 of the projection table, built one by one.
    Returns (row_len u64[cnt], bend u16[cnt, D], records bytes)."""
    c = cfg(net)
    D = n_delays(net)
    grow = cap is None   # no capacity given: start from the in-degree and grow on overflow
    if cap is None:
        cap = int(cnt * (net["k_in"] * 1.5 + 200))
    while True:
        row_len = np.zeros(cnt, dtype=np.uint64)
        bend = np.zeros((cnt, D), dtype=np.uint16)
        recs = np.zeros(cap * rec_bytes(net), dtype=np.uint8)
        n_out = C.c_uint64(0)
        st = lib().or_build_rows(C.byref(c), pre0, cnt, _p(row_len), _p(bend), _p(recs), cap,
                                 C.byref(n_out))
        if st == -5 and grow:
            cap *= 4
            continue
        if st != 0:
            raise ValueError(f"oracle build_rows: status {st}")
        break
    return row_len, bend, recs[: int(n_out.value) * rec_bytes(net)].copy()


def col_pending(net: dict, j: int, raster, T: int) -> np.ndarray:
    """Charge in flight for target j after steps 0 .. T-1 of the (step, gid)
    raster: int64[d_max], entry a arriving at step T + a."""
    c = cfg(net)
    r = np.ascontiguousarray(raster, dtype=np.uint32).reshape(-1, 2)
    keep = r[:, 0].astype(np.int64) >= T - net["d_max"]
    st_ = np.ascontiguousarray(r[keep, 0])
    pr = np.ascontiguousarray(r[keep, 1])
    out = np.zeros(net["d_max"], dtype=np.int64)
    st = lib().or_col_pending(C.byref(c), j, _p(st_), _p(pr), pr.size, T, _p(out))
    if st != 0:
        raise ValueError(f"oracle col_pending: status {st}")
    return out


def col_input(net: dict, j: int, pres) -> np.ndarray:
    """Fixed-point charge per delay that presynaptic set `pres` sends to j."""
    c = cfg(net)
    p = np.ascontiguousarray(pres, dtype=np.uint32)
    out = np.zeros(n_delays(net), dtype=np.int64)
    st = lib().or_col_input(C.byref(c), j, _p(p), p.size, _p(out))
    if st != 0:
        raise ValueError(f"oracle col_input: status {st}")
    return out


class Net:
    """One oracle network: FP64 state, int32 fixed-point delay ring."""

    def __init__(self, net: dict, fp64_weights: bool = False):
        self.net = dict(net)
        self._c = cfg(net)
        self.h = lib().or_net_create(C.byref(self._c), 1 if fp64_weights else 0)
        if not self.h:
            raise ValueError("oracle: invalid network description")
        self.N = n_neurons(net)
        self.D = n_delays(net)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_net_free(h)
            self.h = None

    def build(self):
        st = lib().or_net_build(self.h)
        if st != 0:
            raise ValueError(f"oracle build: status {st}")
        return self

    def csr(self):
        nnz = int(lib().or_net_nnz(self.h))
        row_ptr = np.zeros(self.N + 1, dtype=np.uint64)
        bend = np.zeros((self.N, self.D), dtype=np.uint16)
        recs = np.zeros(max(nnz, 1) * rec_bytes(self.net), dtype=np.uint8)
        st = lib().or_net_csr(self.h, _p(row_ptr), _p(bend), _p(recs), nnz)
        if st != 0:
            raise ValueError(f"oracle csr: status {st}")
        return row_ptr, bend, recs[: nnz * rec_bytes(self.net)]

    def set_csr(self, row_ptr, bend, tgt, delay, wq):
        args = [np.ascontiguousarray(row_ptr, dtype=np.uint64),
                np.ascontiguousarray(bend, dtype=np.uint16),
                np.ascontiguousarray(tgt, dtype=np.uint32),
                np.ascontiguousarray(delay, dtype=np.uint32),
                np.ascontiguousarray(wq, dtype=np.int32)]
        st = lib().or_net_set_csr(self.h, *[_p(a) for a in args])
        if st != 0:
            raise ValueError(f"oracle set_csr: status {st}")

    def step(self, n=1):
        st = lib().or_net_step(self.h, n)
        if st != 0:
            raise OverflowError(f"oracle step: status {st}")

    def step_forced(self, gids):
        g = np.ascontiguousarray(gids, dtype=np.uint32)
        st = lib().or_net_step_forced(self.h, _p(g), g.size)
        if st != 0:
            raise ValueError(f"oracle step_forced: status {st}")

    def state(self):
        V = np.zeros(self.N, dtype=np.float64)
        w = np.zeros(self.N, dtype=np.float64)
        ref = np.zeros(self.N, dtype=np.int32)
        lib().or_net_state(self.h, _p(V), _p(w), _p(ref))
        return V, w, ref

    def ring(self):
        r = np.zeros((RING, self.N), dtype=np.int32)
        lib().or_net_ring(self.h, _p(r))
        return r

    def spikes(self):
        n = int(lib().or_net_hist(self.h, None, 0))
        out = np.zeros((max(n, 1), 2), dtype=np.uint32)
        lib().or_net_hist(self.h, _p(out), n)
        return out[:n]

    def step_forced_exact(self, gids, fracs):
        """Exact solver, lock-step: neuron gids[k] spikes at offset fracs[k]."""
        g = np.ascontiguousarray(gids, dtype=np.uint32)
        f = np.ascontiguousarray(fracs, dtype=np.uint32)
        assert g.size == f.size
        st = lib().or_net_step_forced_exact(self.h, _p(g), _p(f), g.size)
        if st != 0:
            raise ValueError(f"oracle step_forced_exact: status {st}")

    def spike_fracs(self):
        """Emission offsets (2^-32 ms) of the history, aligned with spikes()."""
        n = int(lib().or_net_hist_frac(self.h, None, 0))
        out = np.zeros(max(n, 1), dtype=np.uint32)
        lib().or_net_hist_frac(self.h, _p(out), n)
        return out[:n]

    def queue(self, slot):
        """Exact solver: inputs queued for ring slot `slot` as (target, offset,
        charge) rows, ordered."""
        n = int(lib().or_net_queue(self.h, slot, None, None, None, 0))
        tgt = np.zeros(max(n, 1), dtype=np.uint32)
        fr = np.zeros(max(n, 1), dtype=np.uint32)
        wq = np.zeros(max(n, 1), dtype=np.int32)
        lib().or_net_queue(self.h, slot, _p(tgt), _p(fr), _p(wq), n)
        return np.stack([tgt[:n].astype(np.int64), fr[:n].astype(np.int64), wq[:n].astype(np.int64)], axis=1)

    def ext_counts(self, t0, t1):
        """External Poisson counts u8[t1 - t0, N] of steps t0 .. t1-1."""
        out = np.zeros((t1 - t0, self.N), dtype=np.uint8)
        st = lib().or_net_ext_counts(self.h, t0, t1, _p(out))
        if st != 0:
            raise ValueError(f"oracle ext_counts: status {st}")
        return out

    def rend(self):
        re = np.zeros(self.N, dtype=np.uint64)
        lib().or_net_rend(self.h, _p(re))
        return re

    def stats(self):
        out = np.zeros(6, dtype=np.uint64)
        lib().or_net_stats(self.h, _p(out))
        return dict(t=int(out[0]), spikes=int(out[1]), rec_events=int(out[2]),
                    ext_events=int(out[3]), nnz=int(out[4]), overflow=int(out[5]))
