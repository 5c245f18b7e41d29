"""Pins of the oracle's projections (Sec. II.B, Sec. III.B) against the
statistics the connection law fixes, on the 4x4 Gaussian workload:

* in-degree: Poisson-binomial with mean k_in and variance sum n p (1 - p);
* synapse counts per torus offset: N n(off) p(off), with p = B f(r) from the
  paper's lateral law (z-scores and chi^2);
* delays uniform on [d_min, d_max]; excitatory weights distributed as the
  weight table, inhibitory weight exact;
* structure: no self-connections, no repeated pair, rows ordered by (delay,
  target) with consistent bucket ends; rows and columns built one by one equal
  the full table.
"""
import numpy as np
import pytest
from scipy import stats

from paper_1803_08833_amd import workloads as W


def decode(net, row_ptr, bend, recs):
    N = W.n_neurons(net)
    D = net["d_max"] - net["d_min"] + 1
    r = recs.view(np.uint32).reshape(-1, 2)
    tgt = r[:, 0].astype(np.int64)
    wq = np.rint(r[:, 1].view(np.float32).astype(np.float64) * 65536).astype(np.int64)
    lens = np.diff(row_ptr.astype(np.int64))
    pre = np.repeat(np.arange(N), lens)
    # delay of each record from its row's bucket ends
    k = np.arange(tgt.size) - np.repeat(row_ptr[:-1].astype(np.int64), lens)
    be = bend.astype(np.int64)[pre]
    delay = net["d_min"] + (be <= k[:, None]).sum(axis=1)
    return pre, tgt, wq, delay


@pytest.fixture(scope="module")
def c0(oracle_mod):
    net = W.workload("grid4_gauss")["net"]
    o = oracle_mod.Net(net).build()
    row_ptr, bend, recs = o.csr()
    return net, o, row_ptr, bend, recs, decode(net, row_ptr, bend, recs), oracle_mod.tables(net)


def _p_offset(net, tb):
    return tb["T"].astype(np.float64) / 2**32


def test_structure(c0):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    N = W.n_neurons(net)
    assert row_ptr[0] == 0 and row_ptr[-1] == tgt.size
    assert np.all(pre != tgt)
    assert np.all(bend[:, -1] == np.diff(row_ptr.astype(np.int64)))
    assert np.all(np.diff(bend.astype(np.int64), axis=1) >= 0)
    key = pre * N + tgt
    assert np.unique(key).size == key.size                      # no repeated pair
    order = (pre * 64 + (delay - net["d_min"])) * N + tgt
    assert np.all(np.diff(order) > 0)                           # (delay, target) order


def test_in_degree_distribution(c0):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    N = W.n_neurons(net)
    M = net["n_exc"] + net["n_inh"]
    p = _p_offset(net, tb)
    n = np.full(p.shape, float(M))
    n[0, 0] = M - 1
    mean = (n * p).sum()
    var = (n * p * (1 - p)).sum()
    indeg = np.bincount(tgt, minlength=N)
    outdeg = np.diff(row_ptr.astype(np.int64))
    assert mean == pytest.approx(net["k_in"], abs=1e-6)
    for deg in (indeg, outdeg):
        assert abs(deg.mean() - mean) < 5 * np.sqrt(var / N)
        assert deg.var() == pytest.approx(var, rel=0.1)


def test_offset_histogram_follows_law(c0):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    gx, gy = net["gx"], net["gy"]
    M = net["n_exc"] + net["n_inh"]
    N = W.n_neurons(net)
    mi, mj = pre // M, tgt // M
    dxr = (mj % gx - mi % gx) % gx
    dyr = (mj // gx - mi // gx) % gy
    counts = np.zeros((gy, gx))
    np.add.at(counts, (dyr, dxr), 1)
    # the paper's Gaussian law with the prefactor fixing the total
    dx = np.where(2 * np.arange(gx) <= gx, np.arange(gx), np.arange(gx) - gx)
    dy = np.where(2 * np.arange(gy) <= gy, np.arange(gy), np.arange(gy) - gy)
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    f = np.exp(-r2 / (2 * net["range"] ** 2))
    n = np.full((gy, gx), float(M))
    n[0, 0] = M - 1
    B = net["k_in"] / (n * f).sum()
    exp_counts = N * n * B * f
    z = (counts - exp_counts) / np.sqrt(exp_counts * (1 - B * f))
    assert np.abs(z).max() < 5
    chi2 = (((counts - exp_counts) ** 2) / exp_counts).sum()
    assert stats.chi2.sf(chi2, gx * gy - 1) > 1e-4
    # mean target distance (1.06 module spacings for this workload, summed by
    # hand over the law's offsets)
    dist = np.sqrt(r2[dyr, dxr].astype(np.float64))
    assert dist.mean() == pytest.approx(1.06, abs=0.02)


def test_delays_uniform(c0):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    D = net["d_max"] - net["d_min"] + 1
    h = np.bincount(delay - net["d_min"], minlength=D)
    assert h.size == D
    chi2 = ((h - h.mean()) ** 2 / h.mean()).sum()
    assert stats.chi2.sf(chi2, D - 1) > 1e-4


def test_weights(c0):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    M = net["n_exc"] + net["n_inh"]
    exc = (pre % M) < net["n_exc"]
    assert np.all(wq[~exc] == round(net["w_inh"] * 65536))
    we = wq[exc] / 65536
    assert we.mean() == pytest.approx(net["w_exc"], abs=5 * net["w_exc_sd"] / np.sqrt(we.size))
    assert we.std() == pytest.approx(net["w_exc_sd"], rel=0.01)
    assert np.isin(wq[exc], tb["wtab"]).all()
    # roughly 80 % of the synapses are excitatory
    assert exc.mean() == pytest.approx(net["n_exc"] / M, abs=0.005)


def test_rows_built_alone_equal_table(c0, oracle_mod):
    net, o, row_ptr, bend, recs, *_ = c0
    for pre0, cnt in ((0, 3), (991, 3), (19837, 3), (5000, 2)):
        rl, be, rc = oracle_mod.build_rows(net, pre0, cnt)
        lo, hi = int(row_ptr[pre0]), int(row_ptr[pre0 + cnt])
        np.testing.assert_array_equal(rl, np.diff(row_ptr[pre0:pre0 + cnt + 1].astype(np.int64)))
        np.testing.assert_array_equal(be, bend[pre0:pre0 + cnt])
        np.testing.assert_array_equal(rc, recs[lo * 8:hi * 8])


def test_column_input_equals_table(c0, oracle_mod):
    net, o, row_ptr, bend, recs, (pre, tgt, wq, delay), tb = c0
    rng = np.random.default_rng(3)
    pres = np.sort(rng.choice(W.n_neurons(net), 500, replace=False)).astype(np.uint32)
    D = net["d_max"] - net["d_min"] + 1
    sel = np.isin(pre, pres)
    for j in (0, 17, 12345, 19839):
        got = oracle_mod.col_input(net, j, pres)
        m = sel & (tgt == j)
        want = np.bincount(delay[m] - net["d_min"], weights=wq[m], minlength=D).astype(np.int64)
        np.testing.assert_array_equal(got, want)
