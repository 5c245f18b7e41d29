"""Pins of the oracle's delay distributions (Sec. II.B: delays uniform or
exponential).  Exponential: bucket k of the D integer delays has probability
proportional to exp(-k / tau), i.e. a geometric law truncated to D values,
whose closed-form CDF (1 - q^(k+1)) / (1 - q^D), q = exp(-1/tau), the built
rows' delay histogram must follow (chi^2); uniform: every bucket 1/D."""
import math

import numpy as np
from scipy import stats

from paper_1803_08833_amd import workloads as W


def _bucket_counts(oracle_mod, net):
    o = oracle_mod.Net(net).build()
    _, bend, _ = o.csr()
    be = bend.astype(np.int64)
    return np.diff(np.concatenate([np.zeros((be.shape[0], 1), dtype=np.int64), be], axis=1), axis=1).sum(0)


def test_exponential_delays_follow_truncated_geometric(oracle_mod):
    for tau in (2.0, 6.5):
        net = W.make(4, 4, W.GAUSS, 1.0, 300, 61, n_exc=80, n_inh=20, delay_dist=W.DELAY_EXP, delay_tau=tau)
        obs = _bucket_counts(oracle_mod, net).astype(np.float64)
        D = net["d_max"] - net["d_min"] + 1
        q = math.exp(-1.0 / tau)
        cdf = np.array([(1 - q ** (k + 1)) / (1 - q**D) for k in range(D)])
        pmf = np.diff(np.concatenate([[0.0], cdf]))
        exp = pmf * obs.sum()
        keep = exp >= 5
        o2 = np.append(obs[keep], obs[~keep].sum())
        e2 = np.append(exp[keep], exp[~keep].sum())
        if e2[-1] == 0:
            o2, e2 = o2[:-1], e2[:-1]
        assert stats.chisquare(o2, e2).pvalue > 1e-3, tau


def test_uniform_delays_are_uniform(oracle_mod):
    net = W.make(4, 4, W.GAUSS, 1.0, 300, 62, n_exc=80, n_inh=20)
    obs = _bucket_counts(oracle_mod, net).astype(np.float64)
    assert stats.chisquare(obs).pvalue > 1e-3
