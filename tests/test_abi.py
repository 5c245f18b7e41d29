"""CPU checks of the C ABI: the library loads, exports every call include/snn.h
declares, validates descriptions on the host, and derives exactly the oracle's
integer tables (host-only computation, no device work)."""
import os
import re

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snn.h")
PKG = os.path.join(ROOT, "paper_1803_08833_amd")


@pytest.fixture(scope="module")
def snn():
    from paper_1803_08833_amd import build

    if not os.path.exists(os.path.join(PKG, "libsnn.so")):
        build.build()
    from paper_1803_08833_amd import snn as S

    S.lib()
    return S


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("snn_build_grid", "snn_build_synapses", "snn_step", "snn_read_spikes"):
        assert required in names


def test_library_exports_every_declared_symbol(snn):
    L = snn.lib()
    for name in declared():
        assert hasattr(L, name), name
    assert sorted(snn.EXPORTS) == declared()


def test_allocator_arguments_are_checked_on_the_host(snn):
    L = snn.lib()
    assert L.snn_set_allocator(snn.ALLOC_FN(lambda n, c: None), snn.FREE_FN(), None) == snn.SNN_E_INVAL
    assert b"both" in L.snn_last_error(None)
    assert L.snn_set_allocator(snn.ALLOC_FN(), snn.FREE_FN(lambda p, c: None), None) == snn.SNN_E_INVAL
    with pytest.raises(ValueError):
        snn.set_allocator(alloc=lambda n: 0)
    snn.set_allocator(lambda n: 0, lambda p: None)   # installs (nothing is allocated here)
    snn.set_allocator()                              # and back to hipMalloc / hipFree
    assert L.snn_set_allocator(snn.ALLOC_FN(), snn.FREE_FN(), None) == snn.SNN_OK


def test_product_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), f
                assert "or_net" not in src and "liboracle" not in src, f


@pytest.mark.parametrize("name", ["grid4_gauss", "grid24_gauss", "grid24_exp", "grid96_exp_code8",
                                  "grid24_gauss_paper", "grid48_exp_paper_code8"])
def test_library_tables_equal_oracle_tables(snn, oracle_mod, name):
    net = W.workload(name)["net"]
    lt = snn.host_tables(net)
    ot = oracle_mod.tables(net)
    np.testing.assert_array_equal(lt["T"], ot["T"])
    np.testing.assert_array_equal(lt["T_inh"], ot["T_inh"])
    np.testing.assert_array_equal(lt["wtab"], ot["wtab"])
    np.testing.assert_array_equal(lt["cb"], ot["cb"])
    np.testing.assert_array_equal(lt["poisc"], ot["poisc"])
    for k in ("dm", "dw", "kappa"):
        assert lt[k] == pytest.approx(ot[k], rel=1e-13)


def test_invalid_descriptions_are_rejected_on_the_host(snn):
    import ctypes as C

    base = W.workload("grid4_gauss")["net"]
    bad = [dict(gx=0), dict(n_exc=990, n_inh=249), dict(periodic=0), dict(tau_m=0.0),
           dict(v_th=-1.0), dict(gx=4000, gy=4000)]
    for over in bad:
        net = dict(base, **over)
        g = snn.grid_desc(net)
        h = C.c_void_p()
        st = snn.lib().snn_build_grid(C.byref(g), None, C.byref(h))
        assert st == snn.SNN_E_INVAL, over
        assert not h.value
        assert snn.lib().snn_last_error(None)
    # tables: probability reaching one, bad Poisson mean
    with pytest.raises(snn.SNNError):
        snn.host_tables(dict(base, k_in=19839.0))
    with pytest.raises(snn.SNNError):
        snn.host_tables(dict(base, ext_rate_hz=1e5))
    # paper preset: probabilities outside [0, 1), no cut-off
    paper = W.make_paper(4, 4, W.PAPER_GAUSS, 1)
    for over in (dict(p_local=1.0), dict(amp=-0.1), dict(p_cut=0.0)):
        with pytest.raises(snn.SNNError):
            snn.host_tables(dict(paper, **over))


@pytest.mark.parametrize("over", [dict(), dict(a_plus=0.01, a_minus=0.012, tau_plus=16.8, tau_minus=33.7),
                                  dict(a_plus=0.0, a_minus=0.005, tau_minus=5.0, w_max=0.999969),
                                  dict(a_plus=0.05, a_minus=0.0, tau_plus=25.0)])
def test_library_stdp_tables_equal_oracle_tables(snn, oracle_mod, over):
    net = dict(W.workload("grid4_gauss")["net"], stdp=1, **over)
    lt = snn.host_stdp_tables(net)
    ot = oracle_mod.stdp_tables(net)
    assert lt["win"] == ot["win"] and lt["wmax_q"] == ot["wmax_q"]
    np.testing.assert_array_equal(lt["kp"], ot["kp"])
    np.testing.assert_array_equal(lt["km"], ot["km"])


def test_invalid_plasticity_is_rejected_on_the_host(snn):
    base = dict(W.workload("grid4_gauss")["net"], stdp=1)
    for over in (dict(tau_plus=0.0), dict(a_minus=-0.001), dict(tau_plus=200.0, a_plus=0.5), dict(stdp=2)):
        with pytest.raises(snn.SNNError):
            snn.host_stdp_tables(dict(base, **over))
    with pytest.raises(snn.SNNError):
        snn.host_stdp_tables(dict(base, stdp=0))
