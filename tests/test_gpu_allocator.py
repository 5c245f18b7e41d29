"""GPU tests of snn_set_allocator.

Networks whose device memory comes from torch's caching allocator must step
to exactly the result of networks on hipMalloc memory, under every delivery
schedule.  The cache is first filled with blocks holding a garbage byte
pattern, so nothing the library reads may rely on fresh memory being zero.
The memory is torch's while a network lives and goes back when it is
destroyed; handles keep the allocator they were created with; a failing or
misaligned allocator fails the create cleanly; a batch built under the
allocator gives every job its raster alone.
"""
import sys

import numpy as np
import pytest

from paper_1803_08833_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def snn():
    from paper_1803_08833_amd import snn as S

    S.lib()
    import torch

    assert torch.cuda.is_available()
    return S


@pytest.fixture
def torch_alloc(snn):
    import torch

    snn.use_torch_allocator()
    try:
        yield torch
    finally:
        snn.set_allocator()


def dirty_cache(torch):
    """Leave cached blocks of many sizes filled with 0xA5 bytes."""
    sizes = [64 << 10, 256 << 10, 768 << 10, 2 << 20, 8 << 20, 32 << 20, 128 << 20]
    ts = [torch.full((n,), 0xA5, dtype=torch.uint8, device="cuda") for n in sizes for _ in range(3)]
    torch.cuda.synchronize()
    del ts


def run(snn, net, mode, steps=300):
    with snn.Net(net) as g:
        if mode == 2:
            g.set_option(snn.OPT_DELIVER_MODE, 2)   # before the build: two-level bins
        g.build_synapses()
        g.set_option(snn.OPT_DELIVER_MODE, mode)
        g.set_option(snn.OPT_BIN_THRESHOLD, 0)
        g.step(steps)
        st = g.stats()
        assert st["deliver_mode"] == mode
        return g.read_ring(), g.read_spikes(), g.read_state(), st


@pytest.mark.parametrize("mode,record", [(0, W.REC_F32), (1, W.REC_F32), (2, W.REC_CODE8)])
def test_torch_memory_steps_like_hipmalloc(snn, mode, record):
    import torch

    net = W.make(4, 4, W.EXP, 3.0, 400, 83, record=record, ext_rate_hz=2.6)
    say(f"case: allocator parity, schedule {mode}, record {record}")
    ref = run(snn, net, mode)
    snn.use_torch_allocator()
    try:
        dirty_cache(torch)
        got = run(snn, net, mode)
    finally:
        snn.set_allocator()
    np.testing.assert_array_equal(got[0], ref[0])
    np.testing.assert_array_equal(got[1], ref[1])
    assert len(ref[1]) > 0
    for a, b in zip(got[2], ref[2]):
        np.testing.assert_array_equal(a, b)
    for k in ("spikes", "rec_events", "ext_events", "nnz", "bytes_device"):
        assert got[3][k] == ref[3][k], k


def test_memory_is_torch_and_returned(snn, torch_alloc):
    torch = torch_alloc
    net = W.make(3, 3, W.GAUSS, 1.5, 300, 5)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    g = snn.Net(net)
    g.build_synapses()
    g.step(50)
    held = torch.cuda.memory_allocated() - m0
    dev = g.stats()["bytes_device"]
    assert held >= dev, (held, dev)   # torch rounds blocks up
    g.close()
    assert torch.cuda.memory_allocated() == m0


def test_handles_keep_their_allocator(snn):
    import torch

    net = W.make(2, 2, W.GAUSS, 1.5, 300, 6)
    a = snn.Net(net)          # hipMalloc memory
    a.build_synapses()
    snn.use_torch_allocator()
    try:
        torch.cuda.synchronize()
        m0 = torch.cuda.memory_allocated()
        b = snn.Net(net)      # torch memory
        b.build_synapses()
        m1 = torch.cuda.memory_allocated()
        assert m1 > m0
        a.step(40)
        b.step(40)
        np.testing.assert_array_equal(a.read_spikes(), b.read_spikes())
        a.close()             # goes back to hipFree, not to torch
        assert torch.cuda.memory_allocated() == m1
        snn.set_allocator()   # b still frees through torch
        b.close()
        assert torch.cuda.memory_allocated() == m0
    finally:
        snn.set_allocator()


def test_failing_and_misaligned_allocators(snn):
    import torch

    net = W.make(2, 2, W.GAUSS, 1.5, 300, 7)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    calls = {"n": 0}

    def fail_after_four(n):
        calls["n"] += 1
        if calls["n"] > 4:
            return 0
        return torch.cuda.caching_allocator_alloc(n)

    try:
        snn.set_allocator(fail_after_four, torch.cuda.caching_allocator_delete)
        with pytest.raises(snn.SNNError) as e:
            snn.Net(net)
        assert e.value.status == snn.SNN_E_NOMEM
        assert calls["n"] == 5
        assert torch.cuda.memory_allocated() == m0   # the four blocks were given back

        given = []

        def misaligned(n):
            p = torch.cuda.caching_allocator_alloc(n + 256)
            given.append(p)
            return p + 16

        snn.set_allocator(misaligned, lambda p: torch.cuda.caching_allocator_delete(p - 16))
        with pytest.raises(snn.SNNError) as e:
            snn.Net(net)
        assert e.value.status == snn.SNN_E_NOMEM
        assert len(given) == 1
        assert torch.cuda.memory_allocated() == m0
    finally:
        snn.set_allocator()


def test_batch_under_torch_allocator(snn, torch_alloc):
    torch = torch_alloc
    r = np.random.default_rng(21)
    jobs = [dict(net=W.make(g, g, W.EXP, 3.0, 400, 900 + i, ext_rate_hz=2.5), steps=int(r.integers(60, 200)))
            for i, g in enumerate((1, 2, 3, 2))]
    say("case: batch of 4 jobs built on torch memory vs each alone on hipMalloc memory")
    snn.set_allocator()
    ref = []
    for j in jobs:
        with snn.Net(j["net"], hist_cap=1 << 22) as g:
            g.build_synapses()
            g.step(j["steps"])
            ref.append(g.read_spikes())
    snn.use_torch_allocator()
    dirty_cache(torch)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    got = {}
    with snn.Batch(8 << 30, 1 << 20) as b:
        slots = {b.admit(j["net"], j["steps"]): i for i, j in enumerate(jobs)}
        assert None not in slots
        while len(got) < len(jobs):
            b.step(32)
            for s in b.poll():
                got[slots[s]] = b.read_spikes(s)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
    for i, rs in enumerate(ref):
        assert len(rs) > 0
        np.testing.assert_array_equal(got[i], rs, err_msg=f"job {i}")
