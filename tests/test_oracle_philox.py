"""Pins of the oracle's Philox4x32-10 against something other than itself.

* rocRAND's philox4x32_10 engine (a library implementation of the same
  published generator, Salmon et al. SC'11) compiled as a host program: the
  oracle must give identical words for arbitrary counters and keys.
* Statistical sanity of the output words (uniformity, bit balance).
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

HIPCC = "/opt/rocm/bin/hipcc"
ROCRAND_H = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// rocRAND maps (seed, subsequence, offset) to key = seed, counter words 2-3 =
// subsequence, counter words 0-1 = offset / 4 (offset a multiple of 4).
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_prog():
    if not (os.path.exists(HIPCC) and os.path.exists(ROCRAND_H)):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp(prefix="philox_pin_")
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(PROG)
    subprocess.check_call([HIPCC, "-O1", src, "-o", exe], stderr=subprocess.DEVNULL)
    return exe


def _cases(n, seed=7):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64)
    c[:, 1] %= 2**30            # rocRAND's offset argument must not overflow
    fixed = np.array([[0, 0, 0, 0, 0, 0], [1, 2, 3, 4, 5, 6], [2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1,
                      2**32 - 1, 2**32 - 1], [12345, 77, 1, 0, 3, 0], [714239, 178559, 2, 0, 3, 0]],
                     dtype=np.uint64)
    return np.concatenate([fixed, c]).astype(np.uint32)


def test_philox_matches_rocrand(oracle_mod, rocrand_prog):
    cases = _cases(2000)
    inp = "\n".join(" ".join("%x" % v for v in row) for row in cases) + "\n"
    out = subprocess.run([rocrand_prog], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()], dtype=np.uint32)
    got = np.array([oracle_mod.philox(r[:4], r[4:]) for r in cases])
    assert ref.shape == got.shape
    np.testing.assert_array_equal(got, ref)


def test_philox_statistics(oracle_mod):
    # 40000 draws x 4 words: top-byte histogram chi^2 and per-bit balance
    words = np.array([oracle_mod.philox([i, 3, 1, 0], [11, 0]) for i in range(40000)], dtype=np.uint32).ravel()
    hist = np.bincount(words >> 24, minlength=256)
    exp = words.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 400  # 255 dof: mean 255, sd 22.6
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(words.size))


def test_philox_counter_sensitivity(oracle_mod):
    # flipping any single counter or key bit changes about half of the output bits
    base = oracle_mod.philox([5, 6, 7, 8], [9, 10])
    for word in range(6):
        for bit in (0, 13, 31):
            v = [5, 6, 7, 8, 9, 10]
            v[word] ^= 1 << bit
            o = oracle_mod.philox(v[:4], v[4:])
            diff = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, o))
            assert 32 <= diff <= 96
