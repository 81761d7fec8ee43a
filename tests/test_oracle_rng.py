"""Pins of the counter-based RNG used by every workload (oracle side)."""
import os

import numpy as np

from oracle import core
from paper_1810_11765_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_kat.txt")
GAMMA = 0x9E3779B97F4A7C15


def _kat():
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            s, k, out = (int(t) for t in line.split())
            yield s, k, out


def test_splitmix64_known_answers_oracle():
    for s, k, out in _kat():
        assert core.splitmix64((s + k * GAMMA) % 2**64) == out


def test_splitmix64_known_answers_inputs_module():
    for s, k, out in _kat():
        assert int(inputs.splitmix64(np.uint64((s + k * GAMMA) % 2**64))) == out


def test_ctr_is_the_stated_composition_and_matches_inputs_module():
    rng = np.random.default_rng(0)
    for _ in range(200):
        seed, step, ident, stream = (int(v) for v in rng.integers(0, 2**63, 4))
        stream %= 256
        want = core.ctr(seed, step, ident, stream)
        assert int(inputs.ctr(seed, step, np.array([ident], dtype=np.uint64), stream)[0]) == want


def test_u01_is_exact_24_bit_grid():
    h = inputs.ctr(42, 0, np.arange(100000, dtype=np.uint64), 0)
    u = inputs.u01(h)
    assert u.dtype == np.float32
    assert (u >= 0).all() and (u < 1).all()
    k = u.astype(np.float64) * 2**24
    assert np.array_equal(k, np.round(k))          # exactly k / 2^24
    assert abs(u.mean() - 0.5) < 0.01


def test_bernoulli_thresholds():
    assert inputs.threshold(0.3) == 5033165
    assert inputs.threshold(0.2) == 3355443
    assert inputs.threshold(0.25) == 4194304
    g = inputs.life_initial(42, 512, 512)
    assert abs(g.mean() - 0.3) < 0.005
    k = inputs.wator_initial(42, 1024, 1024)
    assert abs((k == 1).mean() - 0.2) < 0.003 and abs((k == 2).mean() - 0.05) < 0.002
