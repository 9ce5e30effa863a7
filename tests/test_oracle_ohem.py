"""Pins of the oracle's point-OHEM sampling (Sec. 3.3, Eq. 6 right): the inverse
probability formula at its closed-form cases, the counter-based generator against its
published outputs, and the weighted draw against a brute force over explicit intervals
and against the frequencies it must produce."""
import json
import math
import os

import numpy as np
import pytest

from oracle import pifu_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_point_weight_closed_forms():
    L = np.array([0.0, 0.35, 0.7, 2.1])
    # beta = 0: exp(L / alpha)
    assert np.allclose(O.ohem_point_weight(L, 0.7, 0.0), np.exp(L / 0.7), rtol=1e-15)
    # a perfectly predicted point (L = 0) has inverse probability 1 / (1 + beta)
    assert O.ohem_point_weight(np.array([0.0]), 0.7, 0.25)[0] == pytest.approx(0.8, rel=1e-15)
    # large beta bounds the weight by 1 / beta from below the cap
    assert O.ohem_point_weight(np.array([50.0]), 0.7, 0.5)[0] == pytest.approx(2.0, rel=1e-12)
    # the cap keeps the inverse probability finite
    assert O.ohem_point_weight(np.array([1e4]), 0.7, 0.0)[0] == O.OHEM_W_MAX


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))
    for c, hx in enumerate(g["outputs_hex"]):
        assert O.splitmix64(g["seed"], c) == int(hx, 16)


def _brute(weights, batch, seed, counter):
    """Explicit integer intervals [lo, hi) per index, a linear search per draw."""
    q = [int(math.floor(float(np.float32(w)) * 65536)) for w in weights]
    total = sum(q)
    out = []
    for b in range(batch):
        r = O.splitmix64(seed, counter * batch + b)
        t = (r * total) >> 64
        lo = 0
        for m, qm in enumerate(q):
            if lo <= t < lo + qm:
                out.append(m)
                break
            lo += qm
    return np.array(out)


@pytest.mark.parametrize("n,seed,counter", [(1, 3, 0), (7, 11, 2), (40, 5, 9)])
def test_sample_matches_brute_force(n, seed, counter):
    rng = np.random.default_rng(n)
    w = rng.uniform(1.0, 30.0, n).astype(np.float32)
    w[rng.integers(0, n)] = 1.0
    got = O.ohem_sample(w, 64, seed, counter)
    assert np.array_equal(got, _brute(w, 64, seed, counter))


def test_equal_weights_reduce_to_uniform_scaling():
    """With n equal weights every interval has the same length: index = floor(r n / 2^64)."""
    n, batch = 13, 200
    got = O.ohem_sample(np.full(n, 3.5, np.float32), batch, 21, 4)
    want = [(O.splitmix64(21, 4 * batch + b) * n) >> 64 for b in range(batch)]
    assert np.array_equal(got, want)


def test_one_weight_dominates():
    w = np.ones(10, np.float32)
    w[6] = O.OHEM_W_MAX
    got = O.ohem_sample(w, 500, 1, 0)
    assert np.mean(got == 6) > 0.999


def test_frequencies_follow_the_weights():
    w = np.array([1, 2, 4, 8, 16, 1, 1, 32], np.float32)
    got = O.ohem_sample(w, 40000, 123, 0)
    freq = np.bincount(got, minlength=w.size) / got.size
    expect = w / w.sum()
    # chi-square with 7 degrees of freedom: 99.9% quantile 24.3
    chi2 = float(np.sum((freq - expect) ** 2 / expect) * got.size)
    assert chi2 < 24.3, chi2
