"""Pins of the oracle's counter-based generator: published Philox4x32-10
known-answer vectors, and the distribution of the uniforms and normals."""
import os

import numpy as np
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(a, 16) for a in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(orc.philox4x32_10(ctr, key)) == out


def test_u53_bit_layout(orc):
    """u53 = top 53 bits of (out0 << 32 | out1) for counter (e, stream), key seed."""
    seed, stream = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    U = orc.u53(seed, stream, 3)
    for e in range(3):
        o = orc.philox4x32_10([e, 0, stream & 0xFFFFFFFF, stream >> 32],
                              [seed & 0xFFFFFFFF, seed >> 32])
        assert int(U[e]) == ((int(o[0]) << 32) | int(o[1])) >> 11
    assert int(U.max()) < (1 << 53)


def test_uniforms_distribution(orc):
    u = orc.uniforms(5, 77, 200_000)
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_normals_distribution(orc):
    z = orc.normals(11, 3, 50_000, 7)
    flat = z.ravel()
    assert abs(flat.mean()) < 4 / np.sqrt(flat.size)
    assert abs(flat.var() - 1.0) < 4 * np.sqrt(2.0 / flat.size)
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    # columns are uncorrelated (including the two halves of one Box-Muller pair)
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(7)).max() < 5 / np.sqrt(50_000)


def test_streams_are_distinct(orc):
    a = orc.u53(1, 1, 1000)
    b = orc.u53(1, 2, 1000)
    c = orc.u53(2, 1, 1000)
    assert len(set(a.tolist()) & set(b.tolist())) == 0
    assert len(set(a.tolist()) & set(c.tolist())) == 0


def test_init_prior_moments(orc):
    mean = np.array([0.0, 1.0, -2.0])
    sd = np.array([1.0, 5.0, 0.5])
    th = orc.init_prior(mean, sd, 100_000, seed=3, stream=1)
    assert np.all(np.abs(th.mean(0) - mean) < 4 * sd / np.sqrt(100_000))
    assert np.all(np.abs(th.std(0) / sd - 1) < 4 * np.sqrt(0.5 / 100_000))
