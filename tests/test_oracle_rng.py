"""Pins of the oracle's random-number plumbing and samplers.

Philox is pinned to the published known-answer vectors; the direction and
source-radius samplers to moments and CDFs that follow from their densities
(Sec. 4.4 uniform directions, Sec. 4.4.4 hemisphere, Sec. 4.6 source radius
with density proportional to the ball Green's function of App. A.1).
"""
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert list(O.philox(ctr, key)) == out


def test_uniform_grid_and_moments():
    U = np.array([O.uniforms(7, i, 3, 5, 0) for i in range(20000)]).ravel()
    assert U.min() >= 0.0 and U.max() < 1.0
    assert np.all(U * 2 ** 24 == np.floor(U * 2 ** 24))      # 24-bit grid, exact
    assert abs(U.mean() - 0.5) < 4 * math.sqrt(1 / 12 / U.size)
    assert abs(U.var() - 1 / 12) < 0.003


def test_stream_keys_are_distinct():
    a = O.uniforms(1, 0, 0, 0, 0)
    assert not np.allclose(a, O.uniforms(1, 1, 0, 0, 0))
    assert not np.allclose(a, O.uniforms(1, 0, 1, 0, 0))
    assert not np.allclose(a, O.uniforms(1, 0, 0, 1, 0))
    assert not np.allclose(a, O.uniforms(1, 0, 0, 0, 1))
    assert not np.allclose(a, O.uniforms(2, 0, 0, 0, 0))
    assert not np.allclose(a, O.uniforms(1 << 32, 0, 0, 0, 0))


def _dirs(dim, n=40000):
    rng = np.random.default_rng(1)
    u = rng.random((n, 2))
    return np.array([O.sample_direction(dim, a, b) for a, b in u])


@pytest.mark.parametrize("dim", [2, 3])
def test_direction_moments(dim):
    v = _dirs(dim)
    n = v.shape[0]
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-12)
    assert np.all(np.abs(v.mean(0)) < 4 * math.sqrt(1 / dim / n))
    C = v.T @ v / n
    assert np.allclose(C, np.eye(dim) / dim, atol=0.01)


@pytest.mark.parametrize("dim,expect", [(3, -0.5), (2, -2 / math.pi)])
def test_hemisphere_flip_mean(dim, expect):
    """Flipping v when n.v > 0 gives the hemisphere around -n: E[v.n] is
    -1/2 (3D) and -2/pi (2D)."""
    v = _dirs(dim)
    n = np.zeros(dim)
    n[-1] = 1.0
    d = v @ n
    d = np.where(d > 0, -d, d)
    assert abs(d.mean() - expect) < 4 * d.std() / math.sqrt(d.size)


def _cdf3(s):
    return 3 * s ** 2 - 2 * s ** 3


def _cdf2(s):
    return s ** 2 * (1 - 2 * np.log(np.maximum(s, 1e-300)))


@pytest.mark.parametrize("dim,mean,cdf", [(3, 0.5, _cdf3), (2, 4 / 9, _cdf2)])
def test_source_fraction_distribution(dim, mean, cdf):
    """The source distance t = s r has density proportional to
    G^B(t) t^(N-1): Beta(2,2) in 3D, -4 s ln s in 2D."""
    from scipy import stats
    rng = np.random.default_rng(2)
    u = rng.random((30000, 2))
    s = np.array([O.source_fraction(dim, a, b) for a, b in u])
    assert s.min() >= 0 and s.max() <= 1
    assert abs(s.mean() - mean) < 4 * s.std() / math.sqrt(s.size)
    assert stats.kstest(s, cdf).pvalue > 1e-3
