"""The seeded generators: determinism, minimum separation, neutrality, density."""
import math

import numpy as np
import pytest

from paper_1611_04474_amd import workloads as W


def _min_sep_sample(s, n_check=400, seed=0):
    rng = np.random.default_rng(seed)
    L = s.box
    idx = rng.choice(s.n, min(n_check, s.n), replace=False)
    p = s.pos.astype(np.float64)
    best = np.inf
    for i in idx:
        d = p - p[i]
        d -= L * np.round(d / L)
        r2 = (d * d).sum(axis=1)
        r2[i] = np.inf
        best = min(best, r2.min())
    return math.sqrt(best)


def test_same_seed_same_arrays():
    a = W.gen_system(2000, (30.0, 30.0, 30.0), 9)
    b = W.gen_system(2000, (30.0, 30.0, 30.0), 9)
    for x, y in ((a.pos, b.pos), (a.types, b.types), (a.charges, b.charges), (a.sigma, b.sigma)):
        assert np.array_equal(x, y)
    c = W.gen_system(2000, (30.0, 30.0, 30.0), 10)
    assert not np.array_equal(a.pos, c.pos)


@pytest.mark.parametrize("make", [W.small_system, W.apoa1_system])
def test_config_shapes(make):
    s = make()
    assert s.pos.dtype == np.float32 and s.types.dtype == np.int32 and s.charges.dtype == np.float32
    assert np.all(s.pos >= 0) and np.all(s.pos < s.box.astype(np.float32))
    assert np.all(s.box == s.box.astype(np.float32).astype(np.float64))
    assert s.types.min() >= 0 and s.types.max() < W.N_TYPES
    assert np.all((s.sigma >= 2) & (s.sigma <= 4)) and np.all((s.epsilon >= 0.01) & (s.epsilon <= 0.2))
    assert abs(s.charges.astype(np.float64).sum()) < 1e-3 * s.n ** 0.5
    assert _min_sep_sample(s) >= 1.0 - 1e-4


def test_densities():
    s = W.small_system()
    assert s.n / np.prod(s.box) == pytest.approx(3000 / 27000, rel=1e-6)
    s = W.apoa1_system()
    assert s.n / np.prod(s.box) == pytest.approx(0.1, rel=0.002)


def test_serving_trace():
    reqs, table = W.serving_trace()
    sizes = np.array([r.n for r in reqs])
    assert len(reqs) == 512 and sizes.min() >= 2000 and sizes.max() <= 200000
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) >= 0)
    assert 512 / arr[-1] == pytest.approx(200.0, rel=0.15)
    s = W.request_system(reqs[3], table)
    assert s.n == reqs[3].n and s.n / np.prod(s.box) == pytest.approx(0.1, rel=0.01)
    assert np.array_equal(s.sigma, table[0])
    s2 = W.request_system(reqs[3], table)
    assert np.array_equal(s.pos, s2.pos)


def test_perturbation_stream():
    s = W.small_system()
    a = [d.copy() for d in W.perturbation_stream(s.n, 3)]
    b = [d.copy() for d in W.perturbation_stream(s.n, 3)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert a[0].std() == pytest.approx(0.01, rel=0.05)
    p = W.perturb(s.pos, a[0])
    assert p.dtype == np.float32
