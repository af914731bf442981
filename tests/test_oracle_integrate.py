"""Pins of the oracle's motion update (velocity Verlet around the force call), each against
something other than its own formulas: exact free flight, the kinetic-energy unit from
physical constants, time reversibility, and second-order energy error on an LJ dimer."""
import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import workloads as W


def _free_params():
    return dict(box=(30.0, 30.0, 30.0), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
                sigma=np.array([2.0]), epsilon=np.array([0.0]), flags=0)


def test_free_flight_is_exact():
    # no LJ and no charges: no force, so x(t) = x0 + v t (mod L) and v, KE stay constant
    rng = np.random.default_rng(0)
    n = 50
    x0 = rng.uniform(0, 30, (n, 3))
    v0 = rng.normal(0, 0.01, (n, 3))
    im = np.full(n, 1 / 12.0)
    x, v, F, pe, ke = oracle.vv_steps(_free_params(), x0, v0, np.zeros(n, np.int32),
                                      np.zeros(n), im, 1.0, 10, method="bruteforce")
    assert np.array_equal(v, v0) and np.all(F == 0) and np.all(pe == 0)
    assert np.abs(np.mod(x0 + 10.0 * v0, 30.0) - x).max() < 1e-12
    assert np.allclose(ke, ke[0], rtol=0, atol=0)


def test_kinetic_energy_unit_from_physical_constants():
    # 1 amu at 1 A/fs: m v^2 / 2 with m = 1.66053906660e-27 kg, v = 1e5 m/s, times N_A,
    # in kcal (4184 J)
    expect = 0.5 * 1.66053906660e-27 * 1e5 ** 2 * 6.02214076e23 / 4184.0
    got = oracle.kinetic_energy(np.array([[1.0, 0.0, 0.0]]), np.array([1.0]))
    assert got == pytest.approx(expect, rel=1e-9)


def _lattice_system(n=200, L=30.0, seed=3):
    rng = np.random.default_rng(seed)
    g = np.arange(6) * 5.0
    pos = np.array([[a, b, c] for a in g for b in g for c in g])[:n] + rng.uniform(-0.3, 0.3, (n, 3))
    p = dict(box=(L, L, L), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([2.5, 3.0]), epsilon=np.array([0.1, 0.15]), flags=0)
    t = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.3, n)
    q -= q.mean()
    im = 1.0 / np.where(t == 0, 12.0, 16.0)
    v = rng.normal(0, 0.005, (n, 3))
    return p, pos, v, t, q, im


def test_time_reversible():
    # velocity Verlet is symmetric in time: n steps, reversed velocities, n steps back
    p, x0, v0, t, q, im = _lattice_system()
    x1, v1, _, pe, ke = oracle.vv_steps(p, x0, v0, t, q, im, 1.0, 20)
    x2, v2, _, _, _ = oracle.vv_steps(p, x1, -v1, t, q, im, 1.0, 20)
    d = x2 - np.mod(x0, 30.0)
    d -= 30.0 * np.round(d / 30.0)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v2 + v0).max() < 1e-12
    assert np.abs(v1 - v0).max() > 1e-4          # the atoms did move under forces


def test_energy_error_is_second_order():
    # LJ dimer released at rest beyond the minimum: the largest deviation of E = PE + KE
    # from its start shrinks 4x when dt halves (a first-order scheme would give 2x)
    p = dict(box=(40.0, 40.0, 40.0), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([3.0]), epsilon=np.array([0.2]), flags=0)
    x0 = np.array([[10.0, 10.0, 10.0], [13.6, 10.0, 10.0]])
    t = np.zeros(2, np.int32)
    q = np.zeros(2)
    im = np.full(2, 1 / 12.0)
    e0 = oracle.forces(p, x0, t, q, "bruteforce").energy
    err = []
    for dt in (1.0, 0.5):
        _, _, _, pe, ke = oracle.vv_steps(p, x0, np.zeros((2, 3)), t, q, im, dt,
                                          int(round(400.0 / dt)), method="bruteforce")
        assert pe.min() < -0.19          # it oscillates through the well (depth 0.2)
        err.append(np.max(np.abs(pe + ke - e0)))
    assert 3.5 < err[0] / err[1] < 4.5, err
