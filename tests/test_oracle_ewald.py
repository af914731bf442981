"""Pins for the oracle's Ewald summation of the Coulomb energy beyond the cutoff (the
long-range part that Section 2.1 leaves to an O(N) approximation outside the short-range
kernel): the rock-salt Madelung constant, independence of the total from the splitting
parameter alpha (with and without net charge, in a non-cubic box), and forces equal to
minus the gradient of the total energy."""
import math

import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import workloads as W

K = W.COULOMB_K
MADELUNG_NACL = 1.747564594633     # rock salt, referred to the nearest-neighbour distance


def ewald_params(box, alpha, rc=12.0, sigma=(1.0,), eps=(0.0,)):
    return dict(box=tuple(box), r_cut=rc, r_switch=rc, coulomb_k=K, sigma=np.array(sigma, float),
                epsilon=np.array(eps, float), flags=oracle.FLAG_EWALD, ewald_alpha=alpha)


def kmax_for(box, alpha, tol=1e-13):
    """Smallest per-axis wave-vector range whose first omitted term exp(-pi^2 h^2/alpha^2)
    is below tol."""
    h = alpha * math.sqrt(-math.log(tol)) / math.pi
    return [int(math.ceil(h * L)) for L in box]


def total_coulomb(p, pos, q, kmax):
    """Real-space sum inside the cutoff + reciprocal + self + background: energy, forces."""
    t = np.zeros(len(q), np.int32)
    real = oracle.forces(p, pos, t, q, "bruteforce")
    F, er, es, eb = oracle.ewald_recip(p, pos, q, kmax)
    return real.energy + er + es + eb, real.force + F, (real.energy, er, es, eb)


def rock_salt(n_cells, a):
    basis_na = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    basis_cl = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    pos, q = [], []
    for i in range(n_cells):
        for j in range(n_cells):
            for k in range(n_cells):
                for b, s in ((basis_na, 1.0), (basis_cl, -1.0)):
                    for f in b:
                        pos.append(((i + f[0]) * a + 0.01, (j + f[1]) * a + 0.01, (k + f[2]) * a + 0.01))
                        q.append(s)
    return np.array(pos), np.array(q)


def test_rock_salt_madelung_constant():
    """512 ions of rock salt (4x4x4 conventional cells, nearest neighbours 3.1 A apart):
    E = -(N/2) M k q^2 / d with M = 1.747565, and every force vanishes by symmetry."""
    a = 6.2
    pos, q = rock_salt(4, a)
    box = (4 * a,) * 3
    alpha = 0.38
    p = ewald_params(box, alpha)
    E, F, parts = total_coulomb(p, pos, q, kmax_for(box, alpha))
    expect = -(len(q) / 2) * MADELUNG_NACL * K / (a / 2)
    assert E == pytest.approx(expect, rel=1e-8), parts
    assert np.abs(F).max() < 1e-7 * K / (a / 2) ** 2


@pytest.mark.parametrize("net", [0.0, 1.3])
def test_total_independent_of_alpha(net):
    """The split between real and reciprocal space is arbitrary: two splitting parameters
    give the same total energy and forces (a neutral system, and one with net charge, where
    the neutralising-background term is what keeps the total independent of alpha)."""
    rng = np.random.default_rng(17)
    box = (24.5, 26.0, 31.0)
    n = 100
    pos = rng.uniform(0, 1, (n, 3)) * np.array(box)
    q = rng.normal(0, 0.6, n)
    q += (net - q.sum()) / n
    res = []
    for alpha in (0.34, 0.40):
        p = ewald_params(box, alpha)
        res.append(total_coulomb(p, pos, q, kmax_for(box, alpha)))
    (E1, F1, parts1), (E2, F2, parts2) = res
    assert abs(parts1[1] - parts2[1]) > 1e-3 * abs(E1)      # the split really differs
    # agreement to the real-space truncation at the cutoff (erfc(0.34 x 12) = 6e-9)
    assert E1 == pytest.approx(E2, rel=1e-8)
    if net:
        assert abs(parts1[3] - parts2[3]) > 1e3 * 1e-8 * abs(E1)   # the background term matters
    np.testing.assert_allclose(F1, F2, rtol=0, atol=1e-7 * np.abs(F1).max())


def test_forces_are_minus_energy_gradient():
    """Every force component of the total (real + reciprocal) equals minus the central
    difference of the total energy."""
    rng = np.random.default_rng(5)
    box = (24.5, 25.0, 27.0)
    n = 40
    pos = rng.uniform(0, 1, (n, 3)) * np.array(box)
    q = rng.normal(0, 0.5, n)
    q -= q.mean()
    alpha = 0.3
    p = ewald_params(box, alpha)
    km = kmax_for(box, alpha)
    E0, F0, _ = total_coulomb(p, pos, q, km)
    h = 1e-5
    for i in (0, 7, 23):
        for d in range(3):
            pp = pos.copy(); pp[i, d] += h
            pm = pos.copy(); pm[i, d] -= h
            g = -(total_coulomb(p, pp, q, km)[0] - total_coulomb(p, pm, q, km)[0]) / (2 * h)
            assert F0[i, d] == pytest.approx(g, rel=1e-6, abs=1e-6 * np.abs(F0).max())


def test_real_space_term_limits():
    """The real-space pair term is the Coulomb law screened by erfc(alpha r): for a tiny
    alpha it is Eq. 2 itself, and at alpha r = 2 it carries erfc(2) = 0.004677735 of it."""
    r = 6.0
    for alpha, frac in ((1e-9, 1.0), (2.0 / r, 0.004677734981047266)):
        p = ewald_params((30.0, 30.0, 30.0), alpha)
        e, f = oracle.pair_terms(p, 0, 0, 0.5, -0.8, r * r)
        assert e == pytest.approx(frac * K * 0.5 * -0.8 / r, rel=1e-7)
    p0 = ewald_params((30.0, 30.0, 30.0), 1e-9)
    e, f = oracle.pair_terms(p0, 0, 0, 0.5, -0.8, r * r)
    assert f * r == pytest.approx(K * 0.5 * -0.8 / r ** 2, rel=1e-7)    # Eq. 2 magnitude
