"""Pins for the FP64 oracle, checked against facts that do not come from the
oracle itself: textbook special values of the Lennard-Jones and Coulomb laws
(Eq. 1 and Eq. 2, Section 2.1), properties of the switching polynomial,
symmetry and conservation laws, finite differences of the energy, lattice sums
enumerated independently, and brute force against the cell list (Algorithm 1)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import workloads as W

K = W.COULOMB_K


def params(box=(30.0, 30.0, 30.0), rc=12.0, rs=10.0, k=K, sigma=(3.0,), eps=(0.1,), flags=0):
    return dict(box=box, r_cut=rc, r_switch=rs, coulomb_k=k, sigma=np.array(sigma, float),
                epsilon=np.array(eps, float), flags=flags)


def two_atoms(r, ti=0, tj=0, qi=0.0, qj=0.0, box=(30.0, 30.0, 30.0), axis=0, x0=5.0):
    pos = np.zeros((2, 3))
    pos[:, :] = 7.0
    pos[0, axis] = x0
    pos[1, axis] = x0 + r
    return pos, np.array([ti, tj], np.int32), np.array([qi, qj], float)


# ---------------------------------------------------------------- pair law ---

def test_lj_zero_crossing_and_minimum():
    """Textbook LJ: energy 0 at r = sigma, minimum -eps at r = 2^(1/6) sigma with zero force."""
    s, e = 3.2, 0.15
    p = params(sigma=(s,), eps=(e,), rs=12.0)           # no switching
    E0, _ = oracle.pair_terms(p, 0, 0, 0, 0, s * s)
    assert abs(E0) < 1e-12
    rmin = 2 ** (1 / 6) * s
    Em, fm = oracle.pair_terms(p, 0, 0, 0, 0, rmin * rmin)
    assert Em == pytest.approx(-e, rel=1e-12)
    assert abs(fm) < 1e-12
    # repulsive inside the minimum, attractive outside (F_i = f (x_i - x_j))
    assert oracle.pair_terms(p, 0, 0, 0, 0, (0.9 * rmin) ** 2)[1] > 0
    assert oracle.pair_terms(p, 0, 0, 0, 0, (1.1 * rmin) ** 2)[1] < 0


def test_lorentz_berthelot_mixing():
    """Mixed pair: zero crossing at (s1+s2)/2 and well depth sqrt(e1 e2)."""
    p = params(sigma=(2.2, 3.8), eps=(0.02, 0.18), rs=12.0)
    sm = 0.5 * (2.2 + 3.8)
    assert abs(oracle.pair_terms(p, 0, 1, 0, 0, sm * sm)[0]) < 1e-12
    rmin = 2 ** (1 / 6) * sm
    assert oracle.pair_terms(p, 1, 0, 0, 0, rmin * rmin)[0] == pytest.approx(-math.sqrt(0.02 * 0.18), rel=1e-12)


def test_lj_force_matches_eq1_constants():
    """Eq. 1 with A = 48 eps s^12, B = 24 eps s^6: |F| = A/r^13 - B/r^7 at r = 3 A."""
    s, e, r = 3.0, 0.1, 3.0
    p = params(sigma=(s,), eps=(e,))
    _, f = oracle.pair_terms(p, 0, 0, 0, 0, r * r)
    A, B = 48 * e * s ** 12, 24 * e * s ** 6
    assert f * r == pytest.approx(A / r ** 13 - B / r ** 7, rel=1e-12)


def test_coulomb_law():
    """Eq. 2: energy k q1 q2 / r, force magnitude k q1 q2 / r^2, like charges repel."""
    p = params(eps=(0.0,))
    for qi, qj in ((1.0, 1.0), (0.5, -0.7)):
        for r in (1.5, 3.0, 9.9):
            E, f = oracle.pair_terms(p, 0, 0, qi, qj, r * r)
            assert E == pytest.approx(K * qi * qj / r, rel=1e-13)
            assert f * r == pytest.approx(K * qi * qj / r ** 2, rel=1e-13)
    assert oracle.pair_terms(p, 0, 0, 1, 1, 9.0)[1] > 0
    assert oracle.pair_terms(p, 0, 0, 1, -1, 9.0)[1] < 0


def test_cutoff_is_strict():
    p = params(eps=(0.0,))
    assert oracle.pair_terms(p, 0, 0, 1, 1, 144.0) == (0.0, 0.0)
    assert oracle.pair_terms(p, 0, 0, 1, 1, 200.0) == (0.0, 0.0)
    E, f = oracle.pair_terms(p, 0, 0, 1, 1, np.nextafter(144.0, 0.0))
    assert E != 0.0 and f != 0.0
    # two atoms exactly rc apart along x do not interact; just inside they do
    pos, t, q = two_atoms(12.0, qi=1, qj=1)
    r = oracle.forces(p, pos, t, q, "bruteforce")
    assert r.n_pairs == 0 and np.all(r.force == 0)
    pos, t, q = two_atoms(11.999, qi=1, qj=1)
    assert oracle.forces(p, pos, t, q, "bruteforce").n_pairs == 1


def test_switch_polynomial_properties():
    """Smoothstep from rs^2 to rc^2: S = 1 up to rs^2, 1/2 at the midpoint,
    S(u) + S(rs^2 + rc^2 - u) = 1, and 0 at rc^2 (read off a Coulomb pair)."""
    p = params(eps=(0.0,))
    rs2, rc2 = 100.0, 144.0

    def S(u):
        E, _ = oracle.pair_terms(p, 0, 0, 1, 1, u)
        return E / (K / math.sqrt(u))

    assert S(rs2) == 1.0
    assert S(50.0) == 1.0
    assert S(0.5 * (rs2 + rc2)) == pytest.approx(0.5, abs=1e-14)
    for u in (101.0, 110.0, 120.0, 133.0, 143.0):
        assert S(u) + S(rs2 + rc2 - u) == pytest.approx(1.0, abs=1e-13)
        assert 0.0 < S(u) < 1.0
    assert S(np.nextafter(rc2, 0)) < 1e-25
    us = np.linspace(100.0, 143.9, 200)
    vals = [S(u) for u in us]
    assert all(a >= b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("r", [3.0, 9.5, 10.0, 10.0001, 11.0, 11.9])
@pytest.mark.parametrize("flags", [0, oracle.FLAG_TRUNCATED_COULOMB])
def test_force_is_minus_energy_gradient_pair(r, flags):
    """F = -dE/dr by central differences, inside, at and across the switching region."""
    p = params(sigma=(2.6,), eps=(0.12,), flags=flags)
    h = 1e-6

    def E(rr):
        return oracle.pair_terms(p, 0, 0, 0.4, -0.3, rr * rr)[0]

    _, f = oracle.pair_terms(p, 0, 0, 0.4, -0.3, r * r)
    dEdr = (E(r + h) - E(r - h)) / (2 * h)
    # at r = rs the second derivative jumps, so the central difference is O(h) there
    tol = 2e-5 if r == 10.0 else 1e-6
    assert f * r == pytest.approx(-dEdr, rel=tol, abs=1e-9)


def test_switch_continuity_at_rs():
    """Energy and force are continuous at rs (C1 switching)."""
    p = params(sigma=(2.6,), eps=(0.12,))
    below = oracle.pair_terms(p, 0, 0, 0.4, 0.3, np.nextafter(100.0, 0.0))
    above = oracle.pair_terms(p, 0, 0, 0.4, 0.3, np.nextafter(100.0, 200.0))
    assert above[0] == pytest.approx(below[0], rel=1e-12)
    assert above[1] == pytest.approx(below[1], rel=1e-10)


def test_truncated_coulomb_keeps_eq2_to_cutoff():
    p = params(eps=(0.0,), flags=oracle.FLAG_TRUNCATED_COULOMB)
    E, f = oracle.pair_terms(p, 0, 0, 1, 1, 121.0)
    assert E == pytest.approx(K / 11.0, rel=1e-13)
    assert f * 11.0 == pytest.approx(K / 121.0, rel=1e-13)


def test_no_switching_when_rs_equals_rc():
    p = params(rs=12.0, eps=(0.0,))
    E, _ = oracle.pair_terms(p, 0, 0, 1, 1, 143.0)
    assert E == pytest.approx(K / math.sqrt(143.0), rel=1e-14)


# ---------------------------------------------------------- whole systems ---

def test_periodic_image_pair():
    """A pair across the box face interacts exactly like the same pair inside."""
    p = params(sigma=(2.0,), eps=(0.1,))
    inner = oracle.forces(p, *two_atoms(3.0, qi=0.3, qj=-0.2, x0=10.0), "bruteforce")
    pos, t, q = two_atoms(3.0, qi=0.3, qj=-0.2, x0=28.5)
    pos[1, 0] -= 30.0                  # second atom at 1.5, seen through the face
    for method in ("bruteforce", "celllist"):
        wrap = oracle.forces(p, pos, t, q, method)
        assert wrap.n_pairs == 1
        np.testing.assert_allclose(wrap.force, inner.force, rtol=1e-12)
        assert wrap.energy == pytest.approx(inner.energy, rel=1e-12)


def _random_system(n, box, seed, sigma=(2.5, 3.0, 3.5), eps=(0.05, 0.1, 0.15)):
    rng = np.random.default_rng(seed)
    nt = len(sigma)
    # rejection sampling to keep pairs >= 1.6 A apart
    pos = []
    L = np.array(box, float)
    while len(pos) < n:
        x = rng.uniform(0, 1, 3) * L
        ok = True
        for y in pos:
            d = x - y
            d -= L * np.round(d / L)
            if d @ d < 1.6 ** 2:
                ok = False
                break
        if ok:
            pos.append(x)
    pos = np.array(pos)
    t = rng.integers(0, nt, n).astype(np.int32)
    q = rng.normal(0, 0.5, n)
    q -= q.mean()
    return pos, t, q, params(box=box, sigma=sigma, eps=eps)


def test_energy_gradient_system():
    """Every force component equals minus the central difference of the total energy."""
    pos, t, q, p = _random_system(60, (24.5, 26.0, 25.0), 7)
    r0 = oracle.forces(p, pos, t, q, "celllist")
    h = 1e-5
    rng = np.random.default_rng(3)
    for i in rng.choice(60, 12, replace=False):
        for d in range(3):
            pp = pos.copy(); pp[i, d] += h
            pm = pos.copy(); pm[i, d] -= h
            ep = oracle.forces(p, pp, t, q, "bruteforce").energy
            em = oracle.forces(p, pm, t, q, "bruteforce").energy
            g = -(ep - em) / (2 * h)
            assert r0.force[i, d] == pytest.approx(g, rel=1e-5, abs=1e-5 * (1 + abs(g)))


def test_newton_third_law_small_config():
    s = W.small_system()
    r = oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist")
    assert np.linalg.norm(r.force.sum(axis=0)) <= 1e-9 * np.abs(r.force).sum()


def test_translation_invariance():
    pos, t, q, p = _random_system(80, (25.0, 25.0, 25.0), 11)
    r0 = oracle.forces(p, pos, t, q, "celllist")
    shift = np.array([3.7, -11.2, 20.05])
    pos2 = np.mod(pos + shift, 25.0)
    r1 = oracle.forces(p, pos2, t, q, "celllist")
    np.testing.assert_allclose(r1.force, r0.force, rtol=1e-10, atol=1e-10 * np.abs(r0.force).max())
    assert r1.energy == pytest.approx(r0.energy, rel=1e-12)
    assert r1.n_pairs == r0.n_pairs


def test_cubic_symmetries():
    """Axis permutation permutes forces; the reflection x -> L - x negates F_x."""
    pos, t, q, p = _random_system(70, (26.0, 26.0, 26.0), 13)
    r0 = oracle.forces(p, pos, t, q, "celllist")
    perm = [2, 0, 1]
    r1 = oracle.forces(p, pos[:, perm], t, q, "celllist")
    np.testing.assert_allclose(r1.force, r0.force[:, perm], rtol=1e-10, atol=1e-9)
    ref = pos.copy(); ref[:, 0] = 26.0 - ref[:, 0]
    ref[ref[:, 0] >= 26.0, 0] -= 26.0
    r2 = oracle.forces(p, ref, t, q, "celllist")
    exp = r0.force.copy(); exp[:, 0] *= -1
    np.testing.assert_allclose(r2.force, exp, rtol=1e-10, atol=1e-9)
    assert r2.energy == pytest.approx(r0.energy, rel=1e-12)


@pytest.mark.parametrize("box,n,seed", [
    ((24.5, 24.5, 24.5), 150, 1),      # 2x2x2 cells
    ((36.5, 36.5, 36.5), 200, 2),      # 3x3x3 cells
    ((24.5, 37.0, 50.0), 220, 3),      # mixed 2x3x4
])
def test_celllist_pairs_equal_bruteforce(box, n, seed):
    """Algorithm 1's cell list finds exactly the pairs of the O(N^2) definition."""
    pos, t, q, p = _random_system(n, box, seed)
    a = oracle.pairs(p, pos, "bruteforce")
    b = oracle.pairs(p, pos, "celllist")
    assert a.shape == b.shape and np.array_equal(a, b)
    ra = oracle.forces(p, pos, t, q, "bruteforce")
    rb = oracle.forces(p, pos, t, q, "celllist")
    assert ra.n_pairs == rb.n_pairs == a.shape[0]
    np.testing.assert_allclose(rb.force, ra.force, rtol=1e-11, atol=1e-11 * np.abs(ra.force).max())
    assert rb.energy == pytest.approx(ra.energy, rel=1e-12)
    assert np.array_equal(ra.count, rb.count)


def test_small_config_pairs_and_forces_match():
    s = W.small_system()
    p = s.params()
    a = oracle.pairs(p, s.pos, "bruteforce")
    b = oracle.pairs(p, s.pos, "celllist")
    assert np.array_equal(a, b)
    ra = oracle.forces(p, s.pos, s.types, s.charges, "bruteforce")
    rb = oracle.forces(p, s.pos, s.types, s.charges, "celllist")
    np.testing.assert_allclose(rb.force, ra.force, rtol=1e-10, atol=1e-12 * np.abs(ra.force).max())
    assert ra.energy == pytest.approx(rb.energy, rel=1e-13)


def _lattice_vectors(rmax):
    m = int(math.ceil(rmax))
    for v in itertools.product(range(-m, m + 1), repeat=3):
        d2 = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
        if 0 < d2 < rmax * rmax:
            yield v, d2


def test_simple_cubic_lattice_sum():
    """Perfect simple-cubic LJ lattice: zero force on every atom (symmetry) and an
    energy per atom equal to half the sum over integer lattice vectors inside the
    cutoff, with the textbook LJ energy 4 eps ((s/r)^12 - (s/r)^6) and no switching."""
    a, n_side = 2.5, 10                    # 25 A box, 2x2x2 cells, 1000 atoms
    L = a * n_side
    g = np.arange(n_side) * a + 0.3
    pos = np.array(list(itertools.product(g, g, g)))
    s, e = 2.7, 0.08
    p = params(box=(L, L, L), sigma=(s,), eps=(e,), rs=12.0)
    t = np.zeros(len(pos), np.int32)
    q = np.zeros(len(pos))
    r = oracle.forces(p, pos, t, q, "celllist")
    assert np.abs(r.force).max() < 1e-10
    per_atom = 0.0
    count = 0
    for v, d2 in _lattice_vectors(12.0 / a):
        rr = a * math.sqrt(d2)
        per_atom += 4 * e * ((s / rr) ** 12 - (s / rr) ** 6)
        count += 1
    assert r.energy == pytest.approx(0.5 * len(pos) * per_atom, rel=1e-12)
    assert np.all(r.count == count)
    assert r.n_pairs == len(pos) * count // 2


def test_rock_salt_lattice_sum():
    """Alternating +/- charges on a cubic lattice (rock salt): zero forces, and the
    Coulomb energy per ion is half the switched lattice sum over integer vectors,
    with charge sign (-1)^(i+j+k) and the smoothstep evaluated independently."""
    a, n_side = 2.5, 10
    L = a * n_side
    idx = np.array(list(itertools.product(range(n_side), repeat=3)))
    pos = idx * a + 0.1
    q = np.where(idx.sum(axis=1) % 2 == 0, 1.0, -1.0)
    p = params(box=(L, L, L), eps=(0.0,))
    t = np.zeros(len(pos), np.int32)
    r = oracle.forces(p, pos, t, q, "celllist")
    assert np.abs(r.force).max() < 1e-9
    rs2, rc2 = 100.0, 144.0
    per_ion = 0.0
    for v, d2 in _lattice_vectors(12.0 / a):
        u = a * a * d2
        x = min(max((u - rs2) / (rc2 - rs2), 0.0), 1.0)
        sw = 1 - 3 * x * x + 2 * x ** 3       # smoothstep from 1 to 0
        sign = -1.0 if (v[0] + v[1] + v[2]) % 2 else 1.0
        per_ion += sign * K / math.sqrt(u) * sw
    assert r.energy == pytest.approx(0.5 * len(pos) * per_ion, rel=1e-12)


def test_subset_matches_full():
    s = W.small_system()
    p = s.params()
    full = oracle.forces(p, s.pos, s.types, s.charges, "celllist")
    idx = np.array([0, 17, 512, 2999])
    sub = oracle.forces_subset(p, s.pos, s.types, s.charges, idx)
    np.testing.assert_allclose(sub.force, full.force[idx], rtol=1e-11, atol=1e-6)
    assert np.array_equal(sub.count, full.count[idx])


def test_grid_rule():
    assert oracle.grid(params(box=(30.0, 30.0, 30.0))) == (2, 2, 2)
    assert oracle.grid(params(box=tuple(W.f32_box(W.APOA1_BOX)))) == (9, 9, 6)
    assert oracle.grid(params(box=tuple(W.f32_box(W.STMV_BOX)))) == (18, 18, 18)
    # cell edge within 1e-3 A of the cutoff: one cell fewer
    assert oracle.grid(params(box=(36.002, 36.0, 30.0))) == (2, 2, 2)
    for bad in ((23.9, 30.0, 30.0), (24.0005, 30.0, 30.0)):   # < 2 cells after the margin
        with pytest.raises(oracle.OracleError):
            oracle.grid(params(box=bad))


def test_canonicalize_float32_rounding():
    box = np.array([30.0, 30.0, 30.0])
    pos = np.array([[-1e-3, 30.0, 59.99], [-30.0, 0.0, 12.0]], np.float32)
    out, st = oracle.canonicalize(pos, box)
    assert st == 0
    assert out[0, 0] == float(np.float32(-1e-3) + np.float32(30.0))
    assert out[0, 1] == 0.0
    assert out[0, 2] == float(np.float32(59.99) - np.float32(30.0))
    assert out[1, 0] == 0.0
    _, st = oracle.canonicalize(np.array([[np.nan, 0, 0]], np.float32), box)
    assert st & oracle.STATUS_NAN
    _, st = oracle.canonicalize(np.array([[60.0, 0, 0]], np.float32), box)
    assert st & oracle.STATUS_OUT_OF_BOX


def test_pair_count_small_config():
    """Density ~0.111 and rc = 12: the within-cutoff pair count of the 3,000-atom
    system lies near N^2 rho (4/3) pi rc^3 / (2 N) per atom (uniform-density estimate)."""
    s = W.small_system()
    r = oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist")
    est = 0.5 * s.n * (s.n / 27000.0) * 4 / 3 * math.pi * 12.0 ** 3
    assert abs(r.n_pairs / est - 1) < 0.01


def test_small_config_golden():
    """Regression against the stored oracle output for the 3,000-atom system."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small_system_oracle.json")))
    s = W.small_system()
    r = oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist")
    assert r.n_pairs == g["n_pairs"] == 1201501
    assert r.energy == pytest.approx(g["energy"], rel=1e-12)
    np.testing.assert_allclose(r.force[g["atoms"]], np.array(g["forces"]), rtol=1e-10, atol=1e-6)


# ------------------------------------------------- parity scaffolding ----
# Two oracle outputs decide how strict the GPU parity bars are: the per-atom sum of
# pair-force magnitudes (the denominator of the normalised force error) and the atoms
# with a partner in the float32/float64 cutoff band (excused from the exact partner-count
# check). Both are pinned here to closed forms and to an independent enumeration.

def _eq12_magnitude(s, e, qi, qj, r):
    """|F| of one pair from Eq. 1 and Eq. 2 (inside the switching radius): LJ with
    A = 48 eps s^12, B = 24 eps s^6, plus Coulomb k qi qj / r^2."""
    A = 48 * e * s ** 12
    B = 24 * e * s ** 6
    return abs(A / r ** 13 - B / r ** 7 + K * qi * qj / r ** 2)


@pytest.mark.parametrize("r", [2.9, 3.3, 6.0, 9.9])
@pytest.mark.parametrize("method", ["bruteforce", "celllist"])
def test_abs_sum_two_atoms_equals_force_magnitude(r, method):
    """With one partner the sum of pair-force magnitudes is |F_i| itself, and |F_i| is
    the Eq. 1 + Eq. 2 magnitude (|f| u in place of |f| sqrt(u) would miss by a factor r)."""
    s, e = 3.1, 0.12
    p = params(sigma=(s,), eps=(e,))
    pos, t, q = two_atoms(r, qi=0.4, qj=-0.3, axis=1)
    res = oracle.forces(p, pos, t, q, method)
    mag = _eq12_magnitude(s, e, 0.4, -0.3, r)
    assert res.abs_sum[0] == pytest.approx(mag, rel=1e-12)
    assert res.abs_sum[1] == pytest.approx(mag, rel=1e-12)
    assert np.linalg.norm(res.force[0]) == pytest.approx(mag, rel=1e-12)
    sub = oracle.forces_subset(p, pos, t, q, [1])
    assert sub.abs_sum[0] == pytest.approx(mag, rel=1e-12)


@pytest.mark.parametrize("method", ["bruteforce", "celllist"])
def test_abs_sum_three_collinear_atoms(method):
    """Three atoms on a line, 3.4 A apart, the middle one with two equal partners: its
    force cancels exactly while its magnitude sum is twice the pair magnitude; an end
    atom sums its near partner (3.4 A) and its far one (6.8 A)."""
    s, e, d = 3.0, 0.1, 3.4
    p = params(sigma=(s,), eps=(e,))
    pos = np.full((3, 3), 9.0)
    pos[:, 0] = [4.0, 4.0 + d, 4.0 + 2 * d]
    t = np.zeros(3, np.int32)
    q = np.array([0.25, 0.5, 0.25])
    res = oracle.forces(p, pos, t, q, method)
    near = _eq12_magnitude(s, e, 0.25, 0.5, d)
    far = _eq12_magnitude(s, e, 0.25, 0.25, 2 * d)
    assert np.linalg.norm(res.force[1]) < 1e-12 * near
    assert res.abs_sum[1] == pytest.approx(2 * near, rel=1e-12)
    assert res.abs_sum[0] == pytest.approx(near + far, rel=1e-12)
    assert res.abs_sum[2] == pytest.approx(near + far, rel=1e-12)
    assert list(res.count) == [2, 2, 2]


def _band_enumeration(p, pos, band):
    """Independent count of partners with |u - rc^2| <= band, every pair by minimum image
    in numpy (no cells): per atom, and unique pairs."""
    L = np.asarray(p["box"], float)
    x = np.asarray(pos, float)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    u = (d * d).sum(axis=2)
    inb = np.abs(u - p["r_cut"] ** 2) <= band
    np.fill_diagonal(inb, False)
    return inb.sum(axis=1), int(np.triu(inb, 1).sum())


@pytest.mark.parametrize("box,seed", [((24.5, 24.5, 24.5), 21), ((24.5, 37.0, 50.0), 22)])
def test_band_atoms_match_enumeration(box, seed):
    """The band finder against a plain enumeration, on a 2x2x2 and a mixed 2x3x4 grid, with
    a wide band (so that many pairs fall in it, also across every periodic face) and with
    the 8-ulp float32 band around rc^2 = 144."""
    pos, t, q, p = _random_system(260, box, seed)
    for band in (3.0, 0.4, 8 * 2.0 ** (7 - 23)):
        per, tot = oracle.band_atoms(p, pos, band)
        eper, etot = _band_enumeration(p, pos, band)
        assert np.array_equal(per, eper), band
        assert tot == etot
    per, tot = oracle.band_atoms(p, pos, 3.0)
    assert tot > 50 and per.sum() == 2 * tot


def test_band_atoms_constructed_pairs():
    """Pairs placed a few float32 ulps of rc^2 from the cutoff are in the band, pairs
    beyond it are not; across a periodic face as inside the box."""
    ulp = 2.0 ** (7 - 23)                       # float32 ulp of 144
    band = 8 * ulp
    p = params(box=(40.0, 40.0, 40.0))
    rows = []
    # (x_i, distance^2 - rc^2): inside the box, and through the x face at 0 / 40
    for k, (x0, du) in enumerate([(3.0, 2 * ulp), (3.0, -2 * ulp), (3.0, 7.5 * ulp),
                                  (3.0, 30 * ulp), (34.0, -3 * ulp), (34.0, 40 * ulp)]):
        r = math.sqrt(144.0 + du)
        y = 2.0 + 4.5 * k
        rows.append(((x0, y, 5.0), ((x0 + r) % 40.0, y, 5.0)))
    pos = np.array([a for pr in rows for a in pr])
    expect_in = [True, True, True, False, True, False]
    per, tot = oracle.band_atoms(p, pos, band)
    eper, etot = _band_enumeration(p, pos, band)
    assert np.array_equal(per, eper)
    for k, want in enumerate(expect_in):
        assert per[2 * k] == per[2 * k + 1] == int(want), k
    assert tot == sum(expect_in)


def test_canonicalize_float64_wrap_branches():
    """float64 inputs: [-L, 0) gets +L, [L, 2L) gets -L, both exactly; outside, NaN flagged."""
    box = np.array([30.0, 20.0, 10.0])
    pos = np.array([[-29.5, 20.0, 19.25], [-1e-9, 39.0, 0.0]])
    out, st = oracle.canonicalize(pos, box)
    assert st == 0
    np.testing.assert_array_equal(out, [[0.5, 0.0, 9.25], [-1e-9 + 30.0, 19.0, 0.0]])
    _, st = oracle.canonicalize(np.array([[-30.0001, 0.0, 0.0]]), box)
    assert st == oracle.STATUS_OUT_OF_BOX
    _, st = oracle.canonicalize(np.array([[0.0, 40.0, 0.0]]), box)
    assert st == oracle.STATUS_OUT_OF_BOX
    _, st = oracle.canonicalize(np.array([[0.0, 0.0, np.nan]]), box)
    assert st == oracle.STATUS_NAN
