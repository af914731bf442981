"""FP64 CPU oracle for the short-range non-bonded force path (ctypes binding).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package. It shares no code with the
GPU library and never calls it; the two meet only on the seeded inputs.

Every function takes host numpy arrays, works in float64, and is synchronous.
See mdoracle.c for what each computation follows in the paper (Eq. 1, Eq. 2,
the cutoff of Section 2.1 and Algorithm 1).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmdoracle.so")
_lib = None

FLAG_TRUNCATED_COULOMB = 1 << 1
FLAG_EWALD = 1 << 7
STATUS_NAN = 1 << 0
STATUS_OUT_OF_BOX = 1 << 1


class _Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("r_cut", C.c_double), ("r_switch", C.c_double),
                ("coulomb_k", C.c_double), ("n_types", C.c_int32),
                ("sigma", C.POINTER(C.c_double)), ("epsilon", C.POINTER(C.c_double)),
                ("flags", C.c_uint32), ("ewald_alpha", C.c_double)]


class OracleError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        pp = C.POINTER(_Params)
        _lib.mdo_grid.argtypes = [pp, ip]
        _lib.mdo_bin.argtypes = [pp, C.c_int64, dp, ip, ip]
        _lib.mdo_canonicalize_f32.argtypes = [C.c_int64, C.POINTER(C.c_float), dp, dp,
                                              C.POINTER(C.c_uint32)]
        _lib.mdo_canonicalize_f64.argtypes = [C.c_int64, dp, dp, dp, C.POINTER(C.c_uint32)]
        _lib.mdo_pair_terms.argtypes = [pp, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        C.c_double, dp, dp]
        _lib.mdo_forces_bruteforce.argtypes = [pp, C.c_int64, dp, ip, dp, dp, dp, lp, dp, lp,
                                               C.c_int]
        _lib.mdo_forces_celllist.argtypes = [pp, C.c_int64, dp, ip, dp, dp, dp, lp, dp, lp,
                                             C.c_int]
        _lib.mdo_forces_subset.argtypes = [pp, C.c_int64, dp, ip, dp, C.c_int64, lp, dp, dp, lp,
                                           C.c_int]
        _lib.mdo_pairs_bruteforce.argtypes = [pp, C.c_int64, dp, C.c_int64, lp, ip]
        _lib.mdo_pairs_celllist.argtypes = [pp, C.c_int64, dp, C.c_int64, lp, ip]
        _lib.mdo_band_atoms.argtypes = [pp, C.c_int64, dp, C.c_double, lp, lp, C.c_int]
        _lib.mdo_ewald_recip.argtypes = [pp, C.c_int64, dp, dp, ip, dp, dp, dp, dp, C.c_int]
        for f in ("mdo_grid", "mdo_bin", "mdo_canonicalize_f32", "mdo_canonicalize_f64",
                  "mdo_pair_terms", "mdo_forces_bruteforce", "mdo_forces_celllist",
                  "mdo_forces_subset", "mdo_pairs_bruteforce", "mdo_pairs_celllist",
                  "mdo_band_atoms", "mdo_ewald_recip"):
            getattr(_lib, f).restype = C.c_int
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Params:
    """Holds a C parameter struct and keeps its arrays alive."""

    def __init__(self, box, r_cut, r_switch, coulomb_k, sigma, epsilon, flags=0, ewald_alpha=0.0):
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.epsilon = np.ascontiguousarray(epsilon, dtype=np.float64)
        self.box = np.asarray(box, dtype=np.float64)
        self.c = _Params((C.c_double * 3)(*[float(b) for b in self.box]), float(r_cut),
                         float(r_switch), float(coulomb_k), int(self.sigma.shape[0]),
                         _ptr(self.sigma, C.c_double), _ptr(self.epsilon, C.c_double),
                         int(flags), float(ewald_alpha))

    @classmethod
    def from_dict(cls, d):
        return cls(d["box"], d["r_cut"], d["r_switch"], d["coulomb_k"], d["sigma"],
                   d["epsilon"], d.get("flags", 0), d.get("ewald_alpha", 0.0))

    def ref(self):
        return C.byref(self.c)


def _as_params(p):
    return p if isinstance(p, Params) else Params.from_dict(p)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def grid(params):
    p = _as_params(params)
    dims = np.zeros(3, dtype=np.int32)
    _check(lib().mdo_grid(p.ref(), _ptr(dims, C.c_int32)), "mdo_grid")
    return tuple(int(d) for d in dims)


def canonicalize(pos, box):
    """Wraps [-L, 2L) into [0, L] in the input's precision; returns (float64 pos, status)."""
    box = np.ascontiguousarray(box, dtype=np.float64)
    st = C.c_uint32(0)
    if pos.dtype == np.float32:
        src = np.ascontiguousarray(pos, dtype=np.float32)
        out = np.empty(src.shape, dtype=np.float64)
        _check(lib().mdo_canonicalize_f32(src.shape[0], _ptr(src, C.c_float),
                                          _ptr(box, C.c_double), _ptr(out, C.c_double),
                                          C.byref(st)), "canonicalize")
    else:
        src = np.ascontiguousarray(pos, dtype=np.float64)
        out = np.empty(src.shape, dtype=np.float64)
        _check(lib().mdo_canonicalize_f64(src.shape[0], _ptr(src, C.c_double),
                                          _ptr(box, C.c_double), _ptr(out, C.c_double),
                                          C.byref(st)), "canonicalize")
    return out, int(st.value)


def bin_atoms(params, pos64):
    p = _as_params(params)
    pos64 = np.ascontiguousarray(pos64, dtype=np.float64)
    cell = np.empty(pos64.shape[0], dtype=np.int32)
    dims = np.zeros(3, dtype=np.int32)
    _check(lib().mdo_bin(p.ref(), pos64.shape[0], _ptr(pos64, C.c_double),
                         _ptr(cell, C.c_int32), _ptr(dims, C.c_int32)), "mdo_bin")
    return cell, tuple(int(d) for d in dims)


def pair_terms(params, ti, tj, qi, qj, u):
    """(energy, f) of one pair at squared distance u; F_i = f (x_i - x_j)."""
    p = _as_params(params)
    e = C.c_double(0)
    f = C.c_double(0)
    _check(lib().mdo_pair_terms(p.ref(), int(ti), int(tj), float(qi), float(qj), float(u),
                                C.byref(e), C.byref(f)), "mdo_pair_terms")
    return e.value, f.value


class Result:
    def __init__(self, force, energy=None, n_pairs=None, abs_sum=None, count=None):
        self.force = force
        self.energy = energy
        self.n_pairs = n_pairs
        self.abs_sum = abs_sum
        self.count = count


def _inputs(pos, types, charges, box):
    if pos.dtype != np.float64:
        pos64, st = canonicalize(pos, box)
        if st:
            raise OracleError(f"input positions rejected (status {st:#x})")
    else:
        pos64, st = canonicalize(pos, box)
        if st:
            raise OracleError(f"input positions rejected (status {st:#x})")
    t = np.ascontiguousarray(types, dtype=np.int32)
    q = np.ascontiguousarray(np.asarray(charges).astype(np.float64))
    return pos64, t, q


def forces(params, pos, types, charges, method="celllist", n_threads=0):
    """Forces [n,3] float64, total energy, unique pair count, per-atom sum of pair-force
    magnitudes and per-atom partner counts. float32 positions are wrapped in float32."""
    p = _as_params(params)
    pos64, t, q = _inputs(pos, types, charges, p.box)
    n = pos64.shape[0]
    F = np.zeros((n, 3), dtype=np.float64)
    absum = np.zeros(n, dtype=np.float64)
    cnt = np.zeros(n, dtype=np.int64)
    E = C.c_double(0)
    P = C.c_int64(0)
    fn = {"celllist": lib().mdo_forces_celllist,
          "bruteforce": lib().mdo_forces_bruteforce}[method]
    _check(fn(p.ref(), n, _ptr(pos64, C.c_double), _ptr(t, C.c_int32), _ptr(q, C.c_double),
              _ptr(F, C.c_double), C.byref(E), C.byref(P), _ptr(absum, C.c_double),
              _ptr(cnt, C.c_int64), int(n_threads)), f"mdo_forces_{method}")
    return Result(F, E.value, P.value, absum, cnt)


def forces_subset(params, pos, types, charges, idx, n_threads=0):
    """Forces on the atoms idx only, each summed over all atoms by minimum image."""
    p = _as_params(params)
    pos64, t, q = _inputs(pos, types, charges, p.box)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    F = np.zeros((idx.shape[0], 3), dtype=np.float64)
    absum = np.zeros(idx.shape[0], dtype=np.float64)
    cnt = np.zeros(idx.shape[0], dtype=np.int64)
    _check(lib().mdo_forces_subset(p.ref(), pos64.shape[0], _ptr(pos64, C.c_double),
                                   _ptr(t, C.c_int32), _ptr(q, C.c_double), idx.shape[0],
                                   _ptr(idx, C.c_int64), _ptr(F, C.c_double),
                                   _ptr(absum, C.c_double), _ptr(cnt, C.c_int64),
                                   int(n_threads)), "mdo_forces_subset")
    return Result(F, None, None, absum, cnt)


def pairs(params, pos, method="bruteforce", cap=None):
    """Unique within-cutoff pairs (i < j), lexicographically sorted, int32 [k,2]."""
    p = _as_params(params)
    pos64, st = canonicalize(pos, p.box)
    if st:
        raise OracleError(f"input positions rejected (status {st:#x})")
    n = pos64.shape[0]
    if cap is None:
        cap = max(1024, n * 256)
    out = np.empty((cap, 2), dtype=np.int32)
    k = C.c_int64(0)
    fn = {"celllist": lib().mdo_pairs_celllist,
          "bruteforce": lib().mdo_pairs_bruteforce}[method]
    rc = fn(p.ref(), n, _ptr(pos64, C.c_double), cap, C.byref(k), _ptr(out, C.c_int32))
    if rc == -6:
        return pairs(params, pos, method, cap=int(k.value))
    _check(rc, f"mdo_pairs_{method}")
    return out[: k.value].copy()


def band_atoms(params, pos, band, n_threads=0):
    """Per-atom number of partners with |u - rc^2| <= band, and the unique band-pair count."""
    p = _as_params(params)
    pos64, st = canonicalize(pos, p.box)
    if st:
        raise OracleError(f"input positions rejected (status {st:#x})")
    n = pos64.shape[0]
    per = np.zeros(n, dtype=np.int64)
    tot = C.c_int64(0)
    _check(lib().mdo_band_atoms(p.ref(), n, _ptr(pos64, C.c_double), float(band), C.byref(tot),
                                _ptr(per, C.c_int64), int(n_threads)), "mdo_band_atoms")
    return per, int(tot.value)


def ewald_recip(params, pos, charges, kmax, n_threads=0):
    """Ewald reciprocal-space forces [n,3] and the energies (recip, self, background) for
    positions pos (canonicalised like the force path) and charges, over every wave vector
    with |m_d| <= kmax[d] (params['ewald_alpha'] is the splitting parameter)."""
    p = _as_params(params)
    pos64, st = canonicalize(pos, p.box)
    if st:
        raise OracleError(f"input positions rejected (status {st:#x})")
    q = np.ascontiguousarray(np.asarray(charges).astype(np.float64))
    km = np.ascontiguousarray(kmax, dtype=np.int32)
    n = pos64.shape[0]
    F = np.zeros((n, 3), dtype=np.float64)
    er, es, eb = C.c_double(0), C.c_double(0), C.c_double(0)
    _check(lib().mdo_ewald_recip(p.ref(), n, _ptr(pos64, C.c_double), _ptr(q, C.c_double),
                                 _ptr(km, C.c_int32), _ptr(F, C.c_double), C.byref(er),
                                 C.byref(es), C.byref(eb), int(n_threads)), "mdo_ewald_recip")
    return F, er.value, es.value, eb.value


# ---------------------------------------------------------------------------------------
# Motion update around the force call. Each MD iteration first computes the forces on
# every atom and then updates the atoms' motion (Section 1; Section 2.1). The paper names
# no integrator; this is velocity Verlet, written out plainly in float64:
#   v(t + dt/2) = v(t) + (dt/2) a(t)
#   x(t + dt)   = x(t) + dt v(t + dt/2), wrapped into [0, L)
#   a(t + dt)   = F(x(t + dt)) / m
#   v(t + dt)   = v(t + dt/2) + (dt/2) a(t + dt)
# Units: A, fs, amu, kcal/mol. (kcal/mol/A)/amu = 4.184e-4 A/fs^2: 1 cal = 4.184 J and an
# amu times Avogadro's number is one gram.

ACCEL = 4.184e-4


def kinetic_energy(vel, inv_mass):
    """sum of m v^2 / 2 in kcal/mol, for velocities in A/fs and 1/m in 1/amu."""
    v = np.asarray(vel, dtype=np.float64)
    return float(0.5 * np.sum(np.sum(v * v, axis=1) / np.asarray(inv_mass, dtype=np.float64)) / ACCEL)


def vv_steps(params, pos, vel, types, charges, inv_mass, dt, n_steps, method="celllist",
             n_threads=0):
    """n_steps velocity-Verlet steps of dt fs from positions pos [n,3] and velocities vel
    [n,3] (A/fs). Returns (pos, vel, force, pe [n_steps], ke [n_steps]), all float64; pe[k]
    and ke[k] are the potential and kinetic energy after step k + 1."""
    L = np.asarray(params["box"], dtype=np.float64)
    x, _ = canonicalize(pos, L)
    v = np.array(vel, dtype=np.float64)
    im = np.asarray(inv_mass, dtype=np.float64)[:, None]
    F = forces(params, x, types, charges, method, n_threads).force
    pe = np.zeros(n_steps)
    ke = np.zeros(n_steps)
    for k in range(n_steps):
        v = v + 0.5 * dt * (F * im * ACCEL)
        x = x + dt * v
        x = x - L * np.floor(x / L)
        r = forces(params, x, types, charges, method, n_threads)
        F = r.force
        v = v + 0.5 * dt * (F * im * ACCEL)
        pe[k] = r.energy
        ke[k] = kinetic_energy(v, im[:, 0])
    return x, v, F, pe, ke
