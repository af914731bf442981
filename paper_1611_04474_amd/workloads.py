"""Seeded synthetic workloads for the short-range non-bonded force path.

This module only draws inputs: positions, types, charges, per-type Lennard-Jones
parameters, boxes and arrival traces. It holds none of the force method's
arithmetic, so both the HIP path and the FP64 oracle consume the same arrays.

The paper benchmarks ApoA1 (about 100,000 atoms in about 700 cells, Section 3
"Experimental Setup"); that input is not available, so these generators stand in
for it with jittered-lattice systems of the same density, atom count and box shape.

Draw order (numpy PCG64 ``default_rng``), for ``gen_system(n, box, seed)``:
  1. the box is rounded to float32 once; that value is the box everywhere;
  2. lattice constant a0 = (V/n)^(1/3); n_d = ceil(L_d/a0) sites per axis,
     spacing s_d = L_d/n_d, jitter half-width j = (min_d s_d - 1.0)/2, so any two
     atoms are at least 1.0 A apart along some axis;
  3. ``rng.choice(prod n_d, n, replace=False)`` picks the occupied sites;
  4. x = (ijk + 0.5) s + U(-j, j), wrapped into [0, L) and cast to float32;
  5. types ``rng.integers(0, n_types, n)``;
  6. sigma ~ U(2, 4) A and epsilon ~ U(0.01, 0.2) kcal/mol per type (skipped when a
     shared table is passed in);
  7. charges N(0, 0.5) e, shifted to a zero mean in float64, cast to float32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Physical constants of the workload (units: A, e, kcal/mol).
COULOMB_K = 332.0636          # kcal*A/(mol*e^2), dielectric 1
R_CUT = 12.0                  # A
R_SWITCH = 10.0               # A
N_TYPES = 8

# Shapes of the benchmark systems.
SMALL_BOX = (30.0, 30.0, 30.0)            # 3,000 atoms, FP64-everywhere case
SMALL_N = 3000
APOA1_BOX = (108.86, 108.86, 77.76)       # ApoA1-sized box, 92,224 atoms
APOA1_N = 92224
STMV_BOX = (216.83, 216.83, 216.83)       # 1,066,628-atom cube
STMV_N = 1066628
SERVING_DENSITY = 0.1                     # atoms / A^3

SEED_SMALL = 1
SEED_APOA1 = 2
SEED_STMV = 4
SEED_STMV_PERTURB = 40
SEED_SERVING = 5


@dataclasses.dataclass
class System:
    """One periodic system: float32 positions [n,3], int32 types, float32 charges."""
    pos: np.ndarray
    types: np.ndarray
    charges: np.ndarray
    box: np.ndarray            # float64 array holding float32-representable values
    sigma: np.ndarray          # float64 [n_types]
    epsilon: np.ndarray        # float64 [n_types]
    seed: object = None

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def params(self, r_cut=R_CUT, r_switch=R_SWITCH, coulomb_k=COULOMB_K, flags=0) -> dict:
        return dict(box=tuple(float(b) for b in self.box), r_cut=r_cut, r_switch=r_switch,
                    coulomb_k=coulomb_k, sigma=self.sigma, epsilon=self.epsilon, flags=flags)


def f32_box(box) -> np.ndarray:
    """Round a box to float32 once and return it as float64 (exactly representable)."""
    return np.asarray(box, dtype=np.float32).astype(np.float64)


def draw_type_table(rng: np.random.Generator, n_types: int = N_TYPES):
    sigma = rng.uniform(2.0, 4.0, n_types)
    epsilon = rng.uniform(0.01, 0.2, n_types)
    return sigma.astype(np.float64), epsilon.astype(np.float64)


def gen_system(n: int, box, seed, n_types: int = N_TYPES, type_table=None,
               min_sep: float = 1.0) -> System:
    """Jittered-lattice system of n atoms in an orthorhombic periodic box."""
    rng = np.random.default_rng(seed)
    L = f32_box(box)
    vol = float(np.prod(L))
    a0 = (vol / n) ** (1.0 / 3.0)
    nd = np.array([int(math.ceil(L[d] / a0)) for d in range(3)], dtype=np.int64)
    s = L / nd
    jit = (float(s.min()) - min_sep) / 2.0
    if jit < 0:
        raise ValueError("density too high for the requested minimum separation")
    n_sites = int(np.prod(nd))
    if n > n_sites:
        raise ValueError("more atoms than lattice sites")
    sites = rng.choice(n_sites, n, replace=False)
    ix = sites % nd[0]
    iy = (sites // nd[0]) % nd[1]
    iz = sites // (nd[0] * nd[1])
    ijk = np.stack([ix, iy, iz], axis=1).astype(np.float64)
    x = (ijk + 0.5) * s + rng.uniform(-jit, jit, (n, 3))
    x = np.mod(x, L)
    pos = x.astype(np.float32)
    L32 = L.astype(np.float32)
    for d in range(3):   # a value that rounds up to L in float32 wraps to 0
        col = pos[:, d]
        col[col >= L32[d]] = np.float32(0.0)
    types = rng.integers(0, n_types, n).astype(np.int32)
    if type_table is None:
        sigma, epsilon = draw_type_table(rng, n_types)
    else:
        sigma, epsilon = (np.asarray(t, dtype=np.float64) for t in type_table)
    q = rng.normal(0.0, 0.5, n).astype(np.float64)
    q -= q.mean()
    charges = q.astype(np.float32)
    return System(pos=pos, types=types, charges=charges, box=L, sigma=sigma,
                  epsilon=epsilon, seed=seed)


def small_system() -> System:
    """3,000 atoms in a 30 A cube (density ~0.11 / A^3), seed 1."""
    return gen_system(SMALL_N, SMALL_BOX, SEED_SMALL)


def apoa1_system() -> System:
    """92,224 atoms in a 108.86 x 108.86 x 77.76 A box (density 0.1 / A^3), seed 2."""
    return gen_system(APOA1_N, APOA1_BOX, SEED_APOA1)


def stmv_system() -> System:
    """1,066,628 atoms in a 216.83 A cube (density ~0.1 / A^3), seed 4."""
    return gen_system(STMV_N, STMV_BOX, SEED_STMV)


def perturbation_stream(n: int, n_steps: int, sigma: float = 0.01, seed=SEED_STMV_PERTURB):
    """Yields float32 displacement fields N(0, sigma) A, one per force evaluation."""
    rng = np.random.default_rng(seed)
    for _ in range(n_steps):
        yield rng.normal(0.0, sigma, (n, 3)).astype(np.float32)


def perturb(pos: np.ndarray, disp: np.ndarray) -> np.ndarray:
    """x + dx in float32; values may leave [0, L) and are wrapped by the force call."""
    return (pos.astype(np.float32) + disp.astype(np.float32)).astype(np.float32)


def cube_for(n: int, density: float = SERVING_DENSITY) -> float:
    return float(np.float32((n / density) ** (1.0 / 3.0)))


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    seed: object


def serving_trace(n_req: int = 512, rate_hz: float = 200.0, n_min: int = 2000,
                  n_max: int = 200000, seed=SEED_SERVING):
    """Request sizes log-uniform in [n_min, n_max], Poisson arrivals at rate_hz.

    Returns (requests, (sigma, epsilon)); one type table is shared by every request.
    Request r draws its own system from SeedSequence([seed, r]).
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_req))).astype(np.int64)
    if rate_hz is None or math.isinf(rate_hz):
        arrivals = np.zeros(n_req)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, n_req))
        arrivals -= arrivals[0]
    table = draw_type_table(np.random.default_rng(np.random.SeedSequence([seed, 1_000_000])))
    reqs = [Request(rid=r, arrival_s=float(arrivals[r]), n=int(sizes[r]),
                    seed=np.random.SeedSequence([seed, r])) for r in range(n_req)]
    return reqs, table


def request_system(req: Request, table, density: float = SERVING_DENSITY) -> System:
    L = cube_for(req.n, density)
    return gen_system(req.n, (L, L, L), req.seed, type_table=table)


# Masses (amu) of the 8 synthetic atom types for the motion update: H, C, N, O, P, S, Na,
# Cl -- an input table, like sigma and epsilon.
TYPE_MASS = np.array([1.008, 12.011, 14.007, 15.999, 30.974, 32.06, 22.990, 35.45])
SEED_VELOCITIES = 7


def velocities(types, masses=TYPE_MASS, scale=0.005, seed=SEED_VELOCITIES):
    """Seeded initial velocities (A/fs): each component normal with standard deviation
    scale * sqrt(12 / m) for an atom of mass m (about 300 K for scale 0.005), total
    momentum removed. Returns (float32 [n,3] velocities, float32 [n] inverse masses)."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)[np.asarray(types)]
    v = rng.normal(0.0, 1.0, (m.shape[0], 3)) * (scale * np.sqrt(12.0 / m))[:, None]
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return v.astype(np.float32), (1.0 / m).astype(np.float32)


SEED_LIQUID = 9


def liquid_system(n: int, box, seed=SEED_LIQUID, n_types: int = N_TYPES) -> System:
    """Input for the motion update: a jittered lattice of n atoms in the box (the same
    lattice rule as gen_system, jitter 0.1 A), with LJ sigma 1.8-2.0 A so that lattice
    neighbours (about 2.1 A apart at 0.1 atoms/A^3) sit near the LJ minimum, epsilon
    0.05-0.2 kcal/mol and charges N(0, 0.2) e, neutral in total: a system whose dynamics
    stays bounded, unlike the force benchmark's (sigma up to 4 A at the same spacing)."""
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(1.8, 2.0, n_types)
    epsilon = rng.uniform(0.05, 0.2, n_types)
    base = gen_system(n, box, seed, n_types, type_table=(sigma, epsilon))
    L = base.box
    a0 = (float(np.prod(L)) / n) ** (1.0 / 3.0)
    # redraw the jitter at 0.1 A around the same lattice sites
    nd = np.array([int(math.ceil(L[d] / a0)) for d in range(3)], dtype=np.int64)
    sp = L / nd
    site = np.floor(base.pos.astype(np.float64) / sp)   # each atom's lattice site (jitter < s/2)
    x = (site + 0.5) * sp + rng.uniform(-0.1, 0.1, (n, 3))
    pos = np.mod(x, L).astype(np.float32)
    L32 = L.astype(np.float32)
    for d in range(3):
        col = pos[:, d]
        col[col >= L32[d]] = np.float32(0.0)
    q = rng.normal(0.0, 0.2, n)
    q -= q.mean()
    return System(pos=pos, types=base.types, charges=q.astype(np.float32), box=L, sigma=sigma,
                  epsilon=epsilon, seed=seed)
