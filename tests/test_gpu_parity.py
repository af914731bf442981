"""Parity of the HIP force path with the FP64 oracle, through the C ABI.

Bars: float64 path -- forces and energy to 1e-12 relative (metric (ii) and (iii)),
per-atom partner counts bit-exact; float32 path -- metrics (ii) and (iii) <= 1e-5,
energy <= 1e-6 relative, partner counts exact except atoms with a partner whose
squared distance lies within 8 float32 ulps of rc^2 (where a float32 and a float64
cutoff test may disagree)."""
import math

import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import api
from paper_1611_04474_amd import workloads as W

from _gpu import run
from _metrics import force_errors

pytestmark = pytest.mark.gpu

BAND = 8 * 2.0 ** (math.floor(math.log2(144.0)) - 23)    # 8 ulp32 of rc^2


def _say(*a):
    print(*a, flush=True)


def _ref(params, pos, types, q, method="celllist"):
    return oracle.forces(params, pos, types, q, method, n_threads=0)


def _check_fp32(params, pos, types, q, g_force, g_energy, g_counts, tol=1e-5):
    r = _ref(params, pos, types, q)
    err = force_errors(g_force, r.force, r.abs_sum)
    _say("fp32 errors", err, "energy", g_energy, r.energy)
    assert err["max_norm"] <= tol and err["rms"] <= tol, err
    assert g_energy == pytest.approx(r.energy, rel=1e-6, abs=1e-6)
    if g_counts is not None:
        band, nb = oracle.band_atoms(params, pos, BAND)
        ok = (g_counts == r.count) | (band > 0)
        assert ok.all(), np.nonzero(~ok)[0][:10]
    return r, err


@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL, api.PAIR_PREDICATED])
def test_fp64_small_config_exact(gpu, flags):
    """FP64 everywhere: the compacted kernel instantiated for float64 (half and full
    shell) and the predicated kernel, to 1e-12 with bit-exact partner counts."""
    _say("case: 3,000-atom system, float64 path, flags", flags)
    s = W.small_system()
    p = s.params()
    f, e, ws, cnt = run(p, s.pos.astype(np.float64), s.types, s.charges.astype(np.float64), gpu,
                        double=True, flags=flags | api.DIAG_COUNTERS)
    r = _ref(p, s.pos, s.types, s.charges, "bruteforce")
    err = force_errors(f, r.force, r.abs_sum)
    _say("fp64 errors", err)
    assert err["max_norm"] <= 1e-12 and err["rms"] <= 1e-12
    assert e == pytest.approx(r.energy, rel=1e-12)
    assert np.array_equal(cnt, r.count)
    diag = api.read_diag(ws)
    assert diag[2] == r.n_pairs == 1201501
    assert diag[0] == sum_candidates(p, s.pos)
    assert api.read_status(ws) == 0


def sum_candidates(params, pos):
    """Half-shell candidate count from the oracle's binning: for each home cell,
    m(m-1)/2 home pairs plus m * m' for its 13 forward neighbour images."""
    pos64, _ = oracle.canonicalize(pos, np.asarray(params["box"], float))
    cell, dims = oracle.bin_atoms(params, pos64)
    cnt = np.bincount(cell, minlength=int(np.prod(dims))).astype(np.int64)
    nx, ny, nz = dims
    total = int((cnt * (cnt - 1) // 2).sum())
    fwd = [(1, 0, 0), (-1, 1, 0), (0, 1, 0), (1, 1, 0)] + [(x, y, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)]
    for c in range(len(cnt)):
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        for ox, oy, oz in fwd:
            b = (((z + oz) % nz) * ny + (y + oy) % ny) * nx + (x + ox) % nx
            total += int(cnt[c] * cnt[b])
    return total


@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL, api.PAIR_PREDICATED])
def test_fp32_small_config(gpu, flags):
    _say("case: 3,000-atom system, float32 path, flags", flags)
    s = W.small_system()
    p = s.params()
    f, e, ws, cnt = run(p, s.pos, s.types, s.charges, gpu, flags=flags | api.DIAG_COUNTERS)
    _check_fp32(p, s.pos, s.types, s.charges, f, e, cnt)
    assert api.read_status(ws) == 0


@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL])
def test_fp32_apoa1_full(gpu, flags):
    _say("case: 92,224-atom system, float32 path, all atoms, flags", flags)
    s = W.apoa1_system()
    p = s.params()
    f, e, ws, cnt = run(p, s.pos, s.types, s.charges, gpu, flags=flags | api.DIAG_COUNTERS)
    r, err = _check_fp32(p, s.pos, s.types, s.charges, f, e, cnt)
    diag = api.read_diag(ws)
    band, nb = oracle.band_atoms(p, s.pos, BAND)
    _say("pairs gpu", diag[2], "oracle", r.n_pairs, "band pairs", nb, "candidates", diag[0])
    assert abs(diag[2] - r.n_pairs) <= nb
    assert diag[0] == sum_candidates(p, s.pos)


def _check_binning(p, pos, ws, n):
    """The sorted layout in the workspace against the oracle's cells: cell ranges that
    cover every atom once, each cell ordered by (z half, wrapped x, original index) with
    the z half in float32 as the kernel computes it, the lower-half counts, and each atom
    in the oracle's cell unless it sits within 1e-4 A of a cell face."""
    import torch
    lay = api.workspace_layout(p, n)
    nc = lay["n_cells"]
    start = ws[lay["cell_start"]: lay["cell_start"] + 4 * (nc + 1)].view(torch.int32).cpu().numpy()
    perm = ws[lay["perm"]: lay["perm"] + 4 * n].view(torch.int32).cpu().numpy().astype(np.int64)
    zsplit = ws[lay["z_split"]: lay["z_split"] + 4 * nc].view(torch.int32).cpu().numpy()
    assert start[0] == 0 and start[-1] == n and np.all(np.diff(start) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    box = np.asarray(p["box"], np.float64)
    pos64, _ = oracle.canonicalize(pos, box)   # wrapped in float32, as the kernels do
    dims_g = lay["dims"]
    inv_wz = np.float32(dims_g[2] / float(np.float32(box[2])))
    scell = np.repeat(np.arange(nc), np.diff(start))          # cell of each sorted slot
    cz = scell // (dims_g[0] * dims_g[1])
    zf = pos64[perm, 2].astype(np.float32)
    half = ((zf * inv_wz * np.float32(2)).astype(np.int64) >= 2 * cz + 1).astype(np.int64)
    assert np.array_equal(np.bincount(scell[half == 0], minlength=nc), zsplit)
    x = pos64[perm, 0]
    same = np.diff(scell) == 0
    dh, dx, di = np.diff(half), np.diff(x), np.diff(perm)
    ordered = (dh > 0) | ((dh == 0) & ((dx > 0) | ((dx == 0) & (di > 0))))
    assert np.all(ordered[same])
    gcell = np.empty(n, np.int64)
    gcell[perm] = scell
    ocell, dims = oracle.bin_atoms(p, pos64)
    diff = np.nonzero(gcell != ocell)[0]
    w = box / np.array(dims)
    frac = pos64[diff] / w
    assert np.all(np.min(np.abs(frac - np.round(frac)) * w, axis=1) < 1e-4), diff[:10]
    return lay


def test_binning_matches_oracle(gpu):
    _say("case: binning of the 92,224-atom system")
    s = W.apoa1_system()
    p = s.params()
    f, e, ws, _ = run(p, s.pos, s.types, s.charges, gpu)
    _check_binning(p, s.pos, ws, s.n)


def test_binning_many_blocks(gpu):
    """2,500,000 atoms in a 280 A cube (23^3 cells, more than the fused scan takes): 611
    histogram blocks of 4,096 atoms (two rounds of 4 atoms per thread), 39 blocks per wave in
    the column scan, the cell counts of the scan kernel in LDS; sampled forces against the
    oracle."""
    _say("case: binning of 2,500,000 atoms, 280 A cube")
    import torch
    s = W.gen_system(2_500_000, (280.0, 280.0, 280.0), seed=21)
    p = s.params()
    lay = api.workspace_layout(p, s.n)
    assert lay["n_cells"] == 23 ** 3
    f, e, ws, _ = run(p, s.pos, s.types, s.charges, gpu)
    assert api.read_status(ws) == 0
    _check_binning(p, s.pos, ws, s.n)
    idx = np.sort(np.random.default_rng(3).choice(s.n, 200, replace=False))
    ref = oracle.forces_subset(p, s.pos, s.types, s.charges, idx)
    err = force_errors(f[idx], ref.force, ref.abs_sum)
    _say("sampled", err)
    assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5
    del ws
    torch.cuda.empty_cache()


def test_binning_fused_one_wave_gather(gpu):
    """300,000 atoms in 10 x 10 x 8 cells: 147 histogram blocks of 2,048 atoms, so the
    in-cell sort's first wave gathers each cell from three blocks per lane (up to 256
    blocks take that path); sampled forces against the oracle."""
    _say("case: binning of 300,000 atoms, 130 x 130 x 100 A")
    import torch
    s = W.gen_system(300_000, (130.0, 130.0, 100.0), seed=23)
    p = s.params()
    lay = api.workspace_layout(p, s.n)
    assert tuple(lay["dims"]) == (10, 10, 8)
    f, e, ws, _ = run(p, s.pos, s.types, s.charges, gpu)
    assert api.read_status(ws) == 0
    _check_binning(p, s.pos, ws, s.n)
    idx = np.sort(np.random.default_rng(5).choice(s.n, 200, replace=False))
    ref = oracle.forces_subset(p, s.pos, s.types, s.charges, idx)
    err = force_errors(f[idx], ref.force, ref.abs_sum)
    _say("sampled", err)
    assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5
    del ws
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n, box, r_cut, cells, blocks", [
    (524_288, (172.0, 172.0, 172.0), 17.0, 1000, 256),   # the most blocks one wave gathers
    (524_289, (172.0, 172.0, 172.0), 17.0, 1000, 257),   # the fewest the block scans take
    (181_000, (194.0, 97.0, 97.0), 12.0, 1024, 89),      # the largest grid of the fused scan
])
def test_binning_fused_limits(gpu, n, box, r_cut, cells, blocks):
    """The edges of the two-kernel binning: 256 and 257 histogram blocks of 2,048 atoms
    (the in-cell sort's single-wave gather and its block scans), and a grid of exactly 1,024
    cells (16 x 8 x 8, each histogram block scanning 1,024 counts). Binning stage only, from
    a workspace filled with a byte pattern, against the oracle's cells and order."""
    _say("case: binning of", n, "atoms,", cells, "cells,", blocks, "histogram blocks")
    import torch
    from _gpu import to_dev
    rng = np.random.default_rng(n % 1000)
    pos = rng.uniform(0.0, 1.0, (n, 3)) * np.asarray(box)
    pos = pos.astype(np.float32).astype(np.float64)
    types = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.2, n)
    p = dict(box=box, r_cut=r_cut, r_switch=r_cut - 2.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([0.8, 0.9]), epsilon=np.array([0.05, 0.1]), flags=0)
    lay = api.workspace_layout(p, n)
    assert lay["n_cells"] == cells
    chunk = -(-(-(-n // 1024)) // 2048) * 2048
    assert -(-n // chunk) == blocks
    d = to_dev((pos, types, q), gpu)
    ws = api.alloc_workspace(p, n, gpu)
    ws.fill_(0xAB)
    force = torch.empty((n, 3), dtype=torch.float32, device=gpu)
    energy = torch.empty(1, dtype=torch.float64, device=gpu)
    api.forces_stages(p, *d, force, energy, ws, api.STAGE_BIN)
    torch.cuda.synchronize()
    assert api.read_status(ws) == 0
    _check_binning(p, pos, ws, n)
    del ws
    torch.cuda.empty_cache()


def test_binning_fused_several_rounds(gpu):
    """2,200,000 atoms, uniform in a 120 A cube of 9^3 cells (at most 1,024: each histogram
    block writes its atoms in cell order within its range and the in-cell sort gathers the
    cells): 538 blocks of 4,096 atoms, two rounds each, so the blocks read their atoms' cells
    and slots back, and every cell holds more than 1,024 atoms, so the sort keeps its member
    list in the workspace. Binning stage only (the pair stage of a cell this dense is not
    the point here), from a workspace filled with a byte pattern."""
    _say("case: binning of 2,200,000 atoms, 120 A cube, 9^3 cells")
    import torch
    from _gpu import to_dev
    rng = np.random.default_rng(33)
    n = 2_200_000
    pos = rng.uniform(0.0, 120.0, (n, 3)).astype(np.float32).astype(np.float64)
    types = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.2, n)
    p = dict(box=(120.0, 120.0, 120.0), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([0.8, 0.9]), epsilon=np.array([0.05, 0.1]), flags=0)
    lay = api.workspace_layout(p, n)
    assert lay["n_cells"] == 9 ** 3
    d = to_dev((pos, types, q), gpu)
    ws = api.alloc_workspace(p, n, gpu)
    ws.fill_(0xAB)
    force = torch.empty((n, 3), dtype=torch.float32, device=gpu)
    energy = torch.empty(1, dtype=torch.float64, device=gpu)
    api.forces_stages(p, *d, force, energy, ws, api.STAGE_BIN)
    torch.cuda.synchronize()
    assert api.read_status(ws) == 0
    _check_binning(p, pos, ws, n)
    del ws
    torch.cuda.empty_cache()


@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL])
def test_fixed64_bitwise_reproducible(gpu, flags):
    """Ten calls on one workspace give the same bits. The first call (workspace filled with
    a byte pattern) launches the home cells by atom count; the later ones by the cell times
    the call before recorded in the workspace, so this also pins that the launch order
    never changes a result."""
    _say("case: 92,224 atoms, 10 runs, fixed-point accumulation, flags", flags)
    import torch
    from _gpu import to_dev
    s = W.apoa1_system()
    p = api.Params.from_dict(s.params(), flags)
    d = to_dev((s.pos, s.types, s.charges), gpu)
    ws = api.alloc_workspace(p, s.n, gpu)
    ws.fill_(0xAB)
    f0, e0 = api.forces(p, *d, workspace=ws)
    f0 = f0.clone(); e0 = e0.clone()
    for k in range(9):
        f1, e1 = api.forces(p, *d, workspace=ws)
        assert torch.equal(f1, f0) and torch.equal(e1, e0), k


def test_clock_under_load(gpu):
    """The pair kernel's own clock reading: a shader clock between 0.5 GHz and the
    2.4 GHz maximum after the compacted kernel (the roofline's peak at the clock under
    load comes from it), 0 after the predicated kernel, which does not record one."""
    _say("case: 92,224 atoms, clock of the compacted and of the predicated pair kernel")
    from _gpu import to_dev
    s = W.apoa1_system()
    d = to_dev((s.pos, s.types, s.charges), gpu)
    for flags in (0, api.PAIR_PREDICATED):
        p = api.Params.from_dict(s.params(), flags)
        ws = api.alloc_workspace(p, s.n, gpu)
        ws.fill_(0xAB)
        api.forces(p, *d, workspace=ws)
        ghz = api.read_clock(ws)
        _say("flags", flags, "clock GHz", ghz)
        if flags == 0:
            assert 0.5 < ghz < 2.45, ghz
        else:
            assert ghz == 0.0


def test_f32_atomic_mode(gpu):
    _say("case: 92,224 atoms, float32 atomic accumulation")
    s = W.apoa1_system()
    p = s.params()
    f, e, ws, _ = run(p, s.pos, s.types, s.charges, gpu, flags=api.ACCUM_F32_ATOMIC)
    _check_fp32(p, s.pos, s.types, s.charges, f, e, None)


def test_truncated_coulomb(gpu):
    _say("case: 3,000 atoms, truncated Coulomb")
    s = W.small_system()
    p = dict(s.params(), flags=oracle.FLAG_TRUNCATED_COULOMB)
    f, e, _, _ = run(p, s.pos.astype(np.float64), s.types, s.charges.astype(np.float64), gpu,
                     double=True, flags=api.COULOMB_TRUNCATED)
    r = _ref(p, s.pos, s.types, s.charges)
    err = force_errors(f, r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-12 and e == pytest.approx(r.energy, rel=1e-12)


def _random_system(n, box, seed, min_sep=1.2):
    rng = np.random.default_rng(seed)
    L = np.array(box)
    pts = []
    while len(pts) < n:
        x = rng.uniform(0, 1, 3) * L
        if all(((x - y - L * np.round((x - y) / L)) ** 2).sum() >= min_sep ** 2 for y in pts[-400:]):
            pts.append(x)
    pos = np.array(pts).astype(np.float32).astype(np.float64)
    t = rng.integers(0, 3, n).astype(np.int32)
    q = rng.normal(0, 0.5, n)
    params = dict(box=tuple(float(np.float32(b)) for b in box), r_cut=12.0, r_switch=10.0,
                  coulomb_k=W.COULOMB_K, sigma=np.array([2.5, 3.0, 3.5]),
                  epsilon=np.array([0.05, 0.1, 0.15]), flags=0)
    return pos, t, q, params


@pytest.mark.parametrize("box,n,seed", [((24.5, 24.5, 24.5), 150, 1), ((36.5, 36.5, 36.5), 300, 2),
                                        ((24.5, 37.0, 50.0), 260, 3), ((40.0, 26.0, 31.0), 5, 4)])
@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL, api.PAIR_PREDICATED])
def test_fp64_tiny_grids(gpu, box, n, seed, flags):
    _say("case: tiny system", box, n, seed, flags)
    pos, t, q, p = _random_system(n, box, seed)
    f, e, ws, cnt = run(p, pos, t, q, gpu, double=True, flags=flags | api.DIAG_COUNTERS)
    r = oracle.forces(p, pos, t, q, "bruteforce")
    err = force_errors(f, r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-12, err
    assert e == pytest.approx(r.energy, rel=1e-12, abs=1e-12)
    assert np.array_equal(cnt, r.count)


def test_clustered_cell_beyond_one_tile(gpu):
    """600 atoms packed into one 12 A cell of a 3x3x3 grid: the home cell holds more
    atoms than one LDS tile, exercising the multi-tile path. Its atoms share 9 values of x,
    about 33 per (z half, x) bucket of the in-cell sort's rank count, more than a bucket
    takes, so that cell is ranked by counting all pairs; ties in x are ordered by index."""
    _say("case: clustered cell, 600 + 200 atoms")
    rng = np.random.default_rng(5)
    g = np.arange(0, 12.0, 1.45)
    lat = np.array([[x, y, z] for x in g for y in g for z in g])[:600] + 0.3
    rest = rng.uniform(12.5, 36.0, (200, 3))
    pos = np.vstack([lat, rest]).astype(np.float32).astype(np.float64)
    n = len(pos)
    t = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.3, n)
    p = dict(box=(37.0, 37.0, 37.0), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([1.0, 1.2]), epsilon=np.array([0.05, 0.1]), flags=0)
    for flags in (0, api.PAIR_PREDICATED):
        f, e, ws, cnt = run(p, pos, t, q, gpu, double=True, flags=flags | api.DIAG_COUNTERS)
        r = oracle.forces(p, pos, t, q, "celllist")
        err = force_errors(f, r.force, r.abs_sum)
        assert err["max_norm"] <= 1e-12, (flags, err)
        assert e == pytest.approx(r.energy, rel=1e-12)
        assert np.array_equal(cnt, r.count)
        for f32_flags in ((flags,) if flags else (0, api.PAIR_FULL_SHELL)):
            f32, e32, ws32, _ = run(p, pos, t, q, gpu, flags=f32_flags)
            _check_binning(dict(p, flags=f32_flags), pos, ws32, n)
            err32 = force_errors(f32, r.force, r.abs_sum)
            assert err32["max_norm"] <= 1e-5 and err32["rms"] <= 1e-5, (f32_flags, err32)
            assert e32 == pytest.approx(r.energy, rel=1e-6), f32_flags


def _lattice_blob(rng, origin, n_side, spacing, jitter):
    g = np.arange(n_side) * spacing
    pts = np.array([[x, y, z] for x in g for y in g for z in g], dtype=np.float64)
    return origin + pts + rng.uniform(-jitter, jitter, pts.shape)


@pytest.mark.parametrize("double", [False, True])
@pytest.mark.parametrize("flags", [0, api.PAIR_FULL_SHELL])
def test_compact_multi_pass(gpu, flags, double):
    """8,000 atoms in a 3x3x3 grid: every home cell sees all of them (27 images, or 14
    in the half shell), more than one LDS load of neighbours, so the compacted kernel
    stages, filters and (half shell) hands back neighbour sums in several passes; in
    float32 and in float64 (1e-12, bit-exact partner counts)."""
    _say("case: 8,000 atoms, 37 A box, neighbour list beyond LDS, flags", flags, "double", double)
    rng = np.random.default_rng(11)
    L = 37.0
    pos = np.mod(_lattice_blob(rng, np.zeros(3), 20, 1.85, 0.3), L)
    pos = pos.astype(np.float32).astype(np.float64)
    n = len(pos)
    t = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.3, n)
    p = dict(box=(L, L, L), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([1.0, 1.2]), epsilon=np.array([0.05, 0.1]), flags=0)
    f, e, ws, cnt = run(p, pos, t, q, gpu, double=double, flags=flags | api.DIAG_COUNTERS)
    if not double:
        _check_fp32(p, pos, t, q, f, e, cnt)
        return
    r = _ref(p, pos, t, q)
    err = force_errors(f, r.force, r.abs_sum)
    _say("fp64 errors", err)
    assert err["max_norm"] <= 1e-12 and err["rms"] <= 1e-12
    assert e == pytest.approx(r.energy, rel=1e-12)
    assert np.array_equal(cnt, r.count)
    assert api.read_status(ws) == 0


def test_cell_beyond_one_sort_chunk(gpu):
    """1,200 atoms in one cell of a 3x3x3 grid: the in-cell sort ranks them over several
    LDS chunks of keys (a cell of at most 1,024 atoms takes one), and the pair kernels
    take a home cell of that size, in both shells and in float64."""
    _say("case: 1,200 atoms in one cell + 300 elsewhere, 37 A box")
    import torch
    rng = np.random.default_rng(21)
    g = np.arange(11) * 1.1 + 0.3
    lat = np.array([[x, y, z] for x in g for y in g for z in g])[:1200]
    rest = rng.uniform(13.0, 36.5, (300, 3))
    pos = np.vstack([lat, rest]).astype(np.float32).astype(np.float64)
    n = len(pos)
    t = rng.integers(0, 2, n).astype(np.int32)
    q = rng.normal(0, 0.2, n)
    p = dict(box=(37.0, 37.0, 37.0), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([0.8, 0.9]), epsilon=np.array([0.05, 0.1]), flags=0)
    f, e, ws, cnt = run(p, pos, t, q, gpu, flags=api.DIAG_COUNTERS)
    _check_fp32(p, pos, t, q, f, e, cnt)
    lay = api.workspace_layout(p, n)
    start = ws[lay["cell_start"]: lay["cell_start"] + 4 * (lay["n_cells"] + 1)].view(torch.int32).cpu().numpy()
    perm = ws[lay["perm"]: lay["perm"] + 4 * n].view(torch.int32).cpu().numpy()
    big = int(np.argmax(np.diff(start)))
    seg = perm[start[big]:start[big + 1]]
    assert len(seg) >= 1200
    pos64, _ = oracle.canonicalize(pos.astype(np.float32), np.asarray(p["box"]))
    dims = lay["dims"]
    cz = big // (dims[0] * dims[1])
    inv_wz = np.float32(dims[2] / float(np.float32(37.0)))
    half = ((pos64[seg, 2].astype(np.float32) * inv_wz * np.float32(2)).astype(np.int64) >= 2 * cz + 1)
    key = list(zip(half.astype(int), pos64[seg, 0], seg))
    assert key == sorted(key)
    f2, e2, _, cnt2 = run(p, pos, t, q, gpu, flags=api.PAIR_FULL_SHELL | api.DIAG_COUNTERS)
    _check_fp32(p, pos, t, q, f2, e2, cnt2)
    f64, e64, _, cnt64 = run(p, pos, t, q, gpu, double=True, flags=api.DIAG_COUNTERS)
    r = _ref(p, pos, t, q)
    err = force_errors(f64, r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-12 and e64 == pytest.approx(r.energy, rel=1e-12)
    assert np.array_equal(cnt64, r.count)


def test_global_atomic_binning_path(gpu):
    """A 400 A box has 33^3 cells, more than the per-block LDS histogram holds, so the
    binning takes the global-atomic path; atoms sit in dense blobs, one across the
    periodic corner."""
    _say("case: 400 A box, 35,937 cells, 3 blobs of 1,728 atoms")
    rng = np.random.default_rng(12)
    L = 400.0
    blobs = [_lattice_blob(rng, o, 12, 1.9, 0.3) for o in
             (np.array([30.0, 40.0, 50.0]), np.array([200.0, 210.0, 190.0]),
              np.array([390.0, 392.0, 389.0]))]
    pos = np.mod(np.vstack(blobs), L).astype(np.float32).astype(np.float64)
    n = len(pos)
    t = rng.integers(0, 3, n).astype(np.int32)
    q = rng.normal(0, 0.5, n)
    p = dict(box=(L, L, L), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
             sigma=np.array([2.5, 3.0, 3.5]), epsilon=np.array([0.05, 0.1, 0.15]), flags=0)
    lay = api.workspace_layout(p, n)
    assert lay["n_cells"] == 33 ** 3
    f, e, ws, cnt = run(p, pos, t, q, gpu, flags=api.DIAG_COUNTERS)
    _check_fp32(p, pos, t, q, f, e, cnt)
    f64, e64, _, cnt64 = run(p, pos, t, q, gpu, double=True, flags=api.DIAG_COUNTERS)
    r = _ref(p, pos, t, q)
    err = force_errors(f64, r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-12 and e64 == pytest.approx(r.energy, rel=1e-12)
    assert np.array_equal(cnt64, r.count)


def test_empty_and_single_atom(gpu):
    _say("case: n = 0 and n = 1")
    import torch
    s = W.small_system()
    p = api.Params.from_dict(s.params())
    for n in (0, 1):
        pos = torch.full((n, 3), 3.0, device=gpu)
        t = torch.zeros(n, dtype=torch.int32, device=gpu)
        q = torch.ones(n, device=gpu)
        f, e = api.forces(p, pos, t, q)
        torch.cuda.synchronize()
        assert e.item() == 0.0
        if n:
            assert torch.all(f == 0)


def test_wrapping_and_status_bits(gpu):
    _say("case: wrapped positions and device status bits")
    import torch
    s = W.small_system()
    p = s.params()
    pos = s.pos.copy()
    L = np.float32(30.0)
    pos[:100, 0] -= L        # in [-L, 0)
    pos[100:200, 1] += L     # in [L, 2L)
    f, e, ws, _ = run(p, pos, s.types, s.charges, gpu)
    assert api.read_status(ws) == 0
    f0, e0, _, _ = run(p, s.pos, s.types, s.charges, gpu)
    r = _ref(p, pos, s.types, s.charges)
    err = force_errors(f, r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-5
    bad = s.pos.copy(); bad[7, 2] = np.nan
    _, _, ws, _ = run(p, bad, s.types, s.charges, gpu)
    assert api.read_status(ws) & api.STATUS_NAN
    bad = s.pos.copy(); bad[9, 0] = 61.0
    _, _, ws, _ = run(p, bad, s.types, s.charges, gpu)
    assert api.read_status(ws) & api.STATUS_OUT_OF_BOX
    bt = s.types.copy(); bt[3] = 99
    _, _, ws, _ = run(p, s.pos, bt, s.charges, gpu)
    assert api.read_status(ws) & api.STATUS_BAD_TYPE
    # two atoms 0.02 A apart: a pair force far beyond the fixed-point range, in either shell
    close = s.pos.copy(); close[11] = close[10] + np.float32(0.02)
    for flags in (0, api.PAIR_FULL_SHELL):
        _, _, ws, _ = run(p, close, s.types, s.charges, gpu, flags=flags)
        assert api.read_status(ws) & api.STATUS_FIXED_OVERFLOW, flags
    # a clean call on the same workspace clears the sticky word
    run(p, s.pos, s.types, s.charges, gpu, ws=ws)
    assert api.read_status(ws) == 0


def test_stmv_sampled(gpu):
    """1,066,628 atoms: forces of 400 sampled atoms against the oracle's per-atom
    definition, Newton's third law on the whole system, two perturbed evaluations."""
    _say("case: 1,066,628-atom system, sampled atoms")
    import torch
    from _gpu import to_dev
    s = W.stmv_system()
    p = s.params()
    P = api.Params.from_dict(p)
    ws = api.alloc_workspace(P, s.n, gpu)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(s.n, 400, replace=False))
    pos = s.pos
    for step, disp in enumerate(W.perturbation_stream(s.n, 2)):
        if step:
            pos = W.perturb(pos, disp)
        d = to_dev((pos, s.types, s.charges), gpu)
        f, e = api.forces(P, *d, workspace=ws)
        torch.cuda.synchronize()
        assert api.read_status(ws) == 0
        fh = f.double().cpu().numpy()
        ref = oracle.forces_subset(p, pos, s.types, s.charges, idx)
        err = force_errors(fh[idx], ref.force, ref.abs_sum)
        _say("step", step, err)
        assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5
        assert np.linalg.norm(fh.sum(axis=0)) <= 1e-6 * np.abs(fh).sum()


def test_batched_matches_alone(gpu):
    """Serving form: systems of different sizes in one batched call give bitwise the
    results of evaluating each alone. 14 systems exceed one launch batch, one predicated
    system is evaluated on its own inside the call, and two full-shell systems split
    the batches by kind. The last system has 1,728 cells, so its binning takes the path
    for grids of more than 1024 cells while the others take the two-kernel binning."""
    _say("case: 13 serving requests and one 150,000-atom cube, batched vs alone")
    import torch
    from _gpu import to_dev
    reqs, table = W.serving_trace(n_req=64)
    picks = [0, 1, 2, 3, 5, 8, 13, 21, 34, 40, 50, 55, 63, None]
    systems, alone = [], []
    for k, r in enumerate(picks):
        if r is None:
            s = W.gen_system(150_000, (150.0, 150.0, 150.0), seed=31)
            assert api.workspace_layout(s.params(), s.n)["n_cells"] == 12 ** 3
        else:
            s = W.request_system(reqs[r], table)
        flags = api.PAIR_PREDICATED if k == 6 else api.PAIR_FULL_SHELL if k in (3, 4) else 0
        p = api.Params.from_dict(s.params(), flags)
        d = to_dev((s.pos, s.types, s.charges), gpu)
        f, e = api.forces(p, *d)
        alone.append((f.clone(), e.clone()))
        ws = api.alloc_workspace(p, s.n, gpu)
        ws.fill_(0xAB)   # the batched call must not depend on workspace contents
        systems.append(dict(params=p, pos=d[0], types=d[1], charges=d[2],
                            force=torch.full_like(f, float("nan")),
                            energy=torch.full_like(e, float("nan")), workspace=ws))
        _say("  request", r, "atoms", s.n, "box", s.box[0])
    api.forces_batched(systems)
    torch.cuda.synchronize()
    for k, (sysd, (f, e)) in enumerate(zip(systems, alone)):
        assert torch.equal(sysd["force"], f), k
        assert torch.equal(sysd["energy"], e), k
        assert api.read_status(sysd["workspace"]) == 0
    # one of them against the oracle
    s = W.request_system(reqs[picks[0]], table)
    r = _ref(s.params(), s.pos, s.types, s.charges)
    err = force_errors(systems[0]["force"].double().cpu().numpy(), r.force, r.abs_sum)
    assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5, err


def test_serving_loop_outputs(gpu):
    """The serving loop's results equal the plain call's on the same requests, bit for bit:
    inputs copied in and forces copied out with hipMemcpyAsync between pinned host memory
    and slots of one preallocated device pool, batched launches of up to 4 requests; and
    so do the results of the one-at-a-time replay."""
    _say("case: serving loop and plain replay, 12 trace requests, against direct calls")
    import torch
    from paper_1611_04474_amd import serving as S
    from _gpu import to_dev
    reqs, table = W.serving_trace(n_req=12)
    systems = [W.request_system(r, table) for r in reqs]
    items = S.prepare(systems, gpu)
    for it in items:
        it.force_out.fill_(float("nan"))
        it.energy_out.fill_(float("nan"))
    be = S.GpuBackend(gpu, S.pool_bytes(items, 64 << 30), len(items), 2)
    st = S.run_policy(items, np.zeros(len(items)), be, 64 << 30, 4, 2)
    assert st.failed == []
    assert max(st.batches) > 1
    torch.cuda.synchronize()
    got = [(it.force_out.clone(), it.energy_out.clone()) for it in items]
    for it in items:
        it.force_out.fill_(float("nan"))
        it.energy_out.fill_(float("nan"))
    S.replay_plain(items, np.zeros(len(items)), gpu)
    for k, (it, s) in enumerate(zip(items, systems)):
        d = to_dev((s.pos, s.types, s.charges), gpu)
        f, e = api.forces(it.params, *d)
        f, e = f.cpu(), e.cpu()
        assert torch.equal(got[k][0], f) and torch.equal(got[k][1], e), ("batched", k)
        assert torch.equal(it.force_out, f) and torch.equal(it.energy_out, e), ("plain", k)


def test_precision_form_report(gpu):
    """Precision form on the 92,224-atom system: float32 pair arithmetic with 64-bit
    fixed-point per-atom sums against float32-atomic sums, each against the FP64 oracle
    (metrics (i)-(iii) and energy), and bit-reproducibility over 10 runs of each."""
    _say("case: precision form, 92,224 atoms, fixed64 vs f32 atomic vs FP64 oracle")
    import json
    import torch
    from _gpu import to_dev
    s = W.apoa1_system()
    r = _ref(s.params(), s.pos, s.types, s.charges)
    d = to_dev((s.pos, s.types, s.charges), gpu)
    report = {}
    # float32 sums: the compacted full-shell kernel owns each atom in one wave, so its
    # float32 sums run in a fixed order too; the predicated half-shell kernel adds them
    # with float32 atomics
    for name, flags in (("fixed64", 0), ("fixed64_full_shell", api.PAIR_FULL_SHELL),
                        ("f32_sums_full_shell", api.ACCUM_F32_ATOMIC),
                        ("f32_atomic_half_shell", api.ACCUM_F32_ATOMIC | api.PAIR_PREDICATED)):
        p = api.Params.from_dict(s.params(), flags)
        ws = api.alloc_workspace(p, s.n, gpu)
        runs = []
        for k in range(10):
            f, e = api.forces(p, *d, workspace=ws)
            runs.append((f.clone(), e.clone()))
        torch.cuda.synchronize()
        same = sum(torch.equal(runs[k][0], runs[0][0]) and torch.equal(runs[k][1], runs[0][1])
                   for k in range(10))
        err = force_errors(runs[0][0].double().cpu().numpy(), r.force, r.abs_sum)
        e0 = float(runs[0][1].item())
        err["energy_rel"] = abs(e0 - r.energy) / abs(r.energy)
        err["bitwise_identical_runs_of_10"] = int(same)
        report[name] = err
    _say("PRECISION_REPORT " + json.dumps(report))
    assert report["fixed64"]["bitwise_identical_runs_of_10"] == 10
    assert report["fixed64_full_shell"]["bitwise_identical_runs_of_10"] == 10
    for name in report:
        assert report[name]["max_norm"] <= 1e-5 and report[name]["rms"] <= 1e-5, report
        assert report[name]["energy_rel"] <= 1e-6, report


@pytest.mark.parametrize("drain", [1, 3, 4])
def test_drain_depths(gpu, drain):
    """The half-shell kernel instantiated with other drain depths (the candidate-batches
    per force pass sweep) against the oracle, with a multi-pass neighbour load too."""
    _say("case: drain depth", drain)
    s = W.small_system()
    p = s.params()
    f, e, ws, cnt = run(p, s.pos, s.types, s.charges, gpu,
                        flags=api.PAIR_DRAIN(drain) | api.DIAG_COUNTERS)
    _check_fp32(p, s.pos, s.types, s.charges, f, e, cnt)
    assert api.read_status(ws) == 0
    rng = np.random.default_rng(11)
    L = 37.0
    pos = np.mod(_lattice_blob(rng, np.zeros(3), 20, 1.85, 0.3), L).astype(np.float32).astype(np.float64)
    t = rng.integers(0, 2, len(pos)).astype(np.int32)
    q = rng.normal(0, 0.3, len(pos))
    p2 = dict(box=(L, L, L), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
              sigma=np.array([1.0, 1.2]), epsilon=np.array([0.05, 0.1]), flags=0)
    f2, e2, ws2, cnt2 = run(p2, pos, t, q, gpu, flags=api.PAIR_DRAIN(drain) | api.DIAG_COUNTERS)
    _check_fp32(p2, pos, t, q, f2, e2, cnt2)


@pytest.mark.parametrize("shell", [0, api.PAIR_FULL_SHELL])
@pytest.mark.parametrize("case", ["truncated_coulomb", "no_switch", "sixty_four_types"])
def test_fp32_kernel_variants(gpu, case, shell):
    """The float32 compacted kernel's other instantiations against the oracle: Coulomb
    truncated (only LJ switched), switching off (r_switch = r_cut: lanes are masked, not
    clamped), and 64 atom types (the largest LJ table, the smallest LDS neighbour load)."""
    _say("case: float32 kernel variant", case, "flags", shell)
    if case == "sixty_four_types":
        s = W.gen_system(20000, (60.0, 60.0, 55.0), 13, n_types=64)
        p = s.params()
    else:
        s = W.small_system()
        p = s.params()
        if case == "truncated_coulomb":
            p = dict(p, flags=api.COULOMB_TRUNCATED)
        else:
            p = dict(p, r_switch=p["r_cut"])
    f, e, ws, cnt = run(p, s.pos, s.types, s.charges, gpu,
                        flags=p.get("flags", 0) | shell | api.DIAG_COUNTERS)
    if case == "sixty_four_types":
        _check_fp32(p, s.pos, s.types, s.charges, f, e, cnt)
        return
    # without a switch at r_cut the force jumps there: an atom with a partner within 8
    # float32 ulps of rc^2 may see that pair classified differently in float32 and FP64,
    # so those atoms are compared for partner counts only and reported
    r = _ref(p, s.pos, s.types, s.charges)
    band, nb = oracle.band_atoms(p, s.pos, BAND)
    keep = band == 0
    err = force_errors(f[keep], r.force[keep], r.abs_sum[keep])
    _say("fp32 errors (atoms off the cutoff band)", err, "band atoms", int((~keep).sum()))
    assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5, err
    ok = (cnt == r.count) | (band > 0)
    assert ok.all()
    if nb == 0:
        assert e == pytest.approx(r.energy, rel=1e-6, abs=1e-6)


_TINY = [((24.5, 24.5, 24.5), 150, 1), ((36.5, 36.5, 36.5), 300, 2), ((24.5, 37.0, 50.0), 260, 3),
         ((40.0, 26.0, 31.0), 5, 4)]
_COMPACT_FORMS = [(0, "half shell, 2 batches per drain"),
                  (api.PAIR_DRAIN(1), "half shell, 1 batch per drain"),
                  (api.PAIR_FULL_SHELL, "full shell")]


@pytest.mark.parametrize("box,n,seed", _TINY)
@pytest.mark.parametrize("form", range(len(_COMPACT_FORMS)))
def test_fp32_compacted_tiny_grids(gpu, box, n, seed, form):
    """The float32 compacted kernel on the grids the oracle's cell list is pinned on:
    2x2x2 and 3x3x3 cells, a mixed 2x3x4 grid (two images of one cell on some axes only,
    the n_d = 2 case of the 27-cell stencil) and a 5-atom system on a 3x2x2 grid."""
    flags, what = _COMPACT_FORMS[form]
    _say("case: float32 compacted kernel, tiny system", box, n, seed, what)
    pos, t, q, p = _random_system(n, box, seed)
    f, e, ws, cnt = run(p, pos, t, q, gpu, flags=flags | api.DIAG_COUNTERS)
    r, err = _check_fp32(p, pos, t, q, f, e, cnt)
    band, nb = oracle.band_atoms(p, pos, BAND)
    assert abs(api.read_diag(ws)[2] - r.n_pairs) <= nb
    assert api.read_status(ws) == 0


def _cutoff_pairs():
    """Four pairs in a 40 A box, each atom at least 20 A from every atom of another pair:
    exactly r_cut apart inside the box and through the x face (both excluded by the strict
    test u < rc^2), and one float32 step closer than r_cut, inside and through the face
    (both included). Every coordinate and every displacement is exact in float32."""
    x_in = float(np.nextafter(np.float32(15.0), np.float32(0.0)))
    x_face = float(np.nextafter(np.float32(28.5), np.float32(40.0)))
    pos = np.array([[3.0, 5.0, 5.0], [15.0, 5.0, 5.0],          # 12 A exactly
                    [3.0, 25.0, 5.0], [x_in, 25.0, 5.0],         # just inside
                    [0.5, 5.0, 25.0], [28.5, 5.0, 25.0],         # 12 A through the face
                    [0.5, 25.0, 25.0], [x_face, 25.0, 25.0]])    # just inside, through it
    t = np.array([0, 1, 0, 1, 1, 0, 1, 0], np.int32)
    q = np.array([0.5, -0.4, 0.3, 0.6, -0.2, 0.5, 0.4, 0.4])
    return pos, t, q


@pytest.mark.parametrize("switch", [10.0, 11.5, 12.0])
def test_exact_cutoff_pairs(gpu, switch):
    """Algorithm 1's strict cutoff on pairs exactly r_cut apart and one float32 step
    inside, with the switch on and off, in both shells of the float32 kernel and in
    float64: partner counts 0 / 1 exactly, zero force on the excluded pairs. At
    r_switch = 11.5 A the float32 product (rc^2 - rs^2) * fl(1/(rc^2 - rs^2)) rounds to
    just below 1, so a switch variable t = (u - rs^2) / (rc^2 - rs^2) would stop short of 1
    at the cutoff; and 1 - t near the cutoff is a few ulps of 1, where the switch's force
    term, which dominates there, is proportional to it.
    The float32 kernel's u of a pair just inside is rc^2 less one to three ulps (1.5e-5 A^2
    each), so u itself fixes rc^2 - u only to about a third for the first pair. Its forces
    are compared with the oracle's pair terms at that float32 u, float64's with the oracle's
    exact forces."""
    _say("case: pairs at and just inside r_cut, r_switch", switch)
    pos, t, q = _cutoff_pairs()
    p = dict(box=(40.0, 40.0, 40.0), r_cut=12.0, r_switch=switch, coulomb_k=W.COULOMB_K,
             sigma=np.array([2.5, 3.0]), epsilon=np.array([0.05, 0.1]), flags=0)
    r = oracle.forces(p, pos, t, q, "bruteforce")
    scale = oracle.forces(dict(p, r_switch=12.0), pos, t, q, "bruteforce")
    assert list(r.count) == [0, 0, 1, 1, 0, 0, 1, 1]
    # the pairs just inside: displacement (exact in float32) and the float32 u = fl(dx^2)
    ref32 = np.zeros((8, 3))
    q32 = q.astype(np.float32).astype(np.float64)
    for i, j in ((2, 3), (6, 7)):
        dx = pos[i, 0] - pos[j, 0]
        dx -= 40.0 * np.round(dx / 40.0)
        u32 = float(np.float32(dx) * np.float32(dx))
        fij = oracle.pair_terms(p, t[i], t[j], q32[i], q32[j], u32)[1]
        ref32[i, 0], ref32[j, 0] = fij * dx, -fij * dx
    for flags, double in ((0, False), (api.PAIR_FULL_SHELL, False), (0, True)):
        f, e, ws, cnt = run(p, pos, t, q, gpu, double=double, flags=flags | api.DIAG_COUNTERS)
        _say("flags", flags, "double", double, "counts", cnt.tolist())
        assert list(cnt) == [0, 0, 1, 1, 0, 0, 1, 1], (flags, double)
        assert np.all(f[[0, 1, 4, 5]] == 0.0), (flags, double)
        # errors on the scale of the unswitched pair (the switch is near 0 at r_cut)
        tol = 1e-12 if double else 1e-5
        ref = r.force if double else ref32
        for i in (2, 3, 6, 7):
            assert np.linalg.norm(f[i] - ref[i]) <= tol * np.linalg.norm(scale.force[i]), (i, flags)
        assert abs(e - r.energy) <= tol * abs(scale.energy), (flags, double)
        assert api.read_diag(ws)[2] == 2


def test_overflow_bound_per_partial(gpu):
    """The float32 per-atom sums have a 2^35 kcal/mol/A range; every partial added into one
    is checked against its share (one pair's or one workgroup's neighbour-side term below
    2^27, home-side partials below what the 14 n_split neighbour-side ones leave, divided
    by the LDS slices), so a sum can never wrap. A pair force of 1.1e8 (below 2^27) sets no
    status bit, in a system whose neighbour lists take three slices and in one that takes
    one; a pair force of 1.5e8 (above) sets it in both."""
    _say("case: 1.1e8 and 1.5e8 kcal/mol/A pair forces, three slices and one slice")
    p_of = lambda L: dict(box=(L, L, L), r_cut=12.0, r_switch=10.0, coulomb_k=W.COULOMB_K,
                          sigma=np.array([1.0, 1.2]), epsilon=np.array([0.05, 0.1]), flags=0)

    def distance_for(target):
        lo, hi = 0.1, 0.6              # |F| of a type-0 pair falls with r on [0.1, 0.6] A
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            f = oracle.pair_terms(p_of(24.5), 0, 0, 0.0, 0.0, mid * mid)[1] * mid
            lo, hi = (mid, hi) if f > target else (lo, mid)
        return np.float32(lo)

    rng = np.random.default_rng(31)
    # 4,096 atoms on a 16^3 lattice in a 24.5 A box (2x2x2 cells): 14 x 512 atoms in each
    # home cell's half-shell list, three LDS slices; 60 atoms in a 40 A box: one slice
    dense = np.mod(_lattice_blob(rng, np.full(3, 0.4), 16, 1.53, 0.05), 24.5)
    sparse = np.mod(_lattice_blob(rng, np.full(3, 1.0), 4, 9.5, 0.5), 40.0)[:60]
    for target, want in ((1.1e8, False), (1.5e8, True)):
        r = distance_for(target)
        for base, L in ((dense, 24.5), (sparse, 40.0)):
            pos = base.astype(np.float32)
            pos[1] = pos[0] + np.array([r, 0, 0], np.float32)   # the close pair, along x
            n = len(pos)
            t = np.zeros(n, np.int32)
            q = np.zeros(n)
            p = p_of(L)
            f, e, ws, _ = run(p, pos.astype(np.float64), t, q, gpu)
            st = api.read_status(ws)
            _say("target", target, "box", L, "atoms", n, "status", st, "pair force", f[0, 0])
            assert bool(st & api.STATUS_FIXED_OVERFLOW) == want, (target, L, st)
            if not want:
                # the pair's own forces (the other atoms carry ~1e-6 kcal/mol/A, below the
                # 2^-24 rounding of the neighbour-side sums)
                ref = oracle.forces(p, pos, t, q, "bruteforce")
                err = force_errors(f[:2], ref.force[:2], ref.abs_sum[:2])
                assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5, err


def test_serving_failed_request_alone(gpu):
    """A request with a NaN position in a batch of six comes back failed (its device status
    word, copied back behind the results); the other five give the plain call's bits. A
    request whose box the library rejects fails at admission and is never launched."""
    _say("case: serving loop with a NaN request and a rejected one")
    import torch
    from paper_1611_04474_amd import serving as S
    from _gpu import to_dev
    reqs, table = W.serving_trace(n_req=7)
    systems = [W.request_system(r, table) for r in reqs]
    systems[5].box = np.array([20.0, 20.0, 20.0])      # under 2 r_cut: rejected
    items = S.prepare(systems, gpu)
    assert not items[5].valid and all(it.valid for k, it in enumerate(items) if k != 5)
    items[3].pos[5, 0] = float("nan")
    be = S.GpuBackend(gpu, S.pool_bytes(items, 64 << 30), len(items), 2)
    st = S.run_policy(items, np.zeros(len(items)), be, 64 << 30, 8, 2)
    assert sorted(st.failed) == [3, 5], st.failed
    assert items[3].status & api.STATUS_NAN
    for k, (it, s) in enumerate(zip(items, systems)):
        if k in (3, 5):
            continue
        assert it.status == 0
        d = to_dev((s.pos, s.types, s.charges), gpu)
        f, e = api.forces(it.params, *d)
        assert torch.equal(it.force_out, f.cpu()) and torch.equal(it.energy_out, e.cpu()), k
    st = S.replay_plain(items, np.zeros(len(items)), gpu)
    assert sorted(st.failed) == [3, 5]


def test_copy_segments(gpu):
    """md_copy_segments moves byte ranges pinned host -> device and device -> pinned host
    with one kernel launch per call: 16-byte and byte-wise paths (misaligned ends), ranges
    of several 64 KB chunks, and empty ranges."""
    _say("case: md_copy_segments")
    import torch
    from paper_1611_04474_amd import serving as S
    rng = np.random.default_rng(8)
    sizes = [0, 1, 15, 16, 4096 + 3, 3 * 65536 + 40, 1 << 20]
    host = [torch.from_numpy(rng.integers(0, 256, n + 32, dtype=np.uint8)).pin_memory() for n in sizes]
    for h in host:
        assert S.device_mapped(h)
    dev = [torch.zeros(n + 32, dtype=torch.uint8, device=gpu) for n in sizes]
    back = [torch.zeros(n + 32, dtype=torch.uint8).pin_memory() for n in sizes]
    stream = torch.cuda.current_stream()
    # host -> device at offsets 0 (aligned) and 3 (misaligned), then device -> host
    for off in (0, 3):
        api.copy_segments([(d.data_ptr() + off, h.data_ptr() + off, n)
                           for d, h, n in zip(dev, host, sizes)], stream.cuda_stream)
        api.copy_segments([(b.data_ptr() + off, d.data_ptr() + off, n)
                           for b, d, n in zip(back, dev, sizes)], stream.cuda_stream)
        torch.cuda.synchronize()
        for d, h, b, n in zip(dev, host, back, sizes):
            assert torch.equal(d.cpu()[off:off + n], h[off:off + n]), n
            assert torch.equal(b[off:off + n], h[off:off + n]), n


@pytest.mark.parametrize("shell", [0, api.PAIR_FULL_SHELL])
@pytest.mark.parametrize("double", [False, True])
def test_work_split_same_bits(gpu, shell, double):
    """One, two or four workgroups per home cell (each taking every s-th group of home atoms;
    automatic choice too) give the same bits: forces from integer sums, and the energy from
    the workgroups' exact integer partials added as integers. A 20,000-atom cube of 4^3
    cells and the 3,000-atom system of 2^3 cells."""
    _say("case: work split 1/2/4/auto, shell", shell, "double", double)
    for s in (W.gen_system(20000, (58.5, 58.5, 58.5), 12), W.small_system()):
        p = s.params()
        pos = s.pos.astype(np.float64) if double else s.pos
        q = s.charges.astype(np.float64) if double else s.charges
        res = [run(p, pos, s.types, q, gpu, double=double, flags=shell | fl)[:2]
               for fl in (api.PAIR_SPLIT(1), api.PAIR_SPLIT(2), api.PAIR_SPLIT(4), 0)]
        for f, e in res[1:]:
            assert np.array_equal(f, res[0][0]) and e == res[0][1]
    r = oracle.forces(p, s.pos, s.types, s.charges, "celllist")
    err = force_errors(res[0][0], r.force, r.abs_sum)
    assert err["max_norm"] <= (1e-12 if double else 1e-5)
