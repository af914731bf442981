"""Ewald summation on the GPU against the FP64 oracle, through the C ABI: the real-space
erfc term inside the cutoff (MD_COULOMB_EWALD on the compacted kernel, float32 in both
shells and float64), the reciprocal-space sum with self and background terms
(md_ewald_recip_f32), and the two together against the oracle's total.

Bars: the real-space term as every short-range parity test (float32: metrics (ii) and (iii)
<= 1e-5, energy <= 1e-6; float64: 1e-12). Reciprocal space (float32 products, exact phases,
float64 sums across tiles): energy <= 1e-6 relative, RMS force error <= 1e-5 of the RMS
force, largest per-atom error <= 1e-5 of the largest force."""
import math

import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import api
from paper_1611_04474_amd import workloads as W

from _gpu import run, to_dev
from _metrics import force_errors

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def kmax_for(box, alpha, tol=1e-6):
    h = alpha * math.sqrt(-math.log(tol)) / math.pi
    return [int(math.ceil(h * float(np.float32(L)))) for L in box]


def ewald_params(s, alpha):
    return dict(s.params(), flags=api.COULOMB_EWALD, ewald_alpha=alpha)


def _recip_gpu(p, s, kmax, gpu, force=None, accumulate=False):
    import torch
    d = to_dev((s.pos, s.types, s.charges), gpu)
    f, e, ws = api.ewald_recip(api.Params.from_dict(p), d[0], d[2], kmax, force=force,
                               accumulate=accumulate)
    torch.cuda.synchronize()
    return f, float(e.item()), ws


def _recip_errors(fg, eg, ref_f, ref_e):
    d = np.linalg.norm(fg - ref_f, axis=1)
    rms = float(np.linalg.norm(fg - ref_f) / np.linalg.norm(ref_f))
    mx = float(d.max() / np.linalg.norm(ref_f, axis=1).max())
    return dict(rms=rms, max_rel_to_largest=mx, energy_rel=abs(eg - ref_e) / abs(ref_e))


@pytest.mark.parametrize("flags,double", [(0, False), (api.PAIR_FULL_SHELL, False), (0, True)])
def test_real_space_term(gpu, flags, double):
    _say("case: Ewald real-space term, 3,000 atoms, flags", flags, "double", double)
    s = W.small_system()
    p = ewald_params(s, 0.3)
    pos = s.pos.astype(np.float64) if double else s.pos
    q = s.charges.astype(np.float64) if double else s.charges
    f, e, ws, cnt = run(p, pos, s.types, q, gpu, double=double,
                        flags=api.COULOMB_EWALD | flags | api.DIAG_COUNTERS)
    r = oracle.forces(dict(p, flags=oracle.FLAG_EWALD), s.pos, s.types, s.charges, "celllist")
    err = force_errors(f, r.force, r.abs_sum)
    _say("errors", err, "energy", e, r.energy)
    tol, etol = (1e-12, 1e-12) if double else (1e-5, 1e-6)
    assert err["max_norm"] <= tol and err["rms"] <= tol
    assert e == pytest.approx(r.energy, rel=etol)
    assert api.read_status(ws) == 0


@pytest.mark.parametrize("box,n,seed,net", [((30.0, 30.0, 30.0), 3000, 1, 0.0),
                                            ((40.0, 43.0, 47.0), 8000, 3, 0.0),
                                            ((26.0, 31.0, 29.0), 2000, 5, 2.5),
                                            # 87 values of mz: two mz chunks of the force
                                            # kernel and two mz blocks of the structure factors
                                            ((26.0, 27.0, 120.0), 2000, 6, 0.0)])
def test_reciprocal_sum(gpu, box, n, seed, net):
    """Reciprocal forces and energy against the oracle's plain sum over wave vectors, on a
    cube, a non-cubic box (its axes' wave numbers differ) and a system with net charge."""
    _say("case: Ewald reciprocal sum", box, n, seed, "net charge", net)
    s = W.gen_system(n, box, seed)
    s.charges = (s.charges + np.float32(net / n)).astype(np.float32)
    alpha = 0.3
    p = ewald_params(s, alpha)
    km = kmax_for(s.box, alpha)
    f, e, ws = _recip_gpu(p, s, km, gpu)
    ref_f, er, es, eb = oracle.ewald_recip(p, s.pos, s.charges, km)
    err = _recip_errors(f.double().cpu().numpy(), e, ref_f, er + es + eb)
    _say("kmax", km, "errors", err, "energy", e, er + es + eb)
    assert err["energy_rel"] <= 1e-6 and err["rms"] <= 1e-5 and err["max_rel_to_largest"] <= 1e-5
    assert api.read_status(ws) == 0
    # the same bits again
    f2, e2, _ = _recip_gpu(p, s, km, gpu)
    assert e2 == e and bool((f2 == f).all())


def test_total_coulomb_short_plus_reciprocal(gpu):
    """Short-range forces with the erfc term plus the reciprocal forces added onto them
    (accumulate) against the oracle's real-space + reciprocal total."""
    _say("case: Ewald total, 3,000 atoms")
    s = W.small_system()
    alpha = 0.3
    p = ewald_params(s, alpha)
    km = kmax_for(s.box, alpha)
    f_short, e_short, ws, _ = run(p, s.pos, s.types, s.charges, gpu, flags=api.COULOMB_EWALD)
    import torch
    fs = torch.as_tensor(f_short.astype(np.float32)).to(gpu)
    f, e_rec, _ = _recip_gpu(p, s, km, gpu, force=fs, accumulate=True)
    real = oracle.forces(dict(p, flags=oracle.FLAG_EWALD), s.pos, s.types, s.charges, "celllist")
    ref_f, er, es, eb = oracle.ewald_recip(p, s.pos, s.charges, km)
    total_ref = real.force + ref_f
    fg = f.double().cpu().numpy()
    rms = np.linalg.norm(fg - total_ref) / np.linalg.norm(total_ref)
    etot, eref = e_short + e_rec, real.energy + er + es + eb
    _say("total rms", rms, "energy", etot, eref)
    assert rms <= 1e-5
    assert etot == pytest.approx(eref, rel=1e-6)


def test_reciprocal_edge_cases(gpu):
    import torch
    _say("case: Ewald reciprocal sum, no atoms, one atom, NaN")
    s = W.small_system()
    p = api.Params.from_dict(ewald_params(s, 0.3))
    for n in (0, 1):
        pos = torch.full((n, 3), 3.0, device=gpu)
        q = torch.full((n,), 0.7, device=gpu)
        f, e, ws = api.ewald_recip(p, pos, q, (5, 5, 5))
        torch.cuda.synchronize()
        if n == 0:
            assert e.item() == 0.0
        else:
            # one charge: |S|^2 = q^2 for every wave vector, no force, and the energy is the
            # oracle's recip + self + background
            F, er, es, eb = oracle.ewald_recip(dict(ewald_params(s, 0.3)), np.full((1, 3), 3.0),
                                               [0.7], (5, 5, 5))
            assert e.item() == pytest.approx(er + es + eb, rel=1e-6)
            assert float(f.abs().max()) < 1e-5
    pos = torch.as_tensor(s.pos).to(gpu)
    pos[4, 1] = float("nan")
    q = torch.as_tensor(s.charges).to(gpu)
    _, _, ws = api.ewald_recip(p, pos, q, (5, 5, 5))
    assert api.read_status(ws) & api.STATUS_NAN
