"""The motion update (md_run_vv_f32: velocity Verlet around the force path) against the
oracle's velocity Verlet around the FP64 force call, through the C ABI.

Bars, from the float32 state the GPU keeps: after 20 steps of 0.5 fs, positions within
1e-4 A (a float32 rounding of a 30 A coordinate is 1.9e-6 A per step), velocities within
1e-5 A/fs plus 1e-4 of the largest (the force error of 1e-6 relative integrated over 10 fs
gives under 4e-7 A/fs for the lightest atom), potential and kinetic energy within 1e-5
relative to the sum of their magnitudes; results bitwise identical across runs."""
import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import api
from paper_1611_04474_amd import workloads as W

from _gpu import to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _state(gpu, n=3000, box=(30.0, 30.0, 30.0)):
    import torch
    s = W.liquid_system(n, box)
    v, im = W.velocities(s.types)
    p = api.Params.from_dict(s.params())
    pos, t, q = to_dev((s.pos, s.types, s.charges), gpu)
    vel = torch.as_tensor(v).to(gpu)
    inv_m = torch.as_tensor(im).to(gpu)
    ws = api.alloc_workspace(p, s.n, gpu)
    f, _ = api.forces(p, pos, t, q, workspace=ws)
    return s, v, im, p, pos, t, q, vel, inv_m, f, ws


def test_vv_matches_oracle(gpu):
    _say("case: velocity Verlet, 3,000 atoms, 20 steps of 0.5 fs")
    import torch
    s, v0, im, p, pos, t, q, vel, inv_m, f, ws = _state(gpu)
    en = api.run_vv(p, pos, vel, t, q, inv_m, f, 0.5, 20, workspace=ws)
    torch.cuda.synchronize()
    assert api.read_status(ws) == 0
    x, v, F, pe, ke = oracle.vv_steps(s.params(), s.pos, v0.astype(np.float64), s.types, s.charges,
                                      im.astype(np.float64), 0.5, 20)
    gx = pos.double().cpu().numpy()
    gv = vel.double().cpu().numpy()
    ge = en.cpu().numpy()
    dx = gx - x
    dx -= 30.0 * np.round(dx / 30.0)
    dv = np.abs(gv - v).max()
    _say("max |dx|", np.abs(dx).max(), "max |dv|", dv, "max |v|", np.abs(v).max())
    assert np.abs(dx).max() <= 1e-4
    assert dv <= 1e-5 + 1e-4 * np.abs(v).max()
    scale = np.abs(pe) + np.abs(ke)
    _say("pe rel", np.max(np.abs(ge[:, 0] - pe) / scale), "ke rel", np.max(np.abs(ge[:, 1] - ke) / scale))
    assert np.all(np.abs(ge[:, 0] - pe) <= 1e-5 * scale)
    assert np.all(np.abs(ge[:, 1] - ke) <= 1e-5 * scale)
    # the forces left behind are the forces at the final positions
    r = oracle.forces(s.params(), gx.astype(np.float32), s.types, s.charges)
    fn = f.double().cpu().numpy()
    assert np.linalg.norm(fn - r.force) <= 1e-5 * np.linalg.norm(r.force)


def test_vv_bitwise_reproducible_and_conserves_energy(gpu):
    """Two runs of 200 steps of 0.5 fs give the same bits, and the total energy deviates
    from its start by at most twice what the oracle's FP64 velocity Verlet shows on the
    same system and step (the integrator's own O(dt^2) error, plus room for float32)."""
    _say("case: velocity Verlet, 3,000 atoms, 2 x 200 steps")
    import torch
    out = []
    for rep in range(2):
        s, v0, im, p, pos, t, q, vel, inv_m, f, ws = _state(gpu)
        en = api.run_vv(p, pos, vel, t, q, inv_m, f, 0.5, 200, workspace=ws)
        torch.cuda.synchronize()
        assert api.read_status(ws) == 0
        out.append((pos.clone(), vel.clone(), en.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])
    e = out[0][2].cpu().numpy()
    tot = e[:, 0] + e[:, 1]
    _, _, _, pe, ke = oracle.vv_steps(s.params(), s.pos, v0.astype(np.float64), s.types,
                                      s.charges, im.astype(np.float64), 0.5, 200)
    ref = np.abs(pe + ke - (pe + ke)[0]).max()
    dev = np.abs(tot - tot[0]).max()
    _say("E0", tot[0], "max dev gpu", dev, "oracle", ref, "ke", e[0, 1], e[-1, 1])
    assert dev <= 2 * ref


def test_vv_zero_steps_and_pinned_atoms(gpu):
    _say("case: velocity Verlet, 0 steps; atoms with 1/m = 0 stay put")
    import torch
    s, v0, im, p, pos, t, q, vel, inv_m, f, ws = _state(gpu, n=500, box=(30.0, 30.0, 30.0))
    p0 = pos.clone()
    api.run_vv(p, pos, vel, t, q, inv_m, f, 0.5, 0, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(pos, p0)
    vel[:10] = 0
    inv_m[:10] = 0
    api.run_vv(p, pos, vel, t, q, inv_m, f, 0.5, 5, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(pos[:10], p0[:10]) and torch.all(vel[:10] == 0)
    assert not torch.equal(pos[10:], p0[10:])
