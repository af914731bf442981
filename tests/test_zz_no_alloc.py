"""md_forces_f32_noalloc (the entry point for callers that cannot allocate) against
md_forces_f32 with a caller-owned workspace, through the C ABI: two calls in a row on the
library's per-device workspace, the second with a smaller system, each bitwise equal to
the plain call (64-bit fixed-point sums are independent of order and of what the
workspace held before), and the smaller one against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import api
from paper_1611_04474_amd import workloads as W

from _gpu import to_dev
from _metrics import force_errors

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _noalloc(p, d, gpu):
    import torch
    n = d[0].shape[0]
    f = torch.empty((n, 3), dtype=torch.float32, device=gpu)
    e = torch.empty(1, dtype=torch.float64, device=gpu)
    st = torch.full((1,), -1, dtype=torch.int32, device=gpu)
    api.forces_noalloc(p, *d, f, e, st)
    torch.cuda.synchronize()
    return f, e, int(st.item())


def test_noalloc_matches_plain_call(gpu):
    import torch
    for name, make in (("92,224 atoms", W.apoa1_system), ("3,000 atoms", W.small_system)):
        _say("case: no-allocation entry point,", name)
        s = make()
        p = api.Params.from_dict(s.params())
        d = to_dev((s.pos, s.types, s.charges), gpu)
        f0, e0 = api.forces(p, *d)
        torch.cuda.synchronize()
        f1, e1, st = _noalloc(p, d, gpu)
        assert st == 0
        assert torch.equal(f0, f1) and torch.equal(e0, e1), name
        if s.n <= 3000:
            r = oracle.forces(s.params(), s.pos, s.types, s.charges, "celllist")
            err = force_errors(f1.double().cpu().numpy(), r.force, r.abs_sum)
            _say("errors against the oracle", err)
            assert err["max_norm"] <= 1e-5 and err["rms"] <= 1e-5
            assert float(e1.item()) == pytest.approx(r.energy, rel=1e-6)


def test_noalloc_status_and_limit(gpu):
    import torch
    _say("case: no-allocation entry point, status word and size limit")
    s = W.small_system()
    p = api.Params.from_dict(s.params())
    bad = s.pos.copy()
    bad[5, 1] = np.nan
    _, _, st = _noalloc(p, to_dev((bad, s.types, s.charges), gpu), gpu)
    assert st & api.STATUS_NAN
    _, _, st = _noalloc(p, to_dev((s.pos, s.types, s.charges), gpu), gpu)
    assert st == 0
    big = W.stmv_system()
    pb = api.Params.from_dict(big.params())
    d = to_dev((big.pos, big.types, big.charges), gpu)
    f = torch.zeros((big.n, 3), dtype=torch.float32, device=gpu)
    e = torch.zeros(1, dtype=torch.float64, device=gpu)
    with pytest.raises(api.MDError) as ex:
        api.forces_noalloc(pb, *d, f, e)
    assert ex.value.code == -6
    torch.cuda.synchronize()
    assert torch.count_nonzero(f).item() == 0      # nothing was enqueued
