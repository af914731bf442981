"""Host-side checks of the C ABI: the library loads and exports every declared
entry point, the workspace and grid logic, and synchronous argument errors. No
call here reaches the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1611_04474_amd import api
from paper_1611_04474_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mdforce.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 8
    lib = api.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(api.EXPORTED)


def test_read_calls_reject_null_workspace():
    """The read calls check their pointers before any device call."""
    v = C.c_double(1.0)
    assert api.lib().md_read_clock(None, None, C.byref(v)) == -1
    assert v.value == 1.0
    w = (C.c_uint64 * 5)()
    assert api.lib().md_read_diag(None, None, w) == -1


def test_status_strings():
    assert api.status_string(0) == "ok"
    assert "workspace" in api.status_string(-3)


@pytest.mark.parametrize("make", [W.small_system, W.apoa1_system])
def test_grid_matches_oracle_rule(make):
    s = make()
    for dp in (False, True):
        lay = api.workspace_layout(s.params(), s.n, dp)
        assert lay["dims"] == oracle.grid(s.params())
        assert lay["total_bytes"] == api.workspace_bytes(s.params(), s.n, dp)


def test_grid_margin_and_rejection():
    p = W.small_system().params()
    p2 = dict(p, box=(36.002, 36.0, 30.0))
    assert api.workspace_layout(p2, 10)["dims"] == (2, 2, 2)
    for bad in ((23.9, 30.0, 30.0), (24.0005, 30.0, 30.0)):
        with pytest.raises(api.MDError) as e:
            api.workspace_layout(dict(p, box=bad), 10)
        assert e.value.code == -2


def test_workspace_grows_with_atoms():
    p = W.apoa1_system().params()
    a = api.workspace_bytes(p, 1000)
    b = api.workspace_bytes(p, 92224)
    c = api.workspace_bytes(p, 92224, True)
    assert 0 < a < b < c
    # the compacted kernel keeps three int64 sums per atom (float64: two words each); the
    # predicated kernel 27 partial-force slots
    assert b >= 3 * 8 * 92224
    assert c >= 3 * 16 * 92224
    pred = dict(p, flags=api.PAIR_PREDICATED)
    assert api.workspace_bytes(pred, 92224) >= 27 * 3 * 4 * 92224 > b
    assert api.workspace_bytes(pred, 92224, True) >= 27 * 3 * 8 * 92224 > c


def _call_f32(params, n=10, ws_bytes=1 << 20, ws_ptr=256, ptr=4096):
    return api.forces_raw(params, n, ptr, ptr, ptr, ptr, ptr, ws_ptr, ws_bytes, 0)


def test_argument_errors_are_synchronous():
    base = W.small_system().params()
    need = api.workspace_bytes(base, 10)
    assert _call_f32(dict(base, r_switch=13.0), ws_bytes=need) == -1
    assert _call_f32(dict(base, r_cut=-1.0), ws_bytes=need) == -1
    assert _call_f32(dict(base, box=(20.0, 30.0, 30.0)), ws_bytes=need) == -2
    assert _call_f32(dict(base, sigma=np.zeros(0), epsilon=np.zeros(0)), ws_bytes=need) == -1
    assert _call_f32(dict(base, sigma=np.ones(65), epsilon=np.ones(65)), ws_bytes=need) == -6
    assert _call_f32(dict(base, epsilon=-np.ones(8)), ws_bytes=need) == -1
    assert _call_f32(dict(base, flags=1 << 20), ws_bytes=need) == -1
    assert _call_f32(base, ws_bytes=need - 1) == -3
    assert _call_f32(base, ws_bytes=need, ws_ptr=0) == -3
    assert _call_f32(base, ws_bytes=need, ws_ptr=300) == -3      # not 256-aligned
    assert _call_f32(base, n=-1, ws_bytes=need) == -1
    assert _call_f32(base, ws_bytes=need, ptr=0) == -1
    assert _call_f32(base, ws_bytes=need, ptr=4098) == -1         # misaligned float pointer
    assert api.forces_raw(base, 10, 4096, 4096, 4096, 4096, 4096, 256, need, 0,
                          double_precision=True) == -3             # f64 needs more workspace


def test_drain_depth_only_where_the_kernel_has_it():
    base = W.small_system().params()
    need = api.workspace_bytes(base, 10)
    assert [api.PAIR_DRAIN(d) for d in (2, 1, 3, 4)] == [0, 1 << 5, 2 << 5, 3 << 5]
    for bad in (api.PAIR_FULL_SHELL, api.PAIR_PREDICATED, api.ACCUM_F32_ATOMIC,
                api.COULOMB_TRUNCATED):
        assert _call_f32(dict(base, flags=api.PAIR_DRAIN(3) | bad), ws_bytes=need) == -1
    # r_switch == r_cut: no clamp, so no other drain depth
    assert _call_f32(dict(base, r_switch=base["r_cut"], flags=api.PAIR_DRAIN(1)),
                     ws_bytes=need) == -1
    need64 = api.workspace_bytes(base, 10, True)
    assert api.forces_raw(dict(base, flags=api.PAIR_DRAIN(4)), 10, 4096, 4096, 4096, 4096, 4096,
                          256, need64, 0, double_precision=True) == -1


def test_batched_rejects_before_enqueue():
    base = W.small_system().params()

    class Fake:
        def __init__(self, shape, ptr=4096):
            self.shape = shape
            self._p = ptr

        def data_ptr(self):
            return self._p

        def numel(self):
            return 64

    sys_ok = dict(params=base, pos=Fake((10, 3)), types=Fake((10,)), charges=Fake((10,)),
                  force=Fake((10, 3)), energy=Fake((1,)), workspace=Fake((64,), 256))
    with pytest.raises(api.MDError) as e:
        api.forces_batched([sys_ok], stream=0)
    assert e.value.code == -3


def test_motion_update_argument_errors_are_synchronous():
    import ctypes as C
    base = W.small_system().params()
    P = api.Params.from_dict(base)
    need = api.workspace_bytes(base, 10)
    L = api.lib()

    def call(n=10, vel=4096, inv_m=4096, dt=0.5, steps=3, ws_bytes=need, energies=4096, p=P):
        return L.md_run_vv_f32(p.ref(), n, C.c_void_p(4096), C.c_void_p(vel), C.c_void_p(4096),
                               C.c_void_p(4096), C.c_void_p(inv_m), C.c_void_p(4096), float(dt),
                               int(steps), C.c_void_p(energies), C.c_void_p(256), ws_bytes, None)

    assert call(steps=-1) == -1
    assert call(dt=float("nan")) == -1
    assert call(dt=float("inf")) == -1
    assert call(vel=0) == -1
    assert call(inv_m=0) == -1
    assert call(inv_m=4098) == -1          # misaligned
    assert call(energies=4100) == -1       # an FP64 array needs 8-byte alignment
    assert call(ws_bytes=need - 1) == -3
    assert call(p=api.Params.from_dict(dict(base, r_switch=13.0))) == -1


def test_noalloc_rejects_before_any_device_call():
    """md_forces_f32_noalloc checks every argument, and the size of the system against its
    32 MiB per-device workspace, before it touches the device (these calls run without one)."""
    L = api.lib()
    base = W.small_system().params()
    p = api.Params.from_dict(base)
    f = L.md_forces_f32_noalloc
    ptr = C.c_void_p(4096)
    # n large enough that the workspace exceeds the array: MD_ERR_CAPACITY
    n_big = 400_000
    big = api.Params.from_dict(dict(base, box=(160.0, 160.0, 160.0)))
    assert api.workspace_bytes(big, n_big) > api.NOALLOC_MAX_WORKSPACE_BYTES
    assert f(big.ref(), n_big, ptr, ptr, ptr, ptr, ptr, None, None) == -6
    # ordinary argument errors as for md_forces_f32
    assert f(p.ref(), -1, ptr, ptr, ptr, ptr, ptr, None, None) == -1
    assert f(p.ref(), 10, ptr, ptr, ptr, None, ptr, None, None) == -1
    assert f(p.ref(), 10, ptr, ptr, ptr, ptr, C.c_void_p(4100), None, None) == -1   # energy alignment
    assert f(p.ref(), 10, ptr, ptr, ptr, ptr, ptr, C.c_void_p(4098), None) == -1    # status alignment
    bad = api.Params.from_dict(dict(base, box=(20.0, 30.0, 30.0)))
    assert f(bad.ref(), 10, ptr, ptr, ptr, ptr, ptr, None, None) == -2


def test_ewald_arguments():
    """Ewald: real-space flag needs a positive splitting parameter and the compacted kernel;
    the reciprocal call checks alpha, kmax and pointers before anything is enqueued."""
    base = W.small_system().params()
    need = api.workspace_bytes(base, 10)
    ew = dict(base, flags=api.COULOMB_EWALD, ewald_alpha=0.3)
    assert api.workspace_bytes(ew, 10) > 0
    assert api.workspace_bytes(dict(ew, ewald_alpha=0.0), 10) == 0
    assert api.workspace_bytes(dict(ew, flags=api.COULOMB_EWALD | api.PAIR_PREDICATED), 10) == 0
    assert api.workspace_bytes(dict(ew, flags=api.COULOMB_EWALD | api.COULOMB_TRUNCATED), 10) == 0
    assert _call_f32(dict(ew, flags=api.COULOMB_EWALD | api.PAIR_DRAIN(3)), ws_bytes=need) == -1
    assert api.ewald_workspace_bytes(ew, 100, (5, 6, 7)) > 0
    assert api.ewald_workspace_bytes(dict(ew, ewald_alpha=-1.0), 100, (5, 6, 7)) == 0
    assert api.ewald_workspace_bytes(ew, 100, (0, 0, 0)) == 0
    assert api.ewald_workspace_bytes(ew, 100, (256, 1, 1)) == 0
    L = api.lib()
    p = api.Params.from_dict(ew)
    km = (C.c_int32 * 3)(5, 5, 5)
    ptr = C.c_void_p(4096)
    nb = api.ewald_workspace_bytes(ew, 10, (5, 5, 5))
    assert L.md_ewald_recip_f32(p.ref(), 10, ptr, ptr, km, ptr, ptr, 0, C.c_void_p(256), nb - 1,
                                None) == -3
    assert L.md_ewald_recip_f32(p.ref(), 10, ptr, ptr, km, None, ptr, 0, C.c_void_p(256), nb,
                                None) == -1
    assert L.md_ewald_recip_f32(p.ref(), 10, ptr, ptr, km, ptr, C.c_void_p(4100), 0,
                                C.c_void_p(256), nb, None) == -1
