"""Thin Python binding of the C ABI in include/mdforce.h.

Argument marshalling only: every step of the force path runs in the HIP library.
Tensors must already live on the GPU; the caller's current torch stream is used
unless a stream is given. The library must be built (``python -m
paper_1611_04474_amd.build``); a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmdforce.so")

MD_OK = 0
STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "box too small", -3: "workspace",
                -4: "HIP error", -5: "device status", -6: "capacity"}

ACCUM_F32_ATOMIC = 1 << 0
COULOMB_TRUNCATED = 1 << 1
DIAG_COUNTERS = 1 << 2
PAIR_PREDICATED = 1 << 3
PAIR_FULL_SHELL = 1 << 4
COULOMB_EWALD = 1 << 7
PAIR_DRAIN_MASK = 3 << 5


PAIR_SPLIT_MASK = 3 << 8


def PAIR_SPLIT(s):
    """Flag bits forcing s = 1, 2 or 4 workgroups per home cell (0: automatic)."""
    return {1: 1 << 8, 2: 2 << 8, 4: 3 << 8}[int(s)]


def PAIR_DRAIN(d):
    """Flag bits selecting d force batches per FIFO drain (d = 1..4; 2 is the default)."""
    return {2: 0, 1: 1 << 5, 3: 2 << 5, 4: 3 << 5}[int(d)]


STATUS_NAN = 1 << 0
STATUS_OUT_OF_BOX = 1 << 1
STATUS_BAD_TYPE = 1 << 2
STATUS_FIXED_OVERFLOW = 1 << 3

MAX_TYPES = 64


class MDError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {STATUS_NAMES.get(code, code)} ({code})")


class _Params(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("r_cut", C.c_double), ("r_switch", C.c_double),
                ("coulomb_k", C.c_double), ("n_types", C.c_int32),
                ("sigma", C.POINTER(C.c_double)), ("epsilon", C.POINTER(C.c_double)),
                ("flags", C.c_uint32), ("ewald_alpha", C.c_double)]


class _System(C.Structure):
    _fields_ = [("p", _Params), ("n_atoms", C.c_int64), ("d_pos", C.c_void_p),
                ("d_type", C.c_void_p), ("d_charge", C.c_void_p), ("d_force", C.c_void_p),
                ("d_energy", C.c_void_p), ("d_ws", C.c_void_p), ("ws_bytes", C.c_size_t)]


class _CopySegment(C.Structure):
    _fields_ = [("dst", C.c_void_p), ("src", C.c_void_p), ("bytes", C.c_size_t)]


class _Layout(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("n_cells", C.c_int64), ("cell_start", C.c_size_t),
                ("perm", C.c_size_t), ("pair_count", C.c_size_t), ("energy_partials", C.c_size_t),
                ("n_energy_partials", C.c_int64), ("z_split", C.c_size_t),
                ("total_bytes", C.c_size_t)]


_lib = None


def lib():
    """Loads libmdforce.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1611_04474_amd.build`")
        L = C.CDLL(LIB_PATH)
        pp = C.POINTER(_Params)
        vp = C.c_void_p
        L.md_workspace_bytes.argtypes = [pp, C.c_int64, C.c_int]
        L.md_workspace_bytes.restype = C.c_size_t
        L.md_workspace_layout.argtypes = [pp, C.c_int64, C.c_int, C.POINTER(_Layout)]
        L.md_workspace_layout.restype = C.c_int
        for name in ("md_forces_f32", "md_forces_f64"):
            f = getattr(L, name)
            f.argtypes = [pp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
            f.restype = C.c_int
        L.md_forces_f32_stages.argtypes = [pp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_size_t,
                                           C.c_uint32, vp]
        L.md_forces_f32_stages.restype = C.c_int
        L.md_forces_batched.argtypes = [C.POINTER(_System), C.c_int32, vp]
        L.md_forces_batched.restype = C.c_int
        L.md_forces_f32_noalloc.argtypes = [pp, C.c_int64, vp, vp, vp, vp, vp, vp, vp]
        L.md_forces_f32_noalloc.restype = C.c_int
        L.md_copy_segments.argtypes = [C.POINTER(_CopySegment), C.c_int32, vp]
        L.md_copy_segments.restype = C.c_int
        ip3 = C.POINTER(C.c_int32)
        L.md_ewald_workspace_bytes.argtypes = [pp, C.c_int64, ip3]
        L.md_ewald_workspace_bytes.restype = C.c_size_t
        L.md_ewald_recip_f32.argtypes = [pp, C.c_int64, vp, vp, ip3, vp, vp, C.c_int32, vp,
                                         C.c_size_t, vp]
        L.md_ewald_recip_f32.restype = C.c_int
        L.md_run_vv_f32.argtypes = [pp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_double, C.c_int32,
                                    vp, vp, C.c_size_t, vp]
        L.md_run_vv_f32.restype = C.c_int
        L.md_read_device_status.argtypes = [vp, vp, C.POINTER(C.c_uint32)]
        L.md_read_device_status.restype = C.c_int
        L.md_read_diag.argtypes = [vp, vp, C.POINTER(C.c_uint64)]
        L.md_read_diag.restype = C.c_int
        L.md_read_clock.argtypes = [vp, vp, C.POINTER(C.c_double)]
        L.md_read_clock.restype = C.c_int
        L.md_status_string.argtypes = [C.c_int]
        L.md_status_string.restype = C.c_char_p
        _lib = L
    return _lib


EXPORTED = ("md_workspace_bytes", "md_forces_f32", "md_forces_f32_stages", "md_forces_f64",
            "md_forces_batched", "md_forces_f32_noalloc", "md_copy_segments",
            "md_ewald_workspace_bytes", "md_ewald_recip_f32", "md_run_vv_f32",
            "md_read_device_status", "md_read_diag", "md_read_clock", "md_workspace_layout",
            "md_status_string")


class Params:
    """md_params plus the host arrays it points to."""

    def __init__(self, box, r_cut, r_switch, coulomb_k, sigma, epsilon, flags=0, ewald_alpha=0.0):
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.epsilon = np.ascontiguousarray(epsilon, dtype=np.float64)
        self.box = tuple(float(b) for b in box)
        self.r_cut, self.r_switch, self.coulomb_k = float(r_cut), float(r_switch), float(coulomb_k)
        self.flags = int(flags)
        self.ewald_alpha = float(ewald_alpha)
        self.c = _Params((C.c_double * 3)(*self.box), self.r_cut, self.r_switch, self.coulomb_k,
                         int(self.sigma.shape[0]),
                         self.sigma.ctypes.data_as(C.POINTER(C.c_double)),
                         self.epsilon.ctypes.data_as(C.POINTER(C.c_double)), self.flags,
                         self.ewald_alpha)

    @classmethod
    def from_dict(cls, d, flags=None):
        f = d.get("flags", 0) if flags is None else flags
        return cls(d["box"], d["r_cut"], d["r_switch"], d["coulomb_k"], d["sigma"], d["epsilon"], f,
                   d.get("ewald_alpha", 0.0))

    def with_flags(self, flags):
        return Params(self.box, self.r_cut, self.r_switch, self.coulomb_k, self.sigma,
                      self.epsilon, flags, self.ewald_alpha)

    def ref(self):
        return C.byref(self.c)


def _as_params(p, flags=None):
    if isinstance(p, Params):
        return p if flags is None else p.with_flags(flags)
    return Params.from_dict(p, flags)


def workspace_bytes(params, n_atoms, double_precision=False):
    p = _as_params(params)
    return int(lib().md_workspace_bytes(p.ref(), int(n_atoms), int(bool(double_precision))))


def workspace_layout(params, n_atoms, double_precision=False):
    p = _as_params(params)
    out = _Layout()
    rc = lib().md_workspace_layout(p.ref(), int(n_atoms), int(bool(double_precision)), C.byref(out))
    if rc != MD_OK:
        raise MDError(rc, "md_workspace_layout")
    return dict(dims=tuple(out.dims), n_cells=int(out.n_cells), cell_start=int(out.cell_start),
                perm=int(out.perm), pair_count=int(out.pair_count),
                energy_partials=int(out.energy_partials),
                n_energy_partials=int(out.n_energy_partials), z_split=int(out.z_split),
                total_bytes=int(out.total_bytes))


def _stream_ptr(stream):
    if isinstance(stream, int):
        return C.c_void_p(stream)
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def alloc_workspace(params, n_atoms, device, double_precision=False):
    import torch
    nb = workspace_bytes(params, n_atoms, double_precision)
    if nb == 0:
        raise MDError(-1, "md_workspace_bytes")
    return torch.empty(nb, dtype=torch.uint8, device=device)


class Workspace:
    """Reusable device workspace that grows on demand."""

    def __init__(self, device=None):
        self.buf = None
        self.device = device

    def get(self, params, n_atoms, device, double_precision=False):
        import torch
        need = workspace_bytes(params, n_atoms, double_precision)
        if need == 0:
            raise MDError(-1, "md_workspace_bytes")
        if self.buf is None or self.buf.numel() < need or self.buf.device != device:
            self.buf = torch.empty(need, dtype=torch.uint8, device=device)
        return self.buf


def _check_tensor(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def forces(params, pos, types, charges, *, flags=None, force=None, energy=None, workspace=None,
           stream=None, check=True):
    """One force evaluation. pos float32 [n,3] (float64 for the FP64 path), types int32 [n],
    charges same dtype as pos. Returns (force [n,3], energy [1] float64), both on the device.
    Raises MDError if the library rejects the arguments."""
    import torch
    p = _as_params(params, flags)
    dp = pos.dtype == torch.float64
    n = int(pos.shape[0])
    dt = torch.float64 if dp else torch.float32
    if check:
        _check_tensor(pos, dt, (n, 3), "pos")
        _check_tensor(types, torch.int32, (n,), "types")
        _check_tensor(charges, dt, (n,), "charges")
    if force is None:
        force = torch.empty((n, 3), dtype=dt, device=pos.device)
    if energy is None:
        energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    if workspace is None:
        workspace = alloc_workspace(p, n, pos.device, dp)
    elif isinstance(workspace, Workspace):
        workspace = workspace.get(p, n, pos.device, dp)
    fn = lib().md_forces_f64 if dp else lib().md_forces_f32
    rc = fn(p.ref(), n, C.c_void_p(pos.data_ptr()), C.c_void_p(types.data_ptr()),
            C.c_void_p(charges.data_ptr()), C.c_void_p(force.data_ptr()),
            C.c_void_p(energy.data_ptr()), C.c_void_p(workspace.data_ptr()),
            int(workspace.numel()), _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_forces_f64" if dp else "md_forces_f32")
    return force, energy


NOALLOC_MAX_WORKSPACE_BYTES = 32 << 20


def forces_noalloc(params, pos, types, charges, force, energy, status=None, stream=None):
    """md_forces_f32_noalloc: one float32 evaluation in the library's own per-device
    workspace, allocating nothing. pos, types, charges, force [n,3] float32, energy [1]
    float64 and the optional status (int32 [1]) are caller-allocated device tensors."""
    p = _as_params(params)
    n = int(pos.shape[0])
    rc = lib().md_forces_f32_noalloc(p.ref(), n, C.c_void_p(pos.data_ptr()),
                                     C.c_void_p(types.data_ptr()), C.c_void_p(charges.data_ptr()),
                                     C.c_void_p(force.data_ptr()), C.c_void_p(energy.data_ptr()),
                                     C.c_void_p(status.data_ptr() if status is not None else 0),
                                     _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_forces_f32_noalloc")


STAGE_BIN, STAGE_PAIR, STAGE_FINALIZE, STAGE_ALL = 1, 2, 4, 7


def forces_stages(params, pos, types, charges, force, energy, workspace, stages, stream=None):
    """Enqueues the given stages of one float32 evaluation (see md_forces_f32_stages)."""
    p = _as_params(params)
    rc = lib().md_forces_f32_stages(p.ref(), int(pos.shape[0]), C.c_void_p(pos.data_ptr()),
                                    C.c_void_p(types.data_ptr()), C.c_void_p(charges.data_ptr()),
                                    C.c_void_p(force.data_ptr()), C.c_void_p(energy.data_ptr()),
                                    C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                                    int(stages), _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_forces_f32_stages")


def forces_raw(params, n, pos_ptr, type_ptr, q_ptr, force_ptr, energy_ptr, ws_ptr, ws_bytes,
               stream_ptr, double_precision=False):
    """Direct call with integer device pointers; returns the md_status code."""
    p = _as_params(params)
    fn = lib().md_forces_f64 if double_precision else lib().md_forces_f32
    return fn(p.ref(), int(n), C.c_void_p(pos_ptr), C.c_void_p(type_ptr), C.c_void_p(q_ptr),
              C.c_void_p(force_ptr), C.c_void_p(energy_ptr), C.c_void_p(ws_ptr), int(ws_bytes),
              C.c_void_p(stream_ptr))


def forces_batched(systems, stream=None):
    """systems: list of dicts with keys params, pos, types, charges, force, energy, workspace
    (float32 path). Enqueues every system in one call."""
    arr = (_System * len(systems))()
    keep = []
    for k, s in enumerate(systems):
        p = _as_params(s["params"])
        keep.append(p)
        arr[k].p = p.c
        arr[k].n_atoms = int(s["pos"].shape[0])
        arr[k].d_pos = s["pos"].data_ptr()
        arr[k].d_type = s["types"].data_ptr()
        arr[k].d_charge = s["charges"].data_ptr()
        arr[k].d_force = s["force"].data_ptr()
        arr[k].d_energy = s["energy"].data_ptr()
        arr[k].d_ws = s["workspace"].data_ptr()
        arr[k].ws_bytes = int(s["workspace"].numel())
    rc = lib().md_forces_batched(arr, len(systems), _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_forces_batched")


def forces_batched_raw(systems, stream_ptr):
    """md_forces_batched on raw device addresses: systems is a list of tuples
    (params, n_atoms, pos, types, charges, force, energy, workspace, workspace_bytes)."""
    arr = (_System * len(systems))()
    keep = []
    for k, (prm, n, pos, typ, q, f, e, ws, wsb) in enumerate(systems):
        p = _as_params(prm)
        keep.append(p)
        arr[k].p = p.c
        arr[k].n_atoms = n
        arr[k].d_pos = pos
        arr[k].d_type = typ
        arr[k].d_charge = q
        arr[k].d_force = f
        arr[k].d_energy = e
        arr[k].d_ws = ws
        arr[k].ws_bytes = wsb
    rc = lib().md_forces_batched(arr, len(systems), C.c_void_p(stream_ptr))
    if rc != MD_OK:
        raise MDError(rc, "md_forces_batched")


def ewald_workspace_bytes(params, n_atoms, kmax):
    p = _as_params(params)
    km = (C.c_int32 * 3)(*[int(k) for k in kmax])
    return int(lib().md_ewald_workspace_bytes(p.ref(), int(n_atoms), km))


def ewald_recip(params, pos, charges, kmax, *, force=None, energy=None, accumulate=False,
                workspace=None, stream=None):
    """md_ewald_recip_f32: reciprocal-space forces (written, or added into `force` with
    accumulate=True) and the reciprocal + self + background energy, for float32 device
    tensors pos [n,3] and charges [n]. Returns (force, energy, workspace)."""
    import torch
    p = _as_params(params)
    n = int(pos.shape[0])
    _check_tensor(pos, torch.float32, (n, 3), "pos")
    _check_tensor(charges, torch.float32, (n,), "charges")
    if force is None:
        force = torch.zeros((n, 3), dtype=torch.float32, device=pos.device)
    if energy is None:
        energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    km = (C.c_int32 * 3)(*[int(k) for k in kmax])
    nb = lib().md_ewald_workspace_bytes(p.ref(), n, km)
    if nb == 0:
        raise MDError(-1, "md_ewald_workspace_bytes")
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=pos.device)
    rc = lib().md_ewald_recip_f32(p.ref(), n, C.c_void_p(pos.data_ptr()),
                                  C.c_void_p(charges.data_ptr()), km, C.c_void_p(force.data_ptr()),
                                  C.c_void_p(energy.data_ptr()), int(bool(accumulate)),
                                  C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                                  _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_ewald_recip_f32")
    return force, energy, workspace


def copy_segments(segments, stream_ptr):
    """md_copy_segments: (dst, src, nbytes) address triples between device memory and
    pinned host memory, copied by kernel on the stream."""
    arr = (_CopySegment * len(segments))()
    for k, (d, s_, nb) in enumerate(segments):
        arr[k].dst, arr[k].src, arr[k].bytes = d, s_, nb
    rc = lib().md_copy_segments(arr, len(segments), C.c_void_p(stream_ptr))
    if rc != MD_OK:
        raise MDError(rc, "md_copy_segments")


def run_vv(params, pos, vel, types, charges, inv_mass, force, dt, n_steps, *, energies=None,
           workspace=None, stream=None):
    """n_steps velocity-Verlet steps of dt fs (md_run_vv_f32). pos, vel, force float32 [n,3]
    on the device, updated in place; force must hold the forces at pos on entry. Returns
    the energies tensor [n_steps, 2] float64 (potential, kinetic) on the device."""
    import torch
    p = _as_params(params)
    n = int(pos.shape[0])
    _check_tensor(pos, torch.float32, (n, 3), "pos")
    _check_tensor(vel, torch.float32, (n, 3), "vel")
    _check_tensor(force, torch.float32, (n, 3), "force")
    _check_tensor(types, torch.int32, (n,), "types")
    _check_tensor(charges, torch.float32, (n,), "charges")
    _check_tensor(inv_mass, torch.float32, (n,), "inv_mass")
    if energies is None:
        energies = torch.empty((max(int(n_steps), 1), 2), dtype=torch.float64, device=pos.device)
    if workspace is None:
        workspace = alloc_workspace(p, n, pos.device)
    elif isinstance(workspace, Workspace):
        workspace = workspace.get(p, n, pos.device, False)
    rc = lib().md_run_vv_f32(p.ref(), n, C.c_void_p(pos.data_ptr()), C.c_void_p(vel.data_ptr()),
                             C.c_void_p(types.data_ptr()), C.c_void_p(charges.data_ptr()),
                             C.c_void_p(inv_mass.data_ptr()), C.c_void_p(force.data_ptr()),
                             float(dt), int(n_steps), C.c_void_p(energies.data_ptr()),
                             C.c_void_p(workspace.data_ptr()), int(workspace.numel()),
                             _stream_ptr(stream))
    if rc != MD_OK:
        raise MDError(rc, "md_run_vv_f32")
    return energies


def read_status(workspace, stream=None):
    v = C.c_uint32(0)
    rc = lib().md_read_device_status(C.c_void_p(workspace.data_ptr()), _stream_ptr(stream),
                                     C.byref(v))
    if rc != MD_OK:
        raise MDError(rc, "md_read_device_status")
    return int(v.value)


def read_diag(workspace, stream=None):
    v = (C.c_uint64 * 5)()
    rc = lib().md_read_diag(C.c_void_p(workspace.data_ptr()), _stream_ptr(stream), v)
    if rc != MD_OK:
        raise MDError(rc, "md_read_diag")
    return [int(x) for x in v]


def read_clock(workspace, stream=None):
    """Shader clock (GHz) of the last compacted pair kernel on this workspace, 0.0 if none."""
    v = C.c_double(0.0)
    rc = lib().md_read_clock(C.c_void_p(workspace.data_ptr()), _stream_ptr(stream), C.byref(v))
    if rc != MD_OK:
        raise MDError(rc, "md_read_clock")
    return float(v.value)


def status_string(code):
    return lib().md_status_string(int(code)).decode()
