"""Helpers for the GPU tests: move a workload to the device, call the library
through its C ABI, and bring results back."""
import numpy as np

from paper_1611_04474_amd import api


def to_dev(sys_or_arrays, device, double=False):
    import torch
    pos, types, q = sys_or_arrays
    dt = torch.float64 if double else torch.float32
    p = torch.as_tensor(np.ascontiguousarray(pos).astype(np.float64 if double else np.float32))
    return (p.to(device=device, dtype=dt).contiguous(),
            torch.as_tensor(np.ascontiguousarray(types, dtype=np.int32)).to(device),
            torch.as_tensor(np.ascontiguousarray(q).astype(np.float64 if double else np.float32)).to(device))


def run(params, pos, types, q, device, double=False, flags=0, ws=None, extra=False):
    """Returns (forces float64 [n,3], energy, workspace tensor, pair counts or None)."""
    import torch
    d = to_dev((pos, types, q), device, double)
    p = api.Params.from_dict(params, flags)
    if ws is None:
        ws = api.alloc_workspace(p, d[0].shape[0], device, double)
    f, e = api.forces(p, *d, workspace=ws)
    torch.cuda.synchronize()
    counts = None
    if flags & api.DIAG_COUNTERS:
        lay = api.workspace_layout(p, d[0].shape[0], double)
        n = d[0].shape[0]
        counts = ws[lay["pair_count"]: lay["pair_count"] + 4 * n].view(torch.int32).cpu().numpy().copy()
    out = (f.double().cpu().numpy(), float(e.cpu().item()), ws, counts)
    if extra:
        return out + (f, e)
    return out
