"""Serving loop for force-evaluation requests: continuous batching on one GPU.

Requests (a periodic system each: positions, types, charges) arrive over time. The
loop keeps each admitted request's inputs, cell lists and outputs resident in device
memory until its result is back on the host, and:

  * admits arrived requests in arrival order while the bytes they need stay within
    an HBM budget (workspace from md_workspace_bytes plus inputs and outputs);
  * copies an admitted request's inputs to the device on a copy stream as soon as it
    is admitted, so copies overlap the batches already running;
  * launches every admitted, not yet launched request as one batched call
    (md_forces_batched: one launch per kernel of the path for up to 10 systems of one
    kind) whenever fewer than `max_inflight` batches are on the GPU, so requests that
    arrive while others run join the next batch instead of waiting for the queue to
    drain;
  * copies forces and energy back to pinned host memory behind each batch and retires
    the batch when its event completes, releasing its budget.

`replay_plain` serves the same trace one request at a time with the plain call, the
baseline. Both report per-request latency = host time at which the request's
completion was observed minus its arrival time.

The policy (admission, batching, retirement) is written against a small backend
interface so that it can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

IO_BYTES_PER_ATOM = 12 + 4 + 4 + 12     # float32 xyz, int32 type, float32 charge, float32 force


@dataclass
class Item:
    """One request: its host arrays and what it costs on the device."""
    rid: int
    n: int
    params: object                       # api.Params
    pos: object = None                   # pinned host tensors
    types: object = None
    charges: object = None
    force_out: object = None             # pinned host output
    energy_out: object = None
    pairs: int = 0                       # unique pairs within the cutoff (for throughput)
    bytes: int = 0                       # device bytes while resident


@dataclass
class Stats:
    latency_s: np.ndarray
    arrival_s: np.ndarray
    done_s: np.ndarray
    batches: list = field(default_factory=list)     # sizes of launched batches
    busy_s: float = 0.0                              # GPU time of the batches (events)
    peak_bytes: int = 0

    def summary(self, pairs):
        lat = self.latency_s * 1e3
        span = float(np.max(self.done_s) - np.min(self.arrival_s))
        return {
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(np.mean(lat)),
            "pairs_per_s": float(np.sum(pairs) / span) if span > 0 else None,
            "pairs_per_gpu_busy_s": float(np.sum(pairs) / self.busy_s) if self.busy_s > 0 else None,
            "span_s": span,
            "batches": len(self.batches),
            "mean_batch": float(np.mean(self.batches)) if self.batches else None,
            "max_batch": int(np.max(self.batches)) if self.batches else None,
            "peak_resident_MB": self.peak_bytes / 2 ** 20,
        }


def run_policy(items, arrivals, backend, budget_bytes, max_batch=32, max_inflight=2,
               clock=time.perf_counter):
    """Continuous batching over `items` arriving at `arrivals` (seconds from start).

    backend: admit(item) -> handle; launch(handles) -> batch; done(batch) -> bool;
             release(handle); busy(batch) -> seconds of GPU time (after done).
    Returns Stats."""
    n = len(items)
    order = sorted(range(n), key=lambda k: arrivals[k])
    for k in order:
        if items[k].bytes > budget_bytes:
            raise ValueError(f"request {items[k].rid} needs {items[k].bytes} bytes, "
                             f"more than the budget {budget_bytes}")
    waiting = collections.deque(order)
    ready = collections.deque()          # admitted, not launched: (k, handle)
    inflight = collections.deque()       # (batch, [(k, handle)])
    used = peak = 0
    done_s = np.full(n, np.nan)
    sizes = []
    busy = 0.0
    t0 = clock()
    remaining = n
    while remaining:
        now = clock() - t0
        # retire finished batches (one stream: they finish in launch order)
        while inflight and backend.done(inflight[0][0]):
            batch, members = inflight.popleft()
            t = clock() - t0
            busy += backend.busy(batch)
            for k, h in members:
                done_s[k] = t
                used -= items[k].bytes
                backend.release(h)
                remaining -= 1
        # admit arrived requests, in arrival order, within the budget
        while waiting and arrivals[waiting[0]] <= now and used + items[waiting[0]].bytes <= budget_bytes:
            k = waiting.popleft()
            ready.append((k, backend.admit(items[k])))
            used += items[k].bytes
            peak = max(peak, used)
        # launch what is admitted while the GPU has room for another batch
        if ready and len(inflight) < max_inflight:
            members = [ready.popleft() for _ in range(min(max_batch, len(ready)))]
            inflight.append((backend.launch([h for _, h in members]), members))
            sizes.append(len(members))
    arr = np.asarray(arrivals, dtype=np.float64)
    return Stats(latency_s=done_s - arr, arrival_s=arr, done_s=done_s, batches=sizes,
                 busy_s=busy, peak_bytes=peak)


_HIP = None


def copy_async(dst, src, stream):
    """Stream-ordered copy between a pinned host tensor and a device tensor of the same
    byte size, through hipMemcpyAsync itself. torch's non-blocking copy also records an
    event on the pinned host block for each copy; the serving buffers live for the whole
    run, so those events pile up, and now and then recording one held the host for 7-10 ms,
    which showed as the batched tail at high request rates."""
    global _HIP
    import ctypes as C
    if _HIP is None:
        lib = C.CDLL("libamdhip64.so")
        lib.hipMemcpyAsync.restype = C.c_int
        lib.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _HIP = lib
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_async: sizes differ")
    host = src if dst.is_cuda else dst
    if host.is_cuda or not host.is_pinned() or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy_async: needs one pinned host and one device tensor, contiguous")
    kind = 1 if dst.is_cuda else 2          # hipMemcpyHostToDevice, hipMemcpyDeviceToHost
    rc = _HIP.hipMemcpyAsync(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, kind,
                             C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed with code {rc}")


def _to_device(t, device, stream):
    import torch
    d = torch.empty(t.shape, dtype=t.dtype, device=device)
    copy_async(d, t, stream)
    return d


class GpuBackend:
    """Backend of run_policy on one HIP device: device tensors per admitted request,
    host-to-device copies on a copy stream, batched force calls and device-to-host
    copies on a compute stream, one event pair per batch."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.copy = torch.cuda.Stream(device)       # default priority
        self.compute = torch.cuda.Stream(device)

    def admit(self, it):
        from . import api
        torch = self.torch
        with torch.cuda.stream(self.copy):
            h = dict(item=it,
                     pos=_to_device(it.pos, self.device, self.copy),
                     types=_to_device(it.types, self.device, self.copy),
                     charges=_to_device(it.charges, self.device, self.copy),
                     force=torch.empty((it.n, 3), dtype=torch.float32, device=self.device),
                     energy=torch.empty(1, dtype=torch.float64, device=self.device),
                     workspace=api.alloc_workspace(it.params, it.n, self.device))
            h["copied"] = torch.cuda.Event()
            h["copied"].record(self.copy)
        return h

    def launch(self, handles):
        from . import api
        torch = self.torch
        for h in handles:
            self.compute.wait_event(h["copied"])
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(self.compute)
        api.forces_batched([dict(params=h["item"].params, pos=h["pos"], types=h["types"],
                                 charges=h["charges"], force=h["force"], energy=h["energy"],
                                 workspace=h["workspace"]) for h in handles],
                           stream=self.compute)
        for h in handles:
            copy_async(h["item"].force_out, h["force"], self.compute)
            copy_async(h["item"].energy_out, h["energy"], self.compute)
        end.record(self.compute)
        return (start, end)

    def done(self, batch):
        return batch[1].query()

    def busy(self, batch):
        return batch[0].elapsed_time(batch[1]) * 1e-3

    def release(self, h):
        h.clear()


def replay_plain(items, arrivals, device, clock=time.perf_counter):
    """Baseline: FIFO, one request at a time with the plain call (copy in, md_forces_f32,
    copy out, wait)."""
    import torch
    from . import api
    n = len(items)
    order = sorted(range(n), key=lambda k: arrivals[k])
    done_s = np.full(n, np.nan)
    stream = torch.cuda.Stream(device)
    busy = 0.0
    t0 = clock()
    for k in order:
        while clock() - t0 < arrivals[k]:
            pass
        it = items[k]
        with torch.cuda.stream(stream):
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            pos = _to_device(it.pos, device, stream)
            types = _to_device(it.types, device, stream)
            q = _to_device(it.charges, device, stream)
            f, e = api.forces(it.params, pos, types, q, stream=stream)
            copy_async(it.force_out, f, stream)
            copy_async(it.energy_out, e, stream)
            end.record(stream)
        end.synchronize()
        done_s[k] = clock() - t0
        busy += start.elapsed_time(end) * 1e-3
    arr = np.asarray(arrivals, dtype=np.float64)
    return Stats(latency_s=done_s - arr, arrival_s=arr, done_s=done_s, batches=[1] * n,
                 busy_s=busy)


def prepare(systems, device, pairs=None):
    """Items with pinned host inputs and outputs for a list of workloads.System."""
    import torch
    from . import api
    items = []
    for k, s in enumerate(systems):
        p = api.Params.from_dict(s.params())
        it = Item(rid=k, n=s.n, params=p,
                  pos=torch.from_numpy(np.ascontiguousarray(s.pos, dtype=np.float32)).pin_memory(),
                  types=torch.from_numpy(np.ascontiguousarray(s.types, dtype=np.int32)).pin_memory(),
                  charges=torch.from_numpy(np.ascontiguousarray(s.charges, dtype=np.float32)).pin_memory(),
                  force_out=torch.empty((s.n, 3), dtype=torch.float32).pin_memory(),
                  energy_out=torch.empty(1, dtype=torch.float64).pin_memory())
        it.bytes = api.workspace_bytes(p, s.n) + IO_BYTES_PER_ATOM * s.n + 8
        if pairs is not None:
            it.pairs = int(pairs[k])
        items.append(it)
    return items


def count_pairs(items, device):
    """Unique pairs within the cutoff of each item, from the kernels' diagnostic counters."""
    import torch
    from . import api
    out = []
    for it in items:
        p = it.params.with_flags(it.params.flags | api.DIAG_COUNTERS)
        pos, t, q = (x.to(device) for x in (it.pos, it.types, it.charges))
        ws = api.alloc_workspace(p, it.n, device)
        api.forces(p, pos, t, q, workspace=ws)
        out.append(api.read_diag(ws)[2])
        it.pairs = out[-1]
    torch.cuda.synchronize()
    return out
