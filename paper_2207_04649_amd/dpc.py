"""Python binding of libdpc.so (include/dpc.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Tensors are
torch device tensors (torch provides device memory and streams); every step of
the computation runs in the library's HIP kernels.  There is no fallback: if
the library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpc.so")

DPC_OK, DPC_EINVAL, DPC_ERANGE, DPC_EWORKSPACE, DPC_EDEVICE = 0, -1, -2, -3, -4
DPC_REUSE_GRID = 1
DPC_LABEL_WS_BYTES = 256
COORD_LIMIT = 131072
MAX_POINTS = 1 << 27

_lib = None


class DpcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dpc status {status}: {message}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "R", "cell_side", "cells_per_dim", "cells", "strip_cells", "strips", "max_tasks", "mode",
        "workspace_bytes", "window_radius", "stages", "grid_dims", "lanes", "open_radius")]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    """dpc_tuning: plan options of one problem (0 = default)."""
    _fields_ = [("subdiv", ctypes.c_int32), ("strip_cells", ctypes.c_int32), ("nstages", ctypes.c_int32),
                ("stage_radius", ctypes.c_int32 * 4), ("stage_group", ctypes.c_int32 * 4),
                ("ring_cap", ctypes.c_int32), ("grid_dims", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("open_radius", ctypes.c_int32)]

    @classmethod
    def make(cls, subdiv=0, strip_cells=0, stages=(), ring_cap=0, grid_dims=0, lanes=0, open_radius=0) -> "Tuning":
        t = cls()
        t.subdiv, t.strip_cells, t.ring_cap = int(subdiv), int(strip_cells), int(ring_cap)
        t.grid_dims, t.lanes, t.open_radius = int(grid_dims), int(lanes), int(open_radius)
        t.nstages = len(stages)
        for k, (radius, group) in enumerate(stages):
            t.stage_radius[k], t.stage_group[k] = int(radius), int(group)
        return t

    def as_dict(self) -> dict:
        return {"subdiv": self.subdiv, "strip_cells": self.strip_cells, "ring_cap": self.ring_cap,
                "grid_dims": self.grid_dims, "lanes": self.lanes, "open_radius": self.open_radius,
                "stages": [(self.stage_radius[k], self.stage_group[k]) for k in range(self.nstages)]}


class Job(ctypes.Structure):
    """dpc_job: one problem of a batch (device pointers)."""
    _fields_ = [("pts", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("d_cut", ctypes.c_double),
                ("rho_min", ctypes.c_int32), ("delta_min", ctypes.c_double), ("rho", ctypes.c_void_p),
                ("dep", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("ncenters", ctypes.c_void_p)]


def lib() -> ctypes.CDLL:
    """Load libdpc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2207_04649_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, U32, D, SZ = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                   ctypes.c_double, ctypes.c_size_t)
        sig = {
            "dpc_workspace_bytes": (SZ, [I64, I32, D]),
            "dpc_density": (I32, [P, I64, I32, D, P, P, SZ, P]),
            "dpc_dependent": (I32, [P, I64, I32, D, P, P, P, U32, P, SZ, P]),
            "dpc_label": (I32, [I64, P, P, P, I32, D, P, P, P, SZ, P]),
            "dpc_run": (I32, [P, I64, I32, D, I32, D, P, P, P, P, P, P, SZ, P]),
            "dpc_run_static": (I32, [P, I64, I32, D, I32, D, P, P, P, P, P, P, P]),
            "dpc_approx_workspace_bytes": (SZ, [I64, I32, D]),
            "dpc_sapprox_workspace_bytes": (SZ, [I64, I32, D, D]),
            "dpc_sapprox_run": (I32, [P, I64, I32, D, D, I32, D, P, P, P, P, P, P, P, SZ, P]),
            "dpc_decision_top": (I32, [I64, P, P, I32, I32, P, P, P, P, P, SZ, P]),
            "dpc_decision_histogram": (I32, [I64, P, P, P, I32, P, I32, P, P]),
            "dpc_decision_suggest": (I32, [P, P, D, P, P, P]),
            "dpc_approx_run": (I32, [P, I64, I32, D, I32, D, P, P, P, P, P, P, P, SZ, P]),
            "dpc_sync_status": (I32, [P, P]),
            "dpc_last_error": (ctypes.c_char_p, []),
            "dpc_version": (I32, []),
            "dpc_cutoff_square": (I64, [D]),
            "dpc_plan": (I32, [I64, I32, D, ctypes.POINTER(PlanInfo)]),
            "dpc_plan_tuned": (I32, [I64, I32, D, ctypes.POINTER(Tuning), ctypes.POINTER(PlanInfo)]),
            "dpc_batch_plan": (I32, [ctypes.POINTER(Job), I32, ctypes.POINTER(Tuning), ctypes.POINTER(P),
                                     ctypes.POINTER(SZ)]),
            "dpc_batch_bind": (I32, [P, P, SZ]),
            "dpc_batch_run": (I32, [P, P, P]),
            "dpc_batch_sync_status": (I32, [P, P, P, ctypes.POINTER(I32)]),
            "dpc_batch_job_plan": (I32, [P, I32, ctypes.POINTER(PlanInfo)]),
            "dpc_batch_free": (None, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != DPC_OK:
        raise DpcError(status, lib().dpc_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t: torch.Tensor, dtype: torch.dtype, shape: tuple, name: str) -> None:
    if t.dtype != dtype or tuple(t.shape) != shape or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {shape}")


def dpc_version() -> int:
    return int(lib().dpc_version())


def dpc_cutoff_square(d_cut: float) -> int:
    return int(lib().dpc_cutoff_square(float(d_cut)))


def dpc_plan(n: int, d: int, d_cut: float) -> dict:
    info = PlanInfo()
    _check(lib().dpc_plan(int(n), int(d), float(d_cut), ctypes.byref(info)))
    return info.as_dict()


def dpc_plan_tuned(n: int, d: int, d_cut: float, tuning: Tuning | None = None) -> dict:
    info = PlanInfo()
    _check(lib().dpc_plan_tuned(int(n), int(d), float(d_cut), ctypes.byref(tuning) if tuning else None,
                                ctypes.byref(info)))
    return info.as_dict()


def dpc_workspace_bytes(n: int, d: int, d_cut: float) -> int:
    return int(lib().dpc_workspace_bytes(int(n), int(d), float(d_cut)))


def workspace(n: int, d: int, d_cut: float, device="cuda") -> torch.Tensor:
    nbytes = dpc_workspace_bytes(n, d, d_cut)
    if nbytes == 0:
        raise DpcError(DPC_EINVAL, "no workspace for these sizes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _pts(pts: torch.Tensor) -> tuple[int, int]:
    if pts.dim() != 2:
        raise ValueError("pts must be [n, d]")
    n, d = int(pts.shape[0]), int(pts.shape[1])
    _need(pts, torch.int32, (n, d), "pts")
    return n, d


def dpc_density(pts: torch.Tensor, d_cut: float, rho: torch.Tensor | None = None,
                ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    n, d = _pts(pts)
    rho = torch.empty(n, dtype=torch.int32, device=pts.device) if rho is None else rho
    _need(rho, torch.int32, (n,), "rho")
    ws = workspace(n, d, d_cut, pts.device) if ws is None else ws
    _check(lib().dpc_density(_ptr(pts), n, d, float(d_cut), _ptr(rho), _ptr(ws), ws.numel(), _stream(stream)))
    return rho


def dpc_dependent(pts: torch.Tensor, d_cut: float, rho: torch.Tensor, dep: torch.Tensor | None = None,
                  delta: torch.Tensor | None = None, flags: int = 0, ws: torch.Tensor | None = None,
                  stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    n, d = _pts(pts)
    _need(rho, torch.int32, (n,), "rho")
    dep = torch.empty(n, dtype=torch.int32, device=pts.device) if dep is None else dep
    delta = torch.empty(n, dtype=torch.float64, device=pts.device) if delta is None else delta
    _need(dep, torch.int32, (n,), "dep")
    _need(delta, torch.float64, (n,), "delta")
    ws = workspace(n, d, d_cut, pts.device) if ws is None else ws
    _check(lib().dpc_dependent(_ptr(pts), n, d, float(d_cut), _ptr(rho), _ptr(dep), _ptr(delta), int(flags),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return dep, delta


def dpc_label(rho: torch.Tensor, dep: torch.Tensor, delta: torch.Tensor, rho_min: int, delta_min: float,
              label: torch.Tensor | None = None, ncenters: torch.Tensor | None = None,
              ws: torch.Tensor | None = None, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    n = int(rho.shape[0])
    _need(rho, torch.int32, (n,), "rho")
    _need(dep, torch.int32, (n,), "dep")
    _need(delta, torch.float64, (n,), "delta")
    label = torch.empty(n, dtype=torch.int32, device=rho.device) if label is None else label
    ncenters = torch.empty(1, dtype=torch.int64, device=rho.device) if ncenters is None else ncenters
    _need(label, torch.int32, (n,), "label")
    _need(ncenters, torch.int64, (1,), "ncenters")
    ws = torch.empty(DPC_LABEL_WS_BYTES, dtype=torch.uint8, device=rho.device) if ws is None else ws
    _check(lib().dpc_label(n, _ptr(rho), _ptr(dep), _ptr(delta), int(rho_min), float(delta_min), _ptr(label),
                           _ptr(ncenters), _ptr(ws), ws.numel(), _stream(stream)))
    return label, ncenters


def dpc_run(pts: torch.Tensor, d_cut: float, rho_min: int, delta_min: float, ws: torch.Tensor | None = None,
            out: dict | None = None, stream=None) -> dict:
    """rho, dep, delta, label and ncenters in one call (device tensors)."""
    n, d = _pts(pts)
    dev = pts.device
    out = out if out is not None else {}
    rho = out.setdefault("rho", torch.empty(n, dtype=torch.int32, device=dev))
    dep = out.setdefault("dep", torch.empty(n, dtype=torch.int32, device=dev))
    delta = out.setdefault("delta", torch.empty(n, dtype=torch.float64, device=dev))
    label = out.setdefault("label", torch.empty(n, dtype=torch.int32, device=dev))
    ncent = out.setdefault("ncenters", torch.empty(1, dtype=torch.int64, device=dev))
    ws = workspace(n, d, d_cut, dev) if ws is None else ws
    _check(lib().dpc_run(_ptr(pts), n, d, float(d_cut), int(rho_min), float(delta_min), _ptr(rho), _ptr(dep),
                         _ptr(delta), _ptr(label), _ptr(ncent), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def dpc_approx_workspace_bytes(n: int, d: int, d_cut: float) -> int:
    return int(lib().dpc_approx_workspace_bytes(int(n), int(d), float(d_cut)))


def dpc_approx_run(pts: torch.Tensor, d_cut: float, rho_min: int, delta_min: float,
                   ws: torch.Tensor | None = None, out: dict | None = None, stream=None) -> dict:
    """Approx-DPC: rho, dep, delta, label, ncenters and the approx flags (device tensors)."""
    n, d = _pts(pts)
    dev = pts.device
    out = out if out is not None else {}
    rho = out.setdefault("rho", torch.empty(n, dtype=torch.int32, device=dev))
    dep = out.setdefault("dep", torch.empty(n, dtype=torch.int32, device=dev))
    delta = out.setdefault("delta", torch.empty(n, dtype=torch.float64, device=dev))
    label = out.setdefault("label", torch.empty(n, dtype=torch.int32, device=dev))
    ncent = out.setdefault("ncenters", torch.empty(1, dtype=torch.int64, device=dev))
    approx = out.setdefault("approx", torch.empty(n, dtype=torch.uint8, device=dev))
    if ws is None:
        nb = dpc_approx_workspace_bytes(n, d, d_cut)
        if nb == 0:
            raise DpcError(DPC_EINVAL, "no plan for these sizes")
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib().dpc_approx_run(_ptr(pts), n, d, float(d_cut), int(rho_min), float(delta_min), _ptr(rho),
                                _ptr(dep), _ptr(delta), _ptr(label), _ptr(ncent), _ptr(approx), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return out


def dpc_sapprox_workspace_bytes(n: int, d: int, d_cut: float, eps: float) -> int:
    return int(lib().dpc_sapprox_workspace_bytes(int(n), int(d), float(d_cut), float(eps)))


def dpc_sapprox_run(pts: torch.Tensor, d_cut: float, eps: float, rho_min: int, delta_min: float,
                    ws: torch.Tensor | None = None, out: dict | None = None, stream=None) -> dict:
    """S-Approx-DPC: rho, dep, delta, label, ncenters and the picked flags (device tensors)."""
    n, d = _pts(pts)
    dev = pts.device
    out = out if out is not None else {}
    rho = out.setdefault("rho", torch.empty(n, dtype=torch.int32, device=dev))
    dep = out.setdefault("dep", torch.empty(n, dtype=torch.int32, device=dev))
    delta = out.setdefault("delta", torch.empty(n, dtype=torch.float64, device=dev))
    label = out.setdefault("label", torch.empty(n, dtype=torch.int32, device=dev))
    ncent = out.setdefault("ncenters", torch.empty(1, dtype=torch.int64, device=dev))
    picked = out.setdefault("picked", torch.empty(n, dtype=torch.uint8, device=dev))
    if ws is None:
        nb = dpc_sapprox_workspace_bytes(n, d, d_cut, eps)
        if nb == 0:
            raise DpcError(DPC_EINVAL, "no plan for these sizes")
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib().dpc_sapprox_run(_ptr(pts), n, d, float(d_cut), float(eps), int(rho_min), float(delta_min),
                                 _ptr(rho), _ptr(dep), _ptr(delta), _ptr(label), _ptr(ncent), _ptr(picked),
                                 _ptr(ws), ws.numel(), _stream(stream)))
    return out


DECISION_TOP_MAX = 4096
DECISION_WS_BYTES = 128 << 10


def dpc_decision_top(rho: torch.Tensor, delta: torch.Tensor, rho_min: int, k: int, ws: torch.Tensor | None = None,
                     stream=None) -> dict:
    """The top-k non-noise points by delta (device tensors: ids, deltas, rhos, count)."""
    n = int(rho.shape[0])
    _need(rho, torch.int32, (n,), "rho")
    _need(delta, torch.float64, (n,), "delta")
    dev = rho.device
    out = {"ids": torch.empty(k, dtype=torch.int32, device=dev), "deltas": torch.empty(k, dtype=torch.float64, device=dev),
           "rhos": torch.empty(k, dtype=torch.int32, device=dev), "count": torch.empty(1, dtype=torch.int64, device=dev)}
    ws = torch.empty(DECISION_WS_BYTES, dtype=torch.uint8, device=dev) if ws is None else ws
    _check(lib().dpc_decision_top(n, _ptr(rho), _ptr(delta), int(rho_min), int(k), _ptr(out["ids"]),
                                  _ptr(out["deltas"]), _ptr(out["rhos"]), _ptr(out["count"]), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return out


def dpc_decision_histogram(rho: torch.Tensor, delta: torch.Tensor, rho_edges: torch.Tensor,
                           delta_edges: torch.Tensor, stream=None) -> torch.Tensor:
    """[n_rho_bins, n_delta_bins] int64 counts of <rho, delta> (device tensors; float64 edges)."""
    n = int(rho.shape[0])
    _need(rho, torch.int32, (n,), "rho")
    _need(delta, torch.float64, (n,), "delta")
    nr, nd = int(rho_edges.numel()) - 1, int(delta_edges.numel()) - 1
    _need(rho_edges, torch.float64, (nr + 1,), "rho_edges")
    _need(delta_edges, torch.float64, (nd + 1,), "delta_edges")
    counts = torch.empty((max(nr, 0), max(nd, 0)), dtype=torch.int64, device=rho.device)
    _check(lib().dpc_decision_histogram(n, _ptr(rho), _ptr(delta), _ptr(rho_edges), nr, _ptr(delta_edges), nd,
                                        _ptr(counts), _stream(stream)))
    return counts


def dpc_decision_suggest(top: dict, d_cut: float, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    """Suggested delta_min (NaN if none) and its number of centers in the top list."""
    dev = top["deltas"].device
    dmin = torch.empty(1, dtype=torch.float64, device=dev)
    cent = torch.empty(1, dtype=torch.int64, device=dev)
    _check(lib().dpc_decision_suggest(_ptr(top["deltas"]), _ptr(top["count"]), float(d_cut), _ptr(dmin),
                                      _ptr(cent), _stream(stream)))
    return dmin, cent


STATIC_SCRATCH_BYTES = 64 << 20


def dpc_run_static(pts: torch.Tensor, d_cut: float, rho_min: int, delta_min: float, out: dict,
                   status: torch.Tensor | None = None, stream=None) -> dict:
    """dpc_run with the library's static scratch array (no workspace, no allocation).

    ``out`` must hold preallocated rho, dep, delta, label and ncenters tensors (as
    dpc_run fills them); ``status``, if given, is a 1-element int32 device tensor
    that receives the device status word.
    """
    n, d = _pts(pts)
    _need(out["rho"], torch.int32, (n,), "rho")
    _need(out["dep"], torch.int32, (n,), "dep")
    _need(out["delta"], torch.float64, (n,), "delta")
    _need(out["label"], torch.int32, (n,), "label")
    _need(out["ncenters"], torch.int64, (1,), "ncenters")
    if status is not None:
        _need(status, torch.int32, (1,), "status")
    _check(lib().dpc_run_static(_ptr(pts), n, d, float(d_cut), int(rho_min), float(delta_min), _ptr(out["rho"]),
                                _ptr(out["dep"]), _ptr(out["delta"]), _ptr(out["label"]), _ptr(out["ncenters"]),
                                _ptr(status), _stream(stream)))
    return out


def dpc_sync_status(ws: torch.Tensor, stream=None) -> None:
    """Synchronise and raise DpcError if the device flagged an error on this workspace."""
    _check(lib().dpc_sync_status(_ptr(ws), _stream(stream)))


# ---------------------------------------------------------------- batches

def dpc_batch_plan(jobs, tunings=None) -> tuple[ctypes.c_void_p, int]:
    """Plan a batch of Job structs; returns (handle, workspace bytes)."""
    arr = (Job * len(jobs))(*jobs)
    tarr = None if tunings is None else (Tuning * len(jobs))(*tunings)
    handle, nbytes = ctypes.c_void_p(), ctypes.c_size_t()
    _check(lib().dpc_batch_plan(arr, len(jobs), tarr, ctypes.byref(handle), ctypes.byref(nbytes)))
    return handle, int(nbytes.value)


def dpc_batch_bind(handle, ws: torch.Tensor) -> None:
    _check(lib().dpc_batch_bind(handle, _ptr(ws), ws.numel()))


def dpc_batch_run(handle, ws: torch.Tensor, stream=None) -> None:
    _check(lib().dpc_batch_run(handle, _ptr(ws), _stream(stream)))


def dpc_batch_sync_status(handle, ws: torch.Tensor, stream=None) -> int:
    """Synchronise; raise DpcError (naming the first bad job) if any job flagged an error."""
    bad = ctypes.c_int32(-1)
    st = lib().dpc_batch_sync_status(handle, _ptr(ws), _stream(stream), ctypes.byref(bad))
    if st != DPC_OK:
        raise DpcError(st, f"job {bad.value}: " + lib().dpc_last_error().decode())
    return bad.value


def dpc_batch_job_plan(handle, i: int) -> dict:
    info = PlanInfo()
    _check(lib().dpc_batch_job_plan(handle, int(i), ctypes.byref(info)))
    return info.as_dict()


def dpc_batch_free(handle) -> None:
    if handle:
        lib().dpc_batch_free(handle)


class Batch:
    """Many problems run with one launch per phase (dpc_batch_*).

    ``problems`` is a list of (pts, d_cut, rho_min, delta_min) with pts an int32
    [n, d] device tensor.  Outputs are allocated here, one dict per problem with
    rho, dep, delta, label and ncenters; ``run()`` refills them.
    """

    def __init__(self, problems, tunings=None, device="cuda"):
        self.out, jobs = [], []
        for pts, d_cut, rho_min, delta_min in problems:
            n, d = _pts(pts)
            o = {"rho": torch.empty(n, dtype=torch.int32, device=pts.device),
                 "dep": torch.empty(n, dtype=torch.int32, device=pts.device),
                 "delta": torch.empty(n, dtype=torch.float64, device=pts.device),
                 "label": torch.empty(n, dtype=torch.int32, device=pts.device),
                 "ncenters": torch.empty(1, dtype=torch.int64, device=pts.device)}
            self.out.append(o)
            jobs.append(Job(pts.data_ptr(), n, d, float(d_cut), int(rho_min), float(delta_min), o["rho"].data_ptr(),
                            o["dep"].data_ptr(), o["delta"].data_ptr(), o["label"].data_ptr(),
                            o["ncenters"].data_ptr()))
        self._inputs = [p[0] for p in problems]  # keep the points alive
        self.handle, nbytes = dpc_batch_plan(jobs, tunings)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        dpc_batch_bind(self.handle, self.ws)

    def run(self, stream=None) -> list[dict]:
        dpc_batch_run(self.handle, self.ws, stream)
        return self.out

    def sync_status(self, stream=None) -> int:
        return dpc_batch_sync_status(self.handle, self.ws, stream)

    def job_plan(self, i: int) -> dict:
        return dpc_batch_job_plan(self.handle, i)

    def close(self) -> None:
        dpc_batch_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                self.close()
        except Exception:
            pass
