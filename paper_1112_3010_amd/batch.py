"""Python binding of the batched 2D path of libdt (many instances per call).

Argument marshalling only: the passes run in libdt.so.  Outputs are packed
(instance i's [ny][nx] field at ``node_offset(i)``); :meth:`BatchPlan.views`
splits them into per-instance tensors without copying.
"""

from __future__ import annotations

import ctypes
import hashlib
import json
import os
from typing import Optional, Sequence

import torch

from . import _lib as L
from .field import PRECISIONS, OUTPUT_BITS, _stream


def _cache_path():
    return os.environ.get("DT_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                           "paper_1112_3010_amd", "batch_tiles.json")


class BatchPlan:
    """Plan for ``len(dims)`` independent 2D instances.

    dims: sequence of (nx, ny); spacing/origin: per-instance pairs (default
    1/n and 0); taus: per-instance tau (physical units).  k_max (an int or
    one per instance; None or 0 = full padding): the most sources a call
    will give an instance, which enables the reduced padding with truncated
    kernels (results change only below the validity threshold).
    """

    def __init__(self, dims: Sequence, taus: Sequence[float], spacing: Optional[Sequence] = None,
                 origin: Optional[Sequence] = None, precision="fp32", outputs=("S", "grad"), c_theta=0.0,
                 graph=True, device="cuda", k_max=None):
        lib = L.load()
        n = len(dims)
        if n < 1 or len(taus) != n:
            raise ValueError("need one tau per instance")
        desc = (L.DtInstanceDesc * n)()
        for i in range(n):
            nx, ny = (int(v) for v in dims[i])
            h = spacing[i] if spacing is not None else (1.0 / nx, 1.0 / ny)
            o = origin[i] if origin is not None else (0.0, 0.0)
            desc[i].dims[0], desc[i].dims[1] = nx, ny
            desc[i].spacing[0], desc[i].spacing[1] = float(h[0]), float(h[1])
            desc[i].origin[0], desc[i].origin[1] = float(o[0]), float(o[1])
            desc[i].tau = float(taus[i])
            if k_max is not None:
                desc[i].k_max = int(k_max[i] if isinstance(k_max, (list, tuple)) else k_max)
        mask = 0
        for o in outputs:
            mask |= OUTPUT_BITS[o]
        self.n = n
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.outputs = tuple(outputs)
        self._h = ctypes.c_void_p()
        L.check(lib.dt_create_batch_plan(ctypes.byref(self._h), n, desc, PRECISIONS[precision], mask,
                                         float(c_theta)), "dt_create_batch_plan")
        self.device = torch.device(device)
        nbytes = ctypes.c_size_t()
        L.check(lib.dt_batch_workspace_size(self._h, ctypes.byref(nbytes)), "dt_batch_workspace_size")
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        L.check(lib.dt_batch_set_workspace(self._h, ctypes.c_void_p(base + off), int(nbytes.value),
                                           _stream(self.device)), "dt_batch_set_workspace")
        self.info = []
        for i in range(n):
            inf = L.DtBatchInstanceInfo()
            L.check(lib.dt_batch_instance_info(self._h, i, ctypes.byref(inf)), "dt_batch_instance_info")
            self.info.append(inf)
        self.total_nodes = int(self.info[0].total_nodes)
        self.dtype = torch.float64 if self.info[0].precision == L.DT_FP64 else torch.float32
        self.precision = "fp64" if self.dtype == torch.float64 else "fp32"
        self.set_graph(graph)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().dt_destroy_batch_plan(h)
            except Exception:
                pass
            self._h = None

    # -- geometry ------------------------------------------------------------
    def padded(self, i):
        return int(self.info[i].padded[0]), int(self.info[i].padded[1])

    def node_offset(self, i):
        return int(self.info[i].node_offset)

    def kernel_l1(self, i):
        return float(self.info[i].kernel_l1)

    def views(self, S=None, grad=None):
        """Per-instance views [(S_i [ny][nx], grad_i [2][ny][nx]), ...]."""
        out = []
        for i, (nx, ny) in enumerate(self.dims):
            o = self.node_offset(i)
            s = S[o:o + nx * ny].view(ny, nx) if S is not None else None
            g = grad[2 * o:2 * o + 2 * nx * ny].view(2, ny, nx) if grad is not None else None
            out.append((s, g))
        return out

    # -- calls -----------------------------------------------------------------
    @staticmethod
    def pack(points: Sequence[torch.Tensor]):
        """Concatenate per-instance (K_i, 2) float32 tensors; returns (Y, offsets)."""
        offs = [0]
        for p in points:
            offs.append(offs[-1] + int(p.shape[0]))
        Y = torch.cat([p.reshape(-1, 2) for p in points], 0) if points else torch.empty(0, 2)
        return Y.to(torch.float32).contiguous(), offs

    def _args(self, Y, offsets):
        if not (Y.is_cuda and Y.dtype == torch.float32 and Y.dim() == 2 and Y.shape[1] == 2 and Y.is_contiguous()):
            raise ValueError("Y must be a contiguous CUDA float32 (K, 2) tensor")
        if len(offsets) != self.n + 1 or int(offsets[-1]) != Y.shape[0]:
            raise ValueError("offsets must have n_inst + 1 entries ending at K")
        return (ctypes.c_int64 * (self.n + 1))(*[int(v) for v in offsets])

    def empty_outputs(self):
        S = torch.empty(self.total_nodes, dtype=self.dtype, device=self.device) if "S" in self.outputs else None
        G = torch.empty(2 * self.total_nodes, dtype=self.dtype, device=self.device) if "grad" in self.outputs \
            else None
        return S, G

    def forward_into(self, Y, offsets, S=None, grad=None):
        koff = self._args(Y, offsets)
        L.check(L.load().dt_forward_batched(self._h, ctypes.c_void_p(Y.data_ptr()), koff,
                                            None if S is None else ctypes.c_void_p(S.data_ptr()),
                                            None if grad is None else ctypes.c_void_p(grad.data_ptr()),
                                            _stream(self.device)), "dt_forward_batched")

    def forward(self, Y, offsets):
        S, G = self.empty_outputs()
        self.forward_into(Y, offsets, S, G)
        return S, G

    def set_graph(self, enable=True):
        L.check(L.load().dt_batch_set_graph(self._h, 1 if enable else 0), "dt_batch_set_graph")

    def tiles(self):
        t = L.DtBatchTiles()
        L.check(L.load().dt_batch_get_tiles(self._h, ctypes.byref(t)), "dt_batch_get_tiles")
        return {"col_nb": t.col_nb, "col_threads": t.col_threads, "row_threads": t.row_threads}

    def set_tiles(self, col_nb, col_threads, row_threads):
        t = L.DtBatchTiles(int(col_nb), int(col_threads), int(row_threads))
        L.check(L.load().dt_batch_set_tiles(self._h, ctypes.byref(t)), "dt_batch_set_tiles")

    def schedule(self):
        """Radix schedule family per instance and pass: a list of n_inst
        triples (forward rows, columns, inverse rows), each in 0..5."""
        arr = (ctypes.c_int * (3 * self.n))()
        L.check(L.load().dt_batch_get_schedule(self._h, arr), "dt_batch_get_schedule")
        return [list(arr[3 * i:3 * i + 3]) for i in range(self.n)]

    def set_schedule(self, fams):
        flat = [int(v) for triple in fams for v in triple]
        if len(flat) != 3 * self.n:
            raise ValueError("one (rows, columns, inverse rows) triple per instance")
        arr = (ctypes.c_int * (3 * self.n))(*flat)
        L.check(L.load().dt_batch_set_schedule(self._h, arr), "dt_batch_set_schedule")

    def _tune_key(self):
        h = hashlib.sha256()
        h.update(json.dumps([self.dims, self.precision, sorted(self.outputs)]).encode())
        dev = torch.cuda.get_device_name(self.device) if torch.cuda.is_available() else "none"
        h.update(dev.encode())
        return h.hexdigest()

    def autotune(self, Y, offsets, reps=3, cache=True):
        """Pick the fastest tiles and radix schedules (measured on this batch)
        and remember them in a JSON cache keyed by the instance sizes,
        precision and device."""
        path = _cache_path()
        key = self._tune_key()
        table = {}
        if cache and os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
            if key in table:
                entry = dict(table[key])
                sched = entry.pop("schedule", None)
                self.set_tiles(**entry)
                if sched is not None:
                    self.set_schedule(sched)
                return dict(table[key])
        S, G = self.empty_outputs()
        koff = self._args(Y, offsets)
        best = L.DtBatchTiles()
        L.check(L.load().dt_batch_autotune(self._h, ctypes.c_void_p(Y.data_ptr()), koff,
                                           None if S is None else ctypes.c_void_p(S.data_ptr()),
                                           None if G is None else ctypes.c_void_p(G.data_ptr()), int(reps),
                                           _stream(self.device), ctypes.byref(best)), "dt_batch_autotune")
        res = {"col_nb": best.col_nb, "col_threads": best.col_threads, "row_threads": best.row_threads,
               "schedule": self.schedule()}
        if cache:
            table[key] = res
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                with open(path, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
            except OSError:
                pass
        return res

    def last_error(self):
        return L.load().dt_batch_last_error(self._h)

    def stats(self, i):
        s = L.DtCallStats()
        L.check(L.load().dt_batch_stats(self._h, int(i), ctypes.byref(s)), "dt_batch_stats")
        return {"g_l2": s.g_l2, "theta": s.theta, "s_max": s.s_max}
