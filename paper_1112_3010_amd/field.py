"""Python binding of libdt: plans, forward fields, sign, adjoint, autograd.

PyTorch only provides device memory and streams here; every step of the
computation runs in the HIP kernels of libdt.so.
"""

from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib as L

PRECISIONS = {"fp32": L.DT_FP32_SCALED, "fp32_scaled": L.DT_FP32_SCALED, "fp64": L.DT_FP64, "auto": L.DT_AUTO,
              "fp64x2": L.DT_FP64X2, "fp64x4": L.DT_FP64X4}
OUTPUT_BITS = {"S": L.DT_OUT_S, "grad": L.DT_OUT_GRAD, "hess": L.DT_OUT_HESS, "sign": L.DT_OUT_SIGN,
               "backward": L.DT_OUT_BACKWARD, "curv": L.DT_OUT_CURV}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A prepared grid: padded sizes, kernel spectra, workspace.

    dims, spacing, origin are given x first.  ``outputs`` is an iterable of
    "S", "grad", "hess", "sign", "backward", "curv" (kernel families to
    prepare; "curv" prepares the gradient and Hessian kernels).  k_max (None
    or 0: full padding): the most sources a call will bring; a smaller
    padded grid with truncated kernels, which changes results only below the
    validity threshold (calls with more sources are refused).  precision:
    "fp32" (float32 with exact power-of-two scaling), "fp64", "fp64x2"
    (double-double), "fp64x4" (quad-double) or "auto" (the narrowest of
    these whose band reaches trunc_dist for k_hint sources); the extended
    formats return float64 fields.
    """

    def __init__(self, dims, spacing=None, origin=None, tau=None, precision="fp32", outputs=("S", "grad"),
                 trunc_dist=0.0, k_hint=0, c_theta=0.0, device="cuda", static_workspace=False, k_max=None):
        lib = L.load()
        self.ndim = len(dims)
        if spacing is None:
            spacing = [1.0 / n for n in dims]
        if origin is None:
            origin = [0.0] * self.ndim
        if tau is None:
            raise ValueError("tau is required")
        mask = 0
        for o in outputs:
            mask |= OUTPUT_BITS[o]
        self.dims = tuple(int(n) for n in dims)
        self.spacing = tuple(float(h) for h in spacing)
        self.origin = tuple(float(o) for o in origin)
        self.tau = float(tau)
        self._h = ctypes.c_void_p()
        d = (ctypes.c_int64 * self.ndim)(*self.dims)
        s = (ctypes.c_double * self.ndim)(*self.spacing)
        o = (ctypes.c_double * self.ndim)(*self.origin)
        if k_max:
            L.check(lib.dt_create_plan_reduced(ctypes.byref(self._h), self.ndim, d, s, o, self.tau,
                                               PRECISIONS[precision], mask, int(k_max), float(c_theta)),
                    "dt_create_plan_reduced")
        else:
            L.check(lib.dt_create_plan(ctypes.byref(self._h), self.ndim, d, s, o, self.tau, PRECISIONS[precision],
                                       mask, float(trunc_dist), int(k_hint), float(c_theta)), "dt_create_plan")
        self.device = torch.device(device)
        if static_workspace:
            # the library's fixed per-device array (no allocation; see dt.h)
            self.workspace = None
            with torch.cuda.device(self.device):
                L.check(lib.dt_plan_set_static_workspace(self._h, _stream(self.device)),
                        "dt_plan_set_static_workspace")
        else:
            nbytes = ctypes.c_size_t()
            L.check(lib.dt_plan_workspace_size(self._h, ctypes.byref(nbytes)), "dt_plan_workspace_size")
            self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            L.check(lib.dt_plan_set_workspace(self._h, ctypes.c_void_p(base + off), int(nbytes.value),
                                              _stream(self.device)), "dt_plan_set_workspace")
        self.info = self._info()
        self.dtype = torch.float64 if self.info.precision in (L.DT_FP64, L.DT_FP64X2, L.DT_FP64X4) else torch.float32

    def rebuild(self):
        """Attach the same workspace again: the kernel spectra are sampled and
        transformed anew (the plan-time cost that a new tau pays)."""
        if self.workspace is None:
            with torch.cuda.device(self.device):
                L.check(L.load().dt_plan_set_static_workspace(self._h, _stream(self.device)),
                        "dt_plan_set_static_workspace")
            return
        nbytes = ctypes.c_size_t()
        L.check(L.load().dt_plan_workspace_size(self._h, ctypes.byref(nbytes)), "dt_plan_workspace_size")
        base = self.workspace.data_ptr()
        L.check(L.load().dt_plan_set_workspace(self._h, ctypes.c_void_p(base + (-base) % 256), int(nbytes.value),
                                               _stream(self.device)), "dt_plan_set_workspace")

    def _info(self):
        info = L.DtPlanInfo()
        L.check(L.load().dt_plan_info(self._h, ctypes.byref(info)), "dt_plan_info")
        return info

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().dt_destroy_plan(h)
            except Exception:
                pass
            self._h = None

    # -- helpers -----------------------------------------------------------
    @property
    def shape(self):
        return tuple(reversed(self.dims))      # torch order [z][y][x]

    @property
    def padded(self):
        return tuple(int(self.info.padded[a]) for a in range(self.ndim))

    @property
    def cut(self):
        """Kernel truncation box in cells per axis (0: untruncated)."""
        return tuple(int(self.info.cut[a]) for a in range(self.ndim))

    @property
    def precision(self):
        return {L.DT_FP64: "fp64", L.DT_FP64X2: "fp64x2", L.DT_FP64X4: "fp64x4"}.get(self.info.precision, "fp32")

    def _points(self, Y):
        if Y is None:
            return None
        if not (Y.is_cuda and Y.dtype == torch.float32 and Y.dim() == 2 and Y.shape[1] == self.ndim):
            raise ValueError(f"Y must be a CUDA float32 tensor of shape (K, {self.ndim})")
        return Y.contiguous()

    def _shape(self, polygon=None, vertices=None, faces=None):
        if polygon is None and vertices is None:
            return None, ()
        sh = L.DtShape()
        keep = []
        if polygon is not None:
            polygon = polygon.contiguous()
            if not (polygon.is_cuda and polygon.dtype == torch.float32 and polygon.shape[1] == 2):
                raise ValueError("polygon must be a CUDA float32 (K, 2) tensor")
            sh.kind = L.DT_SHAPE_POLYGON
            sh.points = polygon.data_ptr()
            sh.n_points = polygon.shape[0]
            keep.append(polygon)
        else:
            vertices = vertices.contiguous()
            faces = faces.contiguous()
            if not (vertices.is_cuda and vertices.dtype == torch.float32 and faces.dtype == torch.int32):
                raise ValueError("mesh needs CUDA float32 vertices (nv, 3) and int32 faces (nf, 3)")
            sh.kind = L.DT_SHAPE_MESH
            sh.vertices = vertices.data_ptr()
            sh.n_vertices = vertices.shape[0]
            sh.faces = faces.data_ptr()
            sh.n_faces = faces.shape[0]
            keep.extend([vertices, faces])
        return sh, keep

    def _empty(self, *lead, dtype=None):
        return torch.empty(*lead, *self.shape, dtype=dtype or self.dtype, device=self.device)

    # -- entry points --------------------------------------------------------
    def forward(self, Y=None, *, polygon=None, vertices=None, faces=None, S=True, grad=False, hess=False,
                label=False, mu=False, signed=False, curv=False):
        """Run one pipeline for any subset of outputs; returns a dict.
        ``curv``: a (4, *grid) tensor of mean, Gaussian, k1, k2."""
        Yc = self._points(Y)
        sh, keep = self._shape(polygon, vertices, faces)
        out = {}
        if S:
            out["S"] = self._empty()
        if grad:
            out["grad"] = self._empty(self.ndim)
        if hess:
            out["hess"] = self._empty(3 if self.ndim == 2 else 6)
        if label:
            out["label"] = self._empty(dtype=torch.int8)
        if mu:
            out["mu"] = self._empty()
        if curv:
            out["curv"] = self._empty(4)
        o = L.DtOutputs()
        o.S = out["S"].data_ptr() if S else None
        o.grad = out["grad"].data_ptr() if grad else None
        o.hess = out["hess"].data_ptr() if hess else None
        o.label = out["label"].data_ptr() if label else None
        o.mu = out["mu"].data_ptr() if mu else None
        o.curv = out["curv"].data_ptr() if curv else None
        o.signed_outputs = 1 if signed else 0
        K = 0 if Yc is None else Yc.shape[0]
        L.check(L.load().dt_forward(self._h, _ptr(Yc), K, ctypes.byref(sh) if sh is not None else None,
                                    ctypes.byref(o), _stream(self.device)), "dt_forward")
        del keep
        return out

    def forward_into(self, out, Y=None, *, polygon=None, vertices=None, faces=None, signed=False):
        """Like forward() but writes into preallocated tensors in ``out``
        (keys among S, grad, hess, label, mu, curv)."""
        Yc = self._points(Y)
        sh, keep = self._shape(polygon, vertices, faces)
        o = L.DtOutputs()
        for key in ("S", "grad", "hess", "label", "mu", "curv"):
            t = out.get(key)
            setattr(o, key, None if t is None else t.data_ptr())
        o.signed_outputs = 1 if signed else 0
        K = 0 if Yc is None else Yc.shape[0]
        L.check(L.load().dt_forward(self._h, _ptr(Yc), K, ctypes.byref(sh) if sh is not None else None,
                                    ctypes.byref(o), _stream(self.device)), "dt_forward")
        del keep
        return out

    def distance_into(self, S, Y):
        """dt_distance into a preallocated tensor S (plan dtype, grid shape)."""
        Yc = self._points(Y)
        L.check(L.load().dt_distance(self._h, _ptr(Yc), Yc.shape[0], _ptr(S), _stream(self.device)), "dt_distance")
        return S

    def distance(self, Y):
        Yc = self._points(Y)
        S = self._empty()
        L.check(L.load().dt_distance(self._h, _ptr(Yc), Yc.shape[0], _ptr(S), _stream(self.device)), "dt_distance")
        return S

    def gradient(self, Y, with_S=True):
        Yc = self._points(Y)
        S = self._empty() if with_S else None
        g = self._empty(self.ndim)
        L.check(L.load().dt_gradient(self._h, _ptr(Yc), Yc.shape[0], _ptr(S), _ptr(g), _stream(self.device)),
                "dt_gradient")
        return (S, g) if with_S else g

    def hessian(self, Y):
        Yc = self._points(Y)
        H = self._empty(3 if self.ndim == 2 else 6)
        L.check(L.load().dt_hessian(self._h, _ptr(Yc), Yc.shape[0], _ptr(H), _stream(self.device)), "dt_hessian")
        return H

    def sign(self, *, polygon=None, vertices=None, faces=None, with_mu=False):
        sh, keep = self._shape(polygon, vertices, faces)
        if sh is None:
            raise ValueError("sign needs a polygon (2D) or a mesh (3D)")
        lab = self._empty(dtype=torch.int8)
        mu = self._empty() if with_mu else None
        L.check(L.load().dt_sign(self._h, ctypes.byref(sh), _ptr(lab), _ptr(mu), _stream(self.device)), "dt_sign")
        del keep
        return (lab, mu) if with_mu else lab

    def backward(self, Y, S, dL_dS, want_tau=True):
        Yc = self._points(Y)
        S = S.contiguous()
        G = dL_dS.contiguous().to(self.dtype)
        dY = torch.empty(Yc.shape[0], self.ndim, dtype=torch.float32, device=self.device)
        dtau = torch.empty((), dtype=torch.float64, device=self.device) if want_tau else None
        L.check(L.load().dt_backward(self._h, _ptr(Yc), Yc.shape[0], _ptr(S), _ptr(G), _ptr(dY), _ptr(dtau),
                                     _stream(self.device)), "dt_backward")
        return dY, dtau

    def backward_into(self, dY, dtau, Y, S, dL_dS):
        """dt_backward into preallocated dY (K x ndim float32) and dtau (a
        float64 scalar tensor, or None); S and dL_dS of the plan's dtype."""
        Yc = self._points(Y)
        L.check(L.load().dt_backward(self._h, _ptr(Yc), Yc.shape[0], _ptr(S), _ptr(dL_dS), _ptr(dY), _ptr(dtau),
                                     _stream(self.device)), "dt_backward")
        return dY, dtau

    def set_timing(self, enable=True):
        L.check(L.load().dt_plan_set_timing(self._h, 1 if enable else 0), "dt_plan_set_timing")

    def timings(self, reset=False):
        """{pass name: (launches, total ms)} since the last reset (synchronises)."""
        lib = L.load()
        arr = (L.DtPassTiming * 64)()
        n = ctypes.c_int()
        L.check(lib.dt_plan_timings(self._h, arr, 64, ctypes.byref(n)), "dt_plan_timings")
        out = {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, 64))}
        if reset:
            L.check(lib.dt_plan_reset_timings(self._h), "dt_plan_reset_timings")
        return out

    def last_error(self):
        return L.load().dt_last_error(self._h)

    def last_stats(self):
        st = L.DtCallStats()
        L.check(L.load().dt_last_stats(self._h, ctypes.byref(st)), "dt_last_stats")
        return {"g_l2": st.g_l2, "theta": st.theta, "s_max": st.s_max, "dL_dtau": st.dL_dtau,
                "error_bits": int(st.error_bits)}


class DistanceField(torch.autograd.Function):
    """S = distance field of the sources Y on ``plan``'s grid; the backward
    pass runs the library's adjoint and returns dL/dY and dL/dtau.  The plan's
    kernel spectra are built for one tau: the tau input must equal plan.tau
    (checked, ValueError otherwise; the check reads the value on the host and
    is skipped while a stream is being captured), and a step in tau needs a
    new plan."""

    @staticmethod
    def forward(ctx, Y, tau, plan):
        if not (tau.is_cuda and torch.cuda.is_current_stream_capturing()):
            t = float(tau)
            if abs(t - plan.tau) > 1e-12 * abs(plan.tau):
                raise ValueError(f"tau = {t!r} differs from the plan's tau = {plan.tau!r}: "
                                 "the kernel spectra are built for the plan's tau; create a plan for the new tau")
        S = plan.distance(Y)
        ctx.plan = plan
        ctx.save_for_backward(Y, S)
        return S

    @staticmethod
    def backward(ctx, grad_S):
        Y, S = ctx.saved_tensors
        dY, dtau = ctx.plan.backward(Y, S, grad_S, want_tau=ctx.needs_input_grad[1])
        dtau_out = None
        if ctx.needs_input_grad[1]:
            dtau_out = dtau.to(torch.float64)
        return dY, dtau_out, None


def distance_field(Y, plan, tau=None):
    """Differentiable S(Y) on ``plan``'s grid (tau: optional tensor that
    receives dL/dtau)."""
    if tau is None:
        tau = torch.tensor(plan.tau, dtype=torch.float64, device=Y.device)
    return DistanceField.apply(Y, tau, plan)
