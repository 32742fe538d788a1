"""GPU parity of the curvature outputs (mean, Gaussian, k1, k2) against the
oracle's curvatures of its own gradient and Hessian.

Compared on nodes where the field is well conditioned: phi >= 10 Theta
(the float32 error of phi there is a fifth of its error at the parity
band's edge), and in 3D |grad S| >= 0.5 (the level-set formulas divide by
|grad S|^3).  Tolerances (float32): 1e-3 (1/tau + 1/h) for the mean
curvature, its square for the Gaussian curvature, and for k1,2 the mean
tolerance plus the square root of the discriminant's tolerance
2 |mean| tol_mean + tol_gauss (the square root amplifies errors near
umbilic points, where the discriminant vanishes).  Float64: the same forms
on the float64 Hessian bound.
"""

import numpy as np
import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_CURV = 1e-3


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


def _check(res, ref, tau, h, prec, tag, D):
    C = res["curv"].detach().cpu().numpy().astype(np.float64).reshape(4, -1)
    c = oracle.curvature(ref["grad"], ref["hess"])
    ok = ref["lnphi"] >= np.log(10 * ref["theta"])
    if D == 3:
        ok &= np.einsum("ni,ni->n", ref["grad"], ref["grad"]) >= 0.25
    assert ok.sum() > 50
    scale = 1.0 / tau + 1.0 / min(h)
    if prec == "fp32":
        tm = np.full(ok.sum(), TOL_CURV * scale)
        tg = np.full(ok.sum(), TOL_CURV * scale ** 2)
    else:
        b = parity.bound(ref, 1e-7, 1.0)[ok]
        tm, tg = b * scale, b * scale ** 2
    tk = tm + np.sqrt(2 * np.abs(c["mean"][ok]) * tm + tg)
    errs = {}
    for i, (k, t) in enumerate((("mean", tm), ("gauss", tg), ("k1", tk), ("k2", tk))):
        d = np.abs(C[i][ok] - c[k][ok])
        errs[k] = float((d / t).max())
        assert np.all(d <= t), f"{tag} {k}: worst {d.max():.3e} vs tol {t[np.argmax(d)]:.3e}"
    print(f"\n[curv {tag}] worst error / tolerance: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    # clearly outside the valid band every curvature is 0
    inval = ref["lnphi"] < np.log(0.5 * ref["theta"])
    if inval.any():
        assert np.all(C[:, inval] == 0)


@pytest.mark.parametrize("dims,K,tau_h,prec", [((90, 70), 40, 2.0, "fp32"), ((90, 70), 40, 2.0, "fp64"),
                                               ((200, 130), 300, 3.0, "fp32"),
                                               ((34, 30, 28), 40, 2.0, "fp32"), ((34, 30, 28), 40, 2.0, "fp64"),
                                               ((90, 70), 5, 0.5, "fp64x2"), ((34, 30, 28), 6, 0.5, "fp64x2"),
                                               ((90, 70), 5, 0.35, "fp64x4"), ((34, 30, 28), 6, 0.3, "fp64x4")])
def test_curvature(dt, dims, K, tau_h, prec):
    D = len(dims)
    pts = synth.generators.uniform_points(D, K, seed=401 + D + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "curv"])
    Y = torch.from_numpy(pts).cuda()
    res = plan.forward(Y, S=True, curv=True)
    both = plan.forward(Y, S=False, grad=True, hess=True, curv=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    # the curvature outputs do not depend on which other outputs are written
    assert torch.equal(res["curv"], both["curv"])
    if prec in ("fp64x2", "fp64x4"):
        # the extended band reaches nodes that the next narrower format
        # (float64, double-double) reports as S_max
        lower = "fp64" if prec == "fp64x2" else "fp64x2"
        ref_low = oracle.theta(lower, tuple(parity.padded(n) for n in dims),
                               oracle.kernel_l1(tuple(parity.padded(n) for n in dims), h, tau),
                               float(plan.last_stats()["g_l2"]))
        assert plan.last_stats()["s_max"] > 1.8 * oracle.s_max(tau, ref_low)
    ref = parity.reference(dims, h, (0.0,) * D, tau, pts, prec, grad=True, hess=True)
    if prec in ("fp64x2", "fp64x4"):
        # checked nodes (phi >= 10 Theta) exist beyond the narrower band
        beyond = (ref["lnphi"] >= np.log(10 * ref["theta"])) & (ref["lnphi"] < np.log(ref_low))
        assert beyond.sum() > 100, beyond.sum()
    _check(res, ref, tau, h, prec, f"{dims} {prec}", D)


def test_curvature_needs_hessian_kernels(dt):
    """A plan without the curvature (or Hessian) kernels rejects a curvature request."""
    plan = dt.Plan((64, 48), None, None, 2.0 / 64, precision="fp32", outputs=["S", "grad"])
    Y = torch.from_numpy(synth.generators.uniform_points(2, 10, seed=3)).cuda()
    with pytest.raises(RuntimeError):
        plan.forward(Y, S=True, curv=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_source_sphere_curvatures(dt, prec):
    """One source in 3D: every level set of S = r is a sphere, so mean
    curvature and both principal curvatures are 1/r and the Gaussian one is
    1/r^2, checked without the oracle on nodes with phi >= 10 Theta and
    r >= 2h.  The k1, k2 bound widens as in the oracle comparison, since
    k = H +/- sqrt(H^2 - K) amplifies errors where H^2 = K."""
    dims = (38, 36, 32)
    h = tuple(1.0 / n for n in dims)
    tau = 2.0 * h[0]
    node = (19, 16, 14)
    Y = np.array([[(node[a] + 0.5) * h[a] for a in range(3)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "curv"])
    res = plan.forward(torch.from_numpy(Y).cuda(), S=True, curv=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    s_max = plan.last_stats()["s_max"]
    C = res["curv"].detach().cpu().numpy().astype(np.float64).reshape(4, -1)
    zz, yy, xx = np.meshgrid(*[np.arange(dims[a]) * h[a] for a in (2, 1, 0)], indexing="ij")
    r = np.sqrt((xx.ravel() - node[0] * h[0]) ** 2 + (yy.ravel() - node[1] * h[1]) ** 2
                + (zz.ravel() - node[2] * h[2]) ** 2)
    ok = (r <= s_max - tau * np.log(10.0)) & (r >= 2.0 * max(h))
    assert ok.sum() > 1000
    inv_r = 1.0 / r[ok]
    scale = 1.0 / tau + 1.0 / min(h)
    if prec == "fp32":
        tm = np.full(ok.sum(), TOL_CURV * scale)
        tg = np.full(ok.sum(), TOL_CURV * scale ** 2)
    else:
        b = 1e-7 + parity.TOL_THETA_FRAC * np.exp((r[ok] - s_max) / tau)   # Theta/phi for one source
        tm, tg = b * scale, b * scale ** 2
    tk = tm + np.sqrt(2 * inv_r * tm + tg)
    errs = {}
    for i, (k, ref, t) in enumerate((("mean", inv_r, tm), ("gauss", inv_r ** 2, tg), ("k1", inv_r, tk),
                                     ("k2", inv_r, tk))):
        d = np.abs(C[i][ok] - ref)
        errs[k] = float((d / t).max())
        assert np.all(d <= t), f"{prec} {k}: worst {d.max():.3e} vs tol {t[np.argmax(d)]:.3e}"
    print(f"\n[sphere curvatures {prec}] nodes={int(ok.sum())} worst error / tolerance: "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
