"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Sizes are small enough for the oracle's direct sums to finish in seconds but
span several column tiles and leave ragged tails (non-power-of-two n, tiles
of 8 or 16 half-spectrum bins).  Each test prints its measured maxima.
"""

import numpy as np
import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _run_fields(dt, dims, pts, tau_h, prec, grad=True, hess=False):
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    outs = ["S", "grad"] + (["hess"] if hess else [])
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=outs)
    assert plan.padded == tuple(parity.padded(n) for n in dims)
    Y = torch.from_numpy(pts).cuda()
    res = plan.forward(Y, S=True, grad=grad, hess=hess)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0,) * len(dims), tau, pts, prec, grad=grad, hess=hess)
    stats = plan.last_stats()
    return plan, res, ref, stats, tau, h


CASES_2D = [
    ((128, 128), 64, 2.0, "fp64", "c1"),      # the 2D float64 workload
    ((100, 77), 50, 1.5, "fp32", "ragged"),
    ((100, 77), 50, 1.5, "fp64", "ragged"),
    ((200, 130), 300, 3.0, "fp32", "ragged_big"),
]


@pytest.mark.parametrize("dims,K,tau_h,prec,name", CASES_2D)
def test_distance_gradient_2d(dt, dims, K, tau_h, prec, name):
    if name == "c1":
        w = synth.workload("c1_2d_128")
        pts = w.points
    else:
        pts = synth.generators.uniform_points(2, K, seed=101 + K)
    plan, res, ref, stats, tau, h = _run_fields(dt, dims, pts, tau_h, prec)
    S = _np(res["S"]).ravel()
    g = _np(res["grad"]).reshape(2, -1)
    assert stats["g_l2"] == pytest.approx(ref["g_l2"], rel=1e-12)
    assert stats["theta"] == pytest.approx(ref["theta"], rel=1e-9)
    dS = np.abs(S - ref["S_ref"])
    deep = ref["deep"]
    dG = np.abs(g - ref["grad"].T)[:, deep]
    print(f"\n[{name} {prec}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"max|dgrad| deep={dG.max():.3e} valid={ref['valid'].mean():.3f} S_max/tau={ref['s_max'] / tau:.2f}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert dG.max() <= parity.TOL_GRAD
    if prec == "fp64":
        assert np.all(dS[deep] <= parity.bound(ref, parity.TOL_S_TAU_FP64, tau)[deep])
        assert np.all(dG <= parity.bound(ref, parity.TOL_GRAD_FP64)[deep])
    # invalid nodes report S_max and zero gradient
    inval = ~ref["valid"] & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    if inval.any():
        np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-6)
        assert np.all(g[:, inval] == 0)


CASES_3D = [
    ((40, 36, 33), 30, 1.5, "fp32"),
    ((40, 36, 33), 30, 1.5, "fp64"),
    ((64, 64, 64), 200, 1.0, "fp32"),
]


@pytest.mark.parametrize("dims,K,tau_h,prec", CASES_3D)
def test_distance_gradient_3d(dt, dims, K, tau_h, prec):
    pts = synth.generators.uniform_points(3, K, seed=201 + K)
    plan, res, ref, stats, tau, h = _run_fields(dt, dims, pts, tau_h, prec)
    S = _np(res["S"]).ravel()
    g = _np(res["grad"]).reshape(3, -1)
    dS = np.abs(S - ref["S_ref"])
    deep = ref["deep"]
    dG = np.abs(g - ref["grad"].T)[:, deep]
    print(f"\n[3d {dims} {prec}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"max|dgrad| deep={dG.max():.3e} valid={ref['valid'].mean():.3f} S_max/tau={ref['s_max'] / tau:.2f}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert dG.max() <= parity.TOL_GRAD
    if prec == "fp64":
        assert np.all(dS[deep] <= parity.bound(ref, parity.TOL_S_TAU_FP64, tau)[deep])
        assert np.all(dG <= parity.bound(ref, parity.TOL_GRAD_FP64)[deep])


@pytest.mark.parametrize("dims,prec", [((90, 70), "fp32"), ((90, 70), "fp64"), ((34, 30, 28), "fp32"),
                                       ((34, 30, 28), "fp64")])
def test_hessian(dt, dims, prec):
    D = len(dims)
    pts = synth.generators.uniform_points(D, 40, seed=301 + D)
    plan, res, ref, stats, tau, h = _run_fields(dt, dims, pts, 2.0, prec, hess=True)
    H = _np(res["hess"]).reshape(3 if D == 2 else 6, -1)
    Href = parity.hess_components(ref["hess"], D)
    deep = ref["deep"]
    dH = np.abs(H - Href)[:, deep]
    scale = 1.0 / tau + 1.0 / min(h)
    print(f"\n[hess {dims} {prec}] max|dH|/(1/tau+1/h) deep={dH.max() / scale:.3e}")
    assert dH.max() <= parity.TOL_HESS * scale
    if prec == "fp64":
        assert np.all(dH <= parity.bound(ref, 1e-7, scale)[deep])


def test_source_outside_grid_sets_sticky_error(dt):
    dims = (64, 48)
    pts = synth.generators.uniform_points(2, 20, seed=7)
    bad = np.concatenate([pts, np.array([[1.5, 0.5], [np.nan, 0.2]], dtype=np.float32)])
    plan = dt.Plan(dims, None, None, 2.0 / 64, precision="fp64", outputs=["S"])
    S = plan.distance(torch.from_numpy(bad).cuda())
    torch.cuda.synchronize()
    assert plan.last_error() == 2       # DT_E_RANGE
    assert plan.last_error() == 0       # cleared
    ref = parity.reference(dims, (1 / 64, 1 / 48), (0.0, 0.0), 2.0 / 64, pts, "fp64")
    np.testing.assert_allclose(_np(S).ravel(), ref["S_ref"], atol=1e-9)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_source_closed_form_3d(dt, prec):
    """One source: phi = exp(-r/tau) exactly, so S = r and grad S = (X - Y)/r
    on every valid node, with no oracle involved.  Nodes lie at cell centres,
    (i + 1/2) h, and the source is placed exactly on one, so snapping is
    unambiguous and exact.  Positions are measured from the first node (only
    differences X - Y enter), in [z][y][x] order (x fastest)."""
    dims = (48, 40, 36)
    h = tuple(1.0 / n for n in dims)
    tau = 1.0 * h[0]
    node = (17, 22, 9)
    Y = np.array([[(node[a] + 0.5) * h[a] for a in range(3)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad"])
    res = plan.forward(torch.from_numpy(Y).cuda(), S=True, grad=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    st = plan.last_stats()
    S = _np(res["S"]).ravel()
    g = _np(res["grad"]).reshape(3, -1)
    zz, yy, xx = np.meshgrid(*[np.arange(dims[a]) * h[a] for a in (2, 1, 0)], indexing="ij")
    d = np.stack([xx.ravel() - node[0] * h[0], yy.ravel() - node[1] * h[1], zz.ravel() - node[2] * h[2]])
    r = np.sqrt((d ** 2).sum(axis=0))
    s_max, theta = st["s_max"], st["theta"]
    assert abs(s_max + tau * np.log(theta)) <= 1e-9 * s_max
    deep = r <= s_max - tau * np.log(2.0)          # phi >= 2 Theta
    far = r >= s_max + 0.05 * tau                  # phi clearly below Theta
    assert deep.sum() > 1000 and far.sum() > 1000
    dS = np.abs(S - r)
    with np.errstate(invalid="ignore", divide="ignore"):
        gx = np.where(r > 0, d / r, 0.0)
    dG = np.abs(g - gx)[:, deep]
    print(f"\n[single source {prec}] S_max/tau={s_max / tau:.2f} max|S-r|/tau deep={dS[deep].max() / tau:.3e} "
          f"max|grad-(X-Y)/r| deep={dG.max():.3e}")
    if prec == "fp32":
        assert dS[deep].max() <= parity.TOL_S_TAU * tau
        assert dG.max() <= parity.TOL_GRAD
    else:
        # float64: a flat part plus the relative noise floor Theta/phi = Theta e^(r/tau)
        ratio = theta * np.exp(r[deep] / tau)
        assert np.all(dS[deep] <= tau * (parity.TOL_S_TAU_FP64 + parity.TOL_THETA_FRAC * ratio))
        assert np.all(dG <= parity.TOL_GRAD_FP64 + parity.TOL_THETA_FRAC * ratio)
    # beyond the band the library writes S_max cast to the plan's type
    smax_t = float(np.float32(s_max)) if prec == "fp32" else s_max
    assert np.all(S[far] == smax_t)
    assert np.all(g[:, far] == 0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_source_hessian_closed_form_3d(dt, prec):
    """One source: S = r, so the Hessian is (I - n n^T)/r with n = (X - Y)/r,
    checked without the oracle on deep nodes at least 2h from the source.
    Components in the order xx, xy, xz, yy, yz, zz."""
    dims = (40, 36, 34)
    h = tuple(1.0 / n for n in dims)
    tau = 2.0 * h[0]
    node = (20, 17, 15)
    Y = np.array([[(node[a] + 0.5) * h[a] for a in range(3)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "hess"])
    res = plan.forward(torch.from_numpy(Y).cuda(), S=True, hess=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    s_max = plan.last_stats()["s_max"]
    H = _np(res["hess"]).reshape(6, -1)
    zz, yy, xx = np.meshgrid(*[np.arange(dims[a]) * h[a] for a in (2, 1, 0)], indexing="ij")
    d = np.stack([xx.ravel() - node[0] * h[0], yy.ravel() - node[1] * h[1], zz.ravel() - node[2] * h[2]])
    r = np.sqrt((d ** 2).sum(axis=0))
    sel = (r <= s_max - tau * np.log(2.0)) & (r >= 2.0 * max(h))
    assert sel.sum() > 1000
    n = d[:, sel] / r[sel]
    inv_r = 1.0 / r[sel]
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Href = np.stack([((1.0 if i == j else 0.0) - n[i] * n[j]) * inv_r for i, j in pairs])
    dH = np.abs(H[:, sel] - Href)
    scale = 1.0 / tau + 1.0 / min(h)
    print(f"\n[single-source hessian {prec}] max|dH|/(1/tau+1/h)={dH.max() / scale:.3e} nodes={int(sel.sum())}")
    if prec == "fp32":
        # about 25 times the error measured on an MI355X (3.8e-5)
        assert dH.max() <= 1e-3 * scale
    else:
        # flat part plus the relative noise floor Theta/phi = exp((r - S_max)/tau)
        ratio = np.exp((r[sel] - s_max) / tau)
        assert np.all(dH <= scale * (1e-7 + parity.TOL_THETA_FRAC * ratio))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_source_closed_form_2d(dt, prec):
    """The 2D kernels on one source: S = r, grad S = (X - Y)/r and
    H = (I - n n^T)/r (components xx, xy, yy), without the oracle; S_max
    and a zero gradient and Hessian beyond the band."""
    dims = (130, 100)
    h = tuple(1.0 / n for n in dims)
    tau = 1.5 * h[0]
    node = (47, 61)
    Y = np.array([[(node[a] + 0.5) * h[a] for a in range(2)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "hess"])
    res = plan.forward(torch.from_numpy(Y).cuda(), S=True, grad=True, hess=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    s_max = plan.last_stats()["s_max"]
    S = _np(res["S"]).ravel()
    g = _np(res["grad"]).reshape(2, -1)
    H = _np(res["hess"]).reshape(3, -1)
    yy, xx = np.meshgrid(np.arange(dims[1]) * h[1], np.arange(dims[0]) * h[0], indexing="ij")
    d = np.stack([xx.ravel() - node[0] * h[0], yy.ravel() - node[1] * h[1]])
    r = np.sqrt((d ** 2).sum(axis=0))
    deep = r <= s_max - tau * np.log(2.0)
    far = r >= s_max + 0.05 * tau
    assert deep.sum() > 300 and far.sum() > 300
    ratio = np.exp((r - s_max) / tau)              # Theta/phi for one source
    with np.errstate(invalid="ignore", divide="ignore"):
        n = np.where(r > 0, d / r, 0.0)
    sel = deep & (r >= 2.0 * max(h))
    ns, rs = n[:, sel], r[sel]
    Href = np.stack([(1.0 - ns[0] * ns[0]) / rs, -ns[0] * ns[1] / rs, (1.0 - ns[1] * ns[1]) / rs])
    dS = np.abs(S - r)[deep]
    dG = np.abs(g - n)[:, deep]
    dH = np.abs(H[:, sel] - Href)
    scale = 1.0 / tau + 1.0 / min(h)
    print(f"\n[single source 2d {prec}] S_max/tau={s_max / tau:.2f} max|S-r|/tau={dS.max() / tau:.3e} "
          f"max|dgrad|={dG.max():.3e} max|dH|/(1/tau+1/h)={dH.max() / scale:.3e}")
    if prec == "fp32":
        assert dS.max() <= parity.TOL_S_TAU * tau
        assert dG.max() <= parity.TOL_GRAD
        assert dH.max() <= parity.TOL_HESS * scale
    else:
        b = parity.TOL_THETA_FRAC * ratio
        assert np.all(dS <= tau * (parity.TOL_S_TAU_FP64 + b[deep]))
        assert np.all(dG <= parity.TOL_GRAD_FP64 + b[deep])
        assert np.all(dH <= scale * (1e-7 + b[sel]))
    smax_t = float(np.float32(s_max)) if prec == "fp32" else s_max
    assert np.all(S[far] == smax_t)
    assert np.all(g[:, far] == 0) and np.all(H[:, far] == 0)
