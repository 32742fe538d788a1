"""GPU parity of the double-double (DT_FP64X2) pipeline against the oracle.

The oracle's S is the float64 log-sum-exp of the direct sum, exact to
float64 rounding at any distance, so it checks the extended band directly:
nodes whose phi lies between the float64 threshold and the double-double one
are wrong (S_max) in the float64 path and must be right here.
"""

import numpy as np
import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_S_TAU_DD = 1e-12   # flat part of the bound, in units of tau (float64 log of phi)


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


def _clustered(n_pts, frac, seed):
    """Points in the left `frac` of the unit square, so that the rest of the
    grid lies far from every source."""
    rng = np.random.default_rng(seed)
    p = rng.random((n_pts, 2))
    p[:, 0] *= frac
    return p.astype(np.float32)


def _run(dt, dims, pts, tau_h, cells=None, prec="fp64x2"):
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S"])
    assert plan.padded == tuple(parity.padded(n) for n in dims)
    S = plan.distance(torch.from_numpy(pts).cuda())
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, prec, cells=cells)
    S = S.detach().cpu().numpy().astype(np.float64).ravel()
    if cells is not None:
        S = S[cells]
    return plan, S, ref, tau, h


CASES = [
    ((100, 77), 5, 0.25, 1.0, "ragged"),
    ((128, 128), 1, 0.5, 0.7, "single"),
    ((333, 200), 40, 0.3, 2.0, "wide"),
]


@pytest.mark.parametrize("dims,K,frac,tau_h,name", CASES)
def test_dd_distance_vs_oracle(dt, dims, K, frac, tau_h, name):
    pts = _clustered(K, frac, seed=700 + K)
    plan, S, ref, tau, h = _run(dt, dims, pts, tau_h)
    assert plan.precision == "fp64x2"
    stats = plan.last_stats()
    assert stats["g_l2"] == pytest.approx(ref["g_l2"], rel=1e-12)
    assert stats["theta"] == pytest.approx(ref["theta"], rel=1e-9)
    dS = np.abs(S - ref["S_ref"])
    deep, valid = ref["deep"], ref["valid"]
    # nodes that only the extended precision resolves
    theta64 = oracle.theta("fp64", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond64 = deep & (ref["lnphi"] < np.log(theta64))
    print(f"\n[dd {name}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"S_max/tau={ref['s_max'] / tau:.2f} (fp64 {oracle.s_max(tau, theta64) / tau:.2f}) "
          f"valid={valid.mean():.3f} beyond fp64={beyond64.sum()}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_DD, tau)[deep])
    assert beyond64.sum() > 0
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    if inval.any():
        np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-12)


TOL_GRAD_DD = 1e-12


@pytest.mark.parametrize("dims,K,frac,tau_h", [((100, 77), 5, 0.25, 1.0), ((333, 200), 40, 0.3, 2.0)])
def test_dd_gradient_vs_oracle(dt, dims, K, frac, tau_h):
    """grad S = (u * g) / (f * g) (eq. SxSyconv) in double-double, on every
    node the extended precision resolves; S identical to the S-only plan's."""
    pts = _clustered(K, frac, seed=900 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad"])
    S, g = plan.gradient(Y)
    S_only = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S"]).distance(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(S, S_only)
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, "fp64x2", grad=True)
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(2, -1)
    deep, valid = ref["deep"], ref["valid"]
    dG = np.abs(g - ref["grad"].T)
    theta64 = oracle.theta("fp64", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond64 = deep & (ref["lnphi"] < np.log(theta64))
    print(f"\n[dd grad {dims}] max|dgrad| deep={dG[:, deep].max():.3e} beyond fp64={beyond64.sum()} "
          f"max|dS|/tau={np.abs(S - ref['S_ref']).max() / tau:.3e}")
    assert np.all(dG[:, deep] <= parity.bound(ref, TOL_GRAD_DD)[deep])
    assert dG[:, valid].max() <= parity.TOL_GRAD
    # |grad S| < 1 (Sec. 5.1); far out it tends to 1, so allow the parity bound
    assert beyond64.sum() > 0
    assert np.all(np.hypot(*g[:, beyond64]) <= 1.0 + 2 * parity.bound(ref, TOL_GRAD_DD)[beyond64])
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    assert np.all(g[:, inval] == 0)


def test_dd_single_source_is_exact_distance(dt):
    """With one source phi = exp(-r/tau), so S = r throughout the valid band."""
    dims = (128, 96)
    pts = np.array([[0.1, 0.5]], dtype=np.float32)
    plan, S, ref, tau, h = _run(dt, dims, pts, 0.5)
    X = ref["X"]
    r = np.sqrt(((X - ref["Yhat"][0]) ** 2).sum(axis=1))
    v = ref["deep"]
    assert v.sum() > 500
    assert np.all(np.abs(S[v] - r[v]) <= parity.bound(ref, TOL_S_TAU_DD, tau)[v] + 1e-14 * r[v])


def test_dd_beats_fp64_in_the_extended_band(dt):
    """The float64 path reports S_max where the double-double one resolves S."""
    dims = (160, 100)
    pts = _clustered(3, 0.2, seed=7)
    _, S_dd, ref, tau, _ = _run(dt, dims, pts, 0.5)
    _, S_64, ref64, _, _ = _run(dt, dims, pts, 0.5, prec="fp64")
    band = ref["deep"] & ~ref64["valid"] & (ref["S_exact"] > ref64["s_max"] + 0.05 * tau)
    assert band.sum() > 100
    np.testing.assert_allclose(S_64[band], ref64["s_max"], rtol=1e-6)
    assert np.all(np.abs(S_dd[band] - ref["S_exact"][band]) <= parity.bound(ref, TOL_S_TAU_DD, tau)[band])


def test_dd_full_size_sampled(dt):
    """1024^2 (the largest plan: 2048^2 padded) on sampled nodes."""
    dims = (1024, 1024)
    pts = synth.generators.uniform_points(2, 64, seed=811)
    rng = np.random.default_rng(812)
    cells = np.sort(rng.choice(dims[0] * dims[1], 4000, replace=False))
    _, S, ref, tau, _ = _run(dt, dims, pts, 1.0, cells=cells)
    dS = np.abs(S - ref["S_ref"])
    deep = ref["deep"]
    print(f"\n[dd 1024^2] max|dS|/tau sampled={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"valid={ref['valid'].mean():.3f}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_DD, tau)[deep])


def test_dd_source_outside_grid_sets_sticky_error(dt):
    dims = (100, 80)
    plan = dt.Plan(dims, (0.01, 0.0125), None, 0.01, precision="fp64x2", outputs=["S"])
    Y = torch.tensor([[0.5, 0.5], [1.5, 0.5], [float("nan"), 0.2]], dtype=torch.float32, device="cuda")
    plan.distance(Y)
    assert plan.last_error() == 2      # DT_E_RANGE
    assert plan.last_error() == 0      # cleared


def test_dd_rejects_what_it_does_not_build(dt):
    with pytest.raises(Exception):
        dt.Plan((64, 64), None, None, 0.02, precision="fp64x2", outputs=["S", "sign"])
    with pytest.raises(Exception):
        dt.Plan((32, 32, 32), None, None, 0.05, precision="fp64x2", outputs=["S", "sign"])
    with pytest.raises(Exception):
        dt.Plan((300, 32, 32), None, None, 0.05, precision="fp64x2", outputs=["S"])


# ---------------------------------------------------------------------------
# 3D double-double plans (S and grad S)
# ---------------------------------------------------------------------------

def _clustered3(n_pts, frac, seed):
    rng = np.random.default_rng(seed)
    p = rng.random((n_pts, 3))
    p[:, 0] *= frac
    return p.astype(np.float32)


# (40, 36, 150): 512-point z lines, four per block, eight spectrum bins per thread
@pytest.mark.parametrize("dims,K,tau_h", [((40, 36, 33), 5, 1.0), ((96, 40, 30), 12, 0.5), ((40, 36, 150), 6, 1.0)])
def test_dd3d_distance_and_gradient_vs_oracle(dt, dims, K, tau_h):
    """3D (rows, strided y lines, fused z lines, all in double-double): S and
    grad S on every node against the oracle, to the float64 per-node bound
    with the double-double unit; nodes beyond the float64 band are resolved;
    S of the S + grad S plan equals the S-only plan's."""
    pts = _clustered3(K, 0.25, seed=720 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad"])
    assert plan.precision == "fp64x2" and plan.padded == tuple(parity.padded(n) for n in dims)
    S, g = plan.gradient(Y)
    S_only = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S"]).distance(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(S, S_only)
    ref = parity.reference(dims, h, (0.0,) * 3, tau, pts, "fp64x2", grad=True)
    stats = plan.last_stats()
    assert stats["g_l2"] == pytest.approx(ref["g_l2"], rel=1e-12)
    assert stats["theta"] == pytest.approx(ref["theta"], rel=1e-9)
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(3, -1)
    dS = np.abs(S - ref["S_ref"])
    dG = np.abs(g - ref["grad"].T)
    deep, valid = ref["deep"], ref["valid"]
    theta64 = oracle.theta("fp64", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond64 = deep & (ref["lnphi"] < np.log(theta64))
    print(f"\n[dd3d {dims}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"max|dgrad| deep={dG[:, deep].max():.3e} S_max/tau={ref['s_max'] / tau:.2f} "
          f"(fp64 {oracle.s_max(tau, theta64) / tau:.2f}) valid={valid.mean():.3f} beyond fp64={beyond64.sum()}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_DD, tau)[deep])
    assert np.all(dG[:, deep] <= parity.bound(ref, TOL_GRAD_DD)[deep])
    assert dG[:, valid].max() <= parity.TOL_GRAD
    assert beyond64.sum() > 0
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    if tau_h < 1:
        assert inval.sum() > 1000, "the grid must reach past the double-double band"
    if inval.any():
        np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-12)
        assert np.all(g[:, inval] == 0)


def test_dd3d_single_source_is_exact_distance(dt):
    """One source in 3D: S = r and grad S = (X - Y)/r over the whole
    double-double band, without the oracle.  The source sits on a node."""
    dims = (48, 40, 36)
    h = (1.0 / 48,) * 3
    tau = 0.5 * h[0]
    node = (5, 20, 18)
    Yc = np.array([[(node[a] + 0.5) * h[a] for a in range(3)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad"])
    S, g = plan.gradient(torch.from_numpy(Yc).cuda())
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    s_max = plan.last_stats()["s_max"]
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(3, -1)
    zz, yy, xx = np.meshgrid(*[np.arange(dims[a]) for a in (2, 1, 0)], indexing="ij")
    d = np.stack([(xx.ravel() - node[0]) * h[0], (yy.ravel() - node[1]) * h[1], (zz.ravel() - node[2]) * h[2]])
    r = np.sqrt((d ** 2).sum(axis=0))
    inside = r < s_max - np.log(2.0) * tau   # phi >= 2 Theta
    assert inside.sum() > 20000 and s_max / tau > 55
    # the per-node bound of the parity tests with Theta / phi = exp((r - S_max) / tau)
    ratio = np.exp((r - s_max) / tau)
    assert np.all(np.abs(S[inside] - r[inside]) <= tau * (TOL_S_TAU_DD + parity.TOL_THETA_FRAC * ratio[inside]))
    away = inside & (r > 0)
    dG = np.abs(g[:, away] - d[:, away] / r[away])
    assert np.all(dG <= TOL_GRAD_DD + parity.TOL_THETA_FRAC * ratio[away])
    beyond = r > s_max + 2.0 * tau
    assert np.all(S[beyond] == s_max) and np.all(g[:, beyond] == 0)


@pytest.mark.parametrize("dims,K,tau_h", [((100, 77), 5, 1.0), ((40, 36, 33), 5, 1.0), ((96, 40, 30), 12, 0.5)])
def test_dd_hessian_vs_oracle(dt, dims, K, tau_h):
    """The Hessian of eqs. Sxx, Syy, Sxy (and its 3D form) in double-double:
    on every node the extended precision resolves, within the per-node
    bound with the double-double unit; S and grad S of the Hessian plan equal
    those of the S + grad S plan (the extra channels leave them untouched)."""
    D = len(dims)
    pts = _clustered(K, 0.25, seed=740 + K) if D == 2 else _clustered3(K, 0.25, seed=740 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad", "hess"])
    res = plan.forward(Y, S=True, grad=True, hess=True)
    S2, g2 = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad"]).gradient(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(res["S"], S2) and torch.equal(res["grad"], g2)
    ref = parity.reference(dims, h, (0.0,) * D, tau, pts, "fp64x2", grad=True, hess=True)
    H = res["hess"].cpu().numpy().reshape(3 if D == 2 else 6, -1)
    Href = parity.hess_components(ref["hess"], D)
    deep, valid = ref["deep"], ref["valid"]
    scale = 1.0 / tau + 1.0 / min(h)
    dH = np.abs(H - Href)
    theta64 = oracle.theta("fp64", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond64 = deep & (ref["lnphi"] < np.log(theta64))
    print(f"\n[dd hess {dims}] max|dH|/(1/tau+1/h) deep={dH[:, deep].max() / scale:.3e} "
          f"beyond fp64={beyond64.sum()} valid={valid.mean():.3f}")
    assert beyond64.sum() > 0
    assert np.all(dH[:, deep] <= parity.bound(ref, TOL_HESS_DD, scale)[deep])
    assert dH[:, valid].max() <= parity.TOL_HESS * scale
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    assert np.all(H[:, inval] == 0)


# The Hessian's two terms are each of order 1/tau and cancel to order 1/r far
# from the sources; in float64 output that costs a few units of 1e-16 times
# r/tau <= 70 on top of the double-double convolution
TOL_HESS_DD = 1e-12


@pytest.mark.parametrize("dims,K,tau_h", [((100, 77), 5, 1.0), ((40, 36, 33), 5, 1.0), ((96, 40, 30), 12, 0.5)])
def test_dd_backward_vs_oracle(dt, dims, K, tau_h):
    """The adjoint (dL/dY, dL/dtau) in double-double against the oracle's
    analytic sums, with G on every valid node off the threshold's shell,
    including nodes beyond the float64 band; per component within the bound
    of the float64 adjoint tests, taken at the double-double threshold."""
    D = len(dims)
    pts = _clustered(K, 0.25, seed=760 + K) if D == 2 else _clustered3(K, 0.25, seed=760 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "backward"])
    ref = parity.reference(dims, h, (0.0,) * D, tau, pts, "fp64x2", rmean=True)
    lnphi = ref["lnphi"]
    G = np.random.default_rng(761).standard_normal(lnphi.shape)
    G[np.abs(lnphi - np.log(ref["theta"])) < np.log(2.0)] = 0.0
    G[~ref["valid"]] = 0.0
    theta64 = oracle.theta("fp64", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond64 = (G != 0) & (lnphi < np.log(theta64))
    assert beyond64.sum() > 100
    Y = torch.from_numpy(pts).cuda()
    S = plan.distance(Y)
    dY, dtau = plan.backward(Y, S, torch.from_numpy(G).cuda().reshape(plan.shape))
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    dY = dY.cpu().numpy().astype(np.float64)
    dtau = float(dtau.cpu())
    dY_ref, dtau_ref = oracle.loss_gradients(ref["X"], ref["Yhat"], tau, G, ref["valid"], workers=parity.WORKERS)
    ratio = np.exp(np.log(ref["theta"]) - lnphi)
    aG = np.abs(G)
    C = np.stack([aG, aG * ratio], axis=1)
    sens = oracle.adjoint.source_weight_sums(ref["X"], ref["Yhat"], tau, C, workers=parity.WORKERS)
    tw = 1.0 + 2.0 * ref["rmean"] / tau
    w_l2 = float(np.sqrt(np.sum((G * np.exp(-lnphi)) ** 2)))
    noise = parity.adjoint_noise("fp64x2", ref["padded"], ref["kernel_l1"], w_l2)
    bY, bt = parity.fp64_adjoint_bounds(sens[:, 0], sens[:, 1], float(aG @ tw), float((aG * ratio) @ tw), noise,
                                        dY_ref)
    rY = float((np.abs(dY - dY_ref) / bY).max())
    rt = abs(dtau - dtau_ref) / bt
    e_y = float(np.linalg.norm(dY - dY_ref) / np.linalg.norm(dY_ref))
    print(f"\n[dd backward {dims}] rel L2 dL/dY={e_y:.3e} rel dL/dtau={abs(dtau - dtau_ref) / abs(dtau_ref):.3e} "
          f"G beyond fp64={beyond64.sum()} max|ddY|/bound={rY:.3f} |ddtau|/bound={rt:.3f}")
    assert rY <= 1.0
    assert rt <= 1.0
