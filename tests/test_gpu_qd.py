"""GPU parity of the quad-double (DT_FP64X4) pipeline against the oracle.

The same kernels as the double-double path, carried in four float64 parts
(unit roundoff taken as 2^-208).  The oracle's S is the float64 log-sum-exp
of the direct sum, exact to float64 rounding at any distance, so it checks
the doubled band directly: nodes whose phi lies between the double-double
threshold and the quad-double one are S_max in the double-double path and
must be right here.  The per-node bounds are those of the double-double
tests with the quad-double threshold.
"""

import numpy as np
import pytest

import oracle
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_S_TAU_XP = 1e-12   # flat part of the bound, in units of tau (float64 log of phi)
TOL_GRAD_XP = 1e-12
TOL_HESS_XP = 1e-12


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


def _clustered(n_pts, frac, seed, D=2):
    """Points in the first `frac` of the unit box along x, so that the rest of
    the grid lies far from every source."""
    rng = np.random.default_rng(seed)
    p = rng.random((n_pts, D))
    p[:, 0] *= frac
    return p.astype(np.float32)


def _beyond_dd(ref):
    theta_dd = oracle.theta("fp64x2", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    return ref["deep"] & (ref["lnphi"] < np.log(theta_dd))


CASES = [
    ((100, 77), 5, 0.25, 1.0, "ragged"),
    ((128, 128), 1, 0.5, 0.7, "single"),
    ((333, 200), 40, 0.3, 2.0, "wide"),
]


@pytest.mark.parametrize("dims,K,frac,tau_h,name", CASES)
def test_qd_distance_vs_oracle(dt, dims, K, frac, tau_h, name):
    pts = _clustered(K, frac, seed=800 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S"])
    assert plan.precision == "fp64x4" and plan.padded == tuple(parity.padded(n) for n in dims)
    S = plan.distance(torch.from_numpy(pts).cuda())
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, "fp64x4")
    stats = plan.last_stats()
    assert stats["g_l2"] == pytest.approx(ref["g_l2"], rel=1e-12)
    assert stats["theta"] == pytest.approx(ref["theta"], rel=1e-9)
    S = S.cpu().numpy().ravel()
    dS = np.abs(S - ref["S_ref"])
    deep, valid = ref["deep"], ref["valid"]
    beyond = _beyond_dd(ref)
    print(f"\n[qd {name}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
          f"S_max/tau={ref['s_max'] / tau:.2f} valid={valid.mean():.3f} beyond double-double={beyond.sum()}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_XP, tau)[deep])
    assert beyond.sum() > 0
    assert ref["s_max"] / tau > 120
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    if inval.any():
        np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-12)


def test_qd_single_source_is_exact_distance(dt):
    """One source: phi = exp(-r/tau), so S = r over the whole band (about
    130 tau), without the oracle."""
    dims = (128, 96)
    h = (1.0 / 128, 1.0 / 128)
    tau = 0.5 * h[0]
    node = (12, 48)
    Yc = np.array([[(node[a] + 0.5) * h[a] for a in range(2)]], dtype=np.float32)
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "grad"])
    S, g = plan.gradient(torch.from_numpy(Yc).cuda())
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    s_max = plan.last_stats()["s_max"]
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(2, -1)
    yy, xx = np.meshgrid(np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    d = np.stack([(xx.ravel() - node[0]) * h[0], (yy.ravel() - node[1]) * h[1]])
    r = np.sqrt((d ** 2).sum(axis=0))
    inside = r < s_max - np.log(2.0) * tau
    assert s_max / tau > 120 and inside.sum() > 5000
    ratio = np.exp((r - s_max) / tau)
    assert np.all(np.abs(S[inside] - r[inside]) <= tau * (TOL_S_TAU_XP + parity.TOL_THETA_FRAC * ratio[inside])
                  + 1e-14 * r[inside])
    away = inside & (r > 0)
    dG = np.abs(g[:, away] - d[:, away] / r[away])
    assert np.all(dG <= TOL_GRAD_XP + parity.TOL_THETA_FRAC * ratio[away])
    beyond = r > s_max + 2.0 * tau
    assert beyond.sum() > 0
    assert np.all(S[beyond] == s_max) and np.all(g[:, beyond] == 0)


@pytest.mark.parametrize("dims,K,frac,tau_h", [((100, 77), 5, 0.25, 1.0), ((333, 200), 40, 0.3, 2.0)])
def test_qd_gradient_vs_oracle(dt, dims, K, frac, tau_h):
    """grad S = (u * g) / (f * g) (eq. SxSyconv) in quad-double on every node
    the extended precision resolves; S identical to the S-only plan's."""
    pts = _clustered(K, frac, seed=900 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "grad"])
    S, g = plan.gradient(Y)
    S_only = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S"]).distance(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(S, S_only)
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, "fp64x4", grad=True)
    g = g.cpu().numpy().reshape(2, -1)
    deep, valid = ref["deep"], ref["valid"]
    dG = np.abs(g - ref["grad"].T)
    beyond = _beyond_dd(ref)
    print(f"\n[qd grad {dims}] max|dgrad| deep={dG[:, deep].max():.3e} beyond double-double={beyond.sum()}")
    assert beyond.sum() > 0
    assert np.all(dG[:, deep] <= parity.bound(ref, TOL_GRAD_XP)[deep])
    assert dG[:, valid].max() <= parity.TOL_GRAD
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    assert np.all(g[:, inval] == 0)


def test_qd3d_distance_and_gradient_vs_oracle(dt):
    """3D (rows, strided y lines, fused z lines, all in quad-double): S and
    grad S on every node against the oracle; nodes beyond the double-double
    band are resolved, nodes beyond the quad-double band report S_max."""
    dims, K, tau_h = (96, 40, 30), 12, 0.5
    pts = _clustered(K, 0.25, seed=820 + K, D=3)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "grad"])
    assert plan.padded == tuple(parity.padded(n) for n in dims)
    S, g = plan.gradient(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0,) * 3, tau, pts, "fp64x4", grad=True)
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(3, -1)
    dS = np.abs(S - ref["S_ref"])
    dG = np.abs(g - ref["grad"].T)
    deep, valid = ref["deep"], ref["valid"]
    beyond = _beyond_dd(ref)
    print(f"\n[qd3d {dims}] max|dS|/tau deep={dS[deep].max() / tau:.3e} max|dgrad| deep={dG[:, deep].max():.3e} "
          f"S_max/tau={ref['s_max'] / tau:.2f} valid={valid.mean():.3f} beyond double-double={beyond.sum()}")
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_XP, tau)[deep])
    assert np.all(dG[:, deep] <= parity.bound(ref, TOL_GRAD_XP)[deep])
    assert beyond.sum() > 0
    inval = ~valid & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    if inval.any():
        np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-12)
        assert np.all(g[:, inval] == 0)


def test_qd_hessian_vs_oracle(dt):
    """The Hessian of eqs. Sxx, Syy, Sxy in quad-double on every node the
    extended precision resolves; S and grad S equal the S + grad S plan's."""
    dims, K, tau_h = (100, 77), 5, 1.0
    pts = _clustered(K, 0.25, seed=840 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "grad", "hess"])
    res = plan.forward(Y, S=True, grad=True, hess=True)
    S2, g2 = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "grad"]).gradient(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(res["S"], S2) and torch.equal(res["grad"], g2)
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, "fp64x4", grad=True, hess=True)
    H = res["hess"].cpu().numpy().reshape(3, -1)
    Href = parity.hess_components(ref["hess"], 2)
    deep, valid = ref["deep"], ref["valid"]
    scale = 1.0 / tau + 1.0 / min(h)
    dH = np.abs(H - Href)
    beyond = _beyond_dd(ref)
    print(f"\n[qd hess {dims}] max|dH|/(1/tau+1/h) deep={dH[:, deep].max() / scale:.3e} "
          f"beyond double-double={beyond.sum()}")
    assert beyond.sum() > 0
    assert np.all(dH[:, deep] <= parity.bound(ref, TOL_HESS_XP, scale)[deep])
    assert dH[:, valid].max() <= parity.TOL_HESS * scale


def test_qd_backward_vs_oracle(dt):
    """The adjoint (dL/dY, dL/dtau) in quad-double against the oracle's
    analytic sums, with G on every valid node off the threshold's shell,
    including nodes beyond the double-double band; per component within the
    bound of the float64 adjoint tests, taken at the quad-double threshold."""
    dims, K, tau_h = (100, 77), 5, 1.0
    pts = _clustered(K, 0.25, seed=860 + K)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    plan = dt.Plan(dims, h, None, tau, precision="fp64x4", outputs=["S", "backward"])
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, "fp64x4", rmean=True)
    lnphi = ref["lnphi"]
    G = np.random.default_rng(861).standard_normal(lnphi.shape)
    G[np.abs(lnphi - np.log(ref["theta"])) < np.log(2.0)] = 0.0
    G[~ref["valid"]] = 0.0
    theta_dd = oracle.theta("fp64x2", ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond = (G != 0) & (lnphi < np.log(theta_dd))
    assert beyond.sum() > 100
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
    noise = parity.adjoint_noise("fp64x4", ref["padded"], ref["kernel_l1"], w_l2)
    bY, bt = parity.fp64_adjoint_bounds(sens[:, 0], sens[:, 1], float(aG @ tw), float((aG * ratio) @ tw), noise,
                                        dY_ref)
    rY = float((np.abs(dY - dY_ref) / bY).max())
    rt = abs(dtau - dtau_ref) / bt
    print(f"\n[qd backward {dims}] G beyond double-double={beyond.sum()} max|ddY|/bound={rY:.3f} "
          f"|ddtau|/bound={rt:.3f}")
    assert rY <= 1.0
    assert rt <= 1.0


def test_qd_rejects_what_it_does_not_build(dt):
    with pytest.raises(RuntimeError):
        dt.Plan((64, 64), None, None, 0.02, precision="fp64x4", outputs=["S", "sign"])
    with pytest.raises(RuntimeError):
        dt.Plan((160, 32, 32), None, None, 0.05, precision="fp64x4", outputs=["S"])


@pytest.mark.parametrize("prec", ["fp64x2", "fp64x4"])
@pytest.mark.parametrize("dims", [(200, 400), (300, 700)])
def test_xp_long_columns_gradient(dt, prec, dims):
    """S + grad S with long padded columns (1024 and 2048 points: one line per
    block; double-double keeps four or eight spectrum bins per thread,
    quad-double four, on 256 or 512 threads): every resolved node against
    the oracle, S equal to the S-only plan's."""
    K, tau_h = 5, 2.0
    pts = _clustered(K, 0.3, seed=880 + dims[1])
    pts[:, [0, 1]] = pts[:, [1, 0]]   # the sources near y = 0: long distances along the columns
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    Y = torch.from_numpy(pts).cuda()
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad"])
    assert plan.padded == tuple(parity.padded(n) for n in dims)
    S, g = plan.gradient(Y)
    S_only = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S"]).distance(Y)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    assert torch.equal(S, S_only)
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, prec, grad=True)
    S = S.cpu().numpy().ravel()
    g = g.cpu().numpy().reshape(2, -1)
    dS = np.abs(S - ref["S_ref"])
    dG = np.abs(g - ref["grad"].T)
    deep, valid = ref["deep"], ref["valid"]
    lower = "fp64" if prec == "fp64x2" else "fp64x2"
    theta_low = oracle.theta(lower, ref["padded"], ref["kernel_l1"], ref["g_l2"])
    beyond = deep & (ref["lnphi"] < np.log(theta_low))
    print(f"\n[{prec} long columns {dims} -> {plan.padded}] max|dS|/tau deep={dS[deep].max() / tau:.3e} "
          f"max|dgrad| deep={dG[:, deep].max():.3e} beyond {lower}={beyond.sum()}")
    assert beyond.sum() > 0
    assert dS.max() <= parity.TOL_S_TAU * tau
    assert np.all(dS[deep] <= parity.bound(ref, TOL_S_TAU_XP, tau)[deep])
    assert np.all(dG[:, deep] <= parity.bound(ref, TOL_GRAD_XP)[deep])
    assert dG[:, valid].max() <= parity.TOL_GRAD
