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
        dt.Plan((64, 64), None, None, 0.02, precision="fp64x2", outputs=["S", "hess"])
    with pytest.raises(Exception):
        dt.Plan((32, 32, 32), None, None, 0.05, precision="fp64x2", outputs=["S"])
