"""GPU parity of plans with reduced padding (calls of at most k_max sources).

The plan pads each axis only to the smallest power of two >= n + c, with the
kernels truncated to |d_a| <= c cells; what the truncation drops is below
Theta / c_theta at every node.  Every check is against the exact
(untruncated) oracle, with the validity threshold of the reduced grid, to
the same tolerances as the fully padded plans.  Sources are clustered so
that part of each grid lies beyond the truncation distance.
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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _plan(dt, dims, tau, K, prec, outputs, iso=False, expect=None):
    """Reduced plan on the unit box (h_a = 1/n_a) or, iso, with cubic cells
    h = 1/n_x on every axis."""
    h = tuple(1.0 / dims[0] for _ in dims) if iso else tuple(1.0 / n for n in dims)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=outputs, k_max=K)
    Mp, cut = parity.padded_reduced(dims, h, tau, K, prec)
    full = tuple(parity.padded(n) for n in dims)
    assert plan.padded == Mp and plan.cut == cut
    assert any(c > 0 for c in cut) and np.prod(Mp) < np.prod(full), "the case must reduce the padding"
    if expect:
        assert expect in Mp, f"the case must use the {expect}-point engines"
    return plan, h, Mp


def _clustered(D, K, seed, h, centre=(0.3, 0.35, 0.3)):
    if D == 3:
        return synth.generators.jittered_sphere_points(K, 0.12, 2 * h, seed=seed, centre=centre)
    pts = synth.generators.uniform_points(2, K, seed=seed, lo=0.1, hi=0.35)
    return pts.astype(np.float32)


def _sample_cells(dims, n_random, seed, z_cluster=None):
    """Every node of three axis planes (through the cluster, at the far
    faces), of the z plane z_cluster if given, and n_random further nodes."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    parts = [idx[:, :, nx // 3].ravel(), idx[:, ny - 1, :].ravel(), idx[nz - 1, :, :].ravel(),
             np.random.default_rng(seed).choice(nx * ny * nz, n_random, replace=False)]
    if z_cluster is not None:
        parts.append(idx[z_cluster].ravel())
    return np.unique(np.concatenate(parts))


def _check(tag, prec, tau, h, ref, stats, S, g, H=None):
    assert stats["theta"] == pytest.approx(ref["theta"], rel=1e-7), tag
    dS = np.abs(S - ref["S_ref"])
    deep = ref["deep"]
    dG = np.abs(g - ref["grad"].T)[:, deep]
    inval = ~ref["valid"] & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    msg = (f"[{tag} {prec}] max|dS|/tau all={dS.max() / tau:.3e} deep={dS[deep].max() / tau:.3e} "
           f"max|dgrad| deep={dG.max():.3e} valid={ref['valid'].mean():.3f} beyond={inval.mean():.3f}")
    assert dS.max() <= parity.TOL_S_TAU * tau, msg
    assert dG.max() <= parity.TOL_GRAD, msg
    if prec == "fp64":
        assert np.all(dS[deep] <= parity.bound(ref, parity.TOL_S_TAU_FP64, tau)[deep]), msg
        assert np.all(dG <= parity.bound(ref, parity.TOL_GRAD_FP64)[deep]), msg
    assert inval.mean() > 0.05, "part of the grid must lie beyond the threshold"
    np.testing.assert_allclose(S[inval], ref["s_max"], rtol=1e-6)
    assert np.all(g[:, inval] == 0), msg
    if H is not None:
        D = g.shape[0]
        Href = parity.hess_components(ref["hess"], D)
        dH = np.abs(H - Href)[:, deep]
        scale = 1.0 / tau + 1.0 / min(h)
        msg += f" max|dH|/(1/tau+1/h) deep={dH.max() / scale:.3e}"
        assert dH.max() <= parity.TOL_HESS * scale, msg
        if prec == "fp64":
            assert np.all(dH <= parity.bound(ref, 1e-7, scale)[deep]), msg
    return msg


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_reduced_fields_2d(dt, prec):
    """300 x 200 nodes, tau = 1 cell, 100 sources: 512 x 256 instead of
    1024 x 512; S, grad S and the Hessian on every node."""
    dims, K = (300, 200), 100
    tau = 1.0 / dims[0]
    plan, h, Mp = _plan(dt, dims, tau, K, prec, ["S", "grad", "hess"])
    pts = _clustered(2, K, 611, h[0])
    res = plan.forward(torch.from_numpy(pts).cuda(), S=True, grad=True, hess=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, prec, grad=True, hess=True, padded_dims=Mp)
    msg = _check(f"reduced 2d M={Mp}", prec, tau, h, ref, plan.last_stats(), _np(res["S"]).ravel(),
                 _np(res["grad"]).reshape(2, -1), _np(res["hess"]).reshape(3, -1))
    print("\n" + msg)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_reduced_fields_3d(dt, prec):
    """150 x 140 x 130 nodes, tau = 2 cells, 300 sources on a small sphere:
    256^3 instead of 512^3; S and grad S on three full planes and 150 000
    further nodes."""
    dims, K = (150, 140, 130), 300
    tau = 2.0 / dims[0]
    plan, h, Mp = _plan(dt, dims, tau, K, prec, ["S", "grad"])
    pts = _clustered(3, K, 612, 1.0 / dims[0])
    res = plan.forward(torch.from_numpy(pts).cuda(), S=True, grad=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    cells = _sample_cells(dims, 150_000, 613)
    ref = parity.reference(dims, h, (0.0,) * 3, tau, pts, prec, grad=True, cells=cells, padded_dims=Mp)
    S = _np(res["S"]).ravel()[cells]
    g = _np(res["grad"]).reshape(3, -1)[:, cells]
    print("\n" + _check(f"reduced 3d M={Mp}", prec, tau, h, ref, plan.last_stats(), S, g))


def _inside(centre, dims, h):
    """The sphere's centre moved into the box where an axis is short."""
    return tuple(min(c, 0.5 * n * hh) for c, n, hh in zip(centre, dims, h))


# The engines at 288 = 2 * 12^2 and 392 = 2 * 14^2 (columns: pair-split;
# rows: 12 x 12 and 14 x 14 Stockham on 144 and 196 complex points): an axis
# that needs more than 256 (384) points pads to 288 (392) instead of 512 (1024).
CASES_EXT_2D = [((300, 262), "fp32", 288), ((262, 240), "fp32", 288), ((240, 230), "fp64", 288),
                ((350, 300), "fp32", 392), ((330, 300), "fp64", 392)]
CASES_EXT_3D = [((120, 250, 250), "fp32", 288), ((250, 120, 250), "fp32", 288), ((120, 230, 230), "fp64", 288),
                ((230, 120, 230), "fp64", 288), ((300, 120, 300), "fp32", 392), ((280, 120, 280), "fp64", 392)]


@pytest.mark.parametrize("dims,prec,length", CASES_EXT_2D)
def test_reduced_nonpow2_2d(dt, dims, prec, length):
    """2D, cubic cells, tau = h, 100 clustered sources: y (the fused pass on
    the pair-split engine) and/or x (the row passes) padded to 288 or 392; S,
    grad S and H on every node."""
    K = 100
    tau = 1.0 / dims[0]
    plan, h, Mp = _plan(dt, dims, tau, K, prec, ["S", "grad", "hess"], iso=True, expect=length)
    pts = _clustered(2, K, 631, h[0])
    res = plan.forward(torch.from_numpy(pts).cuda(), S=True, grad=True, hess=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, prec, grad=True, hess=True, padded_dims=Mp)
    print("\n" + _check(f"reduced 2d M={Mp}", prec, tau, h, ref, plan.last_stats(), _np(res["S"]).ravel(),
                        _np(res["grad"]).reshape(2, -1), _np(res["hess"]).reshape(3, -1)))


@pytest.mark.parametrize("dims,prec,length", CASES_EXT_3D)
def test_reduced_nonpow2_3d(dt, dims, prec, length):
    """3D, cubic cells, tau = h, 300 sources on a small sphere: two of the
    three axes padded to 288 or 392 (x: row passes; y: strided passes; z: the
    fused pass); S and grad S on four full planes and 150 000 further nodes."""
    K = 300
    tau = 1.0 / dims[0]
    plan, h, Mp = _plan(dt, dims, tau, K, prec, ["S", "grad"], iso=True, expect=length)
    pts = _clustered(3, K, 632, h[0], centre=_inside((0.3, 0.35, 0.3), dims, h))
    assert np.all(pts >= 0) and np.all(pts < np.array(dims) * np.array(h)), "sources inside the grid"
    res = plan.forward(torch.from_numpy(pts).cuda(), S=True, grad=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    cells = _sample_cells(dims, 150_000, 633, z_cluster=int(0.3 / h[2]))
    ref = parity.reference(dims, h, (0.0,) * 3, tau, pts, prec, grad=True, cells=cells, padded_dims=Mp)
    S = _np(res["S"]).ravel()[cells]
    g = _np(res["grad"]).reshape(3, -1)[:, cells]
    print("\n" + _check(f"reduced 3d M={Mp}", prec, tau, h, ref, plan.last_stats(), S, g))


# float32: relative L2 error of dL/dY and relative error of dL/dtau (the
# bar of the fully padded adjoint tests)
TOL_ADJ_FP32 = 1e-3


@pytest.mark.parametrize("dims,tau_h,K,prec,iso", [
    ((300, 200), 1.0, 100, "fp64", False), ((300, 200), 1.0, 100, "fp32", False),
    ((72, 70, 66), 1.5, 100, "fp32", False), ((300, 262), 1.0, 100, "fp32", True),
    ((40, 262, 250), 1.0, 100, "fp32", True), ((262, 90, 120), 1.0, 100, "fp32", True)])
def test_reduced_backward(dt, dims, tau_h, K, prec, iso):
    """dL/dY and dL/dtau of a reduced plan against the oracle (G = 0 on the
    shell around the threshold, as for the fully padded plans); the cubic-cell
    cases pad one or two axes to 288."""
    D = len(dims)
    tau = tau_h / dims[0]
    plan, h, Mp = _plan(dt, dims, tau, K, prec, ["S", "backward"], iso=iso, expect=288 if iso else None)
    # the sphere inside the box (cubic cells of 1/n_x leave y and z shorter)
    if D == 3:
        pts = _clustered(D, K, 620 + D, 1.0 / dims[0], centre=_inside((0.3, 0.35, 0.3), dims, h))
    else:
        pts = _clustered(D, K, 620 + D, h[0])
    assert np.all(pts >= 0) and np.all(pts < np.array(dims) * np.array(h)), "sources inside the grid"
    ref = parity.reference(dims, h, (0.0,) * D, tau, pts, prec, padded_dims=Mp, rmean=prec == "fp64")
    rng = np.random.default_rng(621)
    G = rng.standard_normal(ref["S_ref"].shape)
    lnphi = ref["lnphi"]
    G[np.abs(lnphi - np.log(ref["theta"])) < np.log(2.0)] = 0.0
    G[~ref["valid"]] = 0.0
    Y = torch.from_numpy(pts).cuda()
    S = plan.distance(Y)
    dY, dtau = plan.backward(Y, S, torch.from_numpy(G).to(plan.dtype).cuda().reshape(plan.shape))
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    dY = dY.cpu().numpy().astype(np.float64)
    dtau = float(dtau.cpu())
    dY_ref, dtau_ref = oracle.loss_gradients(ref["X"], ref["Yhat"], tau, G, ref["valid"], workers=parity.WORKERS)
    e_y = _rel(dY, dY_ref)
    e_t = abs(dtau - dtau_ref) / abs(dtau_ref)
    msg = (f"[reduced backward {dims} M={Mp} {prec}] rel L2 dL/dY={e_y:.3e} rel dL/dtau={e_t:.3e} "
           f"valid={ref['valid'].mean():.3f}")
    if prec == "fp32":
        print("\n" + msg)
        assert e_y <= TOL_ADJ_FP32, msg
        assert e_t <= TOL_ADJ_FP32, msg
    else:
        # per component: the forward's float64 error bound carried through
        # the node weights (nodes near the threshold carry most of it)
        ratio = np.exp(np.log(ref["theta"]) - lnphi)
        aG = np.abs(G)
        C = np.stack([aG, aG * ratio], axis=1)
        sens = oracle.adjoint.source_weight_sums(ref["X"], ref["Yhat"], tau, C, workers=parity.WORKERS)
        tw = 1.0 + 2.0 * ref["rmean"] / tau
        w_l2 = float(np.sqrt(np.sum((G * np.exp(-lnphi)) ** 2)))
        noise = parity.adjoint_noise("fp64", Mp, ref["kernel_l1"], w_l2)
        bY, bt = parity.fp64_adjoint_bounds(sens[:, 0], sens[:, 1], float(aG @ tw), float((aG * ratio) @ tw),
                                            noise, dY_ref)
        rY = float((np.abs(dY - dY_ref) / bY).max())
        rt = abs(dtau - dtau_ref) / bt
        print(f"\n{msg} max|ddY|/bound={rY:.3f} |ddtau|/bound={rt:.3f}")
        assert rY <= 1.0, msg
        assert rt <= 1.0, msg
    # more sources than the plan was made for are refused
    more = torch.from_numpy(np.concatenate([pts, pts[:1]])).cuda()
    with pytest.raises(RuntimeError):
        plan.distance(more)
    with pytest.raises(RuntimeError):
        plan.backward(more, S, torch.zeros_like(S))
