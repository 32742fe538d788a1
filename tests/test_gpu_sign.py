"""GPU parity of the sign channels (winding number in 2D, topological degree
in 3D) and of distance fields whose sources come from a shape."""

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
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_polygon_sign_and_distance_2d(dt, prec):
    dims = (120, 96)
    h = (1.0 / 120, 1.0 / 96)
    tau = 1.5 * h[0]
    verts = synth.star_polygon(24, 0.2, 0.45, seed=41)
    poly = synth.sample_polygon(verts, 900)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "sign"])
    P = torch.from_numpy(poly).cuda()
    res = plan.forward(polygon=P, S=True, grad=True, label=True, mu=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    # mu against the direct sum on the snapped polygon
    idx, valid = oracle.snap(poly, (0.0, 0.0), h, dims)
    assert valid.all()
    Yh = oracle.node_coords(idx, (0.0, 0.0), h)
    X = oracle.grid_nodes(dims, (0.0, 0.0), h)
    mu_ref = oracle.winding_number(X, Yh)
    mu = _np(res["mu"]).astype(np.float64).ravel()
    lin = idx[:, 0] + dims[0] * idx[:, 1]
    nosrc = np.ones(X.shape[0], bool)
    nosrc[lin] = False
    dmu = np.abs(mu - mu_ref)[nosrc].max()
    # labels against exact geometry outside the one-cell band
    w = oracle.polygon_winding_exact(X, poly.astype(np.float64))
    dist = oracle.polygon_distance(X, poly.astype(np.float64))
    band = dist < np.sqrt(2) * max(h)
    lab = _np(res["label"]).ravel()
    exact = np.where(w != 0, 1, -1)
    mism_out = int(np.sum(lab[~band] != exact[~band]))
    mism_in = int(np.sum(lab[band] != exact[band]))
    # labels agree with the oracle's mu wherever mu is clearly on one side
    clear = nosrc & (np.abs(mu_ref - 0.5) > 1e-2)
    mism_mu = int(np.sum(lab[clear] != oracle.label_from_mu(mu_ref[clear])))
    print(f"\n[polygon {prec}] max|dmu|={dmu:.3e} label mismatches outside band={mism_out} "
          f"inside band={mism_in}/{band.sum()} vs oracle-mu={mism_mu}")
    assert dmu <= parity.TOL_MU
    assert mism_out == 0
    assert mism_mu == 0
    # distance from the polygon's own points (float64: the per-node bound)
    ref = parity.reference(dims, h, (0.0, 0.0), tau, poly, prec, grad=True)
    S = _np(res["S"]).astype(np.float64).ravel()
    dS = np.abs(S - ref["S_ref"])
    lim = parity.bound(ref, parity.TOL_S_TAU_FP64, tau) if prec == "fp64" else parity.TOL_S_TAU * tau
    print(f"[polygon {prec}] max|dS|/bound={(dS / lim).max():.3e}")
    assert np.all(dS <= lim)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mesh_sign_and_distance_3d(dt, prec):
    n = 48
    dims = (n, n, n)
    h = (1.0 / n,) * 3
    tau = 1.5 / n
    V, F = synth.harmonic_star_mesh(seed=43, n_lon=48, n_ring=30, max_radius=0.38)
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "sign"])
    Vd, Fd = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    res = plan.forward(vertices=Vd, faces=Fd, S=True, grad=True, label=True, mu=True)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    Yh, P, idx, valid = oracle.sign.snapped_mesh_sources(V, F, (0.0,) * 3, h, dims)
    assert valid.all()
    rng = np.random.default_rng(44)
    cells = rng.choice(n ** 3, 6000, replace=False)
    X = oracle.grid_nodes(dims, (0.0,) * 3, h, cells)
    mu_ref = oracle.topological_degree(X, Yh, P)
    mu = _np(res["mu"]).astype(np.float64).ravel()[cells]
    src = set((idx[:, 0] + n * (idx[:, 1] + n * idx[:, 2])).tolist())
    nosrc = np.array([c not in src for c in cells])
    dmu = np.abs(mu - mu_ref)[nosrc].max()
    wexact = oracle.mesh_winding_exact(X, V, F)
    dist = oracle.mesh_distance(X, V, F)
    band = dist < np.sqrt(3) * h[0]
    lab = _np(res["label"]).ravel()[cells]
    exact = np.where(wexact > 0.5, 1, -1)
    mism_out = int(np.sum(lab[~band] != exact[~band]))
    mism_in = int(np.sum(lab[band] != exact[band]))
    print(f"\n[mesh {prec}] max|dmu|={dmu:.3e} label mismatches outside band={mism_out} inside={mism_in}/{band.sum()}")
    assert dmu <= parity.TOL_MU
    assert mism_out == 0
    # distance from the snapped incenters
    ref = parity.reference(dims, h, (0.0,) * 3, tau, Yh.astype(np.float32), prec, cells=cells)
    # reference() snaps its input again: snapped node centres map to themselves
    S = _np(res["S"]).astype(np.float64).ravel()[cells]
    dS = np.abs(S - ref["S_ref"])
    lim = parity.bound(ref, parity.TOL_S_TAU_FP64, tau) if prec == "fp64" else parity.TOL_S_TAU * tau
    print(f"[mesh {prec}] max|dS|/tau={dS.max() / tau:.3e} max|dS|/bound={(dS / lim).max():.3e}")
    assert np.all(dS <= lim)


def test_signed_outputs(dt):
    dims = (80, 64)
    h = (1 / 80, 1 / 64)
    verts = synth.star_polygon(24, 0.2, 0.45, seed=45)
    poly = torch.from_numpy(synth.sample_polygon(verts, 700)).cuda()
    plan = dt.Plan(dims, h, None, 2 * h[0], precision="fp64", outputs=["S", "grad", "sign"])
    a = plan.forward(polygon=poly, S=True, grad=True, label=True)
    b = plan.forward(polygon=poly, S=True, grad=True, label=True, signed=True)
    lab = a["label"].to(torch.float64)
    assert torch.equal(b["label"], a["label"])
    assert torch.equal(b["S"], a["S"] * lab)
    assert torch.equal(b["grad"], a["grad"] * lab)
    lab_only = plan.sign(polygon=poly)
    assert torch.equal(lab_only, a["label"])
