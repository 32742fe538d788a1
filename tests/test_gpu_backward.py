"""GPU parity of the adjoint (dL/dY, dL/dtau) and of the autograd wrapper."""

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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# dL/dY is stored in float32 (the type of Y), so the float64 path is held to
# float32 storage rounding (2e-7 relative); dL/dtau is float64 throughout.
CASES = [((64, 56), 20, 3.0, "fp64", (2e-7, 1e-10)), ((64, 56), 20, 3.0, "fp32", (1e-3, 1e-3)),
         ((36, 32, 30), 25, 2.0, "fp64", (2e-7, 1e-10)), ((36, 32, 30), 25, 2.0, "fp32", (1e-3, 1e-3)),
         ((130, 100), 120, 1.0, "fp32", (1e-3, 1e-3))]


@pytest.mark.parametrize("dims,K,tau_h,prec,tol", CASES)
def test_backward_against_oracle(dt, dims, K, tau_h, prec, tol):
    D = len(dims)
    h = tuple(1.0 / n for n in dims)
    tau = tau_h * h[0]
    pts = synth.generators.uniform_points(D, K, seed=501 + K + D)
    ref = parity.reference(dims, h, (0.0,) * D, tau, pts, prec)
    rng = np.random.default_rng(502)
    G = rng.standard_normal(ref["S_ref"].shape)
    # G = 0 on the shell around the threshold, where the two sides may
    # legitimately disagree on validity; elsewhere validity is clear-cut.
    lnphi = -ref["S_exact"] / tau
    shell = np.abs(lnphi - np.log(ref["theta"])) < np.log(2.0)
    G[shell] = 0.0
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "backward"])
    Y = torch.from_numpy(pts).cuda()
    S = plan.distance(Y)
    Gt = torch.from_numpy(G).to(plan.dtype).cuda().reshape(plan.shape)
    dY, dtau = plan.backward(Y, S, Gt)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    dY_ref, dtau_ref = oracle.loss_gradients(ref["X"], ref["Yhat"], tau, G, ref["valid"])
    e_y = _rel(dY.cpu().numpy(), dY_ref)
    e_t = abs(float(dtau.cpu()) - dtau_ref) / abs(dtau_ref)
    print(f"\n[backward {dims} {prec}] rel L2 dL/dY={e_y:.3e} rel dL/dtau={e_t:.3e} valid={ref['valid'].mean():.3f}")
    assert e_y <= tol[0]
    assert e_t <= tol[1]


def test_autograd_matches_oracle_gradient(dt):
    """loss = sum (S - T)^2 through the autograd Function; every node valid."""
    dims = (40, 36, 32)
    h = tuple(1.0 / n for n in dims)
    tau = 3.0 * h[0]
    pts = synth.jittered_sphere_points(60, 0.25, 2 * h[0], seed=503)
    plan = dt.Plan(dims, h, None, tau, precision="fp64", outputs=["S", "backward"])
    ref = parity.reference(dims, h, (0.0,) * 3, tau, pts, "fp64")
    assert ref["valid"].all()
    T = np.random.default_rng(504).random(ref["S_ref"].shape) * 0.3
    Y = torch.from_numpy(pts).cuda().requires_grad_(True)
    tau_t = torch.tensor(tau, dtype=torch.float64, device="cuda", requires_grad=True)
    import paper_1112_3010_amd as dtm
    S = dtm.distance_field(Y, plan, tau_t)
    loss = ((S - torch.from_numpy(T).cuda().reshape(S.shape)) ** 2).sum()
    loss.backward()
    G = 2.0 * (ref["S_exact"] - T)
    dY_ref, dtau_ref = oracle.loss_gradients(ref["X"], ref["Yhat"], tau, G)
    e_y = _rel(Y.grad.cpu().numpy(), dY_ref)
    e_t = abs(float(tau_t.grad.cpu()) - dtau_ref) / abs(dtau_ref)
    print(f"\n[autograd] rel dL/dY={e_y:.3e} rel dL/dtau={e_t:.3e}")
    assert e_y <= 2e-7 and e_t <= 1e-10


def test_autograd_refuses_a_tau_other_than_the_plans(dt):
    """The kernel spectra belong to the plan's tau: a different tau input is
    an error, not a silent forward at the old tau."""
    dims = (40, 36)
    h = tuple(1.0 / n for n in dims)
    plan = dt.Plan(dims, h, None, 2.0 * h[0], precision="fp32", outputs=["S", "backward"])
    Y = torch.from_numpy(synth.generators.uniform_points(2, 10, seed=505)).cuda().requires_grad_(True)
    import paper_1112_3010_amd as dtm
    ok = torch.tensor(plan.tau, dtype=torch.float64, device="cuda", requires_grad=True)
    dtm.distance_field(Y, plan, ok).sum().backward()
    assert ok.grad is not None and Y.grad is not None
    bad = torch.tensor(plan.tau * 1.01, dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        dtm.distance_field(Y, plan, bad)


# dL/dY of the float64 path is held to float32 storage rounding (2e-7); the
# other bounds are about 50 times the errors measured on an MI355X (float32:
# 1.8e-7 and 2.7e-8; float64 dL/dtau: 4e-15).
@pytest.mark.parametrize("prec,tol", [("fp32", (1e-5, 1e-6)), ("fp64", (2e-7, 1e-12))])
def test_single_source_backward_closed_form(dt, prec, tol):
    """One source: S = r for every tau, so dS/dY = -(X - Y)/r and dS/dtau = 0
    on every valid node.  With G vanishing well inside the band (no validity
    question at its edge), dL/dY = -sum G (X - Y)/r and dL/dtau = 0, written
    here without the oracle.  G is skewed so that dL/dY is far from zero."""
    dims = (36, 32, 30)
    h = tuple(1.0 / n for n in dims)
    tau = 2.0 * h[0]
    node = (12, 15, 8)
    Y = torch.tensor([[(node[a] + 0.5) * h[a] for a in range(3)]], dtype=torch.float32).cuda()
    plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "backward"])
    S = plan.distance(Y)
    torch.cuda.synchronize()
    s_max = plan.last_stats()["s_max"]
    zz, yy, xx = np.meshgrid(*[np.arange(dims[a]) * h[a] for a in (2, 1, 0)], indexing="ij")
    d = np.stack([xx.ravel() - node[0] * h[0], yy.ravel() - node[1] * h[1], zz.ravel() - node[2] * h[2]])
    r = np.sqrt((d ** 2).sum(axis=0))
    R = 0.6 * s_max
    G = np.maximum(0.0, 1.0 - r / R) ** 2 * (1.0 + 2.0 * d[0] / R + d[1] / R)
    assert np.count_nonzero(G) > 500
    with np.errstate(invalid="ignore", divide="ignore"):
        unit = np.where(r > 0, d / r, 0.0)
    dY_ref = -(G * unit).sum(axis=1)
    Gt = torch.from_numpy(G).to(plan.dtype).cuda().reshape(plan.shape)
    dY, dtau = plan.backward(Y, S, Gt)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    e_y = _rel(dY.cpu().numpy().ravel(), dY_ref)
    scale_t = float(np.abs(G).sum() * s_max / tau)
    e_t = abs(float(dtau.cpu())) / scale_t
    print(f"\n[single-source backward {prec}] |dL/dY|={np.linalg.norm(dY_ref):.3e} rel err={e_y:.3e} "
          f"|dL/dtau|/(sum|G| S_max/tau)={e_t:.3e}")
    assert e_y <= tol[0]
    assert e_t <= tol[1]
