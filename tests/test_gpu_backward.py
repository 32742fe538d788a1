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
