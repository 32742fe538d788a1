"""Stress test of the batched path's graph replay: random instance sizes,
many replays with new source coordinates copied into the captured input
buffer, the per-instance source counts switching every 50 replays (each
switch re-captures the graph), and the outputs cleared between some replays.
Every replay must equal the eager batched call bit for bit, and the eager
batched call must equal one-instance plans of each instance bit for bit
(same padding, radix schedule and per-instance scaling)."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


N_INST = 12
N_SETS = 4          # coordinate sets per source-count layout


def _problem(seed):
    rng = np.random.default_rng(seed)
    dims = [(int(rng.integers(9, 400)), int(rng.integers(9, 400))) for _ in range(N_INST)]
    taus = [float(rng.uniform(1.0, 3.0)) / d[0] for d in dims]
    layouts = [[int(rng.integers(1, 300)) for _ in range(N_INST)] for _ in range(2)]
    return dims, taus, layouts


def _sets(dt, layouts, seed):
    out = []
    for li, Ks in enumerate(layouts):
        for j in range(N_SETS):
            pts = [synth.generators.uniform_points(2, K, seed=seed + 1000 * li + 100 * j + i)
                   for i, K in enumerate(Ks)]
            Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
            out.append((Y.cuda(), offs, pts))
    return out


@pytest.mark.parametrize("prec,replays", [("fp32", 1000), ("fp64", 200)])
def test_batch_graph_replay_stress(dt, prec, replays):
    dims, taus, layouts = _problem(4242 if prec == "fp32" else 4343)
    print(f"\n[{prec}] dims {dims}", flush=True)
    sets = _sets(dt, layouts, 77)
    eager = dt.BatchPlan(dims, taus, precision=prec, graph=False)
    refs = []
    for Y, offs, _ in sets:
        refs.append(eager.forward(Y, offs))
    torch.cuda.synchronize()
    assert eager.last_error() == 0

    # one-instance plans of each instance, on the first set of each layout
    for li in range(2):
        Y, offs, pts = sets[li * N_SETS]
        views = eager.views(*refs[li * N_SETS])
        for i in range(N_INST):
            one = dt.BatchPlan([dims[i]], [taus[i]], precision=prec, graph=False)
            Yi, oi = dt.BatchPlan.pack([torch.from_numpy(pts[i])])
            S1, G1 = one.forward(Yi.cuda(), oi)
            torch.cuda.synchronize()
            s, g = views[i]
            assert torch.equal(S1.view_as(s), s) and torch.equal(G1.view_as(g), g), \
                f"instance {i} {dims[i]} layout {li}: max|dS| {(S1.view_as(s) - s).abs().max().item():.3e}"

    graph = dt.BatchPlan(dims, taus, precision=prec, graph=True)
    kmax = max(int(Y.shape[0]) for Y, _, _ in sets)
    ybuf = torch.empty(kmax, 2, dtype=torch.float32, device="cuda")
    S, G = graph.empty_outputs()
    for rep in range(replays):
        idx = ((rep // 50) % 2) * N_SETS + rep % N_SETS
        Y, offs, _ = sets[idx]
        yv = ybuf[:Y.shape[0]]
        yv.copy_(Y)
        if rep % 7 == 0:
            S.fill_(float("nan"))
            G.fill_(float("nan"))
        graph.forward_into(yv, offs, S, G)
        Sr, Gr = refs[idx]
        if not (torch.equal(S, Sr) and torch.equal(G, Gr)):
            pytest.fail(f"replay {rep} (set {idx}) differs from the eager call")
    torch.cuda.synchronize()
    assert graph.last_error() == 0
    print(f"[{prec}] {replays} replays equal to the eager calls", flush=True)
