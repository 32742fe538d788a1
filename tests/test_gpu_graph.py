"""dt_forward and dt_backward captured into a HIP graph (torch.cuda.graph).

The calls only enqueue kernels on the caller's stream: no allocation, no host
synchronisation, no memset nodes (buffers are cleared by fill kernels), so a
caller can capture them.  Each graph is replayed several times with new
point coordinates copied into the captured input, with eager work and
synchronisations between replays, and every replay must equal the eager
result bit for bit (the passes are deterministic: the splat's atomics add
exact integers).
"""

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


def _capture(fn):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()                                    # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


# (64, 700) in quad-double: 2048-point columns of 128 KB of LDS per block, whose
# launches raise the kernel's LDS limit while the stream is being captured
@pytest.mark.parametrize("dims,prec", [((40, 36, 33), "fp32"), ((128, 128), "fp64"), ((96, 80), "fp64x2"),
                                       ((96, 80), "fp64x4"), ((64, 700), "fp64x4")])
def test_forward_graph_replays(dt, dims, prec):
    D = len(dims)
    h = tuple(1.0 / n for n in dims)
    plan = dt.Plan(dims, h, None, 2.0 * h[0], precision=prec, outputs=["S", "grad"])
    sets = [torch.from_numpy(synth.generators.uniform_points(D, 64, seed=500 + i)).cuda() for i in range(4)]
    eager = []
    for Y in sets:
        r = plan.forward(Y, S=True, grad=True)
        eager.append({k: v.clone() for k, v in r.items()})
    torch.cuda.synchronize()
    Ystatic = sets[0].clone()
    out = {"S": plan._empty(), "grad": plan._empty(D)}
    g = _capture(lambda: plan.forward_into(out, Ystatic))
    other = dt.Plan((64, 48), None, None, 2.0 / 64, precision="fp32", outputs=["S"])
    Yo = torch.from_numpy(synth.generators.uniform_points(2, 30, seed=9)).cuda()
    for rep in range(3):
        for i in (2, 0, 3, 1):
            Ystatic.copy_(sets[i])
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out["S"], eager[i]["S"]), (rep, i)
            assert torch.equal(out["grad"], eager[i]["grad"]), (rep, i)
            other.distance(Yo)                  # eager work between replays
            torch.cuda.synchronize()
    assert plan.last_error() == 0
    # launch-bound size: time eager calls against graph replays
    n = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        plan.forward_into(out, Ystatic)
    e1.record()
    torch.cuda.synchronize()
    t_eager = e0.elapsed_time(e1) / n
    e0.record()
    for _ in range(n):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    t_graph = e0.elapsed_time(e1) / n
    print(f"\n[graph {dims} {prec}] eager {t_eager * 1e3:.1f} us/call, graph replay {t_graph * 1e3:.1f} us/call")


def test_backward_graph_replays(dt):
    dims = (40, 36, 33)
    D = 3
    plan = dt.Plan(dims, None, None, 2.0 / 40, precision="fp32", outputs=["S", "backward"])
    sets = [torch.from_numpy(synth.generators.uniform_points(D, 64, seed=600 + i)).cuda() for i in range(3)]
    Ss = [plan.distance(Y).clone() for Y in sets]
    Gs = [S.clone() * 0.5 for S in Ss]
    eager = [tuple(t.clone() for t in plan.backward(Y, S, G)) for Y, S, G in zip(sets, Ss, Gs)]
    torch.cuda.synchronize()
    Ystatic, Sstatic, Gstatic = sets[0].clone(), Ss[0].clone(), Gs[0].clone()
    dY = torch.empty(64, D, dtype=torch.float32, device="cuda")
    dtau = torch.empty((), dtype=torch.float64, device="cuda")
    g = _capture(lambda: plan.backward_into(dY, dtau, Ystatic, Sstatic, Gstatic))
    for rep in range(3):
        for i in (1, 2, 0):
            Ystatic.copy_(sets[i])
            Sstatic.copy_(Ss[i])
            Gstatic.copy_(Gs[i])
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(dY, eager[i][0]), (rep, i)
            assert torch.equal(dtau, eager[i][1]), (rep, i)
    assert plan.last_error() == 0
