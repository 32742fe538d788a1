"""Distinct plans on distinct streams: the compute calls of different plans
share no device state (each plan computes in its own workspace), so calls
enqueued on three streams at once, interleaved, must give the same fields bit
for bit as the same calls made one after another on the default stream."""

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


ROUNDS = 6


def test_plans_on_concurrent_streams(dt):
    # plans of different kinds: 3D float32, 2D float64 with the Hessian, 2D
    # double-double, 2D quad-double with the gradient; and a batched plan
    a = dt.Plan((48, 40, 36), None, None, 2.0 / 48, precision="fp32", outputs=["S", "grad"])
    b = dt.Plan((200, 160), None, None, 2.0 / 200, precision="fp64", outputs=["S", "grad", "hess"])
    c = dt.Plan((96, 80), None, None, 2.0 / 96, precision="fp64x2", outputs=["S"])
    e = dt.Plan((64, 48), None, None, 1.0 / 64, precision="fp64x4", outputs=["S", "grad"])
    bdims = [(97, 130), (64, 64), (150, 40)]
    bp = dt.BatchPlan(bdims, [2.0 / d[0] for d in bdims], precision="fp32", graph=False)

    def inputs(r):
        ya = torch.from_numpy(synth.generators.uniform_points(3, 300, seed=7000 + r)).cuda()
        yb = torch.from_numpy(synth.generators.uniform_points(2, 500, seed=7100 + r)).cuda()
        yc = torch.from_numpy(synth.generators.uniform_points(2, 40, seed=7200 + r)).cuda()
        ye = torch.from_numpy(synth.generators.uniform_points(2, 8, seed=7400 + r)).cuda()
        pts = [torch.from_numpy(synth.generators.uniform_points(2, 50 + 10 * i, seed=7300 + 10 * r + i))
               for i in range(len(bdims))]
        yd, offs = dt.BatchPlan.pack(pts)
        return ya, yb, yc, yd.cuda(), offs, ye

    ins = [inputs(r) for r in range(ROUNDS)]
    torch.cuda.synchronize()

    def run_all(r, streams):
        ya, yb, yc, yd, offs, ye = ins[r]
        outs = {}
        with torch.cuda.stream(streams[0]):
            outs["a"] = a.forward(ya, S=True, grad=True)
            outs["e"] = e.forward(ye, S=True, grad=True)
        with torch.cuda.stream(streams[1]):
            outs["b"] = b.forward(yb, S=True, grad=True, hess=True)
        with torch.cuda.stream(streams[2]):
            outs["c"] = c.forward(yc, S=True)
            outs["d"] = dict(zip(("S", "grad"), bp.forward(yd, offs)))
        return outs

    # one after another on the default stream
    cur = torch.cuda.current_stream()
    ref = []
    for r in range(ROUNDS):
        ref.append(run_all(r, [cur, cur, cur]))
        torch.cuda.synchronize()
    # the same calls on three streams at once (default priority), interleaved
    streams = [torch.cuda.Stream() for _ in range(3)]
    for s in streams:
        s.wait_stream(cur)
    got = [run_all(r, streams) for r in range(ROUNDS)]
    torch.cuda.synchronize()
    for r in range(ROUNDS):
        for key in ("a", "b", "c", "d", "e"):
            for field, t in ref[r][key].items():
                assert torch.equal(got[r][key][field], t), (r, key, field)
    for p in (a, b, c, e):
        assert p.last_error() == 0
    assert bp.last_error() == 0
    # the fields are not trivially equal between rounds
    assert not torch.equal(ref[0]["a"]["S"], ref[1]["a"]["S"])
    assert np.isfinite(ref[0]["b"]["S"].cpu().numpy()).all()
