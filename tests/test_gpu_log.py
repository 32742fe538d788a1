"""The plan log's device-side lines (DT_LOG): the attach line reports
||f||_1 and the one-source threshold that dt_plan_info and the validity
contract give, and the per-call line the threshold of the last call."""

import math
import re

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


def _num(pattern, text):
    m = re.search(pattern, text)
    assert m, (pattern, text)
    return float(m.group(1))


def test_single_plan_log(dt, capfd, monkeypatch):
    monkeypatch.setenv("DT_LOG", "1")
    dims = (96, 80)
    tau = 2.0 / 96
    plan = dt.Plan(dims, (1.0 / 96, 1.0 / 80), None, tau, precision="fp64", outputs=["S", "grad"])
    pts = synth.generators.uniform_points(2, 40, seed=17)
    plan.gradient(torch.from_numpy(pts).cuda())
    st = plan.last_stats()
    out = capfd.readouterr().err
    l1 = _num(r"attached: \|\|f\|\|_1 = ([0-9.eE+-]+)", out)
    assert l1 == pytest.approx(plan._info().kernel_l1, rel=1e-8)
    M = plan.padded
    npad = float(np.prod(M))
    theta1 = 256 * 2.0 ** -53 * math.log2(npad) * l1 / math.sqrt(npad)
    assert _num(r"one source: Theta = ([0-9.eE+-]+)", out) == pytest.approx(theta1, rel=1e-3)
    assert _num(r"last call: \|\|g\|\|_2 = ([0-9.eE+-]+)", out) == pytest.approx(st["g_l2"], rel=1e-5)
    assert _num(r"last call: .* Theta = ([0-9.eE+-]+)", out) == pytest.approx(st["theta"], rel=1e-3)
    assert _num(r"S_max = ([0-9.]+) tau, error bits", out) == pytest.approx(st["s_max"] / tau, rel=1e-3)


def test_batch_plan_log(dt, capfd, monkeypatch):
    monkeypatch.setenv("DT_LOG", "1")
    dims = [(97, 130), (64, 64)]
    plan = dt.BatchPlan(dims, [2.0 / d[0] for d in dims], precision="fp32", graph=False)
    out = capfd.readouterr().err
    assert "batch plan" in out and "blocks: tiles col_nb" in out
    for i in range(2):
        assert f"inst {i}: schedule families 4/4/4, radices rows" in out
        l1 = _num(rf"inst {i}: \|\|f\|\|_1 = ([0-9.eE+-]+)", out)
        assert l1 == pytest.approx(plan.kernel_l1(i), rel=1e-8)
