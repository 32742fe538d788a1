"""GPU parity of the batched 2D path (many instances per call): every
instance against the oracle with the batched padding rule, graph replay and
tile choices against the eager default (bitwise), and the 96-instance
workload on sampled nodes."""

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


SMALL_DIMS = [(97, 130), (128, 128), (37, 200), (250, 64), (500, 300), (12, 9), (64, 64)]
SMALL_K = [50, 200, 1, 0, 1500, 5, 40]


def _small_points():
    pts = []
    for i, (dims, K) in enumerate(zip(SMALL_DIMS, SMALL_K)):
        y = synth.generators.uniform_points(2, K, seed=900 + i) if K else np.zeros((0, 2), np.float32)
        pts.append(y)
    return pts


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _cells(dims, pts, n_uniform, n_near, seed):
    nx, ny = dims
    rng = np.random.default_rng(seed)
    a = rng.choice(nx * ny, min(n_uniform, nx * ny), replace=False)
    if len(pts) == 0:
        return np.unique(a)
    idx = np.floor(pts.astype(np.float64) * np.array([nx, ny])).astype(np.int64)
    pick = idx[rng.integers(0, len(idx), n_near)] + rng.integers(-4, 5, size=(n_near, 2))
    pick = np.clip(pick, 0, [nx - 1, ny - 1])
    return np.unique(np.concatenate([a, pick[:, 0] + nx * pick[:, 1]]))


def _check_instance(tag, prec, dims, tau, pts, S, G, cells, stats, Mp=None, theta_rel=1e-9):
    nx, ny = dims
    h = (1.0 / nx, 1.0 / ny)
    if len(pts) == 0:
        assert np.all(np.isinf(S)) and np.all(S > 0), tag
        assert np.all(G == 0), tag
        return
    if Mp is None:
        Mp = (parity.batch_padded(nx), parity.batch_padded(ny))
    ref = parity.reference(dims, h, (0.0, 0.0), tau, pts, prec, grad=True, cells=cells, padded_dims=Mp)
    assert stats["theta"] == pytest.approx(ref["theta"], rel=theta_rel), tag
    S = S.ravel()[cells] if cells is not None else S.ravel()
    g = G.reshape(2, -1)[:, cells] if cells is not None else G.reshape(2, -1)
    dS = np.abs(S - ref["S_ref"])
    deep = ref["deep"]
    dG = np.abs(g - ref["grad"].T)[:, deep]
    msg = f"[{tag} {prec}] max|dS|/tau={dS.max() / tau:.3e} max|dgrad|={dG.max() if dG.size else 0:.3e}"
    assert dS.max() <= parity.TOL_S_TAU * tau, msg
    if dG.size:
        assert dG.max() <= parity.TOL_GRAD, msg
    if prec == "fp64":
        assert np.all(dS[deep] <= parity.bound(ref, parity.TOL_S_TAU_FP64, tau)[deep]), msg
        assert np.all(dG <= parity.bound(ref, parity.TOL_GRAD_FP64)[deep]), msg
    inval = ~ref["valid"] & (ref["S_exact"] > ref["s_max"] + 0.05 * tau)
    assert np.all(g[:, inval] == 0), msg
    return msg


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_small_against_oracle(dt, prec):
    pts = _small_points()
    taus = [2.0 / d[0] for d in SMALL_DIMS]
    plan = dt.BatchPlan(SMALL_DIMS, taus, precision=prec, graph=False)
    for i, (nx, ny) in enumerate(SMALL_DIMS):
        assert plan.padded(i) == (parity.batch_padded(nx), parity.batch_padded(ny))
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    S, G = plan.forward(Y.cuda(), offs)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    for i, (dims, tau) in enumerate(zip(SMALL_DIMS, taus)):
        s, g = plan.views(S, G)[i]
        cells = None if dims[0] * dims[1] <= 40000 else _cells(dims, pts[i], 2000, 2000, 950 + i)
        msg = _check_instance(f"inst {i} {dims} K={len(pts[i])}", prec, dims, tau, pts[i], _np(s), _np(g), cells,
                              plan.stats(i))
        if msg:
            print("\n" + msg, flush=True)


def test_batch_graph_replay_and_tiles_bitwise(dt):
    pts = _small_points()
    taus = [2.0 / d[0] for d in SMALL_DIMS]
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    Y = Y.cuda()
    plan = dt.BatchPlan(SMALL_DIMS, taus, precision="fp32", graph=False)
    S0, G0 = plan.forward(Y, offs)
    torch.cuda.synchronize()
    # tile choices change only which block handles which rows / kx bins
    for t in [(1, 256, 128), (4, 512, 512), (16, 512, 256), (2, 1024, 64)]:
        plan.set_tiles(*t)
        S1, G1 = plan.forward(Y, offs)
        torch.cuda.synchronize()
        assert torch.equal(S1, S0) and torch.equal(G1, G0), t
    # graph replays, with eager work and synchronisation between them
    plan.set_graph(True)
    S2, G2 = plan.empty_outputs()
    for rep in range(4):
        plan.forward_into(Y, offs, S2, G2)
        junk = (S0 * 2.0).sum()
        torch.cuda.synchronize()
        assert torch.equal(S2, S0) and torch.equal(G2, G0), rep
        S2.fill_(-1.0)
        G2.fill_(-1.0)
        del junk
    # a new output buffer makes a new graph
    S3, G3 = plan.forward(Y, offs)
    torch.cuda.synchronize()
    assert torch.equal(S3, S0) and torch.equal(G3, G0)
    assert plan.last_error() == 0


def test_batch_out_of_grid_source(dt):
    dims = [(64, 48), (40, 40)]
    pts = [synth.generators.uniform_points(2, 30, seed=960), synth.generators.uniform_points(2, 20, seed=961)]
    bad = np.concatenate([pts[1], np.array([[1.5, 0.5]], np.float32)])
    plan = dt.BatchPlan(dims, [2.0 / 64, 2.0 / 40], precision="fp64", graph=False)
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(pts[0]), torch.from_numpy(bad)])
    S, G = plan.forward(Y.cuda(), offs)
    torch.cuda.synchronize()
    assert plan.last_error() == 2
    assert plan.last_error() == 0
    for i in range(2):
        s, g = plan.views(S, G)[i]
        _check_instance(f"inst {i}", "fp64", dims[i], 2.0 / dims[i][0], pts[i], _np(s), _np(g), None, plan.stats(i))


def test_batch_96_instances(dt):
    inst = synth.workload("c4_batch_2d").extra["instances"]
    dims = [(n, n) for n, _ in inst]
    taus = [2.0 / n for n, _ in inst]
    plan = dt.BatchPlan(dims, taus, precision="fp32", graph=True)
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(y) for _, y in inst])
    Y = Y.cuda()
    S, G = plan.forward(Y, offs)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    # tiles and radix schedules tuned on this batch: the schedules change the
    # order of the radix stages, so the tuned results are checked against the
    # oracle as well
    tuned = plan.autotune(Y, offs, reps=1, cache=False)
    S1, G1 = plan.forward(Y, offs)
    torch.cuda.synchronize()
    sched = np.array(plan.schedule())
    assert sched.shape == (len(inst), 3) and sched.min() >= 0 and sched.max() <= 5
    assert tuned["schedule"] == sched.tolist()
    # instances of one padded length share each pass's schedule
    for k, lens in ((0, [plan.padded(i)[0] for i in range(len(inst))]), (1, [plan.padded(i)[1] for i in
                                                                              range(len(inst))])):
        by = {}
        for i, L in enumerate(lens):
            by.setdefault(L, set()).add(int(sched[i, k]))
        assert all(len(v) == 1 for v in by.values())
    for i, ((n, y), tau) in enumerate(zip(inst, taus)):
        cells = _cells((n, n), y, 250, 250, 970 + i)
        for tag, (s, g), st in (("default", plan.views(S, G)[i], None), ("tuned", plan.views(S1, G1)[i], None)):
            _check_instance(f"c4 inst {i} n={n} K={len(y)} {tag}", "fp32", (n, n), tau, y, _np(s), _np(g), cells,
                            plan.stats(i))
    fams = np.bincount(sched.ravel(), minlength=6).tolist()
    print(f"\n[batch 96] tuned tiles {dict((k, v) for k, v in tuned.items() if k != 'schedule')}, "
          f"schedule families used {fams}; all instances within tolerance on about 500 nodes each", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_every_radix_schedule(dt, prec, tmp_path, monkeypatch):
    """Each of the six radix schedules (four orders of the prime-power
    radices, two with fused radices), on every pass of every instance, gives
    the transform (checked against the oracle); the schedule round-trips
    through the tuning cache."""
    pts = _small_points()
    taus = [2.0 / d[0] for d in SMALL_DIMS]
    plan = dt.BatchPlan(SMALL_DIMS, taus, precision=prec, graph=False)
    assert plan.schedule() == [[4, 4, 4]] * len(SMALL_DIMS)
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    Y = Y.cuda()
    for fam in range(6):
        mix = [[fam, (fam + i) % 6, (fam + 2 * i) % 6] for i in range(len(SMALL_DIMS))]
        plan.set_schedule(mix)
        assert plan.schedule() == mix
        S, G = plan.forward(Y, offs)
        torch.cuda.synchronize()
        assert plan.last_error() == 0
        for i, (dims, tau) in enumerate(zip(SMALL_DIMS, taus)):
            s, g = plan.views(S, G)[i]
            cells = None if dims[0] * dims[1] <= 40000 else _cells(dims, pts[i], 1000, 1000, 990 + i)
            _check_instance(f"schedule {mix[i]} inst {i}", prec, dims, tau, pts[i], _np(s), _np(g), cells,
                            plan.stats(i))
    with pytest.raises(RuntimeError):
        plan.set_schedule([[0, 6, 0]] + [[0, 0, 0]] * (len(SMALL_DIMS) - 1))
    assert plan.schedule() == mix
    # autotune writes tiles and schedule to the cache; a new plan restores both
    monkeypatch.setenv("DT_TUNE_CACHE", str(tmp_path / "tiles.json"))
    tuned = plan.autotune(Y, offs, reps=1, cache=True)
    S1, G1 = plan.forward(Y, offs)
    plan2 = dt.BatchPlan(SMALL_DIMS, taus, precision=prec, graph=False)
    again = plan2.autotune(Y, offs, reps=1, cache=True)
    assert again == tuned
    assert plan2.schedule() == tuned["schedule"] == plan.schedule()
    S2, G2 = plan2.forward(Y, offs)
    torch.cuda.synchronize()
    assert torch.equal(S2, S1) and torch.equal(G2, G1)


# Lengths whose fused schedules use the fused radices the every-schedule
# test leaves out, and the fallbacks: rows 27 (9, 3), 45 (15, 3), 63 (7, 9),
# 28 (4, 7), 245 (7, 7, 5); columns 144 (16, 9), 336 (16, 7, 3), 560
# (16, 7, 5), 28 (4, 7), 200 (8, 5, 5).
FUSED_DIMS = [(27, 72), (45, 168), (63, 280), (28, 14), (245, 100)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_fused_radices(dt, prec):
    """Schedules 4 and 5 (fused radices, powers of two first or last) on
    every pass of lengths that use 9 and 15 and the leftover rules (the
    every-schedule test covers 6, 10, 12, 14, 15, 16): every node against the
    oracle."""
    pts = [synth.generators.uniform_points(2, 40 + 10 * i, seed=970 + i) for i in range(len(FUSED_DIMS))]
    taus = [2.0 / d[0] for d in FUSED_DIMS]
    plan = dt.BatchPlan(FUSED_DIMS, taus, precision=prec, graph=False)
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    Y = Y.cuda()
    for fam in (4, 5):
        plan.set_schedule([[fam, fam, fam]] * len(FUSED_DIMS))
        S, G = plan.forward(Y, offs)
        torch.cuda.synchronize()
        assert plan.last_error() == 0
        for i, (dims, tau) in enumerate(zip(FUSED_DIMS, taus)):
            s, g = plan.views(S, G)[i]
            _check_instance(f"fused schedule {fam} inst {i} {dims}", prec, dims, tau, pts[i], _np(s), _np(g), None,
                            plan.stats(i))


RED_DIMS = [(300, 300), (200, 260), (128, 96), (90, 400)]
RED_K = [500, 100, 40, 200]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_reduced_padding_against_oracle(dt, prec):
    """k_max = K per instance: smaller padded grids and kernels truncated to
    the box the padding leaves wrap-free; every node against the exact
    (untruncated) oracle with the reduced grid's threshold."""
    pts = [synth.generators.uniform_points(2, K, seed=950 + i) for i, K in enumerate(RED_K)]
    taus = [2.0 / d[0] for d in RED_DIMS]
    plan = dt.BatchPlan(RED_DIMS, taus, precision=prec, graph=False, k_max=RED_K)
    Mps, truncated = [], 0
    for i, dims in enumerate(RED_DIMS):
        Mp, cut = parity.batch_padded_reduced(dims, (1.0 / dims[0], 1.0 / dims[1]), taus[i], RED_K[i], prec)
        assert plan.padded(i) == Mp
        truncated += any(cut)
        Mps.append(Mp)
    assert truncated >= 3, "the case must exercise truncation"
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    S, G = plan.forward(Y.cuda(), offs)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    for i, ((Si, Gi), dims) in enumerate(zip(plan.views(S, G), RED_DIMS)):
        # Theta: the truncated kernel's l1 norm lacks the tail beyond the box
        # (about 1e-9 relative here); the oracle's is the untruncated sum
        msg = _check_instance(f"reduced {i} {dims} M={Mps[i]}", prec, dims, taus[i], pts[i], _np(Si), _np(Gi), None,
                              plan.stats(i), Mp=Mps[i], theta_rel=1e-7)
        print("\n" + msg)
    # more sources than k_max in an instance is refused
    more = [synth.generators.uniform_points(2, K + (1 if i == 1 else 0), seed=950 + i) for i, K in enumerate(RED_K)]
    Y2, offs2 = dt.BatchPlan.pack([torch.from_numpy(p) for p in more])
    with pytest.raises(RuntimeError):
        plan.forward(Y2.cuda(), offs2)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_single_sources_closed_form(dt, prec):
    """One source per instance on uneven grids (7-smooth padding): S = r and
    grad S = (X - Y)/r on every deep node, S_max and a zero gradient beyond the
    band, without the oracle.  Sources lie exactly on nodes (cell centres);
    positions are measured from the first node, x fastest."""
    dims = [(97, 130), (250, 64), (37, 200), (128, 128)]
    nodes = [(40, 71), (201, 30), (18, 150), (64, 10)]
    taus = [2.0 / max(d) for d in dims]
    pts = [np.array([[(nd[0] + 0.5) / d[0], (nd[1] + 0.5) / d[1]]], dtype=np.float32) for d, nd in zip(dims, nodes)]
    plan = dt.BatchPlan(dims, taus, precision=prec, graph=False)
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(p) for p in pts])
    S, G = plan.forward(Y.cuda(), offs)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    for i, ((nx, ny), nd, tau) in enumerate(zip(dims, nodes, taus)):
        s, g = plan.views(S, G)[i]
        s, g = _np(s).ravel(), _np(g).reshape(2, -1)
        s_max = plan.stats(i)["s_max"]
        yy, xx = np.meshgrid(np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
        d = np.stack([xx.ravel() - nd[0] / nx, yy.ravel() - nd[1] / ny])
        r = np.sqrt((d ** 2).sum(axis=0))
        deep = r <= s_max - tau * np.log(2.0)
        far = r >= s_max + 0.05 * tau
        assert deep.sum() > 100 and far.sum() > 100
        with np.errstate(invalid="ignore", divide="ignore"):
            n = np.where(r > 0, d / r, 0.0)
        dS = np.abs(s - r)[deep]
        dG = np.abs(g - n)[:, deep]
        print(f"\n[batch single source {i} {(nx, ny)} {prec}] S_max/tau={s_max / tau:.2f} "
              f"max|S-r|/tau={dS.max() / tau:.3e} max|dgrad|={dG.max():.3e}")
        if prec == "fp32":
            assert dS.max() <= parity.TOL_S_TAU * tau
            assert dG.max() <= parity.TOL_GRAD
        else:
            b = parity.TOL_THETA_FRAC * np.exp((r[deep] - s_max) / tau)   # Theta/phi for one source
            assert np.all(dS <= tau * (parity.TOL_S_TAU_FP64 + b))
            assert np.all(dG <= parity.TOL_GRAD_FP64 + b)
        smax_t = float(np.float32(s_max)) if prec == "fp32" else s_max
        assert np.all(s[far] == smax_t)
        assert np.all(g[:, far] == 0)
