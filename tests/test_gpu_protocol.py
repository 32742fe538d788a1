"""The accuracy experiments of Sec. 6.1 run on the GPU (float64 path).

Example 1: 129 x 129 nodes at spacing 1/512 on [-0.125, 0.125]^2, 5000
distinct random nodes as sources, the percentage error of eq. percentError
over all nodes, maximum over trials compared with Table 2.  With the
validity threshold of the float64 FFT path (S_max ~ 29 tau here), the valid
band reaches (almost) every node only for tau >= 2e-4: those six of Table 2's
nine values are checked against the printed maxima, with the library's S as
reported (S_max at the rare nodes beyond the band, which the test counts).
tau = 1e-4 and 1.5e-4 run on the double-double path, whose band (~64 tau)
reaches the grid there.
From 3e-4 on (S_max >= 4.4 h) every node of every trial must be valid.  Example 2: 257 x 257 nodes at spacing 1/1024,
10000 sources, tau = 1e-4; the paper reports a mean error below 1.5 %.

The true distance R comes from a KD-tree query (scipy), the error from the
oracle's (pinned) metric, and one trial per case is checked node by node
against the oracle's direct sum.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_max_percent_error.json")
LO = -0.125
EX1 = dict(n=129, h=1.0 / 512, k=5000)
EX2 = dict(n=257, h=1.0 / 1024, k=10000)
FULL_BAND_TAUS = [2e-4, 2.5e-4, 3e-4, 3.5e-4, 4e-4, 4.5e-4]


@pytest.fixture(scope="module")
def dt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1112_3010_amd as dtm
    dtm.load_library()
    return dtm


def _nodes(n, h):
    c = LO + h * np.arange(n)
    xx, yy = np.meshgrid(c, c)
    return np.stack([xx.ravel(), yy.ravel()], axis=1)


def _plan(dt, ex, tau):
    n, h = ex["n"], ex["h"]
    # cell-centred nodes o + (i + 1/2) h land on LO + i h
    return dt.Plan((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, precision="fp64", outputs=["S"])


def _trial(ex, seed):
    from scipy.spatial import cKDTree
    Y = synth.generators.grid_node_subset(ex["n"], LO, ex["h"], ex["k"], seed)
    R, _ = cKDTree(Y.astype(np.float64)).query(_nodes(ex["n"], ex["h"]))
    return Y, R


def test_example1_trial_matches_oracle(dt):
    ex = EX1
    n, h = ex["n"], ex["h"]
    Y, R = _trial(ex, 6000)
    for tau in (2.5e-4, 4.5e-4):
        plan = _plan(dt, ex, tau)
        S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
        ref = parity.reference((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, Y, "fp64")
        assert np.all(ref["valid"])
        dS = np.abs(S - ref["S_exact"])
        assert np.all(dS <= parity.bound(ref, parity.TOL_S_TAU_FP64, tau))
        e_gpu, e_ref = oracle.percent_error(S, R), oracle.percent_error(ref["S_exact"], R)
        print(f"\n[example 1, tau {tau:g}] E gpu {e_gpu:.6f} % oracle {e_ref:.6f} %  max|dS|/tau {dS.max() / tau:.2e}")
        assert abs(e_gpu - e_ref) <= 1e-9 * e_ref


def test_example1_table2(dt):
    """Maximum percentage error over 100 trials per tau against Table 2 (the
    paper: 1000 trials), at the six tau whose valid band covers the grid."""
    with open(GOLDEN) as fh:
        g = json.load(fh)
    printed = dict(zip(g["tau"], g["max_percent_error"]))
    ex = EX1
    trials = [_trial(ex, 6000 + t) for t in range(100)]
    ratios, means = [], []
    for tau in FULL_BAND_TAUS:
        plan = _plan(dt, ex, tau)
        E, invalid = [], 0
        for Y, R in trials:
            S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
            invalid += int(np.sum(S >= plan.last_stats()["s_max"]))
            E.append(oracle.percent_error(S, R))
        if tau >= 3e-4:
            assert invalid == 0
        E = np.array(E)
        ratios.append(E.max() / printed[tau])
        means.append(E.mean())
        print(f"\n[table 2, tau {tau:g}] max E {E.max():.4f} % (printed {printed[tau]:.4f} %), mean {E.mean():.4f} %,"
              f" nodes beyond the band {invalid} of {len(trials) * len(trials[0][1])}")
    ratios = np.array(ratios)
    assert np.all(np.abs(ratios - 1.0) < 0.10), ratios
    # the error grows almost linearly with tau (the paper's observation)
    slope = np.array(means) / np.array(FULL_BAND_TAUS)
    assert slope.std() / slope.mean() < 0.15
    # below 2e-4 the float64 band no longer reaches every node
    plan = _plan(dt, ex, 1e-4)
    Y, _ = trials[0]
    S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().ravel()
    frac = float(np.mean(S < plan.last_stats()["s_max"]))
    print(f"\n[table 2, tau 1e-4] valid fraction {frac:.4f}")
    assert frac < 1.0


def test_example1_table2_extended_precision(dt):
    """Table 2 at tau = 1e-4 and 1.5e-4, where the float64 band (about 29 tau)
    stops short of the nodes farthest from the sources: the double-double
    path's band (about 64 tau, 3.3 h and 4.9 h here) reaches them.  Maximum
    percentage error over 100 trials against the printed maxima (+-10 %),
    nodes beyond the band counted (they report S_max)."""
    with open(GOLDEN) as fh:
        g = json.load(fh)
    printed = dict(zip(g["tau"], g["max_percent_error"]))
    ex = EX1
    n, h = ex["n"], ex["h"]
    trials = [_trial(ex, 6000 + t) for t in range(100)]
    for tau, max_invalid in ((1e-4, 50), (1.5e-4, 0)):
        plan = dt.Plan((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, precision="fp64x2", outputs=["S"])
        E, invalid = [], 0
        for Y, R in trials:
            S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
            invalid += int(np.sum(S >= plan.last_stats()["s_max"]))
            E.append(oracle.percent_error(S, R))
        E = np.array(E)
        s_max_h = plan.last_stats()["s_max"] / h
        print(f"\n[table 2 double-double, tau {tau:g}] max E {E.max():.4f} % (printed {printed[tau]:.4f} %), "
              f"mean {E.mean():.4f} %, S_max {s_max_h:.2f} h, nodes beyond the band {invalid} of "
              f"{len(trials) * len(trials[0][1])}")
        assert invalid <= max_invalid
        assert abs(E.max() / printed[tau] - 1.0) < 0.10
    # one trial node by node against the oracle's direct sum
    Y, R = trials[0]
    tau = 1.5e-4
    plan = dt.Plan((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, precision="fp64x2", outputs=["S"])
    S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
    ref = parity.reference((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, Y, "fp64x2", padded_dims=plan.padded)
    assert np.all(ref["valid"])
    dS = np.abs(S - ref["S_exact"])
    print(f"[table 2 double-double, tau {tau:g}] max|dS|/tau {dS.max() / tau:.2e}")
    assert np.all(dS <= parity.bound(ref, 1e-12, tau))


def test_example1_table2_quad_double(dt):
    """Table 2 at tau = 5e-5, the one tau that double-double does not reach:
    the nodes farthest from the sources sit about 3 h = 117 tau away, past
    double-double's band (about 64 tau); the quad-double path's band (about
    130 tau) reaches them.  Maximum percentage error over 100 trials against
    the printed maximum (+-10 %), nodes beyond the band counted; one trial
    node by node against the oracle's direct sum."""
    with open(GOLDEN) as fh:
        g = json.load(fh)
    printed = dict(zip(g["tau"], g["max_percent_error"]))
    ex = EX1
    n, h = ex["n"], ex["h"]
    tau = 5e-5
    plan = dt.Plan((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, precision="fp64x4", outputs=["S"])
    assert plan.precision == "fp64x4"
    E, invalid = [], 0
    trials = [_trial(ex, 6000 + t) for t in range(100)]
    for Y, R in trials:
        S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
        invalid += int(np.sum(S >= plan.last_stats()["s_max"]))
        E.append(oracle.percent_error(S, R))
    E = np.array(E)
    s_max_h = plan.last_stats()["s_max"] / h
    print(f"\n[table 2 quad-double, tau {tau:g}] max E {E.max():.4f} % (printed {printed[tau]:.4f} %), "
          f"mean {E.mean():.4f} %, S_max {s_max_h:.2f} h, nodes beyond the band {invalid} of "
          f"{len(trials) * len(trials[0][1])}")
    assert invalid <= 50
    assert abs(E.max() / printed[tau] - 1.0) < 0.10
    Y, R = trials[0]
    S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
    ref = parity.reference((n, n), (h, h), (LO - h / 2, LO - h / 2), tau, Y, "fp64x4", padded_dims=plan.padded)
    v = ref["valid"]
    dS = np.abs(S - ref["S_exact"])
    print(f"[table 2 quad-double, tau {tau:g}] max|dS|/tau {dS[v].max() / tau:.2e}, valid {v.mean():.6f}")
    assert np.all(dS[v] <= parity.bound(ref, 1e-12, tau)[v])


def test_example2_mean_error(dt):
    ex = EX2
    tau = 1e-4
    plan = _plan(dt, ex, tau)
    E, frac = [], []
    for t in range(20):
        Y, R = _trial(ex, 7000 + t)
        S = plan.distance(torch.from_numpy(Y).cuda()).cpu().numpy().astype(np.float64).ravel()
        E.append(oracle.percent_error(S, R))
        frac.append(np.mean(S < plan.last_stats()["s_max"]))
    print(f"\n[example 2] mean E {np.mean(E):.4f} % over 20 trials, valid fraction {np.mean(frac):.4f}")
    assert np.mean(E) < 1.5
