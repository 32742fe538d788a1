"""Throughput of the distance-field hot path on one MI355X.

Default workload (the headline metric): 3D grid 256^3 on [0,1]^3 (h = 1/256,
padded to 512^3), sources = the 60 000 snapped triangle incenters of a
closed mesh (a sphere perturbed by random spherical harmonics of degree
1-6, amplitude 0.1, scaled to 0.8 of the box), tau = h, outputs S and grad S.
One step = one dt_forward call (splat -> FFT passes -> epilogue) with the
mesh already resident in device memory.  The float32-with-scaling path is
the headline value; the float64 path is reported beside it.

Prints one JSON line with the metric (mean over the timed calls, with their
median, minimum and 90th percentile), a roofline entry for the dominant
kernel (algorithmic bytes per launch over its average duration, measured
with HIP events on the launch stream), the GPU clocks and power cap, and a
CPU baseline (the FP64 oracle on a bounded sample of grid nodes of the same
workload, on the host's cores).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid pts/s for S+∇S at 256^3: FP64 plain vs FP32-scaled; % HBM roofline"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters_3d_256.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(dims, Mp, w, c_in, c_out, n_tab, out_fields):
    """Algorithmic HBM bytes per launch of each pass (each array read or
    written once; kernel tables counted once at their folded size)."""
    D = len(dims)
    nx, ny = dims[0], dims[1]
    nz = dims[2] if D == 3 else 1
    Mx, My = Mp[0], Mp[1]
    Mz = Mp[2] if D == 3 else 1
    Mh = Mx // 2 + 1
    cs = 2 * w
    N = nx * ny * nz
    tab = n_tab * Mh * (My // 2 + 1) * ((Mz // 2 + 1) if D == 3 else 1) * w
    b = {
        "fill": c_in * N * w,
        # reads the splat's sum of squared multiplicities, writes Theta, S_max, ||g||_2
        "validity": 4 * 8,
        "row_r2c": c_in * N * w + c_in * ny * nz * Mh * cs,
    }
    if D == 3:
        b["col_fwd_y"] = c_in * nz * ny * Mh * cs + c_in * nz * My * Mh * cs
        b["col_fused"] = c_in * nz * My * Mh * cs + tab + c_out * nz * My * Mh * cs
        b["col_inv_y"] = c_out * nz * My * Mh * cs + c_out * nz * ny * Mh * cs
    else:
        b["col_fused"] = c_in * ny * Mh * cs + tab + c_out * ny * Mh * cs
    b["row_c2r_epi"] = c_out * nz * ny * Mh * cs + out_fields * N * w
    return b


def counters_for(kernel_file_hash, precision, pass_name):
    """HBM bytes of one call's launches of a pass (calibrated FETCH_SIZE +
    WRITE_SIZE, summed over the pass's launches in one call) measured by
    rocprofv3 for the current kernel sources, else None.  The summary file
    holds lines `sources <sha256>` and `<precision> <pass> fetch=<B> write=<B>`."""
    try:
        lines = open(COUNTERS).read().splitlines()
    except OSError:
        return None
    src = None
    for ln in lines:
        f = ln.split()
        if len(f) == 2 and f[0] == "sources":
            src = f[1]
        if src == kernel_file_hash and len(f) >= 4 and f[0] == precision and f[1] == pass_name:
            kv = dict(x.split("=") for x in f[2:])
            return int(kv["fetch"]) + int(kv["write"])
    return None


# sources of the double-double pipeline only (no float32/float64 launch uses them)
DD_SOURCES = ("dd.hpp", "qd.hpp", "dt_dd.hpp", "k_dd.hip")
# sources of the batched 2D path and of the fixed workspace only (the 3D
# passes of the headline workload do not use them)
OTHER_SOURCES = ("batch.cpp", "dt_batch.hpp", "fft_mixed.hpp", "k_batch.hip", "k_static_ws.hip", "dt_static.hpp")


def kernel_hash(include_dd=False):
    """Hash of the kernel and host sources that build the single-grid passes
    (without the double-double pipeline's own files unless include_dd, and
    without the batched path's)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1112_3010_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if (f in DD_SOURCES and not include_dd) or f in OTHER_SOURCES:
            continue
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def per_call(per, calls):
    """Per-pass time and launch count per call from the library's timings
    (a pass may run as several launches per call)."""
    ms = {k: v[1] / calls for k, v in per.items() if v[0] > 0}
    launches = {k: v[0] / calls for k, v in per.items() if v[0] > 0}
    return ms, launches


def roofline_entry(nbytes, ms, launches, dom, traffic=None):
    """Roofline of the dominant pass: its algorithmic bytes per call over its
    time per call (the same ratio as bytes per launch over the average launch
    duration)."""
    gbs = nbytes[dom] / (ms[dom] * 1e-3) / 1e9
    per_launch = None if traffic is None else int(round(traffic / launches[dom]))
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": per_launch, "kernel": dom,
            "bytes_per_launch": int(round(nbytes[dom] / launches[dom])), "launches_per_call": launches[dom],
            "avg_launch_us": round(1e3 * ms[dom] / launches[dom], 2)}


def timed_calls(fn, steps):
    """Run fn() `steps` times on the current stream with an event between
    consecutive calls.  Returns (mean ms per call over the whole span,
    {"median", "min", "p90"} of the per-call durations)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    mean = ev[0].elapsed_time(ev[-1]) / steps
    return mean, {"median": round(float(np.median(per)), 4), "min": round(float(per.min()), 4),
                  "p90": round(float(np.percentile(per, 90)), 4)}


def gpu_clocks():
    """Current SCLK/MCLK levels and the power cap of the GPUs, read from the
    amdgpu driver's sysfs files (plain reads: no other program is started)."""
    import glob
    out = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        card = dev.split("/")[-2]
        info = {}
        for name in ("pp_dpm_sclk", "pp_dpm_mclk"):
            try:
                cur = [ln.strip() for ln in open(os.path.join(dev, name)) if ln.strip().endswith("*")]
                info[name] = cur[0] if cur else None
            except OSError:
                pass
        for cap in glob.glob(os.path.join(dev, "hwmon", "hwmon*", "power1_cap")):
            try:
                info["power_cap_w"] = int(open(cap).read()) / 1e6
            except (OSError, ValueError):
                pass
        if info:
            out[card] = info
    return out or None


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sample_cells(dims, n_cells, seed=0):
    """Random node sample shared by the CPU baseline and the accuracy report."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(dims)), n_cells, replace=False))


def run_gpu(prec, V, F, dims, tau, steps, warmup, timing_calls, cells=None, k_max=None):
    import torch
    import paper_1112_3010_amd as dt
    t0 = time.time()
    plan = dt.Plan(dims, None, None, tau, precision=prec, outputs=["S", "grad"], k_max=k_max)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    # the kernel spectra alone (what a new tau costs once the workspace exists)
    tab_s = []
    for _ in range(3):
        t0 = time.time()
        plan.rebuild()
        torch.cuda.synchronize()
        tab_s.append(time.time() - t0)
    Vd = torch.from_numpy(V).cuda()
    Fd = torch.from_numpy(F).cuda()
    out = {"S": plan._empty(), "grad": plan._empty(len(dims))}
    for _ in range(warmup):
        plan.forward_into(out, vertices=Vd, faces=Fd)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ms, ms_stats = timed_calls(lambda: plan.forward_into(out, vertices=Vd, faces=Fd), steps)
    # per-pass timing in a separate set of calls (events inside the library)
    plan.set_timing(True)
    plan.timings(reset=True)
    for _ in range(timing_calls):
        plan.forward_into(out, vertices=Vd, faces=Fd)
    per = plan.timings(reset=True)
    plan.set_timing(False)
    stats = plan.last_stats()
    w = 8 if prec == "fp64" else 4
    Mp = plan.padded
    nbytes = pass_bytes(dims, Mp, w, c_in=1, c_out=1 + len(dims), n_tab=1 + len(dims), out_fields=1 + len(dims))
    avg, launches = per_call(per, timing_calls)
    dom = max((k for k in avg if k in nbytes), key=lambda k: avg[k])
    achieved = nbytes[dom] / (avg[dom] * 1e-3) / 1e9
    total_model = sum(nbytes.values())
    N = int(np.prod(dims))
    res = {
        "value": N / (ms * 1e-3),
        "ms_per_step": ms,
        "ms_stats": ms_stats,
        "plan_setup_s": plan_s,
        "plan_tables_s": float(np.median(tab_s)),
        "dominant": dom,
        "achieved": achieved,
        "pass_ms": {k: round(v, 4) for k, v in avg.items()},
        "pass_gbs": {k: round(nbytes[k] / (avg[k] * 1e-3) / 1e9, 1) for k in avg if k in nbytes},
        "dom_bytes": nbytes[dom],
        "launches": launches,
        "model_bytes": total_model,
        "pass_bytes": nbytes,
        "path_gbs": total_model / (ms * 1e-3) / 1e9,
        "s_max_over_tau": stats["s_max"] / tau,
        "padded": list(Mp),
        "cut": list(plan.cut),
    }
    if cells is not None:
        idx = torch.from_numpy(cells).cuda()
        res["sample_S"] = out["S"].reshape(-1)[idx].double().cpu().numpy()
        res["sample_grad"] = out["grad"].reshape(len(dims), -1)[:, idx].double().cpu().numpy().T
    del plan
    torch.cuda.empty_cache()
    return res


def triangle_centres(V, F):
    """Incenters of the mesh triangles (float32, K x 3): the sources of the
    backward workload, given to dt_backward as points."""
    V = np.asarray(V, dtype=np.float64)
    v0, v1, v2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    a = np.linalg.norm(v1 - v2, axis=1)[:, None]
    b = np.linalg.norm(v2 - v0, axis=1)[:, None]
    c = np.linalg.norm(v0 - v1, axis=1)[:, None]
    return ((a * v0 + b * v1 + c * v2) / (a + b + c)).astype(np.float32)


def backward_bytes(dims, Mp, w, K):
    """Algorithmic HBM bytes per launch of the backward passes (dL/dY and
    dL/dtau): the forward transform of w = G e^(S/tau), the products with the
    D gradient kernels and the r f kernel, and the gather at the K sources."""
    D = len(dims)
    b = pass_bytes(dims, Mp, w, c_in=1, c_out=D + 1, n_tab=D + 1, out_fields=0)
    del b["row_c2r_epi"]
    N = int(np.prod(dims))
    Mh = Mp[0] // 2 + 1
    b["prep_w"] = 3 * N * w
    b["gather"] = K * (D + 1) * Mh * 2 * w + K * D * 4
    return b


def run_backward(prec, Y, dims, tau, steps, warmup, timing_calls, k_max=None):
    """Time dt_backward on the 256^3 grid with the mesh's triangle centres as
    sources and dL/dS = S (the loss S^2 / 2)."""
    import torch
    import paper_1112_3010_amd as dt
    plan = dt.Plan(dims, None, None, tau, precision=prec, outputs=["S", "backward"], k_max=k_max)
    Yd = torch.from_numpy(Y).cuda()
    S = plan.distance(Yd)
    G = S.clone()
    for _ in range(warmup):
        plan.backward(Yd, S, G)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ms, ms_stats = timed_calls(lambda: plan.backward(Yd, S, G), steps)
    plan.set_timing(True)
    plan.timings(reset=True)
    for _ in range(timing_calls):
        plan.backward(Yd, S, G)
    per = plan.timings(reset=True)
    plan.set_timing(False)
    w = 8 if prec == "fp64" else 4
    nbytes = backward_bytes(dims, plan.padded, w, len(Y))
    avg, launches = per_call(per, timing_calls)
    dom = max((k for k in avg if k in nbytes), key=lambda k: avg[k])
    total = sum(nbytes.values())
    N = int(np.prod(dims))
    res = {"value": round(N / (ms * 1e-3), 1), "unit": "grid pts/s", "ms_per_call": round(ms, 4),
           "ms_stats": ms_stats, "sources": len(Y), "padded": list(plan.padded),
           "roofline": roofline_entry(nbytes, avg, launches, dom),
           "path": {"model_bytes": total, "achieved_gbs": round(total / (ms * 1e-3) / 1e9, 1),
                    "frac": round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "pass_ms": {k: round(v, 4) for k, v in avg.items()},
                    "pass_gbs": {k: round(nbytes[k] / (avg[k] * 1e-3) / 1e9, 1) for k in avg if k in nbytes}}}
    del plan
    torch.cuda.empty_cache()
    return res


def run_curvature(prec, Y, dims, tau, steps, warmup, timing_calls):
    """Time dt_forward with S and the curvature outputs (mean, Gaussian, k1,
    k2) on the 256^3 grid: the gradient and Hessian channels (1 + D + D(D+1)/2
    output channels through the fused pass) and the curvature epilogue."""
    import torch
    import paper_1112_3010_amd as dt
    plan = dt.Plan(dims, None, None, tau, precision=prec, outputs=["S", "curv"])
    Yd = torch.from_numpy(Y).cuda()
    out = {"S": plan._empty(), "curv": plan._empty(4)}
    for _ in range(warmup):
        plan.forward_into(out, Yd)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.forward_into(out, Yd)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.set_timing(True)
    plan.timings(reset=True)
    for _ in range(timing_calls):
        plan.forward_into(out, Yd)
    per = plan.timings(reset=True)
    plan.set_timing(False)
    D = len(dims)
    C = 1 + D + D * (D + 1) // 2
    w = 8 if prec == "fp64" else 4
    nbytes = pass_bytes(dims, plan.padded, w, c_in=1, c_out=C, n_tab=C, out_fields=5)
    avg, launches = per_call(per, timing_calls)
    dom = max((k for k in avg if k in nbytes), key=lambda k: avg[k])
    total = sum(nbytes.values())
    N = int(np.prod(dims))
    res = {"value": round(N / (ms * 1e-3), 1), "unit": "grid pts/s", "ms_per_call": round(ms, 4),
           "outputs": "S + mean, Gaussian, k1, k2 (10 channels)",
           "roofline": roofline_entry(nbytes, avg, launches, dom),
           "path": {"model_bytes": total, "achieved_gbs": round(total / (ms * 1e-3) / 1e9, 1),
                    "frac": round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "pass_ms": {k: round(v, 4) for k, v in avg.items()}}}
    del plan, out
    torch.cuda.empty_cache()
    return res


def cpu_baseline(V, F, dims, tau, cells, gpu_results=()):
    """The oracle (FP64 direct sums, S and grad S) on a bounded random sample
    of nodes of the same workload, on the host's cores (one oracle thread per
    core available to this process, at most 16; NumPy's BLAS pool held at one
    thread so the threads do not oversubscribe).  Its fields also give the GPU
    results' errors on that sample: |S - min(S_exact, S_max)| on every sampled
    node, the gradient on nodes with phi >= 2 Theta."""
    import oracle
    from threadpoolctl import threadpool_limits
    inc, _ = oracle.mesh_sources(V, F)
    h = tuple(1.0 / n for n in dims)
    o = (0.0,) * len(dims)
    idx, valid = oracle.sign.snap_f64(inc, o, h, dims)
    Yh = oracle.node_coords(idx[valid], o, h)
    X = oracle.grid_nodes(dims, o, h, cells)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        f = oracle.fields(X, Yh, tau, grad=True, workers=workers)
        dt_s = time.perf_counter() - t0
    out = {"value": len(cells) / dt_s, "unit": "grid pts/s", "cores": workers, "kind": "oracle",
           "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
           "sample": f"{len(cells)} random nodes of the {'x'.join(str(n) for n in dims)} grid, all "
                     f"{int(valid.sum())} sources each, S and grad S in float64 on {workers} threads ({dt_s:.1f} s)"}
    _, mult = oracle.cell_multiplicities(idx[valid], dims)
    g_l2 = float(np.sqrt(np.sum(mult.astype(np.float64) ** 2)))
    acc = {}
    for label, prec, r in gpu_results:
        if r is None or "sample_S" not in r:
            continue
        # the threshold of the grid the GPU result was computed on
        Mp = tuple(r["padded"])
        th = oracle.theta(prec, Mp, oracle.kernel_l1(Mp, h, tau), g_l2)
        s_ref = np.minimum(f["S"], oracle.s_max(tau, th))
        deep = f["lnphi"] >= np.log(2.0 * th)
        eS = np.abs(r["sample_S"] - s_ref)
        eG = np.abs(r["sample_grad"] - f["grad"])[deep]
        acc[label] = {"max_abs_S_over_tau": float(eS.max() / tau),
                     "max_abs_S_over_tau_deep": float(eS[deep].max() / tau) if deep.any() else None,
                     "max_abs_grad_deep": float(eG.max()) if eG.size else None,
                     "deep_nodes": int(deep.sum()), "s_max_over_tau": oracle.s_max(tau, th) / tau}
    return out, acc


def batch_bytes(dims, padded, w, C):
    """Algorithmic HBM bytes of one batched call (S and grad S) for the given
    padded sizes: each array read or written once, kernel tables at their
    folded size."""
    total = 0
    for (nx, ny), (Mx, My) in zip(dims, padded):
        sx = Mx // 2
        N = nx * ny
        spec = ny * (sx + 1) * 2 * w
        total += N * w                                   # fill
        total += N * w + spec                            # row_r2c
        total += spec + C * (My // 2 + 1) * (sx + 1) * w + C * spec   # col_fused
        total += C * spec + C * N * w                    # row_c2r_epi (S + 2 gradient fields)
    return total


def run_protocol(trials):
    """Example 1 of Sec. 6.1 on the float64 path: 129 x 129 nodes at spacing
    1/512 on [-0.125, 0.125]^2, 5000 distinct random nodes per trial, the
    nine tau of Table 2; the three smallest again in double-double and
    quad-double.  Timed: the dt_distance calls with the points on the
    device.  Reported per tau: max and mean percentage error over the trials
    (true distance by KD-tree) and the fraction of nodes inside the valid
    band.  A 2D grid of this size is cache-resident: no roofline claim."""
    import torch
    from scipy.spatial import cKDTree
    import paper_1112_3010_amd as dt
    import synth
    n, h, lo, k = 129, 1.0 / 512, -0.125, 5000
    c = lo + h * np.arange(n)
    xx, yy = np.meshgrid(c, c)
    X = np.stack([xx.ravel(), yy.ravel()], axis=1)
    pts, Rs = [], []
    for t in range(trials):
        Y = synth.generators.grid_node_subset(n, lo, h, k, 6000 + t)
        pts.append(torch.from_numpy(Y).cuda())
        Rs.append(cKDTree(Y.astype(np.float64)).query(X)[0])
    printed = [0.5728, 1.1482, 1.7461, 2.4046, 3.1550, 4.0146, 4.9959, 6.1033, 7.3380]   # Table 2
    taus = [5e-5 * (i + 1) for i in range(9)]

    def run_tau(tau, pr, precision):
        plan = dt.Plan((n, n), (h, h), (lo - h / 2, lo - h / 2), tau, precision=precision, outputs=["S"])
        S = plan._empty()
        for Yd in pts[:3]:
            plan.distance_into(S, Yd)
        torch.cuda.synchronize()
        outs = [plan._empty() for _ in pts]
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for Yd, o in zip(pts, outs):
            plan.distance_into(o, Yd)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        smax = plan.last_stats()["s_max"]
        E, valid = [], []
        for o, R in zip(outs, Rs):
            Sv = o.cpu().numpy().astype(np.float64).ravel()
            keep = R > 0
            E.append(100.0 * np.sum(np.abs(Sv[keep] - R[keep]) / R[keep]) / len(R))   # eq. percentError
            valid.append(np.mean(Sv < smax))
        del plan
        return ms, {"tau": tau, "precision": precision, "max_percent_error": round(max(E), 4), "printed_max": pr,
                    "ratio": round(max(E) / pr, 4), "mean_percent_error": round(float(np.mean(E)), 4),
                    "valid_fraction": round(float(np.mean(valid)), 5), "ms_per_trial": round(ms / trials, 4)}

    rows, total_ms = [], 0.0
    for tau, pr in zip(taus, printed):
        ms, row = run_tau(tau, pr, "fp64")
        total_ms += ms
        rows.append(row)
    # the three smallest tau, where the float64 band stops short of the farthest
    # nodes, in the precision whose band reaches them
    extended = [run_tau(tau, pr, prec)[1] for tau, pr, prec in
                ((5e-5, printed[0], "fp64x4"), (1e-4, printed[1], "fp64x2"), (1.5e-4, printed[2], "fp64x2"))]
    line = {"metric": "Sec. 6.1 Example 1 trials/s (129^2, K=5000, float64) with Table 2 maxima",
            "value": round(trials * len(taus) / (total_ms * 1e-3), 1), "unit": "trials/s", "n_gpus": 1,
            "steps": trials * len(taus), "warmup": 3, "ms_per_step": round(total_ms / (trials * len(taus)), 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "example1_2d_129_K5000_table2_taus", "trials_per_tau": trials},
            "roofline": None, "note": "cache-resident 2D size: no roofline claim", "table2": rows,
            "table2_extended_precision": extended}
    print(json.dumps(line), flush=True)


def run_batch(steps, warmup):
    """96 square 2D instances (n log-uniform in [128, 1024], K log-uniform in
    [100, 20000] uniform points, tau = 2h), S and grad S in float32, one
    batched call per step, replayed from a HIP graph."""
    import torch
    import synth
    import paper_1112_3010_amd as dt
    inst = synth.workload("c4_batch_2d").extra["instances"]
    dims = [(n, n) for n, _ in inst]
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(y) for _, y in inst])
    Y = Y.cuda()
    nodes = sum(n * n for n, _ in inst)

    def run(plan, S, G, graph):
        plan.set_graph(graph)
        for _ in range(warmup):
            plan.forward_into(Y, offs, S, G)
        ms, _ = timed_calls(lambda: plan.forward_into(Y, offs, S, G), steps)
        return ms

    def timed(plan):
        S, G = plan.empty_outputs()
        res = {"default": run(plan, S, G, True)}      # default tiles and radix schedules
        tuned = plan.autotune(Y, offs, reps=2, cache=False)
        res["eager"] = run(plan, S, G, False)
        res["graph"] = run(plan, S, G, True)
        assert plan.last_error() == 0
        sched = np.array(tuned.pop("schedule"))
        tuned["schedule_families"] = {p: np.bincount(sched[:, k], minlength=6).tolist()
                                      for k, p in enumerate(("rows", "columns", "inverse_rows"))}
        padded = [plan.padded(i) for i in range(len(dims))]
        return res, tuned, batch_bytes(dims, padded, 4, 3), int(sum(a * b for a, b in padded))

    taus = [2.0 / n for n, _ in inst]
    res, tiles, nbytes, full_points = timed(dt.BatchPlan(dims, taus, precision="fp32", graph=False))
    ms = res["graph"]
    line = {"metric": "grid pts/s for S+grad S over a batch of 96 2D instances (n 128-1024)",
            "value": round(nodes / (ms * 1e-3), 1), "unit": "grid pts/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 4), "ms_per_step_eager": round(res["eager"], 4),
            "ms_per_step_default_tuning": round(res["default"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batch96_2d_n128-1024_K100-20000_tau2h_S_gradS", "instances": len(inst),
                       "nodes": nodes, "tiles": tiles},
            "path": {"model_bytes": nbytes, "achieved_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    # the same batch with reduced padding (k_max = each instance's source count)
    rplan = dt.BatchPlan(dims, taus, precision="fp32", graph=False, k_max=[len(y) for _, y in inst])
    rres, rtiles, rbytes, red_points = timed(rplan)
    rms = rres["graph"]
    line["reduced_padding"] = {
        "value": round(nodes / (rms * 1e-3), 1), "unit": "grid pts/s", "ms_per_step": round(rms, 4),
        "ms_per_step_eager": round(rres["eager"], 4), "ms_per_step_default_tuning": round(rres["default"], 4),
        "tiles": rtiles,
        "padded_points": red_points, "padded_points_full": full_points,
        "path": {"model_bytes": rbytes, "achieved_gbs": round(rbytes / (rms * 1e-3) / 1e9, 1),
                 "frac": round(rbytes / (rms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    print(json.dumps(line), flush=True)


# float64 VALU operations of the double-double primitives (each add, mul or
# fma one operation): the accurate add is two TwoSums (6 each), two
# Fast2Sums (3 each) and two adds; the product is TwoProd (mul + fma), two
# cross products, two adds and a Fast2Sum.
DD_ADD_OPS, DD_MUL_OPS = 20, 9
# one float64 VALU operation per lane per clock: 256 CUs x 64 lanes x 2.4 GHz
# (78.6 TFLOP/s with an FMA counted as two)
F64_OPS_PEAK_T = 256 * 64 * 2.4e9 / 1e12


def dd_col_ops(Mx, My):
    """Operations of the fused double-double column pass: per column a
    forward and an inverse radix-2 transform of My points (My/2 log2 My
    butterflies, each a complex multiply of 4 products and 2 adds plus a
    complex add and subtract) and My real-by-complex products."""
    bfly = (4 * DD_MUL_OPS + 2 * DD_ADD_OPS) + 4 * DD_ADD_OPS
    logM = int(round(np.log2(My)))
    return Mx * (2 * (My // 2) * logM * bfly + My * 2 * DD_MUL_OPS)


def run_dd(steps, warmup, no_cpu, cpu_cells):
    """The double-double path on the 1024^2 polygon workload (K = 8000,
    tau = 0.5 h: the smallest tau of that workload, where float64 loses the
    most of the grid), S only, timed beside the quad-double and float64 paths
    on the same input.  ALU-bound: the roofline counts float64 operations of
    the double-double column pass."""
    import torch
    import paper_1112_3010_amd as dt
    import synth
    w = synth.workload("c2_2d_1024_polygon")
    dims = w.dims
    h = tuple(1.0 / n for n in dims)
    tau = w.taus[0]
    Yd = torch.from_numpy(w.points).cuda()
    res = {}
    for prec in ("fp64x2", "fp64x4", "fp64"):
        plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S"])
        S = plan._empty()
        for _ in range(warmup):
            plan.distance_into(S, Yd)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            plan.distance_into(S, Yd)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        plan.set_timing(True)
        plan.timings(reset=True)
        for _ in range(5):
            plan.distance_into(S, Yd)
        per = plan.timings(reset=True)
        plan.set_timing(False)
        st = plan.last_stats()
        res[prec] = {"ms": ms, "pass_ms": {k: round(v[1] / v[0], 4) for k, v in per.items() if v[0] > 0},
                     "s_max_over_tau": st["s_max"] / tau, "S": S.cpu().numpy().astype(np.float64).ravel(),
                     "padded": plan.padded, "theta": st["theta"]}
        log(f"{prec}: {ms:.3f} ms, S_max/tau {st['s_max'] / tau:.2f}, passes {res[prec]['pass_ms']}")
        del plan
    # S and grad S in double-double (three channels through the column pass)
    plan = dt.Plan(dims, h, None, tau, precision="fp64x2", outputs=["S", "grad"])
    out = {"S": plan._empty(), "grad": plan._empty(2)}
    for _ in range(warmup):
        plan.forward_into(out, Yd)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.forward_into(out, Yd)
    e1.record()
    torch.cuda.synchronize()
    grad_ms = e0.elapsed_time(e1) / steps
    log(f"fp64x2 S + grad: {grad_ms:.3f} ms")
    del plan
    # 3D: 128^3 with 4096 points near a sphere, tau = h (256^3 padded), S and
    # S + grad S in double-double beside float64
    n3 = 128
    dims3 = (n3,) * 3
    h3 = (1.0 / n3,) * 3
    Y3 = torch.from_numpy(synth.jittered_sphere_points(4096, 0.3, 2.0 / n3, seed=11)).cuda()
    d3 = {}
    for prec, outs in (("fp64x2", ["S"]), ("fp64x2", ["S", "grad"]), ("fp64", ["S", "grad"]),
                       ("fp64x2", ["S", "backward"]), ("fp64x4", ["S"]), ("fp64x4", ["S", "grad"])):
        plan = dt.Plan(dims3, h3, None, h3[0], precision=prec, outputs=outs)
        if outs == ["S"]:
            fwd = lambda: plan.distance(Y3)
        elif outs == ["S", "grad"]:
            fwd = lambda: plan.gradient(Y3)
        else:
            S3 = plan.distance(Y3)
            G3 = S3.clone()
            fwd = lambda: plan.backward(Y3, S3, G3)
        for _ in range(max(1, warmup // 2)):
            fwd()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = max(3, steps // 4)
        for _ in range(reps):
            fwd()
        e1.record()
        torch.cuda.synchronize()
        key = f"{prec}_{'_'.join(outs)}"
        d3[key] = {"ms": round(e0.elapsed_time(e1) / reps, 3),
                   "s_max_over_tau": round(plan.last_stats()["s_max"] / h3[0], 2), "padded": list(plan.padded)}
        log(f"3D 128^3 {key}: {d3[key]}")
        del plan
    torch.cuda.empty_cache()
    r = res["fp64x2"]
    Mx, My = r["padded"]
    col_ms = r["pass_ms"]["dd_col_fused"]
    ops = dd_col_ops(Mx, My)
    achieved = ops / (col_ms * 1e-3) / 1e12
    nodes = dims[0] * dims[1]
    line = {"metric": "grid pts/s for S at 1024^2 in double-double (extended valid band)",
            "value": round(nodes / (r["ms"] * 1e-3), 1), "unit": "grid pts/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(r["ms"], 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64x2", "data": "synthetic",
            "config": {"workload": "polygon_2d_1024_K8000_tau0.5h_S", "padded": [Mx, My]},
            "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(F64_OPS_PEAK_T, 2),
                         "unit": "T f64-ops/s", "frac": round(achieved / F64_OPS_PEAK_T, 4), "traffic": None,
                         "kernel": "dd_col_fused", "ops_per_launch": ops},
            "pass_ms": r["pass_ms"], "s_max_over_tau": round(r["s_max_over_tau"], 2),
            "with_grad_ms_per_step": round(grad_ms, 4),
            "3d_128cube_sphere4096_tau1h": d3,
            "fp64": {"ms_per_step": round(res["fp64"]["ms"], 4), "pass_ms": res["fp64"]["pass_ms"],
                     "s_max_over_tau": round(res["fp64"]["s_max_over_tau"], 2)},
            "fp64x4": {"ms_per_step": round(res["fp64x4"]["ms"], 4), "pass_ms": res["fp64x4"]["pass_ms"],
                       "s_max_over_tau": round(res["fp64x4"]["s_max_over_tau"], 2)}}
    if not no_cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        rng = np.random.default_rng(2024)
        cells = np.sort(rng.choice(nodes, cpu_cells, replace=False))
        o = (0.0, 0.0)
        idx, valid = oracle.snap(w.points, o, h, dims)
        Yh = oracle.node_coords(idx[valid], o, h)
        X = oracle.grid_nodes(dims, o, h, cells)
        with threadpool_limits(1):
            t0 = time.perf_counter()
            f = oracle.fields(X, Yh, tau)
            dt_s = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(len(cells) / dt_s, 2), "unit": "grid pts/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{len(cells)} random nodes of the 1024^2 grid, all {int(valid.sum())} "
                                          f"sources each, S in float64 ({dt_s:.1f} s)"}
        acc = {}
        for prec in ("fp64x2", "fp64x4", "fp64"):
            smax = res[prec]["s_max_over_tau"] * tau
            ref = np.minimum(f["S"], smax)
            Sg = res[prec]["S"][cells]
            deep = f["lnphi"] >= np.log(2.0 * res[prec]["theta"])
            acc[prec] = {"max_dS_over_tau": float(np.abs(Sg - ref).max() / tau),
                         "resolved_fraction": round(float(deep.mean()), 4)}
        line["accuracy_vs_oracle"] = acc
    print(json.dumps(line), flush=True)


def run_reduced(steps, warmup, timing_calls, no_cpu, cpu_cells):
    """The 256^3 mesh workload with its source count known to the plan
    (k_max = the 60 000 triangles): every axis pads to 288 instead of 512,
    with kernels truncated where they fall below the rounding floor.
    Forward S+grad S and the backward, each beside the fully padded plan on
    the same inputs; the forward fields of both are compared with the oracle
    on a node sample."""
    import synth
    n = 256
    dims = (n, n, n)
    tau = 1.0 / n
    V, F = synth.harmonic_star_mesh(seed=3)
    log(f"workload: 256^3, {len(F)} triangles, tau = h, full vs reduced padding")
    cells = sample_cells(dims, cpu_cells, seed=1)
    full = run_gpu("fp32", V, F, dims, tau, steps, warmup, timing_calls, cells)
    log("fp32 full padding:", json.dumps({k: v for k, v in full.items() if not k.startswith("sample_")}))
    red = run_gpu("fp32", V, F, dims, tau, steps, warmup, timing_calls, cells, k_max=len(F))
    log("fp32 reduced padding:", json.dumps({k: v for k, v in red.items() if not k.startswith("sample_")}))
    Yc = triangle_centres(V, F)
    bsteps = max(5, steps // 2)
    b_full = run_backward("fp32", Yc, dims, tau, bsteps, warmup, timing_calls)
    b_red = run_backward("fp32", Yc, dims, tau, bsteps, warmup, timing_calls, k_max=len(F))
    log("fp32 backward full / reduced:", json.dumps(b_full), json.dumps(b_red))
    # float64: the truncation distance is longer (c = 49), and every axis pads to 392
    f64 = run_gpu("fp64", V, F, dims, tau, bsteps, warmup, timing_calls, cells)
    r64 = run_gpu("fp64", V, F, dims, tau, bsteps, warmup, timing_calls, cells, k_max=len(F))
    log("fp64 full / reduced:", json.dumps({k: v for k, v in f64.items() if not k.startswith("sample_")}),
        json.dumps({k: v for k, v in r64.items() if not k.startswith("sample_")}))
    line = {
        "metric": METRIC, "value": round(red["value"], 1), "unit": "grid pts/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(red["ms_per_step"], 4), "ms_stats": red["ms_stats"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3d_256cube_mesh60000_tau1h_S_gradS_reduced_padding", "grid": list(dims),
                   "padded": red["padded"], "cut": red["cut"], "k_max": int(len(F)), "sources": int(len(F)),
                   "tau_over_h": 1.0, "precision": "fp32_scaled"},
        "roofline": roofline_entry(red["pass_bytes"], red["pass_ms"], red["launches"], red["dominant"]),
        "path": {"model_bytes": red["model_bytes"], "achieved_gbs": round(red["path_gbs"], 1),
                 "frac": round(red["path_gbs"] / HBM_PEAK_GBS, 4), "pass_ms": red["pass_ms"],
                 "pass_gbs": red["pass_gbs"], "s_max_over_tau": round(red["s_max_over_tau"], 3),
                 "plan_setup_s": round(red["plan_setup_s"], 3), "plan_tables_s": round(red["plan_tables_s"], 4)},
        "full_padding": {"value": round(full["value"], 1), "ms_per_step": round(full["ms_per_step"], 4),
                         "padded": full["padded"], "pass_ms": full["pass_ms"],
                         "s_max_over_tau": round(full["s_max_over_tau"], 3)},
        "speedup_vs_full_padding": round(full["ms_per_step"] / red["ms_per_step"], 3),
        "backward": b_red,
        "backward_full_padding": {"ms_per_call": b_full["ms_per_call"], "padded": b_full["padded"],
                                  "path": b_full["path"]},
        "backward_speedup_vs_full_padding": round(b_full["ms_per_call"] / b_red["ms_per_call"], 3),
        "fp64": {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 4),
                 "ms_stats": r64["ms_stats"], "dtype": "f64", "padded": r64["padded"], "cut": r64["cut"],
                 "roofline": roofline_entry(r64["pass_bytes"], r64["pass_ms"], r64["launches"], r64["dominant"]),
                 "path": {"model_bytes": r64["model_bytes"], "achieved_gbs": round(r64["path_gbs"], 1),
                          "frac": round(r64["path_gbs"] / HBM_PEAK_GBS, 4), "pass_ms": r64["pass_ms"],
                          "s_max_over_tau": round(r64["s_max_over_tau"], 3)},
                 "full_padding": {"ms_per_step": round(f64["ms_per_step"], 4), "padded": f64["padded"],
                                  "pass_ms": f64["pass_ms"], "s_max_over_tau": round(f64["s_max_over_tau"], 3)},
                 "speedup_vs_full_padding": round(f64["ms_per_step"] / r64["ms_per_step"], 3)},
    }
    if not no_cpu:
        cb, acc = cpu_baseline(V, F, dims, tau, cells, [("fp32_reduced", "fp32", red), ("fp32_full", "fp32", full),
                                                        ("fp64_reduced", "fp64", r64), ("fp64_full", "fp64", f64)])
        cb["value"] = round(cb["value"], 2)
        line["cpu_baseline"] = cb
        line["accuracy_vs_oracle"] = dict(acc, sample=f"the cpu_baseline's {len(cells)} nodes")
    print(json.dumps(line), flush=True)


def run_configs(steps, warmup, no_cpu):
    """Every workload configuration once: the GPU forward call in float32 with
    scaling and in float64 (median of `steps` calls), and on the host's cores
    the oracle's direct sums timed on a bounded node sample (throughput, and
    the full grid's time extrapolated from it), beside the paper's Table 1
    FFT convolution in float64 with scipy (context)."""
    import torch
    import oracle
    import synth
    import paper_1112_3010_amd as dt
    from oracle import table1
    from threadpoolctl import threadpool_limits
    workers = max(1, min(16, len(os.sched_getaffinity(0))))

    def gpu_ms(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        _, st = timed_calls(fn, steps)
        return st["median"]

    def oracle_rate(dims, h, Y, tau, n_cells, hess=False, sign=None, seed=0):
        """Nodes per second of the oracle's S, grad S (and H, and the sign
        sum) on n_cells sampled nodes; the sign sums run on one thread."""
        X = oracle.grid_nodes(dims, (0.0,) * len(dims), h, sample_cells(dims, n_cells, seed))
        with threadpool_limits(1):
            t0 = time.perf_counter()
            oracle.fields(X, Y, tau, grad=True, hess=hess, workers=workers)
            t_f = time.perf_counter() - t0
        out = {"sample_nodes": n_cells, "fields_s": round(t_f, 2), "cores": workers}
        rate = n_cells / t_f
        if sign is not None:
            m = max(64, n_cells // 8)
            t0 = time.perf_counter()
            sign(X[:m])
            t_s = (time.perf_counter() - t0) * n_cells / m
            out["sign_s"] = round(t_s, 2)
            out["sign_cores"] = 1
            rate = n_cells / (t_f + t_s)
        out["nodes_per_s"] = round(rate, 1)
        out["full_grid_s_extrapolated"] = round(float(np.prod(dims)) / rate, 1)
        return out

    def table1_s(idx, dims, h, tau):
        t0 = time.perf_counter()
        table1.table1_phi(idx, dims, h, tau, workers=workers)
        return round(time.perf_counter() - t0, 3)

    res = {}
    # C1: 2D 128^2, 64 points at random cells, tau = 2h, S and grad S
    w = synth.workload("c1_2d_128")
    dims, h, tau = w.dims, (1.0 / 128,) * 2, w.taus[0]
    Yd = torch.from_numpy(w.points).cuda()
    c = {"grid": list(dims), "K": len(w.points), "tau_over_h": 2.0, "outputs": "S, grad S"}
    for prec in ("fp32", "fp64"):
        plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad"])
        c[f"gpu_{prec}_ms"] = gpu_ms(lambda: plan.gradient(Yd))
    idx, valid = oracle.snap(w.points, (0.0, 0.0), h, dims)
    Yh = oracle.node_coords(idx[valid], (0.0, 0.0), h)
    if not no_cpu:
        c["oracle"] = oracle_rate(dims, h, Yh, tau, 16384)
        c["table1_fft_f64_s"] = table1_s(idx[valid], dims, h, tau)
    res["c1_2d_128"] = c
    log("c1:", json.dumps(c))

    # C2: 2D 1024^2, 8000 points on a star polygon, tau in {0.5, 2, 8} h, S, grad S, Hessian, winding number
    w = synth.workload("c2_2d_1024_polygon")
    dims, h = w.dims, (1.0 / 1024,) * 2
    poly = torch.from_numpy(w.polygon).cuda()
    idx, valid = oracle.snap(w.points, (0.0, 0.0), h, dims)
    Yh = oracle.node_coords(idx[valid], (0.0, 0.0), h)
    for tau in w.taus:
        c = {"grid": list(dims), "K": len(w.points), "tau_over_h": tau * 1024,
             "outputs": "S, grad S, Hessian, winding-number label"}
        for prec in ("fp32", "fp64"):
            plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "hess", "sign"])
            out = {"S": plan._empty(), "grad": plan._empty(2), "hess": plan._empty(3),
                   "label": plan._empty(dtype=torch.int8)}
            c[f"gpu_{prec}_ms"] = gpu_ms(lambda: plan.forward_into(out, polygon=poly))
            c[f"gpu_{prec}_s_max_over_tau"] = round(plan.last_stats()["s_max"] / tau, 2)
        if not no_cpu:
            c["oracle"] = oracle_rate(dims, h, Yh, tau, 16384, hess=True,
                                      sign=lambda X: oracle.sign.winding_number(X, w.polygon))
            c["table1_fft_f64_s"] = table1_s(idx[valid], dims, h, tau)
        res[f"c2_2d_1024_tau{tau * 1024:g}h"] = c
        log("c2:", json.dumps(c))

    # C3: 3D 256^3, the mesh's 60 000 triangles, tau = h, S, grad S, topological degree
    w = synth.workload("c3_3d_256_mesh")
    dims, h, tau = w.dims, (1.0 / 256,) * 3, w.taus[0]
    Vd, Fd = torch.from_numpy(w.vertices).cuda(), torch.from_numpy(w.faces).cuda()
    c = {"grid": list(dims), "K": len(w.faces), "tau_over_h": 1.0, "outputs": "S, grad S, degree label"}
    for prec in ("fp32", "fp64"):
        plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "sign"])
        out = {"S": plan._empty(), "grad": plan._empty(3), "label": plan._empty(dtype=torch.int8)}
        c[f"gpu_{prec}_ms"] = gpu_ms(lambda: plan.forward_into(out, vertices=Vd, faces=Fd))
        del plan, out
        torch.cuda.empty_cache()
    if not no_cpu:
        Ym, P, idx, valid = oracle.sign.snapped_mesh_sources(w.vertices, w.faces, (0.0,) * 3, h, dims)
        c["oracle"] = oracle_rate(dims, h, Ym[valid], tau, 4096,
                                  sign=lambda X: oracle.sign.topological_degree(X, Ym[valid], P[valid]))
        c["table1_fft_f64_s"] = table1_s(idx[valid], dims, h, tau)
    res["c3_3d_256_mesh"] = c
    log("c3:", json.dumps(c))

    # C4: 96 2D instances in one batched call (graph replay, default tiles and schedules)
    inst = synth.workload("c4_batch_2d").extra["instances"]
    bd = [(n, n) for n, _ in inst]
    Y, offs = dt.BatchPlan.pack([torch.from_numpy(y) for _, y in inst])
    Y = Y.cuda()
    c = {"instances": len(inst), "nodes": int(sum(n * n for n, _ in inst)), "outputs": "S, grad S"}
    for prec in ("fp32", "fp64"):
        plan = dt.BatchPlan(bd, [2.0 / n for n, _ in inst], precision=prec, graph=True)
        S, G = plan.empty_outputs()
        c[f"gpu_{prec}_ms"] = gpu_ms(lambda: plan.forward_into(Y, offs, S, G))
        del plan, S, G
    if not no_cpu:
        # 256 sampled nodes of every instance, all of its sources
        n_nodes, t_all = 0, 0.0
        for i, (n, y) in enumerate(inst):
            hh = (1.0 / n,) * 2
            ii, vv = oracle.snap(y, (0.0, 0.0), hh, (n, n))
            X = oracle.grid_nodes((n, n), (0.0, 0.0), hh, sample_cells((n, n), 256, i))
            with threadpool_limits(1):
                t0 = time.perf_counter()
                oracle.fields(X, oracle.node_coords(ii[vv], (0.0, 0.0), hh), 2.0 / n, grad=True, workers=workers)
                t_all += time.perf_counter() - t0
            n_nodes += 256
        c["oracle"] = {"sample_nodes": n_nodes, "fields_s": round(t_all, 2), "cores": workers,
                       "nodes_per_s_of_an_average_instance": round(n_nodes / t_all, 1),
                       "full_batch_s_extrapolated": round(c["nodes"] / (n_nodes / t_all), 1)}
    res["c4_batch_2d"] = c
    log("c4:", json.dumps(c))

    # C5: 3D 128^3, 4096 points around a sphere, tau = 4h: forward S and grad S,
    # and the backward of sum (S - S_target)^2
    w = synth.workload("c5_3d_128_grad")
    dims, h, tau = w.dims, (1.0 / 128,) * 3, w.taus[0]
    Yd = torch.from_numpy(w.points).cuda()
    T = torch.from_numpy(np.ascontiguousarray(w.target)).cuda()
    c = {"grid": list(dims), "K": len(w.points), "tau_over_h": tau * 128,
         "outputs": "forward S, grad S; backward dL/dY, dL/dtau"}
    for prec in ("fp32", "fp64"):
        plan = dt.Plan(dims, h, None, tau, precision=prec, outputs=["S", "grad", "backward"])
        c[f"gpu_{prec}_forward_ms"] = gpu_ms(lambda: plan.gradient(Yd))
        S = plan.distance(Yd)
        G = (2.0 * (S - T.to(S.dtype))).contiguous()
        c[f"gpu_{prec}_backward_ms"] = gpu_ms(lambda: plan.backward(Yd, S, G))
    if not no_cpu:
        idx, valid = oracle.snap(w.points, (0.0,) * 3, h, dims)
        Yh = oracle.node_coords(idx[valid], (0.0,) * 3, h)
        c["oracle"] = oracle_rate(dims, h, Yh, tau, 32768)
        c["table1_fft_f64_s"] = table1_s(idx[valid], dims, h, tau)
    res["c5_3d_128_grad"] = c
    log("c5:", json.dumps(c))
    line = {"metric": "per-configuration GPU call time and oracle throughput", "unit": "ms", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "higher_is_better": False, "data": "synthetic",
            "host": {"cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "oracle_threads": workers},
            "config": {"workload": "all_configurations"}, "configs": res}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--timing-calls", type=int, default=10)
    ap.add_argument("--cpu-cells", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-curv", action="store_true", help="skip the 256^3 curvature timing")
    ap.add_argument("--workload", choices=["mesh256", "batch", "protocol", "dd", "reduced", "configs"],
                    default="mesh256",
                    help="mesh256: the 256^3 mesh headline (default); batch: 96 mixed-size 2D instances; "
                         "protocol: Example 1 of Sec. 6.1 against Table 2; dd: 1024^2 polygon S in double-double; "
                         "reduced: the 256^3 mesh with k_max reduced padding, beside full padding; "
                         "configs: every workload configuration, GPU beside the oracle")
    ap.add_argument("--trials", type=int, default=200, help="trials per tau of --workload protocol")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy (3 times) to calibrate HBM traffic counters, then exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {a.numel() * 4} bytes x 3")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (got --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args.steps, args.warmup)
        return
    if args.workload == "protocol":
        run_protocol(args.trials)
        return
    if args.workload == "dd":
        run_dd(args.steps, args.warmup, args.no_cpu, min(args.cpu_cells, 4096))
        return
    if args.workload == "reduced":
        run_reduced(args.steps, args.warmup, args.timing_calls, args.no_cpu, min(args.cpu_cells, 8192))
        return
    if args.workload == "configs":
        run_configs(min(args.steps, 20), args.warmup, args.no_cpu)
        return
    import synth
    n = 256
    dims = (n, n, n)
    tau = 1.0 / n
    V, F = synth.harmonic_star_mesh(seed=3)
    log(f"workload: 256^3, {len(F)} triangles, tau = h")
    cells = sample_cells(dims, args.cpu_cells)
    r32 = run_gpu("fp32", V, F, dims, tau, args.steps, args.warmup, args.timing_calls, cells)
    log("fp32:", json.dumps({k: v for k, v in r32.items() if not k.startswith("sample_")}))
    Yc = triangle_centres(V, F)
    b32 = run_backward("fp32", Yc, dims, tau, max(5, args.steps // 2), args.warmup, args.timing_calls)
    log("fp32 backward:", json.dumps(b32))
    c32 = None
    if not args.no_curv:
        c32 = run_curvature("fp32", Yc, dims, tau, max(5, args.steps // 5), args.warmup, args.timing_calls)
        log("fp32 curvature:", json.dumps(c32))
    r64 = b64 = None
    if not args.no_fp64:
        r64 = run_gpu("fp64", V, F, dims, tau, max(5, args.steps // 2), args.warmup, args.timing_calls, cells)
        log("fp64:", json.dumps({k: v for k, v in r64.items() if not k.startswith("sample_")}))
        b64 = run_backward("fp64", Yc, dims, tau, max(5, args.steps // 4), args.warmup, args.timing_calls)
        log("fp64 backward:", json.dumps(b64))
    clocks_after = gpu_clocks()
    khash = kernel_hash()

    def counter_frac(r, prec):
        """Whole-path HBM bytes from the rocprofv3 counters of the passes that
        have them (the rest at their algorithmic bytes), over the call's time."""
        got = {k: counters_for(khash, prec, k) for k in r["pass_bytes"]}
        if got.get(r["dominant"]) is None:
            return None
        total = sum(v if v is not None else r["pass_bytes"][k] for k, v in got.items())
        gbs = total / (r["ms_per_step"] * 1e-3) / 1e9
        return {"bytes": int(total), "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                "passes_with_counters": sorted(k for k, v in got.items() if v is not None)}

    def roof(r, prec):
        traffic = counters_for(khash, prec, r["dominant"])
        return roofline_entry(r["pass_bytes"], r["pass_ms"], r["launches"], r["dominant"], traffic)

    line = {
        "metric": METRIC,
        "value": round(r32["value"], 1),
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "ms_stats": r32["ms_stats"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3d_256cube_mesh60000_tau1h_S_gradS", "grid": list(dims), "padded": r32["padded"],
                   "sources": int(len(F)), "tau_over_h": 1.0, "precision": "fp32_scaled"},
        "roofline": roof(r32, "fp32"),
        "path": {"model_bytes": r32["model_bytes"], "achieved_gbs": round(r32["path_gbs"], 1),
                 "frac": round(r32["path_gbs"] / HBM_PEAK_GBS, 4), "pass_ms": r32["pass_ms"],
                 "pass_gbs": r32["pass_gbs"], "s_max_over_tau": round(r32["s_max_over_tau"], 3),
                 "plan_setup_s": round(r32["plan_setup_s"], 3), "plan_tables_s": round(r32["plan_tables_s"], 4),
                 "counters": counter_frac(r32, "fp32")},
    }
    line["gpu_clocks"] = clocks_after
    line["backward"] = b32
    if c32 is not None:
        line["curvature"] = c32
    if r64 is not None:
        line["fp64"] = {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 4),
                        "ms_stats": r64["ms_stats"], "dtype": "f64", "roofline": roof(r64, "fp64"),
                        "path": {"model_bytes": r64["model_bytes"], "achieved_gbs": round(r64["path_gbs"], 1),
                                 "frac": round(r64["path_gbs"] / HBM_PEAK_GBS, 4), "pass_ms": r64["pass_ms"],
                                 "pass_gbs": r64["pass_gbs"], "s_max_over_tau": round(r64["s_max_over_tau"], 3),
                                 "plan_tables_s": round(r64["plan_tables_s"], 4),
                                 "counters": counter_frac(r64, "fp64")},
                        "backward": b64}
    if not args.no_cpu:
        cb, acc = cpu_baseline(V, F, dims, tau, cells, [("fp32", "fp32", r32), ("fp64", "fp64", r64)])
        cb["value"] = round(cb["value"], 2)
        line["cpu_baseline"] = cb
        line["accuracy_vs_oracle"] = dict(acc, sample=f"the cpu_baseline's {len(cells)} nodes")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
