"""Walk-on-stars throughput on one MI355X.

Workload: the 2D star-polygon Laplace problem (16,384 segments, half of the
arc length Neumann in 4 arcs, exact u = exp(x) cos(y)), 262,144 interior
points, 1024 walks per point, eps = 1e-4.  One "step" is a whole solve of
that workload: every walk of every point, from the points already resident
in HBM to the per-point FP64 mean and variance in HBM.

Prints one JSON line: walk steps/s (the metric), points/s at the measured
standard error, the plain-launch figure beside the chosen (persistent,
lane-refill) form, the walk kernel's roofline figures and the FP64 oracle's
throughput on the host cores for a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=262144)
    ap.add_argument("--walks", type=int, default=1024)
    ap.add_argument("--count-points", type=int, default=16384,
                    help="points of the traffic-accounting solve (a prefix of the workload)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec, pts, walks, eps, seed, seconds, threads):
    """The FP64 brute-force oracle on a growing prefix of the workload until
    about `seconds` of wall time; steps/s of that sample."""
    import oracle as O
    R = O.Scene(spec)
    nthreads = max(1, min(threads, os.cpu_count() or 1))
    n = nthreads
    w = 16
    while True:
        t0 = time.perf_counter()
        r = R.solve(pts[:n], w, eps, seed=seed, nthreads=nthreads)
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= pts.shape[0]:
            break
        scale = max(2.0, min(8.0, seconds / max(dt, 1e-3)))
        n = min(pts.shape[0], int(n * scale))
    return {"value": r["steps"] / dt, "unit": "steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} points x {w} walks of the workload ({r['steps']} steps, {dt:.1f} s)",
            "walks_per_s": n * w / dt}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "single-GPU build: run with --gpus 1"}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W

    torch.cuda.set_device(0)
    cfg = I.config2(n_points=a.points, walks=a.walks)
    spec, pts, Wk, eps, seed = cfg["scene"], cfg["points"], cfg["walks"], cfg["eps"], cfg["seed"]
    S = W.Scene(spec)
    n = pts.shape[0]
    d_pts = torch.from_numpy(pts).cuda()
    d_mean = torch.empty(n, dtype=torch.float64, device="cuda")
    d_var = torch.empty_like(d_mean)
    stream = torch.cuda.current_stream()
    opts = W.make_opts(mode=0)
    log(f"scene: {spec.n_prims} segments, {S.info.n_neumann} Neumann; {n} points x {Wk} walks")

    def solve(o, npts=n):
        W.wost_solve_ex(S.handle, d_pts, npts, Wk, eps, seed, 0, 0, o, d_mean, d_var, stream.cuda_stream)
        return W.wost_get_stats(S.handle)

    for i in range(a.warmup):
        st = solve(opts)
        log(f"warmup {i}: {st.kernel_ms:.1f} ms, {st.steps} steps, grid {st.grid_blocks}")
    steps_total = 0
    kms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        st = solve(opts)
        steps_total += st.steps
        kms.append(st.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed: {a.steps} solves in {dt:.2f} s; walk kernel {np.mean(kms):.1f} ms")
    mean = d_mean.cpu().numpy()
    var = d_var.cpu().numpy()
    se = np.sqrt(var / Wk)
    u = spec.exact(pts)
    pos = se > 0
    z = (mean[pos] - u[pos]) / se[pos]
    eps_bound = float(eps * np.exp(spec.vertices[:, 0].astype(np.float64).max()))
    steps_per_solve = steps_total / a.steps
    kernel_s = float(np.mean(kms)) / 1e3

    plain = None
    if not a.no_plain:
        stp = solve(W.make_opts(mode=1))
        plain = {"steps_per_s": stp.steps / (stp.kernel_ms / 1e3), "kernel_ms": stp.kernel_ms,
                 "points_per_s": n / (stp.kernel_ms / 1e3)}
        same = bool(np.array_equal(d_mean.cpu().numpy(), mean))
        plain["identical_estimates"] = same
        log(f"plain launch: {stp.kernel_ms:.1f} ms (identical estimates: {same})")

    # algorithmic bytes per step from the traffic-accounting variant on a prefix
    nc = min(a.count_points, n)
    solve(W.make_opts(flags=W.WOST_SOLVE_COUNT_TRAFFIC), nc)
    tr = W.wost_get_traffic(S.handle)
    stc = W.wost_get_stats(S.handle)
    bytes_per_step = tr.bytes / stc.steps
    traffic_bytes_per_launch = bytes_per_step * steps_per_solve
    achieved = traffic_bytes_per_launch / kernel_s / 1e9
    fetch = {k: getattr(tr, k) / stc.steps for k in ("q1_nodes", "q1_prims", "q2_nodes", "q2_cones", "q2_elems",
                                                       "q3_nodes", "q3_prims", "q4_nodes", "q4_prims",
                                                       "vis_nodes", "vis_prims")}
    log(f"traffic: {bytes_per_step:.0f} B/step; per step {json.dumps({k: round(v, 2) for k, v in fetch.items()})}")

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(spec, pts, Wk, eps, seed, a.cpu_seconds, a.cpu_threads)
        log(f"cpu baseline: {cpu['value']:.3g} steps/s on {cpu['cores']} threads ({cpu['sample']})")

    out = {
        "metric": "walk steps/s",
        "value": steps_per_solve * a.steps / dt,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D star polygon Laplace: 16384 segments (50% Neumann), "
                               "262144 points x 1024 walks, eps 1e-4",
                   "points": n, "walks_per_point": Wk, "form": "persistent lane-refill kernel"},
        "points_per_s": n * a.steps / dt,
        "walks_per_s": n * Wk * a.steps / dt,
        "se_median": float(np.median(se)),
        "se_p90": float(np.percentile(se, 90)),
        "mean_steps_per_walk": steps_per_solve / (n * Wk),
        "exact_error_rmse": float(np.sqrt(np.mean((mean - u) ** 2))),
        "exact_bias": float(np.mean(mean - u)),
        "z_beyond_4": int(np.sum(np.abs(z) > 4)),
        "z_allowed": 2 * z.size * 6.33e-5 + 3,
        # a walk stops within eps of the Dirichlet boundary and returns g at
        # the closest point, so each estimate carries a bias of at most
        # eps * sup|grad u| (here sup e^x over the domain)
        "eps_shell_bound": eps_bound,
        "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mean - u) > 4 * se + eps_bound)),
        "plain": plain,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_step": bytes_per_step, "kernel_ms": float(np.mean(kms)),
                     "fetches_per_step": fetch},
        "cpu_baseline": cpu,
    }
    if a.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB (fetch 1 GiB, write 1 GiB each)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
