"""Walk-on-stars throughput on one MI355X.

Default workload: the 2D star-polygon Laplace problem (16,384 segments, half
of the arc length Neumann in 4 arcs, exact u = exp(x) cos(y)), 262,144
interior points, 1024 walks per point, eps = 1e-4.  One "step" is a whole
solve of that workload: every walk of every point, from the points already
resident in HBM to the per-point FP64 mean and variance in HBM.

Prints one JSON line: walk steps/s (the metric), points/s at the measured
standard error, the plain-launch figure beside the chosen (persistent,
lane-refill) form, the walk kernel's roofline figures and the FP64 oracle's
throughput on the host cores for a bounded sample of the same workload.

Other workloads (--workload): icosphere3d (3D displaced icosphere, 1.3M
triangles), geodesic64 (64 scenes: batched launch vs per-scene launches),
serving (Poisson arrivals over a pool of icosphere scenes, progressive
refinement, latency percentiles), and the extensions, sweep and mixed
studies; each prints its own JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# L2 bandwidth of MI355X: 8 XCDs x 16 L2 channels x 128 B per clock x 2.4 GHz.
# The star-polygon scene (about 1 MB of trees and primitives) stays in L2
# (hit rate 99.96 % by counter), so the walk kernel's algorithmic bytes are
# served by L2, not HBM, and L2 is the memory roofline that applies.
L2_PEAK_GBS = 8 * 16 * 128 * 2.4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="star2d",
                    choices=["star2d", "icosphere3d", "geodesic64", "serving", "extensions", "sweep", "mixed"])
    ap.add_argument("--walk-div", type=int, default=1,
                    help="icosphere3d/geodesic64: divide every walk count by this (stated in the output)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--window", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--drain", type=float, default=60.0, help="serving: extra seconds to finish work")
    ap.add_argument("--budget-mb", type=float, default=256.0, help="serving: admission budget (MiB)")
    ap.add_argument("--pool", type=int, default=8, help="serving: scenes in the pool")
    ap.add_argument("--max-points", type=int, default=65536, help="serving: largest request (points)")
    ap.add_argument("--se-lo", type=float, default=1e-3, help="serving: smallest target SE")
    ap.add_argument("--se-hi", type=float, default=1e-2, help="serving: largest target SE")
    ap.add_argument("--fixed-rounds", action="store_true", help="serving: 64 walks every round")
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


PROFILE_C2 = os.path.join(ROOT, "profiles", "k_walk_persistent_2d_star_262144x1024.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("wost_device.hpp", "wost_walks.hip", "wost_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2302_11815_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(path):
    """HBM bytes per launch of the walk kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy), or
    None when the kernel sources changed since the counters were taken."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ": " in line and not line.startswith(("|", "#", "`")):
                    k, v = line.strip().split(": ", 1)
                    kv[k] = v
        if kv.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


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
        print(json.dumps({"error": "the solver runs on one GPU: run with --gpus 1 (a job larger than one "
                                   "GPU splits by point range, with point_base keeping the random streams)"}),
              flush=True)
        sys.exit(2)
    if a.workload == "icosphere3d":
        return bench_icosphere(a)
    if a.workload == "mixed":
        return bench_mixed(a)
    if a.workload == "geodesic64":
        return bench_geodesic_batch(a)
    if a.workload == "serving":
        return bench_serving(a)
    if a.workload == "extensions":
        return bench_extensions(a)
    if a.workload == "sweep":
        return bench_sweep(a)
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W

    torch.cuda.set_device(0)
    cfg = I.star_polygon_case(n_points=a.points, walks=a.walks)
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

    plain = per_lane = None
    if not a.no_plain:
        stp = solve(W.make_opts(mode=1))
        plain = {"steps_per_s": stp.steps / (stp.kernel_ms / 1e3), "kernel_ms": stp.kernel_ms,
                 "points_per_s": n / (stp.kernel_ms / 1e3)}
        same = bool(np.array_equal(d_mean.cpu().numpy(), mean))
        plain["identical_estimates"] = same
        log(f"plain launch: {stp.kernel_ms:.1f} ms (identical estimates: {same})")
        stl = solve(W.make_opts(mode=2))
        per_lane = {"steps_per_s": stl.steps / (stl.kernel_ms / 1e3), "kernel_ms": stl.kernel_ms,
                    "identical_estimates": bool(np.array_equal(d_mean.cpu().numpy(), mean))}
        log(f"persistent, per-lane searches: {stl.kernel_ms:.1f} ms "
            f"(identical estimates: {per_lane['identical_estimates']})")

    # algorithmic bytes per step from the traffic-accounting variant on a prefix
    nc = min(a.count_points, n)
    solve(W.make_opts(flags=W.WOST_SOLVE_COUNT_TRAFFIC), nc)
    tr = W.wost_get_traffic(S.handle)
    stc = W.wost_get_stats(S.handle)
    bytes_per_step = tr.bytes / stc.steps
    traffic_bytes_per_launch = bytes_per_step * steps_per_solve
    achieved = traffic_bytes_per_launch / kernel_s / 1e9
    l2_stream = max(W.wost_measure_l2_read(2 << 20, 16) for _ in range(3))
    log(f"L2-resident streaming read: {l2_stream:.0f} GB/s")
    fetch = {k: getattr(tr, k) / stc.steps for k in ("q1_nodes", "q1_prims", "q2_nodes", "q2_cones", "q2_elems",
                                                       "q3_nodes", "q3_prims", "q4_nodes", "q4_prims",
                                                       "vis_nodes", "vis_prims")}
    log(f"traffic: {bytes_per_step:.0f} B/step; per step {json.dumps({k: round(v, 2) for k, v in fetch.items()})}")

    traffic = profiled_traffic(PROFILE_C2) if (n, Wk) == (262144, 1024) else None
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
                   "points": n, "walks_per_point": Wk,
                   "form": "persistent lane-refill kernel, wave-cooperative tree searches"},
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
        "persistent_per_lane": per_lane,
        "roofline": {"bound": "l2", "achieved": achieved, "peak": L2_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / L2_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "traffic_hbm_frac": (traffic / kernel_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "bytes_per_step": bytes_per_step, "kernel_ms": float(np.mean(kms)),
                     "fetches_per_step": fetch,
                     # what a streaming kernel reaches over an L2-resident
                     # buffer on this GPU, beside the derived peak
                     "l2_stream_gbs": l2_stream, "frac_of_l2_stream": achieved / l2_stream if l2_stream else None},
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


def _timed_solve(W, S, d, n, walks, eps, seed, opts, m, v, prims=None):
    import torch
    torch.cuda.synchronize()
    if prims is None:
        W.wost_solve_ex(S.handle, d, n, walks, eps, seed, 0, 0, opts, m, v, None)
    else:
        W.wost_solve_boundary_ex(S.handle, d, prims, n, walks, eps, seed, 0, 0, opts, m, v, None)
    st = W.wost_get_stats(S.handle)
    return st, m[:n].cpu().numpy(), v[:n].cpu().numpy()


def bench_extensions(a):
    """Evaluation points on the Neumann boundary, the screened Poisson
    equation and pure-Neumann problems with the Tikhonov switch, on the
    16,384-segment star polygon, and double-sided sheets (16,384 segments):
    throughput and error against closed forms."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    base = I.star_polygon_scene(16384, 0)
    n, walks, eps = min(a.points, 65536), a.walks, 1e-4
    m = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    out = {"workload": "extensions on the 2D star polygon (16384 segments)", "points": n, "walks_per_point": walks}

    def record(name, u, st, mean, var, extra=None):
        """u: the exact solution at the points, or None"""
        se = np.sqrt(var / walks)
        r = {"steps_per_s": st.steps / (st.kernel_ms / 1e3), "kernel_ms": st.kernel_ms,
             "steps_per_walk": st.steps / st.walks, "se_median": float(np.median(se)),
             "capped": st.capped, "escaped": st.escaped}
        if u is not None:
            r["exact_bias"] = float(np.mean(mean - u))
            r["beyond_4se"] = int(np.sum(np.abs(mean - u) > 4 * se + 3e-4))
        if extra:
            r.update(extra)
        out[name] = r
        log(f"{name}: {r['steps_per_s']:.3g} steps/s, {r['steps_per_walk']:.1f} steps/walk")

    # boundary evaluation points (Neumann arcs of the mixed problem)
    S = W.Scene(base)
    pts, prims = I.neumann_boundary_points(base, n, seed=1)
    d = torch.from_numpy(pts).cuda()
    st, mean, var = _timed_solve(W, S, d, n, walks, eps, 3, None, m, v, prims=prims)
    record("boundary_points", base.exact(pts), st, mean, var)
    # screened Poisson, u = exp(0.8 x - 0.6 y), sigma = 1 (mixed)
    spec = I.with_data(base, I.FN_EXPLIN, (1.0, 0.8, -0.6))
    S = W.Scene(spec)
    pts = I.star_polygon_points(n, seed=2, vertices=base.vertices)
    d = torch.from_numpy(pts).cuda()
    st, mean, var = _timed_solve(W, S, d, n, walks, eps, 4, W.make_opts(sigma=1.0), m, v)
    record("screened_sigma1", spec.exact(pts), st, mean, var)
    # the same problem with the boundary made all Neumann (well posed for sigma > 0)
    specN = I.with_data(base, I.FN_EXPLIN, (1.0, 0.8, -0.6), bc=np.full(base.n_prims, I.NEUMANN))
    S = W.Scene(specN)
    st, mean, var = _timed_solve(W, S, d, n, walks, eps, 5, W.make_opts(sigma=1.0), m, v)
    record("screened_pure_neumann", specN.exact(pts), st, mean, var)
    # pure-Neumann Poisson with the Tikhonov switch (u = e^x cos y up to a constant)
    specT = I.dataclasses.replace(base, bc=np.full(base.n_prims, I.NEUMANN, np.uint8))
    S = W.Scene(specT)
    st, mean, var = _timed_solve(W, S, d, n, walks, eps, 6, W.make_opts(tikhonov_sigma=0.2, tikhonov_steps=10),
                                 m, v)
    u = specT.exact(pts)
    dev = (mean - u) - np.mean(mean - u)
    record("tikhonov_pure_neumann", None, st, mean, var,
           {"rms_error_up_to_constant": float(np.sqrt(np.mean(dev ** 2)))})
    # double-sided sheets in a square of 8192 one-sided Dirichlet segments: an
    # open curved sheet of 8192 segments (30 % Dirichlet, 70 % Neumann, data
    # from one harmonic u on both sides), and a closed circle of 8192
    # segments with different solutions inside and outside
    for name, specS, seed in (("double_sided_open_sheet", I.crack_scene_2d(n_crack=8192, n_side=2048), 7),
                              ("double_sided_closed_circle", I.double_sided_disk_scene(n_circle=8192, n_side=2048), 8)):
        S = W.Scene(specS)
        pts = I.box_points(n, 2, seed, half=0.9, avoid_radius=0.5 if "circle" in name else None, margin=0.01)
        d = torch.from_numpy(pts).cuda()
        st, mean, var = _timed_solve(W, S, d, n, walks, eps, seed, None, m, v)
        # the one-sided kernels on the same geometry (sheets flagged one-sided:
        # other walks and wrong data on the "-" side), for the cost per step
        S1 = W.Scene(I.dataclasses.replace(specS, bc=(specS.bc & 1).astype(np.uint8)))
        st1, _, _ = _timed_solve(W, S1, d, n, walks, eps, seed, None, m, v)
        record(name, specS.exact(pts), st, mean, var,
               {"one_sided_kernel_same_geometry_steps_per_s": st1.steps / (st1.kernel_ms / 1e3)})
    print(json.dumps(out), flush=True)


def bench_sweep(a):
    """r_min / eps sweep on the star polygon (the paper's study of the
    eps-shell and minimum-radius trade-off): steps per walk, throughput and
    the error against the exact solution for each setting."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    n, walks = min(a.points, 65536), a.walks
    cfg = I.star_polygon_case(n_points=n, walks=walks)
    spec, pts = cfg["scene"], cfg["points"]
    S = W.Scene(spec)
    d = torch.from_numpy(pts).cuda()
    m = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    u = spec.exact(pts)
    rows = []
    for eps in (1e-2, 1e-3, 1e-4, 1e-5):
        for rmin_f in (1.0, 10.0, 100.0):
            st, mean, var = _timed_solve(W, S, d, n, walks, eps, 7, W.make_opts(r_min=eps * rmin_f), m, v)
            se = np.sqrt(var / walks)
            rows.append({"eps": eps, "r_min": eps * rmin_f, "steps_per_walk": st.steps / st.walks,
                         "steps_per_s": st.steps / (st.kernel_ms / 1e3), "points_per_s": n / (st.kernel_ms / 1e3),
                         "bias": float(np.mean(mean - u)), "bias_se": float(np.sqrt(np.sum(var / walks))) / n,
                         "rmse": float(np.sqrt(np.mean((mean - u) ** 2))), "se_rms": float(np.sqrt(np.mean(se ** 2)))})
            log(f"eps {eps:g} r_min {eps * rmin_f:g}: {rows[-1]['steps_per_walk']:.1f} steps/walk, "
                f"bias {rows[-1]['bias']:.2e}")
    print(json.dumps({"workload": "r_min / eps sweep, 2D star polygon (16384 segments)", "points": n,
                      "walks_per_point": walks, "rows": rows}), flush=True)


def bench_icosphere(a):
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    npts = min(a.points, 1_000_000) if a.points != 262144 else 1_000_000
    walks = max(1, 512 // a.walk_div)
    mesh = I.displaced_icosphere(8, 0)
    spec = I.displaced_icosphere_scene(8, 0, mesh=mesh)
    pts = I.radial_mesh_points(mesh, npts, 0)
    S = W.Scene(spec)
    log(f"icosphere scene built: {spec.n_prims} triangles, {npts} points x {walks} walks")
    d = torch.from_numpy(pts).cuda()
    m = torch.empty(npts, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    out = {"workload": "3D displaced icosphere, 1310720 triangles (55% Neumann), Poisson f=1",
           "points": npts, "walks_per_point": walks, "walk_div": a.walk_div}
    for mode, name in ((0, "persistent"), (1, "plain")):
        W.wost_solve_ex(S.handle, d, npts, walks, 1e-4, 0, 0, 0, W.make_opts(mode=mode), m, v, None)
        st = W.wost_get_stats(S.handle)
        out[name] = {"steps_per_s": st.steps / (st.kernel_ms / 1e3), "kernel_ms": st.kernel_ms,
                     "points_per_s": npts / (st.kernel_ms / 1e3), "steps_per_walk": st.steps / st.walks,
                     "capped": st.capped, "escaped": st.escaped}
        log(f"{name}: {st.kernel_ms:.0f} ms, {st.steps / (st.kernel_ms / 1e3):.3g} steps/s")
    mean, var = m.cpu().numpy(), v.cpu().numpy()
    u = spec.exact(pts)
    se = np.sqrt(var / walks)
    V = spec.vertices.astype(np.float64)
    gmax = float(np.linalg.norm(np.stack([V[:, 0] / 3 + V[:, 1], V[:, 1] / 3 + V[:, 0], V[:, 2] / 3], 1), axis=1).max())
    out.update({"se_median": float(np.median(se)), "exact_bias": float(np.mean(mean - u)),
                "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mean - u) > 4 * se + 1e-4 * gmax))})
    W.wost_solve_ex(S.handle, d, min(npts, 8192), walks, 1e-4, 0, 0, 0, W.make_opts(flags=1), m, v, None)
    tr = W.wost_get_traffic(S.handle)
    stc = W.wost_get_stats(S.handle)
    out["bytes_per_step"] = tr.bytes / stc.steps
    out["achieved_gbs"] = out["bytes_per_step"] * out["persistent"]["steps_per_s"] / 1e9
    print(json.dumps(out), flush=True)


def bench_mixed(a):
    """Mixed representations (the paper's heat scene with a 1.2M-element
    Neumann mesh on rocks given as signed distance functions, evaluated at
    285k boundary points with 1024 walks): the 1,310,720-triangle displaced
    icosphere as a Neumann obstacle on 16 analytic rocks inside a Dirichlet
    ball, 285,000 points on the mesh, 1024 / walk_div walks each."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    spec = I.mixed_scene(level=8, seed=0)
    npts = 285_000
    walks = max(1, 1024 // a.walk_div)
    pts, prims = I.neumann_boundary_points(spec, npts, seed=2)
    S = W.Scene(spec)
    log(f"mixed scene built: {spec.n_prims} triangles, {len(spec.sdf)} shapes, {npts} boundary points x {walks} walks")
    d = torch.from_numpy(pts).cuda()
    m = torch.empty(npts, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    eps = 1e-4
    st, mean, var = _timed_solve(W, S, d, npts, walks, eps, 0, None, m, v, prims=prims)
    u = spec.exact(pts)
    se = np.sqrt(var / walks)
    out = {"workload": "mixed: 1310720-triangle Neumann mesh on 16 analytic rocks in a Dirichlet ball, "
                       "285000 boundary points", "walks_per_point": walks, "walk_div": a.walk_div, "eps": eps,
           "steps_per_s": st.steps / (st.kernel_ms / 1e3), "kernel_ms": st.kernel_ms,
           "walks_per_s": st.walks / (st.kernel_ms / 1e3), "steps_per_walk": st.steps / st.walks,
           "us_per_walk": st.kernel_ms * 1e3 / st.walks, "capped": st.capped, "escaped": st.escaped,
           "se_median": float(np.median(se)), "exact_bias": float(np.mean(mean - u)),
           "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mean - u) > 4 * se + eps * 8.0))}
    log(f"mixed: {out['steps_per_s']:.3g} steps/s, {out['steps_per_walk']:.1f} steps/walk")
    print(json.dumps(out), flush=True)


def bench_geodesic_batch(a):
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    cfg = I.geodesic_batch_case()
    items = []
    for c in cfg:
        S = W.Scene(c["scene"])
        n = len(c["points"])
        items.append(dict(S=S, d=torch.from_numpy(c["points"]).cuda(), n=n, wk=max(1, c["walks"] // a.walk_div),
                          eps=c["eps"], seed=c["seed"], m=torch.zeros(n, dtype=torch.float64, device="cuda"),
                          v=torch.zeros(n, dtype=torch.float64, device="cuda")))
    npts = sum(i["n"] for i in items)
    out = {"workload": "64 displaced geodesic spheres (2k-800k triangles), per-scene points and walks",
           "triangles": int(sum(c["scene"].n_prims for c in cfg)), "points": npts,
           "walks": int(sum(i["n"] * i["wk"] for i in items)), "walk_div": a.walk_div}
    for mode, name in ((0, "per_scene_persistent"), (1, "per_scene_plain")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for it in items:
            W.wost_solve_ex(it["S"].handle, it["d"], it["n"], it["wk"], it["eps"], it["seed"], 0, 0,
                            W.make_opts(mode=mode), it["m"], it["v"], None)
            steps += W.wost_get_stats(it["S"].handle).steps
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "steps_per_s": steps / dt, "points_per_s": npts / dt}
        log(f"{name}: {dt:.1f} s")
    ref = [it["m"].cpu().numpy().copy() for it in items]
    B = W.wost_batch_create()
    bitems = [W.make_batch_item(it["S"].handle, it["d"], it["n"], it["wk"], it["eps"], it["seed"], it["m"], it["v"])
              for it in items]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W.wost_solve_batch(B, bitems, None)
    st = W.wost_batch_get_stats(B)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["batched"] = {"seconds": dt, "steps_per_s": st.steps / dt, "points_per_s": npts / dt,
                      "identical_to_per_scene": bool(all(np.array_equal(it["m"].cpu().numpy(), r)
                                                         for it, r in zip(items, ref)))}
    log(f"batched: {dt:.1f} s")
    W.wost_batch_destroy(B)
    print(json.dumps(out), flush=True)


def bench_serving(a):
    """Serving over a pool of displaced-icosphere scenes: Poisson arrivals at --rate for
    --window seconds, each request a uniform scene, 1..65536 fresh interior
    points (log-uniform) and a target SE in [1e-3, 1e-2] (log-uniform)."""
    import math
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    rng = np.random.Generator(np.random.PCG64(5))
    pool, pts_pool = [], []
    for s in range(a.pool):
        mesh = I.displaced_icosphere(8, s)
        pool.append(W.Scene(I.displaced_icosphere_scene(8, s, mesh=mesh)))
        pts_pool.append(I.radial_mesh_points(mesh, 65536, 100 + s))
        log(f"scene {s} ready")
    cfg = W.make_server_config(max_device_bytes=int(a.budget_mb * 2 ** 20), round_walks=64, min_walks=64,
                               max_walks=65536, adaptive=0 if a.fixed_rounds else 1, max_round_walks=4096)
    srv = W.wost_server_create(cfg)
    arrivals = np.cumsum(rng.exponential(1.0 / a.rate, int(a.rate * a.window * 1.5) + 10))
    arrivals = arrivals[arrivals < a.window]
    reqs = []
    for t in arrivals:
        sc = int(rng.integers(0, a.pool))
        n = int(round(math.exp(rng.uniform(0, math.log(a.max_points)))))
        tau = math.exp(rng.uniform(math.log(a.se_lo), math.log(a.se_hi)))
        off = int(rng.integers(0, 65536 - n + 1))
        reqs.append((t, sc, n, tau, off))
    t0 = time.perf_counter()
    ids, k, rounds = [], 0, 0
    queue_len = []
    while True:
        now = time.perf_counter() - t0
        while k < len(reqs) and reqs[k][0] <= now:
            t, sc, n, tau, off = reqs[k]
            ids.append((W.wost_server_submit(srv, pool[sc].handle, pts_pool[sc][off:off + n], 1e-4, 1000 + k, tau), n))
            k += 1
        n_open = W.wost_server_step(srv)
        rounds += 1
        queue_len.append((round(now, 2), n_open))
        if now > a.window + a.drain or (k == len(reqs) and n_open == 0):
            break
        if n_open == 0 and k < len(reqs):
            time.sleep(max(0.0, min(0.05, reqs[k][0] - (time.perf_counter() - t0))))
    elapsed = time.perf_counter() - t0
    lat, done_pts, done_walks, rdone = [], 0, 0, []
    states = {0: 0, 1: 0, 2: 0, 3: 0}
    for rid, n in ids:
        info, _, _ = W.wost_server_poll(srv, rid)
        states[info.state] += 1
        if info.state == W.REQ_DONE:
            lat.append(info.t_done_ms - info.t_submit_ms)
            rdone.append(info.rounds)
            done_pts += n
        done_walks += n * info.walks_per_point
    W.wost_server_destroy(srv)
    lat = np.array(lat) if lat else np.array([np.nan])
    rounds_done = float(np.mean(rdone)) if rdone else None
    out = {"workload": "serving: pool of %d displaced-icosphere scenes (1.3M triangles each), Poisson %g req/s for %g s, "
                       "1..%d points, target SE %g..%g" % (a.pool, a.rate, a.window, a.max_points, a.se_lo, a.se_hi),
           "submitted": len(ids), "done": states[2], "active_at_end": states[1], "queued_at_end": states[0],
           "rejected": states[3], "elapsed_s": elapsed, "rounds": rounds,
           "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
           "points_done_per_s": done_pts / elapsed, "walks_per_s": done_walks / elapsed,
           "open_requests_timeline": queue_len[:: max(1, len(queue_len) // 20)], "budget_mb": a.budget_mb,
           "adaptive_rounds": not a.fixed_rounds, "rounds_per_done_request": rounds_done}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
