"""Walk-on-stars throughput on one MI355X.

Default workload (the largest single-GPU configuration): 3D Poisson in the
1,310,720-triangle displaced icosphere (55 % Neumann, exact
u = (x^2 + y^2 + z^2)/6 + xy, f = 1), 1,000,000 interior points, 512 walks
per point, eps = 1e-4.  One "step" is one slice of 62,500 points (1/16 of
the point set) solved completely: all 512 walks of each of its points, from
the points resident in HBM to their FP64 mean and variance in HBM, with the
random-number point ids of the full solve, so that K steps are exactly K
slices of the full 10^6-point solve.

Prints one JSON line: walk steps/s (the metric), points/s at the measured
standard error, capped and escaped walk counts, the walk kernel's roofline
figures, the one-lane-per-walk launch on the same points, a star-polygon
leg (the 2D workload: 16,384 segments, 262,144 points x 1024 walks), a
unit-square leg (1,024 points x 256 walks) against the vector-ALU roofline,
and the FP64 oracle's throughput on the host cores for a bounded sample of
the headline workload.  --full adds one solve of all 10^6 points.

Other workloads (--workload): star2d (the star polygon alone, with the
per-lane form), geodesic64 (64 scenes: batched launch vs per-scene
launches), serving (Poisson arrivals over a pool of icosphere scenes,
progressive refinement, latency percentiles), and the extensions, sweep
and mixed studies; each prints its own JSON line.
"""
import argparse
import json
import math
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
    ap.add_argument("--workload", default="icosphere3d",
                    choices=["star2d", "icosphere3d", "geodesic64", "serving", "extensions", "sweep", "sweep3d", "mixed"])
    ap.add_argument("--batch-points", type=int, default=62500,
                    help="icosphere3d: points per step (a divisor of 10^6)")
    ap.add_argument("--full-chunk", type=int, default=125000,
                    help="icosphere3d --full: points per launch of the full solve")
    ap.add_argument("--full", action="store_true",
                    help="icosphere3d: also solve all 10^6 points x 512 walks; geodesic64: run the batch at "
                         "its full walk counts, as --walk-ranges batched launches over consecutive walk ranges")
    ap.add_argument("--walk-ranges", type=int, default=8,
                    help="geodesic64 --full: batched launches, each over 1/this of every item's walks")
    ap.add_argument("--no-legs", action="store_true", help="icosphere3d: skip the star-polygon and unit-square legs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="icosphere3d: time the default launch options instead of the autotuned ones")
    ap.add_argument("--tune-walks", type=int, default=1 << 21, help="icosphere3d: walks per autotuner trial")
    ap.add_argument("--walk-div", type=int, default=1,
                    help="icosphere3d/geodesic64: divide every walk count by this (stated in the output)")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: arrivals per second")
    ap.add_argument("--window", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--drain", type=float, default=60.0, help="serving: extra seconds to finish work")
    ap.add_argument("--budget-mb", type=float, default=16384.0, help="serving: admission budget (MiB)")
    ap.add_argument("--rounds-in-flight", type=int, default=2, help="serving: rounds in flight at once")
    ap.add_argument("--pool", type=int, default=8, help="serving: scenes in the pool")
    ap.add_argument("--max-points", type=int, default=65536, help="serving: largest request (points)")
    ap.add_argument("--se-lo", type=float, default=1e-3, help="serving: smallest target SE")
    ap.add_argument("--se-hi", type=float, default=1e-2, help="serving: largest target SE")
    ap.add_argument("--fixed-rounds", action="store_true",
                    help="serving: 64 walks per point every round instead of rounds sized from the request's "
                         "standard error (up to 4096 walks per point, within the round budget)")
    ap.add_argument("--max-active", type=int, default=256,
                    help="serving: requests admitted at once (the rest queue)")
    ap.add_argument("--round-budget", type=int, default=1 << 22,
                    help="serving: walks per round over all its requests (a request larger than this runs alone)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=262144)
    ap.add_argument("--walks", type=int, default=1024)
    ap.add_argument("--count-points", type=int, default=16384,
                    help="points of the traffic-accounting solve (a prefix of the workload)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="oracle threads: the host cores this process may use, at most this many "
                         "(the GPU box's share of cores for one GPU is 16)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


PROFILE_C2 = os.path.join(ROOT, "profiles", "k_walk_persistent_2d_star_262144x1024.md")
PROFILE_C3 = os.path.join(ROOT, "profiles", "k_walk_persistent_3d_icosphere_slice_62500x512.md")
PROFILE_C1 = os.path.join(ROOT, "profiles", "k_walk_persistent_2d_unit_square_1024x256.md")
# vector-ALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
# (a wave64 instruction occupies a SIMD for 4 clocks), in giga lane-instructions/s
VALU_PEAK_GLANES = 256 * 4 * 16 * 2.4


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("wost_device.hpp", "wost_walks.hip", "wost_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2302_11815_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_value(path, key):
    """A figure from a committed rocprofv3 summary ("key: value" lines), or
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
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def profiled_traffic(path):
    """HBM bytes per launch of the walk kernel (FETCH_SIZE + WRITE_SIZE, scaled
    by a 1 GiB copy) from a committed summary, or None (see profiled_value)."""
    return profiled_value(path, "traffic_bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec, pts, walks, eps, seed, seconds, threads, walks_per_point=16):
    """The FP64 brute-force oracle on a growing prefix of the workload (its
    points with their own random-number ids, walks_per_point walks each)
    until about `seconds` of wall time; steps/s of that sample.  It runs on
    the host cores this process may use, at most `threads` of them."""
    import oracle as O
    R = O.Scene(spec)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    nthreads = max(1, min(threads, avail))
    n = nthreads
    w = walks_per_point
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
            "walks_per_s": n * w / dt, "host_cpus": os.cpu_count(), "cpus_available": avail}


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
    if a.workload == "sweep3d":
        return bench_sweep3d(a)
    out = star_polygon_leg(a, a.steps, a.warmup, per_lane=not a.no_plain)
    out.update({"n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"})
    cfg = I_star_cfg(a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg["scene"], cfg["points"], cfg["walks"], cfg["eps"], cfg["seed"],
                                           a.cpu_seconds, a.cpu_threads)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3g} steps/s on {out['cpu_baseline']['cores']} threads")
    if a.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


_STAR_CFG = {}


def I_star_cfg(a):
    """The star-polygon workload (built once)."""
    if "cfg" not in _STAR_CFG:
        from paper_2302_11815_amd import inputs as I
        _STAR_CFG["cfg"] = I.star_polygon_case(n_points=a.points, walks=a.walks)
    return _STAR_CFG["cfg"]


def star_polygon_leg(a, steps, warmup, plain=True, per_lane=False, counting=True):
    """The 2D star polygon (16,384 segments, 262,144 points x 1024 walks):
    `steps` whole solves timed after `warmup`, the one-lane-per-walk launch
    on the same points, and the walk kernel against the L2 roofline (its
    trees stay in L2)."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    cfg = I_star_cfg(a)
    spec, pts, Wk, eps, seed = cfg["scene"], cfg["points"], cfg["walks"], cfg["eps"], cfg["seed"]
    S = W.Scene(spec)
    n = pts.shape[0]
    d_pts = torch.from_numpy(pts).cuda()
    d_mean = torch.empty(n, dtype=torch.float64, device="cuda")
    d_var = torch.empty_like(d_mean)
    stream = torch.cuda.current_stream()
    opts = W.make_opts(mode=0)
    log(f"star polygon: {spec.n_prims} segments, {S.info.n_neumann} Neumann; {n} points x {Wk} walks")

    def solve(o, npts=n):
        W.wost_solve_ex(S.handle, d_pts, npts, Wk, eps, seed, 0, 0, o, d_mean, d_var, stream.cuda_stream)
        return W.wost_get_stats(S.handle)

    for i in range(warmup):
        st = solve(opts)
        log(f"star warmup {i}: {st.kernel_ms:.1f} ms, {st.steps} steps, grid {st.grid_blocks}")
    steps_total = capped = escaped = 0
    kms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = solve(opts)
        steps_total += st.steps
        capped += st.capped
        escaped += st.escaped
        kms.append(st.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"star timed: {steps} solves in {dt:.2f} s; walk kernel {np.mean(kms):.1f} ms")
    mean = d_mean.cpu().numpy()
    var = d_var.cpu().numpy()
    se = np.sqrt(var / Wk)
    u = spec.exact(pts)
    pos = se > 0
    z = (mean[pos] - u[pos]) / se[pos]
    eps_bound = float(eps * np.exp(spec.vertices[:, 0].astype(np.float64).max()))
    steps_per_solve = steps_total / steps
    kernel_s = float(np.mean(kms)) / 1e3
    plain_r = per_lane_r = None
    if plain:
        stp = solve(W.make_opts(mode=1))
        plain_r = {"steps_per_s": stp.steps / (stp.kernel_ms / 1e3), "kernel_ms": stp.kernel_ms,
                   "points_per_s": n / (stp.kernel_ms / 1e3),
                   "identical_estimates": bool(np.array_equal(d_mean.cpu().numpy(), mean))}
        log(f"star plain launch: {stp.kernel_ms:.1f} ms (identical estimates: {plain_r['identical_estimates']})")
    if per_lane:
        stl = solve(W.make_opts(mode=2))
        per_lane_r = {"steps_per_s": stl.steps / (stl.kernel_ms / 1e3), "kernel_ms": stl.kernel_ms,
                      "identical_estimates": bool(np.array_equal(d_mean.cpu().numpy(), mean))}
    roof = None
    if counting:
        nc = min(a.count_points, n)
        solve(W.make_opts(flags=W.WOST_SOLVE_COUNT_TRAFFIC), nc)
        tr = W.wost_get_traffic(S.handle)
        stc = W.wost_get_stats(S.handle)
        bytes_per_step = tr.bytes / stc.steps
        achieved = bytes_per_step * steps_per_solve / kernel_s / 1e9
        l2_stream = max(W.wost_measure_l2_read(2 << 20, 16) for _ in range(3))
        fetch = {k: getattr(tr, k) / stc.steps for k in ("q1_nodes", "q1_prims", "q2_nodes", "q2_cones",
                                                           "q2_elems", "q3_nodes", "q3_prims", "q4_nodes",
                                                           "q4_prims", "vis_nodes", "vis_prims")}
        traffic = profiled_traffic(PROFILE_C2) if (n, Wk) == (262144, 1024) else None
        roof = {"bound": "l2", "achieved": achieved, "peak": L2_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / L2_PEAK_GBS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                "bytes_per_step": bytes_per_step, "kernel_ms": float(np.mean(kms)), "fetches_per_step": fetch,
                "l2_stream_gbs": l2_stream, "frac_of_l2_stream": achieved / l2_stream,
                "valu": valu_issue(PROFILE_C2 if (n, Wk) == (262144, 1024) else None, steps_per_solve / kernel_s)}
        log(f"star roofline: {achieved:.0f} GB/s of algorithmic bytes ({bytes_per_step:.0f} B/step), "
            f"L2 stream {l2_stream:.0f} GB/s")
    return {
        "metric": "walk steps/s", "value": steps_total / dt, "unit": "steps/s", "ms_per_step": 1000 * dt / steps,
        "config": {"workload": "2D star polygon Laplace: 16384 segments (50% Neumann), "
                               f"{n} points x {Wk} walks, eps 1e-4",
                   "points": n, "walks_per_point": Wk,
                   "form": "persistent lane-refill kernel, wave-cooperative tree searches"},
        "points_per_s": n * steps / dt, "walks_per_s": n * Wk * steps / dt,
        "se_median": float(np.median(se)), "se_p90": float(np.percentile(se, 90)),
        "mean_steps_per_walk": steps_per_solve / (n * Wk), "capped": capped, "escaped": escaped,
        "exact_error_rmse": float(np.sqrt(np.mean((mean - u) ** 2))), "exact_bias": float(np.mean(mean - u)),
        "z_beyond_4": int(np.sum(np.abs(z) > 4)), "z_allowed": 2 * z.size * 6.33e-5 + 3,
        "z_rule_met": bool(np.sum(np.abs(z) > 4) <= 2 * z.size * 6.33e-5 + 3),
        # a walk stops within eps of the Dirichlet boundary and returns g at
        # the closest point, so each estimate carries a bias of at most
        # eps * sup|grad u| (here sup e^x over the domain)
        "eps_shell_bound": eps_bound,
        "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mean - u) > 4 * se + eps_bound)),
        "plain": plain_r, "persistent_per_lane": per_lane_r, "roofline": roof,
    }


_VALU_STREAMS = {}


def valu_issue(profile, steps_per_s):
    """VALU lane instructions per second of a walk kernel (steps/s x the
    committed profile's VALU wave instructions per step x 64), beside the
    issue rates measured here for FP32 FMA chains and integer xor + add
    chains (the kernels mix both; integer work issues faster)."""
    from paper_2302_11815_amd import wost as W
    if not _VALU_STREAMS:
        _VALU_STREAMS["fp32"] = max(W.wost_measure_valu(0, 1024) for _ in range(3))
        _VALU_STREAMS["int"] = max(W.wost_measure_valu(1, 1024) for _ in range(3))
    per_step = profiled_value(profile, "valu_instructions_per_step") if profile else None
    achieved = steps_per_s * per_step * 64 / 1e9 if per_step else None
    return {"valu_instructions_per_step": per_step, "achieved_glanes": achieved,
            "stream_fp32_glanes": _VALU_STREAMS["fp32"], "stream_int_glanes": _VALU_STREAMS["int"],
            "frac_of_fp32_stream": achieved / _VALU_STREAMS["fp32"] if achieved else None,
            "frac_of_int_stream": achieved / _VALU_STREAMS["int"] if achieved else None}


def unit_square_leg(a):
    """The unit square (4 segments, 1,024 points x 256 walks, eps 1e-3):
    every byte it reads stays in the caches, so the vector ALU bounds it;
    reported against the VALU issue roofline with the VALU instructions per
    step of the committed counter profile."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    c = I.unit_square_case()
    S = W.Scene(c["scene"])
    n = c["points"].shape[0]
    d = torch.from_numpy(c["points"]).cuda()
    m = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    runs = []
    for _ in range(6):
        W.wost_solve_ex(S.handle, d, n, c["walks"], c["eps"], c["seed"], 0, 0, None, m, v, None)
        runs.append(W.wost_get_stats(S.handle))
    st = sorted(runs[1:], key=lambda r: r.kernel_ms)[len(runs[1:]) // 2]
    mean, var = m.cpu().numpy(), v.cpu().numpy()
    u = c["scene"].exact(c["points"])
    se = np.sqrt(u * (1 - u) / c["walks"])
    steps_s = st.steps / (st.kernel_ms / 1e3)
    valu = profiled_value(PROFILE_C1, "valu_instructions_per_step")
    achieved = steps_s * valu * 64 / 1e9 if valu else None
    vi = valu_issue(PROFILE_C1, steps_s)
    out = {"workload": "2D unit square Laplace: 4 segments, 1024 points x 256 walks, eps 1e-3",
           "steps_per_s": steps_s, "kernel_ms": st.kernel_ms, "points_per_s": n / (st.kernel_ms / 1e3),
           "steps_per_walk": st.steps / st.walks, "capped": st.capped, "escaped": st.escaped,
           "z_beyond_4": int(np.sum(np.abs(mean - u) > 4 * se)),
           "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GLANES, "unit": "Glane-instr/s",
                        "frac": achieved / VALU_PEAK_GLANES if achieved else None,
                        "valu_instructions_per_step": valu, "valu_stream_fp32_glanes": vi["stream_fp32_glanes"],
                        "valu_stream_int_glanes": vi["stream_int_glanes"],
                        "frac_of_fp32_stream": vi["frac_of_fp32_stream"], "frac_of_int_stream": vi["frac_of_int_stream"]}}
    log(f"unit square: {steps_s:.3g} steps/s, {st.kernel_ms:.2f} ms")
    return out


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


def bench_sweep3d(a):
    """r_min / eps sweep on the displaced icosphere (1,310,720 triangles):
    15,625 of its points x 128 walks per setting; steps per walk, throughput
    and the error against the exact solution."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    n, walks = 15625, 128
    mesh = I.displaced_icosphere(8, 0)
    spec = I.displaced_icosphere_scene(8, 0, mesh=mesh)
    pts = I.radial_mesh_points(mesh, n, 0)
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
                         "capped": st.capped, "escaped": st.escaped,
                         "bias": float(np.mean(mean - u)), "bias_se": float(np.sqrt(np.sum(var / walks))) / n,
                         "rmse": float(np.sqrt(np.mean((mean - u) ** 2))), "se_rms": float(np.sqrt(np.mean(se ** 2)))})
            log(f"eps {eps:g} r_min {eps * rmin_f:g}: {rows[-1]['steps_per_walk']:.1f} steps/walk, "
                f"{rows[-1]['steps_per_s']:.3g} steps/s, bias {rows[-1]['bias']:.2e} +- {rows[-1]['bias_se']:.1e}")
    print(json.dumps({"workload": "r_min / eps sweep, 3D displaced icosphere (1310720 triangles)", "points": n,
                      "walks_per_point": walks, "rows": rows}), flush=True)


def bench_icosphere(a):
    """The headline: slices of the 10^6-point displaced-icosphere solve."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    N_ALL, Wk, eps, seed = 1_000_000, max(1, 512 // a.walk_div), 1e-4, 0
    B = a.batch_points
    assert N_ALL % B == 0, "--batch-points must divide 10^6"
    n_slices = N_ALL // B
    need = N_ALL if a.full else min(N_ALL, (a.warmup + a.steps) * B)
    mesh = I.displaced_icosphere(8, 0)
    spec = I.displaced_icosphere_scene(8, 0, mesh=mesh)
    pts = I.radial_mesh_points(mesh, need, seed)
    log(f"icosphere: {spec.n_prims} triangles, {need} of {N_ALL} points generated "
        f"({time.perf_counter() - t_start:.0f} s)")
    t_b = time.perf_counter()
    S = W.Scene(spec)
    log(f"scene built and uploaded in {time.perf_counter() - t_b:.1f} s")
    d_pts = torch.from_numpy(pts).cuda()
    d_mean = torch.empty(need, dtype=torch.float64, device="cuda")
    d_var = torch.empty_like(d_mean)
    stream = torch.cuda.current_stream()
    have = need // B   # slices whose points exist

    def slice_solve(k, opts=None, npts=B):
        j = k % have
        lo = j * B
        W.wost_solve_ex(S.handle, d_pts[lo:lo + npts], npts, Wk, eps, seed, lo, 0, opts, d_mean[lo:lo + npts],
                        d_var[lo:lo + npts], stream.cuda_stream)
        return W.wost_get_stats(S.handle)

    # launch options: the autotuner's choice on the first points, outside the
    # timed region (every candidate gives the same bits)
    tuned = None
    if not a.no_autotune:
        t_t = time.perf_counter()
        tuned = W.wost_autotune(S.handle, d_pts, need, Wk, eps, seed, sample_walks=a.tune_walks,
                                stream=stream.cuda_stream)
        tuned_info = {k: getattr(tuned, k) for k in ("refill", "grid", "walk_order", "claim_walks", "steal_lanes")}
        tuned_info["seconds"] = time.perf_counter() - t_t
        tuned_info["sample_walks"] = a.tune_walks
        log(f"autotuned in {tuned_info['seconds']:.0f} s: {tuned_info}")
        # the tuner's sample is a quarter of a step: confirm its choice on a
        # whole slice against the default options (same bits either way)
        st_d = slice_solve(0, None)
        st_t = slice_solve(0, tuned)
        tuned_info["confirm_ms"] = {"defaults": st_d.kernel_ms, "tuned": st_t.kernel_ms}
        if st_t.kernel_ms >= st_d.kernel_ms:
            tuned = None
            tuned_info["kept"] = "defaults"
        else:
            tuned_info["kept"] = "tuned"
        log(f"on a whole slice: defaults {st_d.kernel_ms:.0f} ms, tuned {st_t.kernel_ms:.0f} ms: "
            f"keeping {tuned_info['kept']}")
    for i in range(a.warmup):
        st = slice_solve(i, tuned)
        log(f"warmup {i}: {st.kernel_ms:.0f} ms, {st.steps / st.kernel_ms * 1e3:.3g} steps/s")
    steps_total = walks_total = capped = escaped = 0
    kms, ksteps, timed = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        k = a.warmup + i
        st = slice_solve(k, tuned)
        steps_total += st.steps
        walks_total += st.walks
        capped += st.capped
        escaped += st.escaped
        kms.append(st.kernel_ms)
        ksteps.append(st.steps)
        timed.append(k % have)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed: {a.steps} slices in {dt:.2f} s; walk kernel {np.mean(kms):.0f} ms per slice")
    # accuracy over the timed slices' points
    idx = np.concatenate([np.arange(j * B, (j + 1) * B) for j in sorted(set(timed))])
    mean, var = d_mean.cpu().numpy()[idx], d_var.cpu().numpy()[idx]
    u = spec.exact(pts[idx])
    se = np.sqrt(var / Wk)
    V = spec.vertices.astype(np.float64)
    gmax = float(np.linalg.norm(np.stack([V[:, 0] / 3 + V[:, 1], V[:, 1] / 3 + V[:, 0], V[:, 2] / 3], 1),
                                axis=1).max())
    pos = se > 0
    z = (mean[pos] - u[pos]) / se[pos]
    kernel_s = float(np.mean(kms)) / 1e3
    steps_per_launch = float(np.mean(ksteps))
    # the one-lane-per-walk launch and the chosen form on the same 1,024 points
    ref = slice_solve(0, None, 1024)
    stp = slice_solve(0, W.make_opts(mode=1), 1024)
    plain = {"points": 1024, "steps_per_s": stp.steps / (stp.kernel_ms / 1e3), "kernel_ms": stp.kernel_ms,
             "persistent_steps_per_s_same_points": ref.steps / (ref.kernel_ms / 1e3)}
    log(f"plain launch (1024 points): {plain['steps_per_s']:.3g} steps/s against "
        f"{plain['persistent_steps_per_s_same_points']:.3g}")
    # algorithmic bytes per step: the counting variant on 1,024 points x 64 walks of slice 0
    W.wost_solve_ex(S.handle, d_pts[:1024], 1024, 64, eps, seed, 0, 0, W.make_opts(flags=W.WOST_SOLVE_COUNT_TRAFFIC),
                    d_mean[:1024], d_var[:1024], stream.cuda_stream)
    tr = W.wost_get_traffic(S.handle)
    stc = W.wost_get_stats(S.handle)
    bytes_per_step = tr.bytes / stc.steps
    achieved = bytes_per_step * steps_per_launch / kernel_s / 1e9
    traffic = profiled_traffic(PROFILE_C3) if (B, Wk) == (62500, 512) else None
    fetch = {k: getattr(tr, k) / stc.steps for k in ("q1_nodes", "q1_prims", "q2_nodes", "q2_cones", "q2_elems",
                                                       "q3_nodes", "q3_prims", "q4_nodes", "q4_prims",
                                                       "vis_nodes", "vis_prims")}
    log(f"roofline: {achieved:.0f} GB/s of algorithmic bytes ({bytes_per_step:.0f} B/step) against "
        f"{HBM_PEAK_GBS:.0f} GB/s")
    rate = steps_total / dt
    full = None
    if a.full:
        # all 10^6 points in launches of --full-chunk points (each with its
        # own point_base, so the walks are those of one launch), logging
        # after each
        C = a.full_chunk
        assert N_ALL % C == 0, "--full-chunk must divide 10^6"
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f_ms, f_steps, f_capped, f_escaped = 0.0, 0, 0, 0
        for lo in range(0, N_ALL, C):
            W.wost_solve_ex(S.handle, d_pts[lo:lo + C], C, Wk, eps, seed, lo, 0, None, d_mean[lo:lo + C],
                            d_var[lo:lo + C], stream.cuda_stream)
            stc = W.wost_get_stats(S.handle)
            f_ms += stc.kernel_ms
            f_steps += stc.steps
            f_capped += stc.capped
            f_escaped += stc.escaped
            log(f"full solve: points {lo}..{lo + C} done, walk kernel {stc.kernel_ms / 1e3:.1f} s")
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t1
        mf, vf = d_mean.cpu().numpy(), d_var.cpu().numpy()
        uf = spec.exact(pts)
        sef = np.sqrt(vf / Wk)
        full = {"points": N_ALL, "walks_per_point": Wk, "launches": N_ALL // C, "seconds": dtf,
                "kernel_ms": f_ms, "steps_per_s": f_steps / (f_ms / 1e3), "points_per_s": N_ALL / dtf,
                "steps": f_steps, "capped": f_capped, "escaped": f_escaped,
                "exact_bias": float(np.mean(mf - uf)),
                "exact_bias_se": float(np.sqrt(np.sum(vf / Wk))) / N_ALL,
                "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mf - uf) > 4 * sef + eps * gmax))}
        log(f"full solve: {dtf:.0f} s, {full['steps_per_s']:.3g} steps/s")
    else:
        est = steps_per_launch * n_slices / rate
        full = {"skipped": f"one launch over all 10^6 points takes about {est:.0f} s at the measured rate "
                           "(run bench.py --full)", "estimated_seconds": est}
    legs = {}
    if not a.no_legs:
        legs["star2d"] = star_polygon_leg(a, 1, 1, plain=True, per_lane=False, counting=True)
        legs["unit_square"] = unit_square_leg(a)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(spec, pts, Wk, eps, seed, a.cpu_seconds, a.cpu_threads, walks_per_point=1)
        log(f"cpu baseline: {cpu['value']:.3g} steps/s on {cpu['cores']} threads ({cpu['sample']})")
    out = {
        "metric": "walk steps/s", "value": rate, "unit": "steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1000 * dt / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D Poisson in the displaced icosphere: 1310720 triangles (55% Neumann), "
                               f"10^6 points x {Wk} walks, eps 1e-4; one step = {B} points (1/{n_slices} of the "
                               "point set) solved completely",
                   "points_per_step": B, "walks_per_point": Wk,
                   "form": "persistent lane-refill kernel, wave-cooperative tree searches"},
        "points_per_s": B * a.steps / dt, "walks_per_s": walks_total / dt,
        "mean_steps_per_walk": steps_total / walks_total, "capped": capped, "escaped": escaped,
        "se_median": float(np.median(se)), "se_p90": float(np.percentile(se, 90)),
        "exact_bias": float(np.mean(mean - u)), "exact_bias_se": float(np.sqrt(np.sum(var / Wk))) / len(idx),
        "exact_error_rmse": float(np.sqrt(np.mean((mean - u) ** 2))),
        "z_beyond_4": int(np.sum(np.abs(z) > 4)), "z_allowed": 2 * z.size * 6.33e-5 + 3,
        "z_rule_met": bool(np.sum(np.abs(z) > 4) <= 2 * z.size * 6.33e-5 + 3),
        "eps_shell_bound": eps * gmax,
        "beyond_4se_plus_eps_bound": int(np.sum(np.abs(mean - u) > 4 * se + eps * gmax)),
        "plain": plain,
        "launch_options": tuned_info if not a.no_autotune else "defaults",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM and Infinity Cache bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "bytes_per_step": bytes_per_step, "steps_per_launch": steps_per_launch,
                     "kernel_ms": float(np.mean(kms)), "fetches_per_step": fetch},
        "full_solve": full, "legs": legs, "cpu_baseline": cpu,
        "wall_s": time.perf_counter() - t_start,
    }
    if a.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


def copy_calibration():
    """Three device copies of 1 GiB (each reads 1 GiB and writes 1 GiB): the
    reference that scales rocprofv3's FETCH_SIZE and WRITE_SIZE counters."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 3 copies of 1 GiB (fetch 1 GiB, write 1 GiB each)")


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


def bench_geodesic_full(a, cfg):
    """The 64-mesh batch at its full walk counts: every item's walks split
    into consecutive walk ranges (walk_base keeps the random streams of one
    whole launch), one batched graph launch per range, the ranges' FP64
    (n, mean, M2) merged per point with Chan's pairwise formula."""
    import numpy as np
    import torch
    from paper_2302_11815_amd import wost as W
    J = a.walk_ranges
    items = []
    t_b = time.perf_counter()
    for c in cfg:
        n = len(c["points"])
        items.append(dict(S=W.Scene(c["scene"]), d=torch.from_numpy(c["points"]).cuda(), n=n, wk=c["walks"],
                          eps=c["eps"], seed=c["seed"],
                          m=torch.zeros(n, dtype=torch.float64, device="cuda"),
                          v=torch.zeros(n, dtype=torch.float64, device="cuda"),
                          cnt=torch.zeros(n, dtype=torch.float64, device="cuda"),
                          mean=torch.zeros(n, dtype=torch.float64, device="cuda"),
                          m2=torch.zeros(n, dtype=torch.float64, device="cuda")))
    log(f"64 scenes built and uploaded in {time.perf_counter() - t_b:.1f} s")
    npts = sum(i["n"] for i in items)
    walks = int(sum(i["n"] * i["wk"] for i in items))
    B = W.wost_batch_create()
    steps = capped = escaped = 0
    launch_s = []
    for j in range(J):
        bitems = []
        for it in items:
            lo, hi = it["wk"] * j // J, it["wk"] * (j + 1) // J
            it["part"] = hi - lo
            bitems.append(W.make_batch_item(it["S"].handle, it["d"], it["n"], hi - lo, it["eps"], it["seed"],
                                            it["m"], it["v"], walk_base=lo))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W.wost_solve_batch(B, bitems, None)
        st = W.wost_batch_get_stats(B)
        torch.cuda.synchronize()
        launch_s.append(time.perf_counter() - t0)
        steps += st.steps
        capped += st.capped
        escaped += st.escaped
        for it in items:
            nb = float(it["part"])
            m2b = it["v"] * (nb - 1.0)
            na = it["cnt"]
            tot = na + nb
            delta = it["m"] - it["mean"]
            it["mean"] += delta * (nb / tot)
            it["m2"] += m2b + delta * delta * (na * nb / tot)
            it["cnt"] = tot
        log(f"walk range {j + 1} of {J}: {launch_s[-1]:.1f} s, {st.steps / launch_s[-1]:.3g} steps/s")
    W.wost_batch_destroy(B)
    dt = float(sum(launch_s))
    err, ses = [], []
    for c, it in zip(cfg, items):
        mean = it["mean"].cpu().numpy()
        var = it["m2"].cpu().numpy() / (it["wk"] - 1.0)
        err.append(mean - c["scene"].exact(c["points"].astype(np.float64)))
        ses.append(np.sqrt(np.maximum(var, 0.0) / it["wk"]))
    err = np.concatenate(err)
    se = np.concatenate(ses)
    z = err / np.maximum(se, 1e-300)
    # u = x^2 - y^2 + z inside a sphere displaced to radius <= 1.2:
    # |grad u| <= sqrt(4 * 1.2^2 + 1)
    eps_bound = cfg[0]["eps"] * math.sqrt(4 * 1.44 + 1)
    out = {"workload": "64 displaced geodesic spheres (2k-800k triangles), per-scene points and walks, "
                       "full walk counts",
           "triangles": int(sum(c["scene"].n_prims for c in cfg)), "points": npts, "walks": walks,
           "walk_ranges": J,
           "batched": {"seconds": dt, "steps": int(steps), "steps_per_s": steps / dt, "points_per_s": npts / dt,
                       "walks_per_s": walks / dt, "launch_seconds": launch_s,
                       "mean_steps_per_walk": steps / walks, "capped": int(capped), "escaped": int(escaped)},
           "exact_bias": float(np.mean(err)), "exact_error_rmse": float(np.sqrt(np.mean(err ** 2))),
           "z_beyond_4": int(np.sum(np.abs(z) > 4)), "z_allowed": 2 * z.size * 6.33e-5 + 3,
           "eps_shell_bound": eps_bound,
           "beyond_4se_plus_eps_bound": int(np.sum(np.abs(err) > 4 * se + eps_bound)),
           "se_median": float(np.median(se))}
    print(json.dumps(out), flush=True)


def bench_geodesic_batch(a):
    import numpy as np
    import torch
    from paper_2302_11815_amd import inputs as I
    from paper_2302_11815_amd import wost as W
    torch.cuda.set_device(0)
    cfg = I.geodesic_batch_case()
    if a.full:
        if a.walk_div != 1:
            sys.exit("--full runs the full walk counts; drop --walk-div")
        return bench_geodesic_full(a, cfg)
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
    forms = ((0, "per_scene_persistent"),) if a.no_plain else ((0, "per_scene_persistent"), (1, "per_scene_plain"))
    for mode, name in forms:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for k, it in enumerate(items):
            W.wost_solve_ex(it["S"].handle, it["d"], it["n"], it["wk"], it["eps"], it["seed"], 0, 0,
                            W.make_opts(mode=mode), it["m"], it["v"], None)
            steps += W.wost_get_stats(it["S"].handle).steps
            if k % 16 == 15:
                log(f"{name}: {k + 1} of {len(items)} scenes")
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
                               max_walks=65536, adaptive=0 if a.fixed_rounds else 1, max_round_walks=4096,
                               max_active=a.max_active, max_rounds=a.rounds_in_flight,
                               round_budget_walks=a.round_budget)
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
    next_log = 0.0
    while True:
        now = time.perf_counter() - t0
        while k < len(reqs) and reqs[k][0] <= now:
            t, sc, n, tau, off = reqs[k]
            ids.append((W.wost_server_submit(srv, pool[sc].handle, pts_pool[sc][off:off + n], 1e-4, 1000 + k, tau), n))
            k += 1
        n_open = W.wost_server_step(srv)
        rounds += 1
        queue_len.append((round(now, 2), n_open))
        if now >= next_log:
            log(f"serving t={now:.0f} s: {k} submitted, {n_open} open")
            next_log += 5.0
        if now > a.window + a.drain or (k == len(reqs) and n_open == 0):
            break
        if n_open == 0 and k < len(reqs):
            time.sleep(max(0.0, min(0.05, reqs[k][0] - (time.perf_counter() - t0))))
    elapsed = time.perf_counter() - t0
    end_ms = elapsed * 1e3
    lat_done, lat_all, done_pts, done_walks, rdone = [], [], 0, 0, []
    states = {0: 0, 1: 0, 2: 0, 3: 0}
    for rid, n in ids:
        info, _, _ = W.wost_server_poll(srv, rid)
        states[info.state] += 1
        if info.state == W.REQ_DONE:
            lat_done.append(info.t_done_ms - info.t_submit_ms)
            lat_all.append(info.t_done_ms - info.t_submit_ms)
            rdone.append(info.rounds)
            done_pts += n
        elif info.state != W.REQ_REJECTED:
            # unfinished at the end of the run: censored, its latency is at least this
            lat_all.append(end_ms - info.t_submit_ms)
        done_walks += n * info.walks_per_point
    W.wost_server_destroy(srv)
    lat_done = np.array(lat_done) if lat_done else np.array([np.nan])
    lat_all = np.array(lat_all) if lat_all else np.array([np.nan])
    rounds_done = float(np.mean(rdone)) if rdone else None
    # open requests against time during the arrival window: the slope of a
    # least-squares line is the queue growth (requests/s); the rate the GPU
    # sustains is the finished requests per second of the run
    tl = np.array([(t, q) for t, q in queue_len if t <= a.window], dtype=np.float64)
    slope = float(np.polyfit(tl[:, 0], tl[:, 1], 1)[0]) if len(tl) >= 2 else None
    out = {"workload": "serving: pool of %d displaced-icosphere scenes (1.3M triangles each), Poisson %g req/s for %g s, "
                       "1..%d points, target SE %g..%g" % (a.pool, a.rate, a.window, a.max_points, a.se_lo, a.se_hi),
           "submitted": len(ids), "done": states[2], "active_at_end": states[1], "queued_at_end": states[0],
           "rejected": states[3], "elapsed_s": elapsed, "rounds": rounds,
           "latency_ms_p50": float(np.percentile(lat_all, 50)), "latency_ms_p99": float(np.percentile(lat_all, 99)),
           "latency_censored": int(states[0] + states[1]),
           "latency_note": "p50/p99 over every submitted request; unfinished ones count with their time "
                           "so far at the end of the run (censored, so the true percentiles are at least these)",
           "latency_ms_p50_finished": float(np.percentile(lat_done, 50)),
           "latency_ms_p99_finished": float(np.percentile(lat_done, 99)),
           "offered_req_per_s": a.rate, "sustained_req_per_s": states[2] / elapsed,
           "queue_growth_req_per_s": slope,
           "points_done_per_s": done_pts / elapsed, "walks_per_s": done_walks / elapsed,
           "open_requests_timeline": queue_len[:: max(1, len(queue_len) // 20)], "budget_mb": a.budget_mb,
           "rounds_in_flight": a.rounds_in_flight,
           "adaptive_rounds": not a.fixed_rounds, "round_budget_walks": a.round_budget, "max_active": a.max_active, "rounds_per_done_request": rounds_done}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
