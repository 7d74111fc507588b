"""ctypes binding of libwost.so (include/wost.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Functions keep the C names; a non-OK status raises WostError.
Device-pointer entry points accept torch tensors (their data pointers are
passed through) and the current torch stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwost.so")
_LIB = None

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NOT_SUPPORTED", 5: "INTERNAL"}
WOST_OK, WOST_ERR_INVALID_ARG, WOST_ERR_OUT_OF_MEMORY, WOST_ERR_DEVICE, WOST_ERR_NOT_SUPPORTED = 0, 1, 2, 3, 4

EXPORTED = ["wost_build_scene", "wost_destroy_scene", "wost_get_scene_info", "wost_check_scene_host",
            "wost_solve", "wost_solve_ex", "wost_solve_boundary_ex", "wost_autotune", "wost_get_stats", "wost_get_traffic",
            "wost_get_walk_events", "wost_trace_walks", "wost_solve_ex_noalloc",
            "wost_probe_closest_point", "wost_probe_silhouette", "wost_probe_ray",
            "wost_probe_neumann_sample", "wost_get_neumann_tree", "wost_batch_create", "wost_batch_destroy", "wost_solve_batch",
            "wost_batch_get_stats", "wost_server_create", "wost_server_destroy", "wost_server_submit",
            "wost_server_step", "wost_server_poll", "wost_measure_l2_read", "wost_measure_valu",
            "wost_last_error"]


class WostError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class wost_fn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("as_normal_derivative", C.c_int32), ("coef", C.c_double * 10),
                ("per_corner", C.c_void_p)]


class wost_sdf(C.Structure):
    _fields_ = [("kind", C.c_int32), ("inside", C.c_int32), ("p", C.c_double * 8)]


class wost_scene_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64), ("vertices", C.c_void_p),
                ("n_prims", C.c_int64), ("prims", C.c_void_p), ("bc", C.c_void_p),
                ("g", wost_fn), ("h", wost_fn), ("f", wost_fn), ("g_minus", wost_fn), ("h_minus", wost_fn),
                ("n_sdf", C.c_int64), ("sdf", C.c_void_p)]


class wost_solve_opts(C.Structure):
    _fields_ = [("r_min", C.c_float), ("max_steps", C.c_int32), ("offset_rel", C.c_float),
                ("escape_rel", C.c_float), ("mode", C.c_int32), ("grid", C.c_int32),
                ("refill", C.c_int32), ("flags", C.c_uint32), ("chunk_walks", C.c_int32),
                ("walk_order", C.c_int32), ("sigma", C.c_float), ("tikhonov_sigma", C.c_float),
                ("tikhonov_steps", C.c_int32), ("claim_walks", C.c_int32), ("steal_lanes", C.c_int32)]


WOST_SOLVE_COUNT_TRAFFIC = 1


class wost_stats(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("walks", C.c_uint64), ("capped", C.c_uint64),
                ("escaped", C.c_uint64), ("kernel_ms", C.c_double), ("mode", C.c_int32),
                ("grid_blocks", C.c_int32), ("graph_captures", C.c_int32)]


class wost_traffic(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("q1_nodes", "q1_prims", "q2_nodes", "q2_cones", "q2_elems",
                                          "q3_nodes", "q3_prims", "q4_nodes", "q4_prims",
                                          "vis_nodes", "vis_prims",
                                          "wave_q1", "wave_q1_leaf", "wave_q2", "wave_q2_leaf",
                                          "wave_q3", "wave_q3_leaf", "wave_q4", "wave_vis",
                                          "wave_vis_leaf", "wave_steps", "cyc_q1", "cyc_q2", "cyc_q3",
                                          "cyc_q4", "cyc_rest")] + \
               [(n, C.c_uint32) for n in ("node_bytes", "cone_bytes", "prim_bytes", "elem_bytes")] + \
               [("io_bytes", C.c_uint64), ("bytes", C.c_uint64), ("wide_node_bytes", C.c_uint32)]


class wost_scene_info(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_prims", C.c_int64), ("n_dirichlet", C.c_int64),
                ("n_neumann", C.c_int64), ("n_silhouette_elements", C.c_int64),
                ("nodes_dirichlet", C.c_int64), ("nodes_neumann", C.c_int64),
                ("nodes_silhouette", C.c_int64), ("depth_dirichlet", C.c_int32),
                ("depth_neumann", C.c_int32), ("depth_silhouette", C.c_int32),
                ("device_bytes", C.c_int64), ("half_diagonal", C.c_double), ("center", C.c_double * 3),
                ("n_sdf", C.c_int64)]


class wost_batch_item(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("d_points", C.c_void_p), ("n_points", C.c_int64),
                ("walks_per_point", C.c_int32), ("eps", C.c_float), ("seed", C.c_uint64),
                ("point_base", C.c_uint32), ("walk_base", C.c_uint32), ("d_mean", C.c_void_p),
                ("d_var", C.c_void_p)]


class wost_server_config(C.Structure):
    _fields_ = [("max_device_bytes", C.c_int64), ("round_walks", C.c_int32), ("min_walks", C.c_int32),
                ("max_walks", C.c_int32), ("max_active", C.c_int32), ("solve", wost_solve_opts),
                ("adaptive", C.c_int32), ("max_round_walks", C.c_int32), ("max_rounds", C.c_int32),
                ("wait_us", C.c_int32), ("round_budget_walks", C.c_int64)]


class wost_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("rounds", C.c_int32), ("n_points", C.c_int64),
                ("walks_per_point", C.c_int64), ("max_se", C.c_double), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("in_flight", C.c_int32)]


REQ_QUEUED, REQ_ACTIVE, REQ_DONE, REQ_REJECTED = 0, 1, 2, 3


class wost_step_rec(C.Structure):
    _fields_ = [("x", C.c_float * 3), ("n", C.c_float * 3), ("on_neumann", C.c_int32), ("cur", C.c_int32),
                ("d_dirichlet", C.c_float), ("xbar", C.c_float * 3), ("prim_dirichlet", C.c_int32),
                ("term", C.c_int32), ("g_term", C.c_float), ("d_silhouette", C.c_float), ("r", C.c_float),
                ("v", C.c_float * 3), ("hit", C.c_int32), ("hit_prim", C.c_int32), ("t", C.c_float),
                ("p", C.c_float * 3), ("n_prim", C.c_int32), ("valid", C.c_int32), ("z", C.c_float * 3),
                ("pdf", C.c_float), ("n_hat", C.c_float), ("s_frac", C.c_float), ("s_hat", C.c_float),
                ("acc", C.c_float), ("q", C.c_float), ("roulette", C.c_int32),
                ("side_g", C.c_int32), ("side_h", C.c_int32)]


def lib():
    """Loads libwost.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(the solver has no CPU fallback)")
        # torch ships its own HIP runtime under the same soname as ROCm's; load
        # it first so that the library binds to that single runtime and torch
        # device pointers and streams are valid inside it
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, I64, I32, U32, U64, F = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_uint64, C.c_float
        sig = {
            "wost_build_scene": [P, P],
            "wost_destroy_scene": [P],
            "wost_get_scene_info": [P, P],
            "wost_check_scene_host": [P, P],
            "wost_solve": [P, P, I64, I32, F, U64, P, P],
            "wost_solve_ex": [P, P, I64, I32, F, U64, U32, U32, P, P, P, P],
            "wost_solve_ex_noalloc": [P, P, I64, I32, F, U64, U32, U32, P, P, P, P],
            "wost_solve_boundary_ex": [P, P, P, I64, I32, F, U64, U32, U32, P, P, P, P],
            "wost_get_stats": [P, P],
            "wost_autotune": [P, P, I64, I32, F, U64, I64, P, P],
            "wost_get_traffic": [P, P],
            "wost_get_walk_events": [P, I32, P, P, P, P, P],
            "wost_trace_walks": [P, P, P, P, P, I64, F, U64, P, I32, P, P, P],
            "wost_probe_closest_point": [P, P, I64, P, P, P],
            "wost_probe_silhouette": [P, P, P, I64, P],
            "wost_probe_ray": [P, P, P, P, P, I64, P, P],
            "wost_probe_neumann_sample": [P, P, P, I64, U64, P, P, P],
            "wost_get_neumann_tree": [P, P, P, P, P, P],
            "wost_batch_create": [P],
            "wost_batch_destroy": [P],
            "wost_solve_batch": [P, P, I32, P, P],
            "wost_batch_get_stats": [P, P],
            "wost_server_create": [P, P],
            "wost_server_destroy": [P],
            "wost_server_submit": [P, P, P, I64, F, U64, C.c_double, P],
            "wost_server_step": [P, P],
            "wost_server_poll": [P, I64, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.wost_last_error.argtypes = []
        L.wost_last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


def _check(status):
    if status != WOST_OK:
        raise WostError(status, lib().wost_last_error().decode())


def _p(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _fn(f, keep) -> wost_fn:
    s = wost_fn()
    s.kind = f.kind
    s.as_normal_derivative = f.as_nd
    c = f.coef10()
    for i in range(10):
        s.coef[i] = c[i]
    if f.per_corner is not None:
        pc = np.ascontiguousarray(f.per_corner, dtype=np.float32)
        keep.append(pc)
        s.per_corner = pc.ctypes.data
    return s


def make_desc(spec):
    """wost_scene_desc for an inputs.Scene; returns (desc, keepalive)."""
    keep = []
    V = np.ascontiguousarray(spec.vertices, dtype=np.float32)
    Pm = np.ascontiguousarray(spec.prims, dtype=np.int32)
    B = np.ascontiguousarray(spec.bc, dtype=np.uint8)
    keep += [V, Pm, B]
    d = wost_scene_desc()
    d.dim = spec.dim
    d.n_vertices = V.shape[0]
    d.vertices = V.ctypes.data
    d.n_prims = Pm.shape[0]
    d.prims = Pm.ctypes.data
    d.bc = B.ctypes.data
    d.g, d.h, d.f = _fn(spec.g, keep), _fn(spec.h, keep), _fn(spec.f, keep)
    d.g_minus, d.h_minus = _fn(spec.g_minus, keep), _fn(spec.h_minus, keep)
    shapes = getattr(spec, "sdf", None) or []
    d.n_sdf = len(shapes)
    if shapes:
        arr = (wost_sdf * len(shapes))()
        for i, f in enumerate(shapes):
            arr[i].kind, arr[i].inside = f.kind, f.inside
            for k, v in enumerate(f.p8()):
                arr[i].p[k] = v
        keep.append(arr)
        d.sdf = C.cast(arr, C.c_void_p)
    return d, keep


def make_opts(r_min=0.0, max_steps=0, offset_rel=0.0, escape_rel=0.0, mode=0, grid=0, refill=0,
              flags=0, chunk_walks=0, walk_order=0, sigma=0.0, tikhonov_sigma=0.0, tikhonov_steps=0,
              claim_walks=0, steal_lanes=0):
    o = wost_solve_opts()
    o.r_min, o.max_steps, o.offset_rel, o.escape_rel = r_min, max_steps, offset_rel, escape_rel
    o.mode, o.grid, o.refill, o.flags = mode, grid, refill, flags
    o.chunk_walks, o.walk_order = chunk_walks, walk_order
    o.sigma, o.tikhonov_sigma, o.tikhonov_steps = sigma, tikhonov_sigma, tikhonov_steps
    o.claim_walks, o.steal_lanes = claim_walks, steal_lanes
    return o


# ---- thin wrappers with the C names -----------------------------------------

def wost_build_scene(desc) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().wost_build_scene(C.byref(desc), C.byref(h)))
    return h


def wost_destroy_scene(scene):
    _check(lib().wost_destroy_scene(scene))


def wost_get_scene_info(scene) -> wost_scene_info:
    info = wost_scene_info()
    _check(lib().wost_get_scene_info(scene, C.byref(info)))
    return info


def wost_check_scene_host(desc) -> wost_scene_info:
    info = wost_scene_info()
    _check(lib().wost_check_scene_host(C.byref(desc), C.byref(info)))
    return info


def wost_solve(scene, points, walks, eps, seed):
    pts = np.ascontiguousarray(points, dtype=np.float32)
    n = pts.shape[0]
    mean = np.zeros(n)
    var = np.zeros(n)
    _check(lib().wost_solve(scene, _p(pts), n, walks, eps, seed, _p(mean), _p(var)))
    return mean, var


def wost_solve_ex(scene, d_points, n, walks, eps, seed, point_base=0, walk_base=0, opts=None,
                  d_mean=None, d_var=None, stream=None):
    """d_points, d_mean, d_var: device tensors (or raw pointers as ints)."""
    def ptr(t):
        return C.c_void_p(t) if isinstance(t, int) else _p(t)
    st = None if stream is None else C.c_void_p(stream)
    _check(lib().wost_solve_ex(scene, ptr(d_points), n, walks, eps, seed, point_base, walk_base,
                               C.byref(opts) if opts is not None else None, ptr(d_mean), ptr(d_var), st))


def wost_solve_ex_noalloc(scene, d_points, n, walks, eps, seed, point_base=0, walk_base=0, opts=None,
                          d_mean=None, d_var=None, stream=None):
    """wost_solve_ex without device allocations (the library's fixed array)."""
    def ptr(t):
        return C.c_void_p(t) if isinstance(t, int) else _p(t)
    st = None if stream is None else C.c_void_p(stream)
    _check(lib().wost_solve_ex_noalloc(scene, ptr(d_points), n, walks, eps, seed, point_base, walk_base,
                                       C.byref(opts) if opts is not None else None, ptr(d_mean), ptr(d_var),
                                       st))


def wost_solve_boundary_ex(scene, d_points, prims, n, walks, eps, seed, point_base=0, walk_base=0,
                           opts=None, d_mean=None, d_var=None, stream=None):
    """As wost_solve_ex; prims (host int32 [n]): the Neumann primitive each
    point lies on, or -1 for an interior point; -2 - p starts on the "-" side
    of the double-sided Neumann primitive p."""
    def ptr(t):
        return C.c_void_p(t) if isinstance(t, int) else _p(t)
    pr = np.ascontiguousarray(prims, dtype=np.int32)
    st = None if stream is None else C.c_void_p(stream)
    _check(lib().wost_solve_boundary_ex(scene, ptr(d_points), _p(pr), n, walks, eps, seed, point_base,
                                        walk_base, C.byref(opts) if opts is not None else None,
                                        ptr(d_mean), ptr(d_var), st))


def wost_autotune(scene, d_points, n, walks, eps, seed, sample_walks=0, opts=None, stream=None):
    """Returns tuned wost_solve_opts (a copy of `opts`, or the defaults)."""
    o = wost_solve_opts()
    C.pointer(o)[0] = opts if opts is not None else make_opts()
    st = None if stream is None else C.c_void_p(stream)
    ptr = C.c_void_p(d_points) if isinstance(d_points, int) else _p(d_points)
    _check(lib().wost_autotune(scene, ptr, n, walks, eps, seed, sample_walks, C.byref(o), st))
    return o


def wost_get_stats(scene) -> wost_stats:
    s = wost_stats()
    _check(lib().wost_get_stats(scene, C.byref(s)))
    return s


def wost_get_walk_events(scene, max_events=64):
    """Walks of the last solve that ended capped (kind 2) or escaped (kind 3):
    arrays (point_ids, walk_ids, steps, kinds)."""
    pid = np.zeros(max_events, np.uint32)
    wid = np.zeros(max_events, np.uint32)
    st = np.zeros(max_events, np.int32)
    kd = np.zeros(max_events, np.int32)
    n = C.c_int32(0)
    _check(lib().wost_get_walk_events(scene, max_events, _p(pid), _p(wid), _p(st), _p(kd), C.byref(n)))
    k = n.value
    return pid[:k], wid[:k], st[:k], kd[:k]


def wost_get_traffic(scene) -> wost_traffic:
    t = wost_traffic()
    _check(lib().wost_get_traffic(scene, C.byref(t)))
    return t


def wost_trace_walks(scene, points, point_ids, walk_ids, eps, seed, max_rec, opts=None, prims=None):
    pts = np.ascontiguousarray(points, dtype=np.float32)
    n = pts.shape[0]
    pid = np.ascontiguousarray(point_ids, dtype=np.uint32)
    wid = np.ascontiguousarray(walk_ids, dtype=np.uint32)
    pr = np.ascontiguousarray(prims, dtype=np.int32) if prims is not None else None
    recs = (wost_step_rec * (n * max_rec))()
    ns = np.zeros(n, dtype=np.int32)
    vals = np.zeros(n, dtype=np.float32)
    _check(lib().wost_trace_walks(scene, _p(pts), _p(pid), _p(wid), _p(pr) if pr is not None else None,
                                  n, eps, seed,
                                  C.byref(opts) if opts is not None else None, max_rec, recs, _p(ns),
                                  _p(vals)))
    return recs, ns, vals


def wost_measure_l2_read(nbytes=0, reps=0) -> float:
    """Read bandwidth (GB/s) of a streaming kernel over an L2-resident buffer."""
    g = C.c_double(0)
    _check(lib().wost_measure_l2_read(C.c_int64(nbytes), C.c_int32(reps), C.byref(g)))
    return g.value


def wost_measure_valu(kind=0, iters=0) -> float:
    """Vector ALU issue rate (10^9 lane instructions per second) of
    independent chains: kind 0 FP32 fused multiply-adds, kind 1 integer
    xor + add pairs."""
    g = C.c_double(0)
    _check(lib().wost_measure_valu(C.c_int32(kind), C.c_int32(iters), C.byref(g)))
    return g.value


def wost_probe_closest_point(scene, x, dim):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, dim)
    n = x.shape[0]
    d = np.zeros(n, np.float32)
    xb = np.zeros((n, dim), np.float32)
    pr = np.zeros(n, np.int32)
    _check(lib().wost_probe_closest_point(scene, _p(x), n, _p(d), _p(xb), _p(pr)))
    return d, xb, pr


def wost_probe_silhouette(scene, x, rmax, dim):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, dim)
    n = x.shape[0]
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(rmax, np.float32), (n,)))
    d = np.zeros(n, np.float32)
    _check(lib().wost_probe_silhouette(scene, _p(x), _p(r), n, _p(d)))
    return d


def wost_probe_ray(scene, o, v, tmax, skip, dim):
    o = np.ascontiguousarray(o, dtype=np.float32).reshape(-1, dim)
    v = np.ascontiguousarray(v, dtype=np.float32).reshape(-1, dim)
    n = o.shape[0]
    tm = np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float32), (n,)))
    sk = np.ascontiguousarray(np.broadcast_to(np.asarray(skip, np.int32), (n,)))
    t = np.zeros(n, np.float32)
    pr = np.zeros(n, np.int32)
    _check(lib().wost_probe_ray(scene, _p(o), _p(v), _p(tm), _p(sk), n, _p(t), _p(pr)))
    return t, pr


def wost_probe_neumann_sample(scene, x, r, seed, dim):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, dim)
    n = x.shape[0]
    rr = np.ascontiguousarray(np.broadcast_to(np.asarray(r, np.float32), (n,)))
    z = np.zeros((n, dim), np.float32)
    pdf = np.zeros(n, np.float32)
    pr = np.zeros(n, np.int32)
    _check(lib().wost_probe_neumann_sample(scene, _p(x), _p(rr), n, seed, _p(z), _p(pdf), _p(pr)))
    return z, pdf, pr


def wost_get_neumann_tree(scene, dim):
    """The binary Neumann tree Q.4 descends: nodes [n][16 (3D) / 12 (2D)]
    float32, slot_prim [n_slots] int32, slot_measure [n_slots] float32."""
    nn, ns = C.c_int64(0), C.c_int64(0)
    _check(lib().wost_get_neumann_tree(scene, C.byref(nn), None, C.byref(ns), None, None))
    nodes = np.zeros((nn.value, 16 if dim == 3 else 12), np.float32)
    sp = np.zeros(ns.value, np.int32)
    sm = np.zeros(ns.value, np.float32)
    _check(lib().wost_get_neumann_tree(scene, C.byref(nn), _p(nodes), C.byref(ns), _p(sp), _p(sm)))
    return nodes, sp, sm


def _ptr_of(t):
    if t is None:
        return None
    return t if isinstance(t, int) else t.data_ptr()


def make_batch_item(scene_handle, d_points, n_points, walks, eps, seed, d_mean, d_var,
                    point_base=0, walk_base=0) -> wost_batch_item:
    it = wost_batch_item()
    it.scene = scene_handle.value if hasattr(scene_handle, "value") else scene_handle
    it.d_points, it.n_points, it.walks_per_point = _ptr_of(d_points), n_points, walks
    it.eps, it.seed, it.point_base, it.walk_base = eps, seed, point_base, walk_base
    it.d_mean, it.d_var = _ptr_of(d_mean), _ptr_of(d_var)
    return it


def wost_batch_create() -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().wost_batch_create(C.byref(h)))
    return h


def wost_batch_destroy(batch):
    _check(lib().wost_batch_destroy(batch))


def wost_solve_batch(batch, items, opts=None, stream=None):
    arr = (wost_batch_item * max(1, len(items)))(*items)
    st = None if stream is None else C.c_void_p(stream)
    _check(lib().wost_solve_batch(batch, arr, len(items), C.byref(opts) if opts is not None else None, st))


def wost_batch_get_stats(batch) -> wost_stats:
    s = wost_stats()
    _check(lib().wost_batch_get_stats(batch, C.byref(s)))
    return s


def make_server_config(max_device_bytes=0, round_walks=0, min_walks=0, max_walks=0, max_active=0,
                       solve=None, adaptive=0, max_round_walks=0, max_rounds=0, wait_us=0,
                       round_budget_walks=0) -> wost_server_config:
    c = wost_server_config()
    c.max_device_bytes, c.round_walks, c.min_walks = max_device_bytes, round_walks, min_walks
    c.max_walks, c.max_active = max_walks, max_active
    c.adaptive, c.max_round_walks = adaptive, max_round_walks
    c.max_rounds, c.wait_us, c.round_budget_walks = max_rounds, wait_us, round_budget_walks
    c.solve = solve if solve is not None else make_opts()
    return c


def wost_server_create(cfg=None) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().wost_server_create(C.byref(cfg) if cfg is not None else None, C.byref(h)))
    return h


def wost_server_destroy(server):
    _check(lib().wost_server_destroy(server))


def wost_server_submit(server, scene_handle, points, eps, seed, target_se) -> int:
    pts = np.ascontiguousarray(points, dtype=np.float32)
    rid = C.c_int64(-1)
    _check(lib().wost_server_submit(server, scene_handle, _p(pts), pts.shape[0], eps, seed, target_se,
                                    C.byref(rid)))
    return rid.value


def wost_server_step(server) -> int:
    n = C.c_int32(0)
    _check(lib().wost_server_step(server, C.byref(n)))
    return n.value


def wost_server_poll(server, request_id, with_results=False):
    info = wost_request_info()
    _check(lib().wost_server_poll(server, request_id, C.byref(info), None, None))
    if not with_results or info.state != REQ_DONE:
        return info, None, None
    mean = np.zeros(info.n_points)
    var = np.zeros(info.n_points)
    _check(lib().wost_server_poll(server, request_id, C.byref(info), _p(mean), _p(var)))
    return info, mean, var


class Scene:
    """Owns a built scene: Scene(inputs.Scene) -> library handle."""

    def __init__(self, spec):
        self.spec = spec
        self.dim = spec.dim
        desc, keep = make_desc(spec)
        self.handle = wost_build_scene(desc)
        self.info = wost_get_scene_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            wost_destroy_scene(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
