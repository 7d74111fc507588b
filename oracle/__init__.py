"""ctypes binding of the FP64 brute-force walk-on-stars oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and
by the CPU-baseline leg of bench.py.  The product path never imports it.
It shares no code with the HIP library; only the seeded inputs of
paper_2302_11815_amd.inputs feed both.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_LIB = None

FN_PER_CORNER = 4
OFFSET_REL = 2.0 ** -18      # inward offset, relative to the scene half-diagonal L
ESCAPE_REL = 2.0             # escape radius, relative to L
MAX_STEPS = 1 << 16


class OrcFn(C.Structure):
    _fields_ = [("kind", C.c_int), ("as_nd", C.c_int), ("coef", C.c_double * 10),
                ("per_corner", C.c_void_p)]


class OrcSdf(C.Structure):
    _fields_ = [("kind", C.c_int), ("inside", C.c_int), ("p", C.c_double * 8)]


class OrcParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("rmin", C.c_double), ("offset", C.c_double),
                ("escape_radius", C.c_double), ("max_steps", C.c_int), ("seed", C.c_uint64),
                ("sigma", C.c_double), ("tik_sigma", C.c_double), ("tik_steps", C.c_int)]


class OrcState(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("n", C.c_double * 3), ("onN", C.c_int), ("cur", C.c_int),
                ("q", C.c_double * 3), ("q_set", C.c_int)]


class OrcStepRec(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("onN", C.c_int), ("cur", C.c_int),
                ("dD", C.c_double), ("xbar", C.c_double * 3), ("primD", C.c_int),
                ("term", C.c_int), ("g_term", C.c_double),
                ("dsil", C.c_double), ("r", C.c_double), ("v", C.c_double * 3),
                ("hit", C.c_int), ("hit_prim", C.c_int), ("t", C.c_double), ("p", C.c_double * 3),
                ("n_prim", C.c_int), ("valid", C.c_int), ("z", C.c_double * 3), ("pdf", C.c_double),
                ("Nhat", C.c_double), ("s_frac", C.c_double), ("Shat", C.c_double),
                ("q", C.c_double), ("roulette", C.c_int), ("side_g", C.c_int), ("side_h", C.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        D, P, I, U32 = C.c_double, C.c_void_p, C.c_int, C.c_uint32
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_uniforms.argtypes = [C.c_uint64, U32, U32, U32, U32, P]
        L.orc_scene_create.restype = P
        L.orc_scene_create.argtypes = [I, C.c_long, P, C.c_long, P, P, P, P, P, P, P]
        L.orc_scene_free.argtypes = [P]
        L.orc_scene_set_sdf.argtypes = [P, C.c_long, P]
        L.orc_sdf_closest.restype = D
        L.orc_sdf_closest.argtypes = [I, P, P, P]
        L.orc_scene_L.restype = D
        L.orc_scene_L.argtypes = [P]
        L.orc_scene_center.argtypes = [P, P]
        L.orc_scene_n_elements.restype = C.c_long
        L.orc_scene_n_elements.argtypes = [P]
        L.orc_closest_dirichlet.restype = D
        L.orc_closest_dirichlet.argtypes = [P, P, P, P]
        L.orc_silhouette.restype = D
        L.orc_silhouette.argtypes = [P, P, D]
        L.orc_ray_neumann.restype = C.c_long
        L.orc_ray_neumann.argtypes = [P, P, P, D, C.c_long, C.c_long, D, P]
        L.orc_silhouette_margin.restype = D
        L.orc_silhouette_margin.argtypes = [P, P, D, D, D]
        L.orc_ray_margin.restype = D
        L.orc_ray_margin.argtypes = [P, P, P, D, D, C.c_long, C.c_long, D]
        L.orc_sample_direction.argtypes = [I, D, D, P]
        L.orc_source_fraction.restype = D
        L.orc_source_fraction.argtypes = [I, D, D]
        L.orc_green_ball.restype = D
        L.orc_green_ball.argtypes = [I, D, D]
        L.orc_green_ball_norm.restype = D
        L.orc_green_ball_norm.argtypes = [I, D]
        for nm, at in (("orc_bessel_ie", [I, D]), ("orc_bessel_ke", [I, D]),
                       ("orc_screened_q", [I, D, D, D]), ("orc_green_ball_screened", [I, D, D, D]),
                       ("orc_green_ball_norm_screened", [I, D, D])):
            getattr(L, nm).restype = D
            getattr(L, nm).argtypes = at
        L.orc_neumann_sample.restype = C.c_long
        L.orc_neumann_sample.argtypes = [P, P, D, D, D, D, P, P]
        L.orc_step.restype = D
        L.orc_step.argtypes = [P, P, U32, U32, U32, P, P, P]
        L.orc_walk.restype = D
        L.orc_walk.argtypes = [P, P, P, U32, U32, P, P, P, I]
        L.orc_solve.restype = I
        L.orc_solve.argtypes = [P, P, P, P, C.c_long, I, I, P, P, P, P]
        L.orc_walk_from.restype = D
        L.orc_walk_from.argtypes = [P, P, P, C.c_long, U32, U32, P, P, P, I]
        L.orc_solve_from.restype = I
        L.orc_solve_from.argtypes = [P, P, P, P, P, C.c_long, I, U32, I, P, P, P, P]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def uniforms(seed, point, walk, step, slot):
    o = np.zeros(4)
    lib().orc_uniforms(C.c_uint64(seed), point, walk, step, slot, _ptr(o))
    return o


def _mkfn(fn, keep):
    s = OrcFn()
    s.kind = fn.kind
    s.as_nd = fn.as_nd
    c = fn.coef10()
    for i in range(10):
        s.coef[i] = c[i]
    if fn.kind == FN_PER_CORNER:
        pc = np.ascontiguousarray(fn.per_corner, dtype=np.float32)
        keep.append(pc)
        s.per_corner = pc.ctypes.data
    return s


class Scene:
    """Oracle-side scene: the brute-force data of one problem instance."""

    def __init__(self, spec):
        self.spec = spec
        self.dim = spec.dim
        keep = []
        V = np.ascontiguousarray(spec.vertices, dtype=np.float32)
        P = np.ascontiguousarray(spec.prims, dtype=np.int32)
        B = np.ascontiguousarray(spec.bc, dtype=np.uint8)
        g, h, f = _mkfn(spec.g, keep), _mkfn(spec.h, keep), _mkfn(spec.f, keep)
        gm, hm = _mkfn(spec.g_minus, keep), _mkfn(spec.h_minus, keep)
        self._h = lib().orc_scene_create(spec.dim, V.shape[0], _ptr(V), P.shape[0], _ptr(P), _ptr(B),
                                         C.byref(g), C.byref(h), C.byref(f), C.byref(gm), C.byref(hm))
        if not self._h:
            raise ValueError("oracle rejected the scene")
        sdf = getattr(spec, "sdf", None) or []
        if sdf:
            arr = (OrcSdf * len(sdf))()
            for i, f in enumerate(sdf):
                arr[i].kind, arr[i].inside = f.kind, f.inside
                for k, v in enumerate(f.p8()):
                    arr[i].p[k] = v
            lib().orc_scene_set_sdf(self._h, len(sdf), arr)
        self.L = lib().orc_scene_L(self._h)
        c = np.zeros(3)
        lib().orc_scene_center(self._h, _ptr(c))
        self.center = c

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_scene_free(self._h)
            self._h = None

    # ---- parameters --------------------------------------------------------
    def params(self, eps, seed=0, rmin=None, max_steps=MAX_STEPS, offset=None, escape=None, sigma=0.0,
               tik_sigma=0.0, tik_steps=0):
        """sigma: screening coefficient (Laplacian(u) - sigma u = f); tik_sigma /
        tik_steps: Tikhonov switch, sigma_T added from step tik_steps on."""
        p = OrcParams()
        p.sigma, p.tik_sigma, p.tik_steps = sigma, tik_sigma, tik_steps
        p.eps = eps
        p.rmin = eps if rmin is None else rmin
        p.offset = OFFSET_REL * self.L if offset is None else offset
        p.escape_radius = ESCAPE_REL * self.L if escape is None else escape
        p.max_steps = max_steps
        p.seed = seed
        return p

    # ---- queries -----------------------------------------------------------
    @staticmethod
    def _x3(x):
        a = np.zeros(3)
        x = np.asarray(x, dtype=np.float64)
        a[: x.shape[0]] = x
        return a

    def closest_dirichlet(self, x):
        xb = np.zeros(3)
        prim = C.c_long(0)
        d = lib().orc_closest_dirichlet(self._h, _ptr(self._x3(x)), _ptr(xb), C.byref(prim))
        return d, xb[: self.dim], prim.value

    def silhouette(self, x, rmax=math.inf):
        return lib().orc_silhouette(self._h, _ptr(self._x3(x)), rmax)

    def ray_neumann(self, o, v, tmax, skip0=-1, skip1=-1, behind=0.0):
        """First crossing with 0 < t <= tmax; behind > 0 also takes a crossing
        at -256 behind < t <= 0 of a one-sided primitive the ray leaves (v a
        unit vector), at t = 0, when o lies outside the primitive's plane by
        less than behind (reading R13, the walk's query uses behind =
        offset / 4)."""
        t = C.c_double(0)
        p = lib().orc_ray_neumann(self._h, _ptr(self._x3(o)), _ptr(self._x3(v)), tmax, skip0, skip1,
                                  float(behind), C.byref(t))
        return p, t.value

    # ---- decision margins (how near a reported result is to a tie) --------
    def silhouette_margin(self, x, rmax, d, tol):
        """Smallest distance of a silhouette decision from its threshold among
        the elements within tol of distance d from x (see orc_silhouette_margin)."""
        return lib().orc_silhouette_margin(self._h, _ptr(self._x3(x)), float(rmax), float(d), float(tol))

    def ray_margin(self, o, v, tmax, t, tol, skip0=-1, skip1=-1):
        """Smallest distance of a crossing decision from its threshold at
        parameter t of the ray o + t v (see orc_ray_margin)."""
        return lib().orc_ray_margin(self._h, _ptr(self._x3(o)), _ptr(self._x3(v)), float(tmax), float(t),
                                    int(skip0), int(skip1), float(tol))

    def neumann_sample(self, x, r, u4, u5, u6):
        z = np.zeros(3)
        pdf = C.c_double(0)
        p = lib().orc_neumann_sample(self._h, _ptr(self._x3(x)), r, u4, u5, u6, _ptr(z), C.byref(pdf))
        return p, z[: self.dim], pdf.value

    # ---- walks -------------------------------------------------------------
    def step(self, params, point, walk, k, x, n=None, onN=False, cur=-1, q=None):
        """q: the walk's last displacement x_k - x_{k-1} (double-sided
        primitives only; None at an interior start)."""
        st = OrcState()
        xx = self._x3(x)
        nn = self._x3(n) if n is not None else np.zeros(3)
        qq = self._x3(q) if q is not None else np.zeros(3)
        for i in range(3):
            st.x[i] = xx[i]
            st.n[i] = nn[i]
            st.q[i] = qq[i]
        st.onN = int(onN)
        st.cur = cur
        st.q_set = int(q is not None)
        rec, nxt = OrcStepRec(), OrcState()
        c = lib().orc_step(self._h, C.byref(params), point, walk, k, C.byref(st), C.byref(rec),
                           C.byref(nxt))
        return c, rec, nxt

    def walk(self, params, x0, point, walk, max_rec=0, start_prim=-1):
        """start_prim >= 0: x0 lies on that Neumann primitive and the walk starts
        on the boundary (on the "+" side of a double-sided one); -2 - p: on the
        "-" side of the double-sided primitive p."""
        ns, how = C.c_int(0), C.c_int(0)
        recs = (OrcStepRec * max_rec)() if max_rec > 0 else None
        v = lib().orc_walk_from(self._h, C.byref(params), _ptr(self._x3(x0)), int(start_prim), point,
                                walk, C.byref(ns), C.byref(how), recs, max_rec)
        out = list(recs[: min(ns.value, max_rec)]) if recs is not None else []
        return v, ns.value, how.value, out

    def solve(self, points, walks, eps, seed=0, rmin=None, max_steps=MAX_STEPS, nthreads=None,
              point_ids=None, return_values=False, params=None, start_prims=None, sigma=0.0,
              tik_sigma=0.0, tik_steps=0, walk_base=0):
        """Per-point mean and unbiased variance over `walks` walks; stats =
        (steps, capped, escaped).  start_prims (optional, [n] int): the Neumann
        primitive each point lies on, or -1 for an interior point.  The walks
        of a point take the RNG walk indices walk_base .. walk_base + walks - 1."""
        pts = np.ascontiguousarray(points, dtype=np.float32)
        n = pts.shape[0]
        if params is None:
            params = self.params(eps, seed, rmin, max_steps, sigma=sigma, tik_sigma=tik_sigma,
                                 tik_steps=tik_steps)
        mean = np.zeros(n)
        var = np.zeros(n)
        vals = np.zeros((n, walks)) if return_values else None
        ids = np.ascontiguousarray(point_ids, dtype=np.uint32) if point_ids is not None else None
        st = np.zeros(3, dtype=np.int64)
        nt = nthreads or os.cpu_count() or 1
        sp = np.ascontiguousarray(start_prims, dtype=np.int32) if start_prims is not None else None
        lib().orc_solve_from(self._h, C.byref(params), _ptr(pts), _ptr(ids), _ptr(sp), n, walks, walk_base, nt,
                             _ptr(mean), _ptr(var), _ptr(vals), _ptr(st))
        out = dict(mean=mean, var=var, steps=int(st[0]), capped=int(st[1]), escaped=int(st[2]))
        if return_values:
            out["values"] = vals
        return out


def sdf_closest(dim, shape, x):
    """Closest point on an analytic shape's surface and the distance."""
    f = OrcSdf()
    f.kind, f.inside = shape.kind, shape.inside
    for k, v in enumerate(shape.p8()):
        f.p[k] = v
    xx = np.zeros(3)
    xx[: len(x)] = x
    o = np.zeros(3)
    d = lib().orc_sdf_closest(dim, C.byref(f), _ptr(xx), _ptr(o))
    return d, o[:dim]


def sample_direction(dim, u0, u1):
    v = np.zeros(3)
    lib().orc_sample_direction(dim, u0, u1, _ptr(v))
    return v[:dim]


def source_fraction(dim, u2, u3):
    return lib().orc_source_fraction(dim, u2, u3)


def green_ball(dim, rho, R):
    return lib().orc_green_ball(dim, rho, R)


def green_ball_norm(dim, R):
    return lib().orc_green_ball_norm(dim, R)


def bessel_ie(n, x):
    """e^-x I_n(x)"""
    return lib().orc_bessel_ie(n, x)


def bessel_ke(n, x):
    """e^x K_n(x)"""
    return lib().orc_bessel_ke(n, x)


def screened_q(dim, sigma, r, R):
    return lib().orc_screened_q(dim, sigma, r, R)


def green_ball_screened(dim, sigma, rho, R):
    return lib().orc_green_ball_screened(dim, sigma, rho, R)


def green_ball_norm_screened(dim, sigma, R):
    return lib().orc_green_ball_norm_screened(dim, sigma, R)
