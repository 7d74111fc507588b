"""Seeded synthetic inputs for the walk-on-stars solver: scenes, evaluation
points and boundary-data descriptors.

This module is shared by the HIP path and the CPU oracle. It builds problem
instances only -- meshes, boundary-condition flags, points inside the domain,
the closed-form solutions used as test targets, and the descriptors of f, g, h
-- and contains none of the estimator's arithmetic (no distances, queries,
kernels or random walks).

The paper evaluates on CT-scan and hand-modelled scenes (toaster, lizard,
lungs) that are not available; the generators below stand in for them at the
paper's scale (about 10^6 boundary elements, 10^5-10^6 evaluation points,
hundreds to a thousand walks per point, models scaled into the unit sphere as
in the paper's experimental setup, Sec. 6).

Problem (Sec. 3.2, Eq. PoissonEquation): Laplacian(u) = f in the domain,
u = g on the Dirichlet part, du/dn = h on the Neumann part, n the unit
outward normal.  Orientation conventions: in 2D a segment (a, b) has outward
normal (b_y - a_y, -(b_x - a_x)) / |b - a| (polygons wound counter-clockwise);
in 3D a triangle (a, b, c) has outward normal (b - a) x (c - a) normalised.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

# Boundary/source data kinds, mirrored by the C-ABI enum wost_fn_kind.
FN_ZERO, FN_CONST, FN_POLY2, FN_EXPCOS, FN_PER_CORNER, FN_EXPLIN = 0, 1, 2, 3, 4, 5

DIRICHLET, NEUMANN = 0, 1
# double-sided primitives (data on both sides; "+" is the side the normal
# points away from, "-" the side it points into)
DIRICHLET2, NEUMANN2 = 2, 3

# analytic Dirichlet shapes, mirrored by the C-ABI enum wost_sdf_kind
SDF_BALL, SDF_BOX, SDF_CAPSULE = 0, 1, 2


@dataclasses.dataclass
class Sdf:
    """An analytic shape whose surface is Dirichlet boundary (data g).

    kind    SDF_BALL: p = (centre[3], -, -, -, radius)
            SDF_BOX: p = (centre[3], half extents[3], rounding radius)
            SDF_CAPSULE: p = (end a[3], end b[3], radius)
            (2D shapes leave the third coordinates 0)
    inside  1: the domain lies inside the shape (a ball, or a box with no
            rounding); 0: outside it.
    """
    kind: int
    inside: int
    p: tuple

    def p8(self) -> np.ndarray:
        c = np.zeros(8, dtype=np.float64)
        c[: len(self.p)] = self.p
        return c

    def value(self, x: np.ndarray) -> np.ndarray:
        """Signed distance, positive on the domain side (problem geometry for
        building inputs: point rejection, not the estimator's query)."""
        x = np.asarray(x, np.float64)
        d = x.shape[-1]
        c = self.p8()
        if self.kind == SDF_BALL:
            s = np.linalg.norm(x - c[:d], axis=-1) - c[6]
        elif self.kind == SDF_BOX:
            q = np.abs(x - c[:d]) - c[3:3 + d]
            s = np.linalg.norm(np.maximum(q, 0), axis=-1) + np.minimum(q.max(-1), 0) - c[6]
        else:
            a, b = c[:d], c[3:3 + d]
            t = np.clip(((x - a) @ (b - a)) / max(float((b - a) @ (b - a)), 1e-300), 0, 1)
            s = np.linalg.norm(x - (a + t[..., None] * (b - a)), axis=-1) - c[6]
        return -s if self.inside else s


@dataclasses.dataclass
class Fn:
    """Descriptor of a scalar field (g, h or f).

    kind       FN_* constant.
    as_nd      1: the field is the outward normal derivative of the analytic
               function given by (kind, coef), evaluated per primitive normal.
    coef       POLY2 in 3D: c, x, y, z, xx, yy, zz, xy, yz, zx.
               POLY2 in 2D: c, x, y, xx, yy, xy.
               EXPCOS (2D): coef[0] * exp(coef[1] x) * cos(coef[1] y).
               EXPLIN: coef[0] * exp(coef[1] x + coef[2] y + coef[3] z); it
               solves Laplacian(u) - sigma u = 0 for sigma = |coef[1:4]|^2.
               CONST: coef[0].
    per_corner [n_prims][dim] float32 values at each primitive's corners,
               interpolated linearly over the primitive (kind PER_CORNER).
    """
    kind: int = FN_ZERO
    as_nd: int = 0
    coef: tuple = ()
    per_corner: Optional[np.ndarray] = None

    def coef10(self) -> np.ndarray:
        c = np.zeros(10, dtype=np.float64)
        c[: len(self.coef)] = self.coef
        return c


@dataclasses.dataclass
class Scene:
    name: str
    dim: int
    vertices: np.ndarray            # float32 [nv, dim]
    prims: np.ndarray               # int32 [np, dim]
    bc: np.ndarray                  # uint8 [np], 0 Dirichlet / 1 Neumann / 2, 3 double-sided
    g: Fn
    h: Fn
    f: Fn
    exact: Optional[Callable[[np.ndarray], np.ndarray]] = None
    g_minus: Fn = dataclasses.field(default_factory=Fn)   # "-" side of double-sided prims
    h_minus: Fn = dataclasses.field(default_factory=Fn)
    sdf: list = dataclasses.field(default_factory=list)   # analytic Dirichlet shapes (Sdf)

    @property
    def n_prims(self) -> int:
        return int(self.prims.shape[0])


# --------------------------------------------------------------------------
# closed-form solutions used as targets
# --------------------------------------------------------------------------

def poly2_eval(coef, x: np.ndarray) -> np.ndarray:
    """Evaluate a POLY2 descriptor (problem data, not estimator arithmetic)."""
    c = np.zeros(10)
    c[: len(coef)] = coef
    x = np.asarray(x, dtype=np.float64)
    if x.shape[-1] == 2:
        X, Y = x[..., 0], x[..., 1]
        return c[0] + c[1] * X + c[2] * Y + c[3] * X * X + c[4] * Y * Y + c[5] * X * Y
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * X + c[5] * Y * Y
            + c[6] * Z * Z + c[7] * X * Y + c[8] * Y * Z + c[9] * Z * X)


def expcos_eval(coef, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return coef[0] * np.exp(coef[1] * x[..., 0]) * np.cos(coef[1] * x[..., 1])


def explin_eval(coef, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    e = coef[1] * x[..., 0] + coef[2] * x[..., 1]
    if x.shape[-1] > 2 and len(coef) > 3:
        e = e + coef[3] * x[..., 2]
    return coef[0] * np.exp(e)


def with_data(spec: "Scene", kind, coef, laplacian_const=None, bc=None, name=None) -> "Scene":
    """A copy of spec with g = u, h = du/dn, f from solution_data (and
    optionally other boundary types)."""
    g, h, f, u = solution_data(kind, coef, laplacian_const)
    return dataclasses.replace(spec, g=g, h=h, f=f, exact=u, name=name or spec.name,
                               bc=spec.bc.copy() if bc is None else np.asarray(bc, np.uint8))


def _analytic(kind, coef):
    if kind == FN_EXPLIN:
        return lambda x: explin_eval(coef, x)
    if kind == FN_POLY2:
        return lambda x: poly2_eval(coef, x)
    if kind == FN_EXPCOS:
        return lambda x: expcos_eval(coef, x)
    if kind == FN_CONST:
        return lambda x: np.full(np.asarray(x).shape[:-1], float(coef[0]))
    if kind == FN_ZERO:
        return lambda x: np.zeros(np.asarray(x).shape[:-1])
    raise ValueError(kind)


def solution_data(kind, coef, laplacian_const: Optional[float] = None):
    """g = u, h = du/dn (as a normal-derivative descriptor) and f for an exact u.

    laplacian_const: the constant Laplacian of u when u is a quadratic.
    """
    g = Fn(kind, 0, tuple(coef))
    h = Fn(kind, 1, tuple(coef))
    if laplacian_const is None or laplacian_const == 0.0:
        f = Fn(FN_ZERO)
    else:
        f = Fn(FN_CONST, 0, (float(laplacian_const),))
    return g, h, f, _analytic(kind, coef)


# --------------------------------------------------------------------------
# 2D scenes
# --------------------------------------------------------------------------

def unit_square_scene() -> Scene:
    """4 segments, counter-clockwise. Dirichlet on x=0 (g=0) and x=1 (g=1),
    zero Neumann on y=0 and y=1; exact u = x."""
    V = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float32)
    P = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], dtype=np.int32)
    bc = np.array([NEUMANN, DIRICHLET, NEUMANN, DIRICHLET], dtype=np.uint8)
    coef = (0.0, 1.0, 0.0)
    g = Fn(FN_POLY2, 0, coef)
    return Scene("unit_square", 2, V, P, bc, g, Fn(FN_ZERO), Fn(FN_ZERO),
                 exact=lambda x: np.asarray(x, np.float64)[..., 0])


def grid_points_2d(n: int = 32) -> np.ndarray:
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float32)


def star_polygon_radius_params(seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.uniform(0.0, 1.0, 8)
    a = w / w.sum()
    phi = rng.uniform(0.0, 2 * math.pi, 8)
    return a, phi


def star_polygon_scene(n_seg: int = 16384, seed: int = 0, neumann_frac: float = 0.5,
                       n_arcs: int = 4) -> Scene:
    """Seeded star polygon r(theta) = 1 + 0.3 sum_k a_k sin(k theta + phi_k),
    a_k >= 0 normalised to sum 1 (so r stays in [0.7, 1.3]), polylined into
    n_seg segments counter-clockwise. n_arcs disjoint contiguous arcs covering
    neumann_frac of the arc length are Neumann, the rest Dirichlet.
    Exact u = exp(x) cos(y), f = 0."""
    a, phi = star_polygon_radius_params(seed)
    th = 2 * math.pi * np.arange(n_seg) / n_seg
    k = np.arange(1, 9)
    r = 1.0 + 0.3 * (a[None, :] * np.sin(k[None, :] * th[:, None] + phi[None, :])).sum(1)
    V = np.stack([r * np.cos(th), r * np.sin(th)], axis=1).astype(np.float32)
    i = np.arange(n_seg, dtype=np.int32)
    P = np.stack([i, (i + 1) % n_seg], axis=1).astype(np.int32)
    # arc-length layout of alternating Neumann / Dirichlet arcs
    Vd = V.astype(np.float64)
    seglen = np.linalg.norm(Vd[P[:, 1]] - Vd[P[:, 0]], axis=1)
    S = seglen.sum()
    mid = np.cumsum(seglen) - 0.5 * seglen
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    wn = rng.uniform(0.5, 1.5, n_arcs)
    wd = rng.uniform(0.5, 1.5, n_arcs)
    ln = neumann_frac * S * wn / wn.sum()
    ld = (1 - neumann_frac) * S * wd / wd.sum()
    start = rng.uniform(0.0, S)
    bc = np.zeros(n_seg, dtype=np.uint8)
    pos = (mid - start) % S
    edges = np.cumsum(np.stack([ln, ld], axis=1).ravel())  # N, D, N, D, ...
    which = np.searchsorted(edges, pos, side="right")
    bc[(which % 2) == 0] = NEUMANN
    g, h, f, u = solution_data(FN_EXPCOS, (1.0, 1.0))
    return Scene(f"star_polygon_{n_seg}_s{seed}", 2, V, P, bc, g, h, f, exact=u)


def neumann_boundary_points(spec: "Scene", n: int, seed: int = 0, margin: float = 0.1):
    """n evaluation points on the Neumann boundary: a uniformly chosen Neumann
    primitive each, and a point on it away from its vertices and edges
    (segment parameter in [margin, 1 - margin]; triangle barycentrics each at
    least margin).  Returns (points [n][dim] float32, primitive ids [n] int32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    neu = np.nonzero(spec.bc == NEUMANN)[0]
    prims = rng.choice(neu, n).astype(np.int32)
    V = spec.vertices.astype(np.float64)
    P = spec.prims[prims]
    if spec.dim == 2:
        t = rng.uniform(margin, 1 - margin, n)[:, None]
        pts = (1 - t) * V[P[:, 0]] + t * V[P[:, 1]]
    else:
        w = rng.dirichlet(np.ones(3), n) * (1 - 3 * margin) + margin
        pts = w[:, :1] * V[P[:, 0]] + w[:, 1:2] * V[P[:, 1]] + w[:, 2:] * V[P[:, 2]]
    return pts.astype(np.float32), prims


def star_polygon_points(n: int, seed: int = 0, poly_seed: int = 0, n_seg: int = 16384,
                        vertices: Optional[np.ndarray] = None) -> np.ndarray:
    """n points uniform inside the star polygon (rejection in the disk of
    radius 1.3); inside test against the exact polyline radius along the
    point's angle, in float64."""
    if vertices is None:
        vertices = star_polygon_scene(n_seg, poly_seed).vertices
    V = vertices.astype(np.float64)
    nv = V.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed + 7777))
    out = []
    have = 0
    while have < n:
        m = max(1024, int((n - have) * 1.6))
        rad = 1.3 * np.sqrt(rng.uniform(0, 1, m))
        ang = rng.uniform(0, 2 * math.pi, m)
        p = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
        seg = np.floor(ang / (2 * math.pi) * nv).astype(np.int64) % nv
        A = V[seg]
        B = V[(seg + 1) % nv]
        d = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        e = B - A
        nrm = np.stack([e[:, 1], -e[:, 0]], axis=1)
        t = (nrm * A).sum(1) / (nrm * d).sum(1)
        keep = p[rad < t]
        out.append(keep)
        have += keep.shape[0]
    return np.concatenate(out)[:n].astype(np.float32)


def polygon_scene(V, bc, name="polygon", g: Fn = None, h: Fn = None, f: Fn = None,
                  exact=None) -> Scene:
    V = np.asarray(V, dtype=np.float32)
    n = V.shape[0]
    i = np.arange(n, dtype=np.int32)
    P = np.stack([i, (i + 1) % n], axis=1).astype(np.int32)
    return Scene(name, 2, V, P, np.asarray(bc, dtype=np.uint8),
                 g or Fn(FN_ZERO), h or Fn(FN_ZERO), f or Fn(FN_ZERO), exact)


def l_shape_2d(bc=None, **kw) -> Scene:
    """[0,2]^2 minus [1,2]^2, counter-clockwise; reflex corner at (1,1)."""
    V = [[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]]
    if bc is None:
        bc = [NEUMANN] * 6
    return polygon_scene(V, bc, name="l_shape", **kw)


# --------------------------------------------------------------------------
# 3D scenes
# --------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return V, F


def icosphere(level: int):
    """Unit icosphere; the children of face f at level L+1 are faces
    4f .. 4f+3 (corner a, corner b, corner c, middle)."""
    V, F = _icosahedron()
    levels = [(V, F)]
    for _ in range(level):
        nf = F.shape[0]
        E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        lo = np.minimum(E[:, 0], E[:, 1])
        hi = np.maximum(E[:, 0], E[:, 1])
        key = lo * (V.shape[0] + 1) + hi
        uk, inv = np.unique(key, return_inverse=True)
        ulo = uk // (V.shape[0] + 1)
        uhi = uk % (V.shape[0] + 1)
        M = V[ulo] + V[uhi]
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        mid = V.shape[0] + inv
        ab, bc_, ca = mid[:nf], mid[nf:2 * nf], mid[2 * nf:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        C = np.empty((nf, 4, 3), dtype=np.int64)
        C[:, 0] = np.stack([a, ab, ca], 1)
        C[:, 1] = np.stack([ab, b, bc_], 1)
        C[:, 2] = np.stack([ca, bc_, c], 1)
        C[:, 3] = np.stack([ab, bc_, ca], 1)
        V = np.concatenate([V, M], axis=0)
        F = C.reshape(-1, 3)
        levels.append((V, F))
    return V, F, levels


def value_noise(p: np.ndarray, seed: int, octaves: int = 4, base_freq: float = 2.0,
                lacunarity: float = 2.0, gain: float = 0.5) -> np.ndarray:
    """Seeded value noise: lattice values uniform in [-1, 1] from an integer
    hash, smoothstep-trilinear interpolation, octaves summed and normalised to
    [-1, 1] by the sum of amplitudes."""
    p = np.asarray(p, dtype=np.float64)
    total = np.zeros(p.shape[0])
    amp, freq, norm = 1.0, base_freq, 0.0
    for o in range(octaves):
        q = p * freq
        i0 = np.floor(q)
        t = q - i0
        w = t * t * (3.0 - 2.0 * t)
        i0 = i0.astype(np.int64)
        acc = np.zeros(p.shape[0])
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    h = _lattice_hash(i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz, seed * 131 + o)
                    wx = w[:, 0] if dx else 1.0 - w[:, 0]
                    wy = w[:, 1] if dy else 1.0 - w[:, 1]
                    wz = w[:, 2] if dz else 1.0 - w[:, 2]
                    acc += wx * wy * wz * h
        total += amp * acc
        norm += amp
        amp *= gain
        freq *= lacunarity
    return total / norm


def _lattice_hash(i, j, k, s):
    M = np.uint64(0xFFFFFFFF)
    h = ((i.astype(np.int64).astype(np.uint64) * np.uint64(0x8DA6B343))
         ^ (j.astype(np.int64).astype(np.uint64) * np.uint64(0xD8163841))
         ^ (k.astype(np.int64).astype(np.uint64) * np.uint64(0xCB1AB31F))
         ^ (np.uint64(s & 0xFFFFFFFF) * np.uint64(0x9E3779B9))) & M
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & M
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & M
    h ^= h >> np.uint64(16)
    return h.astype(np.float64) / 4294967296.0 * 2.0 - 1.0


@dataclasses.dataclass
class RadialMesh:
    """A radially displaced icosphere and the face hierarchy used to locate
    the triangle hit by a ray from the origin (for exact inside tests)."""
    V: np.ndarray        # displaced vertices, float64 [nv, 3]
    F: np.ndarray        # faces [nf, 3]
    levels: list         # (unit vertices, faces) per subdivision level


def displaced_icosphere(level: int, seed: int, amplitude: float = 0.2) -> RadialMesh:
    U, F, levels = icosphere(level)
    rho = 1.0 + amplitude * value_noise(U, seed)
    return RadialMesh(U * rho[:, None], F, levels)


def _locate_faces(levels, d: np.ndarray) -> np.ndarray:
    """Index of the finest-level face whose cone (from the origin) contains
    direction d: descend the subdivision hierarchy, keeping at every level the
    child whose three bounding planes d is most inside."""
    def score(V, F, cand):
        a, b, c = V[F[cand, 0]], V[F[cand, 1]], V[F[cand, 2]]
        dd = d[:, None, :]
        s0 = (np.cross(a, b) * dd).sum(-1)
        s1 = (np.cross(b, c) * dd).sum(-1)
        s2 = (np.cross(c, a) * dd).sum(-1)
        return np.minimum(np.minimum(s0, s1), s2)
    V0, F0 = levels[0]
    cand = np.broadcast_to(np.arange(F0.shape[0]), (d.shape[0], F0.shape[0]))
    face = np.argmax(score(V0, F0, cand), axis=1)
    rows = np.arange(d.shape[0])
    for L in range(1, len(levels)):
        VL, FL = levels[L]
        cand = 4 * face[:, None] + np.arange(4)[None, :]
        face = cand[rows, np.argmax(score(VL, FL, cand), axis=1)]
    return face


def _radial_bounds(mesh: RadialMesh):
    """Radii within which the answer needs no face lookup: every face's plane
    lies at least r_in from the origin (so the surface along any direction is
    farther), and no surface point lies beyond the largest vertex radius."""
    if getattr(mesh, "_bounds", None) is None:
        A, B, C = mesh.V[mesh.F[:, 0]], mesh.V[mesh.F[:, 1]], mesh.V[mesh.F[:, 2]]
        n = np.cross(B - A, C - A)
        r_in = float(((n * A).sum(1) / np.linalg.norm(n, axis=1)).min())
        r_out = float(np.linalg.norm(mesh.V, axis=1).max())
        mesh._bounds = (r_in, r_out)
    return mesh._bounds


def radial_mesh_inside(mesh: RadialMesh, p: np.ndarray, chunk: int = 100000) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    r_in, r_out = _radial_bounds(mesh)
    r_all = np.linalg.norm(p, axis=1)
    out = r_all < r_in
    shell = np.nonzero((r_all >= r_in) & (r_all <= r_out))[0]
    for s in range(0, shell.size, chunk):
        sel = shell[s:s + chunk]
        q = p[sel]
        r = r_all[sel]
        d = q / np.maximum(r, 1e-300)[:, None]
        f = _locate_faces(mesh.levels, d)
        A, B, C = mesh.V[mesh.F[f, 0]], mesh.V[mesh.F[f, 1]], mesh.V[mesh.F[f, 2]]
        n = np.cross(B - A, C - A)
        t = (n * A).sum(1) / (n * d).sum(1)
        out[sel] = r < t
    return out


def displaced_icosphere_scene(level: int = 8, seed: int = 0, z_split: float = 0.1,
                              amplitude: float = 0.2, mesh: RadialMesh = None) -> Scene:
    """Icosphere subdivided `level` times, radially displaced by seeded
    4-octave value noise of the given amplitude. Triangles whose centroid has
    z > z_split are Dirichlet, the rest Neumann. Exact
    u = (x^2 + y^2 + z^2)/6 + xy, so f = Laplacian(u) = 1."""
    if mesh is None:
        mesh = displaced_icosphere(level, seed, amplitude)
    V = mesh.V.astype(np.float32)
    F = mesh.F.astype(np.int32)
    Vd = V.astype(np.float64)
    cen = Vd[F].mean(axis=1)
    nrm = np.cross(Vd[F[:, 1]] - Vd[F[:, 0]], Vd[F[:, 2]] - Vd[F[:, 0]])
    assert np.all((nrm * cen).sum(1) > 0), "displaced mesh must face outward"
    bc = np.where(cen[:, 2] > z_split, DIRICHLET, NEUMANN).astype(np.uint8)
    # u = (x^2+y^2+z^2)/6 + xy  -> POLY2 coefficients c,x,y,z,xx,yy,zz,xy,yz,zx
    coef = (0.0, 0.0, 0.0, 0.0, 1 / 6, 1 / 6, 1 / 6, 1.0, 0.0, 0.0)
    g, h, f, u = solution_data(FN_POLY2, coef, laplacian_const=1.0)
    return Scene(f"displaced_icosphere_L{level}_s{seed}", 3, V, F, bc, g, h, f, exact=u)


def radial_mesh_points(mesh: RadialMesh, n: int, seed: int, box: float = 1.2) -> np.ndarray:
    """n points uniform inside the mesh, by rejection from the box
    [-box, box]^3.  Candidates are drawn in fixed blocks, so the points for
    a smaller n are the first n of the points for a larger one."""
    rng = np.random.Generator(np.random.PCG64(seed + 4242))
    out, have = [], 0
    while have < n:
        p = rng.uniform(-box, box, (1 << 16, 3))
        keep = p[radial_mesh_inside(mesh, p)]
        out.append(keep)
        have += keep.shape[0]
    return np.concatenate(out)[:n].astype(np.float32)


def mesh_scene(V, F, bc, name="mesh", g: Fn = None, h: Fn = None, f: Fn = None,
               exact=None) -> Scene:
    return Scene(name, 3, np.asarray(V, np.float32), np.asarray(F, np.int32),
                 np.asarray(bc, np.uint8), g or Fn(FN_ZERO), h or Fn(FN_ZERO),
                 f or Fn(FN_ZERO), exact)


def cube_mesh(lo=(0, 0, 0), hi=(1, 1, 1)):
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    V = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=np.float64)
    F = np.array([[0, 2, 1], [0, 3, 2],      # z = z0, normal -z
                  [4, 5, 6], [4, 6, 7],      # z = z1, normal +z
                  [0, 1, 5], [0, 5, 4],      # y = y0, normal -y
                  [3, 7, 6], [3, 6, 2],      # y = y1, normal +y
                  [0, 4, 7], [0, 7, 3],      # x = x0, normal -x
                  [1, 2, 6], [1, 6, 5]],     # x = x1, normal +x
                 dtype=np.int64)
    return V, F


def l_prism_mesh(height: float = 1.0):
    """The 2D L-shape [0,2]^2 minus [1,2]^2 extruded along z over [0, height].
    Its reflex edge runs along x = y = 1."""
    L2 = np.array([[0, 0], [2, 0], [2, 1], [1, 1], [1, 2], [0, 2]], dtype=np.float64)
    n = 6
    V = np.concatenate([np.c_[L2, np.zeros(n)], np.c_[L2, np.full(n, height)]], axis=0)
    # bottom cap (normal -z) and top cap (normal +z): triangulate the L as a fan
    # from the convex corner 0 plus the notch-side triangle
    cap = [[0, 1, 2], [0, 2, 3], [0, 3, 4], [0, 4, 5]]
    F = []
    for a, b, c in cap:
        F.append([a, c, b])                  # bottom, reversed
        F.append([a + n, b + n, c + n])      # top
    for i in range(n):
        j = (i + 1) % n
        F.append([i, j, j + n])
        F.append([i, j + n, i + n])
    return V, np.array(F, dtype=np.int64)


def tetrahedron_mesh():
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * 0.5
    F = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int64)
    # make every face outward
    c = V[F].mean(1)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (n * c).sum(1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


# --------------------------------------------------------------------------
# double-sided boundaries (open sheets and two-sided closed surfaces)
# --------------------------------------------------------------------------
# harmonic quadratics (zero Laplacian): 2D (c, x, y, xx, yy, xy);
# 3D (c, x, y, z, xx, yy, zz, xy, yz, zx)
U_OUT_2D = (0.3, 1.0, -0.5, 0.4, -0.4, 0.6)
U_IN_2D = (-0.2, 0.7, 0.9, -0.5, 0.5, 0.3)
U_OUT_3D = (0.2, 0.8, -0.3, 0.5, 0.3, -0.1, -0.2, 0.4, -0.5, 0.2)
U_IN_3D = (-0.3, 0.4, 0.6, -0.7, -0.2, 0.5, -0.3, 0.1, 0.3, -0.4)


def _square_boundary(n_side: int, half: float = 1.0):
    """[-half, half]^2 as a counter-clockwise polyline of 4 n_side segments."""
    t = np.linspace(-half, half, n_side + 1)[:-1]
    V = np.concatenate([np.c_[t, np.full(n_side, -half)], np.c_[np.full(n_side, half), t],
                        np.c_[-t, np.full(n_side, half)], np.c_[np.full(n_side, -half), -t]])
    n = V.shape[0]
    i = np.arange(n)
    return V, np.stack([i, (i + 1) % n], 1)


def double_sided_disk_scene(n_circle: int = 256, n_side: int = 16, radius: float = 0.5) -> Scene:
    """Square [-1, 1]^2 with one-sided Dirichlet data u_out, and inside it a
    circle of n_circle segments wound clockwise (normals towards the centre),
    double-sided: Dirichlet on its upper half, Neumann on its lower half.
    Its "+" side is the annulus (data from u_out), its "-" side the disk
    (data from u_in), so the exact solution is u_in inside the circle and
    u_out outside, two different harmonic quadratics."""
    Vs, Ps = _square_boundary(n_side)
    th = -2.0 * np.pi * np.arange(n_circle) / n_circle
    Vc = radius * np.c_[np.cos(th), np.sin(th)]
    i = np.arange(n_circle)
    Pc = np.stack([i, (i + 1) % n_circle], 1) + Vs.shape[0]
    mid = th - np.pi / n_circle
    bcc = np.where(np.sin(mid) > 0, DIRICHLET2, NEUMANN2)
    V = np.concatenate([Vs, Vc]).astype(np.float32)
    P = np.concatenate([Ps, Pc]).astype(np.int32)
    bc = np.concatenate([np.full(Ps.shape[0], DIRICHLET), bcc]).astype(np.uint8)
    uo, ui = _analytic(FN_POLY2, U_OUT_2D), _analytic(FN_POLY2, U_IN_2D)

    def exact(x):
        x = np.asarray(x, np.float64)
        return np.where(np.linalg.norm(x, axis=-1) < radius, ui(x), uo(x))
    return Scene(f"ds_disk_{n_circle}", 2, V, P, bc, Fn(FN_POLY2, 0, U_OUT_2D), Fn(FN_POLY2, 1, U_OUT_2D),
                 Fn(FN_ZERO), exact, g_minus=Fn(FN_POLY2, 0, U_IN_2D), h_minus=Fn(FN_POLY2, 1, U_IN_2D))


def crack_scene_2d(n_crack: int = 64, n_side: int = 16) -> Scene:
    """Square [-1, 1]^2 (one-sided Dirichlet) around an open curved sheet
    y = 0.05 + 0.25 sin(2.5 x), x in [-0.6, 0.5], of n_crack segments: its
    first 30 % double-sided Dirichlet, the rest double-sided Neumann.  The
    data on both sides come from one harmonic u, so u is the solution; the
    Neumann data differ in sign between the sides (h- = du/dn- = -h+)."""
    Vs, Ps = _square_boundary(n_side)
    x = np.linspace(-0.6, 0.5, n_crack + 1)
    Vk = np.c_[x, 0.05 + 0.25 * np.sin(2.5 * x)]
    i = np.arange(n_crack)
    Pk = np.stack([i, i + 1], 1) + Vs.shape[0]
    bck = np.where(i < int(0.3 * n_crack), DIRICHLET2, NEUMANN2)
    V = np.concatenate([Vs, Vk]).astype(np.float32)
    P = np.concatenate([Ps, Pk]).astype(np.int32)
    bc = np.concatenate([np.full(Ps.shape[0], DIRICHLET), bck]).astype(np.uint8)
    g, h = Fn(FN_POLY2, 0, U_OUT_2D), Fn(FN_POLY2, 1, U_OUT_2D)
    return Scene(f"crack2d_{n_crack}", 2, V, P, bc, g, h, Fn(FN_ZERO), _analytic(FN_POLY2, U_OUT_2D),
                 g_minus=g, h_minus=h)


def double_sided_sphere_scene(level: int = 2, radius: float = 0.5) -> Scene:
    """Cube [-1, 1]^3 (one-sided Dirichlet, u_out) around an icosphere of
    radius `radius` whose faces are wound inwards, double-sided: Dirichlet
    where the face centre has z > 0.1, Neumann below.  Exact solution u_in
    inside the sphere, u_out outside (3D analogue of the disk scene)."""
    Vq, Fq = cube_mesh((-1, -1, -1), (1, 1, 1))
    Vi, Fi, _ = icosphere(level)
    Vi = radius * Vi
    Fi = Fi[:, [0, 2, 1]] + Vq.shape[0]
    cen = np.concatenate([Vq, Vi])[Fi].mean(1)
    bci = np.where(cen[:, 2] > 0.1, DIRICHLET2, NEUMANN2)
    V = np.concatenate([Vq, Vi]).astype(np.float32)
    F = np.concatenate([Fq, Fi]).astype(np.int32)
    bc = np.concatenate([np.full(Fq.shape[0], DIRICHLET), bci]).astype(np.uint8)
    uo, ui = _analytic(FN_POLY2, U_OUT_3D), _analytic(FN_POLY2, U_IN_3D)

    def exact(x):
        x = np.asarray(x, np.float64)
        return np.where(np.linalg.norm(x, axis=-1) < radius, ui(x), uo(x))
    return Scene(f"ds_sphere_L{level}", 3, V, F, bc, Fn(FN_POLY2, 0, U_OUT_3D), Fn(FN_POLY2, 1, U_OUT_3D),
                 Fn(FN_ZERO), exact, g_minus=Fn(FN_POLY2, 0, U_IN_3D), h_minus=Fn(FN_POLY2, 1, U_IN_3D))


def crack_scene_3d(n_grid: int = 12) -> Scene:
    """Cube [-1, 1]^3 (one-sided Dirichlet) around an open wavy sheet
    z = 0.1 + 0.15 sin(2x) cos(2y) over [-0.5, 0.5]^2, 2 n_grid^2 triangles:
    double-sided Dirichlet where x < -0.25, double-sided Neumann elsewhere,
    data from one harmonic u on both sides (u is the solution)."""
    Vq, Fq = cube_mesh((-1, -1, -1), (1, 1, 1))
    t = np.linspace(-0.5, 0.5, n_grid + 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    Vs = np.c_[X.ravel(), Y.ravel(), (0.1 + 0.15 * np.sin(2 * X) * np.cos(2 * Y)).ravel()]
    idx = np.arange((n_grid + 1) ** 2).reshape(n_grid + 1, n_grid + 1)
    a, b = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel()
    c, d = idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    Fs = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]) + Vq.shape[0]
    V = np.concatenate([Vq, Vs])
    cen = V[Fs].mean(1)
    bcs = np.where(cen[:, 0] < -0.25, DIRICHLET2, NEUMANN2)
    F = np.concatenate([Fq, Fs]).astype(np.int32)
    bc = np.concatenate([np.full(Fq.shape[0], DIRICHLET), bcs]).astype(np.uint8)
    g, h = Fn(FN_POLY2, 0, U_OUT_3D), Fn(FN_POLY2, 1, U_OUT_3D)
    return Scene(f"crack3d_{n_grid}", 3, V.astype(np.float32), F, bc, g, h, Fn(FN_ZERO),
                 _analytic(FN_POLY2, U_OUT_3D), g_minus=g, h_minus=h)


# --------------------------------------------------------------------------
# mixed representations: analytic (SDF) Dirichlet shapes with a mesh
# --------------------------------------------------------------------------

def regular_polygon(n: int, radius: float, centre=(0.0, 0.0), clockwise: bool = False):
    th = 2.0 * np.pi * np.arange(n) / n
    if clockwise:
        th = -th
    V = np.c_[centre[0] + radius * np.cos(th), centre[1] + radius * np.sin(th)]
    i = np.arange(n)
    return V, np.stack([i, (i + 1) % n], 1)


def sdf_rocks_scene_2d(n_obstacle: int = 256, with_mesh: bool = True) -> Scene:
    """Disk of radius 1 (an inside ball: Dirichlet) holding three analytic
    rocks (a rounded box, a capsule, a ball: Dirichlet) and a Neumann
    obstacle, a regular polygon of n_obstacle segments and radius 0.18 wound
    clockwise so that its normals point out of the domain.  Data from one
    harmonic quadratic u (g = u, h = du/dn), so u is the solution."""
    shapes = [Sdf(SDF_BALL, 1, (0.0, 0.0, 0.0, 0, 0, 0, 1.0)),
              Sdf(SDF_BOX, 0, (-0.3, -0.45, 0.0, 0.25, 0.12, 0.0, 0.05)),
              Sdf(SDF_CAPSULE, 0, (0.15, -0.55, 0.0, 0.55, -0.3, 0.0, 0.08)),
              Sdf(SDF_BALL, 0, (0.45, 0.35, 0.0, 0, 0, 0, 0.15))]
    if with_mesh:
        V, P = regular_polygon(n_obstacle, 0.18, (-0.25, 0.3), clockwise=True)
        bc = np.full(n_obstacle, NEUMANN, np.uint8)
    else:
        V, P, bc = np.zeros((0, 2)), np.zeros((0, 2), np.int64), np.zeros(0, np.uint8)
    g, h = Fn(FN_POLY2, 0, U_OUT_2D), Fn(FN_POLY2, 1, U_OUT_2D)
    return Scene(f"sdf_rocks2d_{n_obstacle if with_mesh else 0}", 2, V.astype(np.float32), P.astype(np.int32), bc,
                 g, h, Fn(FN_ZERO), _analytic(FN_POLY2, U_OUT_2D), sdf=shapes)


def sdf_rocks_scene_3d(level: int = 3, with_mesh: bool = True) -> Scene:
    """Ball of radius 1.2 (inside: Dirichlet) holding analytic rocks (two
    rounded boxes, a capsule, a ball: Dirichlet) and a Neumann obstacle, an
    icosphere of radius 0.25 wound inwards.  One harmonic quadratic u."""
    shapes = [Sdf(SDF_BALL, 1, (0.0, 0.0, 0.0, 0, 0, 0, 1.2)),
              Sdf(SDF_BOX, 0, (-0.35, -0.5, -0.1, 0.3, 0.12, 0.25, 0.06)),
              Sdf(SDF_BOX, 0, (0.4, -0.45, 0.3, 0.15, 0.15, 0.15, 0.0)),
              Sdf(SDF_CAPSULE, 0, (0.2, -0.6, -0.5, 0.5, -0.3, -0.2, 0.1)),
              Sdf(SDF_BALL, 0, (0.45, 0.4, -0.3, 0, 0, 0, 0.2))]
    if with_mesh:
        Vi, Fi, _ = icosphere(level)
        V = 0.25 * Vi + np.array([-0.2, 0.3, 0.2])
        F = Fi[:, [0, 2, 1]]
        bc = np.full(F.shape[0], NEUMANN, np.uint8)
    else:
        V, F, bc = np.zeros((0, 3)), np.zeros((0, 3), np.int64), np.zeros(0, np.uint8)
    g, h = Fn(FN_POLY2, 0, U_OUT_3D), Fn(FN_POLY2, 1, U_OUT_3D)
    return Scene(f"sdf_rocks3d_L{level if with_mesh else 'none'}", 3, V.astype(np.float32), F.astype(np.int32), bc,
                 g, h, Fn(FN_ZERO), _analytic(FN_POLY2, U_OUT_3D), sdf=shapes)


MIXED_CENTRE = (0.0, 0.35, 0.0)
MIXED_SCALE = 0.35


def mixed_scene(level: int = 8, seed: int = 0, n_rocks: int = 16, mesh: "RadialMesh" = None) -> Scene:
    """Stand-in for the paper's mixed-representation heat scene (a
    1.2-million-triangle Neumann mesh resting on rocks given as signed
    distance functions): a displaced icosphere of 20 * 4^level triangles
    (level 8: 1,310,720), scaled by 0.35 and wound inwards (it is an
    obstacle: its normals point out of the domain), all Neumann; below it a
    seeded pile of n_rocks analytic rocks (rounded boxes, balls, capsules);
    everything inside a Dirichlet ball of radius 1.6.  Data from one
    harmonic quadratic u (g = u on the rocks and the ball, h = du/dn on the
    mesh), so u is the solution."""
    if mesh is None:
        mesh = displaced_icosphere(level, seed)
    V = MIXED_SCALE * mesh.V + np.asarray(MIXED_CENTRE)
    F = mesh.F[:, [0, 2, 1]]
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    reach = 1.2 * MIXED_SCALE + 0.05          # the mesh lies within this of its centre
    shapes = [Sdf(SDF_BALL, 1, (0.0, 0.0, 0.0, 0, 0, 0, 1.6))]
    while len(shapes) < n_rocks + 1:
        kind = int(rng.integers(0, 3))
        size = float(rng.uniform(0.08, 0.25))
        c = np.array([rng.uniform(-1.0, 1.0), rng.uniform(-0.9, -0.15), rng.uniform(-1.0, 1.0)])
        if np.linalg.norm(c) + 2 * size > 1.5 or np.linalg.norm(c - np.asarray(MIXED_CENTRE)) < reach + 2 * size:
            continue
        if kind == SDF_BALL:
            shapes.append(Sdf(SDF_BALL, 0, (*c, 0, 0, 0, size)))
        elif kind == SDF_BOX:
            e = rng.uniform(0.4, 1.0, 3) * size
            shapes.append(Sdf(SDF_BOX, 0, (*c, *e, 0.3 * size)))
        else:
            d = rng.normal(size=3)
            d = 0.8 * size * d / np.linalg.norm(d)
            shapes.append(Sdf(SDF_CAPSULE, 0, (*(c - d), *(c + d), 0.5 * size)))
    g, h = Fn(FN_POLY2, 0, U_OUT_3D), Fn(FN_POLY2, 1, U_OUT_3D)
    return Scene(f"mixed_L{level}_s{seed}", 3, V.astype(np.float32), F.astype(np.int32),
                 np.full(F.shape[0], NEUMANN, np.uint8), g, h, Fn(FN_ZERO), _analytic(FN_POLY2, U_OUT_3D),
                 sdf=shapes)


def crack_in_ball_scene_2d(n_crack: int = 64) -> Scene:
    """The open double-sided sheet of crack_scene_2d (30 % Dirichlet, 70 %
    Neumann) inside an analytic Dirichlet disk of radius 1 instead of the
    meshed square: both extensions in one scene, one harmonic u."""
    base = crack_scene_2d(n_crack=n_crack)
    keep = base.bc >= DIRICHLET2
    used = np.unique(base.prims[keep])
    remap = -np.ones(base.vertices.shape[0], np.int64)
    remap[used] = np.arange(used.size)
    return dataclasses.replace(base, name=f"crack_in_ball_{n_crack}", vertices=base.vertices[used],
                               prims=remap[base.prims[keep]].astype(np.int32), bc=base.bc[keep].copy(),
                               sdf=[Sdf(SDF_BALL, 1, (0.0, 0.0, 0.0, 0, 0, 0, 1.0))])


def sdf_scene_points(spec: Scene, n: int, seed: int, margin: float = 0.02, obstacle=None) -> np.ndarray:
    """Uniform points of the domain of a scene with analytic shapes: inside
    every inside shape and outside every outside one by `margin`, and
    outside the ball (centre, radius) `obstacle` that encloses the mesh."""
    rng = np.random.default_rng(seed)
    dim = spec.dim
    enc = [f for f in spec.sdf if f.inside]
    half = max(f.p8()[6] if f.kind == SDF_BALL else float(np.max(f.p8()[3:3 + dim])) for f in enc)
    out, have = [], 0
    while have < n:
        p = rng.uniform(-half, half, size=(4 * n, dim))
        ok = np.ones(p.shape[0], bool)
        for f in spec.sdf:
            ok &= f.value(p) > margin
        if obstacle is not None:
            ok &= np.linalg.norm(p - np.asarray(obstacle[0])[:dim], axis=1) > obstacle[1] + margin
        out.append(p[ok])
        have += int(ok.sum())
    return np.concatenate(out)[:n].astype(np.float32)


def box_points(n: int, dim: int, seed: int, half: float = 0.95, avoid_radius: float = None,
               margin: float = 0.05) -> np.ndarray:
    """Uniform points in [-half, half]^dim; with avoid_radius, none within
    margin of the sphere of that radius."""
    rng = np.random.default_rng(seed)
    out, have = [], 0
    while have < n:
        p = rng.uniform(-half, half, size=(2 * n, dim))
        if avoid_radius is not None:
            p = p[np.abs(np.linalg.norm(p, axis=1) - avoid_radius) > margin]
        out.append(p)
        have += p.shape[0]
    return np.concatenate(out)[:n].astype(np.float32)


# --------------------------------------------------------------------------
# Workloads: scene, points, walks, eps and seed
# --------------------------------------------------------------------------

def unit_square_case(n_grid: int = 32):
    """Unit square, 32x32 cell-centre points, 256 walks, eps 1e-3, seed 0."""
    return dict(scene=unit_square_scene(), points=grid_points_2d(n_grid),
                walks=256, eps=1e-3, seed=0)


def star_polygon_case(n_points: int = 262144, n_seg: int = 16384, seed: int = 0, walks: int = 1024):
    """Star polygon, 16,384 segments, 262,144 points, 1024 walks, eps 1e-4."""
    sc = star_polygon_scene(n_seg, seed)
    pts = star_polygon_points(n_points, seed=seed, vertices=sc.vertices)
    return dict(scene=sc, points=pts, walks=walks, eps=1e-4, seed=seed)


def icosphere_case(n_points: int = 1_000_000, level: int = 8, seed: int = 0, walks: int = 512):
    """Displaced icosphere, 1.3M triangles, 1M points, 512 walks, eps 1e-4."""
    mesh = displaced_icosphere(level, seed)
    sc = displaced_icosphere_scene(level, seed, mesh=mesh)
    pts = radial_mesh_points(mesh, n_points, seed)
    return dict(scene=sc, points=pts, walks=walks, eps=1e-4, seed=seed, mesh=mesh)


# --------------------------------------------------------------------------
# Many displaced geodesic spheres of uneven sizes (the batched workload)
# --------------------------------------------------------------------------

def geodesic_sphere(freq: int):
    """Class-I geodesic sphere: every icosahedron face split into freq^2
    triangles, vertices projected to the unit sphere (20 freq^2 triangles).
    Vertices shared along icosahedron edges and corners are merged by exact
    integer keys of their barycentric position."""
    V0, F0 = _icosahedron()
    n = freq
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    keep = ii + jj <= n
    I_, J_ = ii[keep], jj[keep]            # weights of corners b and c
    K_ = n - I_ - J_                       # weight of corner a
    nf = F0.shape[0]
    keys, pos = [], []
    base = np.int64(n + 1)
    for f in range(nf):
        a, b, c = F0[f]
        w = {a: K_, b: I_, c: J_}
        # key: sorted (corner, weight) pairs with positive weight
        corners = np.stack([np.full_like(I_, a), np.full_like(I_, b), np.full_like(I_, c)], 1)
        weights = np.stack([K_, I_, J_], 1)
        corners = np.where(weights > 0, corners, 99)     # zero weights sort last
        order = np.argsort(corners, axis=1)
        cs = np.take_along_axis(corners, order, 1)
        ws = np.take_along_axis(weights, order, 1)
        ws_pos = ws > 0
        # encode: for each of the 3 sorted corners, (corner+1)*(n+1)+weight if weight>0 else 0
        code = np.zeros(I_.shape[0], dtype=np.int64)
        for k in range(3):
            term = np.where(ws_pos[:, k], (cs[:, k].astype(np.int64) + 1) * base + ws[:, k], 0)
            code = code * np.int64(13 * (n + 1) + 1) + term
        keys.append(code)
        p = (K_[:, None] * V0[a] + I_[:, None] * V0[b] + J_[:, None] * V0[c]) / n
        pos.append(p)
    keys = np.concatenate(keys)
    pos = np.concatenate(pos)
    uk, first, inv = np.unique(keys, return_index=True, return_inverse=True)
    V = pos[first]
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # local grid index -> global vertex id per face
    npf = I_.shape[0]
    lid = -np.ones((n + 1, n + 1), dtype=np.int64)
    lid[I_, J_] = np.arange(npf)
    tris = []
    for f in range(nf):
        g = inv[f * npf:(f + 1) * npf]
        up_i, up_j = np.nonzero((np.add.outer(np.arange(n + 1), np.arange(n + 1)) <= n - 1))
        t_up = np.stack([g[lid[up_i, up_j]], g[lid[up_i + 1, up_j]], g[lid[up_i, up_j + 1]]], 1)
        dn_i, dn_j = np.nonzero((np.add.outer(np.arange(n + 1), np.arange(n + 1)) <= n - 2))
        t_dn = np.stack([g[lid[dn_i + 1, dn_j]], g[lid[dn_i + 1, dn_j + 1]], g[lid[dn_i, dn_j + 1]]], 1)
        tris.append(t_up)
        tris.append(t_dn)
    F = np.concatenate(tris)
    return V, F


def geodesic_inside(V_disp: np.ndarray, F: np.ndarray, p: np.ndarray, freq: int) -> np.ndarray:
    """Exact inside test for a radially displaced geodesic sphere: the ray
    from the origin along p crosses exactly one triangle (the one whose cone
    contains p); it is found among candidates near the icosahedron-face
    barycentric estimate, then the crossing radius is compared with |p|."""
    Vd = V_disp.astype(np.float64)
    U = Vd / np.linalg.norm(Vd, axis=1, keepdims=True)
    r = np.linalg.norm(p, axis=1)
    d = p / np.maximum(r, 1e-300)[:, None]
    # candidate triangles: a coarse angular hash of triangle centroids
    cen = U[F].mean(1)
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    from scipy.spatial import cKDTree
    tree = cKDTree(cen)
    k = 12
    _, cand = tree.query(d, k=k)
    A, B, C = U[F[cand, 0]], U[F[cand, 1]], U[F[cand, 2]]
    dd = d[:, None, :]
    s0 = (np.cross(A, B) * dd).sum(-1)
    s1 = (np.cross(B, C) * dd).sum(-1)
    s2 = (np.cross(C, A) * dd).sum(-1)
    score = np.minimum(np.minimum(s0, s1), s2)
    best = cand[np.arange(len(d)), np.argmax(score, 1)]
    a, b, c = Vd[F[best, 0]], Vd[F[best, 1]], Vd[F[best, 2]]
    nrm = np.cross(b - a, c - a)
    t = (nrm * a).sum(1) / (nrm * d).sum(1)
    return r < t


def geodesic_outside_distance(V_disp: np.ndarray, F: np.ndarray, p: np.ndarray, freq: int) -> np.ndarray:
    """Signed distance of p from the plane of the triangle that the ray from
    the origin through p crosses, positive outside the displaced geodesic
    sphere (the same triangle search as geodesic_inside)."""
    Vd = V_disp.astype(np.float64)
    p = np.asarray(p, np.float64)
    U = Vd / np.linalg.norm(Vd, axis=1, keepdims=True)
    r = np.linalg.norm(p, axis=1)
    d = p / np.maximum(r, 1e-300)[:, None]
    cen = U[F].mean(1)
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    from scipy.spatial import cKDTree
    _, cand = cKDTree(cen).query(d, k=12)
    A, B, C = U[F[cand, 0]], U[F[cand, 1]], U[F[cand, 2]]
    dd = d[:, None, :]
    score = np.minimum(np.minimum((np.cross(A, B) * dd).sum(-1), (np.cross(B, C) * dd).sum(-1)),
                       (np.cross(C, A) * dd).sum(-1))
    best = cand[np.arange(len(d)), np.argmax(score, 1)]
    a, b, c = Vd[F[best, 0]], Vd[F[best, 1]], Vd[F[best, 2]]
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return ((p - a) * nrm).sum(1)


def geodesic_batch_case(n_scenes: int = 64, seed: int = 0, scale: float = 1.0, only=None):
    """64 displaced geodesic spheres, 2k-800k triangles (log-uniform), a
    random planar Dirichlet/Neumann split each, exact u = x^2 - y^2 + z;
    per scene 1k-256k points and 128-1024 walks (log-uniform).  `scale`
    shrinks triangle and point counts for tests; `only` (a collection of
    scene indices) builds just those scenes, identical to their entries in
    the whole batch."""
    rng = np.random.Generator(np.random.PCG64(seed + 99))
    items = []
    coef = (0.0, 0.0, 0.0, 1.0, 1.0, -1.0, 0.0, 0.0, 0.0, 0.0)   # x^2 - y^2 + z
    for s in range(n_scenes):
        T = math.exp(rng.uniform(math.log(2000), math.log(800000))) * scale
        freq = max(2, int(round(math.sqrt(T / 20))))
        npts = int(round(math.exp(rng.uniform(math.log(1000), math.log(262144))) * scale))
        npts = max(16, npts)
        walks = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        tau = rng.uniform(-0.5, 0.5)
        if only is not None and s not in only:
            continue
        V, F = geodesic_sphere(freq)
        rho = 1.0 + 0.2 * value_noise(V, s)
        Vd = V * rho[:, None]
        cen = Vd[F].mean(1)
        bc = np.where(cen @ a > tau, DIRICHLET, NEUMANN).astype(np.uint8)
        g, h, f, u = solution_data(FN_POLY2, coef)
        spec = Scene(f"geodesic_f{freq}_s{s}", 3, Vd.astype(np.float32), F.astype(np.int32), bc, g, h, f,
                     exact=u)
        prng = np.random.Generator(np.random.PCG64(seed * 1000 + s))
        out, have = [], 0
        while have < npts:
            q = prng.uniform(-1.2, 1.2, (max(2048, 3 * (npts - have)), 3))
            keep = q[geodesic_inside(Vd, F, q, freq)]
            out.append(keep)
            have += keep.shape[0]
        pts = np.concatenate(out)[:npts].astype(np.float32)
        items.append(dict(scene=spec, points=pts, walks=walks, eps=1e-4, seed=seed * 1000 + s))
    return items
