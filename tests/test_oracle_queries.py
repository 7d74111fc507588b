"""Pins of the oracle's geometric queries (Sec. 5: Q.1 closest point, Q.2
closest silhouette point, Q.3 ray intersection, Q.4 point sampling) against
closed forms worked out by hand on tiny meshes and against dense sampling."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I


def _tri_scene(V, bc=I.DIRICHLET):
    return O.Scene(I.mesh_scene(V, [[0, 1, 2]], [bc]))


def test_closest_point_triangle_vs_dense_sampling():
    rng = np.random.default_rng(3)
    m = 200
    a, b = np.meshgrid(np.linspace(0, 1, m + 1), np.linspace(0, 1, m + 1))
    keep = a + b <= 1
    bary = np.stack([1 - a[keep] - b[keep], a[keep], b[keep]], 1)
    for _ in range(25):
        V = rng.normal(size=(3, 3)).astype(np.float32)
        S = _tri_scene(V)
        pts = bary @ V.astype(np.float64)
        h = max(np.linalg.norm(V[i] - V[j]) for i in range(3) for j in range(3)) / m
        for _ in range(8):
            x = rng.normal(size=3) * 1.5
            d, xb, prim = S.closest_dirichlet(x)
            dense = np.linalg.norm(pts - x, axis=1).min()
            assert prim == 0
            assert d <= dense + 1e-12
            assert dense - d <= h
            assert abs(np.linalg.norm(xb - x) - d) < 1e-12


def test_closest_point_unit_square():
    S = O.Scene(I.unit_square_scene())
    for x in I.grid_points_2d(8):
        d, xb, prim = S.closest_dirichlet(x)
        assert d == pytest.approx(min(x[0], 1 - x[0]), abs=1e-15)
        assert prim in (1, 3)


def test_closest_point_cube_all_dirichlet():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.zeros(12)))
    rng = np.random.default_rng(4)
    for x in rng.uniform(0.02, 0.98, (50, 3)):
        d, _, _ = S.closest_dirichlet(x)
        assert d == pytest.approx(min(x.min(), (1 - x).min()), abs=1e-12)


def test_no_dirichlet_gives_infinite_distance():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.ones(12)))
    d, _, prim = S.closest_dirichlet([0.5, 0.5, 0.5])
    assert math.isinf(d) and prim == -1


# ---- Q.2: silhouettes -------------------------------------------------------
# L-shape [0,2]^2 \ [1,2]^2, all Neumann.  Worked by hand from the silhouette
# condition (v.n1)(v.n2) <= 0: from a point of the lower-left block every
# vertex sees both of its edges from the inside, so there is no silhouette;
# from a point in either arm the reflex corner (1,1) is a silhouette and is
# the closest one.

def _l_closed_form(x, rmax):
    if x[0] > 1 or x[1] > 1:
        return min(rmax, math.hypot(x[0] - 1, x[1] - 1))
    return rmax


def test_silhouette_l_shape_2d():
    S = O.Scene(I.l_shape_2d())
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.01, 1.99, (400, 2))
    pts = pts[~((pts[:, 0] > 1) & (pts[:, 1] > 1))]
    for x in pts:
        for rmax in (math.inf, 0.5):
            assert S.silhouette(x, rmax) == pytest.approx(_l_closed_form(x, rmax), abs=1e-14)


def test_silhouette_l_prism_3d():
    V, F = I.l_prism_mesh(1.0)
    S = O.Scene(I.mesh_scene(V, F, np.ones(len(F))))
    rng = np.random.default_rng(6)
    pts = rng.uniform(0.01, 1.99, (300, 2))
    pts = pts[~((pts[:, 0] > 1) & (pts[:, 1] > 1))]
    z = rng.uniform(0.05, 0.95, pts.shape[0])
    for (x, y), zz in zip(pts, z):
        got = S.silhouette([x, y, zz])
        assert got == pytest.approx(_l_closed_form((x, y), math.inf), abs=1e-12)


def test_silhouette_convex_is_empty():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.ones(12)))
    rng = np.random.default_rng(7)
    for x in rng.uniform(0.01, 0.99, (60, 3)):
        assert S.silhouette(x, 5.0) == 5.0


def test_silhouette_open_mesh_boundary_edges():
    """Every boundary edge of the Neumann mesh is a silhouette (Sec. 5.1):
    for the flat square [0,1]^2 x {0} the distance is that to its border."""
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    S = O.Scene(I.mesh_scene(V, [[0, 1, 2], [0, 2, 3]], [1, 1]))
    rng = np.random.default_rng(8)
    for _ in range(50):
        x = np.array([*rng.uniform(0.05, 0.95, 2), rng.uniform(-0.5, 0.5)])
        border = min(x[0], 1 - x[0], x[1], 1 - x[1])
        assert S.silhouette(x) == pytest.approx(math.hypot(border, x[2]), abs=1e-12)


def test_silhouette_from_offset_surface_point():
    """A point just inside a flat Neumann face: coplanar neighbours are not
    silhouettes, a convex fold is not, a concave (reflex) fold is."""
    V, F = I.l_prism_mesh(1.0)
    S = O.Scene(I.mesh_scene(V, F, np.ones(len(F))))
    off = 1e-6
    # on the bottom cap (normal -z) near the middle of the lower-left block
    assert S.silhouette([0.5, 0.5, off], 10.0) == 10.0
    # on the bottom cap inside the right arm: the reflex edge is a silhouette
    d = S.silhouette([1.5, 0.6, off], 10.0)
    assert d == pytest.approx(math.hypot(0.5, 0.4), abs=1e-5)


# ---- Q.3: rays ------------------------------------------------------------

def test_ray_box_closed_form():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.ones(12)))
    rng = np.random.default_rng(9)
    for _ in range(200):
        o = rng.uniform(0.05, 0.95, 3)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        t_exact = min(((1 - o[i]) / v[i]) if v[i] > 0 else (-o[i] / v[i]) for i in range(3))
        prim, t = S.ray_neumann(o, v, 10.0)
        assert prim >= 0 and t == pytest.approx(t_exact, rel=1e-12)
        prim, t = S.ray_neumann(o, v, 0.5 * t_exact)
        assert prim == -1 and t == 0.5 * t_exact


def test_ray_through_shared_vertex_and_edge_hits():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.ones(12)))
    o = np.array([0.5, 0.5, 0.5])
    for target in ([1, 1, 1], [0, 0, 0], [1, 0.5, 1], [0.5, 0.5, 1], [0, 1, 0.25]):
        v = np.array(target, float) - o
        L = np.linalg.norm(v)
        prim, t = S.ray_neumann(o, v / L, 10.0)
        assert prim >= 0 and t == pytest.approx(L, rel=1e-12)
    sq = O.Scene(I.polygon_scene([[0, 0], [1, 0], [1, 1], [0, 1]], [1, 1, 1, 1]))
    prim, t = sq.ray_neumann([0.5, 0.5], np.array([1, 1]) / math.sqrt(2), 10.0)
    assert prim >= 0 and t == pytest.approx(math.sqrt(0.5), rel=1e-12)


def test_ray_skip_lists():
    sq = O.Scene(I.polygon_scene([[0, 0], [1, 0], [1, 1], [0, 1]], [1, 1, 1, 1]))
    prim, t = sq.ray_neumann([0.5, 0.5], [1, 0], 10.0)
    assert prim == 1 and t == pytest.approx(0.5)
    prim, t = sq.ray_neumann([0.5, 0.5], [1, 0], 10.0, skip0=1)
    assert prim == -1


# ---- Q.4: Neumann point sampling ---------------------------------------------

def _flat_neumann_2d(n=64, half=4.0):
    xs = np.linspace(-half, half, n + 1)
    V = np.stack([xs, np.zeros_like(xs)], 1)
    P = np.stack([np.arange(n), np.arange(1, n + 1)], 1)
    return I.Scene("line", 2, V.astype(np.float32), P.astype(np.int32),
                   np.ones(n, np.uint8), I.Fn(), I.Fn(), I.Fn())


def test_neumann_sample_unbiased_chord_2d():
    """E[1{|z-x|<r} / pdf] = length of the Neumann line inside B(x, r)
    (support extension, Sec. 4.5): 2 sqrt(r^2 - d^2)."""
    S = O.Scene(_flat_neumann_2d())
    rng = np.random.default_rng(10)
    for d, r in ((0.3, 1.0), (0.05, 0.4), (0.9, 1.0)):
        x = np.array([0.123, d])
        est = []
        for u in rng.random((4000, 3)):
            prim, z, pdf = S.neumann_sample(x, r, *u)
            assert prim >= 0
            est.append((np.linalg.norm(z - x) < r) / pdf)
        est = np.array(est)
        exact = 2 * math.sqrt(r * r - d * d)
        assert abs(est.mean() - exact) < 4 * est.std() / math.sqrt(est.size) + 1e-12


def test_neumann_sample_unbiased_disk_3d():
    """Same identity on a triangulated Neumann plane: area pi (r^2 - d^2)."""
    n = 16
    xs = np.linspace(-2, 2, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
    idx = lambda i, j: i * (n + 1) + j
    F = []
    for i in range(n):
        for j in range(n):
            F.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)])
            F.append([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)])
    S = O.Scene(I.mesh_scene(V, F, np.ones(len(F))))
    rng = np.random.default_rng(11)
    x = np.array([0.1, -0.2, 0.35])
    r = 0.9
    est = []
    for u in rng.random((6000, 3)):
        prim, z, pdf = S.neumann_sample(x, r, *u)
        est.append((np.linalg.norm(z - x) < r) / pdf)
    est = np.array(est)
    exact = math.pi * (r * r - x[2] ** 2)
    assert abs(est.mean() - exact) < 4 * est.std() / math.sqrt(est.size)


def test_neumann_sample_support_and_empty():
    S = O.Scene(_flat_neumann_2d(n=8, half=4.0))
    x = np.array([0.0, 0.5])
    r = 1.2          # meets the segments over [-1.09, 1.09]: the 4 around 0
    hit = set()
    for u in np.linspace(0, 1, 400, endpoint=False):
        prim, z, pdf = S.neumann_sample(x, r, u, 0.5, 0.5)
        hit.add(prim)
        assert pdf == pytest.approx(1 / 4.0)
    assert hit == {2, 3, 4, 5}
    prim, z, pdf = S.neumann_sample(np.array([0.0, 3.0]), 1.0, 0.3, 0.3, 0.3)
    assert prim == -1 and pdf == 0.0


# ---- Q.3 from a position on the boundary up to rounding (reading R13) -------

def test_ray_just_behind_leaving_counts_at_zero_2d():
    # unit square, Neumann on y = 0 (primitive 0, outward normal -y) and y = 1
    sq = O.Scene(I.unit_square_scene())
    behind = 1e-6
    # just outside y = 0, leaving through it: a crossing at t = -1e-9
    p, t = sq.ray_neumann([0.3, -1e-9], [0.0, -1.0], 10.0, behind=behind)
    assert p == 0 and t == 0.0
    # without the rule the ray passes and finds nothing
    p, t = sq.ray_neumann([0.3, -1e-9], [0.0, -1.0], 10.0)
    assert p == -1 and t == 10.0
    # entering from just outside: an ordinary crossing ahead
    p, t = sq.ray_neumann([0.3, -1e-9], [0.0, 1.0], 10.0, behind=behind)
    assert p == 0 and t == pytest.approx(1e-9, abs=1e-15)
    # farther behind than the bound: no crossing
    p, t = sq.ray_neumann([0.3, -1e-5], [0.0, -1.0], 10.0, behind=behind)
    assert p == -1
    # inside and heading away from y = 0: the crossing behind enters, not counted
    p, t = sq.ray_neumann([0.3, 1e-9], [0.0, 1.0], 10.0, behind=behind)
    assert p == 2 and t == pytest.approx(1.0 - 1e-9, abs=1e-12)


def test_ray_just_behind_leaving_grazing():
    """The distance behind is measured across the primitive's plane: a
    grazing ray from just outside crosses far back along the ray (up to
    256 behind), and still counts; a point farther from the plane than the
    bound does not."""
    sq = O.Scene(I.unit_square_scene())
    behind = 1e-6
    c = 0.008                                   # v . n for the outward normal -y
    v = [math.sqrt(1 - c * c), -c]
    # 1e-7 outside y = 0: the crossing lies at t = -1.25e-5, far beyond -behind
    p, t = sq.ray_neumann([0.3, -1e-7], v, 10.0, behind=behind)
    assert p == 0 and t == 0.0
    # 2e-6 outside: beyond the bound across the plane
    p, t = sq.ray_neumann([0.3, -2e-6], v, 10.0, behind=behind)
    assert p == -1
    # the search reaches back 256 behind along the ray: a crossing at
    # t = -5e-4 (1e-7 across, v . n = 2e-4) lies beyond it
    c2 = 2e-4
    p, t = sq.ray_neumann([0.3, -1e-7], [math.sqrt(1 - c2 * c2), -c2], 10.0, behind=behind)
    assert p == -1
    # 3D: just above the cube's top face z = 1, leaving at a grazing angle
    V, F = I.cube_mesh()
    cube = O.Scene(I.mesh_scene(V, F, np.r_[0, 0, np.ones(10)].astype(np.uint8)))
    w = [math.sqrt(1 - c * c), 0.0, c]
    p, t = cube.ray_neumann([0.5, 0.25, 1.0 + 1e-7], w, 5.0, behind=behind)
    assert p == 2 and t == 0.0
    p, t = cube.ray_neumann([0.5, 0.25, 1.0 + 2e-6], w, 5.0, behind=behind)
    assert p == -1


def test_ray_just_behind_leaving_3d_and_double_sided():
    V, F = I.cube_mesh()
    bc = np.r_[0, 0, np.ones(10)].astype(np.uint8)
    cube = O.Scene(I.mesh_scene(V, F, bc))
    o, v = [0.5, 0.25, 1.0 + 1e-9], [0.0, 0.0, 1.0]     # just above the top face z = 1, leaving
    p, t = cube.ray_neumann(o, v, 5.0, behind=1e-6)
    assert p == 2 and t == 0.0                          # triangle (4, 5, 6) holds (0.5, 0.25)
    # a double-sided primitive has no outside: the rule does not apply
    bc2 = bc.copy()
    bc2[2] = I.NEUMANN2
    sheet = O.Scene(I.mesh_scene(V, F, bc2))
    p, t = sheet.ray_neumann(o, v, 5.0, behind=1e-6)
    assert p == -1
