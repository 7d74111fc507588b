"""Pins of the oracle's analytic Dirichlet shapes (mixed representations,
Sec. 6; Q.1 is the only query a Dirichlet boundary takes part in): closest
points against brute force over densely sampled surfaces, the signed
distance of the input generator, and closed-form solutions of scenes that
mix shapes with a Neumann mesh.  CPU only."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I

SHAPES_2D = [I.Sdf(I.SDF_BALL, 0, (0.1, -0.2, 0, 0, 0, 0, 0.3)),
             I.Sdf(I.SDF_BALL, 1, (0.1, -0.2, 0, 0, 0, 0, 0.9)),
             I.Sdf(I.SDF_BOX, 0, (0.2, 0.1, 0, 0.3, 0.15, 0, 0.0)),
             I.Sdf(I.SDF_BOX, 0, (0.2, 0.1, 0, 0.3, 0.15, 0, 0.07)),
             I.Sdf(I.SDF_BOX, 1, (0.0, 0.0, 0, 0.8, 0.6, 0, 0.0)),
             I.Sdf(I.SDF_CAPSULE, 0, (-0.3, 0.1, 0, 0.4, -0.2, 0, 0.1))]
SHAPES_3D = [I.Sdf(I.SDF_BALL, 0, (0.1, -0.2, 0.05, 0, 0, 0, 0.3)),
             I.Sdf(I.SDF_BALL, 1, (0.0, 0.0, 0.0, 0, 0, 0, 0.9)),
             I.Sdf(I.SDF_BOX, 0, (0.2, 0.1, -0.1, 0.3, 0.15, 0.2, 0.0)),
             I.Sdf(I.SDF_BOX, 0, (0.2, 0.1, -0.1, 0.3, 0.15, 0.2, 0.08)),
             I.Sdf(I.SDF_BOX, 1, (0.0, 0.0, 0.0, 0.8, 0.6, 0.7, 0.0)),
             I.Sdf(I.SDF_CAPSULE, 0, (-0.3, 0.1, 0.2, 0.4, -0.2, -0.1, 0.12))]


def _domain_points(shape, dim, n, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, (20 * n, dim))
    return p[shape.value(p) > 1e-3][:n]


def _surface_cloud(shape, dim, seed, n=4_000_000 // 1, h=1.5e-3):
    """Points within h of the surface, by rejection in a box around it; the
    surface test uses the input generator's signed distance."""
    rng = np.random.default_rng(seed)
    c = shape.p8()
    if shape.kind == I.SDF_BALL:
        lo, hi = c[:dim] - c[6], c[:dim] + c[6]
    elif shape.kind == I.SDF_BOX:
        lo, hi = c[:dim] - c[3:3 + dim] - c[6], c[:dim] + c[3:3 + dim] + c[6]
    else:
        lo = np.minimum(c[:dim], c[3:3 + dim]) - c[6]
        hi = np.maximum(c[:dim], c[3:3 + dim]) + c[6]
    lo, hi = lo - 2 * h, hi + 2 * h
    out = []
    for _ in range(4 if dim == 3 else 1):
        y = rng.uniform(lo, hi, (n if dim == 2 else n // 2, dim))
        out.append(y[np.abs(shape.value(y)) < h])
    return np.concatenate(out)


@pytest.mark.parametrize("dim", [2, 3])
def test_closest_point_is_on_the_surface_at_the_distance(dim):
    """The closest point lies on the surface (the generator's signed distance
    is zero there), at the returned distance, which equals the magnitude of
    the signed distance of the query point."""
    for i, shape in enumerate(SHAPES_2D if dim == 2 else SHAPES_3D):
        for x in _domain_points(shape, dim, 40, i):
            d, o = O.sdf_closest(dim, shape, x)
            assert abs(shape.value(o[None])[0]) < 1e-12, (i, x, o)
            assert np.linalg.norm(x - o) == pytest.approx(d, rel=1e-12, abs=1e-14)
            assert d == pytest.approx(abs(shape.value(x[None])[0]), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_closest_point_matches_brute_force(dim):
    """Against the minimum distance to a dense cloud of surface points: the
    analytic distance may not exceed it (beyond the cloud's thickness) and
    must come within the cloud's spacing of it."""
    for i, shape in enumerate(SHAPES_2D if dim == 2 else SHAPES_3D):
        cloud = _surface_cloud(shape, dim, 10 + i)
        assert cloud.shape[0] > 3000
        for x in _domain_points(shape, dim, 12, 100 + i):
            d, o = O.sdf_closest(dim, shape, x)
            bf = float(np.min(np.linalg.norm(cloud - x, axis=1)))
            assert d <= bf + 2e-3 and bf <= d + (2e-2 if dim == 3 else 6e-3), (i, x, d, bf)


def test_scene_closest_point_mixes_mesh_and_shapes():
    spec = I.sdf_rocks_scene_2d()
    R = O.Scene(spec)
    mesh_only = O.Scene(dataclasses.replace(spec, sdf=[], bc=np.zeros_like(spec.bc)))
    pts = I.sdf_scene_points(spec, 64, 3, obstacle=((-0.25, 0.3), 0.18))
    seen = set()
    for x in pts:
        d, xb, prim = R.closest_dirichlet(x)
        cand = [(O.sdf_closest(2, f, x)[0], spec.n_prims + i) for i, f in enumerate(spec.sdf)]
        assert d == pytest.approx(min(c[0] for c in cand), rel=1e-12)
        assert prim == min(cand)[1]
        seen.add(prim)
        # the Neumann obstacle is not Dirichlet: flagged Dirichlet it competes
        dm, _, pm = mesh_only.closest_dirichlet(x)
        assert pm < spec.n_prims
    assert len(seen) == len(spec.sdf)
    # the scene box covers the shapes: the enclosing unit disk sets L
    assert R.L == pytest.approx(np.sqrt(2.0))


def _check(spec, pts, walks, eps, seed=2, allow=0):
    r = O.Scene(spec).solve(pts, walks, eps, seed=seed, nthreads=8)
    u = spec.exact(pts)
    se = np.sqrt(r["var"] / walks)
    bad = np.abs(r["mean"] - u) > 4 * se + eps * 4.0
    assert int(bad.sum()) <= allow, (np.nonzero(bad)[0], r["mean"][bad], u[bad])
    assert r["capped"] == 0 and r["escaped"] == 0
    return r


def test_rocks_2d_closed_form():
    spec = I.sdf_rocks_scene_2d()
    _check(spec, I.sdf_scene_points(spec, 40, 5, obstacle=((-0.25, 0.3), 0.18)), 600, 1e-3)


def test_shapes_only_2d_closed_form():
    """No mesh at all: walk on spheres inside analytic shapes."""
    spec = I.sdf_rocks_scene_2d(with_mesh=False)
    assert spec.n_prims == 0
    _check(spec, I.sdf_scene_points(spec, 40, 6), 600, 1e-3)


def test_inside_box_enclosure_2d():
    spec = I.sdf_rocks_scene_2d()
    spec = dataclasses.replace(spec, sdf=[I.Sdf(I.SDF_BOX, 1, (0.0, 0.0, 0, 0.95, 0.9, 0, 0.0))] + spec.sdf[1:])
    _check(spec, I.sdf_scene_points(spec, 32, 7, obstacle=((-0.25, 0.3), 0.18)), 600, 1e-3)


def test_rocks_3d_closed_form():
    spec = I.sdf_rocks_scene_3d(level=2)
    _check(spec, I.sdf_scene_points(spec, 16, 8, obstacle=((-0.2, 0.3, 0.2), 0.25)), 256, 1e-3)


def test_double_sided_sheet_inside_an_analytic_disk():
    """Both extensions together: a double-sided sheet (no mesh boundary at
    all) inside an analytic Dirichlet disk."""
    spec = I.crack_in_ball_scene_2d()
    assert spec.n_prims == 64 and set(np.unique(spec.bc)) == {I.DIRICHLET2, I.NEUMANN2}
    _check(spec, I.sdf_scene_points(spec, 32, 9), 600, 1e-3)
