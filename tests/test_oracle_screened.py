"""Screened Poisson equation Laplacian(u) - sigma u = f (Sec. 3.2; ball
kernels of App. A.2) and the Tikhonov switch for pure-Neumann problems
(Sec. 3.4): pins of the oracle's Bessel functions, screened ball kernels and
walks (reading R10 of the oracle)."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from paper_2302_11815_amd import inputs as I
from test_oracle_walks import z_ok


@pytest.mark.parametrize("n", [0, 1])
def test_bessel_functions_match_scipy(n):
    for x in (1e-4, 0.03, 0.7, 2.0, 3.75, 9.0, 40.0, 300.0):
        assert O.bessel_ie(n, x) == pytest.approx(sp.ive(n, x), rel=1e-12)
        assert O.bessel_ke(n, x) == pytest.approx(sp.kve(n, x), rel=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("sigma", [0.3, 4.0, 90.0])
def test_q_on_the_sphere_is_one_minus_sigma_norm(dim, sigma):
    """u = 1 solves Laplacian(u) - sigma u = -sigma, so the screened ball
    kernel on the sphere integrates to 1 - sigma |G^{sigma,B}|; the free-space
    kernel integrates to 1 over the sphere, hence Q(R, R) = 1 - sigma |G|."""
    for R in (0.05, 0.6, 2.0):
        assert O.screened_q(dim, sigma, R, R) == pytest.approx(
            1.0 - sigma * O.green_ball_norm_screened(dim, sigma, R), rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_q_is_the_ratio_of_radial_derivatives(dim):
    """Q(r, R) = dG^{sigma,B}/drho / dG^{R^N}/drho at rho = r (the screened
    ball Poisson kernel over the free-space one), by central differences."""
    sigma, R = 2.5, 0.9
    for r in (0.1, 0.35, 0.7, 0.88):
        h = 1e-5 * r
        dg = (O.green_ball_screened(dim, sigma, r + h, R) - O.green_ball_screened(dim, sigma, r - h, R)) / (2 * h)
        dfree = -1.0 / (2 * math.pi * r) if dim == 2 else -1.0 / (4 * math.pi * r * r)
        assert O.screened_q(dim, sigma, r, R) == pytest.approx(dg / dfree, rel=1e-6)


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_green_function_norm_vanishing_and_limit(dim):
    sigma, R = 3.0, 0.8
    # vanishes on the sphere
    assert abs(O.green_ball_screened(dim, sigma, R, R)) < 1e-12
    # integral over the ball (radial midpoint quadrature)
    m = 200000
    rho = (np.arange(m) + 0.5) * R / m
    w = 2 * math.pi * rho if dim == 2 else 4 * math.pi * rho ** 2
    g = np.array([O.green_ball_screened(dim, sigma, x, R) for x in rho[::100]])
    integ = np.sum(np.interp(rho, rho[::100], g) * w) * R / m
    assert integ == pytest.approx(O.green_ball_norm_screened(dim, sigma, R), rel=2e-3)
    # sigma -> 0 recovers the Poisson kernels
    s0 = 1e-9
    assert O.green_ball_screened(dim, s0, 0.3, R) == pytest.approx(O.green_ball(dim, 0.3, R), rel=1e-6)
    assert O.green_ball_norm_screened(dim, s0, R) == pytest.approx(O.green_ball_norm(dim, R), rel=1e-6)
    assert O.screened_q(dim, s0, 0.3, R) == pytest.approx(1.0, abs=1e-8)
    assert O.screened_q(dim, 0.0, 0.3, R) == 1.0


def _exp_scene(base, a):
    """u = exp(a . x) solves Laplacian(u) - |a|^2 u = 0."""
    return I.with_data(base, I.FN_EXPLIN, (1.0,) + tuple(a))


def test_screened_star_polygon_exp():
    a = (0.8, -0.6)
    spec = _exp_scene(I.star_polygon_scene(512, 0), a)
    pts = I.star_polygon_points(24, seed=2, n_seg=512, vertices=spec.vertices)
    r = O.Scene(spec).solve(pts, 1500, 1e-4, seed=3, sigma=1.0)
    z_ok(r["mean"], r["var"], spec.exact(pts), 1500, "screened star polygon")
    assert r["capped"] == 0 and r["escaped"] == 0


def test_screened_icosphere_exp():
    mesh = I.displaced_icosphere(2, 0)
    a = (0.5, 0.5, -0.7)
    spec = _exp_scene(I.displaced_icosphere_scene(2, 0, mesh=mesh), a)
    pts = I.radial_mesh_points(mesh, 24, 1)
    r = O.Scene(spec).solve(pts, 600, 1e-3, seed=5, sigma=float(np.dot(a, a)))
    z_ok(r["mean"], r["var"], spec.exact(pts), 600, "screened icosphere")


def test_screened_source_term():
    """u = x^2 + y^2: Laplacian(u) = 4, so f = 4 - sigma (x^2 + y^2) (a
    quadratic source) on the mixed star polygon."""
    sigma = 2.0
    base = I.star_polygon_scene(512, 0)
    g, h, _, u = I.solution_data(I.FN_POLY2, (0, 0, 0, 1, 1, 0))
    f = I.Fn(I.FN_POLY2, 0, (4.0, 0, 0, -sigma, -sigma, 0))
    spec = I.dataclasses.replace(base, g=g, h=h, f=f, exact=u)
    pts = I.star_polygon_points(24, seed=5, n_seg=512, vertices=spec.vertices)
    r = O.Scene(spec).solve(pts, 1500, 1e-4, seed=9, sigma=sigma)
    z_ok(r["mean"], r["var"], spec.exact(pts), 1500, "screened source")


@pytest.mark.parametrize("dim", [2, 3])
def test_screened_pure_neumann(dim):
    """No Dirichlet boundary: the screened problem is still well posed; walks
    end by Russian roulette; the star radius is capped at the escape radius."""
    if dim == 2:
        a = (0.9, 0.4)
        base = I.star_polygon_scene(512, 0)
        pts = I.star_polygon_points(16, seed=4, n_seg=512, vertices=base.vertices)
        W, eps = 1500, 1e-4
    else:
        a = (0.6, -0.3, 0.5)
        mesh = I.displaced_icosphere(2, 0)
        base = I.displaced_icosphere_scene(2, 0, mesh=mesh)
        pts = I.radial_mesh_points(mesh, 16, 3)
        W, eps = 600, 1e-3
    spec = I.with_data(base, I.FN_EXPLIN, (1.0,) + a, bc=np.full(base.n_prims, I.NEUMANN))
    r = O.Scene(spec).solve(pts, W, eps, seed=2, sigma=float(np.dot(a, a)))
    z_ok(r["mean"], r["var"], spec.exact(pts), W, f"pure Neumann {dim}D")
    assert r["capped"] == 0 and r["escaped"] == 0


def test_roulette_ends_walks_and_records_q():
    a = (0.8, -0.6)
    spec = I.with_data(I.star_polygon_scene(256, 0), I.FN_EXPLIN, (1.0,) + a,
                       bc=np.full(256, I.NEUMANN))
    S = O.Scene(spec)
    P = S.params(1e-4, 1, sigma=1.0)
    pts = I.star_polygon_points(6, seed=1, n_seg=256, vertices=spec.vertices)
    for i in range(6):
        v, ns, how, recs = S.walk(P, pts[i], i, 0, max_rec=4096)
        assert how == 4 and recs[-1].roulette == 1
        assert all(0.0 < rc.q < 1.0 for rc in recs[:ns])


def test_tikhonov_switch():
    """Pure-Neumann Poisson (harmonic u, compatible flux): the solution is
    fixed only up to a constant.  With the switch at step 0 the walk is the
    screened walk with sigma_T, bit for bit; with a late switch the estimate
    reproduces u up to a constant (differences between points) within a
    small regularisation bias."""
    base = I.star_polygon_scene(512, 0)
    spec = I.dataclasses.replace(base, bc=np.full(512, I.NEUMANN, np.uint8))
    S = O.Scene(spec)
    pts = I.star_polygon_points(8, seed=6, n_seg=512, vertices=spec.vertices)
    a = S.solve(pts, 64, 1e-4, seed=4, tik_sigma=0.5, tik_steps=0)
    b = S.solve(pts, 64, 1e-4, seed=4, sigma=0.5)
    assert np.array_equal(a["mean"], b["mean"])
    W = 1500
    r = S.solve(pts, W, 1e-4, seed=5, tik_sigma=0.2, tik_steps=10)
    u = spec.exact(pts)
    d = (r["mean"] - u) - np.mean(r["mean"] - u)     # the constant removed
    se = np.sqrt(r["var"] / W)
    assert np.all(np.abs(d) < 5 * se + 0.05), (d, se)
    assert r["capped"] == 0
