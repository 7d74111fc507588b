"""Pins of the ball Green's function and its normaliser (App. A.1).

The Green's function is pinned by properties the paper states independently
of its formula: it vanishes on the sphere (zero-Dirichlet ball), its outward
radial derivative there is minus the printed Poisson kernel of the sphere
(1/(2 pi R) in 2D, 1/(4 pi R^2) in 3D), and its integral over the ball,
computed here by quadrature, equals the printed normaliser R^2/4, R^2/6.
"""
import math

import pytest
from scipy import integrate

import oracle as O


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("R", [0.05, 0.7, 3.0])
def test_green_ball_integral(dim, R):
    shell = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    val, _ = integrate.quad(lambda r: O.green_ball(dim, r, R) * shell(r), 0, R, limit=200)
    assert val == pytest.approx(O.green_ball_norm(dim, R), rel=1e-6)
    assert O.green_ball_norm(dim, R) == pytest.approx(R * R / (4 if dim == 2 else 6), rel=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_green_ball_boundary(dim):
    R = 0.8
    assert abs(O.green_ball(dim, R, R)) < 1e-15
    h = 1e-6
    dG = (O.green_ball(dim, R, R) - O.green_ball(dim, R - h, R)) / h
    P = 1 / (2 * math.pi * R) if dim == 2 else 1 / (4 * math.pi * R * R)
    assert -dG == pytest.approx(P, rel=1e-5)
    assert O.green_ball(dim, 0.3, R) > 0
