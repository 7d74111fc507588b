"""Pins of the oracle's decision margins: how far a reported silhouette
distance or ray crossing lies from the thresholds that decide it.  The
parity tests use them to accept a GPU/oracle difference in a discrete
outcome only at a near-tie; values here are worked out by hand on the
L-shape, the unit square and the unit cube."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I

TOL = 1e-9


def test_silhouette_margin_l_shape_2d():
    # reflex vertex (1, 1) between the segments (2,1)-(1,1) (outward normal
    # +y) and (1,1)-(1,2) (outward normal +x); from x = (0.4, 1.3) it is the
    # closest vertex, v = (0.6, -0.3), so the factors are -0.3 and 0.6
    S = O.Scene(I.l_shape_2d())
    x = np.array([0.4, 1.3])
    d = math.hypot(0.6, 0.3)
    assert S.silhouette(x, 10.0) == pytest.approx(d, abs=1e-12)
    assert S.silhouette_margin(x, 10.0, d, TOL) == pytest.approx(0.3, abs=1e-12)
    # the within-radius test is nearer its threshold with rmax = 0.7
    assert S.silhouette_margin(x, 0.7, d, TOL) == pytest.approx(0.7 - d, abs=1e-12)
    # no element at that distance: no decision
    assert math.isinf(S.silhouette_margin(x, 10.0, 0.5, TOL))
    # in line with the segment (2,1)-(1,1): one factor vanishes
    x2 = np.array([0.5, 1.0])
    assert S.silhouette_margin(x2, 10.0, 0.5, TOL) == pytest.approx(0.0, abs=1e-12)


def test_silhouette_margin_l_prism_3d():
    V, F = I.l_prism_mesh(1.0)
    S = O.Scene(I.mesh_scene(V, F, np.ones(len(F), np.uint8)))
    x = np.array([0.4, 1.3, 0.5])
    d = math.hypot(0.6, 0.3)      # to the reflex edge x = y = 1
    assert S.silhouette(x, 10.0) == pytest.approx(d, abs=1e-12)
    assert S.silhouette_margin(x, 10.0, d, TOL) == pytest.approx(0.3, abs=1e-12)


def test_ray_margin_unit_square():
    S = O.Scene(I.unit_square_scene())   # Neumann on y = 0 and y = 1
    o, v = np.array([0.3, 0.5]), np.array([0.0, -1.0])
    p, t = S.ray_neumann(o, v, 2.0)
    assert p == 0 and t == pytest.approx(0.5)
    # crossing at (0.3, 0): 0.3 from the end point (0, 0)
    assert S.ray_margin(o, v, 2.0, t, TOL) == pytest.approx(0.3, abs=1e-12)
    # clipped exactly at the crossing: the t <= tmax test is a tie
    assert S.ray_margin(o, v, 0.5, 0.5, TOL) == pytest.approx(0.0, abs=1e-12)
    # aimed at the corner (1, 0): the crossing is on the rim
    o2, v2 = np.array([0.5, 0.5]), np.array([1.0, -1.0]) / math.sqrt(2.0)
    assert S.ray_margin(o2, v2, 2.0, math.sqrt(0.5), TOL) == pytest.approx(0.0, abs=1e-12)
    # |v| scales the parameter: t is in units of |v|
    assert S.ray_margin(o, 2 * v, 2.0, 0.25, TOL) == pytest.approx(0.3, abs=1e-12)
    # a skipped primitive takes no part
    assert S.ray_margin(o, v, 2.0, 0.5, TOL, skip0=p) == pytest.approx(0.5, abs=1e-12)


def test_ray_margin_cube_face_diagonal():
    V, F = I.cube_mesh()
    S = O.Scene(I.mesh_scene(V, F, np.r_[0, 0, np.ones(10)]))
    # the top face z = 1 is split along x = y; a crossing at (0.5, 0.25, 1)
    # lies 0.25 from the edge y = 0 and 0.25 / sqrt(2) from the diagonal
    o, v = np.array([0.5, 0.25, 0.5]), np.array([0.0, 0.0, 1.0])
    p, t = S.ray_neumann(o, v, 2.0)
    assert p >= 0 and t == pytest.approx(0.5)
    assert S.ray_margin(o, v, 2.0, t, TOL) == pytest.approx(0.25 / math.sqrt(2.0), abs=1e-12)
    # on the diagonal itself
    o2 = np.array([0.5, 0.5, 0.5])
    assert S.ray_margin(o2, v, 2.0, 0.5, TOL) == pytest.approx(0.0, abs=1e-12)
