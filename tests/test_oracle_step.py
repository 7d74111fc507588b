"""One-step identities of the WoSt estimator (Sec. 4.3 boxed estimator,
Sec. 4.7): for an exact solution u, one step satisfies
E[u(x_{k+1}) + N - S] = u(x_k), at interior points and at points on a flat
Neumann face (hemisphere sampling, alpha = 1/2, Sec. 4.4.4).  A sign slip in
the Neumann or source term, a missing 1/alpha, or a wrong kernel normaliser
shifts the mean by O(r) and fails these tests."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I


def _half_space_box_3d(a, coef, lap=0.0, half=10.0, depth=1.0):
    """Box [-half, half]^2 x [-depth, a]; the top face z = a is Neumann, the
    rest Dirichlet; data from the exact u given by POLY2 coefficients."""
    V, F = I.cube_mesh((-half, -half, -depth), (half, half, a))
    bc = np.zeros(12, np.uint8)
    bc[2:4] = I.NEUMANN                      # faces on z = hi
    g, h, f, u = I.solution_data(I.FN_POLY2, coef, laplacian_const=lap)
    return I.mesh_scene(V, F, bc, g=g, h=h, f=f, exact=u)


def _half_plane_box_2d(a, coef, lap=0.0, half=10.0, depth=1.0, n_top=5):
    top = [[half - 2 * half * i / n_top, a] for i in range(n_top + 1)]
    V = [[-half, -depth], [half, -depth]] + top
    nseg = len(V)
    bc = np.zeros(nseg, np.uint8)
    bc[2:2 + n_top] = I.NEUMANN              # segments along y = a
    g, h, f, u = I.solution_data(I.FN_POLY2, coef, laplacian_const=lap)
    return I.polygon_scene(V, bc, g=g, h=h, f=f, exact=u)


def _one_step_mean(spec, x, n_samples, onN=False, normal=None, cur=-1, rmin=1e-3):
    S = O.Scene(spec)
    P = S.params(eps=1e-3, seed=11, rmin=rmin)
    vals = np.empty(n_samples)
    for w in range(n_samples):
        c, rec, nxt = S.step(P, 0, w, 0, x, n=normal, onN=onN, cur=cur)
        assert rec.term == 0
        vals[w] = spec.exact(np.array(nxt.x)[: spec.dim]) + c
    return vals.mean(), vals.std() / math.sqrt(n_samples), rec


U3_LIN = (0.0, 0.0, 0.0, 1.0)                                    # u = z
U3_MIX = (0.0, 0.0, 0.0, 0.0, 1 / 6, 1 / 6, 1 / 6, 1.0, 0.0, 0.0)  # |x|^2/6 + xy
U2_LIN = (0.0, 0.0, 1.0)                                         # u = y
U2_MIX = (0.0, 0.3, 0.0, 0.25, 0.25, 0.7)                        # |x|^2/4 + 0.3x + 0.7xy


@pytest.mark.parametrize("coef,lap", [(U3_LIN, 0.0), (U3_MIX, 1.0)])
def test_one_step_interior_3d(coef, lap):
    spec = _half_space_box_3d(0.5, coef, lap)
    x = np.array([0.0, 0.0, 0.0])
    m, se, rec = _one_step_mean(spec, x, 20000)
    assert rec.r == pytest.approx(1.0)
    assert abs(m - spec.exact(x)) < 4 * se


@pytest.mark.parametrize("coef,lap", [(U3_LIN, 0.0), (U3_MIX, 1.0)])
def test_one_step_on_neumann_3d(coef, lap):
    a = 0.5
    spec = _half_space_box_3d(a, coef, lap)
    x = np.array([0.3, -0.2, a])
    # which top triangle holds x (faces 2, 3 of the cube mesh)
    S = O.Scene(spec)
    cur = 2 if S.ray_neumann([0.3, -0.2, 0.0], [0, 0, 1], 1.0, 3)[0] == 2 else 3
    m, se, rec = _one_step_mean(spec, x, 20000, onN=True, normal=[0, 0, 1], cur=cur)
    assert rec.r == pytest.approx(1.5, rel=1e-4)
    assert abs(m - spec.exact(x)) < 4 * se


@pytest.mark.parametrize("coef,lap", [(U2_LIN, 0.0), (U2_MIX, 1.0)])
def test_one_step_interior_2d(coef, lap):
    spec = _half_plane_box_2d(0.5, coef, lap)
    x = np.array([0.1, 0.0])
    m, se, rec = _one_step_mean(spec, x, 20000)
    assert rec.r == pytest.approx(1.0)
    assert abs(m - spec.exact(x)) < 4 * se


@pytest.mark.parametrize("coef,lap", [(U2_LIN, 0.0), (U2_MIX, 1.0)])
def test_one_step_on_neumann_2d(coef, lap):
    a = 0.5
    spec = _half_plane_box_2d(a, coef, lap)
    x = np.array([0.7, a])
    S = O.Scene(spec)
    cur = S.ray_neumann([0.7, 0.0], [0, 1], 1.0)[0]
    m, se, rec = _one_step_mean(spec, x, 20000, onN=True, normal=[0, 1], cur=cur)
    assert rec.r == pytest.approx(1.5, rel=1e-4)
    assert abs(m - spec.exact(x)) < 4 * se


def test_one_step_poisson_ball_3d():
    """Pure Dirichlet (WoS, Sec. 3.4.2) with u = |x|^2/6, f = 1: the source
    term alone carries E[u(x1)] - u(x0) = r^2/6."""
    V, F = I.cube_mesh((-1, -1, -1), (1, 1, 1))
    g, h, f, u = I.solution_data(I.FN_POLY2, (0, 0, 0, 0, 1 / 6, 1 / 6, 1 / 6), laplacian_const=1.0)
    spec = I.mesh_scene(V, F, np.zeros(12), g=g, h=h, f=f, exact=u)
    x = np.array([0.1, -0.2, 0.15])
    m, se, rec = _one_step_mean(spec, x, 20000)
    assert rec.r == pytest.approx(0.8) and rec.Nhat == 0.0
    assert abs(m - spec.exact(x)) < 4 * se
