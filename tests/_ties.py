"""Near-tie classification for the GPU parity tests (not a test module).

A GPU walk step and the oracle's re-run of it from the GPU's state may
differ in a discrete outcome -- a silhouette accepted or not, a ray crossing
found or not, the hemisphere flip, the source sample inside the star or
not, the eps-shell test -- only where the oracle's deciding quantity lies
within the per-step tolerance of its threshold.  `step_mismatch` names the
first differing quantity in the step's order of computation and returns
whether the oracle's decision there is such a near-tie; a difference in a
continuous quantity (a distance, the radius, the next point along an
agreed ray) is never one."""
import math

import numpy as np


def query_origin(P, x, n, on_neumann):
    """x' = x - offset n on the Neumann boundary (the oracle's reading R4)."""
    return x - (P.offset if on_neumann else 0.0) * n


def step_mismatch(R, P, dim, g, o, tol, hit_prim=False):
    """Compares GPU record g with oracle record o of the same step (oracle
    run from g's state).  Returns None when they agree, else (kind, tie,
    margin): tie is True when the oracle's deciding value is within the
    tolerance of its threshold (tol in length units; 1e-5 for the
    dimensionless hemisphere test)."""
    x = np.array(g.x[:dim], np.float64)
    n = np.array(g.n[:dim], np.float64)
    xq = query_origin(P, x, n, bool(g.on_neumann))
    same_dsil = abs(g.d_silhouette - o.dsil) <= tol or (g.d_silhouette > 1e37 and o.dsil > 1e37)
    if not same_dsil:
        m = R.silhouette_margin(xq, o.dD, min(g.d_silhouette, o.dsil), tol)
        return "silhouette", m <= tol, m
    if abs(g.r - o.r) > tol:
        return "radius", False, math.inf
    if not np.allclose(g.v[:dim], o.v[:dim], atol=1e-5):
        m = abs(float(np.dot(n, np.asarray(o.v[:dim])))) if g.on_neumann else math.inf
        return "hemisphere", m <= 1e-5, m
    if g.hit != o.hit or abs(g.t - o.t) > tol or (hit_prim and g.hit_prim != o.hit_prim):
        m = R.ray_margin(xq, np.asarray(o.v[:dim]), o.r, min(g.t, o.t), tol, skip0=g.cur)
        return "crossing", m <= tol, m
    if not np.allclose(g.p[:dim], o.p[:dim], atol=tol):
        return "next point", False, math.inf
    if abs(g.s_frac - o.s_frac) > 1e-5:
        return "source fraction", False, math.inf
    if abs(g.s_hat - o.Shat) > 1e-4 * abs(o.Shat) + 1e-7:
        m = abs(o.r * o.s_frac - o.t)
        return "source inclusion", m <= tol, m
    if abs(g.q - o.q) > 1e-4 * abs(o.q) + 1e-7:
        return "continuation factor", False, math.inf
    return None


def assert_tie(where, res):
    """Fails unless the mismatch `res` of step_mismatch is a near-tie."""
    kind, tie, margin = res
    assert tie, f"{where}: {kind} differs with the oracle's decision {margin:.3g} from its threshold"
