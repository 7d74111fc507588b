"""Parity of the HIP path with the FP64 oracle, called through the C-ABI.

Per-step geometric results (Q.1-Q.3, radius, direction, next point, source
term) must agree within 1e-5 L (L = scene half-diagonal); a discrete
outcome (hit or miss, silhouette or not, eps-termination) may differ only
where the oracle's deciding quantity lies within 1e-5 L of its threshold,
and such near-ties are counted.  The Neumann sample uses different (both
unbiased) samplers on the two sides (Algorithm 6 on the GPU, a plain
measure-proportional pick in the oracle), so it is compared in
distribution.  Per-point estimates are compared statistically: count of
|z| > 4 within the Gaussian tail allowance."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I
from _ties import assert_tie, step_mismatch

pytestmark = pytest.mark.gpu

W = pytest.importorskip("paper_2302_11815_amd.wost")
Z_TAIL = 6.33e-5


def count_bad(z):
    return int(np.sum(np.abs(z) > 4)), 2 * z.size * Z_TAIL + 3


def _star(n_seg=2048, seed=0):
    return I.star_polygon_scene(n_seg, seed)


def _ico(level=3, seed=0):
    mesh = I.displaced_icosphere(level, seed)
    return I.displaced_icosphere_scene(level, seed, mesh=mesh), mesh


# ---------------------------------------------------------------------------
# probes
# ---------------------------------------------------------------------------

def _probe_points(spec, n, rng):
    V = spec.vertices.astype(np.float64)
    lo, hi = V.min(0), V.max(0)
    pad = 0.1 * (hi - lo)
    return rng.uniform(lo - pad, hi + pad, (n, spec.dim)).astype(np.float32)


@pytest.mark.parametrize("which", ["star", "ico", "square"])
def test_probe_closest_point(which):
    spec = {"star": lambda: _star(), "ico": lambda: _ico()[0], "square": I.unit_square_scene}[which]()
    S, R = W.Scene(spec), O.Scene(spec)
    tol = 1e-5 * R.L
    x = _probe_points(spec, 3000, np.random.default_rng(1))
    d, xb, pr = W.wost_probe_closest_point(S.handle, x, spec.dim)
    for i in range(x.shape[0]):
        dd, xbo, po = R.closest_dirichlet(x[i])
        assert abs(d[i] - dd) <= tol
        assert np.linalg.norm(xb[i] - xbo) <= 10 * tol or po != pr[i]
        if po != pr[i]:  # a tie: the GPU's primitive must be as close
            d2, _, _ = O.Scene(I.Scene("one", spec.dim, spec.vertices, spec.prims[[pr[i]]], np.zeros(1, np.uint8),
                                       I.Fn(), I.Fn(), I.Fn())).closest_dirichlet(x[i])
            assert abs(d2 - dd) <= tol


@pytest.mark.parametrize("which", ["star", "ico", "lshape2", "lprism"])
def test_probe_silhouette(which):
    if which == "lshape2":
        spec = I.l_shape_2d(bc=[0, 1, 1, 1, 1, 1])
    elif which == "lprism":
        V, F = I.l_prism_mesh(1.0)
        bc = np.ones(len(F), np.uint8)
        bc[0] = 0
        spec = I.mesh_scene(V, F, bc)
    elif which == "star":
        spec = _star()
    else:
        spec = _ico()[0]
    S, R = W.Scene(spec), O.Scene(spec)
    tol = 1e-5 * R.L
    x = _probe_points(spec, 2000, np.random.default_rng(2))
    rmax = np.array([R.closest_dirichlet(p)[0] for p in x], np.float32)
    d = W.wost_probe_silhouette(S.handle, x, rmax, spec.dim)
    ties = 0
    for i in range(x.shape[0]):
        do = R.silhouette(x[i], float(rmax[i]))
        if abs(d[i] - do) > tol:
            # allowed only where a silhouette decision of the oracle (an
            # element's predicate factor v . n, or its distance against
            # rmax) lies within the tolerance of its threshold
            m = R.silhouette_margin(x[i], float(rmax[i]), min(float(d[i]), do), tol)
            assert m <= tol, (i, x[i], d[i], do, m)
            ties += 1
    assert ties <= 1e-3 * x.shape[0], f"{ties} near-tie silhouette differences"


@pytest.mark.parametrize("which", ["star", "ico", "cube"])
def test_probe_ray(which):
    if which == "cube":
        V, F = I.cube_mesh()
        spec = I.mesh_scene(V, F, np.r_[0, 0, np.ones(10)])
    else:
        spec = _star() if which == "star" else _ico()[0]
    S, R = W.Scene(spec), O.Scene(spec)
    tol = 1e-5 * R.L
    rng = np.random.default_rng(3)
    o = _probe_points(spec, 3000, rng)
    v = rng.normal(size=o.shape)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v = v.astype(np.float32)
    tmax = rng.uniform(0.05, 2.0, o.shape[0]).astype(np.float32) * R.L
    t, pr = W.wost_probe_ray(S.handle, o, v, tmax, -1, spec.dim)
    ties = 0
    for i in range(o.shape[0]):
        po, to = R.ray_neumann(o[i], v[i], float(tmax[i]), behind=0.25 * O.OFFSET_REL * R.L)
        if (po >= 0) != (pr[i] >= 0) or abs(t[i] - to) > tol:
            # allowed only at a crossing within the tolerance of a
            # primitive's rim, of the clip tmax, or of the origin
            m = R.ray_margin(o[i], v[i], float(tmax[i]), min(float(t[i]), to), tol)
            assert m <= tol, (i, t[i], to, pr[i], po, m)
            ties += 1
    assert ties <= 1e-3 * o.shape[0], f"{ties} near-tie crossing differences"


def test_probe_ray_watertight_cube_corners():
    """Rays aimed exactly at shared vertices and edges of a closed mesh hit."""
    V, F = I.cube_mesh()
    spec = I.mesh_scene(V, F, np.r_[0, 0, np.ones(10)])
    S = W.Scene(spec)
    o = np.tile(np.array([0.5, 0.5, 0.5], np.float32), (6, 1))
    tg = np.array([[1, 1, 1], [0, 1, 1], [1, 0.5, 1], [0.5, 1, 1], [1, 1, 0.3], [0, 0.5, 0.5]], np.float32)
    v = tg - o
    t, pr = W.wost_probe_ray(S.handle, o, v, 10.0, -1, 3)
    assert np.all(pr >= 0)
    assert np.allclose(t, 1.0, atol=1e-6)


def test_probe_ray_grazing_from_just_outside():
    """Reading R13 across the plane: from one or two FP32 ulps above the
    cube's top face (well within offset/4 of its plane), a ray leaving it at
    a grazing angle crosses it far back along the ray and lands at t = 0 on
    it, as in the oracle, while that crossing lies within 64 offsets; from
    2^-17 above (beyond offset/4), or farther back, it does not."""
    V, F = I.cube_mesh()
    spec = I.mesh_scene(V, F, np.r_[0, 0, np.ones(10)])
    S, R = W.Scene(spec), O.Scene(spec)
    offset = O.OFFSET_REL * R.L
    behind, reach = 0.25 * offset, 64.0 * offset
    o, v, want = [], [], []
    for c in (0.0005, 0.002, 0.008, 0.05, 0.3):
        for dz in (2.0 ** -23, 2.0 ** -22, 2.0 ** -17):
            # no case within 10 % of either bound
            assert abs(dz / behind - 1) > 0.1 and abs(dz / c / reach - 1) > 0.1
            o.append([0.5, 0.25, 1.0 + dz])
            v.append([math.sqrt(1 - c * c), 0.0, c])
            want.append(dz < behind and dz / c < reach)
    assert 0 < sum(want) < len(want)
    o = np.array(o, np.float32)
    v = np.array(v, np.float32)
    t, pr = W.wost_probe_ray(S.handle, o, v, np.full(len(o), 5.0, np.float32), -1, 3)
    for i in range(len(o)):
        po, to = R.ray_neumann(o[i], v[i], 5.0, behind=behind)
        assert (po >= 0) == want[i] and (pr[i] >= 0) == want[i], (i, po, pr[i])
        if want[i]:
            assert po == pr[i] and to == 0.0 and t[i] == 0.0, (i, po, pr[i], to, t[i])


def test_walk_grazing_leak_regression():
    """A walk that once left a closed domain (64-mesh batch, mesh 61, point
    53167, walk 417): a step ended by a miss within rounding of a Neumann
    triangle, FP32 put the point 4e-8 outside it, and the next ray left it at
    a grazing angle.  With reading R13 measured across the plane the walk
    lands back on that triangle and ends in the eps-shell; no interior
    position lies outside the mesh by more than rounding (offset / 4, the
    bound under which the next step's ray query brings it back)."""
    c = I.geodesic_batch_case(only={61})[0]
    spec = c["scene"]
    freq = int(spec.name.split("_f")[1].split("_")[0])
    S = W.Scene(spec)
    pid, wid = 53167, 417
    recs, ns, vals = W.wost_trace_walks(S.handle, c["points"][pid:pid + 1], [pid], [wid], c["eps"], c["seed"],
                                        20000)
    k = int(ns[0])
    assert 0 < k < 20000
    assert recs[k - 1].term == 1, [recs[k - 1].term]
    assert all(recs[i].term == 0 for i in range(k - 1))
    x = np.array([list(recs[i].x) for i in range(k)], np.float64)
    interior = np.array([recs[i].on_neumann == 0 for i in range(k)])
    assert k > 120 and recs[115].hit == 0 and recs[116].hit == 1, "the walk no longer takes the path it leaked on"
    out = I.geodesic_outside_distance(spec.vertices, spec.prims, x[interior], freq)
    R = O.Scene(spec)
    assert out.max() < 0.25 * O.OFFSET_REL * R.L, out.max()


@pytest.mark.parametrize("dim", [2, 3])
def test_probe_neumann_sample_unbiased(dim):
    """E[1{|z - x| < r} / pdf] equals the Neumann measure inside B(x, r):
    a chord 2 sqrt(r^2 - d^2) in 2D, a disk pi (r^2 - d^2) in 3D."""
    if dim == 2:
        n = 512
        xs = np.linspace(-4, 4, n + 1)
        V = np.stack([xs, np.zeros_like(xs)], 1)
        P = np.stack([np.arange(n), np.arange(1, n + 1)], 1)
        Vd = np.vstack([V, [[4, -3], [-4, -3]]])
        Pd = np.vstack([P, [[n, n + 1], [n + 1, n + 2]]])
        spec = I.Scene("line", 2, Vd.astype(np.float32), Pd.astype(np.int32),
                       np.r_[np.ones(n), 0, 0].astype(np.uint8), I.Fn(), I.Fn(), I.Fn())
        x, r, exact = np.array([0.123, 0.3]), 1.0, 2 * math.sqrt(1 - 0.09)
    else:
        n = 64
        xs = np.linspace(-2, 2, n + 1)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        Vg = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
        idx = lambda i, j: i * (n + 1) + j
        F = []
        for i in range(n):
            for j in range(n):
                F.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)])
                F.append([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)])
        m = Vg.shape[0]
        Vd = np.vstack([Vg, [[0, 0, -3], [1, 0, -3], [0, 1, -3]]])
        F.append([m, m + 2, m + 1])
        spec = I.mesh_scene(Vd, F, np.r_[np.ones(len(F) - 1), 0])
        x, r = np.array([0.1, -0.2, 0.35]), 0.9
        exact = math.pi * (r * r - x[2] ** 2)
    S = W.Scene(spec)
    N = 200000
    xx = np.tile(x.astype(np.float32), (N, 1))
    z, pdf, pr = W.wost_probe_neumann_sample(S.handle, xx, r, 17, dim)
    assert np.all(pr >= 0) and np.all(pdf > 0)
    inside = np.linalg.norm(z.astype(np.float64) - x, axis=1) < r
    est = inside / pdf.astype(np.float64)
    assert abs(est.mean() - exact) < 4 * est.std() / math.sqrt(N)


def _neumann_area_in_ball(V, F, x, r, k=64):
    """Area of the triangles F (vertices V) inside the ball B(x, r): each
    triangle split into k^2 equal sub-triangles, each counted by whether its
    centroid lies in the ball."""
    i, j = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    keep = i + j <= k - 1
    i, j = i[keep], j[keep]
    # up-pointing sub-triangles (i, j) and down-pointing ones (i, j) with
    # i + j <= k - 2, by their barycentric centroids
    up = np.stack([(i + 1 / 3) / k, (j + 1 / 3) / k], 1)
    dn_keep = i + j <= k - 2
    dn = np.stack([(i[dn_keep] + 2 / 3) / k, (j[dn_keep] + 2 / 3) / k], 1)
    bary = np.vstack([up, dn])                       # k^2 sub-triangle centroids
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    total = 0.0
    for t0 in range(0, F.shape[0], 256):
        a, b, c = A[t0:t0 + 256], B[t0:t0 + 256], C[t0:t0 + 256]
        pts = (a[:, None, :] + bary[None, :, :1] * (b - a)[:, None, :] + bary[None, :, 1:] * (c - a)[:, None, :])
        inside = np.linalg.norm(pts - x, axis=2) < r
        total += float(np.sum(area[t0:t0 + 256] * inside.mean(axis=1)))
    return total


@pytest.mark.parametrize("case", range(4))
def test_probe_neumann_sample_curved_mesh(case):
    """The Neumann sampler on a curved mesh (the displaced icosphere, level
    3, its lower part Neumann): E[1{|z - x| < r} / pdf] equals the Neumann
    area inside B(x, r), which this test integrates itself by subdividing
    every Neumann triangle; every sample lies on the triangle it reports.
    A descent may end without a sample (a node's box meets the ball but none
    of its children's boxes do, or no primitive of the leaf does): such a
    draw contributes 0, and every primitive that meets the ball can still
    be reached, so the mean stays the area."""
    mesh = I.displaced_icosphere(3, 2)
    spec = I.displaced_icosphere_scene(3, 2, mesh=mesh)
    V = spec.vertices.astype(np.float64)
    F = spec.prims.astype(np.int64)
    neu = np.nonzero(spec.bc == 1)[0]
    # a point inside near the Neumann part, and a ball of radius r about it
    dirs = np.array([[0.3, -0.2, -0.9], [-0.6, 0.5, -0.6], [0.8, 0.1, -0.55], [0.0, 0.0, -1.0]])
    d = dirs[case] / np.linalg.norm(dirs[case])
    x = 0.75 * d
    r = [0.35, 0.5, 0.6, 0.8][case]
    exact = _neumann_area_in_ball(V, F[neu], x, r)
    assert exact > 0.05
    S = W.Scene(spec)
    N = 200000
    xx = np.tile(x.astype(np.float32), (N, 1))
    z, pdf, pr = W.wost_probe_neumann_sample(S.handle, xx, r, 23 + case, 3)
    ok = pr >= 0
    assert ok.mean() > 0.02 and np.all(pdf[ok] > 0)
    q = pr[ok]
    assert np.all(spec.bc[q] == 1)
    # each sample on its triangle: in the plane, with barycentric
    # coordinates in [0, 1] up to FP32 rounding
    a, b, c = V[F[q, 0]], V[F[q, 1]], V[F[q, 2]]
    nrm = np.cross(b - a, c - a)
    nn = np.linalg.norm(nrm, axis=1)
    zz = z[ok].astype(np.float64)
    assert np.max(np.abs(np.einsum("ij,ij->i", zz - a, nrm)) / nn) < 1e-5
    wb = np.einsum("ij,ij->i", np.cross(zz - a, c - a), nrm) / nn ** 2
    wc = np.einsum("ij,ij->i", np.cross(b - a, zz - a), nrm) / nn ** 2
    assert wb.min() > -1e-4 and wc.min() > -1e-4 and (wb + wc).max() < 1 + 1e-4
    est = np.zeros(N)
    inside = np.linalg.norm(zz - x, axis=1) < r
    est[ok] = inside / pdf[ok].astype(np.float64)
    # the subdivision's own error is below 0.3 % of the area here
    assert abs(est.mean() - exact) < 4 * est.std() / math.sqrt(N) + 3e-3 * exact


def _seg_dist(x, A, B):
    E = B - A
    t = np.clip(((x - A) * E).sum(1) / (E * E).sum(1), 0.0, 1.0)
    return np.linalg.norm(x - (A + t[:, None] * E), axis=1)


def _prim_dist(spec, x, prims):
    """FP64 distance from x to each primitive (segment or triangle)."""
    V = spec.vertices.astype(np.float64)
    P = spec.prims[np.asarray(prims, np.int64)]
    A, B = V[P[:, 0]], V[P[:, 1]]
    if spec.dim == 2:
        return _seg_dist(x, A, B)
    C = V[P[:, 2]]
    n = np.cross(B - A, C - A)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    h = ((x - A) * n).sum(1)
    y = x - h[:, None] * n                     # projection on each plane
    ins = np.ones(len(A), bool)
    for p, q in ((A, B), (B, C), (C, A)):
        ins &= (np.cross(q - p, y - p) * n).sum(1) >= 0
    edge = np.minimum(np.minimum(_seg_dist(x, A, B), _seg_dist(x, B, C)), _seg_dist(x, C, A))
    return np.where(ins, np.abs(h), edge)


def _alg6_pdfs(nodes, slot_prim, slot_meas, spec, x, r, offset, tol):
    """FP64 re-computation of the Q.4 sampler from the device's own tree:
    one random descent picks, at every node, a child whose box meets
    B(x, r), with probability proportional to 1 / max(|box centre - x|,
    offset) (Algorithm 6); in the leaf, a primitive meeting the ball in
    proportion to its measure (Algorithm 5).  Returns {slot: pdf} for every
    primitive that can be drawn (pdf = P(leaf) / leaf measure in the ball),
    the total probability of reaching a leaf, and `near`: whether any box or
    primitive test made lies within tol of the radius (where FP32 may decide
    otherwise)."""
    dim = spec.dim
    w = 16 if dim == 3 else 12
    N = nodes.reshape(-1, w).astype(np.float64)
    codes = nodes.reshape(-1, w)[:, 4 * dim:4 * dim + 2].copy().view(np.int32)
    empty = np.iinfo(np.int32).min
    out, reach, near = {}, 0.0, False
    stack = [(0, 1.0)]
    while stack:
        i, p = stack.pop()
        wts = [0.0, 0.0]
        for j in range(2):
            if codes[i, j] == empty:
                continue
            lo = N[i, 2 * dim * j:2 * dim * j + dim]
            hi = N[i, 2 * dim * j + dim:2 * dim * (j + 1)]
            db = float(np.linalg.norm(np.maximum(0.0, np.maximum(lo - x, x - hi))))
            near |= abs(db - r) <= tol
            if db <= r:
                wts[j] = 1.0 / max(float(np.linalg.norm(0.5 * (lo + hi) - x)), offset)
        tot = wts[0] + wts[1]
        for j in range(2):
            if wts[j] == 0.0:
                continue
            pj = p * wts[j] / tot
            c = int(codes[i, j])
            if c >= 0:
                stack.append((c, pj))
                continue
            v = -c - 1
            ks = np.arange(v >> 3, (v >> 3) + (v & 7))
            d = _prim_dist(spec, x, slot_prim[ks])
            near |= bool(np.any(np.abs(d - r) <= tol))
            ks = ks[d <= r]
            m = float(np.sum(slot_meas[ks].astype(np.float64)))
            if m > 0:
                reach += pj
                for k in ks:
                    out[int(k)] = out.get(int(k), 0.0) + pj / m
    return out, reach, near


@pytest.mark.parametrize("which", ["star", "ico"])
def test_probe_neumann_pdf_from_device_tree(which):
    """Every Q.4 draw's pdf equals, within FP32 rounding, the pdf that the
    sampler's definition (Algorithms 5-6) gives in FP64 over the device's
    own binary Neumann tree (wost_get_neumann_tree), for balls of many sizes
    around points inside the domain; a draw that FP64 says cannot occur is
    allowed only where a box or primitive test is within 1e-5 L of the
    radius.  Also: the drawn primitive meets the ball, the probability of
    reaching some leaf is at most 1, and every Neumann primitive meeting the
    ball can be drawn."""
    if which == "star":
        spec = _star()
    else:
        spec = I.displaced_icosphere_scene(3, 2, mesh=I.displaced_icosphere(3, 2))
    dim = spec.dim
    S, R = W.Scene(spec), O.Scene(spec)
    tol = 1e-5 * R.L
    offset = O.OFFSET_REL * R.L
    nodes, slot_prim, slot_meas = W.wost_get_neumann_tree(S.handle, dim)
    assert nodes.shape[0] > 1 and sorted(slot_prim.tolist()) == sorted(np.nonzero(spec.bc == 1)[0].tolist())
    slot_of = {int(p): k for k, p in enumerate(slot_prim)}
    rng = np.random.default_rng(11)
    n = 300
    # points in and around the scene (the sampler is defined for any x);
    # each ball reaches 1.05 to 20 times the distance to the nearest Neumann
    # primitive, up to 0.8 L
    x = _probe_points(spec, n, rng)
    neu = np.nonzero(spec.bc == 1)[0]
    dmin = np.array([_prim_dist(spec, xi.astype(np.float64), neu).min() for xi in x])
    r = np.minimum(0.8 * R.L, dmin * np.exp(rng.uniform(math.log(1.05), math.log(20.0), n))).astype(np.float32)
    z, pdf, pr = W.wost_probe_neumann_sample(S.handle, x, r, 29, dim)
    checked = ties = 0
    for i in range(n):
        xi = x[i].astype(np.float64)
        ri = float(r[i])
        pdfs, reach, near = _alg6_pdfs(nodes, slot_prim, slot_meas, spec, xi, ri, offset, tol)
        assert reach <= 1.0 + 1e-12
        # every Neumann primitive meeting the ball can be drawn
        d = _prim_dist(spec, xi, neu)
        for p in neu[d < ri - tol]:
            assert slot_of[int(p)] in pdfs, (i, int(p), ri)
        if pr[i] < 0:
            # no sample: FP64 must give a dead end some probability, or tie
            assert reach < 1.0 - 1e-9 or near, (i, reach)
            continue
        k = slot_of[int(pr[i])]
        assert _prim_dist(spec, xi, [pr[i]])[0] <= ri + tol
        checked += 1
        if k not in pdfs or abs(float(pdf[i]) - pdfs[k]) > 1e-4 * pdfs[k]:
            assert near, (i, k, float(pdf[i]), pdfs.get(k))
            ties += 1
    assert checked > n // 2
    assert ties <= 2 + 0.01 * checked, f"{ties} near-tie pdf differences of {checked}"

# ---------------------------------------------------------------------------
# per-step trace parity
# ---------------------------------------------------------------------------

def _trace_parity(spec, points, eps, seed=5, n_walks=4, max_rec=256, tol_rel=1e-5, prims=None,
                  sigma=0.0, tik_sigma=0.0, tik_steps=0):
    S, R = W.Scene(spec), O.Scene(spec)
    tol = tol_rel * R.L
    P = R.params(eps, seed, sigma=sigma, tik_sigma=tik_sigma, tik_steps=tik_steps)
    opts = W.make_opts(sigma=sigma, tikhonov_sigma=tik_sigma, tikhonov_steps=tik_steps)
    n = points.shape[0]
    pts = np.repeat(points, n_walks, axis=0)
    pid = np.repeat(np.arange(n), n_walks).astype(np.uint32)
    wid = np.tile(np.arange(n_walks), n).astype(np.uint32)
    pr = np.repeat(prims, n_walks).astype(np.int32) if prims is not None else None
    recs, ns, vals = W.wost_trace_walks(S.handle, pts, pid, wid, eps, seed, max_rec, opts=opts, prims=pr)
    if pr is not None:   # boundary starts: the first step sits on the given primitive
        for i in range(pts.shape[0]):
            g = recs[i * max_rec]
            assert g.on_neumann == 1 and g.cur == pr[i]
    dim = spec.dim
    checked = mism = 0
    for i in range(pts.shape[0]):
        for k in range(min(ns[i], max_rec)):
            g = recs[i * max_rec + k]
            x = np.array(g.x[:dim], np.float64)
            nn = np.array(g.n[:dim], np.float64)
            c, o, nxt = R.step(P, int(pid[i]), int(wid[i]), k, x, n=nn, onN=bool(g.on_neumann), cur=g.cur)
            checked += 1
            assert abs(g.d_dirichlet - o.dD) <= tol or (g.d_dirichlet > 1e37 and o.dD > 1e37), \
                (i, k, g.d_dirichlet, o.dD)
            if g.term != o.term:
                if 4 in (g.term, o.term):   # roulette decided on the other side of U = Q
                    assert g.q == pytest.approx(o.q, rel=1e-3, abs=1e-6), (i, k, g.q, o.q)
                else:
                    assert abs(o.dD - eps) <= tol, (i, k, "termination differs away from the shell")
                mism += 1
                break
            if g.term in (1, 2, 3):
                assert g.g_term == pytest.approx(o.g_term, abs=1e-4 * max(1.0, abs(o.g_term)))
                break
            res = step_mismatch(R, P, dim, g, o, tol)
            if res is not None:
                # only a near-tie of the oracle's decision may part the walks
                assert_tie(f"walk {i} step {k}", res)
                mism += 1
                break       # the two walks part ways; the rest is not comparable
    assert checked > 0
    # near-ties are rare: the deciding values fall within 1e-5 L of a threshold
    assert mism <= 2 + 2e-3 * checked, f"{mism} near-tie steps out of {checked}"
    return checked


def test_trace_parity_unit_square():
    c = I.unit_square_case(n_grid=8)
    assert _trace_parity(c["scene"], c["points"], 1e-3) > 500


def test_trace_parity_star_polygon():
    spec = _star(2048)
    pts = I.star_polygon_points(48, seed=3, vertices=spec.vertices)
    assert _trace_parity(spec, pts, 1e-4) > 500


def test_trace_parity_icosphere():
    spec, mesh = _ico(3)
    pts = I.radial_mesh_points(mesh, 32, 2)
    assert _trace_parity(spec, pts, 1e-4, n_walks=3) > 300


# ---------------------------------------------------------------------------
# whole solves
# ---------------------------------------------------------------------------

def test_solve_unit_square_vs_exact_and_oracle():
    c = I.unit_square_case()
    S = W.Scene(c["scene"])
    mean, var = W.wost_solve(S.handle, c["points"], c["walks"], c["eps"], c["seed"])
    u = c["scene"].exact(c["points"])
    se = np.sqrt(u * (1 - u) / c["walks"])
    bad, allowed = count_bad((mean - u) / se)
    assert bad <= allowed
    r = O.Scene(c["scene"]).solve(c["points"], c["walks"], c["eps"], seed=c["seed"])
    se2 = np.sqrt(2 * u * (1 - u) / c["walks"])
    bad, allowed = count_bad((mean - r["mean"]) / se2)
    assert bad <= allowed
    st = W.wost_get_stats(S.handle)
    assert st.walks == 1024 * 256 and st.capped == 0 and st.escaped == 0
    assert st.steps >= st.walks


def test_solve_star_polygon_vs_exact_and_oracle():
    spec = _star(2048)
    pts = I.star_polygon_points(256, seed=1, vertices=spec.vertices)
    S = W.Scene(spec)
    Wk = 512
    mean, var = W.wost_solve(S.handle, pts, Wk, 1e-4, 7)
    u = spec.exact(pts)
    bad, allowed = count_bad((mean - u) / np.sqrt(var / Wk))
    assert bad <= allowed
    sub = slice(0, 64)
    r = O.Scene(spec).solve(pts[sub], 128, 1e-4, seed=11)
    z = (mean[sub] - r["mean"]) / np.sqrt(var[sub] / Wk + r["var"] / 128)
    bad, allowed = count_bad(z)
    assert bad <= allowed


def test_solve_icosphere_poisson_vs_exact_and_oracle():
    spec, mesh = _ico(4)
    pts = I.radial_mesh_points(mesh, 256, 5)
    S = W.Scene(spec)
    Wk = 512
    mean, var = W.wost_solve(S.handle, pts, Wk, 1e-4, 3)
    u = spec.exact(pts)
    bad, allowed = count_bad((mean - u) / np.sqrt(var / Wk))
    assert bad <= allowed
    sub = slice(0, 24)
    r = O.Scene(spec).solve(pts[sub], 128, 1e-4, seed=4)
    z = (mean[sub] - r["mean"]) / np.sqrt(var[sub] / Wk + r["var"] / 128)
    bad, allowed = count_bad(z)
    assert bad <= allowed
    st = W.wost_get_stats(S.handle)
    assert st.capped == 0 and st.escaped == 0


# ---------------------------------------------------------------------------
# determinism, forms, invariants and edge cases
# ---------------------------------------------------------------------------

def _solve_dev(S, pts, Wk, eps, seed, opts):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    m = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    W.wost_solve_ex(S.handle, d, pts.shape[0], Wk, eps, seed, 0, 0, opts, m, v,
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return m.cpu().numpy(), v.cpu().numpy()


def test_launch_forms_bit_identical():
    spec = _star(2048)
    pts = I.star_polygon_points(1000, seed=2, vertices=spec.vertices)   # ragged vs the block size
    S = W.Scene(spec)

    def solve(opts):
        # the per-walk buffer is reused between solves, so equal bits alone
        # would not show a walk that a form skipped: every walk must end once
        r = _solve_dev(S, pts, 96, 1e-4, 9, opts)
        assert W.wost_get_stats(S.handle).walks == 1000 * 96
        return r

    a = solve(W.make_opts(mode=1))
    b = solve(W.make_opts(mode=0))
    c = solve(W.make_opts(mode=0, grid=7, refill=16))
    d = solve(W.make_opts(mode=0, walk_order=1))
    e = solve(W.make_opts(mode=1, walk_order=1))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    assert np.array_equal(a[0], d[0]) and np.array_equal(a[1], d[1])
    assert np.array_equal(a[0], e[0]) and np.array_equal(a[1], e[1])
    # per-lane searches (mode 2) and the default wave-cooperative searches
    # with other grids: same bits, whatever walks share a wave
    f = solve(W.make_opts(mode=2))
    g = solve(W.make_opts(mode=0, grid=3, refill=8, walk_order=1))
    h = solve(W.make_opts(mode=0, grid=1))      # one block: every wave's claims run to the end
    assert np.array_equal(a[0], h[0]) and np.array_equal(a[1], h[1])
    assert np.array_equal(a[0], f[0]) and np.array_equal(a[1], f[1])
    assert np.array_equal(a[0], g[0]) and np.array_equal(a[1], g[1])


def test_cooperative_form_bit_identical_3d():
    """3D mesh with Neumann and source terms: the cooperative kernel (queries
    split over lanes by work stealing, the default form) returns the plain
    kernel's bits, as does the per-lane persistent kernel."""
    spec, mesh = _ico(4, 1)
    pts = I.radial_mesh_points(mesh, 700, 3)
    S = W.Scene(spec)
    a = _solve_dev(S, pts, 40, 1e-3, 11, W.make_opts(mode=1))
    b = _solve_dev(S, pts, 40, 1e-3, 11, W.make_opts(mode=0))
    c = _solve_dev(S, pts, 40, 1e-3, 11, W.make_opts(mode=0, grid=5, walk_order=1))
    d = _solve_dev(S, pts, 40, 1e-3, 11, W.make_opts(mode=2))
    for o in (b, c, d):
        assert np.array_equal(a[0], o[0]) and np.array_equal(a[1], o[1])


def test_autotune_picks_valid_options_and_keeps_results():
    import torch
    spec = _star(2048)
    pts = I.star_polygon_points(2000, seed=2, vertices=spec.vertices)
    S = W.Scene(spec)
    ref = _solve_dev(S, pts, 64, 1e-4, 4, None)
    d = torch.from_numpy(pts).cuda()
    o = W.wost_autotune(S.handle, d, len(pts), 64, 1e-4, 4, sample_walks=1 << 16)
    assert o.mode == 0 and o.refill in (1, 8, 32) and o.grid >= 1 and o.walk_order in (0, 1)
    assert o.claim_walks in (128, 32, 512) and o.steal_lanes == 1
    got = _solve_dev(S, pts, 64, 1e-4, 4, o)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    # every candidate of every knob keeps the bits, 2D and 3D
    for claim in (1, 32, 512):
        for steal in (1, 8, 48):
            got = _solve_dev(S, pts, 64, 1e-4, 4, W.make_opts(claim_walks=claim, steal_lanes=steal, grid=11))
            assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
    spec3, mesh = _ico(3, 1)
    pts3 = I.radial_mesh_points(mesh, 300, 3)
    S3 = W.Scene(spec3)
    ref3 = _solve_dev(S3, pts3, 32, 1e-4, 4, None)
    o3 = W.wost_autotune(S3.handle, torch.from_numpy(pts3).cuda(), len(pts3), 32, 1e-4, 4, sample_walks=1 << 14)
    assert o3.claim_walks == 1 and o3.steal_lanes in (16, 32, 8, 48)
    for steal in (16, 1, 8, 32, 48, 64):
        got = _solve_dev(S3, pts3, 32, 1e-4, 4, W.make_opts(steal_lanes=steal, grid=13))
        assert np.array_equal(ref3[0], got[0]) and np.array_equal(ref3[1], got[1])


def test_split_solve_matches_whole():
    """point_base / walk_base make pieces draw the same random numbers."""
    import torch
    spec = _star(1024)
    pts = I.star_polygon_points(300, seed=4, vertices=spec.vertices)
    S = W.Scene(spec)
    whole = _solve_dev(S, pts, 64, 1e-4, 5, None)
    d = torch.from_numpy(pts[100:]).cuda()
    m = torch.empty(200, dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    W.wost_solve_ex(S.handle, d, 200, 64, 1e-4, 5, 100, 0, None, m, v, None)
    torch.cuda.synchronize()
    assert np.array_equal(m.cpu().numpy(), whole[0][100:])


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_solution_exact(dim):
    if dim == 2:
        spec = _star(512, 1)
        pts = I.star_polygon_points(200, seed=2, vertices=spec.vertices)
    else:
        spec, mesh = _ico(2, 2)
        pts = I.radial_mesh_points(mesh, 100, 1)
    spec.g, spec.h, spec.f = I.Fn(I.FN_CONST, 0, (2.5,)), I.Fn(), I.Fn()
    S = W.Scene(spec)
    mean, var = W.wost_solve(S.handle, pts, 64, 1e-3, 9)
    assert np.all(mean == 2.5) and np.all(var == 0.0)


def test_eps_shell_start_returns_g():
    spec = _star(512, 0)
    Vd = spec.vertices.astype(np.float64)
    D = np.nonzero(spec.bc == I.DIRICHLET)[0][::17]
    mids = 0.5 * (Vd[spec.prims[D, 0]] + Vd[spec.prims[D, 1]])
    pts = (mids * (1 - 2e-5 / np.linalg.norm(mids, axis=1, keepdims=True))).astype(np.float32)
    S = W.Scene(spec)
    mean, var = W.wost_solve(S.handle, pts, 8, 1e-4, 1)
    R = O.Scene(spec)
    for i, x in enumerate(pts):
        d, xb, _ = R.closest_dirichlet(x)
        assert var[i] == 0.0
        assert mean[i] == pytest.approx(math.exp(xb[0]) * math.cos(xb[1]), abs=2e-6)


def test_single_walk_zero_variance_and_empty():
    c = I.unit_square_case(n_grid=4)
    S = W.Scene(c["scene"])
    mean, var = W.wost_solve(S.handle, c["points"], 1, 1e-3, 0)
    assert np.all(var == 0.0) and set(np.unique(mean)) <= {0.0, 1.0}
    m0, v0 = W.wost_solve(S.handle, c["points"][:0], 16, 1e-3, 0)
    assert m0.size == 0


def test_max_steps_cap_counted():
    c = I.unit_square_case(n_grid=4)
    S = W.Scene(c["scene"])
    _solve_dev(S, c["points"], 32, 1e-3, 0, W.make_opts(max_steps=2))
    st = W.wost_get_stats(S.handle)
    assert st.capped > 0 and st.walks == 16 * 32 and st.steps <= 3 * st.walks


def test_solve_argument_errors():
    c = I.unit_square_case(n_grid=4)
    S = W.Scene(c["scene"])
    for args in ((c["points"], 0, 1e-3, 0), (c["points"], 4, 0.0, 0), (c["points"], 4, -1.0, 0)):
        with pytest.raises(W.WostError) as e:
            W.wost_solve(S.handle, *args)
        assert e.value.status == W.WOST_ERR_INVALID_ARG


def test_traffic_variant_identical_and_counted():
    spec = _star(2048)
    pts = I.star_polygon_points(500, seed=6, vertices=spec.vertices)
    S = W.Scene(spec)
    a = _solve_dev(S, pts, 64, 1e-4, 2, None)
    st_a = W.wost_get_stats(S.handle)
    b = _solve_dev(S, pts, 64, 1e-4, 2, W.make_opts(flags=W.WOST_SOLVE_COUNT_TRAFFIC))
    st_b = W.wost_get_stats(S.handle)
    tr = W.wost_get_traffic(S.handle)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert st_a.steps == st_b.steps and st_b.mode == 1
    # one Q.1 descent per step reads at least the root node
    assert tr.q1_nodes >= st_b.steps and tr.q1_prims > 0
    # Q.2..Q.4 and the visibility ray run on every non-terminating step
    assert tr.q3_nodes >= st_b.steps - st_b.walks
    assert tr.q4_nodes >= st_b.steps - st_b.walks
    assert tr.bytes > tr.q1_nodes * tr.node_bytes


def test_valu_measurement():
    """The VALU issue measurements behind the ALU rooflines: positive,
    within a few times the derived FP32 lane rate, bad kinds rejected."""
    for kind in (0, 1):
        g = W.wost_measure_valu(kind, 256)
        assert 1e3 < g < 4 * 256 * 4 * 16 * 2.4
    with pytest.raises(W.WostError):
        W.wost_measure_valu(2, 16)


def test_l2_read_measurement():
    """The streaming-read measurement behind the roofline: positive, below
    the derived L2 peak with margin, and argument errors rejected."""
    g = W.wost_measure_l2_read(2 << 20, 8)
    assert 1e3 < g < 1.5 * 8 * 16 * 128 * 2.4
    with pytest.raises(W.WostError):
        W.wost_measure_l2_read(100, 1)          # not a multiple of 16
