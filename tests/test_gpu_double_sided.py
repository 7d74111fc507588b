"""Double-sided boundaries on the GPU (appendix on open domains and
double-sided boundaries), through the C-ABI: per-step parity with the FP64
oracle re-run from the GPU's own state (side decisions included), whole
solves against the closed forms and the oracle, boundary starts on either
side, and bit-identity across launch forms and the batched form."""
import numpy as np
import pytest

import oracle as O
from paper_2302_11815_amd import inputs as I

pytestmark = pytest.mark.gpu
W = pytest.importorskip("paper_2302_11815_amd.wost")
from _trace import trace_parity  # noqa: E402

SCENES = {
    "disk2d": (I.double_sided_disk_scene, 2),
    "crack2d": (I.crack_scene_2d, 2),
    "sphere3d": (I.double_sided_sphere_scene, 3),
    "crack3d": (I.crack_scene_3d, 3),
}


def _points(name, n, seed):
    make, dim = SCENES[name]
    if name in ("disk2d", "sphere3d"):
        return I.box_points(n, dim, seed, half=0.9, avoid_radius=0.5, margin=0.05)
    return I.box_points(n, dim, seed, half=0.8)


def _dev_solve(S, pts, walks, eps, seed, opts=None):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    m = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    W.wost_solve_ex(S.handle, d, pts.shape[0], walks, eps, seed, 0, 0, opts, m, v, None)
    torch.cuda.synchronize()
    return m.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("name", sorted(SCENES))
def test_trace_parity_double_sided(name):
    make, dim = SCENES[name]
    spec = make()
    pts = _points(name, 40 if dim == 2 else 24, 3)
    if name in ("disk2d", "sphere3d"):      # walks inside the closed sheet too
        pts = np.concatenate([pts, I.box_points(8, dim, 4, half=0.25)])
    checked, sides, flips = trace_parity(spec, pts, 1e-3, n_walks=4 if dim == 2 else 3)
    assert checked > 300 and sides > 20 and flips > 5


@pytest.mark.parametrize("name", sorted(SCENES))
def test_solve_double_sided_vs_exact_and_oracle(name):
    make, dim = SCENES[name]
    spec = make()
    pts = _points(name, 512 if dim == 2 else 256, 5)
    walks, eps = 512, 1e-3
    S = W.Scene(spec)
    mean, var = _dev_solve(S, pts, walks, eps, 21)
    st = W.wost_get_stats(S.handle)
    assert st.capped == 0 and st.escaped == 0
    u = spec.exact(pts)
    se = np.sqrt(var / walks)
    coefs = (I.U_OUT_2D, I.U_IN_2D) if dim == 2 else (I.U_OUT_3D, I.U_IN_3D)
    gb = max(float(np.abs(np.asarray(c[1:], float)).sum()) * 3 for c in coefs)   # loose sup |grad u|
    bad = np.abs(mean - u) > 4 * se + eps * gb
    assert int(bad.sum()) <= max(2, int(0.006 * pts.shape[0])), (np.nonzero(bad)[0][:10])
    # aggregate bias: Gaussian across points
    agg = float(np.mean(mean - u))
    agg_se = float(np.sqrt(np.sum(var / walks))) / pts.shape[0]
    assert abs(agg) <= 5 * agg_se + eps * gb
    # the oracle on a sample of the same streams
    idx = np.arange(0, pts.shape[0], max(1, pts.shape[0] // 24))
    r = O.Scene(spec).solve(pts[idx], walks, eps, seed=21, point_ids=idx.astype(np.uint32), nthreads=8)
    z = (mean[idx] - r["mean"]) / np.sqrt(var[idx] / walks + r["var"] / walks + 1e-300)
    assert np.sum(np.abs(z) > 4) <= 1, z


def test_boundary_starts_on_either_side():
    """Points on the double-sided Neumann arcs of the circle: the "+" start
    estimates the annulus solution, the "-" start the disk solution; a "-"
    start on a one-sided primitive is rejected."""
    import torch
    spec = I.double_sided_disk_scene()
    S = W.Scene(spec)
    V = spec.vertices.astype(np.float64)
    neu = np.nonzero(spec.bc == I.NEUMANN2)[0][3::6]
    mids = (0.5 * (V[spec.prims[neu, 0]] + V[spec.prims[neu, 1]])).astype(np.float32)
    d = torch.from_numpy(mids).cuda()
    m = torch.empty(mids.shape[0], dtype=torch.float64, device="cuda")
    v = torch.empty_like(m)
    walks, eps = 4096, 1e-3
    gb = 6.0
    for codes, want in ((neu, I.poly2_eval(I.U_OUT_2D, mids)), (-2 - neu, I.poly2_eval(I.U_IN_2D, mids))):
        W.wost_solve_boundary_ex(S.handle, d, codes.astype(np.int32), mids.shape[0], walks, eps, 4, d_mean=m, d_var=v)
        torch.cuda.synchronize()
        mean, var = m.cpu().numpy(), v.cpu().numpy()
        bad = np.abs(mean - want) > 4 * np.sqrt(var / walks) + eps * gb
        assert int(bad.sum()) <= 1, (mean[bad], want[bad])
    # the same walks in the oracle (a few points)
    r = O.Scene(spec).solve(mids[:6], walks, eps, seed=4, start_prims=-2 - neu[:6], nthreads=8)
    z = (mean[:6] - r["mean"]) / np.sqrt(var[:6] / walks + r["var"] / walks)
    assert np.sum(np.abs(z) > 4) == 0, z
    one_sided = np.array([-2 - 0], np.int32)      # primitive 0 is a one-sided Dirichlet segment
    with pytest.raises(W.WostError) as e:
        W.wost_solve_boundary_ex(S.handle, d, one_sided, 1, 8, eps, 0, d_mean=m, d_var=v)
    assert e.value.status == W.WOST_ERR_INVALID_ARG


@pytest.mark.parametrize("name", ["crack2d", "sphere3d"])
def test_launch_forms_and_batch_bit_identical(name):
    import torch
    make, dim = SCENES[name]
    spec = make()
    pts = _points(name, 777, 8)                     # ragged against the block size
    S = W.Scene(spec)
    a = _dev_solve(S, pts, 48, 1e-3, 2, W.make_opts(mode=0))
    b = _dev_solve(S, pts, 48, 1e-3, 2, W.make_opts(mode=1))
    c = _dev_solve(S, pts, 48, 1e-3, 2, W.make_opts(mode=2, walk_order=1))
    for x in (b, c):
        assert np.array_equal(a[0], x[0]) and np.array_equal(a[1], x[1])
    # batched with a one-sided scene in the same call
    other = I.unit_square_case(n_grid=8)
    S2 = W.Scene(other["scene"])
    ref2 = _dev_solve(S2, other["points"], 32, 1e-3, 3)
    items = []
    for SS, p, wk, eps, seed in ((S, pts, 48, 1e-3, 2), (S2, other["points"], 32, 1e-3, 3)):
        d = torch.from_numpy(np.ascontiguousarray(p)).cuda()
        m = torch.zeros(p.shape[0], dtype=torch.float64, device="cuda")
        v = torch.zeros_like(m)
        items.append((d, m, v, W.make_batch_item(SS.handle, d, p.shape[0], wk, eps, seed, m, v)))
    B = W.wost_batch_create()
    try:
        W.wost_solve_batch(B, [it[3] for it in items], W.make_opts(chunk_walks=256))
        torch.cuda.synchronize()
    finally:
        W.wost_batch_destroy(B)
    assert np.array_equal(items[0][1].cpu().numpy(), a[0]) and np.array_equal(items[0][2].cpu().numpy(), a[1])
    assert np.array_equal(items[1][1].cpu().numpy(), ref2[0])
