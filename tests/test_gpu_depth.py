"""Depth output for primary rays (Sec. 7: the network can encode the first
hit's depth instead of visibility): the GPU closest-hit caster against the
binary64 tracer, the depth training step's gradients against the oracle's L2
gradients, the depth read-out against the oracle's, and training that lowers
the depth error."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

from gpu_util import make_pair

pytestmark = pytest.mark.gpu


def _grad_close(g, g64, rel_norm=1e-4, rel_max=1e-3):
    err = np.abs(g - g64)
    nrm = np.linalg.norm(err) / max(np.linalg.norm(g64), 1e-300)
    assert nrm <= rel_norm, f"relative norm error {nrm}"
    assert err.max() <= rel_max * np.abs(g64).max(), f"max error {err.max()} vs max |g| {np.abs(g64).max()}"
    return nrm, err.max()


def _camera_rays(n, box, g, dist=4.0):
    """Primary rays of a pinhole camera on a sphere around the box, looking at
    its centre through a 40-degree field of view; t_max = inf."""
    c = 0.5 * (box[:3] + box[3:]).astype(np.float64)
    eye = c + dist * np.array([0.3, 0.5, 0.81])
    fwd = (c - eye) / np.linalg.norm(c - eye)
    right = np.cross(fwd, [0, 1, 0])
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    sx, sy = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    half = np.tan(np.radians(20))
    d = fwd[None] + half * (sx[:, None] * right[None] + sy[:, None] * up[None])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.concatenate([np.broadcast_to(eye, (n, 3)), d], 1).astype(np.float32)
    return rays, np.full(n, np.inf, np.float32)


@pytest.mark.parametrize("case", ["tiny", "frame_mesh"])
def test_closest_hit_matches_oracle(case):
    import torch
    from paper_2306_07191_amd import nif
    g = np.random.default_rng(5)
    if case == "tiny":
        w = S.tiny_workload(n_rays=16384)
        tris, rays, tmax = w["tris"], w["rays"], w["tmax"]
        tmax = np.where(g.uniform(size=tmax.shape[0]) < 0.3, g.uniform(0.5, 4, tmax.shape[0]), tmax).astype(np.float32)
        ref = O.closest_brute(tris, rays, tmax)
        _, ref32 = O.trace_brute32(tris, rays, tmax)
    else:
        tris = S.frame_mesh()
        rays, tmax = _camera_rays(20000, S.mesh_aabb(tris), g)
        ob = O.BVH(tris)
        ref = ob.closest(rays, tmax)
        _, ref32 = ob.trace32(rays, tmax)
    bvh = nif.BVH(tris)
    t32 = bvh.closest(torch.from_numpy(rays).cuda(), torch.from_numpy(tmax).cuda()).cpu().numpy()
    bvh.close()
    # the nearest binary32 hit distance, decision for decision: bit-exact
    np.testing.assert_array_equal(t32, ref32)
    t = t32.astype(np.float64)
    both = np.isfinite(t) & np.isfinite(ref)
    agree = float((np.isfinite(t) == np.isfinite(ref)).mean())
    rel = np.abs(t[both] - ref[both]) / ref[both]
    close = float((rel <= 1e-5).mean())
    print(f"{case}: hit agreement {agree:.6f}, {both.sum()} hits, within 1e-5: {close:.6f}, max rel {rel.max():.2e}")
    assert both.sum() > 0.2 * t.shape[0]
    # binary32 against binary64 watertight tests: a ray grazing an edge may hit in one and not the other
    assert agree >= 0.9999 and close >= 0.9999


def test_depth_gradients_match_oracle():
    import torch
    w = S.tiny_workload(n_rays=4096)
    w["mlps"] = (w["mlps"].astype(np.float64) * 2.0).astype(np.float32)
    t_hit = O.closest_brute(w["tris"], w["rays"], w["tmax"]).astype(np.float32)  # the caller's binary32 targets
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    ctx.setup_training()
    rays, ids, tmax, th = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (w["rays"], w["ids"], w["tmax"], t_hit))
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros(ctx.mlp_params, device="cuda")
    ctx.train_step_depth(rays, ids, tmax, th, step=1, adam=None, loss=loss, mlp_grad=g)
    torch.cuda.synchronize()
    L64, B, gW, gx = model.depth_loss_backward(w["rays"], w["ids"], w["tmax"], t_hit.astype(np.float64))
    assert B > 1000
    assert abs(loss.item() - L64) <= 1e-5 * abs(L64), (loss.item(), L64)
    st = _grad_close(g.cpu().numpy().astype(np.float64), gW[0])
    gg64 = model.grid_grad_dense(0, w["rays"], w["ids"], w["tmax"], gx)
    gg = ctx.train_bufs[0][0].cpu().numpy().astype(np.float64)
    sg = _grad_close(gg, gg64)
    print("depth: B", B, "mlp grad err", st, "grid grad err", sg)
    ctx.close()


def test_depth_readout_matches_oracle():
    import torch
    w = S.tiny_workload(n_rays=8192)
    w["rays"][:5, 3:] = 0.0  # invalid queries: NaN
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    rays, ids, tmax = (torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in ("rays", "ids", "tmax"))
    y = ctx.query(rays, ids, tmax, dtype="f32")
    dep = ctx.depth_from_visibility(rays, ids, tmax, y).cpu().numpy().astype(np.float64)
    ref = model.depth(w["rays"], w["ids"], w["tmax"])
    st = model.status(w["rays"], w["ids"], w["tmax"])
    assert np.isnan(dep[st == -1]).all()
    assert np.isposinf(dep[st == 0]).all() and np.isposinf(ref[st == 0]).all()
    hit = st == 1
    assert hit.sum() > 4000
    # the binary32 visibility is within 1e-5 y64 of the oracle's (the binary32
    # path's tolerance), scaled by the segment length, plus the rounding of t
    ta, tb = model.segment(w["rays"], w["ids"], w["tmax"])
    y64 = model.forward(w["rays"], w["ids"], w["tmax"])["y"]
    tol = 1e-5 * y64[hit] * (tb[hit] - ta[hit]) + 4e-7 * np.abs(ref[hit]) + 1e-7
    err = np.abs(dep[hit] - ref[hit])
    print(f"depth read-out: max |err| {err.max():.2e}, max err / tol {(err / tol).max():.3f}")
    assert (err <= tol).all()
    ctx.close()


def test_depth_training_lowers_error():
    """Camera rays at the small scene's mesh, closest-hit targets from the GPU
    caster: 60 training steps lower the mean depth error on hit rays."""
    import torch
    from paper_2306_07191_amd import nif
    w = S.tiny_workload(n_rays=16)
    ctx, _ = make_pair(w, grid_amp=1e-4)
    ctx.prepare("f32")
    ctx.setup_training()
    bvh = nif.BVH(w["tris"])
    g = np.random.default_rng(8)
    test_r, test_t = _camera_rays(20000, w["aabb"][0], g)
    tr, tt = torch.from_numpy(test_r).cuda(), torch.from_numpy(test_t).cuda()
    t_ref = bvh.closest(tr, tt)
    tid = torch.zeros(20000, dtype=torch.int32, device="cuda")

    def depth_error():
        ctx.prepare("f32")
        y = ctx.query(tr, tid, tt, dtype="f32")
        dep = ctx.depth_from_visibility(tr, tid, tt, y)
        ok = torch.isfinite(t_ref) & torch.isfinite(dep)
        return float((dep[ok] - t_ref[ok]).abs().mean().item())

    e0 = depth_error()
    nb = 8192
    ids = torch.zeros(nb, dtype=torch.int32, device="cuda")
    for step in range(1, 61):
        r_, t_ = _camera_rays(nb, w["aabb"][0], g)
        r, t = torch.from_numpy(r_).cuda(), torch.from_numpy(t_).cuda()
        ctx.train_step_depth(r, ids, t, bvh.closest(r, t), step=step)
    e1 = depth_error()
    print(f"mean |depth error| on hit rays: {e0:.4f} -> {e1:.4f}")
    assert e1 < 0.5 * e0
    bvh.close()
    ctx.close()
