"""Light importance sampling on the GPU (nif_light_* through the C ABI)
against the binary64 oracle: the chosen triangle bit-exact (a binary32
comparison with the same table on both sides), rays, t_max and density to
binary32 rounding."""
import numpy as np
import pytest

from oracle import light_sampling as LS

pytestmark = pytest.mark.gpu


def _lights(L, g):
    c = np.stack([g.uniform(-3, 3, L), g.uniform(4, 6, L), g.uniform(-3, 3, L)], 1)
    tris = (c[:, None, :] + g.normal(size=(L, 3, 3)) * 0.3).reshape(L, 9).astype(np.float32)
    rad = np.exp(g.normal(size=L) * 1.5).astype(np.float32)
    rad[::7] = 0.0  # dark triangles are never chosen
    return tris, rad


@pytest.mark.parametrize("L,n", [(1, 1000), (300, 100000), (5000, 65537), (16384, 3000), (20000, 40000)])
def test_light_sampling_matches_oracle(L, n):
    import torch
    from paper_2306_07191_amd import nif
    g = np.random.default_rng(L + n)
    tris, rad = _lights(L, g)
    if L == 1:
        rad[:] = 2.0
    pts = np.stack([g.uniform(-4, 4, n), g.uniform(-0.5, 0.5, n), g.uniform(-4, 4, n)], 1).astype(np.float32)
    u = g.uniform(size=(n, 3)).astype(np.float32)
    u[0, 0], u[1, 0] = 0.0, np.nextafter(np.float32(1), np.float32(0))
    light = nif.Light(tris, rad)
    rays, tmax, pdf, tri = light.sample(torch.from_numpy(pts).cuda(), torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    ref = LS.sample(tris, rad, pts, u)
    got_tri = tri.cpu().numpy()
    np.testing.assert_array_equal(got_tri, ref["tri"])
    assert got_tri[0] == int(np.argmax(LS.cdf_table(tris, rad) > 0))  # u0 = 0: the first lit triangle
    r = rays.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(r[:, :3], pts.astype(np.float64))
    np.testing.assert_allclose(r[:, 3:], ref["d"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(tmax.cpu().numpy(), ref["tmax"], rtol=2e-6)
    cos = np.abs((LS.areas_normals(tris)[1][ref["tri"]] * ref["d"]).sum(1))
    ok = cos > 1e-2  # the density divides by the light's cosine: grazing samples are ill-conditioned
    np.testing.assert_allclose(pdf.cpu().numpy()[ok], ref["pdf"][ok], rtol=1e-4)
    assert (rad[got_tri] > 0).all()
    light.close()


def test_light_errors_and_empty():
    import torch
    from paper_2306_07191_amd import nif
    good = np.array([[0, 5, 0, 1, 5, 0, 0, 5, 1]], np.float32)
    with pytest.raises(nif.NifError):   # zero-area triangle
        nif.Light(np.array([[0, 5, 0, 1, 5, 0, 2, 5, 0]], np.float32), np.ones(1, np.float32))
    with pytest.raises(nif.NifError):   # negative radiance
        nif.Light(good, -np.ones(1, np.float32))
    with pytest.raises(nif.NifError):   # no flux at all
        nif.Light(good, np.zeros(1, np.float32))
    light = nif.Light(good, np.ones(1, np.float32))
    z = torch.zeros((0, 3), device="cuda")
    light.sample(z, z)  # n = 0 is a no-op
    light.close()


def test_training_on_sampled_rays():
    """Training batches drawn by light importance sampling (Sec. 5 "Training"):
    shadow rays from points under the small scene's object to an emitter above
    it, exact labels from the GPU BVH, a few training steps; the sampled rays
    start at the given points and end on the emitter, both labels occur, and
    the loss falls."""
    import torch
    from paper_2306_07191_amd import nif, synth as S
    from gpu_util import make_pair
    w = S.tiny_workload(n_rays=16)
    ctx, _ = make_pair(w, grid_amp=1e-4)
    ctx.prepare("f32")
    ctx.setup_training()
    g = np.random.default_rng(3)
    L = 64
    c = np.stack([g.uniform(-1.5, 1.5, L), np.full(L, 4.0), g.uniform(-1.5, 1.5, L)], 1)
    tris = (c[:, None, :] + g.normal(size=(L, 3, 3)) * 0.2).reshape(L, 9).astype(np.float32)
    light = nif.Light(tris, np.exp(g.normal(size=L)).astype(np.float32))
    bvh = nif.BVH(w["tris"])
    nb = 8192
    ids = torch.zeros(nb, dtype=torch.int32, device="cuda")
    losses = []
    for step in range(1, 31):
        pts = np.stack([g.uniform(-1.5, 1.5, nb), np.full(nb, -3.0), g.uniform(-1.5, 1.5, nb)], 1).astype(np.float32)
        p = torch.from_numpy(pts).cuda()
        u = torch.from_numpy(g.uniform(size=(nb, 3)).astype(np.float32)).cuda()
        rays, tmax, _, tri = light.sample(p, u)
        lab = bvh.anyhit(rays, tmax)
        if step == 1:
            r = rays.cpu().numpy().astype(np.float64)
            np.testing.assert_array_equal(r[:, :3], pts)
            end = r[:, :3] + tmax.cpu().numpy()[:, None].astype(np.float64) * r[:, 3:]
            verts = tris.reshape(L, 3, 3)[tri.cpu().numpy()]
            assert (end[:, 1] > verts[:, :, 1].min(1) - 1e-3).all() and (end[:, 1] < verts[:, :, 1].max(1) + 1e-3).all()
            frac = float(lab.float().mean().item())
            assert 0.05 < frac < 0.95, frac
        loss = torch.zeros(1, device="cuda")
        ctx.train_step(rays, ids, tmax, lab, step=step, loss=loss)
        losses.append(float(loss.item()))
    assert np.mean(losses[-5:]) < 0.9 * np.mean(losses[:5]), losses
    light.close()
    bvh.close()
    ctx.close()
