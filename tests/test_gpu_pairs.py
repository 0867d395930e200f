"""Pair expansion and per-ray combination (nif_expand_pairs, nif_combine_pairs)
against the oracle: bit-exact pair lists, then the combined visibility."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

from gpu_util import make_pair

pytestmark = pytest.mark.gpu


def _scene(n=20000, K=12, seed=5):
    g = np.random.default_rng(seed)
    lo = g.uniform(-4, 3, (K, 3))
    boxes = np.concatenate([lo, lo + g.uniform(0.4, 2.0, (K, 3))], axis=1).astype(np.float32)
    o = g.uniform(-6, 6, (n, 3))
    k = g.integers(0, K, n)
    tgt = boxes[k, :3] + g.uniform(size=(n, 3)) * (boxes[k, 3:] - boxes[k, :3])
    rays = np.concatenate([o, tgt - o], axis=1).astype(np.float32)
    tmax = np.where(g.uniform(size=n) < 0.6, np.inf, g.uniform(0.2, 2.0, n) * np.linalg.norm(tgt - o, axis=1))
    tmax = tmax.astype(np.float32)
    rays[::501, 3:] = 0          # invalid: zero direction
    rays[7, 0] = np.nan          # invalid: NaN origin
    tmax[11] = -1.0              # invalid: negative t_max
    rays[13, 3:] = [0, 1, 0]     # axis-parallel
    mlps = np.stack([S.xavier_mlp(S.TINY, S.rng(70, 3, m)) for m in range(3)])
    return dict(shape=S.TINY, aabb=boxes, mlps=mlps, mlp_index=(np.arange(K) % 3).astype(np.int32), rays=rays,
                tmax=tmax, ids=np.zeros(n, np.int32))


@pytest.mark.parametrize("K", [12, 40, 70])  # boxes one by one with hit masks, box groups, no masks
def test_pairs_match_oracle_and_combine(K):
    import torch
    w = _scene(K=K)
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    rays, tmax = torch.from_numpy(w["rays"]).cuda(), torch.from_numpy(w["tmax"]).cuda()
    pr_rays, pr_tmax, pr_ids, pr_ray = ctx.expand_pairs(rays, tmax, max_pairs=100)  # too small: retried
    ref_ray, ref_obj = model.expand_pairs(w["rays"], w["tmax"])
    assert ref_ray.size > 5000
    np.testing.assert_array_equal(pr_ray.cpu().numpy(), ref_ray)
    np.testing.assert_array_equal(pr_ids.cpu().numpy(), ref_obj)
    np.testing.assert_array_equal(pr_rays.cpu().numpy(), w["rays"][ref_ray])
    np.testing.assert_array_equal(pr_tmax.cpu().numpy(), w["tmax"][ref_ray])
    # every pair is a query that meets its box
    y = ctx.query(pr_rays, pr_ids, pr_tmax, dtype="f32")
    ref = model.forward(w["rays"][ref_ray], ref_obj, w["tmax"][ref_ray])
    assert (ref["status"] == 1).all()
    yc = y.cpu().numpy().astype(np.float64)
    assert (np.abs(yc - ref["y"]) <= 1e-5 * ref["y"]).all()
    n = w["tmax"].shape[0]
    vis = ctx.combine_pairs(pr_ray, y, n).cpu().numpy()
    np.testing.assert_array_equal(vis, O.combine_pairs(ref_ray, yc, n))
    assert 0 < vis.mean() < 1


def test_pairs_empty_inputs():
    import torch
    w = _scene(n=40)
    ctx, _ = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    e = torch.empty(0, device="cuda")
    pr_rays, pr_tmax, pr_ids, pr_ray = ctx.expand_pairs(e.view(0, 6), e)
    assert pr_ray.numel() == 0
    out = ctx.combine_pairs(pr_ray, e, 5)
    assert (out.cpu().numpy() == 1).all()  # rays without pairs are visible
