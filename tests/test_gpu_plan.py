"""Batched multi-object form: a tuned, graph-captured query plan over many
objects of uneven size (Zipf-distributed rays), against the eager query and
the oracle."""
import json

import numpy as np
import pytest

from paper_2306_07191_amd import synth as S

from gpu_util import check_outputs, make_pair

pytestmark = pytest.mark.gpu


def _multi_tiny(n_objects=8, n_rays=150000):
    w = S.multi_workload(n_objects=n_objects, n_rays=n_rays)
    w["shape"] = S.TINY
    w["mlps"] = np.stack([S.xavier_mlp(S.TINY, S.rng(60, 3, k)) for k in range(n_objects)])
    return w


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_plan_matches_eager_and_oracle_over_replays(dtype):
    import torch
    from paper_2306_07191_amd import nif
    w = _multi_tiny()
    ctx, model = make_pair(w, grid_amp=0.5, quant="exact" if dtype == "f32" else dtype)
    ctx.prepare(dtype)
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    z = torch.empty(ids.shape[0], device="cuda")
    plan = nif.Plan(ctx, rays, ids, tmax, dtype=dtype, logits=z)
    tun = json.loads(plan.tuning())
    # 4-level grids: orderings x grid sizes (no tile shapes besides the default)
    assert tun["candidates"] == 15 and tun["order"] in (0, 1, 2, 3) and tun["tuned_us"] > 0 and tun["shape"] == 0
    torch.cuda.synchronize()
    check_outputs(plan.out.cpu().numpy().astype(np.float64), z.cpu().numpy().astype(np.float64),
                  model.forward(w["rays"], w["ids"], w["tmax"]), dtype, f"plan {dtype}")
    g = np.random.default_rng(3)
    for rep in range(3):
        # new contents in the same buffers, eager work and a synchronisation between replays
        p = torch.from_numpy(g.permutation(ids.shape[0])).cuda()
        r2, i2, t2 = rays[p].clone(), ids[p].clone(), tmax[p].clone()
        rays.copy_(r2)
        ids.copy_(i2)
        tmax.copy_(t2)
        y_eager = ctx.query(rays, ids, tmax, dtype=dtype)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(plan.out.cpu().numpy(), y_eager.cpu().numpy())
    # a given schedule skips the tuning and gives the same outputs
    plan2 = nif.Plan(ctx, rays, ids, tmax, dtype=dtype, tuning='{"order": 0, "blocks_per_cu": 4}')
    assert json.loads(plan2.tuning())["candidates"] == 0
    plan2.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(plan2.out.cpu().numpy(), plan.out.cpu().numpy())
    plan.close()
    plan2.close()


def test_plan_tile_shapes_and_tuning_cache(tmp_path, monkeypatch):
    """8-level binary16 grids (the frame's shape, two objects): the tuner also
    times the fused kernel's tile shapes; every shape gives bit-identical
    outputs; with NIF_PLAN_CACHE set a tuned schedule is stored, and the next
    plan for the same key reads it instead of tuning."""
    import torch
    from paper_2306_07191_amd import nif
    K, n = 2, 200000
    w = S.multi_workload(n_objects=K, n_rays=n)
    w["shape"] = S.FRAME
    w["mlps"] = np.stack([S.xavier_mlp(S.FRAME, S.rng(61, 3, k)) for k in range(K)])
    ctx, _ = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    ctx.prepare("bf16")
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    outs = []
    for shape in (0, 1, 2):
        p = nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning=f'{{"order": 2, "blocks_per_cu": 8, "shape": {shape}}}')
        t = json.loads(p.tuning())
        assert t["shape"] == shape and t["gather_batch"] == {0: 12, 1: 6, 2: 3}[shape]
        assert t["waves_per_simd"] == {0: 3, 1: 2, 2: 4}[shape]
        p.launch()
        torch.cuda.synchronize()
        outs.append(p.out.cpu().numpy().copy())
        p.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    p = nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning='{"order": 3, "blocks_per_cu": 8, "shape": 1}')
    assert json.loads(p.tuning())["order"] == 3  # by object alone: the same outputs
    p.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p.out.cpu().numpy(), outs[0])
    p.close()
    cache = tmp_path / "plans.jsonl"
    monkeypatch.setenv("NIF_PLAN_CACHE", str(cache))
    p1 = nif.Plan(ctx, rays, ids, tmax, dtype="bf16")
    t1 = json.loads(p1.tuning())
    assert t1["candidates"] == 45 and not t1["from_cache"] and t1["tuned_us"] > 0
    line = json.loads(cache.read_text().strip().splitlines()[-1])
    assert "gfx950" in line["key"] and line["shape"] == t1["shape"] and line["order"] == t1["order"]
    p2 = nif.Plan(ctx, rays, ids, tmax, dtype="bf16")
    t2 = json.loads(p2.tuning())
    assert t2["from_cache"] and t2["candidates"] == 0
    assert (t2["order"], t2["blocks_per_cu"], t2["shape"]) == (t1["order"], t1["blocks_per_cu"], t1["shape"])
    p2.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p2.out.cpu().numpy(), outs[0])
    p1.close()
    p2.close()
    ctx.close()


def test_plan_rejects_bad_arguments():
    import torch
    from paper_2306_07191_amd import nif
    w = _multi_tiny(n_objects=2, n_rays=1000)
    ctx, _ = make_pair(w, grid_amp=0.5)
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    with pytest.raises(nif.NifError):  # not prepared
        nif.Plan(ctx, rays, ids, tmax, dtype="bf16")
    ctx.prepare("bf16")
    with pytest.raises(nif.NifError):
        nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning='{"order": 5, "blocks_per_cu": 4}')
    with pytest.raises(nif.NifError):
        nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning='{"blocks_per_cu": 4}')


def test_plan_refuses_a_changed_context():
    """A captured plan is refused (NIF_ERR_STATE, on the host, before any kernel)
    once the context changed in a way its graph cannot follow: a new query-image
    mode (whose old buffers the caller may free), a re-registered object, or
    weights changed since the last nif_prepare.  After nif_prepare alone it
    launches again; after the others a new plan gives the eager outputs."""
    import torch
    from paper_2306_07191_amd import nif
    sh = S.ModelShape(levels=4, res_min=4, res_max=32, feats=2, hidden=3, width=64, grid_dtype="f16")
    w = _multi_tiny(n_objects=3, n_rays=20000)
    w["shape"] = sh
    ctx, _ = make_pair(w, grid_amp=0.5)
    ctx.prepare("bf16")
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    sched = '{"order": 1, "blocks_per_cu": 4}'
    plan = nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning=sched)
    plan.launch()
    y0 = ctx.query(rays, ids, tmax, dtype="bf16")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(plan.out.cpu().numpy(), y0.cpu().numpy())
    # weights re-registered: refused until nif_prepare, then the same outputs
    ctx.set_mlp(0, ctx.mlps[0])
    with pytest.raises(nif.NifError) as e:
        plan.launch()
    assert e.value.status == -5
    ctx.prepare("bf16")
    plan.out.zero_()
    plan.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(plan.out.cpu().numpy(), y0.cpu().numpy())
    # another image mode: the captured graph read the old images
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 2)
    ctx.prepare("bf16")
    with pytest.raises(nif.NifError) as e:
        plan.launch()
    assert e.value.status == -5
    # an object registered again
    plan2 = nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning=sched)
    ctx.set_object(1, w["aabb"][1], ctx.grids[1], int(w["mlp_index"][1]))
    ctx.prepare("bf16")
    with pytest.raises(nif.NifError) as e:
        plan2.launch()
    assert e.value.status == -5
    plan3 = nif.Plan(ctx, rays, ids, tmax, dtype="bf16", tuning=sched)
    plan3.launch()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(plan3.out.cpu().numpy(), y0.cpu().numpy())
    for p in (plan, plan2, plan3):
        p.close()
