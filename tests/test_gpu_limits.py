"""The largest shapes the library accepts: 8 hidden layers (weight images above
64 KB of LDS), 4,096 objects (ordering with one bucket per object), and grids
of resolution 1024 (offsets past 2^32 bytes), each against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

from gpu_util import check_outputs, fp8_scales_from_oracle, make_pair, run_query

pytestmark = pytest.mark.gpu


def test_eight_hidden_layers_all_dtypes_and_gradients():
    import torch
    sh = S.ModelShape(levels=4, res_min=4, res_max=32, feats=2, hidden=8, width=64, grid_dtype="f32")
    w = S.tiny_workload(n_rays=6000)
    w["shape"] = sh
    w["mlps"] = (S.xavier_mlp(sh, S.rng(90, 3)) * 1.5).astype(np.float32)[None]
    ctx, model = make_pair(w, grid_amp=0.5)
    exact = model.forward(w["rays"], w["ids"], w["tmax"])
    for dtype in ("f32", "bf16", "f16"):
        ref = exact if dtype == "f32" else model.with_(quant=dtype).forward(w["rays"], w["ids"], w["tmax"])
        check_outputs(*run_query(ctx, w, dtype), ref, dtype, f"hidden 8 {dtype}", exact=exact)
    sc = fp8_scales_from_oracle(model, w)
    for m in range(sc.shape[0]):
        ctx.set_fp8_scales(m, sc[m])
    ref = model.with_(quant="fp8", fp8_scales=sc).forward(w["rays"], w["ids"], w["tmax"])
    check_outputs(*run_query(ctx, w, "fp8"), ref, "fp8", "hidden 8 fp8", exact=exact)
    # training gradients through all eight layers
    labels = O.BVH(w["tris"]).anyhit(w["rays"], w["tmax"])
    ctx.prepare("f32")
    ctx.setup_training()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    g = torch.zeros(ctx.mlp_params, device="cuda")
    ctx.train_step(t(w["rays"]), t(w["ids"]), t(w["tmax"]), t(labels), step=1, adam=None, mlp_grad=g)
    torch.cuda.synchronize()
    _, _, gW, _ = model.backward(w["rays"], w["ids"], w["tmax"], labels)
    err = np.linalg.norm(g.cpu().numpy() - gW[0]) / np.linalg.norm(gW[0])
    assert err < 1e-4, err


def test_4096_objects():
    K, n = 4096, 60000
    g = np.random.default_rng(17)
    lo = g.uniform(-50, 50, (K, 3))
    boxes = np.concatenate([lo, lo + g.uniform(0.5, 2.0, (K, 3))], axis=1).astype(np.float32)
    ids = g.integers(0, K, n).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.full(n, np.inf, np.float32)
    tgt = boxes[ids, :3] + g.uniform(size=(n, 3)) * (boxes[ids, 3:] - boxes[ids, :3])
    o = tgt + g.normal(size=(n, 3)) * 3
    rays[:, :3], rays[:, 3:] = o, tgt - o
    mlps = np.stack([S.xavier_mlp(S.TINY, S.rng(91, 3, m)) for m in range(4)])
    w = dict(shape=S.TINY, aabb=boxes, mlps=mlps, mlp_index=(np.arange(K) % 4).astype(np.int32), rays=rays,
             tmax=tmax, ids=ids)
    ctx, model = make_pair(w, grid_amp=0.5)
    from paper_2306_07191_amd import nif
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    ref = model.forward(rays, ids, tmax)
    assert (ref["status"] == 1).mean() > 0.9
    check_outputs(*run_query(ctx, w, "f32"), ref, "f32", "4096 objects")


def test_resolution_1024_sampled():
    """One object at 8 levels 64..1024 in binary16 (12.9 GB of latents): table and
    gather offsets beyond 2^32 bytes, through both image kinds and in place."""
    import torch
    from paper_2306_07191_amd import nif
    sh = S.ModelShape(levels=8, res_min=64, res_max=1024, feats=2, hidden=4, width=64, grid_dtype="f16")
    w = S.frame_workload(with_mesh=False, n_rays=200000)
    w["shape"] = sh
    ctx, model = make_pair(w, grid_amp=0.5)
    assert ctx.grid_elems * 2 > 2 ** 33
    sel = np.random.default_rng(2).choice(w["ids"].shape[0], 3000, replace=False)
    ref = model.forward(w["rays"][sel], w["ids"][sel], w["tmax"][sel])
    outs = []
    for img in (0, 1, 2):
        ctx.set_option(nif.NIF_OPT_GRID_IMAGE, img)
        y, z = run_query(ctx, w, "f32", sel=sel)
        check_outputs(y, z, ref, "f32", f"res 1024 image {img}")
        outs.append(y)
        ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)  # free the image before the next kind
        torch.cuda.empty_cache()
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
