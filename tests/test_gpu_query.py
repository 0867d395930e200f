"""Parity of the HIP query path (nif_query through the C ABI) with the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

from gpu_util import GRID_SEED, check_outputs, fp8_scales_from_oracle, make_pair, run_query

pytestmark = pytest.mark.gpu


def test_init_grid_bit_exact():
    import torch
    for sh in (S.TINY, S.FRAME):
        w = dict(shape=sh, aabb=np.array([[0, 0, 0, 1, 1, 1]], np.float32), mlps=np.zeros((1, sh.mlp_params), np.float32),
                 mlp_index=np.zeros(1, np.int32))
        ctx, _ = make_pair(w, grid_amp=1e-4)
        g = ctx.grids[0]
        torch.cuda.synchronize()
        for begin in (0, 1, 12345, ctx.grid_elems - 999):
            cnt = min(999, ctx.grid_elems - begin)
            ref = O.init_grid(GRID_SEED, 0, 1e-4, sh.grid_dtype, cnt, begin)
            got = g[begin:begin + cnt].cpu().numpy()
            got = got.view(np.uint16) if sh.grid_dtype == "f16" else got
            np.testing.assert_array_equal(got, ref)
        del ctx, g
        torch.cuda.empty_cache()


@pytest.mark.parametrize("amp,gain", [(1e-4, 1.0), (1.0, 1.0), (0.5, 2.0)])
def test_query_f32_tiny(amp, gain):
    w = S.tiny_workload()
    w["mlps"] = (w["mlps"].astype(np.float64) * gain).astype(np.float32)
    ctx, model = make_pair(w, grid_amp=amp)
    ref = model.forward(w["rays"], w["ids"], w["tmax"])
    y, z = run_query(ctx, w, "f32")
    st = check_outputs(y, z, ref, "f32", f"tiny amp={amp}")
    print("f32 tiny", amp, gain, st)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("amp", [1e-4, 1.0])
def test_query_lowp_tiny(dtype, amp):
    w = S.tiny_workload()
    ctx, model = make_pair(w, grid_amp=amp)
    ref_x = model.forward(w["rays"], w["ids"], w["tmax"])
    ref_q = model.with_(quant=dtype).forward(w["rays"], w["ids"], w["tmax"])
    y, z = run_query(ctx, w, dtype)
    st = check_outputs(y, z, ref_q, dtype, f"tiny {dtype} amp={amp}", exact=ref_x)
    print(dtype, "tiny", amp, st)


@pytest.mark.parametrize("amp", [1e-4, 1.0])
def test_query_fp8_tiny(amp):
    w = S.tiny_workload()
    model = O.Model(w["shape"], w["aabb"], w["mlps"], grid_seed=GRID_SEED, grid_amp=amp)
    scales = fp8_scales_from_oracle(model, w)
    ctx, model_q = make_pair(w, grid_amp=amp, quant="fp8", fp8_scales=scales)
    ref_q = model_q.forward(w["rays"], w["ids"], w["tmax"])
    ref_x = model.forward(w["rays"], w["ids"], w["tmax"])
    y, z = run_query(ctx, w, "fp8")
    st = check_outputs(y, z, ref_q, "fp8", f"tiny fp8 amp={amp}", exact=ref_x)
    print("fp8 tiny", amp, st)


@pytest.mark.parametrize("n", [1, 31, 32, 129, 1000, 4097])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_query_ragged_sizes(n, dtype):
    w = S.tiny_workload(n_rays=n)
    ctx, model = make_pair(w, grid_amp=1.0)
    ref = model.with_(quant="exact" if dtype == "f32" else dtype).forward(w["rays"], w["ids"], w["tmax"])
    y, z = run_query(ctx, w, dtype)
    check_outputs(y, z, ref, dtype, f"n={n}")


def test_query_empty_and_errors():
    import torch
    from paper_2306_07191_amd import nif
    w = S.tiny_workload(n_rays=64)
    ctx, _ = make_pair(w, grid_amp=1.0)
    ctx.prepare("f32")
    e = torch.empty(0, device="cuda")
    ctx.query(e.reshape(0, 6), torch.empty(0, dtype=torch.int32, device="cuda"), e, "f32")  # n = 0: no-op
    with pytest.raises(nif.NifError) as ei:
        ctx.query(torch.zeros(64, 6, device="cuda"), torch.zeros(64, dtype=torch.int32, device="cuda"),
                  torch.zeros(64, device="cuda"), "bf16")  # not prepared for bf16
    assert ei.value.status == -5


def test_query_invalid_inputs():
    from paper_2306_07191_amd import nif
    w = S.tiny_workload(n_rays=300)
    rays, tmax, ids = w["rays"], w["tmax"], w["ids"]
    rays[0, 0] = np.nan
    rays[1, 3:] = 0
    tmax[2] = -1.0
    ids[3] = 7
    ids[4] = -1
    rays[5, :3] = [10, 10, 10]
    rays[5, 3:] = [0, 1, 0]
    tmax[6] = 1e-3  # segment ends before the box
    rays[7, 3:] = [0, 0, np.inf]
    ctx, model = make_pair(w, grid_amp=1.0)
    for dtype in ("f32", "bf16"):
        ref = model.with_(quant="exact" if dtype == "f32" else dtype).forward(rays, ids, tmax)
        assert list(ref["status"][:8]) == [-1, -1, -1, -1, -1, 0, 0, -1]
        y, z = run_query(ctx, w, dtype)
        check_outputs(y, z, ref, dtype, "invalid")
        # the context's error word has both kinds of domain error, then clears
        assert ctx.error_flags() == nif.NIF_FLAG_INVALID_RAY | nif.NIF_FLAG_BAD_OBJECT
        assert ctx.error_flags() == 0
    w2 = S.tiny_workload(n_rays=300)
    w2["ids"][9] = 3
    run_query(ctx, w2, "f32")
    assert ctx.error_flags() == nif.NIF_FLAG_BAD_OBJECT


def test_query_multi_object_multi_mlp():
    """Several objects sharing three MLPs, ids shuffled: every wave mixes MLPs."""
    g = np.random.default_rng(5)
    K, M = 6, 3
    boxes = []
    for k in range(K):
        c = g.uniform(-5, 5, 3)
        h = g.uniform(0.3, 1.5, 3)
        boxes.append(np.concatenate([c - h, c + h]))
    boxes = np.array(boxes, np.float32)
    n = 5000
    ids = g.integers(0, K, n).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.empty(n, np.float32)
    for k in range(K):
        s = np.nonzero(ids == k)[0]
        ctr = 0.5 * (boxes[k, :3] + boxes[k, 3:])
        r, t = S.rays_sphere_to_box(s.size, boxes[k], g, radius=4.0, center=ctr)
        rays[s], tmax[s] = r, t
    mlps = np.stack([S.xavier_mlp(S.TINY, S.rng(99, 3, m)) for m in range(M)])
    w = dict(shape=S.TINY, aabb=boxes, mlps=mlps, mlp_index=np.array([0, 1, 2, 0, 1, 2], np.int32),
             rays=rays, tmax=tmax, ids=ids)
    ctx, model = make_pair(w, grid_amp=1.0)
    for dtype in ("f32", "bf16"):
        ref = model.with_(quant="exact" if dtype == "f32" else dtype).forward(rays, ids, tmax)
        y, z = run_query(ctx, w, dtype)
        check_outputs(y, z, ref, dtype, f"multi {dtype}")


@pytest.mark.parametrize("amp", [1e-4, 0.5])
def test_query_frame_full_size_sampled(amp):
    """Frame workload at full size (1920 x 1080 rays, 8 levels 16..512, binary16
    latents, 2.1 GB grid) in the bench's launch configuration; sampled outputs
    checked against the oracle (which regenerates latents lazily)."""
    import torch
    w = S.frame_workload(with_mesh=False)
    ctx, model = make_pair(w, grid_amp=amp)
    sel = np.sort(np.random.default_rng(0).choice(w["ids"].shape[0], 3000, replace=False))
    sel = np.concatenate([sel, np.arange(w["ids"].shape[0] - 40, w["ids"].shape[0])])  # ragged tail
    rays, ids, tmax = w["rays"][sel], w["ids"][sel], w["tmax"][sel]
    scales = fp8_scales_from_oracle(model, dict(w, rays=rays, ids=ids, tmax=tmax))
    for m in range(1):
        ctx.set_fp8_scales(m, scales[m])
    exact = model.forward(rays, ids, tmax)
    for dtype in ("f32", "bf16", "f16", "fp8"):
        mq = model.with_(quant="exact" if dtype == "f32" else dtype, fp8_scales=scales if dtype == "fp8" else None)
        ref = exact if dtype == "f32" else mq.forward(rays, ids, tmax)
        y, z = run_query(ctx, w, dtype, sel=sel)
        st = check_outputs(y, z, ref, dtype, f"frame {dtype} amp={amp}", exact=exact)
        print("frame", dtype, amp, st)
    del ctx
    torch.cuda.empty_cache()


def _binary64_case(name):
    """(workload, sampled query indices or None): all 16,384 tiny queries, or
    3,000 frame queries plus the last 40 (the frame's 2.1 GB grid is regenerated
    lazily by the oracle)."""
    if name == "tiny":
        return S.tiny_workload(), None
    w = S.frame_workload(with_mesh=False)
    sel = np.sort(np.random.default_rng(1).choice(w["ids"].shape[0], 3000, replace=False))
    return w, np.concatenate([sel, np.arange(w["ids"].shape[0] - 40, w["ids"].shape[0])])


def _sub(w, sel):
    return (w["rays"], w["ids"], w["tmax"]) if sel is None else (w["rays"][sel], w["ids"][sel], w["tmax"][sel])


@pytest.mark.parametrize("name", ["tiny", "frame"])
def test_query_f32_vs_binary64_at_init(name):
    """The binary32 path against the binary64 oracle with clip, normalisation
    and cell coordinates in binary64 too (no step in binary32), at the paper's
    initialisation (latents U(-1e-4, 1e-4), Sec. 5 "Initialization"): every
    query within 1e-5 relative of y64, the stated tolerance of the binary32
    path."""
    import torch
    w, sel = _binary64_case(name)
    ctx, _ = make_pair(w, grid_amp=1e-4)
    m64 = O.Model(w["shape"], w["aabb"], w["mlps"], mlp_index=w["mlp_index"], grid_seed=GRID_SEED, grid_amp=1e-4,
                  coord_mode=1)
    ref = m64.forward(*_sub(w, sel))
    y, z = run_query(ctx, w, "f32", sel=sel)
    hit = ref["status"] == 1
    assert hit.sum() > 0.5 * hit.size
    assert (y[~hit] == 1.0).all() and np.isfinite(y[hit]).all()
    rel = np.abs(y[hit] - ref["y"][hit]) / ref["y"][hit]
    print(f"{name}: {hit.sum()} queries, f32 vs binary64 max rel {rel.max():.3e}, p99.9 {np.percentile(rel, 99.9):.3e}")
    assert (rel <= 1e-5).all(), rel.max()
    del ctx
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["tiny", "frame"])
@pytest.mark.parametrize("amp", [0.5, 1.0])
def test_error_split_vs_binary64(name, amp):
    """Latents U(-amp, amp), where the logits span a useful range: the error of
    every dtype against the binary64 oracle (binary64 coordinates), next to the
    part a correct binary32 clip and cell-coordinate step contributes by itself
    (the oracle run with those steps in binary32).  The binary32 path is no
    further from binary64 than that part plus the stated 1e-5 relative."""
    import torch
    w, sel = _binary64_case(name)
    ctx, model = make_pair(w, grid_amp=amp)
    q = _sub(w, sel)
    m64 = model.with_(coord_mode=1)
    ref64 = m64.forward(*q)
    ref32c = model.forward(*q)  # binary32 clip and cell coordinates, binary64 otherwise
    hit = (ref64["status"] == 1) & (ref32c["status"] == 1)
    split = np.abs(ref32c["y"][hit] - ref64["y"][hit])
    scales = fp8_scales_from_oracle(model, dict(w, rays=q[0], ids=q[1], tmax=q[2]))
    ctx.set_fp8_scales(0, scales[0])
    rows = {"binary32 coordinates (oracle)": split}
    for dtype in ("f32", "f16", "bf16", "fp8"):
        y, _ = run_query(ctx, w, dtype, sel=sel)
        dy = np.abs(y[hit] - ref64["y"][hit])
        rows[dtype] = dy
        if dtype == "f32":
            assert (dy <= split + 1e-5 * ref64["y"][hit]).all(), (dy - split).max()
    for k, v in rows.items():
        print(f"{name} amp={amp} {k:>30}: |y - y64| max {v.max():.3e}, p99.9 {np.percentile(v, 99.9):.3e}, "
              f"median {np.median(v):.3e}")
    del ctx
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_ordering_is_transparent(dtype):
    """Queries bucket-sorted by (object, entry-point Morton code) before the kernel give
    bit-identical outputs to the unordered launch: each query is computed on its own."""
    import torch
    from paper_2306_07191_amd import nif
    g = np.random.default_rng(9)
    K = 3
    boxes = np.array([[-1, -1, -1, 1, 1, 1], [2, 0, 0, 3, 1, 2], [-4, -3, 0, -2, -1, 1]], np.float32)
    n = 70000
    ids = g.integers(0, K, n).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.empty(n, np.float32)
    for k in range(K):
        s = np.nonzero(ids == k)[0]
        ctr = 0.5 * (boxes[k, :3] + boxes[k, 3:])
        r, tt = S.rays_sphere_to_box(s.size, boxes[k], g, radius=4.0, center=ctr)
        rays[s], tmax[s] = r, tt
    rays[::97, 3:] = -rays[::97, 3:]  # some misses
    ids[::1001] = 9                   # some invalid ids
    mlps = np.stack([S.xavier_mlp(S.TINY, S.rng(98, 3, m)) for m in range(2)])
    w = dict(shape=S.TINY, aabb=boxes, mlps=mlps, mlp_index=np.array([0, 1, 0], np.int32), rays=rays, tmax=tmax, ids=ids)
    scales = np.ones((2, 2 * S.TINY.hidden)) * 0.01 if dtype == "fp8" else None
    ctx, model = make_pair(w, grid_amp=1.0, quant="exact" if dtype == "f32" else dtype, fp8_scales=scales)
    outs = []
    for mode in (0, 1):
        ctx.set_option(nif.NIF_OPT_ORDER, mode)
        outs.append(run_query(ctx, w, dtype))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    ref = model.forward(rays, ids, tmax)
    exact = model.with_(quant="exact").forward(rays, ids, tmax) if dtype != "f32" else None
    check_outputs(outs[1][0], outs[1][1], ref, dtype, f"ordered {dtype}", exact=exact)


def test_order_is_a_grouped_permutation():
    import torch
    from paper_2306_07191_amd import nif
    g = np.random.default_rng(13)
    K, n = 5, 50000
    boxes = np.array([[k * 3.0, 0, 0, k * 3.0 + 2, 1, 1] for k in range(K)], np.float32)
    ids = g.integers(0, K, n).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.empty(n, np.float32)
    for k in range(K):
        s = np.nonzero(ids == k)[0]
        r, tt = S.rays_sphere_to_box(s.size, boxes[k], g, radius=3.0, center=0.5 * (boxes[k, :3] + boxes[k, 3:]))
        rays[s], tmax[s] = r, tt
    rays[::50, 3:] = -rays[::50, 3:]
    ids[::777] = -3
    w = dict(shape=S.TINY, aabb=boxes, mlps=S.xavier_mlp(S.TINY, S.rng(1, 3))[None], mlp_index=np.zeros(K, np.int32),
             rays=rays, tmax=tmax, ids=ids)
    ctx, model = make_pair(w, grid_amp=1.0)
    ctx.prepare("f32")
    perm = ctx.order(*(torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))).cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(n))  # a permutation
    st = model.forward(rays, ids, tmax)["status"]
    hit = st[perm] == 1
    nh = hit.sum()
    assert hit[:nh].all() and not hit[nh:].any()       # misses and invalid queries last
    assert (np.diff(ids[perm[:nh]]) >= 0).all()          # grouped by object


def test_packed_query_records():
    """The ordering pass can also store every query as one 32-byte record
    (row i = query i, bit for bit); the query on the records through the order
    (nif_query with ordering reads them internally) gives the outputs of the
    unordered query, with and without a query image (bucket order alone, or
    bucket order and the window sort)."""
    import torch
    from paper_2306_07191_amd import nif
    n = 40000
    w = S.frame_workload(n_rays=n, with_mesh=False)
    w["rays"][::89, 3:] *= -1.0     # misses
    w["tmax"][::1003] = np.nan      # invalid queries
    w["ids"][::2001] = 5            # object id out of range
    ctx, model = make_pair(w, grid_amp=0.5)
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    ctx.set_option(nif.NIF_OPT_ORDER, 0)
    base = {dt: run_query(ctx, w, dt) for dt in ("f32", "bf16")}
    check_outputs(*base["f32"], model.forward(w["rays"], w["ids"], w["tmax"]), "f32", "unordered f32")
    expect = np.concatenate([w["rays"], w["tmax"][:, None], w["ids"].view(np.float32)[:, None]], axis=1)
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    for img in (0, 1, 2):
        ctx.set_option(nif.NIF_OPT_GRID_IMAGE, img)
        for dt in ("f32", "bf16"):
            got = run_query(ctx, w, dt)
            np.testing.assert_array_equal(got[0], base[dt][0])
            np.testing.assert_array_equal(got[1], base[dt][1])
        ctx.prepare("bf16")
        perm, rec = ctx.order_packed(rays, ids, tmax)
        p = perm.cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(np.sort(p), np.arange(n))
        np.testing.assert_array_equal(rec.cpu().numpy().view(np.uint32), expect.view(np.uint32))
        y = ctx.query_packed(rec, perm, dtype="bf16")
        torch.cuda.synchronize()
        np.testing.assert_array_equal(y.cpu().numpy().astype(np.float64), base["bf16"][0])
    bad = torch.empty(8 * n + 1, dtype=torch.float32, device="cuda")[1:]  # 4-byte offset
    with pytest.raises(nif.NifError):
        ctx.order_packed(rays, ids, tmax, packed=bad)


def test_gpu_bvh_labels_match_oracle():
    """GPU BVH any-hit (binary32 watertight test): every label equal to the
    oracle's binary32 test over all triangles (the decision is taken in the
    kernel's precision on both sides); agreement with the exact binary64
    labels reported and bounded."""
    import torch
    from oracle import oracle as O
    from paper_2306_07191_amd import nif
    w = S.tiny_workload()
    w["tmax"] = np.where(np.arange(w["tmax"].size) % 3 == 0, 3.0, w["tmax"]).astype(np.float32)
    ref32, _ = O.trace_brute32(w["tris"], w["rays"], w["tmax"])
    ref64 = O.anyhit_brute(w["tris"], w["rays"], w["tmax"])
    bvh = nif.BVH(w["tris"])
    got = bvh.anyhit(torch.from_numpy(w["rays"]).cuda(), torch.from_numpy(w["tmax"]).cuda()).cpu().numpy()
    print("tiny labels: binary32 oracle mismatches", int((got != ref32).sum()), "binary64 agreement",
          (got == ref64).mean(), "visible", ref64.mean())
    np.testing.assert_array_equal(got, ref32)
    assert (got == ref64).mean() >= 0.9999
    # frame mesh, a sample of frame rays against the oracle BVH
    tris = S.frame_mesh()
    rays, tmax = S.rays_ground_to_light(20000, S.rng(2, 1))
    ob = O.BVH(tris)
    ref32, _ = ob.trace32(rays, tmax)
    ref64 = ob.anyhit(rays, tmax)
    bvh2 = nif.BVH(tris)
    got = bvh2.anyhit(torch.from_numpy(rays).cuda(), torch.from_numpy(tmax).cuda()).cpu().numpy()
    print("frame labels: binary32 oracle mismatches", int((got != ref32).sum()), "binary64 agreement",
          (got == ref64).mean(), "visible", ref64.mean(), "nodes", bvh2.num_nodes)
    np.testing.assert_array_equal(got, ref32)
    assert (got == ref64).mean() >= 0.9999
    empty = nif.BVH(np.zeros((0, 9), np.float32))
    assert (empty.anyhit(torch.from_numpy(rays).cuda(), torch.from_numpy(tmax).cuda()).cpu().numpy() == 1).all()


def test_grid_image_is_bit_identical():
    """NIF_OPT_GRID_IMAGE gathers from the y-pair image: same lookups, same
    interpolation order, so features and outputs are bit-identical; it is rebuilt
    by nif_prepare after the grid changes."""
    import torch
    from paper_2306_07191_amd import nif
    w = S.frame_workload(n_rays=30000, with_mesh=False)
    ctx, model = make_pair(w, grid_amp=0.5)
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    outs = {}
    for img in (0, 1, 2):
        ctx.set_option(nif.NIF_OPT_GRID_IMAGE, img)
        for dtype in ("f32", "bf16"):
            outs[img, dtype] = run_query(ctx, w, dtype)
        ctx.prepare("f32")
        outs[img, "x"] = ctx.encode(rays, ids, tmax)[0].cpu().numpy()
    for img in (1, 2):
        for key in ("f32", "bf16", "x"):
            np.testing.assert_array_equal(outs[0, key][0] if key != "x" else outs[0, key],
                                          outs[img, key][0] if key != "x" else outs[img, key])
    check_outputs(*outs[1, "f32"], model.forward(w["rays"], w["ids"], w["tmax"]), "f32", "image f32")
    # a changed grid is seen after nif_prepare
    ctx.init_grid(0, GRID_SEED + 1, 0.5)
    y_img = run_query(ctx, w, "f32")
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    np.testing.assert_array_equal(y_img[0], run_query(ctx, w, "f32")[0])
    with pytest.raises(nif.NifError):  # binary32 grids have no image form
        c2, _ = make_pair(S.tiny_workload(n_rays=10), grid_amp=0.5)
        c2.set_option(nif.NIF_OPT_GRID_IMAGE, 1)


def _order_coarse_offset(n: int, num_objects: int) -> int:
    """Byte offset of the bucket order inside the ordering workspace, as the
    library lays it out: count table (buckets x tiles), bucket totals, 16-bit
    keys, fine keys, then the bucket order; each region 256-byte aligned."""
    al = lambda b: (b + 255) // 256 * 256
    bits = 4
    while bits > 0 and (num_objects << (3 * bits)) > 4096:
        bits -= 1
    nb = (num_objects << (3 * bits)) + 1
    tiles = (n + 8191) // 8192
    return al(nb * tiles * 4) + al(nb * 4) + al(n * 2) + al(n * 4)


def test_window_sort_orders_each_window_stably():
    """The ordering's window sort: each window of 4,096 consecutive entries of
    the bucket order is re-sorted, stably, by the finer key (the Morton code of
    the binary32 entry point with 8 bits per axis, for one object); it permutes
    entries only within their window.  The bucket order ranks a tile's queries
    of one bucket with LDS atomics, so it can differ from call to call: the
    window sort is compared with the bucket order of the same call, which the
    workspace still holds, and with a separate call only through what is fixed
    (each window's bucket counts)."""
    import torch
    from paper_2306_07191_amd import nif
    n, win = 20000, 4096
    w = S.frame_workload(n_rays=n, with_mesh=False)
    w["rays"][::97, 3:] *= -1.0  # misses
    w["rays"][1000:1400] = w["rays"][1000]  # identical queries: equal keys
    w["tmax"][1000:1400] = w["tmax"][1000]
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    ctx.prepare("f32")
    args = [torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax")]
    ctx.set_option(nif.NIF_OPT_WINDOW_SORT, 0)
    other = ctx.order(*args).cpu().numpy().astype(np.int64)
    ctx.set_option(nif.NIF_OPT_WINDOW_SORT, 1)
    ws = torch.empty(int(nif.lib().nif_order_workspace_bytes(ctx.h, n)), dtype=torch.uint8, device="cuda")
    fine = ctx.order(*args, ws=ws).cpu().numpy().astype(np.int64)
    off = _order_coarse_offset(n, 1)
    coarse = ws[off:off + 4 * n].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(np.sort(coarse), np.arange(n)) and np.array_equal(np.sort(fine), np.arange(n))

    def spread3(v):
        r = np.zeros_like(v)
        for b in range(10):
            r |= ((v >> b) & 1) << (3 * b)
        return r

    key = np.full(n, 0xFFFFFFFF, np.int64)
    bucket = np.full(n, 4096, np.int64)
    for i in range(n):
        st, u, *_ = model.detail(w["rays"][i], 0, float(w["tmax"][i]))
        if st == 1:
            c = np.minimum((np.float32(u[0]) * np.float32(256)).astype(np.int64), 255)
            key[i] = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2)
            bucket[i] = key[i] >> 12
    assert (np.diff(bucket[coarse]) >= 0).all() and (np.diff(bucket[other]) >= 0).all()
    ties = 0
    for w0 in range(0, n, win):
        a, b, o = coarse[w0:w0 + win], fine[w0:w0 + win], other[w0:w0 + win]
        assert np.array_equal(np.sort(a), np.sort(b))           # the same entries
        assert np.array_equal(np.sort(bucket[o]), np.sort(bucket[b]))
        kb = key[b]
        assert (np.diff(kb) >= 0).all()                          # sorted by the finer key
        pos = {q: j for j, q in enumerate(a.tolist())}           # stable: ties keep the bucket order
        for k in np.unique(kb):
            same = b[kb == k]
            ties += same.shape[0] - 1
            assert (np.diff([pos[q] for q in same.tolist()]) > 0).all()
    assert ties >= 399


def test_concurrent_calls_on_streams():
    """The fused kernel's blocks take their tiles from per-XCD counters: in the
    caller's workspace for nif_query, from the context's ring of counter blocks
    for nif_query_packed.  Calls in flight together on several streams, with
    several launches per stream, each give the outputs of one call alone, bit
    for bit, and the reference's within the binary32 tolerance."""
    import torch
    from paper_2306_07191_amd import nif
    w = S.frame_workload(n_rays=300000, with_mesh=False)
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    ctx.prepare("f32")
    rays, ids, tmax = (torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in ("rays", "ids", "tmax"))
    n = ids.shape[0]
    alone_z = torch.empty(n, device="cuda")
    alone = ctx.query(rays, ids, tmax, dtype="f32", logits=alone_z)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    recs = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    ows = torch.empty(int(nif.lib().nif_order_workspace_bytes(ctx.h, n)), dtype=torch.uint8, device="cuda")
    ctx.order_packed(rays, ids, tmax, perm=perm, packed=recs, ws=ows)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(4)]
    outs_p = [[torch.full((n,), -1.0, device="cuda") for _ in range(3)] for _ in streams]
    outs_q = [torch.full((n,), -1.0, device="cuda") for _ in streams]
    wss = [torch.empty(int(nif.lib().nif_workspace_bytes(ctx.h, n, 0)), dtype=torch.uint8, device="cuda")
           for _ in streams]
    for si, st in enumerate(streams):
        with torch.cuda.stream(st):
            for o in outs_p[si]:
                ctx.query_packed(recs, perm, dtype="f32", out=o)
            ctx.query(rays, ids, tmax, dtype="f32", out=outs_q[si], ws=wss[si])
    torch.cuda.synchronize()
    for si in range(len(streams)):
        for o in outs_p[si] + [outs_q[si]]:
            assert torch.equal(o, alone)
    check_outputs(alone.cpu().numpy(), alone_z.cpu().numpy(), model.forward(w["rays"], w["ids"], w["tmax"]), "f32",
                  "concurrent")


@pytest.mark.parametrize("dtype", ["f16", "fp8"])
def test_tile_shape_1_many_objects(dtype):
    """Blocks reload their LDS weights when their next tile starts another
    object: with 16 objects of their own MLPs and ordered queries (blocks cross
    object boundaries often), tile shape 1 gives outputs bit-identical to shape
    0 and within the reduced-precision criteria of the oracle, through
    nif_query (tile counters in the workspace) and nif_query_packed (the
    context's ring, launched three times)."""
    import torch
    from paper_2306_07191_amd import nif
    K, n = 16, 120000
    w = S.multi_workload(n_objects=K, n_rays=n)
    w["shape"] = S.FRAME
    w["mlps"] = np.stack([S.xavier_mlp(S.FRAME, S.rng(71, 3, k)) for k in range(K)])
    w["mlp_index"] = np.arange(K, dtype=np.int32)
    scales = None
    if dtype == "fp8":
        exact0 = O.Model(w["shape"], w["aabb"], w["mlps"], mlp_index=w["mlp_index"], grid_seed=GRID_SEED, grid_amp=0.5)
        scales = fp8_scales_from_oracle(exact0, w, n_cal=n)
    ctx, model = make_pair(w, grid_amp=0.5, quant=dtype, fp8_scales=scales)
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    outs = {}
    for shape in (0, 1):
        ctx.set_option(nif.NIF_OPT_TILE_SHAPE, shape)
        outs[shape] = run_query(ctx, w, dtype)
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    rays, ids, tmax = (torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in ("rays", "ids", "tmax"))
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    recs = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    ows = torch.empty(int(nif.lib().nif_order_workspace_bytes(ctx.h, n)), dtype=torch.uint8, device="cuda")
    ctx.order_packed(rays, ids, tmax, perm=perm, packed=recs, ws=ows)
    for _ in range(3):  # the ring's blocks are left at zero by every launch
        y = ctx.query_packed(recs, perm, dtype=dtype)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(y.cpu().numpy().astype(np.float64), outs[1][0])
    ref = model.forward(w["rays"], w["ids"], w["tmax"])
    exact = model.with_(quant="exact").forward(w["rays"], w["ids"], w["tmax"])
    check_outputs(outs[1][0], outs[1][1], ref, dtype, f"shape 1 {dtype}", exact=exact)


def test_image_only_objects():
    """Objects answered from their query image alone: nif_build_image builds
    one object's image, nif_set_object without a grid keeps it and the grid
    buffer is released.  Queries (FP32 and BF16) give the grid path's outputs
    bit for bit, and the oracle's within the FP32 tolerance; nif_init_grid and
    training refuse the context; a grid given again brings the grid back."""
    import torch
    from paper_2306_07191_amd import nif
    n, K = 20000, 3
    w = S.frame_workload(n_rays=n, with_mesh=False)
    w["aabb"] = np.repeat(w["aabb"], K, axis=0)
    w["mlps"] = np.repeat(w["mlps"], K, axis=0)
    w["mlp_index"] = np.arange(K, dtype=np.int32)
    w["ids"] = np.random.default_rng(3).integers(0, K, n).astype(np.int32)
    w["ids"][::7] = 1
    ctx, model = make_pair(w, grid_amp=0.5)
    y_grid = {dt: run_query(ctx, w, dt) for dt in ("f32", "bf16")}
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 1)
    for k in range(K):
        ctx.build_image(k)
    torch.cuda.synchronize()
    for k in (0, 2):  # object 1 keeps its grid (its image is rebuilt by nif_prepare)
        ctx.drop_grid(k)
    torch.cuda.empty_cache()
    for dt in ("f32", "bf16"):
        y, z = run_query(ctx, w, dt)
        np.testing.assert_array_equal(y, y_grid[dt][0])
        np.testing.assert_array_equal(z, y_grid[dt][1])
    check_outputs(*run_query(ctx, w, "f32"), model.forward(w["rays"], w["ids"], w["tmax"]), "f32", "image only")
    with pytest.raises(nif.NifError) as e:
        ctx.init_grid(0, GRID_SEED, 0.5)
    assert e.value.status == nif.NIF_ERR_STATE
    rays, ids, tmax = (torch.from_numpy(w[k][:64]).cuda() for k in ("rays", "ids", "tmax"))
    with pytest.raises(nif.NifError) as e:
        ctx.train_step(rays, ids, tmax, torch.ones(64, dtype=torch.uint8, device="cuda"), step=1)
    assert e.value.status == nif.NIF_ERR_STATE
    # another image mode forgets the images: objects without a grid cannot be prepared
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    with pytest.raises(nif.NifError) as e:
        ctx.prepare("f32")
    assert e.value.status == nif.NIF_ERR_STATE
    # the paths that would read the grids through the last prepared object table refuse too
    with pytest.raises(nif.NifError) as e:
        ctx.encode(rays, ids, tmax)
    assert e.value.status == nif.NIF_ERR_STATE
    with pytest.raises(nif.NifError) as e:
        ctx.calibrate_fp8(rays, ids, tmax, mlp=0)
    assert e.value.status == nif.NIF_ERR_STATE
    for k in (0, 2):  # grids given again (same initial latents): the grid path's outputs
        ctx.set_object(k, w["aabb"][k], ctx.alloc_grid(), int(w["mlp_index"][k]))
        ctx.init_grid(k, GRID_SEED, 0.5)
    np.testing.assert_array_equal(run_query(ctx, w, "f32")[0], y_grid["f32"][0])


def test_order_bits_option_is_transparent():
    """NIF_OPT_ORDER_BITS caps the entry-point Morton bits of the ordering's
    bucket key (0: by object alone): the ordering is a permutation whose
    buckets follow the capped key, and nif_query's outputs are those of the
    automatic setting bit for bit, with and without the window sort."""
    import torch
    from paper_2306_07191_amd import nif
    K, n = 16, 60000
    w = S.multi_workload(n_objects=K, n_rays=n)
    w["shape"] = S.FRAME
    w["mlps"] = np.stack([S.xavier_mlp(S.FRAME, S.rng(71, 3, k)) for k in range(K)])
    w["mlp_index"] = np.arange(K, dtype=np.int32)
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_ORDER, 1)
    ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 0)
    ref = run_query(ctx, w, "bf16")
    rays, ids, tmax = (torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in ("rays", "ids", "tmax"))
    for ws in (0, 1):
        ctx.set_option(nif.NIF_OPT_WINDOW_SORT, ws)
        for bits in (0, 1, 3):
            ctx.set_option(nif.NIF_OPT_ORDER_BITS, bits)
            y, z = run_query(ctx, w, "bf16")
            np.testing.assert_array_equal(y, ref[0])
            np.testing.assert_array_equal(z, ref[1])
            perm = ctx.order(rays, ids, tmax).cpu().numpy().view(np.uint32).astype(np.int64)
            assert np.array_equal(np.sort(perm), np.arange(n))
            if bits == 0 and ws == 0:  # by object alone; misses and invalid queries last
                st = model.forward(w["rays"], w["ids"], w["tmax"])["status"]
                obj = np.where(st == 1, w["ids"], K)
                assert (np.diff(obj[perm]) >= 0).all()
    ctx.set_option(nif.NIF_OPT_ORDER_BITS, -1)
    with pytest.raises(nif.NifError):
        ctx.set_option(nif.NIF_OPT_ORDER_BITS, 5)
