"""The two stages of a query run separately (grid stage, inference stage), each
checked against the oracle."""
import numpy as np
import pytest

from paper_2306_07191_amd import synth as S

from gpu_util import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape_name", ["tiny", "frame_small"])
def test_encode_matches_oracle(shape_name):
    import torch
    if shape_name == "tiny":
        w = S.tiny_workload(n_rays=3000)
    else:
        w = S.frame_workload(n_rays=3000, with_mesh=False)
    amp = 0.5
    ctx, model = make_pair(w, grid_amp=amp)
    ctx.prepare("f32")
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    f, st = ctx.encode(rays, ids, tmax)
    torch.cuda.synchronize()
    f, st = f.cpu().numpy().astype(np.float64), st.cpu().numpy()
    ref = model.forward(w["rays"], w["ids"], w["tmax"], want_x=True)
    np.testing.assert_array_equal(st, ref["status"])
    hit = st == 1
    err = np.abs(f[hit] - ref["x"][hit])
    # binary32 interpolation of latents bounded by amp: a few rounding units of amp
    assert err.max() <= 1e-6 * amp, (err.max(), np.unravel_index(err.argmax(), err.shape))
    assert (f[~hit] == 0).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_mlp_matches_oracle(dtype):
    import torch
    w = S.tiny_workload(n_rays=2000)
    ctx, model = make_pair(w, grid_amp=0.5)
    g = np.random.default_rng(3)
    x = g.uniform(-1, 1, (2000, w["shape"].din)).astype(np.float32)
    ctx.prepare(dtype)
    z = ctx.mlp(torch.from_numpy(x).cuda(), dtype=dtype)
    torch.cuda.synchronize()
    z = z.cpu().numpy().astype(np.float64)
    mq = model.with_(quant="exact" if dtype == "f32" else dtype)
    r = mq.mlp_only(x.astype(np.float64), want_tol=True)
    zr = r["z"]
    err = np.abs(z - zr)
    print(dtype, "max err", err.max(), "median", np.median(err), "max err / ztol", (err / r["ztol"]).max())
    if dtype == "f32":
        assert (err <= 1e-5 * np.maximum(np.abs(zr), 1e-2)).all(), err.max()
    else:
        # emulated rounding: within the binary32-summation tolerance (plus one
        # quantum at flagged rounding decisions) for >= 99.9 %, and every query's
        # visibility within the propagated rounding bound of the unquantised result
        assert (err <= r["ztol"]).mean() >= 0.999, (err / r["ztol"]).max()
        ze = model.with_(quant="exact").mlp_only(x.astype(np.float64))
        dy = np.abs(1 / (1 + np.exp(-z)) - 1 / (1 + np.exp(-ze)))
        assert (dy <= r["ybound"]).all(), (dy / r["ybound"]).max()


@pytest.mark.parametrize("hidden", [1, 2])
def test_fp8_exact_when_representable(hidden):
    """FP8 with unit scales on operands that are E4M3 values whose products stay
    within a factor 2^3 of each other: no quantisation and no truncation inside
    the matrix core, so the result equals the exact one up to binary32 sums."""
    import torch
    from oracle import oracle as O
    from paper_2306_07191_amd import nif
    sh = S.ModelShape(levels=4, res_min=4, res_max=32, feats=2, hidden=hidden, width=64, grid_dtype="f32")
    g = np.random.default_rng(11)
    mant = np.array([1.0, 1.125, 1.25, 1.375, 1.5, 1.625, 1.75, 1.875])
    def e4m3_values(n, lo_exp, hi_exp):
        return g.choice(mant, n) * 2.0 ** g.integers(lo_exp, hi_exp + 1, n) * g.choice([-1.0, 1.0], n)
    P = sh.mlp_params
    W = np.zeros(P)
    n1 = sh.width * sh.din
    W[:n1] = e4m3_values(n1, -1, -1)  # [0.5, 1)
    off = n1
    for j in range(1, hidden):
        # second layer: powers of two only, so every product is exact and within range
        W[off: off + sh.width * sh.width] = 2.0 ** -7 * g.choice([-1.0, 1.0], sh.width * sh.width)
        off += sh.width * sh.width
    W[off:] = g.standard_normal(sh.width)
    x = e4m3_values(500 * sh.din, 0, 0).reshape(500, sh.din)  # [1, 2)
    w = dict(shape=sh, aabb=np.array([[0, 0, 0, 1, 1, 1]], np.float32), mlps=W[None].astype(np.float32),
             mlp_index=np.zeros(1, np.int32))
    ctx = nif.Context(sh)
    ctx.set_mlp(0, torch.from_numpy(W.astype(np.float32)).cuda())
    ctx.set_object(0, w["aabb"][0], ctx.alloc_grid(), 0)
    # unit scales except the input of layer 2 (s_x2 = 16): layer-1 outputs are exact
    # (multiples of 2^-7 below 96), a / 16 rounds identically on both sides, and the
    # layer-2 products (codes x 2^-7) stay within 2^11.6 of each other
    sc = np.array([1.0] * hidden + [1.0, 16.0][:hidden], np.float32)
    ctx.set_fp8_scales(0, sc)
    ctx.prepare("fp8")
    z = ctx.mlp(torch.from_numpy(x.astype(np.float32)).cuda(), dtype="fp8").cpu().numpy().astype(np.float64)
    m = O.Model(sh, w["aabb"], w["mlps"], quant="fp8", fp8_scales=sc.astype(np.float64)[None])
    zr = m.mlp_only(x)
    if hidden == 1:
        W32 = W.astype(np.float32).astype(np.float64)
        h = np.maximum(x @ W32[:n1].reshape(sh.width, sh.din).T, 0)
        np.testing.assert_allclose(zr, h @ W32[-sh.width:], rtol=1e-12, atol=1e-12)  # the oracle's emulation is exact here
    mag = np.abs(W[-sh.width:]).sum() * 200.0
    assert np.abs(z - zr).max() <= 64 * 2.0 ** -24 * mag, np.abs(z - zr).max()


@pytest.mark.parametrize("shape_name", ["tiny", "frame"])
def test_fp8_calibration_matches_oracle(shape_name):
    """nif_calibrate_fp8 (binary32 encode and layers) vs the oracle's binary64 maxima,
    on the calibration set of the frame scene (its first 65,536 queries)."""
    import torch
    if shape_name == "tiny":
        w = S.tiny_workload(n_rays=4096)
    else:
        w = S.frame_workload(n_rays=65536, with_mesh=False)
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    got = ctx.calibrate_fp8(rays, ids, tmax, mlp=0).astype(np.float64)
    ref = model.fp8_calibrate(w["rays"], w["ids"], w["tmax"], mlp=0)
    H = w["shape"].hidden
    # weight maxima are exact; activation maxima carry binary32 accumulation error
    np.testing.assert_array_equal(got[:H], ref[:H].astype(np.float32))
    np.testing.assert_allclose(got[H:], ref[H:], rtol=1e-5)
    # n = 0: unit activation scales
    e = torch.empty(0, device="cuda")
    got0 = ctx.calibrate_fp8(e.view(0, 6), e.int(), e, mlp=0)
    assert (got0[H:] == 1.0).all()


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("shape_name", ["tiny", "frame_small"])
def test_16bit_stages_match_fused_query(fmt, shape_name):
    """nif_encode16 stores the binary32 features rounded to nearest-even (bit
    patterns equal to torch's conversion of nif_encode's features), and nif_mlp16
    on them gives nif_query's logits bit for bit (the MLP rounds its input to
    the same format)."""
    import torch
    from paper_2306_07191_amd import nif
    w = S.tiny_workload(n_rays=3001) if shape_name == "tiny" else S.frame_workload(n_rays=3001, with_mesh=False)
    ctx, _ = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_ORDER, 0)
    ctx.prepare(fmt)
    rays, ids, tmax = (torch.from_numpy(w[k]).cuda() for k in ("rays", "ids", "tmax"))
    f32, st = ctx.encode(rays, ids, tmax)
    f16, st16 = ctx.encode16(rays, ids, tmax, fmt)
    tdt = torch.bfloat16 if fmt == "bf16" else torch.float16
    assert torch.equal(f16, f32.to(tdt).view(torch.int16))
    assert torch.equal(st, st16)
    z = ctx.mlp16(f16, fmt)
    zq = torch.empty_like(z)
    ctx.query(rays, ids, tmax, dtype=fmt, logits=zq)
    torch.cuda.synchronize()
    hit = (st == 1).cpu().numpy()
    np.testing.assert_array_equal(z.cpu().numpy()[hit], zq.cpu().numpy()[hit])
    with pytest.raises(nif.NifError):
        ctx.mlp16(f16, "f32")


def _hand_cases(q, fp8: bool):
    """(hidden, {(layer, row, col): weight}, w_out[0], x[0], scales or None, expected z):
    the hand-computed nets of the oracle's rounding-position pins, embedded in
    unit 0 of a 64-wide MLP whose other weights are zero."""
    e = 0.75 * q
    s2 = [1.0] * 4 if fp8 else None
    s1 = [1.0] * 2 if fp8 else None
    cases = [
        (2, {(0, 0, 0): 1.0, (1, 0, 0): 1.0}, 1.0, 1 + e, s2, 1 + q),            # input rounded
        (2, {(0, 0, 0): 1 + e, (1, 0, 0): 1.0}, 1.0, 1.0, s2, 1 + q),            # W1 rounded
        (2, {(0, 0, 0): 1.0, (1, 0, 0): 1 + e}, 1.0, 1.0, s2, 1 + q),            # W2 rounded
        (2, {(0, 0, 0): 1 + q, (1, 0, 0): 1 + q}, 1.0, 1 + q, s2, 1 + 3 * q + 2 * q * q),  # h1 rounded, h2 not
        (2, {(0, 0, 0): 1.0, (1, 0, 0): 1.0}, 1 + e, 1.0, s2, 1 + e),            # w_out binary32
        (1, {(0, 0, 0): 1 + q}, 1.0, 1 + q, s1, 1 + 2 * q + q * q),               # last activation not rounded
    ]
    if fp8:
        cases += [
            (1, {(0, 0, 0): 1.0}, 1.0, 1.0, [1.0, 0.75], 1.03125),                # s_x: 0.75 E4M3(1 / 0.75)
            (1, {(0, 0, 0): 1.0}, 1.0, 1.0, [0.75, 1.0], 1.03125),                # s_W
            (2, {(0, 0, 0): 1.0, (1, 0, 0): 1.0}, 1.0, 1.0, [1.0, 1.0, 1.0, 0.75], 1.03125),
            (1, {(0, 0, 0): 1.0}, 1.0, 500.0, [1.0, 1.0], 448.0),                # saturation
        ]
    return cases


@pytest.mark.parametrize("dtype,q", [("bf16", 2.0 ** -7), ("f16", 2.0 ** -10), ("fp8", 2.0 ** -3)])
def test_rounding_positions_hand_computed(dtype, q):
    """The reduced-precision MLP rounds its input, its hidden weights and every
    hidden activation except the last, and keeps the output layer in binary32:
    the hand-computed logits of the oracle's pins, bit for bit (every product
    and sum here is exact in binary32)."""
    import torch
    from paper_2306_07191_amd import nif
    for hidden, wts, wout, x0, scales, want in _hand_cases(q, dtype == "fp8"):
        sh = S.ModelShape(levels=4, res_min=4, res_max=32, feats=2, hidden=hidden, width=64, grid_dtype="f32")
        W = np.zeros(sh.mlp_params, np.float32)
        offs = [0, sh.width * sh.din]
        for (layer, r, c), v in wts.items():
            k = sh.din if layer == 0 else sh.width
            W[offs[layer] + r * k + c] = v
        W[sh.mlp_params - sh.width] = wout
        ctx = nif.Context(sh)
        ctx.set_mlp(0, torch.from_numpy(W).cuda())
        ctx.set_object(0, np.array([0, 0, 0, 1, 1, 1], np.float32), ctx.alloc_grid(), 0)
        if scales is not None:
            ctx.set_fp8_scales(0, np.asarray(scales, np.float32))
        ctx.prepare(dtype)
        x = np.zeros((33, sh.din), np.float32)
        x[:, 0] = x0
        z = ctx.mlp(torch.from_numpy(x).cuda(), dtype=dtype).cpu().numpy().astype(np.float64)
        assert (z == want).all(), (dtype, hidden, wts, wout, x0, scales, z[0], want)
        ctx.close()
