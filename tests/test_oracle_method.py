"""Pins of the oracle's clip, encoding, MLP, gradient and Adam against closed
forms, invariants, hand-computed cases and finite differences."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

UNIT_BOX = np.array([[0, 0, 0, 1, 1, 1]], np.float32)


def shape(levels=4, res_min=4, res_max=32, feats=2, hidden=3, width=64, grid_dtype="f32"):
    return S.ModelShape(levels, res_min, res_max, feats, hidden, width, grid_dtype)


def zero_mlp(sh):
    return np.zeros((1, sh.mlp_params), np.float32)


# ---------------------------------------------------------------- levels

def test_level_progression():
    m = O.Model(S.TINY, UNIT_BOX, zero_mlp(S.TINY))
    r = m.level_res()
    assert r[0] == 4 and r[-1] == 32
    m2 = O.Model(S.FRAME, UNIT_BOX, zero_mlp(S.FRAME))
    r2 = m2.level_res().astype(np.float64)
    assert r2[0] == 16 and r2[-1] == 512 and (np.diff(r2) > 0).all()
    # a geometric progression up to rounding to integers: |N_l - N_min b^l| <= 1/2
    b = (512 / 16) ** (1 / 7)
    assert np.all(np.abs(r2 - 16 * b ** np.arange(8)) <= 0.5)
    one = O.Model(shape(levels=1, res_min=8, res_max=8), UNIT_BOX, zero_mlp(shape(levels=1, res_min=8, res_max=8)))
    assert list(one.level_res()) == [8]


def test_grid_sizes():
    m = O.Model(S.FRAME, UNIT_BOX, zero_mlp(S.FRAME))
    off = m.grid_offsets()
    res = m.level_res()
    per = ((res + 1) ** 3 * 2).astype(np.int64)
    assert off[-1] == 3 * per.sum()
    np.testing.assert_array_equal(np.diff(off), np.tile(per, 3))


# ---------------------------------------------------------------- clip

def _detail(m, o, d, tmax=np.inf):
    return m.detail(np.array(list(o) + list(d), np.float32), 0, tmax)


@pytest.mark.parametrize("mode", [0, 1])
def test_clip_axis_aligned(mode):
    m = O.Model(S.TINY, UNIT_BOX, zero_mlp(S.TINY), coord_mode=mode)
    st, u, *_ = _detail(m, (-5, 0.5, 0.25), (1, 0, 0))
    assert st == 1
    np.testing.assert_array_equal(u[0], [0, 0.5, 0.25])  # entry on the x = 0 face
    np.testing.assert_array_equal(u[1], [1, 0.5, 0.25])  # exit on the x = 1 face
    np.testing.assert_array_equal(u[2], [1, 0.5, 0.5])  # (d + 1) / 2
    # t_max cuts the segment inside the box: exit = o + t_max d
    st, u, *_ = _detail(m, (-5, 0.5, 0.25), (1, 0, 0), tmax=5.5)
    np.testing.assert_allclose(u[1], [0.5, 0.5, 0.25])
    # t_max before the box: miss
    st, *_ = _detail(m, (-5, 0.5, 0.25), (1, 0, 0), tmax=4.0)
    assert st == 0
    # box behind the origin: miss
    st, *_ = _detail(m, (-5, 0.5, 0.25), (-1, 0, 0))
    assert st == 0
    # parallel to a slab and outside it: miss; inside it: hit
    assert _detail(m, (-5, 2.0, 0.5), (1, 0, 0))[0] == 0
    assert _detail(m, (0.5, 0.5, -3), (0, 0, 1))[0] == 1


@pytest.mark.parametrize("mode", [0, 1])
def test_clip_origin_inside(mode):
    m = O.Model(S.TINY, UNIT_BOX, zero_mlp(S.TINY), coord_mode=mode)
    st, u, *_ = _detail(m, (0.25, 0.5, 0.75), (0, 1, 0))
    assert st == 1
    np.testing.assert_array_equal(u[0], [0.25, 0.5, 0.75])  # the origin is its own entry point
    np.testing.assert_array_equal(u[1], [0.25, 1.0, 0.75])


def test_clip_corner_ray():
    m = O.Model(S.TINY, UNIT_BOX, zero_mlp(S.TINY), coord_mode=1)
    d = np.array([1, 1, 1]) / np.sqrt(3)
    st, u, *_ = _detail(m, (-1, -1, -1), d)
    assert st == 1
    np.testing.assert_allclose(u[0], [0, 0, 0], atol=1e-7)
    np.testing.assert_allclose(u[1], [1, 1, 1], atol=1e-7)


def test_invalid_and_miss_outputs():
    w = S.tiny_workload(n_rays=8)
    m = O.Model(w["shape"], w["aabb"], w["mlps"], grid_seed=1)
    rays = w["rays"].copy()
    tmax = w["tmax"].copy()
    ids = w["ids"].copy()
    rays[0, 0] = np.nan          # non-finite origin
    rays[1, 3:] = 0              # zero direction
    tmax[2] = -1.0               # negative t_max
    ids[3] = 5                   # object id out of range
    rays[4, :3] = [10, 10, 10]   # aimed away from the box
    rays[4, 3:] = [0, 1, 0]
    out = m.forward(rays, ids, tmax)
    assert (out["status"][:4] == -1).all() and np.isnan(out["y"][:4]).all()
    assert out["status"][4] == 0 and out["y"][4] == 1.0
    assert (out["status"][5:] == 1).all()


def test_aliased_rays_encode_identically():
    """Sec. 2 / Sec. 3.1: moving the origin along d (outside the box) does not change
    the encoding.  Coordinates are dyadic so that o - k d lies exactly on the same line
    in binary32 (d is not unit length: t is measured in units of d)."""
    g = np.random.default_rng(3)
    n = 64
    gd = g.standard_normal((n, 3))
    o = np.round(3.0 * gd / np.linalg.norm(gd, axis=1, keepdims=True) * 64) / 64 + 0.5
    tgt = np.round(g.uniform(0, 1, (n, 3)) * 64) / 64
    d = tgt - o
    sh = S.TINY
    for mode, unit in [(1, 2.0 ** -53), (0, 2.0 ** -24)]:
        m = O.Model(sh, UNIT_BOX, S.xavier_mlp(sh, S.rng(7, 3))[None], grid_seed=1, grid_amp=1.0, coord_mode=mode)
        for k in (1, 2, 3):
            # the entry point o + t_a d carries rounding of order |o| units of the format
            tol = 16 * unit * (1 + np.abs(o - k * d).max())
            r1 = np.concatenate([o, d], axis=1).astype(np.float32)
            r2 = np.concatenate([o - k * d, d], axis=1).astype(np.float32)
            assert (r2[:, :3].astype(np.float64) == o - k * d).all()  # exact
            for i in range(n):
                s1, u1, x1, _, _ = m.detail(r1[i], 0, np.inf)
                s2, u2, x2, _, _ = m.detail(r2[i], 0, np.inf)
                assert s1 == 1 and s2 == 1
                np.testing.assert_allclose(u1, u2, atol=tol, rtol=0)
            a = m.forward(r1, np.zeros(n, np.int32), np.full(n, np.inf, np.float32))
            b = m.forward(r2, np.zeros(n, np.int32), np.full(n, np.inf, np.float32))
            if mode == 1:
                np.testing.assert_allclose(a["z"], b["z"], rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- encoding

def _vertex_grid(m, fn):
    """Grid whose value at vertex (ix, iy, iz) of table (e, l) is fn(e, l, f, ix/N, iy/N, iz/N, N)."""
    res = m.level_res()
    off = m.grid_offsets()
    F = m.shape.feats
    g = np.zeros(m.grid_elems, np.float64)
    for e in range(3):
        for l, N in enumerate(res):
            i = np.arange(N + 1)
            iz, iy, ix = np.meshgrid(i, i, i, indexing="ij")
            for f in range(F):
                vals = fn(e, l, f, ix / N, iy / N, iz / N, N)
                g[off[e * len(res) + l] + f: off[e * len(res) + l + 1]: F] = np.broadcast_to(vals, ix.shape).ravel()
    return g


def test_encoding_reproduces_affine_functions():
    """Trilinear interpolation is exact for affine functions of the vertex position:
    table values a.v + b give feature a.u + b at any u (pins weights, corner order, axis order)."""
    sh = S.TINY
    base = O.Model(sh, UNIT_BOX, zero_mlp(sh))
    coef = lambda e, l, f: (np.array([1.0, 2.0, 4.0]) * (1 + e) + f * np.array([0.5, -3.0, 0.25]), 0.125 * l - f)  # noqa
    def affine(e, l, f, x, y, z, N):
        a, b = coef(e, l, f)
        return a[0] * x + a[1] * y + a[2] * z + b
    g = _vertex_grid(base, affine)
    m = O.Model(sh, UNIT_BOX, zero_mlp(sh), grids=[g.astype(np.float32)], coord_mode=1)
    g_ = np.random.default_rng(8)
    o = g_.standard_normal((300, 3))
    o = 0.5 + 3 * o / np.linalg.norm(o, axis=1, keepdims=True)
    rays = np.concatenate([o, g_.uniform(0, 1, (300, 3)) - o], axis=1).astype(np.float32)
    for i in range(300):
        st, u, x, _, _ = m.detail(rays[i], 0, np.inf)
        if st != 1:
            continue
        for e in range(3):
            for l in range(sh.levels):
                for f in range(sh.feats):
                    a, b = coef(e, l, f)
                    ref = a @ u[e] + b
                    # table values are binary32-rounded; error bounded by their rounding
                    assert abs(x[(e * sh.levels + l) * sh.feats + f] - ref) <= 8 * 2.0 ** -24 * (np.abs(a).sum() + abs(b) + 1)


def test_encoding_partition_of_unity_and_order():
    sh = S.TINY
    base = O.Model(sh, UNIT_BOX, zero_mlp(sh))
    # constant tables: value 100 e + 10 l + f -> features read back in (e, l, f) order
    g = _vertex_grid(base, lambda e, l, f, x, y, z, N: 100.0 * e + 10.0 * l + f)
    m = O.Model(sh, UNIT_BOX, zero_mlp(sh), grids=[g.astype(np.float32)])
    w = S.tiny_workload(n_rays=200)
    out = m.forward(w["rays"], w["ids"], w["tmax"], want_x=True)
    expect = np.array([100.0 * e + 10.0 * l + f for e in range(3) for l in range(sh.levels) for f in range(sh.feats)])
    hit = out["status"] == 1
    np.testing.assert_allclose(out["x"][hit], np.broadcast_to(expect, (hit.sum(), expect.size)), rtol=1e-14, atol=1e-12)


def test_encoding_vertex_exactness_and_corners():
    sh = S.TINY
    g = O.init_grid(seed=9, obj=0, amp=1.0, grid_dtype="f32", count=O.Model(sh, UNIT_BOX, zero_mlp(sh)).grid_elems)
    m = O.Model(sh, UNIT_BOX, zero_mlp(sh), grids=[g], coord_mode=1)
    # ray entering exactly at a vertex of every level: u_in = (0.25, 0.5, 0) on the z = 0 face
    st, u, x, ce, cw = _detail(m, (0.25, 0.5, -2.0), (0, 0, 1))
    assert st == 1
    res = m.level_res()
    off = m.grid_offsets()
    for l, N in enumerate(res):
        ix, iy, iz = int(0.25 * N), int(0.5 * N), 0
        v = (iz * (N + 1) + iy) * (N + 1) + ix
        assert x[l * 2] == g[off[l] + 2 * v] and x[l * 2 + 1] == g[off[l] + 2 * v + 1]
        # weights of one corner are 1, the others 0; weights always sum to 1
        np.testing.assert_allclose(cw[l].sum(), 1.0)
        assert sorted(cw[l])[-1] == 1.0


def test_clamped_cell_at_upper_face():
    sh = S.TINY
    m = O.Model(sh, UNIT_BOX, zero_mlp(sh), coord_mode=1)
    st, u, x, ce, cw = _detail(m, (0.5, 0.5, 3.0), (0, 0, -1))  # exits through z = 0, enters at z = 1
    assert st == 1 and u[0][2] == 1.0
    res = m.level_res()
    off = m.grid_offsets()
    for l, N in enumerate(res):
        # cell N-1 with weight 1 on its upper z corner: all used vertices are valid
        assert (ce[l] >= off[l]).all() and (ce[l] < off[l + 1]).all()
        assert np.isclose(cw[l][4:].sum(), 1.0)


# ---------------------------------------------------------------- MLP

def _small_model(W1, wout):
    sh = S.ModelShape(levels=1, res_min=2, res_max=2, feats=1, hidden=1, width=2, grid_dtype="f32")
    w = np.concatenate([np.ravel(W1), np.ravel(wout)]).astype(np.float32)
    return O.Model(sh, UNIT_BOX, w[None, :])


def test_mlp_hand_computed():
    m = _small_model([[1.0, -1.0, 0.5], [-2.0, 0.5, 1.0]], [3.0, -1.0])
    # a = (1 - 2 + 1.5, -2 + 1 + 3) = (0.5, 2); z = 3*0.5 - 2 = -0.5
    # second input: a = (3, -6) -> h = (3, 0); z = 9
    z = m.mlp_only(np.array([[1.0, 2.0, 3.0], [3.0, 0.0, 0.0]]))
    np.testing.assert_array_equal(z, [-0.5, 9.0])


def test_mlp_two_hidden_hand_computed():
    sh = S.ModelShape(levels=1, res_min=2, res_max=2, feats=1, hidden=2, width=2, grid_dtype="f32")
    # W1 = [[1,0,0],[0,1,0]], W2 = [[1,1],[1,-1]], w_out = [1, 2]
    w = np.array([1, 0, 0, 0, 1, 0, 1, 1, 1, -1, 1, 2], np.float32)
    m = O.Model(sh, UNIT_BOX, w[None, :])
    # x = (2, 3, 7): h1 = (2, 3); h2 = ReLU(5, -1) = (5, 0); z = 5
    np.testing.assert_array_equal(m.mlp_only(np.array([[2.0, 3.0, 7.0]])), [5.0])


def test_zero_weights_give_half_and_visible():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    assert gold["occlusion_threshold"]["value"] == 0.5
    w = S.tiny_workload(n_rays=100)
    m = O.Model(w["shape"], w["aabb"], np.zeros_like(w["mlps"]), grid_seed=1)
    out = m.forward(w["rays"], w["ids"], w["tmax"])
    hit = out["status"] == 1
    assert (out["y"][hit] == 0.5).all()  # z = 0 -> probability 1/2 -> not below 0.5 -> visible


def test_sigmoid_symmetry():
    w = S.tiny_workload(n_rays=200)
    m = O.Model(w["shape"], w["aabb"], w["mlps"], grid_seed=1, grid_amp=1.0)
    neg = w["mlps"].copy()
    neg[:, -w["shape"].width:] *= -1  # negate w_out: z -> -z
    mn = O.Model(w["shape"], w["aabb"], neg, grid_seed=1, grid_amp=1.0)
    a = m.forward(w["rays"], w["ids"], w["tmax"])
    b = mn.forward(w["rays"], w["ids"], w["tmax"])
    np.testing.assert_allclose(a["y"] + b["y"], 1.0, rtol=0, atol=1e-15)


def test_paper_network_size():
    """Sec. 5 "Memory Footprint": the outer network (two 3-latent grids = 6 inputs,
    2 hidden layers of 64) takes about 18 kB in binary32, which fixes the reading
    that H hidden layers means H+1 weight matrices and no biases."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    n_in = 2 * gold["outer_grid"]["N"]
    sh = S.ModelShape(levels=1, res_min=256, res_max=256, feats=n_in // 3, hidden=2, width=64, grid_dtype="f16")
    m = O.Model(sh, UNIT_BOX, np.zeros((1, sh.mlp_params), np.float32))
    P = O.lib().orc_mlp_params(m.ref)
    assert round(P * 4 / 1024) == gold["outer_network_runtime_kB"]["value"]
    # a third weight matrix would no longer round to the printed size
    assert round((P + 64 * 64) * 4 / 1024) != gold["outer_network_runtime_kB"]["value"]


# ---------------------------------------------------------------- quantisation emulation

def test_fp8_identity_when_exact():
    """FP8 with unit scales and every weight/activation exactly representable equals the exact path."""
    sh = S.ModelShape(levels=1, res_min=2, res_max=2, feats=1, hidden=2, width=2, grid_dtype="f32")
    w = np.array([1, 0, 0.5, 0, 1, 0, 1, 0.25, 0.5, -1, 1, 2], np.float32)
    m = O.Model(sh, UNIT_BOX, w[None, :])
    mq = O.Model(sh, UNIT_BOX, w[None, :], quant="fp8", fp8_scales=np.ones((1, 4)))
    x = np.array([[2.0, 3.0, 0.5], [0.25, 1.5, 4.0]])  # all activations E4M3 values
    np.testing.assert_array_equal(m.mlp_only(x), mq.mlp_only(x))


def _two_object_calibration_case(mlp0):
    g = np.random.default_rng(31)
    boxes = np.array([[-1, -1, -1, 1, 1, 1], [3, 0, 0, 4, 2, 1]], np.float32)
    n = 3000
    ids = (np.arange(n) % 2).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.empty(n, np.float32)
    for k in range(2):
        s = np.nonzero(ids == k)[0]
        r, t = S.rays_sphere_to_box(s.size, boxes[k], g, radius=4.0, center=0.5 * (boxes[k, :3] + boxes[k, 3:]))
        rays[s], tmax[s] = r, t
    rays[::7, 3:] = -rays[::7, 3:]  # misses
    mlps = np.stack([mlp0, S.xavier_mlp(S.TINY, S.rng(5, 3))])
    # object 1 (MLP 1) has latents 1e4 times larger: it must not enter MLP 0's scales
    m = O.Model(S.TINY, boxes, mlps, mlp_index=np.array([0, 1], np.int32), grid_seed=3, grid_amp=[1.0, 1e4])
    return m, rays, ids, tmax


def test_fp8_calibration_closed_form():
    """Identity-like layers make every layer input a closed form of the features:
    W_1 = -[I; 0] gives h_1 = ReLU(-x) (zero-padded), W_2 = 2I gives h_2 = 2 ReLU(-x).
    So s_W = [1, 2, 3] / 448 and s_x = [max|x|, max ReLU(-x), 2 max ReLU(-x)] / 448 over
    the MLP's own hitting queries."""
    sh = S.TINY
    din, W = sh.din, sh.width
    w = np.concatenate([-np.eye(W, din).ravel(), 2 * np.eye(W).ravel(), 3 * np.eye(W).ravel(), np.ones(W)])
    m, rays, ids, tmax = _two_object_calibration_case(w.astype(np.float32))
    f = m.forward(rays, ids, tmax, want_x=True)
    sel = (f["status"] == 1) & (ids == 0)
    assert 0 < sel.sum() < (f["status"] == 1).sum()
    x = f["x"][sel]
    r = np.maximum(-x, 0).max()
    assert np.abs(x).max() > r > 0  # the max of |x| and of ReLU(-x) differ here
    s = m.fp8_calibrate(rays, ids, tmax, mlp=0)
    np.testing.assert_array_equal(s[:3], np.array([1.0, 2.0, 3.0]) / 448.0)
    np.testing.assert_array_equal(s[3:], np.array([np.abs(x).max(), r, 2 * r]) / 448.0)
    # the other MLP sees the large latents
    s1 = m.fp8_calibrate(rays, ids, tmax, mlp=1)
    assert s1[3] > 1e3 * s[3]


def test_fp8_calibration_zero_weights_and_no_queries():
    """All-zero weights give unit weight scales and unit scales for the all-zero hidden
    inputs; with no query of the MLP every activation scale is 1."""
    m, rays, ids, tmax = _two_object_calibration_case(np.zeros(S.TINY.mlp_params, np.float32))
    s = m.fp8_calibrate(rays, ids, tmax, mlp=0)
    assert (s[:3] == 1.0).all() and s[3] < 1.0 and (s[4:] == 1.0).all()
    s = m.fp8_calibrate(rays[ids == 1], ids[ids == 1], tmax[ids == 1], mlp=0)
    assert (s == 1.0).all()


def _round_net(H, mats, wout, quant, scales=None):
    """A width-2 net with din = 3 (levels 1, feats 1), weights given row-major."""
    sh = S.ModelShape(levels=1, res_min=2, res_max=2, feats=1, hidden=H, width=2, grid_dtype="f32")
    w = np.concatenate([np.ravel(m) for m in mats] + [np.ravel(wout)]).astype(np.float32)
    assert w.size == sh.mlp_params
    sc = None if scales is None else np.asarray(scales, np.float64)[None, :]
    return O.Model(sh, UNIT_BOX, w[None, :], quant=quant, fp8_scales=sc)


@pytest.mark.parametrize("quant,q", [("bf16", 2.0 ** -7), ("f16", 2.0 ** -10), ("fp8", 2.0 ** -3)])
def test_rounding_positions_hand_computed(quant, q):
    """Where the reduced-precision forms round: the MLP input, every hidden
    weight matrix, every hidden activation except the last, and nothing in
    the binary32 output layer.  q is the spacing of the format on [1, 2)
    (7, 10 and 3 fraction bits); 1 + 3q/4 rounds to 1 + q (nearest), and
    1 + 2q + q^2 to 1 + 2q (q^2 < q/2).  Each net below routes one value
    through unit 0 and has all other weights zero, and its expected logit is
    worked out by hand; moving any one rounding changes that logit (noted per
    case).  FP8 uses unit scales here, so its codes are the E4M3 values."""
    e = 0.75 * q
    sc2 = [1.0] * 4 if quant == "fp8" else None
    sc1 = [1.0] * 2 if quant == "fp8" else None
    I3 = [[1, 0, 0], [0, 0, 0]]
    I2 = [[1, 0], [0, 0]]
    one = np.array([[1.0, 0, 0]])
    # input rounded: x = 1 + 3q/4 -> 1 + q (unrounded input would give 1 + 3q/4)
    assert _round_net(2, [I3, I2], [1, 0], quant, sc2).mlp_only(np.array([[1 + e, 0, 0]]))[0] == 1 + q
    # first-layer weight rounded (else 1 + 3q/4)
    assert _round_net(2, [[[1 + e, 0, 0], [0, 0, 0]], I2], [1, 0], quant, sc2).mlp_only(one)[0] == 1 + q
    # hidden-layer weight rounded (else 1 + 3q/4)
    assert _round_net(2, [I3, [[1 + e, 0], [0, 0]]], [1, 0], quant, sc2).mlp_only(one)[0] == 1 + q
    # h_1 = (1+q)^2 = 1 + 2q + q^2 rounded to 1 + 2q (else the q^2 term stays); the last
    # activation a_2 = (1+q)(1+2q) = 1 + 3q + 2q^2 is not rounded (else 1 + 3q)
    d = _round_net(2, [[[1 + q, 0, 0], [0, 0, 0]], [[1 + q, 0], [0, 0]]], [1, 0], quant, sc2)
    assert d.mlp_only(np.array([[1 + q, 0, 0]]))[0] == 1 + 3 * q + 2 * q * q
    # binary32 output weight, not rounded (else 1 + q)
    assert _round_net(2, [I3, I2], [1 + e, 0], quant, sc2).mlp_only(one)[0] == 1 + e
    # one hidden layer: h_1 is the last activation, not rounded (else 1 + 2q)
    g = _round_net(1, [[[1 + q, 0, 0], [0, 0, 0]]], [1, 0], quant, sc1)
    assert g.mlp_only(np.array([[1 + q, 0, 0]]))[0] == 1 + 2 * q + q * q


def test_fp8_scales_hand_computed():
    """FP8 per-layer scales: a layer input h becomes s_x E4M3(h / s_x) and a weight
    s_W E4M3(w / s_W).  With s = 0.75, 1 / 0.75 = 1.333.. lies between the E4M3
    values 1.25 and 1.375 and rounds to 1.375, so 1 -> 0.75 * 1.375 = 1.03125
    (an unscaled rounding would keep 1).  E4M3 has no infinity: 500 saturates
    to 448."""
    I3 = [[1, 0, 0], [0, 0, 0]]
    I2 = [[1, 0], [0, 0]]
    one = np.array([[1.0, 0, 0]])
    assert _round_net(1, [I3], [1, 0], "fp8", [1.0, 0.75]).mlp_only(one)[0] == 1.03125   # s_x of layer 1
    assert _round_net(1, [I3], [1, 0], "fp8", [0.75, 1.0]).mlp_only(one)[0] == 1.03125   # s_W of layer 1
    assert _round_net(2, [I3, I2], [1, 0], "fp8", [1.0, 1.0, 1.0, 0.75]).mlp_only(one)[0] == 1.03125  # s_x, layer 2
    assert _round_net(1, [I3], [1, 0], "fp8", [1.0, 1.0]).mlp_only(np.array([[500.0, 0, 0]]))[0] == 448.0


@pytest.mark.parametrize("q", ["bf16", "f16"])
def test_quantised_within_bound(q):
    w = S.tiny_workload(n_rays=3000)
    m = O.Model(w["shape"], w["aabb"], w["mlps"], grid_seed=1, grid_amp=1.0)
    a = m.forward(w["rays"], w["ids"], w["tmax"])
    b = m.with_(quant=q).forward(w["rays"], w["ids"], w["tmax"])
    assert (np.abs(b["y"] - a["y"]) <= b["ybound"]).all()
    assert np.abs(b["z"] - a["z"]).max() > 0  # the emulation does round


# ---------------------------------------------------------------- gradients

def _fd_model(grid):
    sh = S.TINY
    w = S.xavier_mlp(sh, S.rng(77, 3)) * 2.0
    return sh, w


def test_backward_matches_finite_differences():
    """Central differences of the binary64 loss against the analytic gradient."""
    sh = S.TINY
    wl = S.tiny_workload(n_rays=256)
    g0 = O.init_grid(seed=4, obj=0, amp=0.5, grid_dtype="f32", count=O.Model(sh, UNIT_BOX, zero_mlp(sh)).grid_elems)
    W = (S.xavier_mlp(sh, S.rng(77, 3)).astype(np.float64) * 2.0)
    labels = (np.random.default_rng(5).uniform(size=256) < 0.5).astype(np.uint8)

    def model(Wv, g):
        return O.Model(sh, wl["aabb"], Wv[None, :], grids=[g.astype(np.float64).astype(np.float32)], coord_mode=1)

    def loss_of(Wv, g):
        mm = O.Model(sh, wl["aabb"], Wv[None, :], grids=[g], coord_mode=1)
        out = mm.forward(wl["rays"], wl["ids"], wl["tmax"])
        hit = out["status"] == 1
        return O.bce_with_logits(out["z"][hit], labels[hit])[0]

    m = model(W, g0)
    loss, B, gW, gx = m.backward(wl["rays"], wl["ids"], wl["tmax"], labels)
    assert B == 256
    # the C loss equals the numpy BCE of the C forward's logits
    assert abs(loss - loss_of(W, g0)) < 1e-14
    # MLP weights: the oracle MLP is exact binary64, so perturb the binary64 copy
    rng = np.random.default_rng(6)
    idx = rng.choice(sh.mlp_params, 40, replace=False)
    Wd = W.copy()
    for k in idx:
        h = 1e-6 * max(1.0, abs(Wd[k]))
        Wp, Wm = Wd.copy(), Wd.copy()
        Wp[k] += h
        Wm[k] -= h
        mp = O.Model(sh, wl["aabb"], Wp[None, :], grids=[g0], coord_mode=1)
        mm = O.Model(sh, wl["aabb"], Wm[None, :], grids=[g0], coord_mode=1)
        zp = mp.forward(wl["rays"], wl["ids"], wl["tmax"])["z"]
        zm = mm.forward(wl["rays"], wl["ids"], wl["tmax"])["z"]
        fd = (O.bce_with_logits(zp, labels)[0] - O.bce_with_logits(zm, labels)[0]) / (2 * h)
        assert abs(fd - gW[0, k]) <= 1e-6 * max(1e-3, abs(gW[0, k])) + 1e-9, (k, fd, gW[0, k])
    # grid latents enter linearly: use the dense scatter of gx
    gg = m.grid_grad_dense(0, wl["rays"], wl["ids"], wl["tmax"], gx)
    touched = np.nonzero(gg)[0]
    assert touched.size > 1000
    pick = rng.choice(touched, 30, replace=False)
    g64 = g0.astype(np.float64)
    for k in pick:
        h = 2.0 ** -14
        gp, gm = g64.copy(), g64.copy()
        gp[k] += h
        gm[k] -= h
        # grid values are binary32 in the model: divide by the step actually taken
        fd = (loss_of(W, gp.astype(np.float32)) - loss_of(W, gm.astype(np.float32))) / (
            gp.astype(np.float32)[k] - gm.astype(np.float32)[k])
        assert abs(fd - gg[k]) <= 1e-5 * abs(gg[k]) + 1e-10, (k, fd, gg[k])


def test_backward_given_matches_finite_differences():
    """Upstream-gradient backward: d/dtheta of sum_i c_i y_i by central differences."""
    sh = S.TINY
    wl = S.tiny_workload(n_rays=256)
    g0 = O.init_grid(seed=8, obj=0, amp=0.5, grid_dtype="f32", count=O.Model(sh, UNIT_BOX, zero_mlp(sh)).grid_elems)
    W = S.xavier_mlp(sh, S.rng(78, 3)).astype(np.float64) * 2.0
    c = np.random.default_rng(9).normal(size=256)

    def obj_of(Wv, g):
        y = O.Model(sh, wl["aabb"], Wv[None, :], grids=[g], coord_mode=1).forward(wl["rays"], wl["ids"], wl["tmax"])["y"]
        return float(np.sum(c * y))

    m = O.Model(sh, wl["aabb"], W[None, :], grids=[g0], coord_mode=1)
    B, gW, gx = m.backward_given(wl["rays"], wl["ids"], wl["tmax"], c)
    assert B == 256
    rng = np.random.default_rng(10)
    for k in rng.choice(sh.mlp_params, 30, replace=False):
        h = 1e-6 * max(1.0, abs(W[k]))
        Wp, Wm = W.copy(), W.copy()
        Wp[k] += h
        Wm[k] -= h
        fd = (obj_of(Wp, g0) - obj_of(Wm, g0)) / (2 * h)
        assert abs(fd - gW[0, k]) <= 1e-6 * max(1e-3, abs(gW[0, k])) + 1e-9, (k, fd, gW[0, k])
    gg = m.grid_grad_dense(0, wl["rays"], wl["ids"], wl["tmax"], gx)
    g64 = g0.astype(np.float64)
    for k in rng.choice(np.nonzero(gg)[0], 20, replace=False):
        gp, gm = g64.copy(), g64.copy()
        gp[k] += 2.0 ** -14
        gm[k] -= 2.0 ** -14
        fd = (obj_of(W, gp.astype(np.float32)) - obj_of(W, gm.astype(np.float32))) / (
            gp.astype(np.float32)[k] - gm.astype(np.float32)[k])
        assert abs(fd - gg[k]) <= 1e-5 * abs(gg[k]) + 1e-10, (k, fd, gg[k])


def test_grid_grad_at_matches_dense():
    sh = S.TINY
    wl = S.tiny_workload(n_rays=128)
    m = O.Model(sh, wl["aabb"], wl["mlps"], grid_seed=2, grid_amp=0.5)
    labels = np.ones(128, np.uint8)
    _, _, _, gx = m.backward(wl["rays"], wl["ids"], wl["tmax"], labels)
    dense = m.grid_grad_dense(0, wl["rays"], wl["ids"], wl["tmax"], gx)
    sel = np.concatenate([np.nonzero(dense)[0][::7], np.array([0, 1, 5])])
    el, vals = m.grid_grad_at(0, wl["rays"], wl["ids"], wl["tmax"], gx, np.unique(sel))
    np.testing.assert_array_equal(vals, dense[el])


def test_bce_closed_form():
    z = np.array([0.0, 2.0, -3.0])
    t = np.array([1.0, 0.0, 1.0])
    L, dz = O.bce_with_logits(z, t)
    ref = (np.log(2) + (2 + np.log1p(np.exp(-2))) + (np.log1p(np.exp(-3)) + 3)) / 3
    assert abs(L - ref) < 1e-15
    s = 1 / (1 + np.exp(-z))
    np.testing.assert_allclose(dz, (s - t) / 3, rtol=1e-15)


def test_adam_first_step_closed_form_and_lazy():
    g = np.array([0.3, -2e-3, 0.0, 1e-12])
    th, m, v = O.adam_step(np.ones(4), np.zeros(4), np.zeros(4), g, step=1, lr=1e-2, beta1=0.9, beta2=0.99,
                           eps=1e-15, lazy=True)
    # step 1: m_hat = g, v_hat = g^2 -> delta = -lr g / (|g| + eps)
    np.testing.assert_allclose(th[[0, 1, 3]], 1 - 1e-2 * g[[0, 1, 3]] / (np.abs(g[[0, 1, 3]]) + 1e-15), rtol=1e-14)
    assert th[2] == 1.0 and m[2] == 0.0 and v[2] == 0.0  # lazy: untouched
    th2, m2, v2 = O.adam_step(th, m, v, np.array([0.0, 0.0, 0.0, 0.0]), step=2, lr=1e-2, beta1=0.9, beta2=0.99,
                              eps=1e-15, lazy=False)
    assert (m2 == 0.9 * m).all()


# ---- depth output for primary rays (Sec. 7) ----

def test_depth_target_closed_form():
    """Axis-aligned rays through the unit box with the hit plane z = 0.3: the
    segment is [t_a, t_b] = [2, 3] for an origin at z = -2 looking up z, so the
    normalised depth of the hit at t = 2.3 is 0.3; a miss of the box has no
    target, nor a ray without a hit."""
    sh = S.TINY
    m = O.Model(sh, UNIT_BOX, zero_mlp(sh), coord_mode=1)
    rays = np.array([[0.5, 0.5, -2, 0, 0, 1], [0.5, 0.5, -2, 0, 0, 2], [3, 3, -2, 0, 0, 1], [0.5, 0.5, -2, 0, 0, 1]],
                    np.float32)
    ids = np.zeros(4, np.int32)
    tmax = np.full(4, np.inf, np.float32)
    ta, tb = m.segment(rays, ids, tmax)
    np.testing.assert_array_equal(ta[:2], [2.0, 1.0])
    np.testing.assert_array_equal(tb[:2], [3.0, 1.5])
    assert np.isinf(ta[2]) and np.isinf(tb[2])
    s = m.depth_targets(rays, ids, tmax, np.array([2.3, 1.15, 5.0, np.inf]))
    np.testing.assert_allclose(s[:2], [0.3, 0.3], rtol=1e-12)
    assert np.isnan(s[2]) and np.isnan(s[3])
    # zero weights: y = 1/2, so the predicted depth is the segment's midpoint
    np.testing.assert_allclose(m.depth(rays[:2], ids[:2], tmax[:2]), [2.5, 1.25], rtol=1e-12)


def test_depth_loss_gradient_matches_finite_differences():
    """L2 depth loss of the oracle: d/dtheta of (1/B) sum (y - s)^2 by central
    differences (MLP weights and latents), targets from the exact closest hit."""
    sh = S.TINY
    wl = S.tiny_workload(n_rays=256)
    t_hit = O.closest_brute(wl["tris"], wl["rays"], wl["tmax"])
    g0 = O.init_grid(seed=8, obj=0, amp=0.5, grid_dtype="f32", count=O.Model(sh, UNIT_BOX, zero_mlp(sh)).grid_elems)
    W = S.xavier_mlp(sh, S.rng(79, 3)).astype(np.float64) * 2.0

    def loss_of(Wv, g):
        return O.Model(sh, wl["aabb"], Wv[None, :], grids=[g], coord_mode=1).depth_loss_backward(
            wl["rays"], wl["ids"], wl["tmax"], t_hit)[0]

    m = O.Model(sh, wl["aabb"], W[None, :], grids=[g0], coord_mode=1)
    loss, B, gW, gx = m.depth_loss_backward(wl["rays"], wl["ids"], wl["tmax"], t_hit)
    assert 50 < B < 256 and loss > 0
    rng = np.random.default_rng(11)
    for k in rng.choice(sh.mlp_params, 20, replace=False):
        h = 1e-6 * max(1.0, abs(W[k]))
        Wp, Wm = W.copy(), W.copy()
        Wp[k] += h
        Wm[k] -= h
        fd = (loss_of(Wp, g0) - loss_of(Wm, g0)) / (2 * h)
        assert abs(fd - gW[0, k]) <= 1e-6 * max(1e-3, abs(gW[0, k])) + 1e-9, (k, fd, gW[0, k])
    gg = m.grid_grad_dense(0, wl["rays"], wl["ids"], wl["tmax"], gx)
    g64 = g0.astype(np.float64)
    for k in rng.choice(np.nonzero(gg)[0], 10, replace=False):
        gp, gm = g64.copy(), g64.copy()
        gp[k] += 2.0 ** -14
        gm[k] -= 2.0 ** -14
        fd = (loss_of(W, gp.astype(np.float32)) - loss_of(W, gm.astype(np.float32))) / (
            gp.astype(np.float32)[k] - gm.astype(np.float32)[k])
        assert abs(fd - gg[k]) <= 1e-5 * abs(gg[k]) + 1e-10, (k, fd, gg[k])
