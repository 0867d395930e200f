"""Pins of the binary64 oracle of the paper's own networks (outer and inner
NIF networks with spherical 2D grids, Sec. 3.1, Sec. 3.2, Sec. 5, Table 1)
against closed forms, invariants and hand-computed cases."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import paper_nets as PN

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
BOX = np.array([[-1.0, -2.0, 0.5, 3.0, 2.0, 1.5]], np.float32)  # non-cubic on purpose


def test_network_sizes_match_table_1_and_memory_footprint():
    """Sec. 5: 18 kB (outer) and 21 kB (inner) of binary32 weights, with the
    inputs of Table 1 (3+3 and 5+5+3 latents) and no biases."""
    assert PN.OUTER["R"] == GOLD["outer_grid"]["R"] and PN.OUTER["N"] == GOLD["outer_grid"]["N"]
    assert PN.INNER["R"] == GOLD["inner_grid_2d"]["R"] and PN.INNER["N"] == GOLD["inner_grid_2d"]["N"]
    assert PN.INNER["R1"] == GOLD["inner_grid_1d"]["R"] and PN.INNER["N1"] == GOLD["inner_grid_1d"]["N"]
    assert PN.mlp_params(0) == 6 * 64 + 64 * 64 + 64 == 4544
    assert PN.mlp_params(1) == 13 * 48 + 2 * 48 * 48 + 48 == 5280
    assert round(PN.mlp_params(0) * 4 / 1024) == GOLD["outer_network_runtime_kB"]["value"]
    assert round(PN.mlp_params(1) * 4 / 1024) == GOLD["inner_network_runtime_kB"]["value"]


def test_rounding_matches_the_c_oracle():
    """numpy RNE to bf16 / f16 agrees with the C oracle's rounding (itself
    pinned on bit patterns and ties) on normal, f16-subnormal and tie values."""
    g = np.random.default_rng(3)
    vals = np.concatenate([g.normal(size=300), g.normal(size=300) * 1e-5, g.normal(size=100) * 1e-7,
                           [1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -11, 2 ** -24 * 1.5, -(2 ** -24) * 2.5, 0.0]])
    for fmt in ("bf16", "f16"):
        np.testing.assert_array_equal(PN.round_to(vals, fmt), O.round_fmt_array(vals, fmt))


def test_spherical_map_closed_forms():
    q = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 0], [1, 1, 0]], float)
    u, v = PN.sph(q)
    np.testing.assert_allclose(u, [0, 1, 0.5, 0.5, 0.5, 0.5, 0, 0.5], atol=1e-15)
    np.testing.assert_allclose(v, [0.5, 0.5, 0.5, 1.0, 0.75, 0.25, 0.5, 0.625], atol=1e-15)


def _outside_rays(g, n, box, back=0.0):
    lo, hi = box[0, :3].astype(float), box[0, 3:].astype(float)
    target = lo + g.uniform(0.05, 0.95, (n, 3)) * (hi - lo)
    dirs = g.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    o = target - (6.0 + back) * dirs
    return np.concatenate([o, dirs], 1).astype(np.float32)


def test_outer_transform_is_invariant_along_the_ray():
    """Sec. 2 and Sec. 3.1: moving the origin back along d (still outside the
    box) gives the same entry point, so the same (p', d')."""
    g = np.random.default_rng(4)
    n = 500
    rays = _outside_rays(g, n, BOX)
    ids = np.zeros(n, np.int32)
    tmax = np.full(n, np.inf, np.float32)
    a = PN.transform(rays, ids, tmax, BOX)
    moved = rays.astype(np.float64).copy()
    moved[:, :3] -= 3.0 * moved[:, 3:]
    b = PN.transform(moved.astype(np.float32), ids, tmax, BOX)
    assert (a[0] == PN.CLS_OUTER).all() and (b[0] == PN.CLS_OUTER).all()
    for k in (1, 2, 3, 4):  # binary32 inputs and clip: a few ulp of the entry point
        np.testing.assert_allclose(a[k], b[k], atol=2e-6)
    np.testing.assert_array_equal(a[3], b[3])  # the direction is exactly the same
    np.testing.assert_array_equal(a[4], b[4])


def test_entry_point_maps_to_its_face():
    """A ray straight down the -z axis enters through the top face centre:
    theta = 0 (u = 0); one along +x enters the x = lo face centre: u = 1/2, v = 1."""
    rays = np.array([[1.0, 0.0, 9.0, 0.0, 0.0, -1.0], [-9.0, 0.0, 1.0, 1.0, 0.0, 0.0]], np.float32)
    cls, pu, pv, du, dv, r = PN.transform(rays, np.zeros(2, np.int32), np.full(2, np.inf, np.float32), BOX)
    assert list(cls) == [PN.CLS_OUTER] * 2
    np.testing.assert_allclose([pu[0], pu[1], pv[1]], [0.0, 0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose([du[0], du[1], dv[1]], [1.0, 0.5, 0.5], atol=1e-15)
    np.testing.assert_allclose(r, [1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)


def test_classes():
    rays = np.array([[1, 0, 1, 0, 0, 1],            # origin inside: inner
                     [1, 0, 9, 0, 0, -1],           # outside, towards the box: outer
                     [1, 0, 9, 0, 0, 1],            # outside, away: miss
                     [1, 0, 9, 0, 0, -1],           # t_max too short: miss
                     [np.nan, 0, 0, 1, 0, 0],       # invalid
                     [1, 0, 9, 0, 0, -1]], np.float32)
    ids = np.array([0, 0, 0, 0, 0, 3], np.int32)
    tmax = np.array([np.inf, np.inf, np.inf, 1.0, 1.0, 1.0], np.float32)
    cls = PN.classify(rays, ids, tmax, BOX)[0]
    assert list(cls) == [2, 1, 0, 0, -1, -1]
    # the inner distance: centre -> 0, near a corner -> nearly 1
    c = 0.5 * (BOX[0, :3] + BOX[0, 3:])
    near = BOX[0, 3:] - 1e-3 * (BOX[0, 3:] - BOX[0, :3])
    rr = np.array([[*c, 0, 0, 1], [*near, 1, 0, 0]], np.float32)
    r = PN.transform(rr, np.zeros(2, np.int32), np.full(2, np.inf, np.float32), BOX)[5]
    assert r[0] == 0.0 and 0.99 < r[1] < 1.0


@pytest.mark.parametrize("R", [4, 256])
def test_bilinear_reproduces_affine_fields(R):
    """G[a, b] = alpha a + beta b + gamma per latent: the lookup returns
    alpha s_u + beta s_v + gamma exactly (up to rounding); an all-ones grid
    interpolates to 1; vertices are reproduced exactly."""
    g = np.random.default_rng(5)
    al, be, ga = g.normal(size=3), g.normal(size=3), g.normal(size=3)
    a = np.arange(R)[:, None, None]
    b = np.arange(R)[None, :, None]
    G = al * a + be * b + ga
    u, v = g.uniform(0, 1, 400), g.uniform(0, 1, 400)
    u[:2], v[:2] = [0.0, 1.0], [1.0, 0.0]
    got = PN.bilinear(G, u, v)
    want = al * (u * (R - 1))[:, None] + be * (v * (R - 1))[:, None] + ga
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * R)
    np.testing.assert_allclose(PN.bilinear(np.ones((R, R, 5)), u, v), 1.0, atol=1e-14)
    iu, iv = g.integers(0, R, 50), g.integers(0, R, 50)
    Gr = g.normal(size=(R, R, 3))
    np.testing.assert_allclose(PN.bilinear(Gr, iu / (R - 1), iv / (R - 1)), Gr[iu, iv], atol=1e-14)
    G1 = g.normal(size=3) * np.arange(R)[:, None] + 2.0
    r = g.uniform(0, 1, 100)
    np.testing.assert_allclose(PN.linear(G1, r), G1[0] + (G1[1] - G1[0]) * (r * (R - 1))[:, None], atol=1e-11 * R)


def test_mlp_hand_computed():
    """2-2-1 leaky-ReLU network by hand: x = (1, 1), W1 = [[1, -2], [0.5, 1]]
    -> pre-activations (-1, 1.5) -> (-s, 1.5) with the slope s -> z = 2(-s) + 3(1.5)."""
    mats = [np.array([[1.0, -2.0], [0.5, 1.0]]), np.array([[2.0, 3.0]])]
    z = PN.mlp_mats(np.array([[1.0, 1.0]]), mats)
    assert z[0] == 2 * (-PN.LEAKY) + 4.5
    # a second hidden layer W2 = identity applies the slope to -s once more
    z2 = PN.mlp_mats(np.array([[1.0, 1.0]]), [mats[0], np.eye(2), mats[1]])
    assert abs(z2[0] - (2 * (-PN.LEAKY * PN.LEAKY) + 4.5)) < 1e-15
    assert abs(PN.LEAKY - 0.01) < 1e-9


def test_quantised_equals_exact_when_representable():
    """Weights, inputs and activations that bf16 and f16 hold exactly, with
    positive pre-activations: the quantised MLP is the exact one."""
    g = np.random.default_rng(6)
    mats = [g.integers(1, 4, (64, 6)) / 8.0, g.integers(1, 4, (64, 64)) / 64.0, g.integers(-3, 4, (1, 64)) / 8.0]
    x = g.integers(1, 4, (20, 6)) / 4.0
    ref = PN.mlp_mats(x, mats)
    for q in ("bf16", "f16"):
        np.testing.assert_array_equal(PN.mlp_mats(x, mats, q), ref)


def test_grid_layout_and_init_stream():
    """One object's buffer: position, direction (and distance) grids back to
    back; the latents are the generator's elements of key 2 obj + network."""
    assert PN.grid_elems(0) == 2 * 256 * 256 * 3
    assert PN.grid_elems(1) == 2 * 128 * 128 * 5 + 128 * 3
    buf = O.init_grid(7, PN.init_key(3, 1), 1e-4, "f16", PN.grid_elems(1))
    p, d, r = PN.split_grid(buf, 1)
    assert p.shape == (128, 128, 5) and d.shape == (128, 128, 5) and r.shape == (128, 3)
    assert np.array_equal(r.ravel(), buf[-384:])
    vals = buf.view(np.float16).astype(np.float64)
    assert np.abs(vals).max() <= PN.round_to(1e-4, "f16") and np.abs(vals).max() > 0.9e-4


def test_forward_routes_by_class():
    """Outer queries use the outer network, inner ones the inner network; a
    miss is visible with z = +inf; invalid input gives NaN."""
    g = np.random.default_rng(8)
    w0 = g.uniform(-0.3, 0.3, PN.mlp_params(0))
    w1 = g.uniform(-0.3, 0.3, PN.mlp_params(1))
    go = [[g.normal(size=s) for s in PN.grid_shapes(0)]]
    gi = [[g.normal(size=s) for s in PN.grid_shapes(1)]]
    rays = np.array([[1, 0, 1, 0, 0, 1], [1, 0, 9, 0, 0, -1], [1, 0, 9, 0, 0, 1], [np.nan, 0, 0, 1, 0, 0]],
                    np.float32)
    ids = np.zeros(4, np.int32)
    tmax = np.full(4, np.inf, np.float32)
    out = PN.forward(rays, ids, tmax, BOX, go, gi, w0, w1)
    assert list(out["cls"]) == [2, 1, 0, -1]
    _, x1 = PN.features(1, rays[:1], ids[:1], tmax[:1], BOX, gi)
    _, x0 = PN.features(0, rays[1:2], ids[1:2], tmax[1:2], BOX, go)
    assert out["z"][0] == PN.mlp(x1, w1, 1)[0]
    assert out["z"][1] == PN.mlp(x0, w0, 0)[0]
    assert out["y"][2] == 1.0 and out["z"][2] == np.inf
    assert np.isnan(out["y"][3])


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("network", [0, 1])
def test_lowp_bound_covers_the_emulated_rounding(fmt, network):
    """The emulated bf16 / f16 forward is one realisation of the rounding the
    bound covers: |y_q - y_exact| stays within it for every query, and the
    bound is far below the decision margin of typical queries."""
    g = np.random.default_rng(10 + network)
    w = np.concatenate([g.uniform(-math.sqrt(6 / (i + o)), math.sqrt(6 / (i + o)), o * i)
                        for o, i in PN.layer_shapes(network)])
    x = g.normal(size=(3000, PN.din(network))) * 0.3
    y = 1 / (1 + np.exp(-PN.mlp(x, w, network)))
    yq = 1 / (1 + np.exp(-PN.mlp(x, w, network, fmt)))
    bnd = PN.lowp_bound(x, w, network, fmt)
    assert (np.abs(yq - y) <= bnd).all() and np.isfinite(bnd).all()
    assert np.median(bnd) < 0.5  # below the decision margin of a typical query


def _train_case(network, n=48, seed=20):
    g = np.random.default_rng(seed)
    if network == 0:
        rays = _outside_rays(g, n, BOX)
    else:
        lo, hi = BOX[0, :3].astype(float), BOX[0, 3:].astype(float)
        o = lo + g.uniform(0.1, 0.9, (n, 3)) * (hi - lo)
        d = g.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rays = np.concatenate([o, d], 1).astype(np.float32)
    ids = np.zeros(n, np.int32)
    tmax = np.full(n, np.inf, np.float32)
    labels = g.integers(0, 2, n).astype(np.uint8)
    w = np.concatenate([g.uniform(-0.6, 0.6, o_ * i_) for o_, i_ in PN.layer_shapes(network)])
    grids = [[g.normal(size=sh) * 0.3 for sh in PN.grid_shapes(network)]]
    return rays, ids, tmax, labels, w, grids


def _loss(network, rays, ids, tmax, labels, w, grids):
    """L2 loss and the sign pattern of every pre-activation (to skip
    perturbations that cross a kink of the leaky ReLU)."""
    cls, x = PN.features(network, rays, ids, tmax, BOX, grids)
    s = cls == (PN.CLS_OUTER if network == 0 else PN.CLS_INNER)
    y = 1 / (1 + np.exp(-PN.mlp(x[s], w, network)))
    mats = PN.split_weights(w, network)
    h, signs = x[s], []
    for m in mats[:-1]:
        a = h @ m.T
        signs.append(a > 0)
        h = PN.leaky(a)
    return np.mean((y - (labels[s] != 0)) ** 2), np.concatenate([g.ravel() for g in signs])


def _fd(network, rays, ids, tmax, labels, wp, wm, gp, gm, h):
    lp, sp = _loss(network, rays, ids, tmax, labels, wp, gp)
    lm, sm = _loss(network, rays, ids, tmax, labels, wm, gm)
    return (lp - lm) / (2 * h) if np.array_equal(sp, sm) else None


@pytest.mark.parametrize("network", [0, 1])
def test_train_gradients_match_finite_differences(network):
    """Central differences of the binary64 L2 loss: MLP weights (all layers)
    and latents of every grid the queries touch."""
    rays, ids, tmax, labels, w, grids = _train_case(network)
    loss, B, dW, gg = PN.train_grads(network, rays, ids, tmax, labels, BOX, grids, w)
    assert B == 48 and abs(loss - _loss(network, rays, ids, tmax, labels, w, grids)[0]) < 1e-15
    g = np.random.default_rng(21)
    h = 1e-6
    checked = 0
    for i in g.choice(w.size, 40, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = _fd(network, rays, ids, tmax, labels, wp, wm, grids, grids, h)
        if fd is not None:
            checked += 1
            assert abs(fd - dW[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, dW[i])
    for gi in range(len(gg[0])):
        nz = np.argwhere(gg[0][gi] != 0)
        assert len(nz) > 0
        for idx in nz[g.choice(len(nz), min(15, len(nz)), replace=False)]:
            idx = tuple(idx)
            gp = [a.copy() for a in grids[0]]
            gm = [a.copy() for a in grids[0]]
            gp[gi][idx] += h
            gm[gi][idx] -= h
            fd = _fd(network, rays, ids, tmax, labels, w, w, [gp], [gm], h)
            if fd is not None:
                checked += 1
                assert abs(fd - gg[0][gi][idx]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (gi, idx, fd, gg[0][gi][idx])
    assert checked >= 60


def test_l2_loss_closed_form():
    """Zero weights: z = 0, y = 1/2, L = 1/4 for any labels, dL/dz = 2 (1/2 - t) / B / 4."""
    rays, ids, tmax, labels, w, grids = _train_case(0, n=10)
    loss, B, dW, _ = PN.train_grads(0, rays, ids, tmax, labels, BOX, grids, np.zeros_like(w))
    assert loss == 0.25 and B == 10 and not dW.any()
    # only the output row sees a gradient when the hidden weights are zero but w_out is not:
    # h = 0, so dW_out = 0 too
    w2 = np.zeros_like(w)
    w2[-64:] = 1.0
    _, _, dW2, gg = PN.train_grads(0, rays, ids, tmax, labels, BOX, grids, w2)
    assert not dW2.any() and not any(a.any() for a in gg[0])


def test_upstream_gradient_form_matches_finite_differences():
    """With a given dL/dy the gradients are those of L = sum g y over the
    network's queries (central differences of that sum)."""
    network = 1
    rays, ids, tmax, labels, w, grids = _train_case(network, n=40, seed=30)
    gy = np.random.default_rng(31).normal(size=rays.shape[0])
    loss, B, dW, gg = PN.train_grads(network, rays, ids, tmax, None, BOX, grids, w, grad_y=gy)
    assert loss is None

    def f(wv, gr):
        cls, x = PN.features(network, rays, ids, tmax, BOX, gr)
        s = cls == PN.CLS_INNER
        y = 1 / (1 + np.exp(-PN.mlp(x[s], wv, network)))
        return float((gy[s] * y).sum())
    h = 1e-6
    g = np.random.default_rng(32)
    for i in g.choice(w.size, 25, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (f(wp, grids) - f(wm, grids)) / (2 * h)
        assert abs(fd - dW[i]) <= 1e-5 * max(1e-3, abs(fd)) + 1e-8, (i, fd, dW[i])
    nz = np.argwhere(gg[0][2] != 0)
    for idx in nz[:6]:
        idx = tuple(idx)
        gp = [a.copy() for a in grids[0]]
        gm = [a.copy() for a in grids[0]]
        gp[2][idx] += h
        gm[2][idx] -= h
        fd = (f(w, [gp]) - f(w, [gm])) / (2 * h)
        assert abs(fd - gg[0][2][idx]) <= 1e-5 * max(1e-3, abs(fd)) + 1e-8
