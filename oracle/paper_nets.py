"""Binary64 oracle of the paper's own networks: the outer and inner NIF
networks with two-dimensional spherical grids (Sec. 3.1, Sec. 3.2, Fig. 2,
Sec. 5 "Architecture" and "Initialization", Table 1).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.

Plain numpy over arrays of queries, in the paper's order of steps:

1. Classify the query (Sec. 3, Sec. 4.1): invalid input; a segment that
   misses the AABB (visible); origin strictly inside the AABB (inner network,
   Sec. 3.2); otherwise the outer network (Sec. 3.1).  The slab test is done
   in binary32 because a binary32 comparison decides the class on both sides.
2. Transform (Eq. 2 and Eq. 4).  Outer: the AABB entry point p = o + t_a d;
   inner: p = o.  Position: q = (p - c) / h with the box centre c and half
   extents h, then spherical angles of q; direction: spherical angles of d.
   Inner also r = |q| / sqrt(3).  (theta, phi) -> (u, v) = (theta / pi,
   (phi + pi) / (2 pi)), clamped to [0, 1].
3. Grid lookup (Fig. 2): bilinear interpolation on an R x R grid of
   N-vectors, vertex-aligned (s = u (R - 1)); the 1D distance grid is
   interpolated linearly.
4. MLP (Sec. 5 "Architecture"): no biases, leaky ReLU after every hidden
   layer, sigmoid output; the decision is visible iff y >= 0.5.

Readings where the paper is silent: the spherical map of a non-cubic box goes
through the unit cube (q = (p - c) / h) so that the box surface maps
bijectively onto the sphere; the angle grids do not wrap around at phi = +-pi;
a zero q maps to theta = 0, phi = 0; the leaky slope is the binary32 value of
0.01, used alike by both sides; inner and outer queries that miss their box
are visible.

Quantised forms (bf16, f16) round exactly where the kernel does: the MLP
input, every weight matrix of the hidden layers, and each hidden activation
after the leaky ReLU except the last, whose binary32 value feeds the binary32
output layer.
"""
from __future__ import annotations

import math

import numpy as np

LEAKY = float(np.float32(0.01))  # leaky ReLU slope, binary32 value

OUTER = dict(R=256, N=3, hidden=2, width=64)  # Table 1; Sec. 5 "Architecture"
INNER = dict(R=128, N=5, R1=128, N1=3, hidden=3, width=48)

CLS_INVALID, CLS_MISS, CLS_OUTER, CLS_INNER = -1, 0, 1, 2


def din(network: int) -> int:
    return 2 * OUTER["N"] if network == 0 else 2 * INNER["N"] + INNER["N1"]


def layer_shapes(network: int):
    """(out, in) of W1 .. WH and w_out, row-major [out][in]."""
    cfg = OUTER if network == 0 else INNER
    w, H = cfg["width"], cfg["hidden"]
    return [(w, din(network))] + [(w, w)] * (H - 1) + [(1, w)]


def mlp_params(network: int) -> int:
    return sum(o * i for o, i in layer_shapes(network))


def grid_shapes(network: int):
    """Arrays of one object's grid buffer, in buffer order: position, direction
    (R x R x N each), and for the inner network the distance grid (R1 x N1)."""
    if network == 0:
        R, N = OUTER["R"], OUTER["N"]
        return [(R, R, N), (R, R, N)]
    R, N, R1, N1 = INNER["R"], INNER["N"], INNER["R1"], INNER["N1"]
    return [(R, R, N), (R, R, N), (R1, N1)]


def grid_elems(network: int) -> int:
    return sum(int(np.prod(s)) for s in grid_shapes(network))


def split_grid(buf, network: int):
    """Views of a flat grid buffer (any dtype) as the arrays of grid_shapes."""
    out, off = [], 0
    for s in grid_shapes(network):
        k = int(np.prod(s))
        out.append(np.asarray(buf[off:off + k]).reshape(s))
        off += k
    return out


def init_key(obj: int, network: int) -> int:
    """Latent-generator key of object obj's grid buffer of `network`."""
    return 2 * obj + network


# --------------------------------------------------------------------------
# rounding (round to nearest, ties to even) of binary64 values
# --------------------------------------------------------------------------

def round_to(x, fmt: str) -> np.ndarray:
    """x rounded to bf16 or f16 (RNE), returned as binary64; overflow is not
    handled (the values here are far from it)."""
    frac, emin = {"bf16": (7, -126), "f16": (10, -14)}[fmt]
    x = np.asarray(x, np.float64)
    _, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    E = np.maximum(e - 1, emin)
    q = np.ldexp(1.0, E - frac)
    return np.where(x == 0.0, x, np.rint(x / q) * q)


# --------------------------------------------------------------------------
# steps
# --------------------------------------------------------------------------

def classify(rays, ids, tmax, aabb):
    """Class per query and the binary32 segment [t_a, t_b] (Sec. 3.1, slab
    test in binary32 without contraction)."""
    rays = np.asarray(rays, np.float32)
    tmax = np.asarray(tmax, np.float32)
    ids = np.asarray(ids, np.int64)
    n = ids.shape[0]
    K = aabb.shape[0]
    o, d = rays[:, :3], rays[:, 3:]
    valid = np.isfinite(o).all(1) & np.isfinite(d).all(1) & (d != 0).any(1) & ~np.isnan(tmax) & (tmax >= 0)
    valid &= (ids >= 0) & (ids < K)
    box = np.asarray(aabb, np.float32)[np.clip(ids, 0, K - 1)]
    lo, hi = box[:, :3], box[:, 3:]
    tn = np.full(n, -np.inf, np.float32)
    tf = np.full(n, np.inf, np.float32)
    empty = np.zeros(n, bool)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            par = d[:, a] == 0
            empty |= par & ((o[:, a] < lo[:, a]) | (o[:, a] > hi[:, a]))
            t0 = np.float32(lo[:, a] - o[:, a]) / d[:, a]
            t1 = np.float32(hi[:, a] - o[:, a]) / d[:, a]
            l, h = np.minimum(t0, t1), np.maximum(t0, t1)
            tn = np.where(par, tn, np.maximum(tn, l))
            tf = np.where(par, tf, np.minimum(tf, h))
    ta = np.maximum(tn, np.float32(0))
    tb = np.minimum(tf, tmax)
    hit = ~empty & (ta <= tb)
    inside = ((o > lo) & (o < hi)).all(1)
    cls = np.where(~valid, CLS_INVALID, np.where(~hit, CLS_MISS, np.where(inside, CLS_INNER, CLS_OUTER)))
    return cls, ta, tb


def sph(q):
    """(u, v) in [0, 1]^2 of the spherical angles of the rows of q (binary64);
    the polar angle as atan2(sqrt(x^2 + y^2), z), well conditioned everywhere."""
    q = np.asarray(q, np.float64)
    theta = np.arctan2(np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]), q[:, 2])  # polar angle, 0 for q = 0
    phi = np.arctan2(q[:, 1], q[:, 0])
    u = np.clip(theta / math.pi, 0.0, 1.0)
    v = np.clip((phi + math.pi) / (2.0 * math.pi), 0.0, 1.0)
    return u, v


def transform(rays, ids, tmax, aabb):
    """Eq. 2 / Eq. 4: class, (pu, pv), (du, dv), r per query (binary64)."""
    cls, ta, _ = classify(rays, ids, tmax, aabb)
    rays64 = np.asarray(rays, np.float32).astype(np.float64)
    o, d = rays64[:, :3], rays64[:, 3:]
    K = aabb.shape[0]
    box = np.asarray(aabb, np.float32).astype(np.float64)[np.clip(np.asarray(ids, np.int64), 0, K - 1)]
    c = 0.5 * (box[:, :3] + box[:, 3:])
    h = 0.5 * (box[:, 3:] - box[:, :3])
    t = np.where(cls == CLS_OUTER, ta.astype(np.float64), 0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        p = o + t[:, None] * d
        q = np.where(np.isfinite(p), (p - c) / h, 0.0)
    pu, pv = sph(q)
    du, dv = sph(np.where(np.isfinite(d), d, 1.0))
    r = np.clip(np.sqrt((q * q).sum(1)) / math.sqrt(3.0), 0.0, 1.0)
    return cls, pu, pv, du, dv, r


def bilinear(G, u, v):
    """Rows of G (R x R x N, binary64) interpolated at (u, v), vertex-aligned."""
    R = G.shape[0]
    su, sv = u * (R - 1), v * (R - 1)
    a = np.minimum(np.floor(su), R - 2).astype(np.int64)
    b = np.minimum(np.floor(sv), R - 2).astype(np.int64)
    wa, wb = (su - a)[:, None], (sv - b)[:, None]
    return ((1 - wa) * (1 - wb) * G[a, b] + wa * (1 - wb) * G[a + 1, b] + (1 - wa) * wb * G[a, b + 1]
            + wa * wb * G[a + 1, b + 1])


def linear(G, r):
    """Rows of G (R x N) interpolated at r in [0, 1], vertex-aligned."""
    R = G.shape[0]
    s = r * (R - 1)
    a = np.minimum(np.floor(s), R - 2).astype(np.int64)
    w = (s - a)[:, None]
    return (1 - w) * G[a] + w * G[a + 1]


def leaky(a):
    return np.where(a > 0, a, LEAKY * a)


def split_weights(w, network: int):
    w = np.asarray(w, np.float64)
    mats, off = [], 0
    for o_, i_ in layer_shapes(network):
        mats.append(w[off:off + o_ * i_].reshape(o_, i_))
        off += o_ * i_
    assert off == w.size, "weight count does not match the network"
    return mats


def mlp(x, w, network: int, quant: str = "exact"):
    """Logit z of the rows of x (n x din) through the network's MLP."""
    return mlp_mats(x, split_weights(w, network), quant)


def mlp_mats(x, mats, quant: str = "exact"):
    """Logit of the rows of x through hidden matrices mats[:-1] (leaky ReLU
    after each) and the output row mats[-1]."""
    H = len(mats) - 1
    rnd = (lambda a: a) if quant == "exact" else (lambda a: round_to(a, quant))
    h = rnd(x)
    for j in range(H):
        a = h @ rnd(mats[j]).T
        h = leaky(a)
        if j < H - 1:
            h = rnd(h)
    return h @ mats[H][0]


def lowp_bound(x, w, network: int, fmt: str):
    """Per-query bound on |y - y_exact| of the bf16 / f16 forms, by first-order
    propagation of the rounding errors through the layers:
      D_0 = (u + 2^-20) |x| + a      (input rounding, plus binary32 feature error)
      E_j = |W_j| D_(j-1) + (u + g_K (1 + u)) |W_j| |h_(j-1)|   (pre-activation)
      D_j = E_j + u |h_j| + a        (activation rounding, j < H; D_H = E_H)
      |dz| <= |w_out| E_H + g_W |w_out| |h_H|,  |dy| <= |dz| / 4
    with u the unit roundoff of fmt (2^-8 bf16, 2^-11 f16), a its subnormal
    half-spacing, g_K = K 2^-24 / (1 - K 2^-24) for binary32 sums of K terms;
    the leaky ReLU is 1-Lipschitz and the sigmoid's slope is at most 1/4.
    h_j are the rounded activations of the emulated forward."""
    u, a = {"bf16": (2.0 ** -8, 2.0 ** -134), "f16": (2.0 ** -11, 2.0 ** -25)}[fmt]
    gam = lambda k: k * 2.0 ** -24 / (1 - k * 2.0 ** -24)
    mats = split_weights(w, network)
    H = len(mats) - 1
    x = np.asarray(x, np.float64)
    h = round_to(x, fmt)
    D = (u + 2.0 ** -20) * np.abs(x) + a
    E = None
    for j in range(H):
        Wj = mats[j]
        aW = np.abs(Wj)
        E = D @ aW.T + (u + gam(Wj.shape[1]) * (1 + u)) * (np.abs(h) @ aW.T)
        hn = leaky(h @ round_to(Wj, fmt).T)
        if j < H - 1:
            hn = round_to(hn, fmt)
            D = E + u * np.abs(hn) + a
        h = hn
    wo = np.abs(mats[H][0])
    dz = E @ wo + gam(wo.size) * (np.abs(h) @ wo)
    return dz / 4.0


def _corners2d(R, u, v):
    """Vertex indices (a, b) and weights of the four corners, order (0,0),
    (1,0), (0,1), (1,1), of a vertex-aligned bilinear lookup."""
    su, sv = u * (R - 1), v * (R - 1)
    a = np.minimum(np.floor(su), R - 2).astype(np.int64)
    b = np.minimum(np.floor(sv), R - 2).astype(np.int64)
    wa, wb = su - a, sv - b
    return [(a, b, (1 - wa) * (1 - wb)), (a + 1, b, wa * (1 - wb)), (a, b + 1, (1 - wa) * wb), (a + 1, b + 1, wa * wb)]


def leaky_grad(a):
    """Derivative of the leaky ReLU, the slope at a = 0."""
    return np.where(a > 0, 1.0, LEAKY)


def train_grads(network: int, rays, ids, tmax, labels, aabb, grids, w, grad_y=None):
    """L2 training loss of `network` (Sec. 5 "Training": L2 loss) over the
    queries of its class, L = (1/B) sum (y - t)^2 with t = label (1 visible),
    and its gradients by back-propagation (Fig. 2: the latents are trained
    with the MLP): returns (loss, B, dW flat like w, per-object grid
    gradients as arrays of grid_shapes).  With grad_y (dL/dy per query) the
    gradients are those of that upstream gradient instead (dL/dz = g y (1 - y),
    no labels, no 1/B) and the loss is None."""
    cls, pu, pv, du, dv, r = transform(rays, ids, tmax, aabb)
    want = CLS_OUTER if network == 0 else CLS_INNER
    s = np.nonzero(cls == want)[0]
    B = s.size
    mats = split_weights(w, network)
    H = len(mats) - 1
    K = len(grids)
    ggrids = [[np.zeros(sh) for sh in grid_shapes(network)] for _ in range(K)]
    dW = [np.zeros_like(m) for m in mats]
    if B == 0:
        return 0.0, 0, np.concatenate([d.ravel() for d in dW]), ggrids
    ids_s = np.asarray(ids, np.int64)[s]
    _, x = features(network, rays, ids, tmax, aabb, grids)
    x = x[s]
    t = None if grad_y is not None else (np.asarray(labels)[s] != 0).astype(np.float64)
    hs, acts = [x], []
    h = x
    for j in range(H):
        a = h @ mats[j].T
        acts.append(a)
        h = leaky(a)
        hs.append(h)
    z = h @ mats[H][0]
    y = 1.0 / (1.0 + np.exp(-z))
    if grad_y is not None:
        loss = None
        dz = np.asarray(grad_y, np.float64)[s] * y * (1.0 - y)
    else:
        loss = float(np.mean((y - t) ** 2))
        dz = 2.0 * (y - t) / B * y * (1.0 - y)
    dW[H][0] = dz @ hs[H]
    delta = dz[:, None] * mats[H][0][None, :] * leaky_grad(acts[H - 1])
    for j in range(H - 1, -1, -1):
        dW[j] = delta.T @ hs[j]
        back = delta @ mats[j]
        if j > 0:
            delta = back * leaky_grad(acts[j - 1])
    gx = back  # dL/dx, n x din
    R, N = (OUTER["R"], OUTER["N"]) if network == 0 else (INNER["R"], INNER["N"])
    for k in range(K):
        sel = np.nonzero(ids_s == k)[0]
        if sel.size == 0:
            continue
        for gi, (uu, vv, cols) in enumerate(((pu[s][sel], pv[s][sel], slice(0, N)),
                                             (du[s][sel], dv[s][sel], slice(N, 2 * N)))):
            for a, b, wt in _corners2d(R, uu, vv):
                np.add.at(ggrids[k][gi], (a, b), wt[:, None] * gx[sel][:, cols])
        if network == 1:
            R1 = INNER["R1"]
            sr = r[s][sel] * (R1 - 1)
            a = np.minimum(np.floor(sr), R1 - 2).astype(np.int64)
            wr = sr - a
            g1 = gx[sel][:, 2 * N:]
            np.add.at(ggrids[k][2], a, (1 - wr)[:, None] * g1)
            np.add.at(ggrids[k][2], a + 1, wr[:, None] * g1)
    return loss, B, np.concatenate([d.ravel() for d in dW]), ggrids


def transform32(rays, ids, tmax, aabb):
    """transform() with every step in binary32 (numpy float32: the entry point,
    q = (p - c) / h, the angles and r), for sizing how far a binary32
    evaluation of the same definitions can move the features."""
    cls, ta, _ = classify(rays, ids, tmax, aabb)
    f = np.float32
    r32 = np.asarray(rays, np.float32)
    o, d = r32[:, :3], r32[:, 3:]
    K = aabb.shape[0]
    box = np.asarray(aabb, np.float32)[np.clip(np.asarray(ids, np.int64), 0, K - 1)]
    c = (box[:, :3] + box[:, 3:]) * f(0.5)
    h = (box[:, 3:] - box[:, :3]) * f(0.5)
    t = np.where(cls == CLS_OUTER, ta, f(0)).astype(np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        p = (o + t[:, None] * d).astype(np.float32)
        q = np.where(np.isfinite(p), (p - c) / h, f(0)).astype(np.float32)

    def sph32(v):
        theta = np.arctan2(np.sqrt(v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]), v[:, 2])
        phi = np.arctan2(v[:, 1], v[:, 0])
        return (np.clip(theta / f(math.pi), 0, 1).astype(np.float64),
                np.clip((phi + f(math.pi)) / f(2 * math.pi), 0, 1).astype(np.float64))
    pu, pv = sph32(q)
    du, dv = sph32(np.where(np.isfinite(d), d, f(1)).astype(np.float32))
    r = np.clip(np.sqrt((q * q).sum(1)) / f(math.sqrt(3.0)), 0, 1).astype(np.float64)
    return cls, pu, pv, du, dv, r


def kink_ambiguous(network: int, rays, ids, tmax, aabb, grids, w, factor: float = 8.0):
    """Per query of `network`'s class: True when some hidden pre-activation a
    lies so close to the leaky ReLU's kink that a binary32 evaluation may put
    it on the other side, so that the query's backward pass (the slope, Sec. 5
    "Architecture") may differ from the binary64 one.  The margin of unit i of
    layer j is factor x (|a32 - a64| + g_K sum_k |W_ik h_k|): a32 from the
    features of transform32, a64 from the binary64 ones, plus the worst-case
    drift of a K-term binary32 sum (g_K = K 2^-24 / (1 - K 2^-24)).  Queries
    of other classes are False."""
    cls, x64 = features(network, rays, ids, tmax, aabb, grids)
    x32 = features(network, rays, ids, tmax, aabb, grids, coords=transform32(rays, ids, tmax, aabb))[1]
    s = np.nonzero(cls == (CLS_OUTER if network == 0 else CLS_INNER))[0]
    mats = split_weights(w, network)
    out = np.zeros(cls.shape[0], bool)
    h64, h32 = x64[s], x32[s]
    near = np.zeros(s.size, bool)
    for m in mats[:-1]:
        a64, a32 = h64 @ m.T, h32 @ m.T
        K = m.shape[1]
        g = K * 2.0 ** -24 / (1 - K * 2.0 ** -24)
        margin = factor * (np.abs(a32 - a64) + g * (np.abs(h64) @ np.abs(m).T))
        near |= (np.abs(a64) <= margin).any(1)
        h64, h32 = leaky(a64), leaky(a32)
    out[s] = near
    return out


def features(network: int, rays, ids, tmax, aabb, grids, coords=None):
    """Class per query and the MLP input x (n x din) of `network`; rows of
    other classes are zero.  grids: per object, the binary64 arrays of
    grid_shapes(network).  coords: the output of transform() to use (default:
    transform() of the queries)."""
    cls, pu, pv, du, dv, r = transform(rays, ids, tmax, aabb) if coords is None else coords
    want = CLS_OUTER if network == 0 else CLS_INNER
    n = cls.shape[0]
    x = np.zeros((n, din(network)))
    ids = np.asarray(ids, np.int64)
    for k in range(len(grids)):
        s = np.nonzero((cls == want) & (ids == k))[0]
        if s.size == 0:
            continue
        g = grids[k]
        parts = [bilinear(g[0], pu[s], pv[s]), bilinear(g[1], du[s], dv[s])]
        if network == 1:
            parts.append(linear(g[2], r[s]))
        x[s] = np.concatenate(parts, axis=1)
    return cls, x


def forward(rays, ids, tmax, aabb, grids_outer, grids_inner, w_outer, w_inner, quant: str = "exact"):
    """Visibility y, logit z and class per query (Sec. 4.1: outer queries
    through the outer network, inner queries through the inner one; a miss
    is visible with z = +inf; invalid queries give NaN)."""
    n = np.asarray(ids).shape[0]
    y = np.full(n, np.nan)
    z = np.full(n, np.nan)
    cls = None
    for net, grids, w in ((0, grids_outer, w_outer), (1, grids_inner, w_inner)):
        cls, x = features(net, rays, ids, tmax, aabb, grids)
        s = np.nonzero(cls == (CLS_OUTER if net == 0 else CLS_INNER))[0]
        if s.size:
            z[s] = mlp(x[s], w, net, quant)
            y[s] = 1.0 / (1.0 + np.exp(-z[s]))
    miss = cls == CLS_MISS
    y[miss], z[miss] = 1.0, np.inf
    return {"y": y, "z": z, "cls": cls}
