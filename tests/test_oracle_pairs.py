"""Pins of the oracle's pair expansion and per-ray combination (Sec. 4.1): hand
cases and a binary64 slab test on rays far from grazing."""
import numpy as np

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

BOXES = np.array([[0, 0, 0, 1, 1, 1],      # A
                  [2, 0, 0, 3, 1, 1],      # B
                  [0, 5, 0, 1, 6, 1]],     # C
                 np.float32)


def _model(boxes):
    K = boxes.shape[0]
    return O.Model(S.TINY, boxes, S.xavier_mlp(S.TINY, S.rng(1, 3))[None], mlp_index=np.zeros(K, np.int32))


def test_pairs_hand_cases():
    rays = np.array([[-1, 0.5, 0.5, 1, 0, 0],     # through A then B
                     [-1, 0.5, 0.5, 1, 0, 0],     # same, t_max 2.5 ends before B (entered at t = 3)
                     [0.5, 0.5, -5, 0, 0, 1],     # A only
                     [10, 10, 10, 1, 0, 0],       # nothing
                     [0.5, 0.5, 0.5, 0, 0, 1],    # starts inside A
                     [0.5, -1, 0.5, 0, 1, 0],     # A and C
                     [0.5, -1, 0.5, 0, 1, 0]],    # t_max 3: A only
                    np.float32)
    tmax = np.array([np.inf, 2.5, np.inf, np.inf, np.inf, np.inf, 3.0], np.float32)
    pr, po = _model(BOXES).expand_pairs(rays, tmax)
    assert list(zip(pr.tolist(), po.tolist())) == [(0, 0), (0, 1), (1, 0), (2, 0), (4, 0), (5, 0), (5, 2), (6, 0)]


def test_pairs_match_binary64_slab_test():
    g = np.random.default_rng(3)
    boxes = np.concatenate([g.uniform(-3, 2, (6, 3)), np.zeros((6, 3))], axis=1)
    boxes[:, 3:] = boxes[:, :3] + g.uniform(0.3, 1.5, (6, 3))
    boxes = boxes.astype(np.float32)
    n = 3000
    o = g.uniform(-5, 5, (n, 3))
    k = g.integers(0, 6, n)  # aim at a point of a random box
    tgt = boxes[k, :3] + g.uniform(size=(n, 3)) * (boxes[k, 3:] - boxes[k, :3])
    d = tgt - o
    rays = np.concatenate([o, d], axis=1).astype(np.float32)
    tmax = np.where(g.uniform(size=n) < 0.5, np.inf, g.uniform(0.5, 8, n)).astype(np.float32)
    o64, d64 = rays[:, :3].astype(np.float64), rays[:, 3:].astype(np.float64)
    lo, hi = boxes[:, :3].astype(np.float64), boxes[:, 3:].astype(np.float64)
    t0 = (lo[None] - o64[:, None]) / d64[:, None]
    t1 = (hi[None] - o64[:, None]) / d64[:, None]
    tn = np.minimum(t0, t1).max(axis=2)
    tf = np.maximum(t0, t1).min(axis=2)
    ta, tb = np.maximum(tn, 0), np.minimum(tf, tmax.astype(np.float64)[:, None])
    margin = tb - ta
    clear = np.abs(margin) > 1e-4 * (1 + np.abs(ta) + np.abs(tb))  # not near grazing or t_max
    pr, po = _model(boxes).expand_pairs(rays, tmax)
    got = np.zeros((n, 6), bool)
    got[pr, po] = True
    assert np.array_equal(got[clear], (margin >= 0)[clear])
    assert clear.mean() > 0.99 and got.sum() > 500


def test_combine_hand_cases():
    pair_ray = np.array([0, 0, 2, 3, 3])
    vis = np.array([0.9, 0.7, 0.2, 0.5, 0.49])
    np.testing.assert_array_equal(O.combine_pairs(pair_ray, vis, 5), [1, 1, 0, 0, 1])
