"""The compulsory-byte count behind the bench line's HBM roofline: the
distinct grid vertices that the trilinear lookups of a set of queries touch
(object, table, level, vertex), counted by bench.latent_footprint, against a
plain per-query enumeration of the eight corners of every lookup."""
import math

import numpy as np

import bench
from paper_2306_07191_amd import synth as S


def _brute(rays, tmax, ids, aabb, res):
    seen, lines = set(), set()
    for r, tm, k in zip(rays.astype(np.float64), tmax.astype(np.float64), ids):
        lo, hi = aabb[k, :3].astype(np.float64), aabb[k, 3:].astype(np.float64)
        o, d = r[:3], r[3:]
        ta, tb = 0.0, tm
        for a in range(3):
            if d[a] == 0.0:
                continue
            t1, t2 = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
            ta, tb = max(ta, min(t1, t2)), min(tb, max(t1, t2))
        if not ta <= tb:
            continue
        ext = hi - lo
        us = [np.clip((o + ta * d - lo) / ext, 0, 1), np.clip((o + tb * d - lo) / ext, 0, 1),
              np.clip((d / math.sqrt((d * d).sum()) + 1) * 0.5, 0, 1)]
        for t, u in enumerate(us):
            for l, N in enumerate(res):
                c = np.minimum(np.floor(u * N).astype(np.int64), N - 1)
                for cz in (0, 1):
                    for cy in (0, 1):
                        for cx in (0, 1):
                            v = ((c[2] + cz) * (N + 1) + (c[1] + cy)) * (N + 1) + (c[0] + cx)
                            seen.add((int(k), t, l, int(v)))
                            lines.add((int(k), t, l, int(v) * 2 * 2 // 64))
    return len(seen), len(lines)


def test_latent_footprint_matches_enumeration():
    import torch
    g = np.random.default_rng(3)
    boxes = np.array([[-1, -1, -1, 1, 1, 1], [2, 0, 0, 3, 1, 2]], np.float32)
    n = 400
    ids = g.integers(0, 2, n).astype(np.int32)
    rays = np.empty((n, 6), np.float32)
    tmax = np.empty(n, np.float32)
    for k in range(2):
        s = np.nonzero(ids == k)[0]
        ctr = 0.5 * (boxes[k, :3] + boxes[k, 3:])
        rays[s], tmax[s] = S.rays_sphere_to_box(s.size, boxes[k], g, radius=4.0, center=ctr)
    rays[::13, 3:] *= -1.0  # misses
    res = [4, 7, 16]
    got = bench.latent_footprint(torch.from_numpy(rays), torch.from_numpy(tmax), torch.from_numpy(ids), boxes, res,
                                 2, 2)
    verts, lines = _brute(rays, tmax, ids, boxes, res)
    assert got[0] == verts and got[1] == verts * 4 and got[2] == lines
    assert verts > 1000
