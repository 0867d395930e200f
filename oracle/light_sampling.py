"""Binary64 oracle of light importance sampling for training rays (Sec. 5
"Training": ray directions drawn by light importance sampling according to
radiant flux, with a tabulated CDF searched by bisection; Sec. 6 "Comparison
of Sampling Method").

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.

Steps, in the paper's order:
1. Radiant flux of every emitting triangle: a Lambertian emitter of radiance
   L and area A emits pi L A.
2. Tabulated CDF: running sums of the fluxes in triangle order (binary64),
   divided by the total, stored as binary32 (the table both sides search), the
   last entry set to 1.
3. Triangle of a sample: the first i with cdf[i] > u0 (u0 in [0, 1), a
   binary32 comparison on both sides, since it decides an integer).
4. Point: uniform on the triangle, v0 + b1 (v1 - v0) + b2 (v2 - v0) with
   b1 = 1 - sqrt(u1), b2 = u2 sqrt(u1).
5. Shadow ray from the shading point x towards the point: unit direction,
   t_max = the distance, and the solid-angle density of the direction,
   P(i) / A_i * dist^2 / |n_i . d|.

The random numbers (u0, u1, u2) are inputs.
"""
from __future__ import annotations

import numpy as np


def areas_normals(tris):
    """Area and unit normal of each triangle (rows of 9: three vertices),
    cross product (e1 y e2 z - e1 z e2 y, ...) in binary64."""
    t = np.asarray(tris, np.float32).astype(np.float64).reshape(-1, 3, 3)
    e1, e2 = t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]
    c = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                  e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                  e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], axis=1)
    ln = np.sqrt(c[:, 0] * c[:, 0] + c[:, 1] * c[:, 1] + c[:, 2] * c[:, 2])
    return 0.5 * ln, c / ln[:, None]


def flux(tris, radiance):
    """Radiant flux pi L A of each Lambertian emitting triangle."""
    return np.pi * np.asarray(radiance, np.float32).astype(np.float64) * areas_normals(tris)[0]


def cdf_table(tris, radiance):
    """The binary32 CDF table: running sums (binary64, in order) / total."""
    f = flux(tris, radiance)
    run = np.cumsum(f)  # sequential, left to right
    tab = (run / run[-1]).astype(np.float32)
    tab[-1] = np.float32(1.0)
    return tab


def pick(tab, u0):
    """Index of the first table entry greater than u0 (binary32 comparison)."""
    u0 = np.asarray(u0, np.float32)
    i = np.searchsorted(tab, u0, side="right")
    return np.minimum(i, tab.size - 1)


def sample(tris, radiance, points, u):
    """Triangle index, ray (origin x, unit direction), t_max and solid-angle
    density of each sample (binary64 after the binary32 pick)."""
    tab = cdf_table(tris, radiance)
    u = np.asarray(u, np.float32)
    i = pick(tab, u[:, 0])
    t = np.asarray(tris, np.float32).astype(np.float64).reshape(-1, 3, 3)[i]
    su = np.sqrt(u[:, 1].astype(np.float64))
    b1 = 1.0 - su
    b2 = u[:, 2].astype(np.float64) * su
    p = t[:, 0] + b1[:, None] * (t[:, 1] - t[:, 0]) + b2[:, None] * (t[:, 2] - t[:, 0])
    x = np.asarray(points, np.float32).astype(np.float64)
    v = p - x
    dist = np.sqrt((v * v).sum(1))
    d = v / dist[:, None]
    area, nrm = areas_normals(tris)
    f = flux(tris, radiance)
    prob = f[i] / f.sum()
    cos = np.abs((nrm[i] * d).sum(1))
    pdf = prob / area[i] * dist * dist / cos
    return {"tri": i, "o": x, "d": d, "tmax": dist, "pdf": pdf, "point": p, "bary": np.stack([1 - b1 - b2, b1, b2], 1)}


def triangle_solid_angle(x, tri):
    """Solid angle of a triangle seen from x (Van Oosterom and Strackee,
    IEEE Trans. Biomed. Eng. 1983): tan(Omega / 2) = |a . (b x c)| /
    (abc + (a.b)c + (a.c)b + (b.c)a) for the vertex vectors a, b, c from x."""
    v = np.asarray(tri, np.float64).reshape(3, 3) - np.asarray(x, np.float64)[None, :]
    a, b, c = v
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    om = 2.0 * np.arctan2(num, den)
    return om if om >= 0 else om + 2 * np.pi
