"""Pins of the light importance sampling oracle (Sec. 5 "Training": training
ray directions drawn in proportion to radiant flux with a tabulated CDF and
bisection) against closed forms and Monte Carlo identities."""
import math

import numpy as np

from oracle import light_sampling as LS


def _tri(p0, p1, p2):
    return np.array([*p0, *p1, *p2], np.float32)


def test_cdf_table_and_pick_closed_form():
    """Four unit right triangles with radiance 1..4: fluxes pi/2 (1, 2, 3, 4),
    CDF (0.1, 0.3, 0.6, 1); the pick is the first entry above u0."""
    tris = np.stack([_tri((k, 0, 0), (k + 1, 0, 0), (k, 1, 0)) for k in range(4)])
    rad = np.array([1, 2, 3, 4], np.float32)
    np.testing.assert_allclose(LS.flux(tris, rad), math.pi / 2 * np.array([1, 2, 3, 4]), rtol=1e-15)
    tab = LS.cdf_table(tris, rad)
    np.testing.assert_array_equal(tab, np.float32([0.1, 0.3, 0.6, 1.0]))
    u0 = np.float32([0.0, 0.05, 0.1, 0.2999, 0.3, 0.6, 0.99999994])
    assert list(LS.pick(tab, u0)) == [0, 0, 1, 1, 2, 3, 3]


def test_pick_frequencies_follow_flux():
    g = np.random.default_rng(1)
    L = 12
    tris = np.stack([_tri((k, 0, 0), (k + g.uniform(0.5, 2), 0, 0), (k, g.uniform(0.5, 2), 0)) for k in range(L)])
    rad = g.uniform(0.1, 5.0, L).astype(np.float32)
    f = LS.flux(tris, rad)
    n = 400000
    idx = LS.pick(LS.cdf_table(tris, rad), g.uniform(size=n).astype(np.float32))
    freq = np.bincount(idx, minlength=L) / n
    p = f / f.sum()
    assert np.all(np.abs(freq - p) <= 5 * np.sqrt(p * (1 - p) / n))


def test_points_are_uniform_on_the_triangle():
    """Barycentric weights are non-negative and sum to 1; the sample mean is the
    centroid, and the mass of the sub-triangle at vertex 0 cut at half height is 1/4."""
    tri = _tri((0, 0, 0), (4, 0, 0), (0, 2, 1))
    g = np.random.default_rng(2)
    n = 200000
    out = LS.sample(tri[None], np.ones(1, np.float32), np.tile([0.0, 0.0, 10.0], (n, 1)),
                    g.uniform(size=(n, 3)).astype(np.float32))
    b = out["bary"]
    assert (b >= -1e-12).all() and np.allclose(b.sum(1), 1.0)
    centroid = tri.reshape(3, 3).astype(np.float64).mean(0)
    assert np.all(np.abs(out["point"].mean(0) - centroid) < 5 * out["point"].std(0) / np.sqrt(n))
    frac = (b[:, 0] > 0.5).mean()  # the corner region b0 > 1/2 holds a quarter of the area
    assert abs(frac - 0.25) < 5 * math.sqrt(0.25 * 0.75 / n)


def test_pdf_integrates_to_the_solid_angle():
    """E[1 / pdf] over directions drawn from one light triangle is the solid angle
    it subtends (Van Oosterom-Strackee closed form), within Monte Carlo error;
    directions are unit and t_max reaches the light point."""
    tri = _tri((-1, 3, -1), (2, 3, -0.5), (0, 3.5, 2))
    x = np.array([0.2, 0.0, 0.1])
    g = np.random.default_rng(3)
    n = 200000
    out = LS.sample(tri[None], np.full(1, 2.0, np.float32), np.tile(x, (n, 1)), g.uniform(size=(n, 3)).astype(np.float32))
    inv = 1.0 / out["pdf"]
    est, err = inv.mean(), inv.std() / np.sqrt(n)
    om = LS.triangle_solid_angle(x, tri)
    assert abs(est - om) < 5 * err, (est, om, err)
    assert np.allclose(np.linalg.norm(out["d"], axis=1), 1.0)
    np.testing.assert_allclose(out["o"] + out["tmax"][:, None] * out["d"], out["point"], atol=1e-12)


def test_solid_angle_formula_closed_form():
    """A triangle that is one face of an octant (vertices on the three axes) seen
    from the origin covers 4 pi / 8."""
    om = LS.triangle_solid_angle(np.zeros(3), _tri((1, 0, 0), (0, 1, 0), (0, 0, 1)))
    assert abs(om - 4 * math.pi / 8) < 1e-12
