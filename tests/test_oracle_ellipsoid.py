"""Ellipsoids (smooth convex bodies, Sec. 1 and Sec. 3.3: the method needs
only a signed distance) in the FP64 oracle.

Pins, none of which re-evaluates the oracle's own formula:
  * equal semi-axes reduce to the sphere, |p| - a, gradient p / |p|;
  * brute force: the nearest point of a dense (theta, phi) surface grid,
    refined by a bounded minimiser, gives |d| within 1e-9 and the sign of the
    inside test sum (p_k / e_k)^2 < 1, at random points inside and outside
    and on the symmetry planes and axes (the degenerate branches);
  * closed forms: beyond an axis tip the distance is y_k - e_k; at the
    centre it is minus the shortest semi-axis;
  * the gradient agrees with central differences of the distance;
  * volume and second moment against a midpoint-rule integral of the
    indicator; circumradius the longest semi-axis;
  * the half extent along a world axis against the largest world coordinate
    over a dense surface sample.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

T_E = 6          # type slots used here (the polyhedron tests use 0..4, 7)
AXES = [(1.0, 0.6, 0.35), (2.0, 1.0, 1.0), (0.5, 0.5, 1.2), (0.8, 1.3, 0.8),
        (1.0, 1.0, 0.5)]
IDENT = np.array([1.0, 0.0, 0.0, 0.0])


def _define(O, axes, t=T_E):
    O.define_ellipsoid(t, axes)
    return O.POLY0 + t


def _surface(axes, th, ph):
    a, b, c = axes
    return np.stack([a * np.sin(th) * np.cos(ph), b * np.sin(th) * np.sin(ph),
                     c * np.cos(th)], axis=-1)


def _brute(axes, y):
    """Nearest surface point of y by grid search and bounded refinement."""
    th = np.linspace(0.0, math.pi, 181)
    ph = np.linspace(-math.pi, math.pi, 361)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    S = _surface(axes, TH, PH)
    D2 = ((S - y) ** 2).sum(-1)
    best = None
    for idx in np.argsort(D2, axis=None)[:8]:
        i, j = np.unravel_index(idx, D2.shape)
        f = lambda v: float(((_surface(axes, v[0], v[1]) - y) ** 2).sum())
        r = minimize(f, [TH[i, j], PH[i, j]], method="L-BFGS-B",
                     bounds=[(0.0, math.pi), (-math.pi, math.pi)],
                     options=dict(ftol=1e-300, gtol=1e-14, maxiter=500))
        if best is None or r.fun < best[0]:
            best = (r.fun, _surface(axes, r.x[0], r.x[1]))
    return math.sqrt(max(best[0], 0.0)), best[1]


def _points(rng, axes, n):
    e = np.asarray(axes)
    pts = [rng.uniform(-2.0, 2.0, 3) * e for _ in range(n)]
    # symmetry planes and axes: the branches where components vanish
    for k in range(3):
        p = rng.uniform(-1.5, 1.5, 3) * e
        p[k] = 0.0
        pts.append(p)
        q = np.zeros(3)
        q[k] = rng.uniform(0.05, 0.9) * e[k]
        pts.append(q)
        pts.append(-q)
    pts.append(np.array([0.1 * e[0], 0.0, 0.0]))
    pts.append(np.array([0.0, 0.05 * e[1], 0.0]))
    return pts


def test_equal_axes_reduce_to_sphere(O):
    sh = _define(O, (1.3, 1.3, 1.3))
    rng = np.random.default_rng(1)
    for _ in range(200):
        r = rng.uniform(-6.0, 6.0, 3)
        size = rng.uniform(0.5, 4.0)
        d, g = O.sdf(sh, size, IDENT, r, want_grad=True)
        n = np.linalg.norm(r)
        assert abs(d - (n - 1.3 * size)) <= 4e-15 * max(n, 1.3 * size)
        assert np.allclose(g, r / n, atol=1e-13)


@pytest.mark.parametrize("axes", AXES)
def test_distance_brute_force(O, axes):
    sh = _define(O, axes)
    rng = np.random.default_rng(7)
    e = np.asarray(axes)
    for y in _points(rng, axes, 24):
        d = O.sdf(sh, 1.0, IDENT, y)
        bd, x = _brute(axes, y)
        inside = ((y / e) ** 2).sum() < 1.0
        assert abs(abs(d) - bd) <= 1e-9, (y, d, bd)
        assert (d < 0.0) == inside, (y, d)


@pytest.mark.parametrize("axes", AXES)
def test_axis_tips_and_centre(O, axes):
    sh = _define(O, axes)
    e = np.asarray(axes)
    assert O.sdf(sh, 1.0, IDENT, np.zeros(3)) == pytest.approx(-e.min(), abs=1e-15)
    for k in range(3):
        for s in (1.0, -1.0):
            for out in (1e-6, 0.3, 2.0):
                y = np.zeros(3)
                y[k] = s * (e[k] + out)
                d, g = O.sdf(sh, 1.0, IDENT, y, want_grad=True)
                assert d == pytest.approx(out, rel=1e-9, abs=1e-15)
                assert g[k] == pytest.approx(s, abs=1e-12)


@pytest.mark.parametrize("axes", AXES)
def test_gradient_matches_differences(O, axes):
    sh = _define(O, axes)
    rng = np.random.default_rng(11)
    e = np.asarray(axes)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    h = 1e-6
    for _ in range(40):
        r = rng.uniform(-2.0, 2.0, 3) * e.max()
        d, g = O.sdf(sh, 1.7, q, r, want_grad=True)
        if d < -0.5 * e.min() * 1.7:
            continue          # deep inside: near the medial axis
        fd = np.array([(O.sdf(sh, 1.7, q, r + h * u) - O.sdf(sh, 1.7, q, r - h * u)) / (2 * h)
                       for u in np.eye(3)])
        assert np.allclose(g, fd, atol=2e-6), (r, g, fd)
        assert abs(np.linalg.norm(g) - 1.0) <= 1e-12


@pytest.mark.parametrize("axes", AXES[:2])
def test_volume_and_second_moment(O, axes):
    sh = _define(O, axes)
    vol, J, rc, _ = O.polyhedron_info(T_E, 0)
    e = np.asarray(axes)
    assert rc == e.max()
    n = 64
    gs = [(np.arange(n) + 0.5) / n * 2 * e[k] - e[k] for k in range(3)]
    X, Y, Z = np.meshgrid(*gs, indexing="ij")
    P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    ins = np.array([O.sdf(sh, 1.0, IDENT, p) < 0.0 for p in P[::7]])
    # every 7th node for the indicator (the rest by the same sampling rate)
    Ps = P[::7]
    dV = (2 * e[0] / n) * (2 * e[1] / n) * (2 * e[2] / n) * 7
    V = ins.sum() * dV
    Jn = (Ps[ins][:, :, None] * Ps[ins][:, None, :]).sum(0) * dV
    assert V == pytest.approx(vol, rel=5e-3)
    assert vol == pytest.approx(4.0 / 3.0 * math.pi * e.prod(), rel=1e-15)
    for k in range(3):
        assert Jn[k, k] == pytest.approx(J[k, k], rel=1e-2)
    assert abs(J - np.diag(np.diag(J))).max() == 0.0


def test_half_extent_is_surface_maximum(O):
    axes = (1.0, 0.6, 0.35)
    sh = _define(O, axes)
    rng = np.random.default_rng(3)
    th = np.linspace(0.0, math.pi, 401)
    ph = np.linspace(-math.pi, math.pi, 801)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    S = _surface(axes, TH, PH).reshape(-1, 3)
    for _ in range(5):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = O.rotation(q)
        W = S @ R.T * 2.5
        for k in range(3):
            he = O.half_extent(sh, 2.5, q, k)
            m = np.abs(W[:, k]).max()
            assert m <= he * (1 + 1e-12)
            assert he - m <= 1e-4 * he


def test_malformed_ellipsoid_rejected(O):
    with pytest.raises(ValueError, match="semi-axes"):
        O.define_ellipsoid(T_E, (1.0, 0.0, 1.0))
    with pytest.raises(ValueError, match="type"):
        O.define_ellipsoid(8, (1.0, 1.0, 1.0))
