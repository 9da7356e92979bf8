"""Pins of the oracle's geometry: rotation, signed distances, coupling weight.

The signed distances are checked against brute-force distances to densely
sampled surfaces, the rotation against scipy, and the weight against its
defining special values.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def _rand_quat(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


@pytest.mark.parametrize("seed", range(4))
def test_rotation_matches_scipy(O, seed):
    rng = np.random.default_rng(seed)
    q = _rand_quat(rng)
    R = O.rotation(q)
    ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    np.testing.assert_allclose(R, ref, atol=1e-15)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-15)


def _cube_surface(a, n):
    """Dense sample of the surface of an axis-aligned cube of edge a."""
    t = (np.arange(n) + 0.5) / n * a - a / 2
    u, v = np.meshgrid(t, t, indexing="ij")
    u, v = u.ravel(), v.ravel()
    pts = []
    for k in range(3):
        for s in (-a / 2, a / 2):
            p = np.zeros((u.size, 3))
            p[:, k] = s
            p[:, (k + 1) % 3] = u
            p[:, (k + 2) % 3] = v
            pts.append(p)
    # edges, densely, so that corner regions are resolved
    e = (np.arange(4 * n) + 0.5) / (4 * n) * a - a / 2
    for k in range(3):
        for s1 in (-a / 2, a / 2):
            for s2 in (-a / 2, a / 2):
                p = np.zeros((e.size, 3))
                p[:, k] = e
                p[:, (k + 1) % 3] = s1
                p[:, (k + 2) % 3] = s2
                pts.append(p)
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1)
                        for sz in (-1, 1)], float) * (a / 2)
    pts.append(corners)
    return np.concatenate(pts)


@pytest.mark.parametrize("seed", range(3))
def test_cube_sdf_brute_force(O, seed):
    """|d| equals the distance to the surface; sign from inside/outside."""
    rng = np.random.default_rng(seed)
    a = 2.0
    q = _rand_quat(rng)
    R = O.rotation(q)
    surf_body = _cube_surface(a, 300)
    surf = surf_body @ R.T
    for _ in range(40):
        r = rng.uniform(-2.0, 2.0, 3)
        d = O.sdf(1, a, q, r)
        dist = np.sqrt(((surf - r) ** 2).sum(1)).min()
        inside = np.all(np.abs(R.T @ r) < a / 2)
        assert (d < 0) == inside
        assert abs(abs(d) - dist) < 2e-4, (r, d, dist)


@pytest.mark.parametrize("seed", range(3))
def test_sphere_sdf_brute_force(O, seed):
    rng = np.random.default_rng(seed)
    R0 = 1.7
    v = rng.standard_normal((400000, 3))
    surf = R0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    q = _rand_quat(rng)
    for _ in range(30):
        r = rng.uniform(-3.0, 3.0, 3)
        d = O.sdf(0, R0, q, r)
        dist = np.sqrt(((surf - r) ** 2).sum(1)).min()
        assert (d < 0) == (np.linalg.norm(r) < R0)
        assert abs(abs(d) - dist) < 5e-3


@pytest.mark.parametrize("shape,size", [(0, 3.0), (1, 5.0), (2, 4.0)])
def test_sdf_gradient_unit_and_fd(O, shape, size):
    """|grad d| = 1, and grad d matches central differences off the ridges."""
    rng = np.random.default_rng(7)
    q = _rand_quat(rng)
    h = 1e-6
    checked = 0
    for _ in range(200):
        r = rng.uniform(-5, 5, 3)
        d, g = O.sdf(shape, size, q, r, want_grad=True)
        assert abs(np.linalg.norm(g) - 1.0) < 1e-12
        fd = np.array([(O.sdf(shape, size, q, r + h * e) -
                        O.sdf(shape, size, q, r - h * e)) / (2 * h)
                       for e in np.eye(3)])
        if shape == 1 and d < 0:
            # inside a cube the gradient jumps across the diagonal planes;
            # skip points close to them
            p = np.abs(O.rotation(q).T @ r)
            srt = np.sort(p)
            if srt[2] - srt[1] < 1e-3:
                continue
        if shape == 2 and np.abs(O.rotation(q).T @ r).min() < 1e-3:
            # the octahedron's gradient flips sign across the body planes
            continue
        np.testing.assert_allclose(g, fd, atol=2e-6)
        checked += 1
    assert checked > 150


def test_sdf_rotation_invariance(O):
    """d(R, r) = d(I, R^T r): the body frame is p = R^T r."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        q = _rand_quat(rng)
        r = rng.uniform(-6, 6, 3)
        R = O.rotation(q)
        d1 = O.sdf(1, 4.0, q, r)
        d2 = O.sdf(1, 4.0, np.array([1.0, 0, 0, 0]), R.T @ r)
        assert abs(d1 - d2) < 1e-13


def test_cube_sdf_special_points(O):
    """Face centre, edge and corner distances of an axis-aligned cube."""
    q = np.array([1.0, 0, 0, 0])
    a = 2.0
    assert O.sdf(1, a, q, [0, 0, 0]) == -1.0
    assert abs(O.sdf(1, a, q, [2.0, 0, 0]) - 1.0) < 1e-15
    assert abs(O.sdf(1, a, q, [2.0, 2.0, 0]) - math.sqrt(2.0)) < 1e-15
    assert abs(O.sdf(1, a, q, [2.0, 2.0, 2.0]) - math.sqrt(3.0)) < 1e-15
    assert abs(O.sdf(1, a, q, [0.5, 0.2, 0]) + 0.5) < 1e-15


def test_weight_special_values(O):
    eps = 1.0
    assert O.weight(-0.5, eps) == 1.0
    assert O.weight(0.5, eps) == 0.0
    assert abs(O.weight(0.0, eps) - 0.5) < 1e-15
    assert O.weight(-3.0, eps) == 1.0 and O.weight(2.0, eps) == 0.0
    ds = np.linspace(-0.6, 0.6, 241)
    B = np.array([O.weight(d, eps) for d in ds])
    assert np.all(np.diff(B) <= 1e-16)            # monotone non-increasing
    # symmetric about the surface: B(d) + B(-d) = 1
    for d in np.linspace(-0.5, 0.5, 21):
        assert abs(O.weight(d, eps) + O.weight(-d, eps) - 1.0) < 1e-15
    # C1 at the band ends: one-sided slopes vanish
    h = 1e-7
    assert abs(O.weight(0.5 - h, eps)) / h < 1e-5
    assert abs(1.0 - O.weight(-0.5 + h, eps)) / h < 1e-5


def _octahedron_surface(a, n):
    """Points of the 8 faces (triangles of vertices a e_i) on a fine grid."""
    pts = []
    for i in range(n + 1):
        for j in range(n + 1 - i):
            u, v = i / n, j / n
            w = 1.0 - u - v
            pts.append([u * a, v * a, w * a])
    tri = np.array(pts)
    out = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                out.append(tri * [sx, sy, sz])
    return np.concatenate(out)


@pytest.mark.parametrize("seed", range(3))
def test_octahedron_sdf_brute_force(O, seed):
    """|d| is the distance to the sampled surface of |x|+|y|+|z| = a (face
    interiors, edges and vertices), the sign that of |x|+|y|+|z| - a."""
    rng = np.random.default_rng(seed)
    a = 2.0
    q = _rand_quat(rng)
    R = O.rotation(q)
    surf = _octahedron_surface(a, 220) @ R.T
    for _ in range(40):
        r = rng.uniform(-3.0, 3.0, 3)
        d = O.sdf(2, a, q, r)
        dist = np.sqrt(((surf - r) ** 2).sum(1)).min()
        inside = np.abs(R.T @ r).sum() < a
        assert (d < 0) == inside
        # the samples lie on the surface (dist >= |d|) and every surface
        # point is within the grid spacing s of a sample
        sp = a * math.sqrt(2.0) / 220
        assert abs(d) <= dist + 1e-12, (r, d, dist)
        assert dist <= math.sqrt(d * d + sp * sp) + 1e-12, (r, d, dist)


def test_octahedron_sdf_special_points(O):
    """Centre, beyond a vertex, beyond an edge midpoint, beyond a face
    centre, of the axis-aligned octahedron |x|+|y|+|z| <= a."""
    q = np.array([1.0, 0, 0, 0])
    a = 3.0
    s3 = math.sqrt(3.0)
    assert abs(O.sdf(2, a, q, [0, 0, 0]) + a / s3) < 1e-15
    assert abs(O.sdf(2, a, q, [a + 0.7, 0, 0]) - 0.7) < 1e-15
    assert abs(O.sdf(2, a, q, [-a - 0.7, 0.2, -0.1]) -
               math.sqrt(0.7 ** 2 + 0.2 ** 2 + 0.1 ** 2)) < 1e-14
    e = np.array([a / 2, a / 2, 0.0]) + 0.4 * np.array([1, 1, 0]) / math.sqrt(2)
    assert abs(O.sdf(2, a, q, e) - 0.4) < 1e-14          # edge region
    f = np.array([a, a, a]) / 3 + 0.25 * np.ones(3) / s3
    assert abs(O.sdf(2, a, q, f) - 0.25) < 1e-14         # face region
    assert abs(O.sdf(2, a, q, -f) - 0.25) < 1e-14


def test_octahedron_volume_and_inertia(O, W):
    """V = 4 a^3 / 3 and I = m a^2 / 5 against a midpoint-rule integral of
    the indicator of |x|+|y|+|z| <= a (the oracle uses them for the mass and
    inertia of the particle update)."""
    a, n = 1.0, 160
    h = 2 * a / n
    g = -a + h * (np.arange(n) + 0.5)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    ins = (np.abs(X) + np.abs(Y) + np.abs(Z)) <= a
    V = ins.sum() * h ** 3
    assert abs(V - 4 * a ** 3 / 3) < 2e-3
    Ixx = ((Y ** 2 + Z ** 2) * ins).sum() * h ** 3
    assert abs(Ixx / V - a * a / 5) < 2e-3
    # the oracle's update uses these: a free octahedron under gravity only
    gz = 1e-4
    p = W.Params(nx=16, ny=16, nz=24, tau=0.7, gravity=(0.0, 0.0, -gz))
    sc = W.Scene(np.array([2], np.int32), np.array([3.0]), np.array([1e12]),
                 np.array([[8.0, 8.0, 12.0]]), np.array([[1.0, 0, 0, 0]]),
                 np.zeros((1, 3)), np.zeros((1, 3)))
    sim = O.OracleSim(p, sc)
    sim.init_equilibrium()
    sim.step(5)
    assert abs(sim.particles()["U"][0, 2] + 5 * gz) < 1e-12
