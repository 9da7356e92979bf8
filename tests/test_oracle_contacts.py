"""Pins of the oracle's discrete contact model (Sec. 2.3, Sec. 3.3).

Closed forms: the lens volume of two overlapping spheres, the spherical cap
cut by a wall, the box overlap of face-on cubes; special values of the
friction law (eqs. (7)-(9)), the damping law (eq. (6)) and the effective
modulus (eq. (5)); symmetry and invariance: centroid and normal of equal
spheres, action-reaction, torque balance, translation across a periodic
boundary.
"""
import math

import numpy as np
import pytest

E_REST = 0.926
MU_S, MU_K = 0.32, 0.16


def lens_volume(R, d):
    return math.pi * (2 * R - d) ** 2 * (d + 4 * R) / 12.0


def _pair(O, R, dist, shape=0, q=(1, 0, 0, 0), centre=(20.0, 20.0, 20.0)):
    c = np.array(centre)
    pa = O.make_particle(shape, R, 2.0, c, q)
    pb = O.make_particle(shape, R, 2.0, c + [dist, 0, 0], q)
    return pa, pb


@pytest.mark.parametrize("dist", [8.0, 7.9, 7.5, 7.0])
def test_lens_volume(O, W, dist):
    """Two spheres R = 4 enlarged by 0.2: V -> pi (2R'-d)^2 (d+4R') / 12."""
    R, Rp = 4.0, 4.2
    ex = lens_volume(Rp, dist)
    pa, pb = _pair(O, R, dist)
    lo = np.array([20 + dist - Rp - 1.0, 17.0, 17.0])
    hi = np.array([20 + Rp + 1.0, 23.0, 23.0])
    p = W.Params(nx=64, ny=64, nz=64)
    errs = {}
    for nc in (8, 64):
        r = O.treat_pair(p.replace(n_c=nc), pa, pb, 1, lo, hi, npass=100)
        errs[nc] = abs(r["volume"] - ex) / ex
        # equal spheres: centroid at the midpoint, normal along the centre line
        np.testing.assert_allclose(r["centroid"], [20 + dist / 2, 20, 20],
                                   atol=1e-9)
        np.testing.assert_allclose(r["normal"], [1.0, 0, 0], atol=1e-12)
        # depth -> 2R' - d from below (max over midpoints on the centre line)
        assert 0 < r["depth"] <= 2 * Rp - dist + 1e-12
        assert r["depth"] > (2 * Rp - dist) * (1 - 2.0 / nc)
    assert errs[8] < 0.015        # the paper's resolution N_c = 8
    assert errs[64] < 1e-3


@pytest.mark.parametrize("sy,sz", [(1.3, -2.1), (0.0, 0.0)])
def test_face_on_cubes_exact(O, W, sy, sz):
    """Aligned cubes, no enlargement: the corrected box is the overlap box,
    so V = t (a - |s_y|)(a - |s_z|) to rounding and depth = t.  With flush
    lateral faces the normal is +x by symmetry (with lateral offsets the
    inside-gradient sum picks up the nearby side faces of one cube)."""
    a, t = 6.0, 0.7
    p = W.Params(nx=64, ny=64, nz=64, enlarge=0.0)
    q = np.array([1.0, 0, 0, 0])
    Xa = np.array([20.0, 20.0, 20.0])
    Xb = Xa + [a - t, sy, sz]
    pa = O.make_particle(1, a, 2.0, Xa, q)
    pb = O.make_particle(1, a, 2.0, Xb, q)
    lo = np.array([Xb[0] - a / 2 - 0.8, 17.5, 15.0])
    hi = np.array([Xa[0] + a / 2 + 0.6, 24.0, 23.5])
    r = O.treat_pair(p, pa, pb, 1, lo, hi, npass=100)
    V = t * (a - abs(sy)) * (a - abs(sz))
    assert abs(r["volume"] - V) <= 1e-12 * V
    if sy == 0.0 and sz == 0.0:
        np.testing.assert_allclose(r["normal"], [1, 0, 0], atol=1e-15)
    else:
        assert r["normal"][0] > 0.98
    assert abs(r["depth"] - t) < 1e-12
    ov_lo = [Xb[0] - a / 2, Xb[1] - a / 2, Xa[2] - a / 2]
    ov_hi = [Xa[0] + a / 2, Xa[1] + a / 2, Xb[2] + a / 2]
    np.testing.assert_allclose(r["lo"], ov_lo, atol=1e-12)
    np.testing.assert_allclose(r["hi"], ov_hi, atol=1e-12)


def test_face_on_cubes_common_rotation(O, W):
    """The flush face-on pair rotated rigidly about x keeps n_c = x and V."""
    a, t, sy, sz = 6.0, 0.7, 0.0, 0.0
    p = W.Params(nx=64, ny=64, nz=64, enlarge=0.0, n_c=16)
    ang = 0.37
    q = np.array([math.cos(ang / 2), math.sin(ang / 2), 0, 0])
    R = O.rotation(q)
    Xa = np.array([20.0, 20.0, 20.0])
    Xb = Xa + R @ np.array([a - t, sy, sz])
    pa = O.make_particle(1, a, 2.0, Xa, q)
    pb = O.make_particle(1, a, 2.0, Xb, q)
    lo = np.minimum(Xa, Xb) - 5.0
    hi = np.maximum(Xa, Xb) + 5.0
    lo[0], hi[0] = Xb[0] - a / 2 - 0.5, Xa[0] + a / 2 + 0.5
    r = O.treat_pair(p, pa, pb, 1, lo, hi, npass=100)
    V = t * (a - abs(sy)) * (a - abs(sz))
    # the overlap is a rotated box: midpoint integration is no longer exact,
    # but the normal is (by symmetry of the face-on contact) the x axis
    np.testing.assert_allclose(r["normal"], [1, 0, 0], atol=1e-12)
    assert abs(r["volume"] - V) / V < 0.08


def test_sphere_wall_cap(O, W):
    """Sphere R enlarged by 0.2 against the bottom wall at z = -1/2."""
    R, Rp, pen = 4.0, 4.2, 0.5
    Z = -0.5 + Rp - pen
    p = W.Params(nx=32, ny=32, nz=32, periodic_z=0, n_c=64)
    pa = O.make_particle(0, R, 2.0, (16.0, 16.0, Z), (1, 0, 0, 0))
    lo = np.array([12.0, 12.0, -1.5])
    hi = np.array([20.0, 20.0, 0.8])
    r = O.treat_pair(p, pa, None, -1, lo, hi, npass=100)
    h = pen
    cap = math.pi * h * h * (3 * Rp - h) / 3.0
    assert abs(r["volume"] - cap) / cap < 5e-3
    np.testing.assert_allclose(r["normal"], [0, 0, -1], atol=1e-12)
    np.testing.assert_allclose(r["centroid"][:2], [16.0, 16.0], atol=1e-9)


def test_friction_law_special_values(O):
    mus_star = MU_S * (1 - 0.09 * (MU_K / MU_S) ** 4)
    assert abs(mus_star - 0.3182) < 1e-12
    assert O.friction_mu(0.0, MU_S, MU_K) == 0.0
    assert abs(O.friction_mu(1.0, MU_S, MU_K) - mus_star) < 1e-15
    assert abs(O.friction_mu(1e8, MU_S, MU_K) - MU_K) < 1e-12
    # the peak (static) coefficient lies between 1 and 2 in a
    a = np.linspace(0.01, 10, 2000)
    mu = np.array([O.friction_mu(v, MU_S, MU_K) for v in a])
    assert mu.max() >= mus_star and a[mu.argmax()] < 2.0


def test_damping_special_values(O):
    assert O.damping(1.0, 0.01) == 0.0
    assert O.damping(E_REST, 0.0) == 0.0
    assert O.damping(E_REST, -0.02) == 0.0
    k = 1.5 * (1 - E_REST) * (11 - E_REST) / (1 + 9 * E_REST)
    assert abs(k - 0.11980) < 5e-6
    assert abs(O.damping(E_REST, 0.004) * 0.004 - k) < 1e-15


def test_effective_modulus(O):
    E, nu = 0.43, 0.3
    assert abs(O.effective_modulus(E, nu, E, nu) - E / (2 * (1 - nu * nu))) < 1e-15
    # a rigid partner leaves only the soft body's term
    assert abs(O.effective_modulus(E, nu, 1e300, 0.0) - E / (1 - nu * nu)) < 1e-15


def _contact_scene(W, dist, U=0.004, periodic_shift=None, L=32):
    X = np.array([[10.0, 16.0, 16.0], [10.0 + dist, 16.0, 16.0]])
    if periodic_shift is not None:
        X = np.mod(X + periodic_shift, L)
    return W.Scene(np.array([0, 0], np.int32), np.array([4.0, 4.0]),
                   np.array([2.0, 2.0]), X, np.tile([1.0, 0, 0, 0], (2, 1)),
                   np.array([[U, 0.001, 0], [-U, 0, 0.0005]]),
                   np.array([[0, 0, 0.001], [0.0005, 0, 0]]))


def test_contact_dynamics_action_reaction(O, W):
    """Spheres whose enlarged surfaces overlap: the contact is established
    with a damping factor from the normal approach rate, the normal force is
    repulsive, forces are equal and opposite (bit-exact) and the contact
    torques balance the force couple."""
    L = 32
    p = W.c1_two_spheres().params
    sc = _contact_scene(W, 8.2)
    s = O.OracleSim(p, sc)
    s.init_equilibrium()
    assert [(c["a"], c["b"]) for c in s.contacts()] == [(0, 1)]
    Xpre = s.particles()
    s.step(1)
    con = s.contacts()
    assert len(con) == 1
    c = con[0]
    assert c["established"] == 1 and c["volume"] > 0 and c["carried"] == 1
    n = np.array(c["normal"])
    assert n[0] > 0.99
    Fa, Fb = np.array(c["force_a"]), np.array(c["force_b"])
    assert np.array_equal(Fa, -Fb)
    assert Fa @ n < 0            # repulsive on a
    # damping factor: c u0 = 1.5 (1-e)(11-e)/(1+9e), u0 = normal approach
    xc = np.array(c["centroid"])
    va = Xpre["U"][0] + np.cross(Xpre["omega"][0], xc - Xpre["X"][0])
    vb = Xpre["U"][1] + np.cross(Xpre["omega"][1], xc - Xpre["X"][1])
    u0 = (va - vb) @ n
    k = 1.5 * (1 - p.restitution) * (11 - p.restitution) / (1 + 9 * p.restitution)
    assert abs(c["damping"] * u0 - k) < 1e-12
    # contact torques: T_a + T_b + X_a x F_a + X_b x F_b = 0 (angular momentum)
    f = s.forces()
    Xa, Xb = Xpre["X"][0], Xpre["X"][1]
    tot = f["Tc"][0] + f["Tc"][1] + np.cross(Xa, f["Fc"][0]) + np.cross(Xb, f["Fc"][1])
    assert np.abs(tot).max() < 1e-14 * max(1.0, np.abs(Xa).max()) * np.abs(Fa).max() * 10


def test_contact_periodic_translation_invariance(O, W):
    """A pair straddling the periodic x boundary gives the same contact as
    the same pair away from it (the box lives in the lower-id frame)."""
    p = W.c1_two_spheres().params
    ref = O.OracleSim(p, _contact_scene(W, 8.1))
    ref.init_equilibrium()
    ref.step(2)
    c0 = ref.contacts()[0]
    sh = np.array([18.0, 5.0, 0.0])       # particle 1 wraps to x ~ 4
    per = O.OracleSim(p, _contact_scene(W, 8.1, periodic_shift=sh))
    per.init_equilibrium()
    per.step(2)
    c1 = per.contacts()[0]
    assert (c0["a"], c0["b"]) == (c1["a"], c1["b"])
    assert c0["n_in"] == c1["n_in"]
    for k in ("volume", "depth", "fn"):
        assert abs(c0[k] - c1[k]) <= 1e-10 * max(abs(c0[k]), 1e-12)
    np.testing.assert_allclose(c1["normal"], c0["normal"], atol=1e-10)
    # the box (lower-id frame) of the shifted case is the reference box + sh
    np.testing.assert_allclose(np.array(c1["lo"]) - sh, c0["lo"], atol=1e-9)


def test_no_contact_when_apart(O, W):
    """C1 as specified: the gap stays wide, no contact ever has volume."""
    wl = W.c1_two_spheres()
    s = O.OracleSim(wl.params, wl.scene)
    s.init_equilibrium()
    for _ in range(4):
        s.step(5)
        for c in s.contacts():
            assert c["volume"] == 0.0
        assert np.abs(s.forces()["Fc"]).max() == 0.0


@pytest.mark.parametrize("D", [4.6, 5.3])
def test_octahedra_vertex_overlap_exact(O, W, D):
    """Two axis-aligned octahedra of centre-to-vertex a, centres D apart
    along x, no enlargement: their overlap is the octahedron of
    centre-to-vertex a - D/2 around the midpoint, V = 4 (a - D/2)^3 / 3; the
    depth max -(d_a + d_b) is attained at the midpoint, 2 (a - D/2) / sqrt 3,
    and the normal is -x ... +x by symmetry."""
    a = 3.0
    p = W.Params(nx=64, ny=64, nz=64, enlarge=0.0, n_c=64)
    q = np.array([1.0, 0, 0, 0])
    Xa = np.array([20.0, 20.0, 20.0])
    Xb = Xa + [D, 0.0, 0.0]
    pa = O.make_particle(2, a, 2.0, Xa, q)
    pb = O.make_particle(2, a, 2.0, Xb, q)
    c = a - D / 2
    mid = (Xa + Xb) / 2
    lo = mid - c - 0.6
    hi = mid + c + 0.45
    r = O.treat_pair(p, pa, pb, 1, lo, hi, npass=100)
    V = 4.0 * c ** 3 / 3.0
    assert abs(r["volume"] - V) < 3e-3 * V
    # the depth is a maximum over cell-midpoint samples: at most the exact
    # value, and short of it by at most twice the half-diagonal of a cell
    # (each distance is 1-Lipschitz)
    cell = (np.array(r["hi"]) - np.array(r["lo"])) / 64
    exact = 2 * c / math.sqrt(3.0)
    assert r["depth"] <= exact + 1e-12
    assert exact - r["depth"] <= np.linalg.norm(cell) + 1e-12
    # the corrected box is the overlap's bounding box to within a cell
    np.testing.assert_allclose(r["lo"], mid - c, atol=cell.max())
    np.testing.assert_allclose(r["hi"], mid + c, atol=cell.max())
    assert abs(abs(r["normal"][0]) - 1.0) < 1e-12
