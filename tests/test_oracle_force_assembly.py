"""Closed-form pins of the oracle's contact-force assembly (Sec. 2.3,
eqs. (4)-(9)) and of the isotropic inertia of spheres and cubes (eq. (3)).

The expected values are written out here from the equations, not taken
from the oracle:

* normal force |F_n| = 4/(3 pi) E* sqrt(V d) (1 + c ddot_n), clamped at 0,
  with E* = E / (2 (1 - nu^2)) for identical materials (eq. (5)) and, at
  the onset of a contact, c = 1.5 (1 - e)(11 - e) / ((1 + 9 e) u0) with u0
  the normal approach rate (eq. (6));
* tangential force -v_t/|v_t| mu(|v_t| / u_k) |F_n| with
  mu(a) = (2 mu_s* - mu_k) a^2 / (a^4 + 1) + mu_k - mu_k / (a^2 + 1) and
  mu_s* = mu_s (1 - 0.09 (mu_k / mu_s)^4) (eqs. (7)-(9));
* the relative velocity at the contact point x_c,
  v = [U_a + w_a x (x_c - X_a)] - [U_b + w_b x (x_c - X_b)];
* the angular response to a contact couple: dw = T / I with
  I = 2/5 m R^2 (sphere) and m a^2 / 6 (cube), m = s V.

Face-on cubes without enlargement give an exact overlap (V = t a^2,
depth t, normal +x, centroid the middle of the overlap slab), so the
force of a treated pair is fixed to rounding.
"""
import math

import numpy as np
import pytest

E_REST, MU_S, MU_K, NU = 0.926, 0.32, 0.16, 0.3


def mu_closed(a):
    mus = MU_S * (1.0 - 0.09 * (MU_K / MU_S) ** 4)
    a2 = a * a
    return (2.0 * mus - MU_K) * a2 / (a2 * a2 + 1.0) + MU_K - MU_K / (a2 + 1.0)


def expected_force(E, V, d, n, v, c_damp, u_k):
    """force on a from eqs. (4)-(9) for relative velocity v = v_a - v_b."""
    estar = E / (2.0 * (1.0 - NU * NU))
    dn = float(v @ n)
    fn = 4.0 / (3.0 * math.pi) * estar * math.sqrt(V * d) * (1.0 + c_damp * dn)
    fn = max(fn, 0.0)
    vt = v - dn * n
    vtn = np.linalg.norm(vt)
    ft = -(vt / vtn) * mu_closed(vtn / u_k) * fn if vtn > 0 else np.zeros(3)
    return fn, -fn * n + ft


def onset_damping(u0):
    return 1.5 * (1 - E_REST) * (11 - E_REST) / ((1 + 9 * E_REST) * u0) if u0 > 0 else 0.0


def _params(W, **kw):
    base = dict(nx=64, ny=64, nz=64, enlarge=0.0, young=0.8, poisson=NU,
                restitution=E_REST, mu_s=MU_S, mu_k=MU_K, u_k=1e-3)
    base.update(kw)
    return W.Params(**base)


@pytest.mark.parametrize("vel", [
    # (U_a, w_a, U_b, w_b): approach along x with a sliding part
    ((0.003, 0.002, -0.001), (0.0, 0.0, 4e-4), (-0.001, 5e-4, 0.0), (2e-4, 0.0, 0.0)),
    ((0.0005, -0.004, 0.0025), (1e-4, -3e-4, 0.0), (0.0, 0.0, -0.001), (0.0, 5e-4, -2e-4)),
])
def test_face_on_cubes_force_at_onset(O, W, vel):
    """Treated face-on cubes: fn and the force on a match eqs. (4)-(9) at the
    onset (damping from the normal approach rate)."""
    a, t = 6.0, 0.7
    p = _params(W)
    q = np.array([1.0, 0, 0, 0])
    Xa = np.array([20.0, 20.0, 20.0])
    Xb = Xa + [a - t, 0.0, 0.0]
    Ua, wa, Ub, wb = (np.array(v) for v in vel)
    pa = O.make_particle(1, a, 2.0, Xa, q, Ua, wa)
    pb = O.make_particle(1, a, 2.0, Xb, q, Ub, wb)
    lo = np.array([Xb[0] - a / 2 - 0.8, 16.5, 16.0])
    hi = np.array([Xa[0] + a / 2 + 0.6, 23.5, 24.0])
    r = O.treat_pair(p, pa, pb, 1, lo, hi, npass=100)
    V = t * a * a
    n = np.array([1.0, 0.0, 0.0])
    xc = np.array([(Xb[0] - a / 2 + Xa[0] + a / 2) / 2, 20.0, 20.0])
    assert abs(r["volume"] - V) <= 1e-12 * V
    assert abs(r["depth"] - t) <= 1e-12
    np.testing.assert_allclose(r["normal"], n, atol=1e-15)
    np.testing.assert_allclose(r["centroid"], xc, atol=1e-12)
    v = (Ua + np.cross(wa, xc - Xa)) - (Ub + np.cross(wb, xc - Xb))
    c = onset_damping(float(v @ n))
    fn, Fa = expected_force(p.young, V, t, n, v, c, p.u_k)
    assert abs(r["damping"] - c) <= 1e-12 * max(c, 1.0)
    assert abs(r["fn"] - fn) <= 1e-12 * fn
    np.testing.assert_allclose(r["force_a"], Fa, rtol=0, atol=1e-12 * fn)
    assert np.array_equal(np.array(r["force_b"]), -np.array(r["force_a"]))


@pytest.mark.parametrize("rate,slide", [
    (0.004, 3.0),     # closing: fn grows by 1 + c ddot_n
    (-0.0015, 3.0),   # opening, 0 < 1 + c ddot_n < 1
    (-0.05, 3.0),     # opening fast: 1 + c ddot_n < 0, force clamped to 0
    (0.002, 0.25),    # slow sliding (a < 1): rising branch of mu(a)
])
def test_established_contact_force(O, W, rate, slide):
    """An established contact keeps its damping factor c; the normal force
    is 4/(3 pi) E* sqrt(V d) (1 + c ddot_n), never negative, and friction
    opposes the sliding velocity with mu(|v_t| / u_k)."""
    p = _params(W, young=0.5, u_k=4e-4)
    V, d = 2.3, 0.41
    n = np.array([2.0, -1.0, 2.0]) / 3.0
    tdir = np.array([1.0, 2.0, 0.0]) / math.sqrt(5.0)      # orthogonal to n
    xc = np.array([21.0, 19.5, 20.25])
    Xa, Xb = xc - 3.0 * n, xc + 3.2 * n
    vt = slide * p.u_k * tdir
    # v_a - v_b = rate n + vt, from translations only
    Ua, Ub = rate * n + vt, np.zeros(3)
    c0 = 37.0                                   # damping fixed at onset
    pa = O.make_particle(1, 6.0, 2.0, Xa, (1, 0, 0, 0), Ua, (0, 0, 0))
    pb = O.make_particle(1, 6.0, 2.0, Xb, (1, 0, 0, 0), Ub, (0, 0, 0))
    r = O.contact_force_of(p, pa, pb, V, d, xc, n, established=1, damping=c0)
    fn, Fa = expected_force(p.young, V, d, n, rate * n + vt, c0, p.u_k)
    assert r["damping"] == c0
    if 1.0 + c0 * rate <= 0.0:
        assert r["fn"] == 0.0 and not np.any(np.array(r["force_a"]))
    else:
        assert abs(r["fn"] - fn) <= 1e-13 * fn
        np.testing.assert_allclose(r["force_a"], Fa, rtol=0, atol=1e-13 * fn)
        # friction along -v_t with mu(a), a = |v_t| / u_k
        ft = np.array(r["force_a"]) + r["fn"] * n
        assert ft @ tdir < 0
        assert abs(np.linalg.norm(ft) - mu_closed(slide) * fn) <= 1e-13 * fn
        assert mu_closed(slide) != pytest.approx(mu_closed(1.0 / slide), rel=1e-3)


def test_wall_partner_at_rest(O, W):
    """A wall partner contributes no velocity: v = v_a at the contact
    point; onset damping from the approach rate towards the wall."""
    p = _params(W, periodic_z=0, young=0.3)
    n = np.array([0.0, 0.0, -1.0])               # from the particle to the wall
    xc = np.array([16.0, 16.0, -0.3])
    X = np.array([16.4, 15.8, 2.4])
    U, w = np.array([0.002, -0.001, -0.003]), np.array([1e-4, 2e-4, -3e-4])
    pa = O.make_particle(1, 6.0, 2.0, X, (1, 0, 0, 0), U, w)
    r = O.contact_force_of(p, pa, None, 1.7, 0.3, xc, n)
    v = U + np.cross(w, xc - X)
    c = onset_damping(float(v @ n))
    fn, Fa = expected_force(p.young, 1.7, 0.3, n, v, c, p.u_k)
    assert abs(r["damping"] - c) <= 1e-12 * c
    assert abs(r["fn"] - fn) <= 1e-13 * fn
    np.testing.assert_allclose(r["force_a"], Fa, rtol=0, atol=1e-13 * fn)


def _first_step_response(O, W, p, scene):
    """Step once from a fluid at rest: the momentum exchange of the first
    step is exactly zero (f* = f after streaming a uniform field), so the
    particles move by the contact force and torque alone (g = 0)."""
    s = O.OracleSim(p, scene)
    s.init_equilibrium()
    X0 = s.particles()
    s.step(1)
    f, X1 = s.forces(), s.particles()
    assert not np.any(f["Fh"]) and not np.any(f["Th"])
    con = s.contacts()
    s.close()
    return X0, X1, f, con


def test_sphere_inertia_from_contact_couple(O, W):
    """Two spheres R = 4 (s = 2) sliding past each other in contact: the
    friction couple spins each one at dw = T_c / (2/5 m R^2), and the
    velocity changes by F_c / m with m = s 4/3 pi R^3."""
    R, s = 4.0, 2.0
    p = _params(W, nx=32, ny=32, nz=32, enlarge=0.2, tau=0.8, young=2.0)
    sc = W.Scene(np.array([0, 0], np.int32), np.array([R, R]), np.array([s, s]),
                 np.array([[10.0, 16.0, 16.0], [18.2, 16.0, 16.0]]),
                 np.tile([1.0, 0, 0, 0], (2, 1)),
                 np.array([[0.001, 0.003, 0.0], [-0.001, -0.002, 0.001]]),
                 np.zeros((2, 3)))
    X0, X1, f, con = _first_step_response(O, W, p, sc)
    assert len(con) == 1 and con[0]["volume"] > 0
    m = s * 4.0 / 3.0 * math.pi * R ** 3
    I = 0.4 * m * R * R
    for k in range(2):
        np.testing.assert_allclose(X1["omega"][k], f["Tc"][k] / I, rtol=1e-13, atol=0)
        dU = X1["U"][k] - X0["U"][k]
        np.testing.assert_allclose(dU, f["Fc"][k] / m, rtol=1e-9, atol=1e-22)
        assert np.abs(f["Tc"][k]).max() > 0
    # the couple of each sphere is its lever arm times its contact force
    xc = np.array(con[0]["centroid"])
    np.testing.assert_allclose(f["Tc"][0], np.cross(xc - X0["X"][0], f["Fc"][0]),
                               rtol=1e-12, atol=1e-14 * np.abs(f["Tc"][0]).max())


def test_cube_inertia_from_contact_couple(O, W):
    """Two cubes of edge 6 (s = 1.7) pressed face-on with their enlarged
    surfaces and sliding: the friction couple spins each one at
    dw = T_c / (m a^2 / 6), m = s a^3."""
    a, s = 6.0, 1.7
    p = _params(W, nx=32, ny=32, nz=32, enlarge=0.2, tau=0.8, young=2.0)
    sc = W.Scene(np.array([1, 1], np.int32), np.array([a, a]), np.array([s, s]),
                 np.array([[12.0, 16.0, 16.0], [18.2, 15.5, 16.3]]),
                 np.tile([1.0, 0, 0, 0], (2, 1)),
                 np.array([[0.002, 0.003, -0.001], [-0.001, -0.002, 0.002]]),
                 np.zeros((2, 3)))
    X0, X1, f, con = _first_step_response(O, W, p, sc)
    assert len(con) == 1 and con[0]["volume"] > 0
    m = s * a ** 3
    I = m * a * a / 6.0
    for k in range(2):
        np.testing.assert_allclose(X1["omega"][k], f["Tc"][k] / I, rtol=1e-13, atol=0)
        np.testing.assert_allclose(X1["U"][k] - X0["U"][k], f["Fc"][k] / m,
                                   rtol=1e-9, atol=1e-22)
        assert np.abs(f["Tc"][k]).max() > 0


@pytest.mark.parametrize("top", [False, True])
def test_cube_through_wall_exact_overlap(O, W, top):
    """An axis-aligned cube (no enlargement) reaching t = 0.2 beyond the
    bottom (or top) wall plane: the contact's box starts on the far side of
    the body, the correction moves its faces onto the cube and the wall
    plane, and the overlap is the exact slab: V = t a^2, depth t, normal
    from the cube into the wall, centroid the slab centre; the force is the
    closed form of eqs. (4)-(9) with the wall at rest."""
    a, t, nz = 6.0, 0.2, 24
    zc = (nz - 0.5 + t - a / 2) if top else (-0.5 - t + a / 2)
    p = _params(W, nx=32, ny=32, nz=nz, periodic_z=0, tau=0.8, young=2.0)
    X = np.array([16.3, 15.7, zc])
    U, w = np.array([0.001, -0.0005, 0.002 if top else -0.002]), np.zeros(3)
    sc = W.Scene(np.array([1], np.int32), np.array([a]), np.array([1.5]),
                 X[None, :], np.array([[1.0, 0, 0, 0]]), U[None, :], w[None, :])
    s = O.OracleSim(p, sc)
    s.init_equilibrium()
    s.step(1)
    con, f = s.contacts(), s.forces()
    s.close()
    assert len(con) == 1 and con[0]["b"] == (-2 if top else -1)
    c = con[0]
    V = t * a * a
    n = np.array([0.0, 0.0, 1.0 if top else -1.0])
    plane = nz - 0.5 if top else -0.5
    xc = np.array([X[0], X[1], plane + (t / 2 if top else -t / 2)])
    assert abs(c["volume"] - V) <= 1e-12 * V
    assert abs(c["depth"] - t) <= 1e-12
    np.testing.assert_allclose(c["normal"], n, atol=1e-15)
    np.testing.assert_allclose(c["centroid"], xc, atol=1e-12)
    v = U + np.cross(w, xc - X)
    fn, Fa = expected_force(p.young, V, t, n, v, onset_damping(float(v @ n)), p.u_k)
    assert abs(c["fn"] - fn) <= 1e-12 * fn
    np.testing.assert_allclose(f["Fc"][0], Fa, rtol=0, atol=1e-12 * fn)
