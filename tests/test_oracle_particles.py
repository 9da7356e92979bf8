"""Pins of the oracle's particle motion (eqs. (2)-(3), Sec. 5.1) and of the
paper's printed constants used by the seeded inputs."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _heavy(W, shape, U, om, s=1e12, X=(10.3, 11.7, 9.2)):
    size = 3.0 if shape == 0 else 5.0
    return W.Scene(np.array([shape], np.int32), np.array([size]),
                   np.array([s]), np.array([X]), np.array([[1.0, 0, 0, 0]]),
                   np.array([U]), np.array([om]))


def _qmul(a, b):
    w1, v1, w2, v2 = a[0], a[1:], b[0], b[1:]
    return np.concatenate([[w1 * w2 - v1 @ v2], w1 * v2 + w2 * v1 + np.cross(v1, v2)])


def test_free_heavy_particle_kinematics(O, W):
    """Hydrodynamic forces cannot move a particle 1e12 times denser than the
    fluid: U and w stay constant, X advances by U per step (wrapped), and the
    orientation is the exact rotation by k |w| about w."""
    U = np.array([0.03, -0.02, 0.011])
    om = np.array([0.01, 0.02, -0.015])
    p = W.Params(nx=20, ny=20, nz=20, tau=0.7)
    for shape in (0, 1):
        s = O.OracleSim(p, _heavy(W, shape, U, om))
        s.init_equilibrium()
        k = 40
        s.step(k)
        st = s.particles()
        np.testing.assert_allclose(st["U"][0], U, rtol=0, atol=1e-12)
        np.testing.assert_allclose(st["omega"][0], om, rtol=0, atol=1e-12)
        X = np.mod(np.array([10.3, 11.7, 9.2]) + k * U, 20.0)
        np.testing.assert_allclose(st["X"][0], X, atol=1e-10)
        th = np.linalg.norm(om) * k
        ax = om / np.linalg.norm(om)
        qe = np.concatenate([[math.cos(th / 2)], math.sin(th / 2) * ax])
        q = st["q"][0]
        assert abs(np.linalg.norm(q) - 1.0) < 1e-15
        assert min(np.abs(q - qe).max(), np.abs(q + qe).max()) < 1e-10


def test_gravity_minus_buoyancy(O, W):
    """F_g = (rho_p - rho_f) V g: a heavy particle accelerates at g (1 - 1/s)."""
    g = 1e-4
    s_ratio = 1e9
    p = W.Params(nx=16, ny=16, nz=32, tau=0.7, gravity=(0.0, 0.0, -g))
    sim = O.OracleSim(p, _heavy(W, 1, [0, 0, 0], [0, 0, 0], s=s_ratio,
                                X=(8.0, 8.0, 16.0)))
    sim.init_equilibrium()
    sim.step(10)
    Uz = sim.particles()["U"][0, 2]
    assert abs(Uz - (-10 * g * (1 - 1 / s_ratio))) < 1e-12


def test_balance_acceleration_cancels_net_weight(O, W):
    """Fully periodic with balance: N_cells a_ext + sum (s-1) V g = 0."""
    wl = W.c5_adjoint_cubes()
    s = O.OracleSim(wl.params, wl.scene)
    a = s.balance()
    V = wl.scene.size ** 3
    net = ((wl.scene.density - 1) * V).sum() * np.array(wl.params.gravity)
    n = wl.params.nx * wl.params.ny * wl.params.nz
    np.testing.assert_allclose(n * a + net, 0.0, atol=1e-15)
    assert a[2] > 0


def test_paper_particle_counts(W):
    """N = phi L^3 / V_p reproduces the particle counts the paper prints."""
    gold = json.load(open(GOLDEN))
    e = gold["largest_run_particles"]
    n = e["phi"] * e["L_over_Ds"] ** 3 / (math.pi / 6.0)
    assert round(n) == e["value"]
    c = gold["cube_run_particles"]
    n = c["phi"] * c["L_over_Ds"] ** 3 / (math.pi / 6.0)
    assert abs(n - c["value"]) <= 1.0          # the paper's phi is approximate


def test_workload_constants_match_paper(W):
    gold = json.load(open(GOLDEN))
    assert W.D_S_PHYS == gold["D_s_m"]["value"]
    assert W.RHO_F_PHYS == gold["rho_f"]["value"]
    assert W.G_PHYS == gold["g"]["value"]
    assert W.E_PHYS == gold["E_Pa"]["value"]
    assert W.U_K_PHYS == gold["u_k_ms"]["value"]
    assert W.RESTITUTION == gold["restitution"]["value"]
    assert (W.MU_K, W.MU_S) == (gold["mu_k"]["value"], gold["mu_s"]["value"])
    assert W.CONTACT_RES == gold["contact_resolution"]["value"]
    assert W.ENLARGE == gold["enlargement_dx"]["value"]
    assert abs(math.sqrt(0.75) - gold["detect_threshold"]["value"]) < 1e-16


def test_archimedes_unit_conversion(W):
    """Ar = g D^3 (s-1) / nu^2 (eq. (25)) holds in lattice units, and the
    cube workloads have the expected particle counts and fractions."""
    for ar, edge in ((500, 12.0), (1000, 14.0)):
        d = W.cube_equiv_diameter(edge)
        lu = W.lattice_units(d, 1.5, ar, 0.55)
        assert abs(lu["g"] * d ** 3 * 0.5 / lu["nu"] ** 2 - ar) < 1e-9 * ar
    assert round(0.3 * 256 ** 3 / 14 ** 3) == 1834
    assert round(0.1 * 128 ** 3 / 12 ** 3) == 121


def test_substeps_constant_force_closed_form(O, W):
    """n sub-steps of length 1/n under a constant force a (gravity minus
    buoyancy, hydrodynamic force zero for a particle 1e12 times denser than
    the fluid): after k steps U = U0 + k a and, per step, X advances by
    U_start + a (n + 1) / (2 n) (the sum of the sub-step velocities / n)."""
    g = 2e-4
    s_ratio = 1e12
    a = -g * (1 - 1 / s_ratio)
    U0 = np.array([0.01, 0.0, 0.002])
    om = np.array([0.0, 0.03, 0.0])
    for n in (1, 3, 8):
        p = W.Params(nx=16, ny=16, nz=32, tau=0.7, gravity=(0.0, 0.0, -g), n_sub=n)
        sim = O.OracleSim(p, _heavy(W, 0, U0, om, s=s_ratio, X=(8.0, 8.0, 20.0)))
        sim.init_equilibrium()
        k = 6
        sim.step(k)
        st = sim.particles()
        Uz = U0[2] + k * a
        Zexp = 20.0 + sum(U0[2] + j * a + a * (n + 1) / (2 * n) for j in range(k))
        assert abs(st["U"][0, 2] - Uz) < 1e-13
        assert abs(st["X"][0, 2] - Zexp) < 1e-12, (n, st["X"][0, 2], Zexp)
        assert abs(st["X"][0, 0] - (8.0 + k * U0[0])) < 1e-12
        # the rotation over a step is the same whatever the sub-division
        th = k * np.linalg.norm(om)
        qe = np.array([math.cos(th / 2), 0.0, math.sin(th / 2), 0.0])
        q = st["q"][0]
        assert min(np.abs(q - qe).max(), np.abs(q + qe).max()) < 1e-12


def _head_on(W, n_sub, young, speed=0.02):
    sc = W.Scene(np.array([0, 0], np.int32), np.array([3.0, 3.0]),
                 np.array([2000.0, 2000.0]),
                 np.array([[9.0, 10.0, 10.0], [15.6, 10.0, 10.0]]),
                 np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
                 np.array([[speed, 0, 0], [-speed, 0, 0]]), np.zeros((2, 3)))
    p = W.Params(nx=26, ny=20, nz=20, tau=0.8, young=young, u_k=3e-4,
                 max_pairs=16, tile_capacity=8, n_sub=n_sub)
    return p, sc


def test_substeps_head_on_momentum_balance(O, W):
    """Contact forces act equal and opposite in every sub-step, and the
    hydrodynamic impulse of a step is F_h whatever the sub-division: the
    particles' momentum changes by the summed hydrodynamic impulse only."""
    for n in (1, 4):
        p, sc = _head_on(W, n, young=50.0)
        sim = O.OracleSim(p, sc)
        sim.init_equilibrium()
        m = 2000.0 * 4.0 / 3.0 * math.pi * 27.0
        P0 = m * (sc.U[0] + sc.U[1])
        imp = np.zeros(3)
        touched = False
        for _ in range(60):
            sim.step(1)
            f = sim.forces()
            imp += f["Fh"][0] + f["Fh"][1]
            touched = touched or np.abs(f["Fc"]).max() > 0
        st = sim.particles()
        P1 = m * (st["U"][0] + st["U"][1])
        assert touched
        np.testing.assert_allclose(P1 - P0, imp, rtol=0, atol=1e-12 * m * 0.02)


def test_substeps_converge_on_a_stiff_collision(O, W):
    """With a stiff contact the collision lasts only a few steps; the
    velocity after the rebound converges as the sub-steps refine it (the
    difference to a 32-sub-step run shrinks from 2 to 8 sub-steps)."""
    def rebound(n):
        p, sc = _head_on(W, n, young=2e4)
        sim = O.OracleSim(p, sc)
        sim.init_equilibrium()
        sim.step(40)
        return sim.particles()["U"][0, 0]
    ref = rebound(32)
    e2, e8 = abs(rebound(2) - ref), abs(rebound(8) - ref)
    assert ref < 0.0                 # the sphere bounced back
    assert e8 < 0.5 * e2, (e2, e8)
