"""GPU parity of the zero-net-flux balance force (balance mode 2): the
controller's hand-derived trajectory on a particle-free box, and a settling
box stepped by the HIP path and the FP64 oracle side by side."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-3}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _momentum(O, f):
    c = O.lattice()[0].astype(float)
    return np.tensordot(c, f, axes=(0, 0)).reshape(3, -1).sum(1), f.sum()


@pytest.mark.parametrize("prec", [0, 1])
def test_constant_drive_trajectory_gpu(O, W, H, prec):
    """fluid_accel g0 on a box at rest: a = g0, -g0, 0, 0, ... and the
    lattice momentum g0 M after the first collision, 0 afterwards."""
    _say("constant drive, precision", prec)
    g0 = np.array([1e-5, 0.0, -3e-5])
    p = W.Params(nx=20, ny=12, nz=9, periodic_z=1, tau=0.7, young=1.0, u_k=1.0,
                 max_pairs=16, tile_capacity=8, precision=prec, balance=2,
                 fluid_accel=tuple(g0))
    g = H.Simulation(p, W.Scene.empty())
    g.init_equilibrium()
    M = 20 * 12 * 9
    tol_a = 1e-14 if prec == 0 else 1e-9
    assert g.fluid_acceleration() == pytest.approx(g0, abs=tol_a)
    expect_a = [-g0, 0 * g0, 0 * g0, 0 * g0]
    expect_P = [g0 * M, 0 * g0, 0 * g0, 0 * g0]
    for t in range(4):
        g.step(1)
        P, _ = _momentum(O, g.populations())
        assert P == pytest.approx(expect_P[t], abs=(1e-10 if prec == 0 else 1e-5) * M * 3e-5)
        assert g.fluid_acceleration() == pytest.approx(expect_a[t], abs=tol_a)


@pytest.mark.parametrize("prec", [0, 1])
def test_settling_box_parity(O, W, H, prec):
    """Twelve spheres in a 24^3 box with balance mode 2, six steps: particle
    velocities, hydrodynamic forces and the fluid acceleration against the
    oracle, per step."""
    _say("settling box, precision", prec)
    wl = W.settling_box(W.SPHERE, 0.1, 6.0, edge_cells=24, ar=500.0,
                        precision=prec, balance=2)
    o = O.OracleSim(wl.params.replace(precision=0), wl.scene)
    g = H.Simulation(wl.params, wl.scene)
    o.init_equilibrium()
    g.init_equilibrium()
    assert g.fluid_acceleration() == pytest.approx(o.balance(), abs=1e-15)
    gz = abs(wl.params.gravity[2])
    for t in range(6):
        o.step(1)
        g.step(1)
        ao, ag = o.balance(), g.fluid_acceleration()
        Fo, Fg = o.forces()["Fh"], g.forces()["Fh"]
        Uo, Ug = o.particles()["U"], g.particles()["U"]
        ea = np.abs(ag - ao).max() / gz
        eF = np.abs(Fg - Fo).max() / max(np.abs(Fo).max(), 1e-300)
        eU = np.abs(Ug - Uo).max() / max(np.abs(Uo).max(), 1e-300)
        _say(f"  step {t + 1}: accel {ea:.2e} (of g), force {eF:.2e}, velocity {eU:.2e}")
        # the acceleration comes from lattice sums whose per-node momenta
        # are small differences of O(0.1) populations: its rounding error is
        # a few ulp of the populations, not of the acceleration itself
        assert ea <= (1e-10 if prec == 0 else TOL[prec])
        assert eF <= TOL[prec]
        assert eU <= TOL[prec]
