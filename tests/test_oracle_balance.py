"""Zero-net-flux balance force (balance mode 2) of the FP64 oracle.

The reading of Sec. 5.1 ("a balance force such that the suspension has a
net volume flow rate of zero"): the uniform fluid acceleration of each
collision is set from the lattice momentum of the last two steps so that
the lattice momentum, i.e. the net volume flow of the suspension, stays at
zero.  Pins: hand-derived trajectories of the controller on particle-free
boxes, and the momentum budget of a settling box against the static
balance of mode 1."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import oracle as O  # noqa: E402
from paper_2401_10878_amd import workloads as W  # noqa: E402


def _momentum(sim):
    c = O.lattice()[0].astype(float)
    f = sim.populations()
    return np.tensordot(c, f, axes=(0, 0)).reshape(3, -1).sum(1), f.sum()


def _box(**kw):
    p = W.Params(nx=12, ny=10, nz=8, periodic_z=1, tau=0.7, young=1.0,
                 u_k=1.0, max_pairs=16, tile_capacity=8, precision=0)
    return p.replace(**kw)


def test_uniform_flow_is_stopped_in_one_step():
    """No particles, fluid moving at u0: b_0 = -u0, so the first collision
    removes the whole momentum and the acceleration is zero afterwards."""
    u0 = np.array([0.02, -0.01, 0.005])
    sim = O.OracleSim(_box(balance=2), W.Scene.empty())
    sim.init_equilibrium(1.0, tuple(u0))
    P, M = _momentum(sim)
    assert P == pytest.approx(M * u0, rel=1e-12)
    assert sim.balance() == pytest.approx(-u0, rel=1e-12)
    sim.step(1)
    P, M = _momentum(sim)
    assert np.abs(P).max() < 1e-12 * M
    assert np.abs(sim.balance()).max() < 1e-13
    sim.step(3)
    P, M = _momentum(sim)
    assert np.abs(P).max() < 1e-12 * M


def test_constant_drive_trajectory():
    """No particles, fluid at rest, a constant fluid_accel g0 (momentum
    g0 M per collision besides the controller).  By hand: a = g0 + b with
    b = 0, -2 g0, -g0, -g0, ...; lattice momentum g0 M after the first
    collision and 0 after every later one."""
    g0 = np.array([1e-5, 0.0, -3e-5])
    sim = O.OracleSim(_box(balance=2, fluid_accel=tuple(g0)), W.Scene.empty())
    sim.init_equilibrium(1.0, (0.0, 0.0, 0.0))
    M = _momentum(sim)[1]
    expect_a = [g0, -g0, 0 * g0, 0 * g0, 0 * g0]
    expect_P = [g0 * M, 0 * g0, 0 * g0, 0 * g0]
    assert sim.balance() == pytest.approx(expect_a[0], abs=1e-18)
    for t in range(4):
        sim.step(1)
        P, _ = _momentum(sim)
        assert P == pytest.approx(expect_P[t], abs=1e-10 * M * 3e-5)
        assert sim.balance() == pytest.approx(expect_a[t + 1], abs=1e-14)


def test_static_balance_unchanged_without_mode_two():
    """Mode 1 keeps the fixed acceleration -sum (s_p - 1) V_p g / N."""
    wl = W.settling_box(W.SPHERE, 0.1, 6.0, edge_cells=24, ar=500.0,
                        precision=0, balance=1)
    sim = O.OracleSim(wl.params, wl.scene)
    sim.init_equilibrium()
    V = np.pi / 6.0 * 6.0 ** 3
    a = -((wl.scene.density - 1.0) * V).sum() * np.asarray(wl.params.gravity) / 24 ** 3
    assert sim.balance() == pytest.approx(a, rel=1e-12)
    sim.step(2)
    assert sim.balance() == pytest.approx(a, rel=1e-12)


def test_settling_box_holds_zero_net_flow():
    """Twelve spheres settling in a 24^3 box for 300 steps: with mode 1 the
    lattice momentum drifts (the momentum exchange over the owned nodes does
    not conserve the total), with mode 2 it stays orders of magnitude
    smaller, and the particles still settle."""
    out = {}
    for mode in (1, 2):
        wl = W.settling_box(W.SPHERE, 0.1, 6.0, edge_cells=24, ar=500.0,
                            precision=0, balance=mode)
        sim = O.OracleSim(wl.params, wl.scene)
        sim.init_equilibrium()
        sim.step(300)
        P, M = _momentum(sim)
        out[mode] = (abs(P[2]), sim.particles()["U"][:, 2].mean())
    drift1, u1 = out[1]
    drift2, u2 = out[2]
    assert drift1 > 1.0
    assert drift2 < 1e-2 * drift1
    assert u1 < 0 and u2 < 0
