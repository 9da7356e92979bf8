"""GPU parity of particle-wall contacts, and the boundary calls added for the
one-call adjoint, the treatment sample counter and the autograd wrapper.

Wall contacts: an axis-aligned cube reaching through the bottom wall plane
and a rotated cube and a sphere pressing on the top wall (periodic x, y;
half-way bounce-back walls in z), stepped in FP64 against the oracle: the
contact records bit for bit in their integer fields (rough counts, node
boxes, inside-sample counts), volumes, depths, normals and forces to 1e-12.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wall_scene(W):
    nz = 26
    q1 = np.array([math.cos(0.2), 0.3 * math.sin(0.2), 0.5 * math.sin(0.2),
                   math.sqrt(1 - 0.34) * math.sin(0.2)])
    sc = W.Scene(shape=np.array([1, 1, 0], np.int32),
                 size=np.array([6.0, 5.0, 3.2]),
                 density=np.array([1.5, 1.8, 2.2]),
                 X=np.array([[9.3, 10.2, 2.3], [20.4, 9.1, nz - 3.0], [11.0, 20.5, nz - 3.4]]),
                 q=np.array([[1.0, 0.0, 0.0, 0.0], q1, [1.0, 0.0, 0.0, 0.0]]),
                 U=np.array([[0.002, -0.001, -0.004], [-0.001, 0.002, 0.003],
                             [0.0, 0.001, 0.004]]),
                 omega=np.array([[0.0, 0.001, 0.0], [0.001, 0.0, -0.002], [0.0, 0.0, 0.001]]))
    sc.q = sc.q / np.linalg.norm(sc.q, axis=1, keepdims=True)
    p = W.Params(nx=30, ny=28, nz=nz, periodic_z=0, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), young=0.6, u_k=3e-4,
                 wall_velocity=((0.0, 0.0, 0.0), (0.002, -0.001, 0.0)),
                 max_pairs=64, tile_capacity=16, precision=0)
    return p, sc


def test_wall_contacts_parity(O, W, H):
    from test_gpu_parity import compare_contacts, force_err
    p, sc = _wall_scene(W)
    o = O.OracleSim(p, sc)
    g = H.Simulation(p, sc)
    o.init_equilibrium()
    g.init_equilibrium()
    Fref = 0.5 * 6.0 ** 3 * 2e-4
    Tref = Fref * 3.0          # torques: the force scale times a lever arm
    walls = 0
    for k in range(6):
        o.step(1)
        g.step(1)
        oc, gc = o.contacts(), g.contacts()
        compare_contacts(oc, gc, 1e-12)
        walls += sum(1 for c in oc if c["b"] < 0 and c["volume"] > 0)
        eo, eg = o.forces(), g.forces()
        fe = max(force_err(eg["Fh"], eo["Fh"], Fref), force_err(eg["Fc"], eo["Fc"], Fref))
        te = max(force_err(eg["Th"], eo["Th"], Tref), force_err(eg["Tc"], eo["Tc"], Tref))
        _say(f"  step {k + 1}: {len(oc)} records, force {fe:.1e} torque {te:.1e}")
        assert fe <= 1e-12 and te <= 1e-12
        assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    # the bodies meet their walls (overlap volume > 0) in most steps
    _say(f"  wall contacts with volume > 0: {walls} over 6 steps")
    assert walls >= 6
    g.close()
    o.close()


def test_treatment_sample_counter(W, H):
    """One overlapping sphere pair: the treatment samples 6 N_c^2 face
    points and N_c^3 volume points."""
    p = W.Params(nx=32, ny=32, nz=32, tau=0.8, young=0.4, u_k=3e-4,
                 max_pairs=16, tile_capacity=16, precision=0)
    sc = W.Scene(np.array([0, 0], np.int32), np.array([4.0, 4.0]), np.array([2.0, 2.0]),
                 np.array([[10.0, 16.0, 16.0], [18.1, 16.0, 16.0]]),
                 np.tile([1.0, 0, 0, 0], (2, 1)), np.zeros((2, 3)), np.zeros((2, 3)))
    g = H.Simulation(p, sc)
    g.init_equilibrium()
    g.step(1)
    c = g.counters()
    assert len(g.contacts()) == 1 and g.contacts()[0]["volume"] > 0
    assert c["samples"] == 6 * p.n_c ** 2 + p.n_c ** 3
    g.close()


def test_one_call_adjoint(W, H):
    """hlbm_adjoint gives the gradients of record + gradient."""
    from test_gpu_adjoint import _scene
    p, sc = _scene(W)
    seed = np.zeros((sc.n, 3))
    seed[:, 2] = 1.0 / sc.n
    a = H.Simulation(p, sc)
    a.init_equilibrium()
    ds, dq = a.adjoint(14, 5, seed)
    a.close()
    b = H.Simulation(p, sc)
    b.init_equilibrium()
    b.adjoint_record(14, 5)
    r = b.adjoint_gradient(seed)
    b.close()
    np.testing.assert_allclose(ds, r["s"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(dq, r["q0"], rtol=1e-12, atol=1e-300)


def test_autograd_on_device_with_unnormalised_q(W, H):
    """Device tensors in, device tensors out; a quaternion given with norm
    2 gets the gradient of J(q / |q|), i.e. half the unit-sphere gradient,
    which matches central differences along a random direction."""
    import torch
    from test_gpu_adjoint import _scene, _J_gpu
    p, sc = _scene(W)
    K = 10
    dev = torch.device("cuda:0")
    dens = torch.tensor(sc.density, dtype=torch.float64, device=dev, requires_grad=True)
    q0 = torch.tensor(2.0 * sc.q, dtype=torch.float64, device=dev, requires_grad=True)
    J = H.mean_settling_velocity(dens, q0, p, sc, K, 4)
    assert J.device == dev
    J.backward()
    assert dens.grad.device == dev and q0.grad.device == dev
    gq = q0.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    v = rng.normal(size=sc.q.shape)
    h = 2e-6

    def Jq(qr):
        s = sc.copy()
        s.q = qr / np.linalg.norm(qr, axis=1, keepdims=True)
        return _J_gpu(H, p, s, K)
    fd = (Jq(2.0 * sc.q + h * v) - Jq(2.0 * sc.q - h * v)) / (2 * h)
    ad = float((gq * v).sum())
    _say(f"  dJ/dq . v: adjoint {ad:+.8e} fd {fd:+.8e}")
    assert abs(ad - fd) <= 1e-5 * max(abs(fd), np.abs(gq).max())
    # a second backward has nothing left to run on
    with pytest.raises(RuntimeError):
        J2 = H.mean_settling_velocity(dens, q0, p, sc, K, 4)
        J2.backward(retain_graph=True)
        J2.backward()
