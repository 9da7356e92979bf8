"""Adjoint of K coupled steps against finite differences.

The gradient is that of J = mean over particles of U_z after K steps from
fluid at rest.  The adjoint holds the owner map and the contact forces of the
forward run fixed, so the references are central differences with a step
small enough that no node changes owner (the scenes keep the particles apart,
so there are no contacts):
  * central differences of the GPU FP64 forward (every parameter kind);
  * central differences of the FP64 CPU oracle (the reference gradient).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _scene(W):
    """Three separated bodies (a sphere and two cubes) in a ragged box."""
    sc = W.Scene(shape=np.array([0, 1, 1], np.int32),
                 size=np.array([3.5, 6.0, 5.0]),
                 density=np.array([1.6, 1.4, 2.0]),
                 X=np.array([[6.3, 7.1, 8.4], [17.2, 12.6, 15.9], [8.8, 16.4, 22.7]]),
                 q=np.array([[1.0, 0.0, 0.0, 0.0],
                             [0.9, 0.3, -0.2, 0.25],
                             [0.7, -0.1, 0.5, 0.4]]),
                 U=np.array([[0.002, -0.001, 0.0], [0.0, 0.001, -0.002], [-0.001, 0.0, 0.001]]),
                 omega=np.array([[0.0, 0.001, 0.0], [0.002, 0.0, -0.001], [0.0, -0.001, 0.002]]))
    sc.q = sc.q / np.linalg.norm(sc.q, axis=1, keepdims=True)
    p = W.Params(nx=26, ny=22, nz=30, periodic_z=1, tau=0.65,
                 gravity=(0.0, 0.0, -3e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=64, tile_capacity=16, precision=0)
    return p, sc


def _rotate(q, axis, ang):
    """q -> exp(ang axis / 2) (x) q (world-frame rotation)."""
    h = 0.5 * ang
    a = np.array([math.cos(h)] + list(math.sin(h) * np.asarray(axis, float)))
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _J_gpu(H, p, sc, K):
    g = H.Simulation(p, sc)
    g.init_equilibrium()
    g.step(K)
    J = g.particles()["U"][:, 2].mean()
    g.close()
    return J


def _J_oracle(O, p, sc, K):
    o = O.OracleSim(p, sc)
    o.init_equilibrium()
    o.step(K)
    J = o.particles()["U"][:, 2].mean()
    o.close()
    return J


def _adjoint(H, p, sc, K, L):
    g = H.Simulation(p, sc)
    g.init_equilibrium()
    g.adjoint_record(K, L)
    J = g.particles()["U"][:, 2].mean()
    seed = np.zeros((sc.n, 3))
    seed[:, 2] = 1.0 / sc.n
    r = g.adjoint_gradient(seed)
    # the context stands at the end of the window afterwards
    assert g.particles()["U"][:, 2].mean() == J
    g.close()
    return J, r


def _perturbations(sc):
    """(name, function scene, h -> perturbed scene, adjoint key, index)."""
    out = []
    for i in range(sc.n):
        def ds(s, h, i=i):
            s = s.copy(); s.density[i] += h; return s
        out.append((f"s[{i}]", ds, 1e-6, "s", (i,)))
    for i in (1, 2):
        for k in range(3):
            def dq(s, h, i=i, k=k):
                s = s.copy(); e = np.zeros(3); e[k] = 1.0
                s.q[i] = _rotate(s.q[i], e, h); return s
            out.append((f"theta0[{i},{k}]", dq, 1e-6, "theta0", (i, k)))
    for key, attr in (("X0", "X"), ("U0", "U"), ("omega0", "omega")):
        for i, k in ((0, 2), (1, 0), (2, 1)):
            def dx(s, h, attr=attr, i=i, k=k):
                s = s.copy(); getattr(s, attr)[i, k] += h; return s
            hh = 1e-6 if key == "X0" else 1e-7
            out.append((f"{key}[{i},{k}]", dx, hh, key, (i, k)))
    return out


def test_adjoint_matches_gpu_finite_differences(W, H):
    p, sc = _scene(W)
    K = 30
    J, r = _adjoint(H, p, sc, K, 7)
    assert abs(J - _J_gpu(H, p, sc, K)) <= 1e-15 + 1e-12 * abs(J)
    worst = 0.0
    scale = dict(s=np.abs(r["s"]).max(), theta0=np.abs(r["theta0"]).max(),
                 X0=np.abs(r["X0"]).max(), U0=np.abs(r["U0"]).max(),
                 omega0=np.abs(r["omega0"]).max())
    for name, fn, h, key, idx in _perturbations(sc):
        fd = (_J_gpu(H, p, fn(sc, h), K) - _J_gpu(H, p, fn(sc, -h), K)) / (2 * h)
        ad = r[key][idx]
        err = abs(ad - fd) / max(scale[key], 1e-30)
        worst = max(worst, err)
        _say(f"  {name}: adjoint {ad:+.8e} fd {fd:+.8e} rel {err:.1e}")
    _say("  worst", worst)
    assert worst <= 1e-5


def test_adjoint_checkpoint_interval_independent(W, H):
    p, sc = _scene(W)
    _, a = _adjoint(H, p, sc, 24, 24)
    _, b = _adjoint(H, p, sc, 24, 5)
    for k in ("s", "theta0", "X0", "U0", "omega0"):
        s = max(np.abs(a[k]).max(), 1e-300)
        assert np.abs(a[k] - b[k]).max() <= 1e-12 * s, k


def test_adjoint_matches_oracle_reference_gradient(O, W, H):
    """FP64 CPU reference gradient: central differences of the oracle."""
    p, sc = _scene(W)
    K = 16
    _, r = _adjoint(H, p, sc, K, 6)
    picks = [q for q in _perturbations(sc) if q[0] in
             ("s[0]", "s[2]", "theta0[1,0]", "theta0[2,2]", "U0[1,0]")]
    for name, fn, h, key, idx in picks:
        fd = (_J_oracle(O, p, fn(sc, h), K) - _J_oracle(O, p, fn(sc, -h), K)) / (2 * h)
        ad = r[key][idx]
        err = abs(ad - fd) / max(np.abs(r[key]).max(), 1e-30)
        _say(f"  oracle {name}: adjoint {ad:+.8e} fd {fd:+.8e} rel {err:.1e}")
        assert err <= 1e-5


def test_autograd_function(W, H):
    import torch
    p, sc = _scene(W)
    K = 12
    dens = torch.tensor(sc.density, dtype=torch.float64, requires_grad=True)
    q0 = torch.tensor(sc.q, dtype=torch.float64, requires_grad=True)
    J = H.mean_settling_velocity(dens, q0, p, sc, K, 5)
    J.backward()
    _, r = _adjoint(H, p, sc, K, 5)
    assert abs(J.item() - _J_gpu(H, p, sc, K)) <= 1e-15
    assert np.allclose(dens.grad.numpy(), r["s"], rtol=1e-12, atol=0)
    assert np.allclose(q0.grad.numpy(), r["q0"], rtol=1e-12, atol=1e-300)
    # the quaternion gradient is tangent to the unit sphere
    assert np.abs((q0.grad.numpy() * sc.q).sum(axis=1)).max() <= 1e-12 * \
        np.abs(q0.grad.numpy()).max()


def test_adjoint_box_workload(W, H):
    """96^3 box, 27 cubes, 500 steps with checkpoints every 50: gradient of
    the mean settling velocity by the (common) density ratio and by initial
    rotations along ten random directions, against GPU central differences,
    and along the two directions of the stored FP64 CPU reference gradient
    (oracle central differences, tests/golden/c5_oracle_fd.json).  A node
    whose distance to a body crosses the edge of the coupling band changes
    owner, which moves the force by a finite amount the adjoint does not
    see.  Over 500 steps with 27 bodies such crossings are frequent: a
    rotation of 1e-9 rad moved a node across in about half of the random
    directions (a jump of about 1e-10 in J, which dominates the difference
    quotient), so rotations take h = 1e-11 rad (FP64 rounding of J then
    contributes about 1e-4 of the smallest directional derivative) and the
    density ratio h = 1e-9.  Agreement is held to 1%.  Holding contact
    forces fixed is exact here: no node is flagged by the rough detection in
    any step of the window, so no contact can start."""
    import json
    import os
    wl = W.c5_adjoint_cubes()
    p = wl.params.replace(precision=0)
    sc = wl.scene
    K, L = 500, 50
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "c5_oracle_fd.json")))
    assert ref["steps"] == K and ref["flagged_nodes_all_steps"] == 0
    g = H.Simulation(p, sc)
    g.init_equilibrium()
    g.adjoint_record(K, L)
    assert g.counters()["total_cells"] == 0          # no contact in the window
    J = g.particles()["U"][:, 2].mean()
    seed = np.zeros((sc.n, 3))
    seed[:, 2] = 1.0 / sc.n
    r = g.adjoint_gradient(seed)
    g.close()
    _say(f"  C5: J = {J:.9e} (oracle {ref['J']:.9e})")
    assert abs(J - ref["J"]) <= 1e-9 * abs(ref["J"])
    h, hr = ref["h_density"], ref["h_rotation"]

    def all_s(s, hh):
        s = s.copy(); s.density = s.density + hh; return s

    def rot_by(v):
        def rot(s, hh):
            s = s.copy()
            for i in range(s.n):
                ang = np.linalg.norm(v[i])
                s.q[i] = _rotate(s.q[i], v[i] / ang, hh * ang)
            return s
        return rot
    fd = (_J_gpu(H, p, all_s(sc, h), K) - _J_gpu(H, p, all_s(sc, -h), K)) / (2 * h)
    ad = r["s"].sum()
    err_s = abs(ad - fd) / abs(fd)
    _say(f"  dJ/ds: adjoint {ad:+.6e} fd {fd:+.6e} rel {err_s:.2e}")
    errs = [err_s]
    # the FP64 CPU reference gradient (oracle central differences)
    e = abs(ad - ref["density"]["fd"]) / abs(ref["density"]["fd"])
    _say(f"  dJ/ds: oracle fd {ref['density']['fd']:+.6e} rel {e:.2e}")
    errs.append(e)
    vref = np.array(ref["rotation_directions"])
    adv = float((r["theta0"] * vref).sum())
    e = abs(adv - ref["rotation"]["fd"]) / max(abs(ref["rotation"]["fd"]),
                                               np.abs(r["theta0"]).max())
    _say(f"  dJ/dtheta . v: adjoint {adv:+.6e} oracle fd {ref['rotation']['fd']:+.6e} "
         f"rel {e:.2e}")
    errs.append(e)
    rng = np.random.default_rng(5)
    for _ in range(10):
        v = rng.normal(size=(sc.n, 3))
        rot = rot_by(v)
        fdv = (_J_gpu(H, p, rot(sc, hr), K) - _J_gpu(H, p, rot(sc, -hr), K)) / (2 * hr)
        adv = float((r["theta0"] * v).sum())
        e = abs(adv - fdv) / max(abs(fdv), np.abs(r["theta0"]).max())
        _say(f"  dJ/dtheta . v: adjoint {adv:+.6e} fd {fdv:+.6e} rel {e:.2e}")
        errs.append(e)
    _say(f"  worst {max(errs):.2e}")
    assert max(errs) <= 1e-2
