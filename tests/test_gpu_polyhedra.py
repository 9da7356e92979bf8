"""GPU parity of convex polyhedra (arbitrary convex bodies): a box, a
regular tetrahedron and a random convex hull mixed with spheres, through
the C ABI against the FP64 oracle.  Owners, pair sets and overlap counts
bit-exact at the start and after every FP64 step; forces, torques and
angular velocities (eq. (3) with the anisotropic inertia tensor) within the
precision's tolerance; malformed definitions rejected."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _polys(W):
    return {0: W.polyhedron_cuboid(1.0, 1.6, 2.2),
            1: W.polyhedron_tetrahedron(2.4),
            2: W.polyhedron_random(np.random.default_rng(5), 14)}


def _scene(O, W, seed, dims, n):
    polys = _polys(W)
    rc = {}
    for k, P in polys.items():
        O.define_polyhedron(k, P.vertices, P.faces)
        rc[W.POLY0 + k] = O.polyhedron_info(k, len(P.vertices))[2]
    sc = W.random_small_scene(seed, dims, n, periodic_z=1, size_range=(1.8, 3.0),
                              gap=-0.8, speed=0.01, spin=0.006,
                              shapes=(0, W.POLY0, W.POLY0 + 1, W.POLY0 + 2), poly_rc=rc)
    return polys, sc


def _rel(a, b, floor):
    return np.abs(a - b).max() / max(np.abs(b).max(), floor) if b.size else 0.0


@pytest.mark.parametrize("prec,eps", [(0, 1.0), (1, 1.0), (0, 3.5), (1, 3.5)])
def test_polyhedra_parity(O, W, H, prec, eps):
    """eps = 3.5: a coupling band reaching 1.75 cells out, beyond which
    screening forms may stop at the plane lower bound."""
    seed, dims, n = 43, (30, 26, 22), 9
    polys, sc = _scene(O, W, seed, dims, n)
    assert (sc.shape >= W.POLY0).sum() >= 5
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=1, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=prec, eps_b=eps)
    f0 = W.perturbed_populations(seed, dims, O.feq(1.0, [0.003, 0.002, -0.001]), amp=0.01)
    o = O.OracleSim(p.replace(precision=0), sc)
    g = H.Simulation(p, sc, polyhedra=polys)
    o.set_populations(f0)
    g.set_populations(f0)
    _say("polyhedra precision", prec, "eps", eps)
    assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    oc = o.contacts()
    assert any(sc.shape[c["a"]] >= W.POLY0 for c in oc)
    assert [(c["a"], c["b"], c["count"]) for c in oc] == \
           [(c["a"], c["b"], c["count"]) for c in g.contacts()]
    Fref = 2e-4 * 0.5 * (4 / 3 * math.pi * 1.8 ** 3)
    tol = TOL[prec]
    for k in range(4):
        o.step(1)
        g.step(1)
        eo, eg = o.forces(), g.forces()
        po, pg = o.particles(), g.particles()
        eF = max(_rel(eg["Fh"], eo["Fh"], Fref), _rel(eg["Fc"], eo["Fc"], Fref))
        eT = max(_rel(eg["Th"], eo["Th"], Fref), _rel(eg["Tc"], eo["Tc"], Fref))
        ew = _rel(pg["omega"], po["omega"], 1e-6)
        eX = np.abs(pg["X"] - po["X"]).max()
        _say(f"  step {k + 1}: force {eF:.2e} torque {eT:.2e} omega {ew:.2e} X {eX:.2e}")
        assert eF <= max(tol, 1e-11)
        assert eT <= max(tol, 1e-11)
        assert ew <= max(tol, 1e-11)
        if prec == 0:
            assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
            assert [(c["a"], c["b"], c["count"]) for c in o.contacts()] == \
                   [(c["a"], c["b"], c["count"]) for c in g.contacts()]


def test_polyhedron_definition_errors(W, H):
    P = W.polyhedron_cuboid(1.0, 1.0, 1.0)
    p = W.Params(nx=16, ny=16, nz=16, periodic_z=1, tau=0.7, young=1.0, u_k=1.0,
                 max_pairs=16, tile_capacity=8, precision=1)
    bad = W.Polyhedron(P.vertices, [f[::-1] for f in P.faces])
    with pytest.raises(H.HlbmError, match="counter-clockwise"):
        H.Simulation(p, W.Scene.empty(), polyhedra={0: bad})
    v = P.vertices.copy()
    v[7] *= 0.5
    with pytest.raises(H.HlbmError, match="convex"):
        H.Simulation(p, W.Scene.empty(), polyhedra={0: W.Polyhedron(v, P.faces)})
    sc = W.Scene(np.array([W.POLY0 + 1], np.int32), np.array([2.0]), np.array([2.0]),
                 np.array([[8.0, 8.0, 8.0]]), np.array([[1.0, 0, 0, 0]]),
                 np.zeros((1, 3)), np.zeros((1, 3)))
    with pytest.raises(H.HlbmError, match="polyhedron type"):
        H.Simulation(p, sc, polyhedra={0: P})
    g = H.Simulation(p, W.Scene(np.array([W.POLY0], np.int32), sc.size, sc.density,
                                sc.X, sc.q, sc.U, sc.omega), polyhedra={0: P})
    v = np.ascontiguousarray(P.vertices, np.float64).reshape(-1)
    fs = np.array([len(f) for f in P.faces], np.int32)
    fi = np.array([j for f in P.faces for j in f], np.int32)
    rc = g.L.hlbm_define_polyhedron(g.h, 1, 8, v.ctypes.data_as(H.C.POINTER(H.C.c_double)), 6,
                                    fs.ctypes.data_as(H.C.POINTER(H.C.c_int)),
                                    fi.ctypes.data_as(H.C.POINTER(H.C.c_int)))
    assert rc != 0 and "before init_particles" in g.L.hlbm_last_error(g.h).decode()
