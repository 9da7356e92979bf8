"""GPU parity of ellipsoid types (smooth convex bodies) through the C ABI
against the FP64 oracle: a triaxial ellipsoid and a spheroid (two equal
shortest axes) mixed with a box and spheres in a periodic box, an
axis-aligned ellipsoid centred on a node (nodes on its symmetry planes and
axes take the degenerate branches of the nearest-point solve) next to a
second one, two chains of overlapping ellipsoids (37 ellipsoid pairs), and
ellipsoids on a wall.  Owners, pair sets and overlap counts
bit-exact at the start and after every FP64 step; forces, torques, angular
velocities and positions within the precision's tolerance; malformed
definitions rejected."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b, floor):
    return np.abs(a - b).max() / max(np.abs(b).max(), floor) if b.size else 0.0


def _types(W):
    return {0: W.Ellipsoid((1.0, 0.6, 0.4)),
            1: W.Ellipsoid((0.7, 0.7, 1.1)),
            2: W.polyhedron_cuboid(1.0, 1.6, 2.2)}


def _define(O, types):
    rc = {}
    for k, T in types.items():
        O.define_body_type(k, T)
        nv = 0 if hasattr(T, "axes") else len(T.vertices)
        rc[O.POLY0 + k] = O.polyhedron_info(k, nv)[2]
    return rc


def _run(O, W, H, p, sc, types, f0, nsteps, Fref):
    o = O.OracleSim(p.replace(precision=0), sc)
    g = H.Simulation(p, sc, polyhedra=types)
    if f0 is not None:
        o.set_populations(f0)
        g.set_populations(f0)
    else:
        o.init_equilibrium()
        g.init_equilibrium()
    prec = p.precision
    assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    oc = o.contacts()
    assert [(c["a"], c["b"], c["count"]) for c in oc] == \
           [(c["a"], c["b"], c["count"]) for c in g.contacts()]
    tol = TOL[prec]
    for k in range(nsteps):
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
        assert eX <= max(tol, 1e-11) * max(p.nx, p.ny, p.nz)
        if prec == 0:
            assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
            assert [(c["a"], c["b"], c["count"]) for c in o.contacts()] == \
                   [(c["a"], c["b"], c["count"]) for c in g.contacts()]
    out = (o.contacts(), g.contacts())
    o.close()
    g.close()
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_ellipsoid_mixed_parity(O, W, H, prec):
    seed, dims, n = 47, (30, 26, 22), 9
    types = _types(W)
    rc = _define(O, types)
    sc = W.random_small_scene(seed, dims, n, periodic_z=1, size_range=(1.8, 3.0),
                              gap=-0.8, speed=0.01, spin=0.006,
                              shapes=(0, W.POLY0, W.POLY0 + 1, W.POLY0 + 2), poly_rc=rc)
    assert (sc.shape == W.POLY0).sum() + (sc.shape == W.POLY0 + 1).sum() >= 3
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=1, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=prec)
    f0 = W.perturbed_populations(seed, dims, O.feq(1.0, [0.003, 0.002, -0.001]), amp=0.01)
    _say("ellipsoids mixed, precision", prec)
    Fref = 2e-4 * 0.5 * (4 / 3 * math.pi * 1.8 ** 3)
    oc, gc = _run(O, W, H, p, sc, types, f0, 4, Fref)
    assert any(sc.shape[c["a"]] in (W.POLY0, W.POLY0 + 1) or
               (c["b"] >= 0 and sc.shape[c["b"]] in (W.POLY0, W.POLY0 + 1)) for c in oc)


@pytest.mark.parametrize("prec", [0, 1])
def test_ellipsoid_axis_aligned_on_node(O, W, H, prec):
    """Identity orientation, centre on a node: the centre node, the nodes on
    the three symmetry planes and on the axes have zero body components.
    A second ellipsoid overlaps its enlarged surface."""
    types = {0: W.Ellipsoid((1.0, 0.6, 0.4)), 1: W.Ellipsoid((0.7, 0.7, 1.1))}
    _define(O, types)
    dims = (24, 24, 24)
    sc = W.Scene(np.array([W.POLY0, W.POLY0 + 1], np.int32), np.array([6.0, 4.0]),
                 np.array([1.5, 1.5]), np.array([[12.0, 12.0, 12.0], [18.1, 12.3, 12.2]]),
                 np.array([[1.0, 0.0, 0.0, 0.0], [0.96, 0.0, 0.28, 0.0]]),
                 np.array([[0.002, 0.0, 0.0], [-0.002, 0.0, 0.0]]),
                 np.array([[0.0, 0.0, 0.001], [0.0, 0.0, 0.0]]))
    sc.q[1] /= np.linalg.norm(sc.q[1])
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=1, tau=0.7,
                 gravity=(0.0, 0.0, -1e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=64, tile_capacity=16, precision=prec)
    _say("ellipsoid on a node, precision", prec)
    oc, gc = _run(O, W, H, p, sc, types, None, 3, 1e-4 * 0.5 * 4 / 3 * math.pi * 6 ** 3 * 0.24)
    assert any(c["b"] == 1 for c in oc)


@pytest.mark.parametrize("prec", [0, 1])
def test_ellipsoid_contact_chains(O, W, H, prec):
    """Two periodic chains, tilted triaxial ellipsoids tip to tip and
    spheroids beside them, every neighbour overlapping its enlarged
    surface: 37 ellipsoid-ellipsoid pairs, across the periodic boundary and
    between the chains, through the box correction and the overlap
    integration with gradients."""
    types = {0: W.Ellipsoid((1.0, 0.6, 0.4)), 1: W.Ellipsoid((0.7, 0.7, 1.1))}
    _define(O, types)
    rng = np.random.default_rng(21)
    L, n0, n1 = 40, 6, 12

    def tilt(ang):
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        a = rng.uniform(-ang, ang)
        return np.array([math.cos(a / 2), *(math.sin(a / 2) * ax)])

    X, q, sh, sz = [], [], [], []
    for i in range(n0):
        X.append([i * L / n0 + 1.3, 6.0, 12.0])
        q.append(tilt(0.2))
        sh.append(W.POLY0)
        sz.append(3.5)
    for i in range(n1):
        X.append([i * L / n1 + 0.4, 9.6, 12.3])
        q.append(tilt(0.25))
        sh.append(W.POLY0 + 1)
        sz.append(2.5)
    n = n0 + n1
    sc = W.Scene(np.array(sh, np.int32), np.array(sz), np.full(n, 1.5), np.array(X),
                 np.array(q), rng.uniform(-0.002, 0.002, (n, 3)),
                 rng.uniform(-0.001, 0.001, (n, 3)))
    p = W.Params(nx=L, ny=20, nz=24, periodic_z=1, tau=0.7, gravity=(0.0, 0.0, -1e-4),
                 balance=1, young=0.4, u_k=3e-4, max_pairs=256, tile_capacity=24,
                 precision=prec)
    _say("ellipsoid chains, precision", prec)
    oc, gc = _run(O, W, H, p, sc, types, None, 3, 1e-4 * 0.5 * 4 / 3 * math.pi * 2.5 ** 3)
    assert len(oc) >= 30


def test_ellipsoid_on_wall(O, W, H):
    """Walls in z: an ellipsoid pressed into the bottom wall, tilted (its
    half extent along z sets the wall pair's first box)."""
    types = {0: W.Ellipsoid((1.0, 0.6, 0.4))}
    _define(O, types)
    dims = (24, 20, 18)
    q = np.array([math.cos(0.3), math.sin(0.3), 0.0, 0.0])
    sc = W.Scene(np.array([W.POLY0, W.POLY0], np.int32), np.array([6.0, 5.0]),
                 np.array([2.0, 2.0]), np.array([[8.0, 10.0, 2.0], [17.0, 9.5, 14.0]]),
                 np.array([q, [1.0, 0.0, 0.0, 0.0]]), np.zeros((2, 3)),
                 np.zeros((2, 3)))
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=0, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=0, young=0.4, u_k=3e-4,
                 max_pairs=64, tile_capacity=16, precision=0)
    _say("ellipsoid on a wall")
    oc, gc = _run(O, W, H, p, sc, types, None, 3, 2e-4 * 4 / 3 * math.pi * 6 ** 3 * 0.24)
    assert any(c["b"] == -1 for c in oc)


def test_ellipsoid_definition_errors(W, H):
    p = W.Params(nx=16, ny=16, nz=16, periodic_z=1, tau=0.7, young=1.0, u_k=1.0,
                 max_pairs=16, tile_capacity=8, precision=1)
    with pytest.raises(H.HlbmError, match="semi-axes"):
        H.Simulation(p, W.Scene.empty(), polyhedra={0: W.Ellipsoid((1.0, -1.0, 1.0))})
    with pytest.raises(H.HlbmError, match="ellipsoid type"):
        H.Simulation(p, W.Scene.empty(), polyhedra={9: W.Ellipsoid((1.0, 1.0, 1.0))})
    sc = W.Scene(np.array([W.POLY0], np.int32), np.array([2.0]), np.array([2.0]),
                 np.array([[8.0, 8.0, 8.0]]), np.array([[1.0, 0, 0, 0]]),
                 np.zeros((1, 3)), np.zeros((1, 3)))
    g = H.Simulation(p, sc, polyhedra={0: W.Ellipsoid((1.0, 0.5, 0.5))})
    rc = g.L.hlbm_define_ellipsoid(g.h, 1, 1.0, 1.0, 1.0)
    assert rc != 0 and "before init_particles" in g.L.hlbm_last_error(g.h).decode()
    g.close()
