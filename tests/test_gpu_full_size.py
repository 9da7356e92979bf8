"""GPU parity at the full sizes of the dense settling boxes, in the launch
configuration the benchmark times (one context, stream execution, the same
workload records; the steps also in one call, as the benchmark issues
them).

256^3 periodic box with 1834 cubes of edge 14 (phi 0.30, Ar 1000) and the
same centres with spheres of the volume-equivalent diameter (Ar 2000).  The
FP64 oracle runs the whole lattice (a few steps take seconds on the host's
cores), so every output is compared, not a sample:
  * at the initial state (identical in every precision): the owner of every
    node, the detected pair set, per-pair overlap node counts and image boxes
    bit for bit;
  * after each step: hydrodynamic and contact forces and torques, particle
    state, and the final population field, within the precision's tolerance
    (forces relative to max(|F_oracle|, (s - 1) V |g|)).
"""
import dataclasses
import sys

import numpy as np
import pytest

from test_gpu_parity import TOL, compare_contacts, force_err, rel_field

pytestmark = pytest.mark.gpu

W_POLY0 = 3      # first body-type shape code

NSTEPS = 3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_run(O, wl, nsteps=NSTEPS):
    """Initial integer outputs, per-step forces and particles, final field."""
    o = O.OracleSim(wl.params.replace(precision=0), wl.scene)
    o.init_equilibrium()
    ref = dict(owner0=o.fields()["owner"], contacts0=o.contacts(),
               counters0=o.counters(), steps=[])
    for _ in range(nsteps):
        o.step(1)
        ref["steps"].append(dict(forces=o.forces(), particles=o.particles(),
                                 contacts=o.contacts(), counters=o.counters()))
    ref["pop"] = o.populations()
    o.close()
    return ref


@pytest.fixture(scope="module")
def dense_cubes(O, W):
    wl = W.c3_dense_cubes()
    _say("oracle: dense cube box", wl.note)
    return wl, _oracle_run(O, wl)


@pytest.fixture(scope="module")
def dense_spheres(O, W):
    wl = W.c4_dense_spheres()
    _say("oracle: dense sphere box", wl.note)
    return wl, _oracle_run(O, wl)


def _check(H, wl, ref, prec):
    nsteps = len(ref["steps"])
    p = wl.params.replace(precision=prec)
    tol = TOL[prec]
    g = H.Simulation(p, wl.scene, polyhedra=wl.polyhedra)
    g.init_equilibrium()
    assert np.array_equal(g.fields()["owner"], ref["owner0"])
    compare_contacts(ref["contacts0"], g.contacts(), 0.0)
    c = g.counters()
    assert (c["pairs"], c["cells"]) == ref["counters0"]
    V = np.where(wl.scene.shape == 1, wl.scene.size ** 3,
                 4.0 / 3.0 * np.pi * wl.scene.size ** 3)
    for k, T in (wl.polyhedra or {}).items():     # ellipsoid types here
        m = wl.scene.shape == W_POLY0 + k
        V[m] = 4.0 / 3.0 * np.pi * float(np.prod(T.axes)) * wl.scene.size[m] ** 3
    Fref = ((wl.scene.density - 1) * V).max() * abs(p.gravity[2])
    Tref = Fref * wl.scene.size.max()
    for k in range(nsteps):
        g.step(1)
        s = ref["steps"][k]
        eo, eg = s["forces"], g.forces()
        ferr = max(force_err(eg["Fh"], eo["Fh"], Fref),
                   force_err(eg["Fc"], eo["Fc"], Fref))
        terr = max(force_err(eg["Th"], eo["Th"], Tref),
                   force_err(eg["Tc"], eo["Tc"], Tref))
        po, pg = s["particles"], g.particles()
        xerr = np.abs(pg["X"] - po["X"]).max()
        _say(f"  precision {prec} step {k + 1}: force {ferr:.2e} torque {terr:.2e} X {xerr:.2e}")
        assert ferr <= tol and terr <= tol
        assert xerr <= tol * max(p.nx, p.ny, p.nz)
        if prec == 0:
            oc, gc = s["contacts"], g.contacts()
            assert [(a["a"], a["b"], a["count"]) for a in oc] == \
                   [(b["a"], b["b"], b["count"]) for b in gc]
    fg = g.populations()
    perr = rel_field(fg, ref["pop"])
    _say(f"  precision {prec}: population error {perr:.2e}")
    assert perr <= tol
    pg = g.particles()
    g.close()
    # the benchmark's launch sequence: the same steps in one call (the
    # contact treatment of steps 2..n beside the previous lattice passes)
    # leaves the same bits as the step-by-step run above
    g2 = H.Simulation(p, wl.scene, polyhedra=wl.polyhedra)
    g2.init_equilibrium()
    g2.step(nsteps)
    assert np.array_equal(g2.populations(), fg)
    p2 = g2.particles()
    for k in pg:
        assert np.array_equal(p2[k], pg[k]), k
    g2.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dense_cube_box_full_size(dense_cubes, H, prec):
    wl, ref = dense_cubes
    _check(H, wl, ref, prec)


@pytest.mark.parametrize("prec", [0, 2])
def test_dense_sphere_box_full_size(dense_spheres, H, prec):
    wl, ref = dense_spheres
    _check(H, wl, ref, prec)


@pytest.fixture(scope="module")
def dense_ellipsoids(O, W):
    wl = W.c3_dense_ellipsoids()
    for k, T in wl.polyhedra.items():
        O.define_body_type(k, T)
    _say("oracle: dense ellipsoid box", wl.note)
    return wl, _oracle_run(O, wl, nsteps=2)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_dense_ellipsoid_box_full_size(dense_ellipsoids, H, prec):
    """The ellipsoid benchmark box (734 ellipsoids, 256^3): every node's
    owner from the exact ellipsoid distance, bit-exact in FP64."""
    wl, ref = dense_ellipsoids
    _check(H, wl, ref, prec)


TREAT_WAVES = 512 * 4    # wavefronts of the contact-treatment grid


@pytest.fixture(scope="module")
def crowded_cubes(O, W):
    """The dense cube box with the contact surfaces enlarged by one lattice
    spacing (enlargement delta_c = 1 of Sec. 3.3.1): about 5500 detected pairs,
    so every wavefront of the treatment grid takes more than one record of
    the pair list."""
    wl = W.c3_dense_cubes()
    wl = dataclasses.replace(wl, params=wl.params.replace(enlarge=1.0))
    _say("oracle: dense cube box, delta_c = 1", wl.note)
    return wl, _oracle_run(O, wl, nsteps=2)


@pytest.mark.parametrize("prec", [0, 1])
def test_dense_cube_box_pair_list_longer_than_grid(crowded_cubes, H, prec):
    wl, ref = crowded_cubes
    npairs = ref["counters0"][0]
    _say(f"  detected pairs {npairs} (treatment wavefronts {TREAT_WAVES})")
    assert npairs > 2 * TREAT_WAVES
    _check(H, wl, ref, prec)


def test_dense_cube_box_graphs_match_stream(W, H):
    """The benchmark's launch mode at full size: 67 FP32 steps in one call
    replayed as graphs (eight chained 8-step graphs with the overlapped
    contact treatment, then three stream steps) leave the same bits as 67
    stream-launched steps."""
    wl = W.c3_dense_cubes()
    out = []
    for graph in (False, True):
        g = H.Simulation(wl.params, wl.scene, graph=graph)
        g.init_equilibrium()
        g.step(67)
        out.append((g.particles(), g.forces(), g.populations()[:, ::5, ::3, :].copy(),
                    [(c["a"], c["b"], c["count"], c["fn"]) for c in g.contacts()]))
        g.close()
    (pa, ea, fa, ca), (pb, eb, fb, cb) = out
    assert len(ca) > 0 and ca == cb
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    for k in ea:
        assert np.array_equal(ea[k], eb[k]), k
    assert np.array_equal(fa, fb)


def test_dense_cube_box_bitwise_reproducible(W, H):
    """Two runs of the benchmark workload (FP32, 30 steps with contacts)
    give identical bits: every reduction on the path has a fixed order."""
    wl = W.c3_dense_cubes()
    out = []
    for _ in range(2):
        g = H.Simulation(wl.params, wl.scene)
        g.init_equilibrium()
        g.step(30)
        e = g.forces()
        out.append((g.particles(), e, g.populations()[:, ::7, ::5, ::3].copy(),
                    [(c["a"], c["b"], c["count"], c["fn"]) for c in g.contacts()]))
        g.close()
    (pa, ea, fa, ca), (pb, eb, fb, cb) = out
    assert len(ca) > 0 and ca == cb
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    for k in ea:
        assert np.array_equal(ea[k], eb[k]), k
    assert np.array_equal(fa, fb)
