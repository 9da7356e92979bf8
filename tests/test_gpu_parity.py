"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Integer outputs (node owners, detected pair set, overlap node counts, rough
boxes, inside-sample counts) must match bit for bit when both start from the
same state; floating-point outputs within 1e-12 (FP64 path), 1e-5 (FP32)
and 1e-3 (FP16 storage), relative to the largest magnitude of the oracle's
field or, for forces, to max(|F_oracle|, a reference force).

Forces (and the particle state they drive) after several steps of the
reduced-precision paths are held to FTOL and STOL, ten times TOL.  The
hydrodynamic force is a sum of about 10^3 link terms (c_i - u)(f*_i - f_i)
per particle of these scenes, each carrying the rounding of the stored
values; the FP32 path stores deviations h = f - w of about 1e-2, whose
rounding (about 1e-9 after a few steps, the population error measured here
being 5e-9 of max |f| = 1/3) adds up as a random walk to about
30 x 2 x 1.7e-9 = 1e-7, or 6e-5 of the reference force 1.7e-3.  Binary16
storage rounds the same deviations with 2^-11 instead of 2^-24 of relative
precision.  Measured worst cases after 18 steps: FP32 1.9e-5, binary16
2.9e-3.  FP64 keeps 1e-11 for forces and 1e-12 for the state.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-3}
FTOL = {0: 1e-11, 1: 1e-4, 2: 1e-2}       # forces after several steps
STOL = {0: 1e-12, 1: 1e-4, 2: 1e-2}       # particle state after several steps


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(O, H, params, scene, f0=None):
    o = O.OracleSim(params, scene)
    g = H.Simulation(params, scene)
    if f0 is None:
        o.init_equilibrium()
        g.init_equilibrium()
    else:
        o.set_populations(f0)
        g.set_populations(f0)
    return o, g


def _key(c):
    return (c["a"], c["b"])


def compare_contacts(oc, gc, tol, exact_ints=True):
    assert [_key(c) for c in gc] == [_key(c) for c in oc]
    for a, b in zip(oc, gc):
        assert a["count"] == b["count"], (_key(a), a["count"], b["count"])
        assert a["rlo"] == b["rlo"] and a["rhi"] == b["rhi"], _key(a)
        assert a["carried"] == b["carried"] and a["established"] == b["established"]
        if exact_ints:
            assert a["n_in"] == b["n_in"], (_key(a), a["n_in"], b["n_in"])
        for k in ("volume", "depth", "fn", "damping"):
            s = max(abs(a[k]), 1e-300)
            assert abs(a[k] - b[k]) <= tol * s + 1e-300, (k, a[k], b[k])
        for k in ("lo", "hi", "centroid", "normal", "force_a"):
            x, y = np.array(a[k]), np.array(b[k])
            s = max(np.abs(x).max(), 1e-300)
            assert np.abs(x - y).max() <= tol * s, (k, x, y)


def rel_field(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def force_err(Fg, Fo, Fref):
    scale = np.maximum(np.abs(Fo), Fref)
    return (np.abs(Fg - Fo) / scale).max() if Fo.size else 0.0


CASES = [
    # (seed, dims, n, periodic_z)  -- sizes span several 4^3 tiles with
    # ragged tails on every axis
    (11, (30, 22, 18), 7, 1),
    (12, (26, 21, 23), 8, 0),
    (13, (17, 19, 25), 5, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_prologue_bit_exact(O, W, H, case):
    seed, dims, n, pz = case
    _say("prologue", case)
    sc = W.random_small_scene(seed, dims, n, periodic_z=pz,
                              size_range=(1.6, 3.0), gap=-0.8)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7,
                 young=0.4, u_k=3e-4, max_pairs=256, tile_capacity=16)
    o, g = _pair(O, H, p, sc)
    fo = o.fields()
    fg = g.fields()
    assert np.array_equal(fg["owner"], fo["owner"])
    oc, gc = o.contacts(), g.contacts()
    assert len(oc) > 0
    compare_contacts(oc, gc, 0.0)
    po, pg = o.counters(), g.counters()
    assert (pg["pairs"], pg["cells"]) == po


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_steps_parity(O, W, H, case, prec):
    """Perturbed populations, moving particles in contact; k steps."""
    seed, dims, n, pz = case
    _say("steps", case, "precision", prec)
    sc = W.random_small_scene(seed, dims, n, periodic_z=pz,
                              size_range=(1.6, 3.0), gap=-0.8, speed=0.01,
                              spin=0.004)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=pz,
                 wall_velocity=((0.0, 0.0, 0.0), (0.003, 0.0, 0.0)),
                 young=0.4, u_k=3e-4, max_pairs=256, tile_capacity=16,
                 precision=prec)
    f0 = W.perturbed_populations(seed, dims, O.feq(1.0, [0.004, -0.002, 0.001]),
                                 amp=0.01)
    o, g = _pair(O, H, p, sc, f0)
    Fref = np.abs(np.array(p.gravity)).max() * 0.5 * (4 / 3 * math.pi * 1.6 ** 3)
    tol = TOL[prec]
    nsteps = 1 if prec == 0 else 6
    for k in range(3):
        o.step(nsteps)
        g.step(nsteps)
        fo, fg = o.fields(), g.fields()
        assert np.array_equal(fg["owner"], fo["owner"]) or prec != 0
        if prec == 0:
            # same imported state at the start: integer outputs bit-exact
            compare_contacts(o.contacts(), g.contacts(), 1e-12,
                             exact_ints=(k == 0))
        eo, eg = o.forces(), g.forces()
        ferr = max(force_err(eg["Fh"], eo["Fh"], Fref),
                   force_err(eg["Fc"], eo["Fc"], Fref))
        pe = rel_field(g.populations(), o.populations())
        _say(f"  step {o.step_count}: pop {pe:.2e} force {ferr:.2e}")
        assert pe <= tol
        assert ferr <= FTOL[prec]
        po, pg = o.particles(), g.particles()
        for key in ("X", "U", "q", "omega"):
            a, b = pg[key], po[key]
            s = max(np.abs(b).max(), 1e-3 if key == "U" else 1e-6)
            assert np.abs(a - b).max() <= STOL[prec] * s, key


def test_two_sphere_workload_parity(O, W, H):
    """C1 (32^3, two spheres head-on, 100 steps) in FP64."""
    wl = W.c1_two_spheres()
    _say("C1 parity")
    o, g = _pair(O, H, wl.params, wl.scene)
    Fref = 0.0        # g = 0: reference force = max |F| over particles and steps
    for _ in range(4):
        o.step(25)
        g.step(25)
        eo, eg = o.forces(), g.forces()
        Fref = max(Fref, np.abs(eo["Fh"]).max())
        err = force_err(eg["Fh"], eo["Fh"], Fref)
        _say(f"  C1 step {o.step_count}: force err {err:.2e}")
        assert err <= 1e-12, err
        assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    assert rel_field(g.populations(), o.populations()) <= 1e-12
    po, pg = o.particles(), g.particles()
    assert np.abs(pg["X"] - po["X"]).max() <= 1e-12 * 32
    # mirror symmetry holds on the GPU too
    F = eg["Fh"]
    assert abs(F[0, 0] + F[1, 0]) <= 1e-12 * abs(F[0, 0])


def test_graph_matches_stream(W, H):
    """The captured step gives the same state as the launch sequence."""
    sc = W.random_small_scene(21, (24, 20, 16), 6, size_range=(1.6, 2.8),
                              gap=-0.6, speed=0.01)
    p = W.Params(nx=24, ny=20, nz=16, tau=0.7, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=1)
    a = H.Simulation(p, sc)
    b = H.Simulation(p, sc, graph=True)
    a.init_equilibrium(u=(0.003, 0, 0))
    b.init_equilibrium(u=(0.003, 0, 0))
    for _ in range(3):
        a.step(5)
        b.step(5)
        a.sync()
        b.sync()
        assert rel_field(b.populations(), a.populations()) <= 1e-6
        ca, cb = a.contacts(), b.contacts()
        assert [_key(c) for c in ca] == [_key(c) for c in cb]
        assert [c["count"] for c in ca] == [c["count"] for c in cb]
        assert np.array_equal(a.fields()["owner"], b.fields()["owner"])


@pytest.mark.parametrize("prec", [0, 1])
def test_overlapped_treatment_matches_ordered_steps(W, H, prec):
    """One call of n steps (the contact treatment of steps 2..n on the side
    stream, beside the previous step's lattice passes) leaves the same bits
    as n calls of one step (strictly ordered)."""
    sc = W.random_small_scene(29, (26, 22, 20), 9, size_range=(1.8, 3.0),
                              gap=-0.7, speed=0.01, spin=0.004)
    p = W.Params(nx=26, ny=22, nz=20, tau=0.7, young=0.4, u_k=3e-4,
                 gravity=(0.0, 0.0, -1e-4), balance=1,
                 max_pairs=256, tile_capacity=16, precision=prec)
    a = H.Simulation(p, sc)
    b = H.Simulation(p, sc)
    a.init_equilibrium(u=(0.002, -0.001, 0))
    b.init_equilibrium(u=(0.002, -0.001, 0))
    assert len(a.contacts()) > 0
    for _ in range(3):
        for _ in range(6):
            a.step(1)
        b.step(6)
        a.sync()
        b.sync()
        assert np.array_equal(a.populations(), b.populations())
        pa, pb = a.particles(), b.particles()
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k
        fa, fb = a.forces(), b.forces()
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
        ca, cb = a.contacts(), b.contacts()
        assert [_key(c) for c in ca] == [_key(c) for c in cb]
        assert [c["count"] for c in ca] == [c["count"] for c in cb]
        assert a.counters() == b.counters()


def test_multistep_graph_matches_stream(W, H):
    """Calls replayed as graphs leave the same bits as stream launches, on
    every path a call can take (8-step graphs with the overlapped contact
    treatment inside, chained across graph boundaries): a long call that
    replays graphs not run before (70 steps: graphs, then six stream steps
    after a joined graph); a short call of graphs already run (19: two
    graphs, three stream steps); a short call whose graphs have not run (19
    from the other parity: stream launches only); a graph whose successor
    has not run (16: one graph, then stream); 64 steps ending in the graph
    that starts no further treatment; that graph chained after another
    (16); one step (its single-step graph); five steps (stream)."""
    sc = W.random_small_scene(31, (26, 22, 20), 9, size_range=(1.8, 3.0),
                              gap=-0.7, speed=0.01, spin=0.004)
    p = W.Params(nx=26, ny=22, nz=20, tau=0.7, young=0.4, u_k=3e-4,
                 gravity=(0.0, 0.0, -1e-4), balance=1,
                 max_pairs=256, tile_capacity=16, precision=1)
    a = H.Simulation(p, sc)
    b = H.Simulation(p, sc, graph=True)
    a.init_equilibrium(u=(0.002, -0.001, 0))
    b.init_equilibrium(u=(0.002, -0.001, 0))
    assert len(a.contacts()) > 0
    for n in (70, 19, 19, 16, 64, 16, 1, 5):
        a.step(n)
        b.step(n)
        a.sync()
        b.sync()
        assert np.array_equal(a.populations(), b.populations()), n
        pa, pb = a.particles(), b.particles()
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (n, k)
        ca, cb = a.contacts(), b.contacts()
        assert [_key(c) for c in ca] == [_key(c) for c in cb]
        assert a.counters() == b.counters()


def test_capacity_overflow_reported(W, H):
    """Too small a tile capacity is reported, not silently truncated."""
    sc = W.random_small_scene(3, (16, 16, 16), 6, size_range=(2.0, 3.0), gap=-0.5)
    p = W.Params(nx=16, ny=16, nz=16, tau=0.7, young=0.4, u_k=3e-4,
                 max_pairs=64, tile_capacity=1)
    g = H.Simulation(p, sc)
    with pytest.raises(H.HlbmError) as e:
        g.init_equilibrium()
    assert e.value.code == -4


def test_invalid_configuration_rejected(W, H):
    wl = W.c1_two_spheres()
    with pytest.raises(H.HlbmError):
        H.Simulation(wl.params.replace(tau=0.5), wl.scene)
    with pytest.raises(H.HlbmError):
        H.Simulation(wl.params.replace(n_sub=0), wl.scene)
    # a periodic box shorter than twice the particle reach
    with pytest.raises(H.HlbmError):
        H.Simulation(wl.params.replace(nx=8), wl.scene)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_adjoint_box_workload_parity(O, W, H, prec):
    """96^3 periodic box, 27 cubes a=10, Ar 500 (balance force): forces,
    trajectories and fields against the FP64 oracle, normalised as stated:
    |F - F_o| / max(|F_o|, F_ref), F_ref = (s - 1) V |g|."""
    wl = W.c5_adjoint_cubes()
    p = wl.params.replace(precision=prec)
    _say("C5 parity precision", prec)
    o, g = _pair(O, H, p, wl.scene)
    V = wl.scene.size ** 3
    Fref = ((wl.scene.density - 1) * V).max() * abs(p.gravity[2])
    tol = TOL[prec]
    worst = dict(F=0.0, T=0.0, pop=0.0, X=0.0, U=0.0)
    for _ in range(4):
        o.step(10)
        g.step(10)
        eo, eg = o.forces(), g.forces()
        worst["F"] = max(worst["F"], force_err(eg["Fh"], eo["Fh"], Fref),
                         force_err(eg["Fc"], eo["Fc"], Fref))
        Tref = Fref * wl.scene.size.max()
        worst["T"] = max(worst["T"], force_err(eg["Th"], eo["Th"], Tref))
        worst["pop"] = max(worst["pop"], rel_field(g.populations(), o.populations()))
        po, pg = o.particles(), g.particles()
        worst["X"] = max(worst["X"], np.abs(pg["X"] - po["X"]).max())
        Uref = max(np.abs(po["U"]).max(), 1e-12)
        worst["U"] = max(worst["U"], np.abs(pg["U"] - po["U"]).max() / Uref)
        if prec == 0:
            assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    _say("  worst", {k: f"{v:.2e}" for k, v in worst.items()})
    assert worst["F"] <= tol and worst["T"] <= tol
    assert worst["pop"] <= tol
    assert worst["U"] <= tol and worst["X"] <= tol


def test_walled_settling_workload_parity(O, W, H):
    """128^3 box with walls in z, 121 cubes a=12 (FP64): 20 coupled steps."""
    wl = W.c2_settling_walls()
    _say("C2 parity")
    o, g = _pair(O, H, wl.params, wl.scene)
    V = wl.scene.size ** 3
    Fref = ((wl.scene.density - 1) * V).max() * abs(wl.params.gravity[2])
    for _ in range(2):
        o.step(10)
        g.step(10)
        eo, eg = o.forces(), g.forces()
        err = max(force_err(eg["Fh"], eo["Fh"], Fref), force_err(eg["Fc"], eo["Fc"], Fref))
        _say(f"  C2 step {o.step_count}: force err {err:.2e}")
        assert err <= 1e-12
        assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
        oc, gc = o.contacts(), g.contacts()
        assert [(c["a"], c["b"], c["count"]) for c in oc] == \
               [(c["a"], c["b"], c["count"]) for c in gc]
    assert rel_field(g.populations(), o.populations()) <= 1e-12


@pytest.mark.parametrize("prec", [0, 2])
def test_state_checkpoint_resume(W, H, prec):
    """A state saved to the host and restored into a fresh context continues
    bit for bit like the original."""
    sc = W.random_small_scene(31, (22, 26, 19), 6, size_range=(1.6, 2.8),
                              gap=-0.6, speed=0.01, spin=0.004)
    p = W.Params(nx=22, ny=26, nz=19, tau=0.7, gravity=(0.0, 0.0, -2e-4),
                 balance=1, young=0.4, u_k=3e-4, max_pairs=256,
                 tile_capacity=16, precision=prec)
    a = H.Simulation(p, sc)
    a.init_equilibrium(u=(0.002, 0.0, -0.001))
    a.step(5)
    blob = a.get_state()
    a.step(7)
    b = H.Simulation(p, sc)
    b.set_state(blob)
    b.step(7)
    assert np.array_equal(a.populations(), b.populations())
    pa, pb = a.particles(), b.particles()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k
    assert [(c["a"], c["b"], c["count"], c["volume"]) for c in a.contacts()] == \
           [(c["a"], c["b"], c["count"], c["volume"]) for c in b.contacts()]
    assert a.counters()["steps"] == b.counters()["steps"]
    # a blob of another configuration is refused
    other = H.Simulation(p.replace(nx=23), sc)
    with pytest.raises(H.HlbmError) as e:
        other.set_state(blob)
    assert e.value.code == -1


@pytest.mark.parametrize("n_sub", [2, 3])
def test_substep_parity(O, W, H, n_sub):
    """Contact sub-steps (treatment, motion over 1/n_sub, detection, with
    the hydrodynamic force held) against the oracle, FP64, with walls."""
    seed, dims, n, pz = CASES[1]
    sc = W.random_small_scene(seed, dims, n, periodic_z=pz,
                              size_range=(1.6, 3.0), gap=-0.8, speed=0.01,
                              spin=0.004)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, n_sub=n_sub)
    f0 = W.perturbed_populations(seed, dims, O.feq(1.0, [0.004, -0.002, 0.001]),
                                 amp=0.01)
    o, g = _pair(O, H, p, sc, f0)
    Fref = np.abs(np.array(p.gravity)).max() * 0.5 * (4 / 3 * math.pi * 1.6 ** 3)
    for _ in range(3):
        o.step(2)
        g.step(2)
        eo, eg = o.forces(), g.forces()
        err = max(force_err(eg["Fh"], eo["Fh"], Fref), force_err(eg["Fc"], eo["Fc"], Fref))
        _say(f"  n_sub {n_sub} step {o.step_count}: force {err:.2e}")
        assert err <= 1e-11
        assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
        assert [(c["a"], c["b"], c["count"]) for c in o.contacts()] == \
               [(c["a"], c["b"], c["count"]) for c in g.contacts()]
        po, pg = o.particles(), g.particles()
        assert np.abs(pg["X"] - po["X"]).max() <= 1e-12 * max(dims)
    assert rel_field(g.populations(), o.populations()) <= 1e-12


def test_substep_graph_matches_stream(W, H):
    sc = W.random_small_scene(22, (24, 20, 16), 6, size_range=(1.6, 2.8),
                              gap=-0.6, speed=0.01)
    p = W.Params(nx=24, ny=20, nz=16, tau=0.7, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=1, n_sub=2)
    a = H.Simulation(p, sc)
    b = H.Simulation(p, sc, graph=True)
    a.init_equilibrium(u=(0.003, 0, 0))
    b.init_equilibrium(u=(0.003, 0, 0))
    for _ in range(3):
        a.step(3)
        b.step(3)
        assert np.array_equal(b.populations(), a.populations())
        pa, pb = a.particles(), b.particles()
        assert np.array_equal(pa["X"], pb["X"])
        assert [(c["a"], c["b"], c["count"]) for c in a.contacts()] == \
               [(c["a"], c["b"], c["count"]) for c in b.contacts()]


@pytest.mark.parametrize("prec", [0, 1])
def test_octahedra_parity(O, W, H, prec):
    """Scenes mixing spheres, cubes and regular octahedra: owner map, pair
    set and counts bit-exact at the start (and after each FP64 step), fields
    and forces within the precision's tolerance."""
    seed, dims, n, pz = 41, (28, 24, 20), 8, 1
    sc = W.random_small_scene(seed, dims, n, periodic_z=pz, size_range=(1.6, 3.0),
                              gap=-0.8, speed=0.01, spin=0.004, shapes=(0, 1, 2))
    assert (sc.shape == 2).sum() >= 3
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7,
                 gravity=(0.0, 0.0, -2e-4), balance=1, young=0.4, u_k=3e-4,
                 max_pairs=256, tile_capacity=16, precision=prec)
    f0 = W.perturbed_populations(seed, dims, O.feq(1.0, [0.003, 0.002, -0.001]),
                                 amp=0.01)
    o, g = _pair(O, H, p, sc, f0)
    assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    oc = o.contacts()
    assert any(sc.shape[c["a"]] == 2 or (c["b"] >= 0 and sc.shape[c["b"]] == 2) for c in oc)
    compare_contacts(oc, g.contacts(), 0.0)
    Fref = np.abs(np.array(p.gravity)).max() * 0.5 * (4 / 3 * math.pi * 1.6 ** 3)
    tol = TOL[prec]
    for k in range(3):
        o.step(2)
        g.step(2)
        eo, eg = o.forces(), g.forces()
        err = max(force_err(eg["Fh"], eo["Fh"], Fref), force_err(eg["Fc"], eo["Fc"], Fref))
        _say(f"  octahedra precision {prec} step {o.step_count}: force {err:.2e}")
        assert err <= FTOL[prec]
        if prec == 0:
            assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
            assert [(c["a"], c["b"], c["count"]) for c in o.contacts()] == \
                   [(c["a"], c["b"], c["count"]) for c in g.contacts()]
    assert rel_field(g.populations(), o.populations()) <= tol


@pytest.mark.parametrize("case", CASES)
def test_coupling_field_parity(O, W, H, case):
    """The per-node coupling weight B(d_owner) and particle velocity u_p
    (Sec. 3.2) against the oracle's, at the start and after moving steps."""
    seed, dims, n, pz = case
    sc = W.random_small_scene(seed, dims, n, periodic_z=pz, size_range=(1.6, 3.0),
                              gap=-0.8, speed=0.01, spin=0.004, shapes=(0, 1, 2))
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7,
                 young=0.4, u_k=3e-4, max_pairs=256, tile_capacity=16)
    o, g = _pair(O, H, p, sc)
    for k in range(2):
        fo, fg = o.fields(), g.coupling()
        assert (fo["B"] > 0).sum() > 100
        assert np.abs(fg["B"] - fo["B"]).max() <= 1e-14
        assert np.abs(fg["up"] - fo["up"]).max() <= 1e-15
        o.step(3)
        g.step(3)


@pytest.mark.parametrize("pz", [1, 0])
def test_no_particles_pure_fluid(O, W, H, pz):
    """An empty particle set: the step is the plain stream-collide (with
    half-way bounce-back at walls), FP64 against the oracle."""
    dims = (21, 18, 23)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.62,
                 fluid_accel=(1e-5, 0.0, 0.0),
                 wall_velocity=((0.0, 0.0, 0.0), (0.002, 0.0, 0.0)),
                 young=0.4, u_k=3e-4, max_pairs=16, tile_capacity=4)
    f0 = W.perturbed_populations(5, dims, O.feq(1.0, [0.002, 0.001, 0.0]), amp=0.02)
    o, g = _pair(O, H, p, W.Scene.empty(), f0)
    o.step(7)
    g.step(7)
    assert rel_field(g.populations(), o.populations()) <= 1e-13
    assert g.contacts() == [] and g.counters()["pairs"] == 0
    assert (g.fields()["owner"] == -1).all()


def test_reach_wraps_through_partial_block(O, W, H):
    """A particle whose reach wraps round a periodic x axis through its last,
    partial lattice block (132 = 2 x 64 + 4 nodes) touches three blocks
    along x; its partial-sum slots must hold them (this was reported as a
    capacity overflow).  FP64 against the oracle over three steps."""
    dims = (132, 24, 24)
    sc = W.Scene(np.array([0, 1], np.int32), np.array([8.5, 7.0]), np.array([1.5, 1.5]),
                 np.array([[125.5, 11.0, 12.0], [60.0, 12.5, 11.0]]),
                 np.array([[1.0, 0, 0, 0], [0.9, 0.3, -0.2, 0.1]]) /
                 np.linalg.norm([[1.0, 0, 0, 0], [0.9, 0.3, -0.2, 0.1]], axis=1)[:, None],
                 np.array([[0.004, 0.001, 0.0], [-0.002, 0.0, 0.001]]), np.zeros((2, 3)))
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=1, tau=0.7,
                 gravity=(0.0, 0.0, -1e-5), young=0.4, u_k=3e-4,
                 max_pairs=16, tile_capacity=8, precision=0)
    f0 = W.perturbed_populations(9, dims, O.feq(1.0, [0.002, 0.0, 0.001]), amp=0.01)
    o, g = _pair(O, H, p, sc, f0)
    assert np.array_equal(g.fields()["owner"], o.fields()["owner"])
    Fref = 1e-5 * 0.5 * 4.0 / 3.0 * math.pi * 8.5 ** 3
    for _ in range(3):
        o.step(1)
        g.step(1)
        eo, eg = o.forces(), g.forces()
        assert np.abs(eg["Fh"] - eo["Fh"]).max() <= 1e-12 * max(np.abs(eo["Fh"]).max(), Fref)
        assert np.abs(eg["Th"] - eo["Th"]).max() <= 1e-12 * max(np.abs(eo["Th"]).max(), Fref * 8.5)


def test_pair_table_overflow_reported(W, H):
    """More contact pairs than the table holds is an error, not a silent
    truncation."""
    sc = W.random_small_scene(3, (20, 20, 20), 10, size_range=(2.0, 3.0), gap=-1.2)
    p = W.Params(nx=20, ny=20, nz=20, tau=0.7, young=0.4, u_k=3e-4,
                 max_pairs=1, tile_capacity=32)
    g = H.Simulation(p, sc)
    with pytest.raises(H.HlbmError) as e:
        g.init_equilibrium()
    assert e.value.code == -4


def test_oversized_lattice_rejected(W, H):
    """32-bit population offsets: a lattice with 19 N >= 2^31 is refused
    before any allocation."""
    p = W.Params(nx=1400, ny=1400, nz=1400, tau=0.7, young=0.4, u_k=3e-4)
    with pytest.raises(H.HlbmError):
        H.Simulation(p, W.Scene.empty())
