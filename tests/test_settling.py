"""Hindered-settling statistics (Sec. 5): correlations, the single-particle
velocity, the time scale and the settling-box generator (CPU), and one
short settling run through the library (GPU)."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2401_10878_amd import settling as S  # noqa: E402
from paper_2401_10878_amd import workloads as W  # noqa: E402


def test_schiller_naumann_closed_form():
    # Re = 1: 24 (1 + 0.15); Re = 100: 0.24 (1 + 0.15 * 100^0.687)
    assert S.schiller_naumann_cd(1.0) == pytest.approx(27.6, rel=1e-15)
    assert S.schiller_naumann_cd(100.0) == pytest.approx(
        0.24 * (1.0 + 0.15 * math.exp(0.687 * math.log(100.0))), rel=1e-14)


@pytest.mark.parametrize("ar", [1.0, 500.0, 1000.0, 2000.0])
def test_single_particle_velocity_solves_its_equation(ar):
    nu, d, s = (0.55 - 0.5) / 3.0, 9.0, 3.3
    g = ar * nu * nu / (d ** 3 * (s - 1.0))
    u = S.single_particle_velocity(g, d, s, nu)
    cd = S.schiller_naumann_cd(u * d / nu)
    assert u == pytest.approx(math.sqrt(4.0 * g * d * (s - 1.0) / (3.0 * cd)),
                              rel=1e-12)
    # below the Stokes velocity, approaching it as Re -> 0
    stokes = g * d * d * (s - 1.0) / (18.0 * nu)
    assert u < stokes
    re = u * d / nu
    assert u == pytest.approx(stokes / (1.0 + 0.15 * re ** 0.687), rel=1e-10)


def test_expansion_indices_piecewise():
    assert S.n_richardson_zaki(0.1) == 4.65
    assert S.n_richardson_zaki(0.5) == pytest.approx(4.35 * 0.5 ** -0.03)
    assert S.n_richardson_zaki(10.0) == pytest.approx(4.45 * 10.0 ** -0.1)
    assert S.n_richardson_zaki(600.0) == 2.39
    # Garside and Al-Dibouni: 5.1 at Re -> 0, 2.7 at Re -> infinity
    assert S.n_garside_al_dibouni(1e-12) == pytest.approx(5.1, rel=1e-9)
    assert S.n_garside_al_dibouni(1e12) == pytest.approx(2.7, rel=1e-6)
    assert S.k_yao(0.0) == 0.89
    assert S.k_yao(1e5) == pytest.approx(0.89 / math.e)
    assert S.power_law(0.0, 0.9, 4.0) == 0.9
    assert S.power_law(0.5, 1.0, 2.0) == 0.25


def test_time_scale_and_average():
    nu, d, s, ar = (0.55 - 0.5) / 3.0, 9.0, 3.3, 1000.0
    g = ar * nu * nu / (d ** 3 * (s - 1.0))
    # with Ar fixed, D g (s-1) / (18 nu) = Ar nu / (18 D^2)
    assert S.tstar_per_step(d, g, s, nu) == pytest.approx(
        ar * nu / (18.0 * d * d), rel=1e-14)
    t = np.linspace(0.0, 10.0, 101)
    v = np.where(t < 2.0, t, 2.0)          # ramp, then a plateau
    assert S.time_average(t, v, 2.0) == pytest.approx(2.0)
    assert S.time_average(t, 3.0 * t, 0.0) == pytest.approx(15.0)
    with pytest.raises(ValueError):
        S.time_average(t, v, 11.0)


@pytest.mark.parametrize("shape", [W.SPHERE, W.CUBE])
@pytest.mark.parametrize("phi", [0.1, 0.3])
def test_settling_box_generator(shape, phi):
    wl = W.settling_box(shape, phi, 9.0, edge_cells=120, ar=1000.0)
    p, sc = wl.params, wl.scene
    assert (p.nx, p.ny, p.nz, p.periodic_z, p.balance) == (120, 120, 120, 1, 2)
    vol = (4.0 / 3.0 * np.pi * sc.size ** 3 if shape == W.SPHERE
           else sc.size ** 3).sum()
    assert vol / 120 ** 3 == pytest.approx(phi, abs=5e-4)
    # same particle volume for both shapes: that of a sphere of diameter 9
    v1 = (4.0 / 3.0 * np.pi * sc.size[0] ** 3 if shape == W.SPHERE
          else sc.size[0] ** 3)
    assert v1 == pytest.approx(np.pi / 6.0 * 729.0, rel=1e-12)
    assert np.all(sc.density == 3.3) and np.all(sc.U == 0.0)
    # gravity from the Archimedes number: Ar = g D^3 (s - 1) / nu^2
    nu = (p.tau - 0.5) / 3.0
    assert -p.gravity[2] * 729.0 * 2.3 / nu ** 2 == pytest.approx(1000.0)
    # no two spheres of diameter 9 (the centre spacing) overlap
    d = W._minimg(sc.X[:, None, :] - sc.X[None, :, :], np.full(3, 120.0),
                  np.ones(3, bool))
    dist = np.sqrt((d * d).sum(-1)) + np.eye(sc.n) * 1e9
    assert dist.min() >= 9.0
    if shape == W.CUBE:
        R = W._rotation_matrices(sc.q)
        h = 0.5 * sc.size[0]
        close = np.argwhere(dist < 2.0 * h * math.sqrt(3.0))
        for i, j in close[close[:, 0] < close[:, 1]]:
            assert not W._obb_overlap(np.zeros(3), R[i], h, d[j, i], R[j], h)


@pytest.mark.parametrize("shape", [W.OCTAHEDRON, "box", "tetrahedron"])
def test_settling_box_other_bodies(shape):
    """Octahedra, 1 : 1.25 : 1.6 boxes and regular tetrahedra of the volume
    of the sphere of diameter 9; the volume fraction from that diameter."""
    wl = W.settling_box(shape, 0.1, 9.0, edge_cells=60, ar=1000.0)
    sc = wl.scene
    vs = np.pi / 6.0 * 729.0
    if shape == W.OCTAHEDRON:
        assert np.all(sc.shape == W.OCTAHEDRON)
        assert 4.0 / 3.0 * sc.size[0] ** 3 == pytest.approx(vs, rel=1e-12)
    else:
        assert np.all(sc.shape == W.POLY0) and np.all(sc.size == 1.0)
        v = wl.polyhedra[0].vertices
        if shape == "box":
            e = v.max(0) - v.min(0)
            assert e[1] / e[0] == pytest.approx(1.25) and e[2] / e[0] == pytest.approx(1.6)
            assert np.prod(e) == pytest.approx(vs, rel=1e-12)
        else:
            edge = np.linalg.norm(v[0] - v[1])
            assert edge ** 3 / (6.0 * np.sqrt(2.0)) == pytest.approx(vs, rel=1e-12)
    assert wl.d_equiv == 9.0
    assert S._phi(wl) == pytest.approx(0.1, abs=5e-3)
    assert np.allclose(np.linalg.norm(sc.q, axis=1), 1.0)


@pytest.mark.gpu
def test_gpu_short_settling_run():
    """A small sphere box settles: the bulk velocity along gravity grows from
    rest, stays finite and below u*, and the run reports its inputs."""
    wl = W.settling_box(W.SPHERE, 0.1, 6.0, edge_cells=36, ar=1000.0)
    r = S.settling_run(wl, t_end=8.0, t_avg=4.0, sample_every=20)
    u = np.asarray(r["series_u_over_u_star"])
    print(f"  n={r['n_particles']} steps={r['steps']} u/u*={r['u_bar_over_u_star']:.4f}"
          f" Re={r['re']:.2f}")
    assert np.all(np.isfinite(u))
    assert u[0] == 0.0 and u[-1] > 0.05
    assert 0.0 < r["u_bar_over_u_star"] < 1.0
    assert r["ar"] == pytest.approx(1000.0, rel=1e-12)
    assert r["n_particles"] == wl.scene.n and r["steps"] % 20 == 0
