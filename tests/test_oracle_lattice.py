"""Pins of the oracle's lattice Boltzmann part (Sec. 3.1, eqs. (10)-(13)).

Each check is fixed by mathematics independent of the code under test:
lattice isotropy identities, moments of the second-order equilibrium,
exact conservation laws, and two closed-form channel flows.
"""
import math

import numpy as np
import pytest


def test_velocity_set_identities(O):
    c, w, opp = O.lattice()
    assert c.shape == (19, 3)
    # all 19 D3Q19 velocities, each exactly once: |c|^2 in {0, 1, 2}
    sq = (c * c).sum(1)
    assert sorted(sq.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c}) == 19
    np.testing.assert_array_equal(c[opp], -c)
    # Gauss-Hermite isotropy: sum w = 1, sum w c c = cs^2 I,
    # sum w c_a c_b c_c c_d = cs^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c),
                               cs2 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    T4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = cs2 * cs2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(T4, iso, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(O, seed):
    """sum f = rho, sum c f = rho u, sum c c f = rho (cs^2 I + u u)."""
    rng = np.random.default_rng(seed)
    c, w, _ = O.lattice()
    rho = rng.uniform(0.8, 1.2)
    u = rng.uniform(-0.05, 0.05, 3)
    f = O.feq(rho, u)
    assert abs(f.sum() - rho) < 1e-15
    np.testing.assert_allclose((c * f[:, None]).sum(0), rho * u, atol=1e-16)
    P = np.einsum("i,ia,ib->ab", f, c, c)
    np.testing.assert_allclose(P, rho * (np.eye(3) / 3.0 + np.outer(u, u)),
                               atol=2e-16)


def test_printed_sign_would_break_mass(O):
    """With '+' on the u.u term (as printed) sum f^eq = rho (1 + 3 u.u):
    the oracle's equilibrium must not show that excess."""
    u = np.array([0.037, 0.0, 0.0])
    f = O.feq(1.0, u)
    assert abs(f.sum() - 1.0) < 1e-15
    assert abs((1.0 + 3.0 * u @ u) - 1.0) > 4e-3


def test_periodic_box_conserves_mass_and_momentum(O, W):
    """Particle-free periodic box: BGK conserves mass and momentum exactly."""
    p = W.Params(nx=12, ny=10, nz=8, tau=0.6)
    s = O.OracleSim(p, W.Scene.empty())
    f0 = W.perturbed_populations(11, (12, 10, 8), O.feq(1.0, [0, 0, 0]), amp=0.05)
    s.set_populations(f0)
    c, _, _ = O.lattice()
    m0 = f0.sum()
    j0 = np.einsum("ia,izyx->a", c.astype(float), f0)
    s.step(300)
    f = s.populations()
    assert abs(f.sum() - m0) / m0 < 1e-13
    j = np.einsum("ia,izyx->a", c.astype(float), f)
    assert np.abs(j - j0).max() / m0 < 1e-13


def test_couette_linear_profile(O, W):
    """Moving top wall, fixed bottom wall, half-way bounce-back: the linear
    profile u_x(z) = U (z + 1/2) / H is an exact steady solution."""
    H, Uw = 16, 0.01
    p = W.Params(nx=2, ny=2, nz=H, periodic_z=0, tau=1.0,
                 wall_velocity=((0.0, 0.0, 0.0), (Uw, 0.0, 0.0)))
    s = O.OracleSim(p, W.Scene.empty())
    s.init_equilibrium()
    s.step(6000)
    u = s.fields()["u"][:, 0, 0, 0]
    z = np.arange(H)
    np.testing.assert_allclose(u, Uw * (z + 0.5) / H, rtol=0, atol=1e-12)


def test_poiseuille_exact_at_magic_tau(O, W):
    """Body-force driven channel between walls at -1/2 and H-1/2 (EDM source,
    eq. (14), with a uniform acceleration).  The physical velocity
    u + du/2 matches a/(2 nu) (z + 1/2)(H - 1/2 - z); with half-way
    bounce-back the BGK solution is exact for tau = 1/2 + sqrt(3/16)."""
    H, a = 8, 1e-6
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    p = W.Params(nx=2, ny=2, nz=H, periodic_z=0, tau=tau, fluid_accel=(a, 0, 0))
    s = O.OracleSim(p, W.Scene.empty())
    s.init_equilibrium()
    s.step(int(30 * H * H / nu))
    ustar = s.fields()["u"][:, 0, 0, 0]   # post-collision moment u + du
    z = np.arange(H)
    ex = a / (2 * nu) * (z + 0.5) * (H - 0.5 - z)
    assert np.abs((ustar - a / 2) - ex).max() / ex.max() < 1e-10


def test_poiseuille_second_order(O, W):
    """Away from the magic tau the wall slip error falls as H^-2."""
    tau, a = 0.8, 1e-6
    nu = (tau - 0.5) / 3.0
    errs = []
    for H in (8, 16):
        p = W.Params(nx=2, ny=2, nz=H, periodic_z=0, tau=tau,
                     fluid_accel=(a, 0, 0))
        s = O.OracleSim(p, W.Scene.empty())
        s.init_equilibrium()
        s.step(int(30 * H * H / nu))
        u = s.fields()["u"][:, 0, 0, 0] - a / 2
        z = np.arange(H)
        ex = a / (2 * nu) * (z + 0.5) * (H - 0.5 - z)
        errs.append(np.abs(u - ex).max() / ex.max())
    order = math.log2(errs[0] / errs[1])
    assert 1.9 < order < 2.1, errs
