"""Pins of the oracle's fluid-particle coupling (Sec. 3.2-3.3, eqs. (14)-(18)).

* node ownership, coupling weight, particle velocity and rough contact
  detection against an all-nodes x all-particles x all-periodic-images brute
  force on small boxes (this pins the bounding-box scatter, the periodic
  image handling and the per-node detection lists);
* the momentum exchange sum against a conservation identity: BGK + EDM
  keep mass and add rho du of momentum at a node, so for every owned node
  S = rho(t-1) du(t-1) + J(t-1) - J(t) - u_p (rho(t-1) - rho(t));
* the drag sign on a sphere driven through resting fluid, and the mirror
  symmetry of the head-on two-sphere workload.
"""
import itertools
import math

import numpy as np
import pytest

THETA = math.sqrt(0.75)


def _images(p):
    shifts = []
    for kx, ky in itertools.product((-1, 0, 1), repeat=2):
        for kz in ((-1, 0, 1) if p.periodic_z else (0,)):
            shifts.append(np.array([kx * p.nx, ky * p.ny, kz * p.nz], float))
    return shifts


def brute_force(O, p, sc):
    """Owner, B, u_p, pair counts and node-image boxes from first principles."""
    nz, ny, nx = p.nz, p.ny, p.nx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    nodes = np.stack([x, y, z], -1).reshape(-1, 3).astype(float)
    n = nodes.shape[0]
    shifts = _images(p)
    D = np.full((sc.n, n), np.inf)
    near_img = np.zeros((sc.n, n, 3))       # image of the node nearest X_p
    for ip in range(sc.n):
        best = np.full(n, np.inf)
        for sh in shifts:
            img = nodes + sh
            dd = np.array([O.sdf(sc.shape[ip], sc.size[ip], sc.q[ip],
                                 v - sc.X[ip]) for v in img])
            D[ip] = np.minimum(D[ip], dd)
            dist = np.linalg.norm(img - sc.X[ip], axis=1)
            better = dist < best
            best[better] = dist[better]
            near_img[ip][better] = img[better]
    owner = np.full(n, -1)
    B = np.zeros(n)
    up = np.zeros((n, 3))
    for c in range(n):
        cand = [(D[ip, c], ip) for ip in range(sc.n) if D[ip, c] < 0.5 * p.eps_b]
        if cand:
            d, ip = min(cand)
            owner[c] = ip
            B[c] = O.weight(d, p.eps_b)
            r = near_img[ip, c] - sc.X[ip]
            up[c] = sc.U[ip] + np.cross(sc.omega[ip], r)
    pairs = {}
    for c in range(n):
        K = [ip for ip in range(sc.n) if D[ip, c] - p.enlarge < THETA]
        members = [(a, b) for a, b in itertools.combinations(sorted(K), 2)]
        if not p.periodic_z:
            zc = nodes[c, 2]
            for ip in K:
                if zc + 0.5 < THETA:
                    members.append((ip, -1))
                if (p.nz - 0.5) - zc < THETA:
                    members.append((ip, -2))
        for a, b in members:
            img = near_img[a, c].astype(int)
            e = pairs.setdefault((a, b), [0, img.copy(), img.copy()])
            e[0] += 1
            e[1] = np.minimum(e[1], img)
            e[2] = np.maximum(e[2], img)
    return owner.reshape(nz, ny, nx), B.reshape(nz, ny, nx), \
        up.reshape(nz, ny, nx, 3), pairs


@pytest.mark.parametrize("seed,dims,npart,pz", [
    (1, (14, 12, 10), 5, 1),
    (2, (13, 11, 12), 6, 0),
    (3, (12, 12, 12), 4, 1),
])
def test_coupling_and_detection_brute_force(O, W, seed, dims, npart, pz):
    sc = W.random_small_scene(seed, dims, npart, periodic_z=pz,
                              size_range=(1.5, 2.6), gap=-0.6)
    p = W.Params(nx=dims[0], ny=dims[1], nz=dims[2], periodic_z=pz, tau=0.7)
    s = O.OracleSim(p, sc)
    s.init_equilibrium()
    owner, B, up, pairs = brute_force(O, p, sc)
    fl = s.fields()
    np.testing.assert_array_equal(fl["owner"], owner)
    np.testing.assert_allclose(fl["B"], B, atol=1e-15)
    np.testing.assert_allclose(fl["up"], up, atol=1e-15)
    con = s.contacts()
    got = {(c["a"], c["b"]): (c["count"], c["rlo"], c["rhi"]) for c in con}
    assert set(got) == set(pairs)
    assert len(pairs) > 0
    for k, (cnt, lo, hi) in pairs.items():
        assert got[k][0] == cnt
        assert tuple(got[k][1]) == tuple(lo.tolist())
        assert tuple(got[k][2]) == tuple(hi.tolist())
    # list is sorted by (a, b) and new boxes are [min - 1/2, max + 1/2]
    keys = [(c["a"], c["b"]) for c in con]
    assert keys == sorted(keys)
    for c in con:
        assert c["lo"] == tuple(v - 0.5 for v in c["rlo"])
        assert c["hi"] == tuple(v + 0.5 for v in c["rhi"])


def test_coverage_lemma(O, W):
    """The rough box [min - 1/2, max + 1/2] contains the enlarged overlap."""
    rng = np.random.default_rng(5)
    p = W.Params(nx=24, ny=24, nz=24, tau=0.7)
    checked = 0
    for trial in range(12):
        shape = rng.integers(0, 2, 2).astype(np.int32)
        size = np.where(shape == 0, rng.uniform(2.0, 3.5, 2),
                        rng.uniform(3.0, 5.0, 2))
        rb = np.where(shape == 0, size, 0.5 * size * math.sqrt(3.0))
        Xa = rng.uniform(0, 24, 3)
        dvec = rng.standard_normal(3)
        dvec /= np.linalg.norm(dvec)
        Xb = Xa + dvec * 0.8 * (rb[0] + rb[1])
        X = np.stack([Xa, np.mod(Xb, 24.0)])
        q = W.random_quaternions(rng, 2)
        sc = W.Scene(shape, size, np.array([1.5, 1.5]), X, q,
                     np.zeros((2, 3)), np.zeros((2, 3)))
        s = O.OracleSim(p, sc)
        s.init_equilibrium()
        for c in s.contacts():
            a, b = c["a"], c["b"]
            Xbi = sc.X[a] + ((sc.X[b] - sc.X[a] + 12.0) % 24.0 - 12.0)
            lo, hi = np.array(c["lo"]), np.array(c["hi"])
            pts = sc.X[a] + rng.uniform(-8, 8, (20000, 3))
            da = np.array([O.sdf(sc.shape[a], sc.size[a], sc.q[a], v - sc.X[a])
                           for v in pts]) - p.enlarge
            db = np.array([O.sdf(sc.shape[b], sc.size[b], sc.q[b], v - Xbi)
                           for v in pts]) - p.enlarge
            inside = (da < 0) & (db < 0)
            if inside.any():
                checked += 1
                q_in = pts[inside]
                assert np.all(q_in >= lo - 1e-12) and np.all(q_in <= hi + 1e-12)
    assert checked >= 8


def _run_and_check_identity(O, s):
    """One step; compare the momentum-exchange sum with the identity."""
    rho_p, J_p, du_p = s.collision_diag()
    up_p = s.fields()["up"]
    owner_p = s.fields()["owner"]
    s.step(1)
    S = s.mea_cells()
    f = s.post_stream()
    c, _, _ = O.lattice()
    rho_t = f.sum(0)
    J_t = np.einsum("ia,izyx->zyxa", c.astype(float), f)
    ident = (rho_p[..., None] * du_p + J_p - J_t
             - up_p * (rho_p - rho_t)[..., None])
    own = owner_p >= 0
    assert own.sum() > 50
    err = np.abs(S[own] - ident[own]).max()
    scale = np.abs(ident[own]).max()
    assert err <= 1e-13 * max(scale, 1e-3), (err, scale)


def test_momentum_exchange_identity(O, W):
    sc = W.random_small_scene(4, (16, 14, 12), 4, size_range=(2.0, 3.0),
                              gap=0.5, speed=0.02, spin=0.01)
    p = W.Params(nx=16, ny=14, nz=12, tau=0.65)
    s = O.OracleSim(p, sc)
    f0 = W.perturbed_populations(9, (16, 14, 12), O.feq(1.0, [0.01, 0, 0]),
                                 amp=0.02)
    s.set_populations(f0)
    s.step(3)
    _run_and_check_identity(O, s)


def test_momentum_exchange_identity_walls(O, W):
    sc = W.random_small_scene(6, (14, 12, 16), 3, periodic_z=0,
                              size_range=(1.6, 2.4), gap=0.5, speed=0.02)
    p = W.Params(nx=14, ny=12, nz=16, periodic_z=0, tau=0.7,
                 wall_velocity=((0.0, 0.0, 0.0), (0.01, 0.0, 0.0)))
    s = O.OracleSim(p, sc)
    s.init_equilibrium()
    s.step(4)
    _run_and_check_identity(O, s)


def test_drag_opposes_motion(O, W):
    """A very heavy sphere moving through resting fluid feels F.U < 0."""
    p = W.Params(nx=32, ny=24, nz=24, tau=0.8)
    sc = W.Scene(np.array([0], np.int32), np.array([4.0]), np.array([1e9]),
                 np.array([[12.0, 12.0, 12.0]]), np.array([[1.0, 0, 0, 0]]),
                 np.array([[0.02, 0.005, 0.0]]), np.zeros((1, 3)))
    s = O.OracleSim(p, sc)
    s.init_equilibrium()
    for _ in range(6):
        s.step(5)
        F = s.forces()["Fh"][0]
        assert F @ sc.U[0] < 0.0


def test_two_sphere_mirror_symmetry(O, W):
    """C1 geometry: forces are mirror images, transverse components vanish."""
    wl = W.c1_two_spheres()
    s = O.OracleSim(wl.params, wl.scene)
    s.init_equilibrium()
    for _ in range(4):
        s.step(5)
        F = s.forces()["Fh"]
        scale = np.abs(F).max()
        assert abs(F[0, 0] + F[1, 0]) <= 1e-12 * scale
        assert np.abs(F[:, 1:]).max() <= 1e-12 * scale
        X = s.particles()["X"]
        assert abs((X[0, 0] - 16.0) + (X[1, 0] - 16.0)) < 1e-12
