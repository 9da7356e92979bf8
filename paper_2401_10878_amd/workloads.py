"""Seeded synthetic inputs: lattice parameters and particle scenes.

This module is the only code that both the FP64 oracle and the GPU library
consume.  It produces *inputs* (parameter records, particle poses, perturbed
population fields) and holds none of the method's arithmetic: no
equilibrium, no signed distance, no coupling, no contact law.

Physical set-up (paper Sec. 5.1, "Simulation setup"): spheres of diameter
D_s = 1.5 mm, fluid density 1000 kg/m^3, standard gravity, a periodic cubic
box, relaxation time tau = 0.55, contact resolution 8, enlargement by
Delta x / 5, restitution 0.926, kinetic/static friction 0.16/0.32,
Young's modulus 5 kPa; u_k = 0.001 m/s (Sec. 2.3, after eq. (9)).
Lattice parameters follow from the Archimedes number (eq. (25)).

Workloads (synthetic random suspensions, as in the paper's own experiments):
  C1  32^3 periodic, 2 spheres D=8 approaching head-on, tau 0.8, no gravity
  C2  128^3, walls in z, ~121 cubes a=12, phi 0.10, s 1.5, Ar 500
  C3  256^3 periodic, 1834 cubes a=14, phi 0.30, s 1.5, Ar 1000
  C4  256^3 periodic, 1834 spheres D=17.37 (volume-equivalent), Ar 2000
  C5  96^3 periodic, 27 cubes a=10 on a jittered 3x3x3 grid, Ar 500
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SPHERE = 0
CUBE = 1
OCTAHEDRON = 2         # size = centre-to-vertex distance
POLY0 = 3              # shape POLY0 + k: convex polyhedron type k, size = scale

# Physical constants of the hindered-settling set-up (Sec. 5.1, Sec. 2.3).
D_S_PHYS = 1.5e-3          # m
RHO_F_PHYS = 1000.0        # kg/m^3
G_PHYS = 9.80665           # m/s^2
E_PHYS = 5.0e3             # Pa
U_K_PHYS = 1.0e-3          # m/s
RESTITUTION = 0.926
MU_K = 0.16
MU_S = 0.32
POISSON = 0.3              # not given in the paper; a common value for solids
CONTACT_RES = 8
ENLARGE = 0.2              # Delta x / 5 in lattice units
EPS_B = 1.0                # width of the coupling-weight transition band


@dataclasses.dataclass
class Params:
    """Flat parameter record; field names mirror the C-ABI struct."""
    nx: int
    ny: int
    nz: int
    periodic_z: int = 1
    tau: float = 0.55
    wall_velocity: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    gravity: tuple = (0.0, 0.0, 0.0)
    fluid_accel: tuple = (0.0, 0.0, 0.0)
    balance: int = 0
    eps_b: float = EPS_B
    enlarge: float = ENLARGE
    n_c: int = CONTACT_RES
    young: float = 0.0
    poisson: float = POISSON
    restitution: float = RESTITUTION
    mu_s: float = MU_S
    mu_k: float = MU_K
    u_k: float = 1.0
    max_pairs: int = 4096
    tile_capacity: int = 48
    precision: int = 0     # 0 FP64, 1 FP32, 2 FP16 storage of deviations
    n_sub: int = 1         # contact sub-steps per time step

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Scene:
    """Particle set in lattice units (float64 / int32 numpy arrays)."""
    shape: np.ndarray      # (n,) int32, SPHERE or CUBE
    size: np.ndarray       # (n,) radius for spheres, edge for cubes
    density: np.ndarray    # (n,) particle/fluid density ratio s
    X: np.ndarray          # (n,3) centre of mass
    q: np.ndarray          # (n,4) unit quaternion (w, x, y, z)
    U: np.ndarray          # (n,3)
    omega: np.ndarray      # (n,3)

    @property
    def n(self) -> int:
        return int(self.shape.shape[0])

    def copy(self) -> "Scene":
        return Scene(*(np.array(getattr(self, f.name), copy=True)
                       for f in dataclasses.fields(self)))

    @staticmethod
    def empty() -> "Scene":
        return Scene(np.zeros(0, np.int32), np.zeros(0), np.zeros(0),
                     np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)),
                     np.zeros((0, 3)))


@dataclasses.dataclass
class Workload:
    name: str
    params: Params
    scene: Scene
    steps: int
    note: str = ""
    polyhedra: Optional[dict] = None   # {type k: Polyhedron or Ellipsoid} for shape POLY0 + k
    d_equiv: Optional[float] = None    # volume-equivalent sphere diameter (settling boxes)


# --------------------------------------------------------------------------
# unit conversion (physical -> lattice), fixed by the Archimedes number
# --------------------------------------------------------------------------
def lattice_units(d_s_cells: float, s: float, ar: float, tau: float) -> dict:
    """Lattice gravity, Young's modulus and u_k for a given resolution.

    nu_lat follows from tau (Sec. 3.1, tau = 3 nu + 1/2 in lattice units);
    Ar = g D^3 (s-1) / nu^2 (eq. (25) with rho_p/rho_f = s) fixes g_lat, and
    the physical viscosity, Delta x and Delta t; E and u_k are then scaled.
    """
    nu = (tau - 0.5) / 3.0
    g_lat = ar * nu * nu / (d_s_cells ** 3 * (s - 1.0))
    nu_phys = math.sqrt(G_PHYS * D_S_PHYS ** 3 * (s - 1.0) / ar)
    dx = D_S_PHYS / d_s_cells
    dt = nu * dx * dx / nu_phys
    e_lat = E_PHYS * dt * dt / (RHO_F_PHYS * dx * dx)
    uk_lat = U_K_PHYS * dt / dx
    return dict(nu=nu, g=g_lat, young=e_lat, u_k=uk_lat, dx=dx, dt=dt,
                nu_phys=nu_phys)


def cube_equiv_diameter(edge: float) -> float:
    """Diameter of the sphere with the volume of a cube of this edge."""
    return edge * (6.0 / math.pi) ** (1.0 / 3.0)


# --------------------------------------------------------------------------
# convex polyhedron geometries (vertices and faces, counter-clockwise seen
# from outside); inputs only, the volume, inertia and distances are the
# method's and live in the library and in the oracle
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Polyhedron:
    vertices: np.ndarray   # (nv, 3)
    faces: list            # vertex-index lists


@dataclasses.dataclass
class Ellipsoid:
    """Smooth convex body type: semi-axes (a, b, c) along the body axes at
    unit scale (registered in the same type slots as the polyhedra)."""
    axes: tuple


def polyhedron_cuboid(a: float, b: float, c: float) -> Polyhedron:
    """Box with edges a, b, c along x, y, z, centred at the origin."""
    h = np.array([a, b, c]) / 2.0
    v = np.array([[sx * h[0], sy * h[1], sz * h[2]]
                  for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)])
    # vertex k = ix + 2 iy + 4 iz with i = 0 for the negative side
    faces = [[0, 2, 3, 1], [4, 5, 7, 6], [0, 1, 5, 4], [2, 6, 7, 3],
             [0, 4, 6, 2], [1, 3, 7, 5]]
    return Polyhedron(v, faces)


def polyhedron_tetrahedron(edge: float = 1.0) -> Polyhedron:
    """Regular tetrahedron on alternate corners of a cube."""
    s = edge / (2.0 * math.sqrt(2.0))
    v = s * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    faces = [[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]]
    return Polyhedron(v, faces)


def polyhedron_octahedron(a: float = 1.0) -> Polyhedron:
    """Regular octahedron |x| + |y| + |z| <= a."""
    v = a * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                      [0, 0, 1], [0, 0, -1]], float)
    faces = [[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
             [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]
    return Polyhedron(v, faces)


def polyhedron_random(rng: np.random.Generator, npts: int = 12,
                      stretch=(1.0, 0.8, 0.6)) -> Polyhedron:
    """Convex hull of random points on a stretched sphere, triangulated,
    each triangle ordered counter-clockwise seen from outside."""
    from scipy.spatial import ConvexHull
    p = rng.normal(size=(npts, 3))
    p /= np.linalg.norm(p, axis=1)[:, None]
    p *= np.asarray(stretch)[None, :]
    hull = ConvexHull(p)
    used = np.unique(hull.simplices)
    remap = -np.ones(npts, int)
    remap[used] = np.arange(used.size)
    faces = []
    for tri, eq in zip(hull.simplices, hull.equations):
        a, b, c = p[tri]
        if np.dot(np.cross(b - a, c - a), eq[:3]) < 0:
            tri = tri[[0, 2, 1]]
        faces.append([int(remap[k]) for k in tri])
    return Polyhedron(p[used], faces)


# --------------------------------------------------------------------------
# random geometry helpers (input generation only)
# --------------------------------------------------------------------------
def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], 1)
    return q


def _rotation_matrices(q: np.ndarray) -> np.ndarray:
    """Rotation matrices for the placement test (scipy, scalar-last order)."""
    from scipy.spatial.transform import Rotation
    return Rotation.from_quat(np.asarray(q)[:, [1, 2, 3, 0]]).as_matrix()


def _obb_overlap(ca, Ra, ha, cb, Rb, hb, margin=0.0) -> bool:
    """Separating-axis test for two cubes (15 axes); True if they overlap.

    Cubes are (centre, rotation whose columns are the body axes, half edge);
    both are grown by `margin` on every face before testing.
    """
    ha = ha + margin
    hb = hb + margin
    t = cb - ca
    axes = [Ra[:, i] for i in range(3)] + [Rb[:, i] for i in range(3)]
    for i in range(3):
        for j in range(3):
            c = np.cross(Ra[:, i], Rb[:, j])
            nn = np.linalg.norm(c)
            if nn > 1e-9:
                axes.append(c / nn)
    for ax in axes:
        ra = ha * np.abs(Ra.T @ ax).sum()
        rb = hb * np.abs(Rb.T @ ax).sum()
        if abs(t @ ax) > ra + rb:
            return False
    return True


def _minimg(v: np.ndarray, L: np.ndarray, periodic: np.ndarray) -> np.ndarray:
    v = v.copy()
    for k in range(3):
        if periodic[k]:
            v[..., k] = v[..., k] - L[k] * np.round(v[..., k] / L[k])
    return v


def rsa_centres(rng, n, dims, min_dist, periodic, lo_margin=None,
                max_tries=2_000_000) -> np.ndarray:
    """Random sequential addition of n centres with pairwise distance >= min_dist.

    Uses a cell list of edge min_dist; periodic axes use the minimal image.
    Along non-periodic axes centres are drawn from [lo_margin, dim-1-lo_margin].
    """
    dims = np.asarray(dims, float)
    periodic = np.asarray(periodic, bool)
    if lo_margin is None:
        lo_margin = np.zeros(3)
    lo_margin = np.asarray(lo_margin, float)
    ncell = np.maximum((dims // min_dist).astype(int), 1)
    csize = dims / ncell
    grid: dict = {}
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"RSA stalled at {k}/{n} centres")
        p = np.empty(3)
        for a in range(3):
            if periodic[a]:
                p[a] = rng.random() * dims[a]
            else:
                lo, hi = lo_margin[a], dims[a] - 1.0 - lo_margin[a]
                p[a] = lo + rng.random() * (hi - lo)
        ci = np.minimum((p // csize).astype(int), ncell - 1)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    cj = ci + np.array([dx, dy, dz])
                    skip = False
                    for a in range(3):
                        if periodic[a]:
                            cj[a] %= ncell[a]
                        elif cj[a] < 0 or cj[a] >= ncell[a]:
                            skip = True
                    if skip:
                        continue
                    for j in grid.get(tuple(cj), ()):
                        d = _minimg(pts[j] - p, dims, periodic)
                        if d @ d < min_dist * min_dist:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            grid.setdefault(tuple(ci), []).append(k)
            k += 1
    return pts


def box_orientations(rng, X, half, dims, periodic, margin=0.3,
                     max_draws=10_000) -> np.ndarray:
    """Random orientations such that no two boxes of half extents `half`
    (grown by margin) overlap; the separating-axis test of
    cube_orientations with unequal half extents."""
    n = X.shape[0]
    dims = np.asarray(dims, float)
    periodic = np.asarray(periodic, bool)
    h = np.asarray(half, float) + margin
    rc = float(np.linalg.norm(h))
    q = np.zeros((n, 4))
    R = np.zeros((n, 3, 3))
    done = np.zeros(n, bool)

    def overlap(Ra, Rb, t):
        axes = [Ra[:, i] for i in range(3)] + [Rb[:, i] for i in range(3)]
        for i in range(3):
            for j in range(3):
                c = np.cross(Ra[:, i], Rb[:, j])
                nn = np.linalg.norm(c)
                if nn > 1e-9:
                    axes.append(c / nn)
        for ax in axes:
            if abs(t @ ax) > (h * np.abs(Ra.T @ ax)).sum() + (h * np.abs(Rb.T @ ax)).sum():
                return False
        return True

    for i in range(n):
        d = _minimg(X - X[i], dims, periodic)
        dist2 = (d * d).sum(1)
        near = np.nonzero(done & (dist2 < (2 * rc) ** 2))[0]
        for draw in range(max_draws):
            qi = random_quaternions(rng, 1)
            Ri = _rotation_matrices(qi)[0]
            if not any(overlap(Ri, R[j], d[j]) for j in near):
                break
        else:
            raise RuntimeError(f"orientation draws stalled at box {i}")
        q[i], R[i], done[i] = qi[0], Ri, True
    return q


def convex_orientations(rng, X, verts, faces, dims, periodic, margin=0.3,
                        max_draws=10_000) -> np.ndarray:
    """Random orientations such that no two copies of the convex body with
    body-frame vertices `verts` and faces `faces` (grown by margin) overlap:
    the separating-axis test over both bodies' face normals and the cross
    products of their edge directions."""
    n = X.shape[0]
    dims = np.asarray(dims, float)
    periodic = np.asarray(periodic, bool)
    verts = np.asarray(verts, float)
    normals = []
    for f in faces:
        a, b, c = verts[f[0]], verts[f[1]], verts[f[2]]
        nv = np.cross(b - a, c - a)
        normals.append(nv / np.linalg.norm(nv))
    normals = np.array(normals)
    edges = set()
    for f in faces:
        for j in range(len(f)):
            i0, i1 = f[j], f[(j + 1) % len(f)]
            edges.add((min(i0, i1), max(i0, i1)))
    edirs = np.array([(verts[b] - verts[a]) / np.linalg.norm(verts[b] - verts[a])
                      for a, b in sorted(edges)])
    rc = float(np.linalg.norm(verts, axis=1).max()) + margin
    q = np.zeros((n, 4))
    R = np.zeros((n, 3, 3))
    done = np.zeros(n, bool)

    def overlap(Ra, Rb, t):
        va, vb = verts @ Ra.T, verts @ Rb.T + t
        axes = list(normals @ Ra.T) + list(normals @ Rb.T)
        ea, eb = edirs @ Ra.T, edirs @ Rb.T
        for u in ea:
            for w in eb:
                c = np.cross(u, w)
                nn = np.linalg.norm(c)
                if nn > 1e-9:
                    axes.append(c / nn)
        for ax in axes:
            pa, pb = va @ ax, vb @ ax
            if pa.max() + margin < pb.min() - margin or pb.max() + margin < pa.min() - margin:
                return False
        return True

    for i in range(n):
        d = _minimg(X - X[i], dims, periodic)
        dist2 = (d * d).sum(1)
        near = np.nonzero(done & (dist2 < (2 * rc) ** 2))[0]
        for draw in range(max_draws):
            qi = random_quaternions(rng, 1)
            Ri = _rotation_matrices(qi)[0]
            if not any(overlap(Ri, R[j], d[j]) for j in near):
                break
        else:
            raise RuntimeError(f"orientation draws stalled at body {i}")
        q[i], R[i], done[i] = qi[0], Ri, True
    return q


def cube_orientations(rng, X, edge, dims, periodic, margin=0.3,
                      max_draws=10_000) -> np.ndarray:
    """Random orientations such that no two cubes (grown by margin) overlap.

    Cubes are processed in index order; each draw is tested with the
    separating-axis theorem against already oriented neighbours within two
    circumradii.  Raises if a cube needs more than max_draws draws.
    """
    n = X.shape[0]
    dims = np.asarray(dims, float)
    periodic = np.asarray(periodic, bool)
    h = 0.5 * edge
    rc = h * math.sqrt(3.0) + margin
    q = np.zeros((n, 4))
    R = np.zeros((n, 3, 3))
    done = np.zeros(n, bool)
    for i in range(n):
        d = _minimg(X - X[i], dims, periodic)
        dist2 = (d * d).sum(1)
        near = np.nonzero(done & (dist2 < (2 * rc) ** 2))[0]
        for draw in range(max_draws):
            qi = random_quaternions(rng, 1)
            Ri = _rotation_matrices(qi)[0]
            if not any(_obb_overlap(np.zeros(3), Ri, h, d[j], R[j], h, margin)
                       for j in near):
                break
        else:
            raise RuntimeError(f"orientation draws stalled at cube {i}")
        q[i], R[i], done[i] = qi[0], Ri, True
    return q


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def _base_params(n, periodic_z, tau, lu, balance) -> Params:
    return Params(nx=n[0], ny=n[1], nz=n[2], periodic_z=periodic_z, tau=tau,
                  gravity=(0.0, 0.0, -lu["g"]), balance=balance,
                  young=lu["young"], u_k=lu["u_k"])


def c1_two_spheres() -> Workload:
    """32^3 periodic, two spheres D=8 approaching head-on at 0.01, tau 0.8."""
    lu2 = lattice_units(cube_equiv_diameter(12.0), 1.5, 500.0, 0.55)
    p = Params(nx=32, ny=32, nz=32, periodic_z=1, tau=0.8,
               young=lu2["young"], u_k=lu2["u_k"], max_pairs=64,
               tile_capacity=16)
    sc = Scene(shape=np.array([SPHERE, SPHERE], np.int32),
               size=np.array([4.0, 4.0]), density=np.array([2.0, 2.0]),
               X=np.array([[10.0, 16.0, 16.0], [22.0, 16.0, 16.0]]),
               q=np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
               U=np.array([[0.01, 0, 0], [-0.01, 0, 0]]),
               omega=np.zeros((2, 3)))
    return Workload("C1", p, sc, 100,
                    "32^3 periodic, 2 spheres D=8 head-on at 0.01, s=2, g=0")


def c2_settling_walls(seed: int = 2, n_override: Optional[int] = None) -> Workload:
    """128^3, walls in z, ~121 cubes a=12 (phi 0.10), s 1.5, Ar 500."""
    a, s, ar, tau, L = 12.0, 1.5, 500.0, 0.55, 128
    lu = lattice_units(cube_equiv_diameter(a), s, ar, tau)
    n = n_override or round(0.10 * L ** 3 / a ** 3)
    rng = np.random.default_rng(seed)
    h = 0.5 * a * math.sqrt(3.0)
    X = rsa_centres(rng, n, (L, L, L), a * math.sqrt(3.0) + 0.6,
                    (True, True, False), lo_margin=(0, 0, h + 1.0))
    q = cube_orientations(rng, X, a, (L, L, L), (True, True, False))
    sc = Scene(np.full(n, CUBE, np.int32), np.full(n, a), np.full(n, s), X, q,
               np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 0, tau, lu, 0).replace(max_pairs=2048,
                                                       tile_capacity=32)
    return Workload("C2", p, sc, 2000,
                    f"128^3 walls z, {n} cubes a=12, phi~0.10, s=1.5, Ar=500")


def _dense_centres(seed: int, L: int, n: int, d: float,
                   jitter: float = 0.5) -> np.ndarray:
    """n centres on a randomly thinned, jittered face-centred cubic lattice.

    Random sequential addition cannot reach a 30% fill of randomly oriented
    cubes, so the dense boxes take the sites of an m^3-cell FCC lattice
    (4 m^3 >= n sites, the largest nearest-neighbour distance for the site
    count), drop random sites down to n, and jitter each centre by +-jitter
    per axis.  Spheres of diameter d never overlap.
    """
    rng = np.random.default_rng(seed)
    m = 1
    while 4 * m ** 3 < n:
        m += 1
    a = L / m
    if a / math.sqrt(2.0) < d + 2.0 * math.sqrt(3.0) * jitter:
        raise ValueError("lattice too tight for the requested diameter")
    basis = np.array([[0.25, 0.25, 0.25], [0.75, 0.75, 0.25],
                      [0.75, 0.25, 0.75], [0.25, 0.75, 0.75]])
    g = np.arange(m)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 1, 3)
    sites = ((cells + basis[None]) * a).reshape(-1, 3)
    keep = np.sort(rng.permutation(sites.shape[0])[:n])
    X = sites[keep] + rng.uniform(-jitter, jitter, (n, 3))
    return np.mod(X, L)


def c3_dense_cubes(seed: int = 3, L: int = 256, phi: float = 0.30,
                   edge: float = 14.0) -> Workload:
    """256^3 periodic, 1834 cubes a=14 (phi 0.30), s 1.5, Ar 1000; zero net
    volume flow held by the balance controller (balance mode 2, Sec. 5.1).

    Centres are the sphere centres of the matching sphere workload (the paper
    keeps the initial positions for spheres and cubes); orientations are
    redrawn until no two cubes overlap.
    """
    s, ar, tau = 1.5, 1000.0, 0.55
    dsph = cube_equiv_diameter(edge)
    lu = lattice_units(dsph, s, ar, tau)
    n = round(phi * L ** 3 / edge ** 3)
    X = _dense_centres(seed, L, n, dsph)
    rng = np.random.default_rng(seed + 1000)
    q = cube_orientations(rng, X, edge, (L, L, L), (True, True, True))
    sc = Scene(np.full(n, CUBE, np.int32), np.full(n, edge), np.full(n, s), X,
               q, np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 1, tau, lu, 2).replace(
        max_pairs=max(1024, 8 * n), tile_capacity=48, precision=1)
    return Workload("C3", p, sc, 1000,
                    f"{L}^3 periodic, {n} cubes a={edge:g}, phi~{phi}, s=1.5, Ar=1000")


def c3_dense_boxes(seed: int = 3, L: int = 256, phi: float = 0.30,
                   edge: float = 14.0) -> Workload:
    """C3 with the cubes replaced by boxes of edge ratio 1 : 1.25 : 1.6 and
    the same volume, given as a convex polyhedron type (anisotropic
    inertia, the general polyhedron signed distance)."""
    s, ar, tau = 1.5, 1000.0, 0.55
    dsph = cube_equiv_diameter(edge)
    lu = lattice_units(dsph, s, ar, tau)
    n = round(phi * L ** 3 / edge ** 3)
    a = (edge ** 3 / 2.0) ** (1.0 / 3.0)
    dims3 = np.array([a, 1.25 * a, 1.6 * a])
    X = _dense_centres(seed, L, n, dsph)
    rng = np.random.default_rng(seed + 2000)
    q = box_orientations(rng, X, 0.5 * dims3, (L, L, L), (True, True, True))
    sc = Scene(np.full(n, POLY0, np.int32), np.ones(n), np.full(n, s), X,
               q, np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 1, tau, lu, 2).replace(
        max_pairs=max(1024, 8 * n), tile_capacity=48, precision=1)
    return Workload("C3B", p, sc, 1000,
                    f"{L}^3 periodic, {n} boxes {dims3[0]:.2f} x {dims3[1]:.2f} x "
                    f"{dims3[2]:.2f} (polyhedra), phi~{phi}, s=1.5, Ar=1000",
                    polyhedra={0: polyhedron_cuboid(*dims3)})


def c3_dense_ellipsoids(seed: int = 3, L: int = 256, phi: float = 0.12,
                        edge: float = 14.0, margin: float = 0.3) -> Workload:
    """256^3 periodic box of ellipsoids with semi-axes ratio 1 : 1.25 : 1.6
    and the volume of the cube of edge 14, as an ellipsoid type (the smooth
    convex body; exact distance by its nearest-point multiplier).

    Orientations are drawn as for the boxes with the ellipsoids' bounding
    boxes (half extents the semi-axes): bounding boxes that do not overlap
    keep the ellipsoids apart.  Those boxes hold twice the body volume, so
    the fill is phi 0.12 (734 bodies) rather than the cubes' 0.30; the
    lattice sites then sit 30 cells apart, more than two long semi-axes, so
    (as in the sphere box) no pair is in contact at the start.
    """
    s, ar, tau = 1.5, 1000.0, 0.55
    dsph = cube_equiv_diameter(edge)
    lu = lattice_units(dsph, s, ar, tau)
    n = round(phi * L ** 3 / edge ** 3)
    a = (edge ** 3 / (4.0 / 3.0 * math.pi * 2.0)) ** (1.0 / 3.0)
    axes = np.array([a, 1.25 * a, 1.6 * a])
    X = _dense_centres(seed, L, n, dsph)
    rng = np.random.default_rng(seed + 3000)
    q = box_orientations(rng, X, axes, (L, L, L), (True, True, True), margin=margin)
    sc = Scene(np.full(n, POLY0, np.int32), np.ones(n), np.full(n, s), X,
               q, np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 1, tau, lu, 2).replace(
        max_pairs=max(1024, 8 * n), tile_capacity=48, precision=1)
    return Workload("C3E", p, sc, 1000,
                    f"{L}^3 periodic, {n} ellipsoids {axes[0]:.2f} x {axes[1]:.2f} x "
                    f"{axes[2]:.2f} (semi-axes), phi~{phi}, s=1.5, Ar=1000",
                    polyhedra={0: Ellipsoid(tuple(float(x) for x in axes))})


def c4_dense_spheres(seed: int = 3, L: int = 256, phi: float = 0.30,
                     edge: float = 14.0) -> Workload:
    """256^3 periodic, 1834 spheres of the cubes' volume-equivalent diameter;
    zero net volume flow (balance mode 2, Sec. 5.1)."""
    s, ar, tau = 1.5, 2000.0, 0.55
    dsph = cube_equiv_diameter(edge)
    lu = lattice_units(dsph, s, ar, tau)
    n = round(phi * L ** 3 / edge ** 3)
    X = _dense_centres(seed, L, n, dsph)
    q = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    sc = Scene(np.full(n, SPHERE, np.int32), np.full(n, 0.5 * dsph),
               np.full(n, s), X, q, np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 1, tau, lu, 2).replace(
        max_pairs=max(1024, 8 * n), tile_capacity=48, precision=2)
    return Workload("C4", p, sc, 1000,
                    f"{L}^3 periodic, {n} spheres D={dsph:.2f}, phi~{phi}, s=1.5, Ar=2000")


def settling_box(shape, phi: float, n_per_d: float = 9.0,
                 l_over_d: float = 12.0, ar: float = 1000.0, s: float = 3.3,
                 tau: float = 0.55, seed: int = 11, precision: int = 1,
                 edge_cells: Optional[int] = None,
                 balance: int = 2) -> Workload:
    """Periodic hindered-settling box of Sec. 5.1: spheres of diameter
    D = n_per_d cells (or other bodies of the same volume), edge
    L = l_over_d * D (or edge_cells), n = phi L^3 / V_s particles at rest
    on a jittered, thinned FCC lattice (non-spherical bodies randomly
    oriented without overlap), density ratio s (3.3 in the paper), gravity
    from the Archimedes number, balance force on.  shape: SPHERE, CUBE,
    OCTAHEDRON, or "box" (edges 1 : 1.25 : 1.6) or "tetrahedron" (regular),
    the last two as polyhedron type 0.  Dense boxes need an edge whose FCC
    cell count leaves the bodies room to turn (e.g. L = 120 for D = 9 at
    phi = 0.3)."""
    d = float(n_per_d)
    L = int(edge_cells) if edge_cells else int(round(l_over_d * d))
    vs = math.pi / 6.0 * d ** 3
    n = max(1, int(round(phi * L ** 3 / vs)))
    lu = lattice_units(d, s, ar, tau)
    X = _dense_centres(seed, L, n, d)
    rng = np.random.default_rng(seed + 1000)
    per3, dims3 = (True, True, True), (L, L, L)
    polys = None
    if isinstance(shape, str):
        # volume-equivalent polyhedron type 0 at unit size
        if shape == "box":
            a = (vs / 2.0) ** (1.0 / 3.0)
            P = polyhedron_cuboid(a, 1.25 * a, 1.6 * a)
        elif shape == "tetrahedron":
            P = polyhedron_tetrahedron((6.0 * math.sqrt(2.0) * vs) ** (1.0 / 3.0))
        else:
            raise ValueError(f"unknown settling body {shape!r}")
        polys = {0: P}
        code, size, kind = POLY0, 1.0, "boxes" if shape == "box" else "tetrahedra"
        q = convex_orientations(rng, X, P.vertices, P.faces, dims3, per3)
    elif shape == SPHERE:
        code, size, kind = SPHERE, 0.5 * d, "spheres"
        q = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (n, 1))
    elif shape == CUBE:
        code, size, kind = CUBE, d * (math.pi / 6.0) ** (1.0 / 3.0), "cubes"
        q = cube_orientations(rng, X, size, dims3, per3)
    elif shape == OCTAHEDRON:
        code, size, kind = OCTAHEDRON, (0.75 * vs) ** (1.0 / 3.0), "octahedra"
        P = polyhedron_octahedron(size)
        q = convex_orientations(rng, X, P.vertices, P.faces, dims3, per3)
    else:
        raise ValueError("settling boxes hold spheres, cubes, octahedra, boxes or tetrahedra")
    sc = Scene(np.full(n, code, np.int32), np.full(n, size), np.full(n, s), X,
               q, np.zeros((n, 3)), np.zeros((n, 3)))
    p = _base_params((L, L, L), 1, tau, lu, balance).replace(
        max_pairs=max(1024, 8 * n), tile_capacity=48, precision=precision)
    return Workload("settling", p, sc, 0,
                    f"{L}^3 periodic, {n} {kind}, D={d:g} cells (volume-equivalent), "
                    f"phi~{phi}, s={s}, Ar={ar:g}", polyhedra=polys, d_equiv=d)


def c5_adjoint_cubes(seed: int = 5) -> Workload:
    """96^3 periodic, 27 cubes a=10 on a jittered 3x3x3 grid, Ar 500."""
    a, s, ar, tau, L = 10.0, 1.5, 500.0, 0.55, 96
    lu = lattice_units(cube_equiv_diameter(a), s, ar, tau)
    rng = np.random.default_rng(seed)
    g = np.arange(3) * 32.0 + 16.0
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    X = X + rng.uniform(-4.0, 4.0, X.shape)
    q = random_quaternions(rng, 27)
    sc = Scene(np.full(27, CUBE, np.int32), np.full(27, a), np.full(27, s), X,
               q, np.zeros((27, 3)), np.zeros((27, 3)))
    p = _base_params((L, L, L), 1, tau, lu, 1).replace(max_pairs=256,
                                                       tile_capacity=16)
    return Workload("C5", p, sc, 500,
                    "96^3 periodic, 27 cubes a=10 jittered 3x3x3, s=1.5, Ar=500")


def random_small_scene(seed: int, dims, n_particles: int, periodic_z=1,
                       size_range=(2.0, 4.5), gap=-0.3, speed=0.01,
                       spin=0.004, shapes=(SPHERE, CUBE),
                       poly_rc=None) -> Scene:
    """Mixed convex bodies (spheres, cubes and, if asked, octahedra or
    polyhedron types POLY0 + k with unit circumradius poly_rc[POLY0 + k]) in
    a small box; neighbours may nearly touch.

    `gap` is the allowed surface gap between bounding spheres (negative
    values let bounding spheres interpenetrate, so that corners and
    enlarged surfaces come into contact and the contact path is exercised).
    """
    rng = np.random.default_rng(seed)
    dims = np.asarray(dims, float)
    periodic = np.array([True, True, bool(periodic_z)])
    shape = np.asarray(shapes, np.int32)[rng.integers(0, len(shapes), n_particles)]
    size = np.empty(n_particles)
    rb = np.empty(n_particles)
    for i in range(n_particles):
        if shape[i] == SPHERE:
            size[i] = rng.uniform(*size_range)
            rb[i] = size[i]
        elif shape[i] == OCTAHEDRON:
            size[i] = 1.3 * rng.uniform(*size_range)
            rb[i] = size[i]
        elif shape[i] >= POLY0:
            rc = poly_rc[int(shape[i])]
            size[i] = 1.2 * rng.uniform(*size_range) / rc
            rb[i] = size[i] * rc
        else:
            size[i] = 2.0 * rng.uniform(*size_range) / math.sqrt(3.0) * 1.4
            rb[i] = 0.5 * size[i] * math.sqrt(3.0)
    X = np.zeros((n_particles, 3))
    for i in range(n_particles):
        for _ in range(100000):
            p = np.empty(3)
            for a in range(3):
                if periodic[a]:
                    p[a] = rng.random() * dims[a]
                else:
                    lo, hi = rb[i] + 0.8, dims[a] - 1.0 - rb[i] - 0.8
                    p[a] = lo + rng.random() * max(hi - lo, 0.0)
            ok = True
            for j in range(i):
                d = _minimg(X[j] - p, dims, periodic)
                if math.sqrt(d @ d) < rb[i] + rb[j] + gap:
                    ok = False
                    break
            if ok:
                X[i] = p
                break
        else:
            raise RuntimeError("small scene placement stalled")
    q = random_quaternions(rng, n_particles)
    U = rng.uniform(-speed, speed, (n_particles, 3))
    om = rng.uniform(-spin, spin, (n_particles, 3))
    dens = rng.uniform(1.2, 3.0, n_particles)
    return Scene(shape, size, dens, X, q, U, om)


def perturbed_populations(seed: int, dims, profile, amp: float = 0.01) -> np.ndarray:
    """Smooth random population field f[19][z][y][x] = profile_i (1 + amp noise).

    `profile` (19 values) is supplied by the caller (for example a rest
    equilibrium); the noise is periodic-smoothed standard normal noise.  Used
    only as an arbitrary starting state that both implementations import.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    profile = np.asarray(profile, float).reshape(19, 1, 1, 1)
    noise = rng.standard_normal((19, nz, ny, nx))
    for ax in (1, 2, 3):
        noise = (noise + np.roll(noise, 1, ax) + np.roll(noise, -1, ax)) / 3.0
    return np.ascontiguousarray(profile * (1.0 + amp * noise))


WORKLOADS = {
    "C1": c1_two_spheres,
    "C2": c2_settling_walls,
    "C3": c3_dense_cubes,
    "C3B": c3_dense_boxes,
    "C3E": c3_dense_ellipsoids,
    "C4": c4_dense_spheres,
    "C5": c5_adjoint_cubes,
}
