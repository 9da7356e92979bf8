"""ctypes binding of the FP64 CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product package.

Build the library with `python oracle/build.py` (or __graft_entry__.build()).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

Q = 19
MAXK = 8


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("periodic_z", C.c_int), ("tau", C.c_double),
                ("wall_u", (C.c_double * 3) * 2),
                ("gravity", C.c_double * 3), ("fluid_accel", C.c_double * 3),
                ("balance", C.c_int), ("eps", C.c_double),
                ("delta_c", C.c_double), ("n_c", C.c_int),
                ("young", C.c_double), ("poisson", C.c_double),
                ("restitution", C.c_double), ("mu_s", C.c_double),
                ("mu_k", C.c_double), ("u_k", C.c_double),
                ("n_sub", C.c_int)]


class OrcParticle(C.Structure):
    _fields_ = [("shape", C.c_int), ("size", C.c_double), ("dens", C.c_double),
                ("X", C.c_double * 3), ("q", C.c_double * 4),
                ("U", C.c_double * 3), ("w", C.c_double * 3)]


class OrcContact(C.Structure):
    _fields_ = [("a", C.c_int), ("b", C.c_int), ("count", C.c_int),
                ("rlo", C.c_int * 3), ("rhi", C.c_int * 3),
                ("carried", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("established", C.c_int), ("damping", C.c_double),
                ("age", C.c_int), ("n_in", C.c_int),
                ("volume", C.c_double), ("centroid", C.c_double * 3),
                ("normal", C.c_double * 3), ("depth", C.c_double),
                ("fn", C.c_double), ("force_a", C.c_double * 3),
                ("force_b", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("oracle library not built: run python oracle/build.py")
        L = C.CDLL(LIBPATH)
        P = C.POINTER
        d, i = C.c_double, C.c_int
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [P(OrcParams), i, P(i), P(d), P(d), P(d), P(d),
                                 P(d), P(d)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init_equilibrium.argtypes = [C.c_void_p, d, P(d)]
        L.orc_set_populations.argtypes = [C.c_void_p, P(d)]
        L.orc_step.argtypes = [C.c_void_p, i]
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_step_count.restype = C.c_long
        L.orc_error.argtypes = [C.c_void_p]
        L.orc_error.restype = C.c_char_p
        L.orc_get_populations.argtypes = [C.c_void_p, P(d)]
        L.orc_get_post_stream.argtypes = [C.c_void_p, P(d)]
        L.orc_get_fields.argtypes = [C.c_void_p, P(d), P(d), P(i), P(d), P(d)]
        L.orc_get_collision_diag.argtypes = [C.c_void_p, P(d), P(d), P(d)]
        L.orc_get_mea_cells.argtypes = [C.c_void_p, P(d)]
        L.orc_get_particles.argtypes = [C.c_void_p, P(d), P(d), P(d), P(d)]
        L.orc_get_forces.argtypes = [C.c_void_p, P(d), P(d), P(d), P(d)]
        L.orc_num_contacts.argtypes = [C.c_void_p]
        L.orc_get_contacts.argtypes = [C.c_void_p, P(OrcContact)]
        L.orc_get_counters.argtypes = [C.c_void_p, P(C.c_longlong),
                                       P(C.c_longlong)]
        L.orc_get_balance.argtypes = [C.c_void_p, P(d)]
        L.orc_feq.argtypes = [d, P(d), P(d)]
        L.orc_lattice.argtypes = [P(i), P(d), P(i)]
        L.orc_rotation.argtypes = [P(d), P(d)]
        L.orc_sdf.argtypes = [i, d, P(d), P(d), P(d)]
        L.orc_sdf.restype = d
        L.orc_weight.argtypes = [d, d]
        L.orc_weight.restype = d
        L.orc_friction_mu.argtypes = [d, d, d]
        L.orc_friction_mu.restype = d
        L.orc_damping.argtypes = [d, d]
        L.orc_damping.restype = d
        L.orc_effective_modulus.argtypes = [d, d, d, d]
        L.orc_effective_modulus.restype = d
        L.orc_treat_pair.argtypes = [P(OrcParams), P(OrcParticle),
                                     P(OrcParticle), i, i, P(d), P(d),
                                     P(OrcContact)]
        L.orc_contact_force_of.argtypes = [P(OrcParams), P(OrcParticle),
                                           P(OrcParticle), P(OrcContact)]
        L.orc_threads.restype = i
        L.orc_define_polyhedron.argtypes = [i, i, P(d), i, P(i), P(i)]
        L.orc_define_polyhedron.restype = i
        L.orc_poly_error.restype = C.c_char_p
        L.orc_define_ellipsoid.argtypes = [i, d, d, d]
        L.orc_define_ellipsoid.restype = i
        L.orc_half_extent.argtypes = [i, d, P(d), i]
        L.orc_half_extent.restype = d
        L.orc_poly_info.argtypes = [i, P(d), P(d), P(d), P(d)]
        L.orc_poly_info.restype = i
        L.orc_poly_angular_accel.argtypes = [i, d, d, P(d), P(d), P(d)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def make_params(p) -> OrcParams:
    """OrcParams from a workloads.Params record."""
    o = OrcParams()
    o.nx, o.ny, o.nz = p.nx, p.ny, p.nz
    o.periodic_z = p.periodic_z
    o.tau = p.tau
    for w in range(2):
        for k in range(3):
            o.wall_u[w][k] = p.wall_velocity[w][k]
    for k in range(3):
        o.gravity[k] = p.gravity[k]
        o.fluid_accel[k] = p.fluid_accel[k]
    o.balance = p.balance
    o.eps = p.eps_b
    o.delta_c = p.enlarge
    o.n_c = p.n_c
    o.young, o.poisson, o.restitution = p.young, p.poisson, p.restitution
    o.mu_s, o.mu_k, o.u_k = p.mu_s, p.mu_k, p.u_k
    o.n_sub = p.n_sub
    return o


def make_particle(shape, size, dens, X, q, U=(0, 0, 0), w=(0, 0, 0)) -> OrcParticle:
    o = OrcParticle()
    o.shape, o.size, o.dens = int(shape), float(size), float(dens)
    for k in range(3):
        o.X[k], o.U[k], o.w[k] = X[k], U[k], w[k]
    for k in range(4):
        o.q[k] = q[k]
    return o


def contacts_to_dicts(arr) -> list:
    out = []
    for c in arr:
        out.append(dict(a=c.a, b=c.b, count=c.count, rlo=tuple(c.rlo),
                        rhi=tuple(c.rhi), carried=c.carried, lo=tuple(c.lo),
                        hi=tuple(c.hi), established=c.established,
                        damping=c.damping, age=c.age, n_in=c.n_in,
                        volume=c.volume, centroid=tuple(c.centroid),
                        normal=tuple(c.normal), depth=c.depth, fn=c.fn,
                        force_a=tuple(c.force_a), force_b=tuple(c.force_b)))
    return out


class OracleSim:
    """Whole-simulation oracle.  Arrays are numpy float64 / int32."""

    def __init__(self, params, scene):
        self.params = params
        self.P = make_params(params)
        self.ncell = params.nx * params.ny * params.nz
        self.np = scene.n
        sh = np.ascontiguousarray(scene.shape, np.int32)
        args = [np.ascontiguousarray(a, np.float64) for a in
                (scene.size, scene.density, scene.X, scene.q, scene.U,
                 scene.omega)]
        self._keep = (sh, args)
        h = lib().orc_create(C.byref(self.P), self.np, _ip(sh),
                             *[_dp(a) for a in args])
        if not h:
            raise MemoryError("orc_create failed")
        self.h = C.c_void_p(h)

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(lib().orc_error(self.h).decode())

    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        uu = np.asarray(u, np.float64)
        self._check(lib().orc_init_equilibrium(self.h, rho, _dp(uu)))

    def set_populations(self, fs):
        fs = np.ascontiguousarray(fs, np.float64)
        assert fs.size == Q * self.ncell
        self._check(lib().orc_set_populations(self.h, _dp(fs)))

    def step(self, n=1):
        self._check(lib().orc_step(self.h, n))

    @property
    def step_count(self):
        return lib().orc_step_count(self.h)

    def shape3(self):
        p = self.params
        return (p.nz, p.ny, p.nx)

    def populations(self):
        out = np.empty((Q,) + self.shape3())
        lib().orc_get_populations(self.h, _dp(out))
        return out

    def post_stream(self):
        out = np.empty((Q,) + self.shape3())
        lib().orc_get_post_stream(self.h, _dp(out))
        return out

    def fields(self):
        s = self.shape3()
        rho = np.empty(s)
        u = np.empty(s + (3,))
        owner = np.empty(s, np.int32)
        B = np.empty(s)
        up = np.empty(s + (3,))
        lib().orc_get_fields(self.h, _dp(rho), _dp(u), _ip(owner), _dp(B),
                             _dp(up))
        return dict(rho=rho, u=u, owner=owner, B=B, up=up)

    def collision_diag(self):
        s = self.shape3()
        rho, J, du = np.empty(s), np.empty(s + (3,)), np.empty(s + (3,))
        lib().orc_get_collision_diag(self.h, _dp(rho), _dp(J), _dp(du))
        return rho, J, du

    def mea_cells(self):
        out = np.empty(self.shape3() + (3,))
        lib().orc_get_mea_cells(self.h, _dp(out))
        return out

    def particles(self):
        n = max(self.np, 1)
        X, q, U, w = (np.empty((n, 3)), np.empty((n, 4)), np.empty((n, 3)),
                      np.empty((n, 3)))
        lib().orc_get_particles(self.h, _dp(X), _dp(q), _dp(U), _dp(w))
        k = self.np
        return dict(X=X[:k], q=q[:k], U=U[:k], omega=w[:k])

    def forces(self):
        n = max(self.np, 1)
        a = [np.zeros((n, 3)) for _ in range(4)]
        lib().orc_get_forces(self.h, *[_dp(x) for x in a])
        k = self.np
        return dict(Fh=a[0][:k], Th=a[1][:k], Fc=a[2][:k], Tc=a[3][:k])

    def contacts(self):
        n = lib().orc_num_contacts(self.h)
        arr = (OrcContact * max(n, 1))()
        lib().orc_get_contacts(self.h, arr)
        return contacts_to_dicts(arr[:n])

    def counters(self):
        a, b = C.c_longlong(), C.c_longlong()
        lib().orc_get_counters(self.h, C.byref(a), C.byref(b))
        return a.value, b.value

    def balance(self):
        out = np.empty(3)
        lib().orc_get_balance(self.h, _dp(out))
        return out


# ---- pieces ------------------------------------------------------------
def feq(rho, u):
    out = np.empty(Q)
    uu = np.asarray(u, np.float64)
    lib().orc_feq(rho, _dp(uu), _dp(out))
    return out


def lattice():
    c = np.empty((Q, 3), np.int32)
    w = np.empty(Q)
    opp = np.empty(Q, np.int32)
    lib().orc_lattice(_ip(c), _dp(w), _ip(opp))
    return c, w, opp


def rotation(q):
    qq = np.ascontiguousarray(q, np.float64)
    R = np.empty(9)
    lib().orc_rotation(_dp(qq), _dp(R))
    return R.reshape(3, 3)


def sdf(shape, size, q, r, want_grad=False):
    R = np.ascontiguousarray(rotation(q).reshape(9))
    rr = np.ascontiguousarray(r, np.float64)
    g = np.empty(3)
    d = lib().orc_sdf(int(shape), float(size), _dp(R), _dp(rr), _dp(g))
    return (d, g) if want_grad else d


POLY0 = 3


def define_polyhedron(ptype, vertices, faces):
    """Register convex polyhedron type ptype (shape code POLY0 + ptype):
    vertices (n, 3), faces as vertex-index lists, counter-clockwise seen
    from outside."""
    v = np.ascontiguousarray(vertices, np.float64).reshape(-1)
    fs = np.array([len(f) for f in faces], np.int32)
    fi = np.array([k for f in faces for k in f], np.int32)
    rc = lib().orc_define_polyhedron(int(ptype), v.size // 3, _dp(v), len(faces),
                                     _ip(fs), _ip(fi))
    if rc != 0:
        raise ValueError(lib().orc_poly_error().decode())


def define_ellipsoid(ptype, axes):
    """Register ellipsoid type ptype (shape code POLY0 + ptype): semi-axes
    (a, b, c) along the body axes at unit scale."""
    a, b, c = (float(x) for x in axes)
    if lib().orc_define_ellipsoid(int(ptype), a, b, c) != 0:
        raise ValueError(lib().orc_poly_error().decode())


def define_body_type(ptype, body):
    """Register a polyhedron (vertices, faces) or an ellipsoid (axes)."""
    if hasattr(body, "axes"):
        define_ellipsoid(ptype, body.axes)
    else:
        define_polyhedron(ptype, body.vertices, body.faces)


def half_extent(shape, size, q, k):
    """Half extent along world axis k of a particle (rotation q)."""
    qq = np.ascontiguousarray(q, np.float64)
    return lib().orc_half_extent(int(shape), float(size), _dp(qq), int(k))


def polyhedron_info(ptype, nv):
    """(unit volume, second moment J (3x3) about the centroid,
    circumradius, re-centred vertices) of a defined type."""
    vol, rc = np.zeros(1), np.zeros(1)
    J, v = np.zeros(9), np.zeros(3 * nv)
    if lib().orc_poly_info(int(ptype), _dp(vol), _dp(J), _dp(rc), _dp(v)) != 0:
        raise ValueError("polyhedron type not defined")
    return vol[0], J.reshape(3, 3), rc[0], v.reshape(nv, 3)


def poly_angular_accel(shape, size, dens, q, T):
    qq = np.ascontiguousarray(q, np.float64)
    tt = np.ascontiguousarray(T, np.float64)
    out = np.empty(3)
    lib().orc_poly_angular_accel(int(shape), float(size), float(dens), _dp(qq),
                                 _dp(tt), _dp(out))
    return out


def weight(d, eps=1.0):
    return lib().orc_weight(float(d), float(eps))


def friction_mu(a, mu_s, mu_k):
    return lib().orc_friction_mu(float(a), float(mu_s), float(mu_k))


def damping(e, u0):
    return lib().orc_damping(float(e), float(u0))


def effective_modulus(Ea, nua, Eb, nub):
    return lib().orc_effective_modulus(Ea, nua, Eb, nub)


def treat_pair(params, pa, pb, b_id, lo, hi, npass=1):
    """Static treatment of one pair from the box [lo, hi] (copied)."""
    P = make_params(params)
    lo = np.ascontiguousarray(lo, np.float64).copy()
    hi = np.ascontiguousarray(hi, np.float64).copy()
    out = OrcContact()
    lib().orc_treat_pair(C.byref(P), C.byref(pa),
                         C.byref(pb) if pb is not None else None, int(b_id),
                         int(npass), _dp(lo), _dp(hi), C.byref(out))
    return contacts_to_dicts([out])[0]


def contact_force_of(params, pa, pb, volume, depth, centroid, normal,
                     established=0, damping=0.0):
    """eqs. (4)-(9) for a contact of the given volume, depth, centroid and
    normal (pb None: wall partner); returns the record with fn, forces and
    the damping factor."""
    P = make_params(params)
    c = OrcContact()
    c.volume, c.depth = float(volume), float(depth)
    for k in range(3):
        c.centroid[k] = float(centroid[k])
        c.normal[k] = float(normal[k])
    c.established, c.damping = int(established), float(damping)
    lib().orc_contact_force_of(C.byref(P), C.byref(pa),
                               C.byref(pb) if pb is not None else None,
                               C.byref(c))
    return contacts_to_dicts([c])[0]


def threads():
    return lib().orc_threads()
