"""Python binding of libhlbm.so (C ABI in include/hlbm.h).

Argument marshalling only: every step of the time step runs in the library's
HIP kernels.  PyTorch supplies the device memory of the two population
buffers and the HIP stream the library runs on.  The library must be built
(`python -m paper_2401_10878_amd.build`); importing this module without it
raises immediately, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhlbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hlbm.h")

Q = 19
STATUS = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_CAPACITY",
          -5: "E_UNSTABLE", -6: "E_STATE"}
BYTES = {0: 8, 1: 4, 2: 2}


class HlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hlbm {STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("periodic_z", C.c_int), ("tau", C.c_double),
                ("wall_velocity", (C.c_double * 3) * 2),
                ("gravity", C.c_double * 3), ("fluid_accel", C.c_double * 3),
                ("balance", C.c_int), ("eps_b", C.c_double),
                ("enlarge", C.c_double), ("n_c", C.c_int),
                ("young", C.c_double), ("poisson", C.c_double),
                ("restitution", C.c_double), ("mu_s", C.c_double),
                ("mu_k", C.c_double), ("u_k", C.c_double),
                ("max_pairs", C.c_int), ("tile_capacity", C.c_int),
                ("precision", C.c_int), ("n_sub", C.c_int)]


class Contact(C.Structure):
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


def header_functions() -> list:
    """Names of the functions include/hlbm.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", txt)))


_lib = None


def load():
    """Load libhlbm.so (no GPU call is made here)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(
            f"{LIBPATH} is missing: build it with python -m paper_2401_10878_amd.build")
    L = C.CDLL(LIBPATH)
    from . import build as _build
    L.hlbm_build_hash.restype = C.c_char_p
    built, here = L.hlbm_build_hash().decode(), _build.source_hash()
    if built != here:
        raise RuntimeError(
            f"{LIBPATH} was built from other sources (hash {built}, sources {here}): "
            "rebuild it with python -m paper_2401_10878_amd.build")
    P, d, i, v = C.POINTER, C.c_double, C.c_int, C.c_void_p
    L.hlbm_create.argtypes = [P(Params), v, P(v)]
    L.hlbm_bind_populations.argtypes = [v, v, v, C.c_size_t]
    L.hlbm_init_particles.argtypes = [v, i, P(i), P(d), P(d), P(d), P(d), P(d), P(d)]
    L.hlbm_define_polyhedron.argtypes = [v, i, i, P(d), i, P(i), P(i)]
    L.hlbm_define_ellipsoid.argtypes = [v, i, d, d, d]
    L.hlbm_init_fluid_equilibrium.argtypes = [v, d, P(d)]
    L.hlbm_set_populations.argtypes = [v, P(d)]
    L.hlbm_step.argtypes = [v, i]
    L.hlbm_use_graph.argtypes = [v, i]
    L.hlbm_sync.argtypes = [v]
    L.hlbm_timing_begin.argtypes = [v, i]
    L.hlbm_timing_end.argtypes = [v, P(d), P(i)]
    L.hlbm_read_forces.argtypes = [v, P(d), P(d), P(d), P(d)]
    L.hlbm_read_particles.argtypes = [v, P(d), P(d), P(d), P(d)]
    L.hlbm_read_contacts.argtypes = [v, i, P(Contact), P(i)]
    L.hlbm_read_fields.argtypes = [v, P(d), P(d), P(i)]
    L.hlbm_read_populations.argtypes = [v, P(d)]
    L.hlbm_read_coupling.argtypes = [v, P(d), P(d)]
    L.hlbm_read_coupling_noalloc.argtypes = [v, P(d), P(d)]
    L.hlbm_counters.argtypes = [v] + [P(C.c_longlong)] * 5
    L.hlbm_stream.argtypes = [v]
    L.hlbm_stream.restype = v
    L.hlbm_fluid_acceleration.argtypes = [v, P(d)]
    L.hlbm_get_state.argtypes = [v, v, P(C.c_size_t)]
    L.hlbm_set_state.argtypes = [v, v, C.c_size_t]
    L.hlbm_adjoint_record.argtypes = [v, i, i]
    L.hlbm_adjoint_gradient.argtypes = [v] + [P(d)] * 7
    L.hlbm_adjoint.argtypes = [v, i, i, P(d), P(d), P(d)]
    L.hlbm_last_error.argtypes = [v]
    L.hlbm_last_error.restype = C.c_char_p
    L.hlbm_destroy.argtypes = [v]
    for name in header_functions():
        f = getattr(L, name)
        if name not in ("hlbm_stream", "hlbm_last_error", "hlbm_destroy",
                        "hlbm_build_hash"):
            f.restype = C.c_int
    L.hlbm_destroy.restype = None
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def make_params(p) -> Params:
    o = Params()
    for f in ("nx", "ny", "nz", "periodic_z", "tau", "balance", "eps_b",
              "enlarge", "n_c", "young", "poisson", "restitution", "mu_s",
              "mu_k", "u_k", "max_pairs", "tile_capacity", "precision", "n_sub"):
        setattr(o, f, getattr(p, f))
    for w in range(2):
        for k in range(3):
            o.wall_velocity[w][k] = p.wall_velocity[w][k]
    for k in range(3):
        o.gravity[k] = p.gravity[k]
        o.fluid_accel[k] = p.fluid_accel[k]
    return o


class Simulation:
    """One coupled HLBM + contact simulation on one GPU.

    params: workloads.Params; scene: workloads.Scene; polyhedra: optional
    {type k: workloads.Polyhedron or workloads.Ellipsoid} for particles of
    shape POLY0 + k.  The two
    population buffers are torch device tensors lent to the library; the
    library runs on a dedicated torch stream (default priority).
    """

    def __init__(self, params, scene, device="cuda:0", graph=False,
                 polyhedra=None):
        import torch
        self.torch = torch
        self.L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("hlbm needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.params = params
        self.ncell = params.nx * params.ny * params.nz
        self.np = scene.n
        self.stream = torch.cuda.Stream(self.device)
        self.P = make_params(params)
        h = C.c_void_p()
        self._check(self.L.hlbm_create(C.byref(self.P),
                                       C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)), None)
        self.h = h
        nbytes = Q * self.ncell * BYTES[params.precision]
        self.fa = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.fb = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self._check(self.L.hlbm_bind_populations(
            self.h, C.c_void_p(self.fa.data_ptr()), C.c_void_p(self.fb.data_ptr()),
            nbytes))
        for k, poly in (polyhedra or {}).items():
            if hasattr(poly, "axes"):
                a, b, c = (float(x) for x in poly.axes)
                self._check(self.L.hlbm_define_ellipsoid(self.h, int(k), a, b, c))
                continue
            v = np.ascontiguousarray(poly.vertices, np.float64).reshape(-1)
            fs = np.array([len(f) for f in poly.faces], np.int32)
            fi = np.array([j for f in poly.faces for j in f], np.int32)
            self._check(self.L.hlbm_define_polyhedron(
                self.h, int(k), v.size // 3, _dp(v), len(poly.faces), _ip(fs), _ip(fi)))
        sh = np.ascontiguousarray(scene.shape, np.int32)
        arrs = [np.ascontiguousarray(a, np.float64) for a in
                (scene.size, scene.density, scene.X, scene.q, scene.U, scene.omega)]
        self._check(self.L.hlbm_init_particles(self.h, self.np, _ip(sh),
                                               *[_dp(a) for a in arrs]))
        if graph:
            self._check(self.L.hlbm_use_graph(self.h, 1))

    # ---- lifecycle ------------------------------------------------------
    def _check(self, rc, h=...):
        if rc != 0:
            hh = self.h if h is ... else h
            msg = self.L.hlbm_last_error(hh).decode() if hh else ""
            raise HlbmError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.hlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- initial conditions and stepping --------------------------------
    def init_equilibrium(self, rho=1.0, u=(0.0, 0.0, 0.0)):
        uu = np.asarray(u, np.float64)
        self._check(self.L.hlbm_init_fluid_equilibrium(self.h, rho, _dp(uu)))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64)
        assert f.size == Q * self.ncell
        self._check(self.L.hlbm_set_populations(self.h, _dp(f)))

    def step(self, n=1):
        """n coupled time steps, queued on the library stream.  Within one
        call the contact treatment of steps 2..n runs on the context's second
        stream beside the previous step's lattice passes; the call ends with
        nothing pending and the same bits as n single-step calls."""
        self._check(self.L.hlbm_step(self.h, n))

    def use_graph(self, on=True):
        """Replay steps as captured HIP graphs (8-step graphs while at least
        8 steps of a call remain, single-step graphs for the rest)."""
        self._check(self.L.hlbm_use_graph(self.h, 1 if on else 0))

    KERNELS = ("clear", "treat", "particles", "keep", "detect", "lattice",
               "mea")

    def timing_begin(self, max_steps):
        self._check(self.L.hlbm_timing_begin(self.h, max_steps))

    def timing_end(self):
        ms = np.zeros(len(self.KERNELS))
        n = C.c_int()
        self._check(self.L.hlbm_timing_end(self.h, _dp(ms), C.byref(n)))
        return dict(zip(self.KERNELS, ms.tolist())), n.value

    def sync(self):
        self._check(self.L.hlbm_sync(self.h))

    # ---- read-out ---------------------------------------------------------
    def shape3(self):
        p = self.params
        return (p.nz, p.ny, p.nx)

    def forces(self):
        n = max(self.np, 1)
        a = [np.zeros((n, 3)) for _ in range(4)]
        self._check(self.L.hlbm_read_forces(self.h, *[_dp(x) for x in a]))
        k = self.np
        return dict(Fh=a[0][:k], Th=a[1][:k], Fc=a[2][:k], Tc=a[3][:k])

    def particles(self):
        n = max(self.np, 1)
        X, q, U, w = (np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3)),
                      np.zeros((n, 3)))
        self._check(self.L.hlbm_read_particles(self.h, _dp(X), _dp(q), _dp(U), _dp(w)))
        k = self.np
        return dict(X=X[:k], q=q[:k], U=U[:k], omega=w[:k])

    def contacts(self):
        n = C.c_int()
        self._check(self.L.hlbm_read_contacts(self.h, 0, None, C.byref(n)))
        arr = (Contact * max(n.value, 1))()
        self._check(self.L.hlbm_read_contacts(self.h, n.value, arr, C.byref(n)))
        out = []
        for c in arr[:n.value]:
            out.append(dict(a=c.a, b=c.b, count=c.count, rlo=tuple(c.rlo),
                            rhi=tuple(c.rhi), carried=c.carried, lo=tuple(c.lo),
                            hi=tuple(c.hi), established=c.established,
                            damping=c.damping, age=c.age, n_in=c.n_in,
                            volume=c.volume, centroid=tuple(c.centroid),
                            normal=tuple(c.normal), depth=c.depth, fn=c.fn,
                            force_a=tuple(c.force_a), force_b=tuple(c.force_b)))
        return out

    def fields(self, rho=True, u=True, owner=True):
        s = self.shape3()
        r = np.zeros(s) if rho else None
        uu = np.zeros(s + (3,)) if u else None
        o = np.zeros(s, np.int32) if owner else None
        self._check(self.L.hlbm_read_fields(
            self.h, _dp(r) if rho else None, _dp(uu) if u else None,
            _ip(o) if owner else None))
        return dict(rho=r, u=uu, owner=o)

    def coupling(self):
        """B(d_owner) and u_p per node (FP64), as in the collision."""
        s = self.shape3()
        B, up = np.zeros(s), np.zeros(s + (3,))
        self._check(self.L.hlbm_read_coupling(self.h, _dp(B), _dp(up)))
        return dict(B=B, up=up)

    def coupling_noalloc(self):
        """The same read-out through the library's fixed device array
        (lattices of at most 2^21 nodes)."""
        s = self.shape3()
        B, up = np.zeros(s), np.zeros(s + (3,))
        self._check(self.L.hlbm_read_coupling_noalloc(self.h, _dp(B), _dp(up)))
        return dict(B=B, up=up)

    def populations(self):
        f = np.zeros((Q,) + self.shape3())
        self._check(self.L.hlbm_read_populations(self.h, _dp(f)))
        return f

    def counters(self):
        v = [C.c_longlong() for _ in range(5)]
        self._check(self.L.hlbm_counters(self.h, *[C.byref(x) for x in v]))
        return dict(pairs=v[0].value, cells=v[1].value, total_cells=v[2].value,
                    steps=v[3].value, samples=v[4].value)

    def fluid_acceleration(self):
        a = np.zeros(3)
        self._check(self.L.hlbm_fluid_acceleration(self.h, _dp(a)))
        return a

    # ---- checkpoint / resume ------------------------------------------------
    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self.L.hlbm_get_state(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        self._check(self.L.hlbm_get_state(self.h, buf, C.byref(n)))
        return bytes(buf)

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.L.hlbm_set_state(self.h, buf, len(blob)))

    # ---- adjoint ------------------------------------------------------------
    def adjoint_record(self, ksteps, ckpt_every):
        """Run ksteps steps keeping checkpoints every ckpt_every steps."""
        self._check(self.L.hlbm_adjoint_record(self.h, ksteps, ckpt_every))

    def adjoint_gradient(self, dJ_dU):
        """Gradients of J = sum_p dJ_dU[p] . U_p(end of window)."""
        n = max(self.np, 1)
        seed = np.zeros((n, 3))
        seed[:self.np] = np.asarray(dJ_dU, np.float64).reshape(self.np, 3)
        out = dict(s=np.zeros(n), theta0=np.zeros((n, 3)), q0=np.zeros((n, 4)),
                   X0=np.zeros((n, 3)), U0=np.zeros((n, 3)), omega0=np.zeros((n, 3)))
        self._check(self.L.hlbm_adjoint_gradient(
            self.h, _dp(seed), _dp(out["s"]), _dp(out["theta0"]), _dp(out["q0"]),
            _dp(out["X0"]), _dp(out["U0"]), _dp(out["omega0"])))
        return {k: v[:self.np] for k, v in out.items()}

    def adjoint(self, ksteps, ckpt_every, dJ_dU):
        """Record ksteps steps and return (dJ/ds, dJ/dq0) of
        J = sum_p dJ_dU[p] . U_p at the end of the window, in one call."""
        n = max(self.np, 1)
        seed = np.zeros((n, 3))
        seed[:self.np] = np.asarray(dJ_dU, np.float64).reshape(self.np, 3)
        ds, dq = np.zeros(n), np.zeros((n, 4))
        self._check(self.L.hlbm_adjoint(self.h, int(ksteps), int(ckpt_every),
                                        _dp(seed), _dp(ds), _dp(dq)))
        return ds[:self.np], dq[:self.np]


def _settling_function():
    import torch
    from torch.autograd.function import once_differentiable

    class MeanSettlingVelocity(torch.autograd.Function):
        """J = mean over particles of the vertical velocity U_z after ksteps
        coupled steps from fluid at rest, as a function of the particles'
        density ratios (n) and initial quaternions (n x 4).  The backward pass
        is the library's adjoint (owners and contact forces of the forward run
        held fixed).  The library runs on the unit quaternions q / |q|; the
        gradient by q is that of J(q / |q|), i.e. the library's gradient
        tangent to the unit sphere divided by |q|.  J and the gradients come
        back on the device and in the dtype of the inputs; the backward pass
        can run once (it releases the recorded window)."""

        @staticmethod
        def forward(ctx, density, q0, params, scene, ksteps, ckpt_every):
            sc = scene.copy()
            sc.density = density.detach().cpu().double().numpy().copy()
            qraw = q0.detach().cpu().double().numpy().copy()
            sc.q = qraw
            sim = Simulation(params.replace(precision=0), sc)
            sim.init_equilibrium()
            sim.adjoint_record(int(ksteps), int(ckpt_every))
            U = sim.particles()["U"]
            ctx.sim = sim
            ctx.n = sc.n
            ctx.qnorm = np.sqrt((qraw * qraw).sum(axis=1))
            ctx.like = ((density.device, density.dtype), (q0.device, q0.dtype))
            return torch.tensor(U[:, 2].mean(), dtype=density.dtype,
                                device=density.device)

        @staticmethod
        @once_differentiable
        def backward(ctx, grad):
            if ctx.sim is None:
                raise RuntimeError("MeanSettlingVelocity: the recorded window was "
                                   "released by an earlier backward pass")
            g = float(grad)
            seed = np.zeros((ctx.n, 3))
            seed[:, 2] = g / ctx.n
            try:
                r = ctx.sim.adjoint_gradient(seed)
            finally:
                ctx.sim.close()
                ctx.sim = None
            (dd, dt), (qd, qt) = ctx.like
            gq = r["q0"] / ctx.qnorm[:, None]
            return (torch.from_numpy(r["s"]).to(device=dd, dtype=dt),
                    torch.from_numpy(gq).to(device=qd, dtype=qt),
                    None, None, None, None)

    return MeanSettlingVelocity


_MSV = None


def mean_settling_velocity(density, q0, params, scene, ksteps, ckpt_every=50):
    """Differentiable J(density, q0); see MeanSettlingVelocity."""
    global _MSV
    if _MSV is None:
        _MSV = _settling_function()
    return _MSV.apply(density, q0, params, scene, ksteps, ckpt_every)
