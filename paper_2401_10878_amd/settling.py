"""Hindered-settling statistics on top of the coupled time step (Sec. 5).

The bulk settling velocity of a periodic suspension, normalised by the
single-particle settling velocity, and the correlations the paper compares
it with.  Everything here is host-side post-processing of particle
velocities read back from the library; every time step runs in the HIP
kernels.

Definitions (lattice units, fluid density 1, eta = nu):
  single-particle velocity u* (Sec. 5, eq. (20)) with the Schiller-Naumann
      drag coefficient C_d = 24/Re (1 + 0.15 Re^0.687), Re = u* D / nu,
      solved for u* (u*^2 C_d(Re) grows monotonically with u*);
  power law  u_p / u* = k (1 - phi)^n (eq. (19)) with
      n from Richardson and Zaki (eq. (22)) or Garside and Al-Dibouni
      (eq. (23)), and k = 1 or k = 0.89 exp(-Ar / 1e5) (Yao et al., eq. (24));
  normalised time  t* = t D g (s - 1) / (18 nu)  (Sec. 5.1);
  the bulk velocity is the mean over particles of the velocity component
      along gravity, averaged in time from t*_avg on (the paper: 50 of 400);
  also reported against the Stokes velocity g D^2 (s - 1) / (18 nu), the
      single-particle velocity with C_d = 24/Re.

    python -m paper_2401_10878_amd.settling --shape sphere cube --phi 0.1 0.3
    (also octahedron, box (edges 1 : 1.25 : 1.6) and tetrahedron, all of the
    sphere's volume)
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W


def schiller_naumann_cd(re: float) -> float:
    """Drag coefficient of a sphere, C_d = 24/Re (1 + 0.15 Re^0.687)."""
    return 24.0 / re * (1.0 + 0.15 * re ** 0.687)


def single_particle_velocity(g: float, d: float, s: float, nu: float) -> float:
    """u* = sqrt(4 g D (s-1) / (3 C_d(u* D / nu))) by bisection.

    The residual u^2 C_d(u D/nu) - 4 g D (s-1)/3 = 24 nu u/D (1 + 0.15
    Re^0.687) - 4 g D (s-1)/3 increases with u; it is negative at 0 and
    non-negative at the Stokes velocity g D^2 (s-1) / (18 nu), where
    C_d >= 24/Re makes u^2 C_d at least the right-hand side."""
    rhs = 4.0 * g * d * (s - 1.0) / 3.0
    lo, hi = 0.0, g * d * d * (s - 1.0) / (18.0 * nu)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if mid * mid * schiller_naumann_cd(mid * d / nu) < rhs:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def n_richardson_zaki(re: float) -> float:
    """Expansion index of Richardson and Zaki (eq. (22))."""
    if re < 0.2:
        return 4.65
    if re < 1.0:
        return 4.35 * re ** -0.03
    if re < 500.0:
        return 4.45 * re ** -0.1
    return 2.39


def n_garside_al_dibouni(re: float) -> float:
    """Expansion index of Garside and Al-Dibouni (eq. (23))."""
    r = re ** 0.9
    return (5.1 + 0.27 * r) / (1.0 + 0.1 * r)


def k_yao(ar: float) -> float:
    """Prefactor of Yao et al. (eq. (24))."""
    return 0.89 * math.exp(-ar / 1.0e5)


def power_law(phi: float, k: float, n: float) -> float:
    """u_p / u* = k (1 - phi)^n (eq. (19))."""
    return k * (1.0 - phi) ** n


def tstar_per_step(d: float, g: float, s: float, nu: float) -> float:
    """Normalised time of one lattice time step, D g (s-1) / (18 nu)."""
    return d * g * (s - 1.0) / (18.0 * nu)


def time_average(t, v, t_from: float) -> float:
    """Mean of the samples v taken at times t >= t_from (trapezoidal in
    time over the sampled interval; a single sample returns itself)."""
    t = np.asarray(t, float)
    v = np.asarray(v, float)
    m = t >= t_from
    t, v = t[m], v[m]
    if t.size == 0:
        raise ValueError("no samples after the averaging start")
    if t.size == 1:
        return float(v[0])
    return float(np.trapezoid(v, t) / (t[-1] - t[0]))


def settling_run(wl: W.Workload, t_end: float, t_avg: float,
                 sample_every: int = 50, graph: bool = True,
                 progress=None, device: str = "cuda:0") -> dict:
    """Run a settling box to t*_end and return the normalised bulk velocity.

    The bulk velocity is sampled every sample_every steps as the mean over
    particles of the velocity component along gravity (positive when
    settling)."""
    from . import hlbm
    p, sc = wl.params, wl.scene
    gvec = np.asarray(p.gravity, float)
    g = float(np.linalg.norm(gvec))
    if g == 0.0:
        raise ValueError("the settling box needs gravity")
    down = gvec / g
    nu = (p.tau - 0.5) / 3.0
    s = float(sc.density[0])
    # sphere diameter of the particle volume (every body is volume-equivalent)
    if wl.d_equiv is not None:
        d = float(wl.d_equiv)
    elif int(sc.shape[0]) == W.SPHERE:
        d = 2.0 * float(sc.size[0])
    else:
        d = float(sc.size[0]) * (6.0 / math.pi) ** (1.0 / 3.0)
    dts = tstar_per_step(d, g, s, nu)
    steps = int(math.ceil(t_end / dts))
    steps = sample_every * int(math.ceil(steps / sample_every))
    ustar = single_particle_velocity(g, d, s, nu)
    ustokes = g * d * d * (s - 1.0) / (18.0 * nu)
    re = ustar * d / nu
    ar = g * d ** 3 * (s - 1.0) / (nu * nu)
    sim = hlbm.Simulation(p, sc, device=device, graph=graph, polyhedra=wl.polyhedra)
    sim.init_equilibrium()
    ts, us = [0.0], [0.0]
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        sim.step(sample_every)
        done += sample_every
        U = sim.particles()["U"]
        ts.append(done * dts)
        us.append(float((U @ down).mean()))
        if progress is not None and done % (sample_every * 100) == 0:
            progress(done, steps, us[-1] / ustar)
    sim.sync()
    wall = time.perf_counter() - t0
    ubar = time_average(ts, us, t_avg)
    k = k_yao(ar)
    return dict(
        n_particles=sc.n, lattice=[p.nx, p.ny, p.nz], d_cells=d, s=s,
        ar=ar, re=re, u_star=ustar, u_stokes=ustokes, steps=steps,
        t_end=steps * dts, t_avg_from=t_avg, u_bar=ubar,
        u_bar_over_u_star=ubar / ustar, u_bar_over_u_stokes=ubar / ustokes,
        richardson_zaki=power_law(_phi(wl), 1.0, n_richardson_zaki(re)),
        garside_al_dibouni_yao=power_law(_phi(wl), k, n_garside_al_dibouni(re)),
        wall_s=wall, ms_per_step=1e3 * wall / steps,
        series_t=ts, series_u_over_u_star=[u / ustar for u in us])


def _phi(wl: W.Workload) -> float:
    p, sc = wl.params, wl.scene
    if wl.d_equiv is not None:
        return sc.n * math.pi / 6.0 * float(wl.d_equiv) ** 3 / float(p.nx * p.ny * p.nz)
    if int(sc.shape[0]) == W.SPHERE:
        v = 4.0 / 3.0 * math.pi * float(sc.size[0]) ** 3
    else:
        v = float(sc.size[0]) ** 3
    return sc.n * v / float(p.nx * p.ny * p.nz)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--shape", nargs="+", default=["sphere", "cube"],
                    choices=["sphere", "cube", "octahedron", "box", "tetrahedron"])
    ap.add_argument("--phi", nargs="+", type=float, default=[0.1, 0.2, 0.3])
    ap.add_argument("--ar", nargs="+", type=float, default=[1000.0])
    ap.add_argument("--n-per-d", type=float, default=9.0,
                    help="cells per sphere diameter")
    ap.add_argument("--edge", type=int, default=120, help="box edge in cells")
    ap.add_argument("--t-end", type=float, default=400.0)
    ap.add_argument("--t-avg", type=float, default=50.0)
    ap.add_argument("--sample-every", type=int, default=50)
    ap.add_argument("--precision", choices=["fp64", "fp32", "fp16s"],
                    default="fp32")
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args(argv)
    prec = {"fp64": 0, "fp32": 1, "fp16s": 2}[args.precision]
    rows = []
    for ar in args.ar:
        for phi in args.phi:
            for shp in args.shape:
                shape = {"sphere": W.SPHERE, "cube": W.CUBE,
                         "octahedron": W.OCTAHEDRON}.get(shp, shp)
                def prog(done, steps, r, shp=shp, phi=phi, ar=ar):
                    print(f"  {shp} phi={phi} Ar={ar:g}: step {done}/{steps} "
                          f"u/u*={r:.4f}", flush=True)

                try:
                    wl = W.settling_box(shape, phi, args.n_per_d, ar=ar,
                                        seed=args.seed, precision=prec,
                                        edge_cells=args.edge)
                    r = settling_run(wl, args.t_end, args.t_avg,
                                     args.sample_every, progress=prog)
                except Exception as e:  # report and go on with the next point
                    print(json.dumps(dict(shape=shp, phi=phi, ar=ar,
                                          error=str(e))), flush=True)
                    continue
                r.pop("series_t")
                r.pop("series_u_over_u_star")
                r.update(shape=shp, phi=round(_phi(wl), 4))
                rows.append(r)
                print(json.dumps(r), flush=True)
    print("| Ar | phi | shape | n | u_bar/u* | RZ | GaD+Yao | u_bar/u_Stokes | ms/step |")
    print("|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['ar']:.0f} | {r['phi']:.3f} | {r['shape']} | "
              f"{r['n_particles']} | {r['u_bar_over_u_star']:.3f} | "
              f"{r['richardson_zaki']:.3f} | {r['garside_al_dibouni_yao']:.3f} | "
              f"{r['u_bar_over_u_stokes']:.3f} | {r['ms_per_step']:.3f} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
