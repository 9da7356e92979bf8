"""FP64 CPU reference gradient of the adjoint workload (test infrastructure).

    python tests/golden/make_c5_oracle_fd.py

J = mean over the 27 cubes of U_z after 500 steps of the 96^3 adjoint box,
from fluid at rest.  Central differences of the FP64 oracle (oracle/) along
two directions, written to tests/golden/c5_oracle_fd.json:

* the common density ratio, s_p -> s_p + h for every particle (h = 1e-9);
* a seeded random rotation of every particle's initial orientation,
  q_p -> exp(h v_p / 2) (x) q_p (h = 1e-11), with the directions v_p stored
  beside the result.

The steps are small because a perturbation that moves a node across the
edge of the coupling band during the 500 steps switches its owner, which
changes the momentum exchange by a finite amount that a gradient with
frozen owners does not contain: a rotation of 1e-9 rad did so in about
half of the directions tried (a jump of about 1e-10 in J), 1e-11 rad in
about one in two hundred.  The run also records that no
node is flagged by the rough detection at any step (no contact can start, so
holding contact forces fixed in the adjoint is exact).
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "oracle")):
    if p not in sys.path:
        sys.path.insert(0, p)

OUT = os.path.join(HERE, "c5_oracle_fd.json")
H_DENSITY = 1e-9
H_ROTATION = 1e-11
SEED = 55


def rotate(q, axis, ang):
    """exp(ang axis / 2) (x) q for a unit axis (world-frame rotation)."""
    h = 0.5 * ang
    w1, x1, y1, z1 = [math.cos(h)] + list(math.sin(h) * np.asarray(axis, float))
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def directions(n):
    return np.random.default_rng(SEED).normal(size=(n, 3))


def run_J(O, wl, scene):
    s = O.OracleSim(wl.params.replace(precision=0), scene)
    s.init_equilibrium()
    flagged = 0
    for _ in range(wl.steps):
        s.step(1)
        flagged += s.counters()[1]
    J = float(s.particles()["U"][:, 2].mean())
    s.close()
    return J, flagged


def main():
    import oracle as O
    from paper_2401_10878_amd import workloads as W
    wl = W.c5_adjoint_cubes()
    sc = wl.scene
    v = directions(sc.n)
    t0 = time.time()

    def dens(hh):
        s = sc.copy()
        s.density = s.density + hh
        return s

    def rot(hh):
        s = sc.copy()
        for i in range(s.n):
            ang = float(np.linalg.norm(v[i]))
            s.q[i] = rotate(s.q[i], v[i] / ang, hh * ang)
        return s

    J0, flagged = run_J(O, wl, sc)
    out = dict(workload=f"{wl.name}: {wl.note}", steps=wl.steps,
               h_density=H_DENSITY, h_rotation=H_ROTATION,
               J=J0, flagged_nodes_all_steps=int(flagged),
               rotation_seed=SEED, rotation_directions=v.tolist())
    for name, fn, h in (("density", dens, H_DENSITY), ("rotation", rot, H_ROTATION)):
        jp, fp = run_J(O, wl, fn(h))
        jm, fm = run_J(O, wl, fn(-h))
        out[name] = dict(J_plus=jp, J_minus=jm, fd=(jp - jm) / (2 * h),
                         flagged_nodes=int(fp + fm))
        print(f"{name}: fd {(jp - jm) / (2 * h):+.9e} ({time.time() - t0:.0f} s)",
              flush=True)
    out["oracle_threads"] = O.threads()
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
