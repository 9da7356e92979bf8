"""Full-length FP64 oracle references of the workloads (test infrastructure).

    python tests/golden/make_fullrun_refs.py C2 C3 C4 C5 [--every N]

Runs each workload through the FP64 CPU oracle (oracle/) for its stated
number of steps and writes tests/golden/fullrun_<name>.npz with:

* every N steps (and after the initial coupling, step 0): particle
  position, orientation, velocity and angular velocity, and the
  hydrodynamic and contact force and torque that moved them;
* every step: the number of detected pairs and flagged nodes (rough
  detection, Sec. 3.3.1), a 64-bit digest of the detected pair set and of
  the set of contacts with a positive overlap volume (the pairs that exert
  a contact force, eqs. (4)-(9));
* every contact episode: pair (a, b), first and last step with a positive
  overlap volume (the onset of eq. (6) and the end of the contact);
* after the last step: lattice mass and momentum, density extremes and the
  largest fluid speed.

Only the oracle and the seeded scene generator are called; nothing here
comes from the GPU path.  The GPU full-run tests summarise their own
contact lists with the functions below, so both sides are reduced the same
way.
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "oracle")):
    if p not in sys.path:
        sys.path.insert(0, p)

SNAP_KEYS = ("X", "q", "U", "omega", "Fh", "Th", "Fc", "Tc")
DEFAULT_EVERY = {"C2": 50, "C3": 100, "C4": 100, "C5": 50}


def ref_path(name):
    return os.path.join(HERE, f"fullrun_{name}.npz")


def digest(pairs):
    """64-bit digest of a sorted list of (a, b) pairs."""
    arr = np.asarray(pairs, np.int64).reshape(-1, 2)
    return int.from_bytes(hashlib.blake2b(arr.tobytes(), digest_size=8).digest(),
                          "little")


def contact_sets(contacts):
    """(detected pairs, pairs with a positive overlap volume), each sorted.
    A record is detected when its latest rough detection flagged nodes; it
    has a positive volume when the latest treatment kept it (carried)."""
    det = sorted((c["a"], c["b"]) for c in contacts if c["count"] > 0)
    act = sorted((c["a"], c["b"]) for c in contacts
                 if c["carried"] and c["volume"] > 0.0)
    return det, act


class Episodes:
    """Contact episodes: (a, b, first step with V > 0, last step with V > 0)."""

    def __init__(self):
        self.open = {}
        self.done = []

    def update(self, step, active):
        cur = set(active)
        for k in list(self.open):
            if k not in cur:
                self.done.append((k[0], k[1], self.open.pop(k), step - 1))
        for k in cur:
            if k not in self.open:
                self.open[k] = step

    def close(self, last_step):
        out = list(self.done) + [(k[0], k[1], s, last_step)
                                 for k, s in self.open.items()]
        return np.array(sorted(out), np.int64).reshape(-1, 4)


def snapshot(particles, forces):
    d = dict(particles)
    d.update(forces)
    return {k: np.array(d[k], np.float64) for k in SNAP_KEYS}


def run(name, every, log=print):
    import oracle as O
    from paper_2401_10878_amd import workloads as W
    wl = W.WORKLOADS[name]()
    for k, P in (wl.polyhedra or {}).items():
        O.define_polyhedron(k, P.vertices, P.faces)
    s = O.OracleSim(wl.params, wl.scene)
    t0 = time.time()
    s.init_equilibrium()
    snaps = {k: [] for k in SNAP_KEYS}
    snap_steps = []

    def take(step):
        sn = snapshot(s.particles(), s.forces())
        for k in SNAP_KEYS:
            snaps[k].append(sn[k])
        snap_steps.append(step)

    take(0)
    nsteps = wl.steps
    det_n = np.zeros(nsteps + 1, np.int64)
    det_cells = np.zeros(nsteps + 1, np.int64)
    det_hash = np.zeros(nsteps + 1, np.uint64)
    act_n = np.zeros(nsteps + 1, np.int64)
    act_hash = np.zeros(nsteps + 1, np.uint64)
    ep = Episodes()

    def record(step):
        det, act = contact_sets(s.contacts())
        det_n[step], det_cells[step] = s.counters()
        det_hash[step] = np.uint64(digest(det))
        act_n[step] = len(act)
        act_hash[step] = np.uint64(digest(act))
        ep.update(step, act)

    record(0)
    for t in range(1, nsteps + 1):
        s.step(1)
        record(t)
        if t % every == 0 or t == nsteps:
            take(t)
            log(f"{name}: step {t}/{nsteps}, {det_n[t]} pairs, {act_n[t]} in contact, "
                f"{time.time() - t0:.0f} s")
    f = s.fields()
    rho, u = f["rho"], f["u"]
    mom = (rho[..., None] * u).reshape(-1, 3).sum(axis=0)
    out = dict(
        workload=np.array(f"{wl.name}: {wl.note}"), steps=np.int64(nsteps),
        snap_steps=np.array(snap_steps, np.int64),
        det_n=det_n, det_cells=det_cells, det_hash=det_hash,
        act_n=act_n, act_hash=act_hash, episodes=ep.close(nsteps),
        mass=np.float64(rho.sum()), momentum=mom,
        rho_min=np.float64(rho.min()), rho_max=np.float64(rho.max()),
        speed_max=np.float64(np.sqrt((u * u).sum(-1)).max()),
        oracle_threads=np.int64(O.threads()),
        wall_s=np.float64(time.time() - t0))
    for k in SNAP_KEYS:
        out["snap_" + k] = np.stack(snaps[k])
    s.close()
    np.savez_compressed(ref_path(name), **out)
    log(f"{name}: wrote {ref_path(name)} ({time.time() - t0:.0f} s)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=sorted(DEFAULT_EVERY))
    ap.add_argument("--every", type=int, default=0,
                    help="snapshot interval (default per workload)")
    a = ap.parse_args()
    for n in a.names:
        run(n, a.every or DEFAULT_EVERY[n], log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
