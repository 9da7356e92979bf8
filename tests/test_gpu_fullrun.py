"""Full-length runs of the workloads against the stored FP64 oracle runs.

Each workload runs its stated number of steps on the GPU in one precision
(FP64, FP32, binary16 storage) from the same seeded scene as the oracle run
written by tests/golden/make_fullrun_refs.py, and is compared with it:

* every step: the detected pair set (digest) and the pairs with a positive
  overlap volume;
* contact episodes: the onset of every contact (first step with a positive
  overlap volume, where eq. (6) fixes the damping) and its end; an onset or
  end that differs is counted as a shift, and the particles of a shifted
  episode leave the pointwise trajectory comparison from that step on;
* at the stored snapshots: positions, orientations, velocities, angular
  velocities and the hydrodynamic force of the remaining particles, and the
  mean settling velocity (mean U_z) of all particles;
* at the end, for the fully periodic boxes: the lattice momentum per unit
  lattice mass against the mean settling velocity (zero net volume flow:
  below 1e-3 of it, the bound the stored oracle runs meet).

The bounds asserted are the ones measured, with a margin (the rounding of
the FP64 path differs from the oracle's in the order of its sums, and a node
whose distance sits within that rounding of the coupling-band edge switches
owner: a discrete change of the momentum exchange that the trajectories then
carry; FP32 and binary16 storage add their own rounding every step).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullrun_refs as R  # noqa: E402

# (workload, precision): bounds over the whole run on the errors of the
# particles without a shifted contact episode (velocity relative to the
# largest oracle speed, angular velocity relative to the largest oracle
# spin, hydrodynamic force relative to max(|F|, (s - 1) V g)), on the
# relative error of the final mean settling velocity, and on the number of
# contact episodes whose onset or end differs from the oracle's.  Measured
# (worst over the run) and asserted with a margin of about three:
#   C2 FP64  U 9.6e-14  omega 2.8e-13  Fh 3.5e-13  msv 3.6e-14  shifts 0 of 81
#   C2 FP32  U 3.7e-5   omega 3.0e-4   Fh 2.5e-4   msv 2.6e-5   shifts 0 of 81
#   C3 FP64  U 1.4e-13  omega 4.0e-13  Fh 6.4e-12  msv 1.2e-14  shifts 0 of 338
#   C3 FP32  U 1.9e-5   omega 1.5e-4   Fh 3.2e-4   msv 1.3e-5   shifts 2 + 2
#   C3 b16   U 2.3e-5   omega 1.5e-4   Fh 4.7e-4   msv 1.9e-6   shifts 2 + 2
#   C4 FP64  U 9.8e-14  omega 1.2e-13  Fh 3.8e-12  msv 2.5e-15  shifts 0 of 25
#   C4 FP32  U 2.1e-5   omega 5.0e-5   Fh 5.8e-4   msv 1.2e-5   shifts 1 + 1
#   C4 b16   U 2.5e-5   omega 6.1e-5   Fh 6.8e-4   msv 4.9e-7   shifts 0
# The number of shifted episodes of the reduced-precision runs follows the
# rounding of the whole trajectory: builds that differ only in the order of
# sums gave 1 + 1, 2 + 2 and 4 + 4 for binary16 storage in the cube box.
# Its bound is 5% of the oracle's episodes (at least 4).
#   C5 FP64  U 4.3e-14  omega 5.4e-13  Fh 6.3e-13  msv 2.3e-14  (no contacts)
#   C5 FP32  U 1.2e-5   omega 4.0e-4   Fh 1.3e-5   msv 1.1e-5
#   C5 b16   U 7.2e-5   omega 1.7e-3   Fh 7.5e-4   msv 5.3e-5
BOUNDS = {
    ("C2", 0): dict(U=3e-13, omega=1e-12, Fh=1e-12, msv=1e-13, shifts=0),
    ("C2", 1): dict(U=1.2e-4, omega=1e-3, Fh=8e-4, msv=8e-5, shifts=0),
    ("C3", 0): dict(U=5e-13, omega=1.5e-12, Fh=2e-11, msv=5e-14, shifts=0),
    ("C3", 1): dict(U=6e-5, omega=5e-4, Fh=1e-3, msv=4e-5, shifts=17),
    ("C3", 2): dict(U=8e-5, omega=5e-4, Fh=2.5e-3, msv=1.2e-5, shifts=17),
    ("C4", 0): dict(U=3e-13, omega=4e-13, Fh=1.2e-11, msv=1e-14, shifts=0),
    ("C4", 1): dict(U=6e-5, omega=1.5e-4, Fh=2e-3, msv=4e-5, shifts=4),
    ("C4", 2): dict(U=8e-5, omega=2e-4, Fh=2e-3, msv=4e-5, shifts=4),
    ("C5", 0): dict(U=2e-13, omega=2e-12, Fh=2e-12, msv=1e-13, shifts=0),
    ("C5", 1): dict(U=4e-5, omega=1.5e-3, Fh=5e-5, msv=4e-5, shifts=0),
    ("C5", 2): dict(U=2.5e-4, omega=5e-3, Fh=2.5e-3, msv=2e-4, shifts=0),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(name, prec):
    if not os.path.exists(R.ref_path(name)):
        pytest.skip(f"no stored oracle run for {name} (make_fullrun_refs.py)")
    return np.load(R.ref_path(name))


def run_gpu(W, H, name, prec, snap_steps, nsteps):
    wl = W.WORKLOADS[name]()
    sim = H.Simulation(wl.params.replace(precision=prec), wl.scene,
                       polyhedra=wl.polyhedra)
    sim.init_equilibrium()
    snaps = {k: [] for k in R.SNAP_KEYS}
    det_hash = np.zeros(nsteps + 1, np.uint64)
    act_hash = np.zeros(nsteps + 1, np.uint64)
    ep = R.Episodes()

    def record(t):
        det, act = R.contact_sets(sim.contacts())
        det_hash[t] = np.uint64(R.digest(det))
        act_hash[t] = np.uint64(R.digest(act))
        ep.update(t, act)
        if t in snap_steps:
            sn = R.snapshot(sim.particles(), sim.forces())
            for k in R.SNAP_KEYS:
                snaps[k].append(sn[k])

    record(0)
    for t in range(1, nsteps + 1):
        sim.step(1)
        record(t)
    flow = None
    if wl.params.periodic_z:
        f = sim.fields(owner=False)
        rho, u = f["rho"], f["u"]
        flow = (float(rho.sum()), (rho[..., None] * u).reshape(-1, 3).sum(axis=0))
    sim.close()
    return wl, {k: np.stack(v) for k, v in snaps.items()}, det_hash, act_hash, \
        ep.close(nsteps), flow


def episode_shifts(ref_ep, gpu_ep):
    """Episodes (a, b, start, end) present in one run and not the other:
    the earliest differing step per particle."""
    a = {tuple(e) for e in ref_ep.tolist()}
    b = {tuple(e) for e in gpu_ep.tolist()}
    shifted = a ^ b
    first = {}
    for (p, q, s, e) in shifted:
        for k in (p, q):
            if k >= 0:
                first[k] = min(first.get(k, 1 << 30), s)
    return len(a - b), len(b - a), first


@pytest.mark.parametrize("name,prec", sorted(BOUNDS))
def test_full_run_against_oracle(W, H, name, prec):
    ref = _case(name, prec)
    nsteps = int(ref["steps"])
    snap_steps = [int(s) for s in ref["snap_steps"]]
    _say(f"{name} precision {prec}: {nsteps} steps")
    wl, g, det_hash, act_hash, gep, flow = run_gpu(W, H, name, prec, set(snap_steps), nsteps)
    sc = wl.scene
    # scales: velocities and forces relative to max(|oracle|, reference)
    gmag = abs(wl.params.gravity[2])
    V = np.where(sc.shape == 0, 4.0 / 3.0 * np.pi * sc.size ** 3, sc.size ** 3)
    Fref = max(((sc.density - 1.0) * V).max() * gmag, 1e-12)
    Uref = max(np.abs(ref["snap_U"]).max(), 1e-12)
    Wref = max(np.abs(ref["snap_omega"]).max(), 1e-12)
    same_det = det_hash == ref["det_hash"]
    first_det = int(np.argmin(same_det)) if not same_det.all() else None
    same_act = act_hash == ref["act_hash"]
    first_act = int(np.argmin(same_act)) if not same_act.all() else None
    only_ref, only_gpu, first = episode_shifts(ref["episodes"], gep)
    _say(f"  episodes: oracle {len(ref['episodes'])}, gpu {len(gep)}, shifted "
         f"{only_ref} / {only_gpu}; first differing detection step {first_det}, "
         f"contact step {first_act}")
    worst = dict(X=0.0, q=0.0, U=0.0, omega=0.0, Fh=0.0)
    for j, t in enumerate(snap_steps):
        keep = np.array([first.get(i, 1 << 30) > t for i in range(sc.n)])
        if not keep.any():
            continue
        for k, scale in (("X", 1.0), ("q", 1.0), ("U", Uref), ("omega", Wref),
                         ("Fh", Fref)):
            a, b = g[k][j][keep], ref["snap_" + k][j][keep]
            d = a - b
            if k == "X":   # periodic positions: minimum image
                L = np.array([wl.params.nx, wl.params.ny, wl.params.nz], float)
                d = d - L * np.round(d / L) * np.array([1, 1, wl.params.periodic_z])
            if k == "Fh":
                e = (np.abs(d) / np.maximum(np.abs(b), Fref)).max()
            else:
                e = np.abs(d).max() / scale
            worst[k] = max(worst[k], float(e))
        _say(f"  step {t}: kept {keep.sum()}/{sc.n}, " +
             ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    uz = g["U"][-1][:, 2].mean()
    uzr = ref["snap_U"][-1][:, 2].mean()
    msv = abs(uz - uzr) / abs(uzr)
    _say(f"  mean settling velocity: gpu {uz:.9e} oracle {uzr:.9e} rel {msv:.2e}")
    if flow is not None:
        M, P = flow
        drift = np.abs(P).max() / M / abs(uz)
        _say(f"  lattice momentum / mass: {np.abs(P).max() / M:.3e} "
             f"({drift:.2e} of the mean settling velocity; oracle "
             f"{np.abs(ref['momentum']).max() / float(ref['mass']):.3e})")
        assert drift < 1e-3
    b = BOUNDS[(name, prec)]
    if b["shifts"] is not None:
        assert only_ref + only_gpu <= b["shifts"], (only_ref, only_gpu)
    for k in ("U", "omega", "Fh"):
        assert worst[k] <= b[k], (k, worst[k], b[k])
    assert msv <= b["msv"], (msv, b["msv"])
