#!/usr/bin/env python3
"""Throughput of the coupled HLBM + discrete-contact time step on one GPU.

Default workload: dense settling box, 256^3 periodic lattice, 1834 cubes of
edge 14 (phi = 0.30, s = 1.5, Ar = 1000), populations in FP32, synthetic
seeded scene.  A step is the whole time step: contact treatment, particle
motion and tile binning, contact carry-over, coupling map with rough
detection, and the stream-collide pass with the coupling, which also sums
the momentum exchange of the populations it writes.  The timed steps are replayed as
captured HIP graphs (8 steps per graph, the contact treatment of each step
on a second stream beside the previous step's lattice passes); --stream
times plain stream launches instead, and the line reports the other mode's
time beside the value.

Prints ONE JSON line with the metric, the roofline of the dominant kernel
(the stream-collide pass, HBM-bound) and the FP64 CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--precision fp32|fp64|fp16s]
                    [--workload C1|C2|C3|C3B|C3E|C4|C5] [--stream]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_TFLOPS = 78.6        # MI355X dense FP64 vector
# FP64 operations of one midpoint sample of the contact treatment for a pair
# of cubes (both bodies; additions, multiplications, divisions and square
# roots count one each, comparisons and selects none): a face sample takes
# the sample point (6), per body the offset (3), the rotation into the body
# frame (15), |p| - h (4), the squared outside part (5), its root (1), the
# sum with the inside part (1) and the enlargement (1); an integration
# sample takes the point (9), per body the same 30 plus the gradient
# (3 divisions, 3 sign products, the rotation back: 15), and the sums of
# position, gradient difference and depth (10)
CUBE_FLOP_FACE = 6 + 2 * 30
CUBE_FLOP_INTEGRATION = 9 + 2 * (30 + 21) + 10
PREC = {"fp64": 0, "fp32": 1, "fp16s": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16s": "f16-storage/f32-compute"}
VALUE_BYTES = {0: 8, 1: 4, 2: 2}
W_POLY0 = 3                    # shape code of the first polyhedron type
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_lattice_c3_traffic.json")
# the sources the stream-collide kernel is built from
LATTICE_SRC = [os.path.join(ROOT, "paper_2401_10878_amd", "csrc", f)
               for f in ("k_lattice.hip", "device_math.h", "context.h")]


def lattice_source_hash():
    h = hashlib.sha256()
    for f in LATTICE_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_for(prec_name, section="per_precision", field="bytes_per_launch",
                workload="C3"):
    """HBM bytes per launch of the stream-collide pass from the committed
    rocprofv3 counters, or None if the counters were taken on another
    workload or another version of the kernels."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != lattice_source_hash():
        return None
    if str(d.get("workload", "")).split(":")[0] != workload:
        return None
    e = d.get(section, {}).get(prec_name)
    return e.get(field) if e else None


def contact_roofline(wl, res):
    """Algorithmic FP64 operations of the contact treatment per second (its
    event-timed kernel time, the last step's pair count) against the FP64
    vector peak; None unless every particle is a cube."""
    if not all(int(s) == 1 for s in wl.scene.shape):
        return None
    nc = wl.params.n_c
    flop = res["pairs"] * (6 * nc ** 2 * CUBE_FLOP_FACE + nc ** 3 * CUBE_FLOP_INTEGRATION)
    tf = flop / (res["kernel_ms_per_step"]["treat"] * 1e-3) / 1e12
    return dict(bound="fp64", kernel="k_treat", achieved=round(tf, 3),
                peak=PEAK_FP64_TFLOPS, unit="TFLOP/s", frac=round(tf / PEAK_FP64_TFLOPS, 4),
                flop_per_step=int(flop), flop_per_face_sample=CUBE_FLOP_FACE,
                flop_per_integration_sample=CUBE_FLOP_INTEGRATION)


def run_gpu(wl, prec, steps, warmup, graph):
    import torch
    from paper_2401_10878_amd import hlbm
    p = wl.params.replace(precision=PREC[prec])
    sim = hlbm.Simulation(p, wl.scene, device="cuda:0", graph=graph,
                          polyhedra=wl.polyhedra)
    sim.init_equilibrium()
    sim.step(warmup)
    sim.sync()
    c0 = sim.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = sim.counters()
    # per-kernel times from a second window of the same length, with HIP
    # events around every launch (those steps run their kernels one after
    # another: the contact treatment does not overlap the lattice passes)
    sim.timing_begin(steps)
    sim.step(steps)
    sim.sync()
    kms, n = sim.timing_end()
    ncell = p.nx * p.ny * p.nz
    wall = t1 - t0
    out = dict(
        mlups=ncell * steps / wall / 1e6,
        ms_per_step=wall * 1e3 / steps,
        contact_cells_per_s=(c1["total_cells"] - c0["total_cells"]) / wall,
        kernel_ms_per_step={k: v / n for k, v in kms.items()},
        pairs=c1["pairs"], overlap_cells=c1["cells"],
    )
    lat_s = kms["lattice"] / n / 1e3
    bytes_alg = 2 * 19 * VALUE_BYTES[PREC[prec]] * ncell
    out["lattice_gbs"] = bytes_alg / lat_s / 1e9
    out["bytes_alg"] = bytes_alg
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def other_ms_per_step(wl, prec, steps, warmup, graph):
    """Wall time per step of the other launch mode: captured HIP graphs
    (graph=True) or stream launches."""
    import torch
    from paper_2401_10878_amd import hlbm
    sim = hlbm.Simulation(wl.params.replace(precision=PREC[prec]), wl.scene,
                          device="cuda:0", graph=graph, polyhedra=wl.polyhedra)
    sim.init_equilibrium()
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return (t1 - t0) * 1e3 / steps


def reference_force(wl):
    """(s - 1) V |g| of the heaviest particle: the force scale of the error
    normalisation max(|F|, F_ref)."""
    import numpy as np
    sc, g = wl.scene, abs(wl.params.gravity[2])
    V = np.where(sc.shape == 0, 4.0 / 3.0 * np.pi * sc.size ** 3,
                 np.where(sc.shape == 2, 4.0 / 3.0, 1.0) * sc.size ** 3)
    for k, P in (wl.polyhedra or {}).items():
        # a normalising scale only: the volume of the polyhedron by the
        # divergence theorem over its faces, fanned into triangles (of an
        # ellipsoid type, 4 pi abc / 3)
        if hasattr(P, "axes"):
            vol = 4.0 / 3.0 * np.pi * float(np.prod(P.axes))
        else:
            v = P.vertices
            vol = sum(np.dot(v[f[0]], np.cross(v[f[j]], v[f[j + 1]]))
                      for f in P.faces for j in range(1, len(f) - 1)) / 6.0
        m = sc.shape == W_POLY0 + k
        V[m] = vol * sc.size[m] ** 3
    return ((sc.density - 1.0) * V).max() * g


def state_errors(wl, got, ref):
    """Errors of a GPU state against a reference state after the same steps:
    mean settling velocity (mean U_z), hydrodynamic force (relative to
    max(|F|, (s - 1) V |g|)) and particle velocity (relative to the largest
    reference speed)."""
    import numpy as np
    Fref = reference_force(wl)
    U, Ur = got["U"], ref["U"]
    F, Fr = got["Fh"], ref["Fh"]
    uz, uzr = U[:, 2].mean(), Ur[:, 2].mean()
    return dict(
        mean_settling_velocity_rel=float(abs(uz - uzr) / abs(uzr)),
        force_rel=float((np.abs(F - Fr) / np.maximum(np.abs(Fr), Fref)).max()),
        velocity_rel=float(np.abs(U - Ur).max() / np.abs(Ur).max()))


def gpu_short_state(wl, prec, steps):
    """Particle velocities and hydrodynamic forces after `steps` steps from
    the initial state (stream launches), for the comparison with the
    oracle's run of the same steps."""
    import torch
    from paper_2401_10878_amd import hlbm
    sim = hlbm.Simulation(wl.params.replace(precision=PREC[prec]), wl.scene,
                          device="cuda:0", polyhedra=wl.polyhedra)
    sim.init_equilibrium()
    sim.step(steps)
    sim.sync()
    out = dict(U=sim.particles()["U"], Fh=sim.forces()["Fh"])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, steps):
    """The FP64 oracle timed on the host cores over `steps` steps of the
    workload; also returns its particle velocities and hydrodynamic forces
    after those steps (the reference of the precision errors)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    for k, P in (wl.polyhedra or {}).items():
        O.define_body_type(k, P)
    s = O.OracleSim(wl.params, wl.scene)
    s.init_equilibrium()
    # one step per call, so that the flagged contact cells of each step can
    # be read between the timed calls
    wall, cells = 0.0, 0
    for _ in range(steps):
        t0 = time.perf_counter()
        s.step(1)
        wall += time.perf_counter() - t0
        cells += s.counters()[1]
    ncell = wl.params.nx * wl.params.ny * wl.params.nz
    res = dict(value=round(ncell * steps / wall / 1e6, 3), unit="MLUPS",
               cores=O.threads(), kind="oracle",
               contact_cells_per_s=round(cells / wall, 1),
               sample=f"{wl.name}: {steps} coupled FP64 steps after the prologue "
                      f"({ncell} nodes, {wl.scene.n} particles), {wall:.1f} s")
    state = dict(U=s.particles()["U"], Fh=s.forces()["Fh"])
    s.close()
    return res, state


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain streaming copy of known size (an elementwise kernel that reads
    nbytes and writes nbytes), profiled beside the lattice kernel to scale the
    HBM byte counters (FETCH_SIZE, WRITE_SIZE)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_read=nbytes, copy_bytes_written=nbytes,
                          launches=reps)), flush=True)


def traffic_summary(outdir, workload_name):
    """Write the counter file from four rocprofv3 --pmc runs (csv output)
    under outdir: pmc_FETCH_SIZE and pmc_WRITE_SIZE of the benchmark command
    and copy_FETCH_SIZE, copy_WRITE_SIZE of --copy-calibration.  FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch) of the stream-collide kernel are
    scaled by what the same counters read for the plain copy of known size."""
    import csv
    import glob

    def rows(sub):
        files = glob.glob(os.path.join(outdir, sub, "**", "*counter_collection.csv"),
                          recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {outdir}/{sub}")
        out = []
        for f in files:
            with open(f) as fh:
                out.extend(csv.DictReader(fh))
        return out

    def per_kernel(sub, counter, match):
        vals = {}
        for r in rows(sub):
            if r.get("Counter_Name") != counter or match not in r.get("Kernel_Name", ""):
                continue
            vals.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
            vals[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: sum(v.values()) / len(v) for k, v in vals.items()}, \
            {k: len(v) for k, v in vals.items()}

    cf, _ = per_kernel("copy_FETCH_SIZE", "FETCH_SIZE", "elementwise")
    cw, _ = per_kernel("copy_WRITE_SIZE", "WRITE_SIZE", "elementwise")
    nbytes = 1 << 30
    fetch_factor = nbytes / (max(cf.values()) * 1024.0)
    write_factor = nbytes / (max(cw.values()) * 1024.0)
    lf, ln = per_kernel("pmc_FETCH_SIZE", "FETCH_SIZE", "k_lattice")
    lw, _ = per_kernel("pmc_WRITE_SIZE", "WRITE_SIZE", "k_lattice")
    mf, mn = per_kernel("pmc_FETCH_SIZE", "FETCH_SIZE", "k_mea")
    mw, _ = per_kernel("pmc_WRITE_SIZE", "WRITE_SIZE", "k_mea")
    kind = {"k_lattice<double": "fp64", "k_lattice<float": "fp32",
            "k_lattice<__half": "fp16s"}
    mkind = {"k_mea<double": "fp64", "k_mea<float": "fp32", "k_mea<__half": "fp16s"}
    per = {}
    for name, fkib in lf.items():
        prec = next((v for k, v in kind.items() if k in name), None)
        wkib = lw.get(name)
        if prec is None or wkib is None:
            continue
        rd, wr = fkib * 1024.0 * fetch_factor, wkib * 1024.0 * write_factor
        alg = 2 * 19 * VALUE_BYTES[PREC[prec]] * 256 ** 3
        per[prec] = dict(fetch_size_kib=round(fkib, 1), write_size_kib=round(wkib, 1),
                         read_bytes=int(rd), write_bytes=int(wr),
                         bytes_per_launch=int(rd + wr), launches=ln[name],
                         algorithmic_bytes=alg,
                         traffic_over_algorithmic=round((rd + wr) / alg, 4))
    # the separate momentum-exchange pass (the initial state only):
    # measured bytes per launch
    for name, fkib in mf.items():
        prec = next((v for k, v in mkind.items() if k in name), None)
        wkib = mw.get(name)
        if prec is None or wkib is None or prec not in per:
            continue
        rd, wr = fkib * 1024.0 * fetch_factor, wkib * 1024.0 * write_factor
        per[prec]["separate_mea"] = dict(read_bytes=int(rd), write_bytes=int(wr),
                                         launches=mn[name])
    d = dict(kernel="k_lattice", workload=workload_name,
             note="HBM bytes per launch of the stream-collide pass (which also sums "
                  "the momentum exchange of the next step), from FETCH_SIZE and "
                  "WRITE_SIZE scaled by a plain 1 GiB copy",
             kernel_source_sha256_16=lattice_source_hash(),
             commands=["cd /tmp && export TMPDIR=/tmp",
                       "rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'k_lattice|k_mea' "
                       "--output-format csv -d <out>/pmc_FETCH_SIZE -o lat -- python3 "
                       "bench.py --steps 4 --warmup 1 --cpu-steps 0",
                       "rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'k_lattice|k_mea' "
                       "--output-format csv -d <out>/pmc_WRITE_SIZE -o lat -- python3 "
                       "bench.py --steps 4 --warmup 1 --cpu-steps 0",
                       "rocprofv3 --pmc FETCH_SIZE --output-format csv -d "
                       "<out>/copy_FETCH_SIZE -o copy -- python3 bench.py --copy-calibration",
                       "rocprofv3 --pmc WRITE_SIZE --output-format csv -d "
                       "<out>/copy_WRITE_SIZE -o copy -- python3 bench.py --copy-calibration",
                       "python3 bench.py --traffic-summary <out>"],
             calibration=dict(copy_bytes_read=nbytes, copy_bytes_written=nbytes,
                              fetch_size_kib=round(max(cf.values()), 1),
                              write_size_kib=round(max(cw.values()), 1),
                              fetch_factor=round(fetch_factor, 4),
                              write_factor=round(write_factor, 4)),
             per_precision=per)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=sorted(PREC))
    ap.add_argument("--workload", default="C3", choices=["C1", "C2", "C3", "C3B", "C3E", "C4", "C5"])
    ap.add_argument("--stream", action="store_true",
                    help="time stream launches instead of captured HIP graphs")
    ap.add_argument("--other-precisions", type=int, default=1,
                    help="also time the other two storage precisions")
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="oracle steps timed for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--traffic-summary", metavar="DIR",
                    help="write the counter file from rocprofv3 --pmc output under DIR")
    args = ap.parse_args()
    if args.traffic_summary:
        from paper_2401_10878_amd import workloads as W
        wl = W.WORKLOADS[args.workload]()
        traffic_summary(args.traffic_summary, f"{wl.name}: {wl.note}")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU "
              "path.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_2401_10878_amd import workloads as W
    wl = W.WORKLOADS[args.workload]()
    graph = not args.stream
    main_res = run_gpu(wl, args.precision, args.steps, args.warmup, graph)
    runs = {args.precision: main_res}
    if args.other_precisions:
        for pr in PREC:
            if pr != args.precision:
                runs[pr] = run_gpu(wl, pr, args.steps, args.warmup, graph)
    others = {}
    for pr, r in runs.items():
        others[pr] = dict(mlups=round(r["mlups"], 1),
                          ms_per_step=round(r["ms_per_step"], 4),
                          lattice_gbs=round(r["lattice_gbs"], 1))
        if "fp64" in runs and pr != "fp64":
            others[pr]["speedup_vs_fp64"] = round(runs["fp64"]["ms_per_step"]
                                                  / r["ms_per_step"], 3)
    other_ms = other_ms_per_step(wl, args.precision, args.steps, args.warmup,
                                 not graph)
    lat_ms = main_res["kernel_ms_per_step"]["lattice"]
    achieved = main_res["lattice_gbs"]
    traffic = traffic_for(args.precision, workload=wl.name)
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS,
                unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4),
                traffic=traffic, kernel="k_lattice",
                bytes_per_launch=main_res["bytes_alg"],
                avg_launch_ms=round(lat_ms, 5),
                # measured HBM bytes (rocprofv3 counters) over the same time
                traffic_gbs=None if traffic is None else round(traffic / (lat_ms * 1e6), 1))
    cpu = None
    if args.cpu_steps > 0:
        cpu, oracle_state = cpu_baseline(wl, args.cpu_steps)
        # each precision against the FP64 oracle after the same steps
        for pr in runs:
            got = gpu_short_state(wl, pr, args.cpu_steps)
            others[pr]["error_vs_oracle"] = dict(
                steps=args.cpu_steps,
                **{k: float(f"{v:.3e}") for k, v in
                   state_errors(wl, got, oracle_state).items()})
    p = wl.params
    line = dict(
        metric="coupled-step MLUPS (+ contact cells/s)",
        value=round(main_res["mlups"], 1), unit="MLUPS", n_gpus=1,
        steps=args.steps, warmup=args.warmup,
        ms_per_step=round(main_res["ms_per_step"], 4),
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=DTYPE[args.precision], data="synthetic",
        config=dict(workload=f"{wl.name}: {wl.note}", lattice=[p.nx, p.ny, p.nz],
                    particles=wl.scene.n, precision=args.precision,
                    graph=graph),
        contact_cells_per_s=round(main_res["contact_cells_per_s"], 1),
        detected_pairs=main_res["pairs"], overlap_cells=main_res["overlap_cells"],
        # the contact treatment alone: its kernel time, and midpoint samples
        # (6 n_c^2 box-correction + n_c^3 integration per pair, two bodies
        # each) per second at the last step's pair count
        contact_kernel_ms_per_step=round(main_res["kernel_ms_per_step"]["treat"], 5),
        contact_samples_per_s=round(
            main_res["pairs"] * (6 * p.n_c ** 2 + p.n_c ** 3)
            / (main_res["kernel_ms_per_step"]["treat"] * 1e-3), 1),
        # the contact treatment against the FP64 vector peak (scenes of
        # cubes only: the FP64 operations per sample are those of a cube
        # pair, every box face sampled)
        contact_roofline=contact_roofline(wl, main_res),
        # the lattice pass includes the momentum exchange of the next step,
        # the particle launch the contact carry-over (their own slots stay
        # empty)
        kernel_ms_per_step={k: round(v, 5) for k, v in
                            main_res["kernel_ms_per_step"].items()
                            if k not in ("mea", "keep")},
        # the other launch mode of the same workload and precision
        **{("stream_ms_per_step" if graph else "graph_ms_per_step"): round(other_ms, 4)},
        precisions=others,
        roofline=roof,
        # the whole step against the same bound: algorithmic population
        # bytes per step over the wall time per step
        step_roofline=dict(bytes_per_step=main_res["bytes_alg"],
                           achieved=round(main_res["bytes_alg"] / (main_res["ms_per_step"] * 1e6), 1),
                           peak=PEAK_HBM_GBS, unit="GB/s",
                           frac=round(main_res["bytes_alg"] / (main_res["ms_per_step"] * 1e6)
                                      / PEAK_HBM_GBS, 4)),
        cpu_baseline=cpu,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
