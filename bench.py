"""Benchmark: Burton-Miller operator matvec (near field on the fly + FMM far
field) and GMRES solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1]

A step is one application of the whole operator (near field, FMM far field,
diagonal) to a seeded complex vector already resident in HBM, in FP64 (the
paper's arithmetic: the headline value); the mixed path (complex-FP32
operator) is timed the same way and reported beside it, with one GMRES solve
per precision and the surface pressure's error against the oracle's LU
solution.  Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic flops per near-field quadrature point of the fused formula (the
# Burton-Miller integrand as a polynomial in the scaled inverse distance U),
# FMA counted as two, rsqrt, sin and cos as one each: the quadratic form for
# the scaled |y - x|^2 (10), rsqrt and phase (2), sin and cos (2), the affine
# normal projection (4), the Horner form in U (16), weight times U^2 and the
# phase factor (4), the complex accumulation (8); 61 with the admittance terms
FLOPS_PER_POINT = 46
FLOPS_PER_POINT_BC = 61
# the same integrand evaluated term by term (G, H, H', E from r, 1/r and
# exp(ikr), then the Burton-Miller combination), the count of a direct
# implementation: 66 flops per point
FLOPS_PER_POINT_DIRECT = 66
# MI355X vector peaks: FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s with packed
# FP32 instructions, which the library's kernels are compiled without (78.6
# without them)
PEAK_TFLOPS = {"fp64": 78.6, "fp32_packed": 157.3, "fp32": 78.6}
SOLVE_TOL = 1e-6

WORKLOADS = {
    # config of the headline metric: 20480-triangle rigid sphere, 6 elements
    # per wavelength, 3-level FMM with ~32-element leaves
    "c2": dict(mesh=("icosphere", 5), use_fmm=1, levels=3, leaf_size=32, preset="tight",
               elems_per_wavelength=6.0),
    # 1280-triangle rigid sphere, k = 1, every pair by direct quadrature
    "c1": dict(mesh=("icosphere", 3), use_fmm=0, preset="tight", k=1.0),
    # head-like graded ellipsoid with a bump (~60k triangles), 16 kHz in air,
    # point source 1 mm off the bump, 5-level FMM
    "c3": dict(mesh=("graded", None), use_fmm=1, levels=5, leaf_size=32, preset="mixed",
               k=2 * math.pi * 16000.0 / 343.0, source="point"),
    # frequency sweep: 40500-triangle geodesic sphere, 64 log-spaced
    # frequencies 100 Hz - 20 kHz in air, per-frequency far-field method
    "c4": dict(mesh=("geodesic", 45), preset="mixed", sweep=True),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target host time of the oracle sample (the one-row probe overestimates a row, "
                         "so the sample usually takes about half of it)")
    ap.add_argument("--streams", type=int, default=1,
                    help="concurrent frequencies in the sweep workload (only 1: concurrent host threads are disabled)")
    ap.add_argument("--profile-near-only", action="store_true",
                    help="run only near-field applications (precision --profile-prec), then a 512 MiB "
                         "copy that calibrates the HBM byte counters (for rocprofv3 --pmc runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) "
                         "of --profile-near-only runs into the traffic record read by the bench")
    ap.add_argument("--traffic-out", default=None,
                    help="traffic record to write (default: the one of --profile-prec)")
    ap.add_argument("--summarize-valu", nargs=2, metavar=("PMC_CSV", "OUT_MD"),
                    help="per-kernel VALU instruction counts from a rocprofv3 --pmc run (SQ_INSTS_VALU, "
                         "SQ_ACTIVE_INST_VALU, SQ_WAVES, GRBM_GUI_ACTIVE) as a markdown summary")
    ap.add_argument("--profile-far-only", action="store_true",
                    help="run only far-field (FMM) applications, then the calibration copy")
    ap.add_argument("--profile-far-direct", action="store_true",
                    help="c4 mesh (40500 elements, depth 4) at 9382.3 Hz, the sweep's first direct-far-field "
                         "frequency: only direct far-field applications (precision --profile-prec, "
                         "--far-rows points per wavefront), then the calibration copy")
    ap.add_argument("--far-rows", type=int, default=0, choices=(0, 1, 4),
                    help="bem_options.far_rows of the --profile-far-direct mesh")
    ap.add_argument("--profile-prec", default="mixed", choices=("mixed", "fp64"),
                    help="operator precision of the --profile-near-only / --profile-far-only applications")
    ap.add_argument("--summarize-translate", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="per-launch HBM bytes of the translation kernel from two counter runs of "
                         "--profile-far-only, written to --translate-out")
    ap.add_argument("--translate-out",
                    default=os.path.join(ROOT, "profiles", "k_translate_c2_sphere20480_traffic.json"))
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


NEAR_KERNEL = "k_near<float, false, false"
NEAR_KERNEL64 = "k_near<double, false, false"
CAL_BYTES = 512 * 2 ** 20
# near-field traffic records per precision (complex FP32, FP64)
TRAFFIC_FILES = {"mixed": os.path.join(ROOT, "profiles", "k_near_c2_sphere20480_traffic.json"),
                 "fp64": os.path.join(ROOT, "profiles", "k_near_fp64_c2_sphere20480_traffic.json")}


def kernel_source_hash():
    """Hash of the sources that define the near-field kernel; a traffic
    record measured on other sources is not used."""
    import hashlib
    h = hashlib.sha256()
    for f in ("near.hip", "device.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2312_00005_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summarize_counters(fetch_csv, write_csv, out, prec="mixed"):
    """Per-dispatch averages of FETCH_SIZE / WRITE_SIZE (KiB) for the
    near-field kernel of precision prec and for the calibration copy, and the
    HBM bytes per near-field launch scaled by the copy's measured/known ratio."""
    import csv
    kernel = NEAR_KERNEL if prec == "mixed" else NEAR_KERNEL64
    out = out or TRAFFIC_FILES[prec]

    def per_kernel(path, counter):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")

    def pick(d, pred):
        keys = [k for k in d if pred(k)]
        if not keys:
            raise SystemExit(f"no dispatch matched in {sorted(d)[:8]}")
        return max(keys, key=lambda k: max(d[k]))

    near_f = pick(fetch, lambda k: kernel in k)
    near_w = pick(write, lambda k: kernel in k)
    cal_f = pick(fetch, lambda k: "copy" in k.lower() or "elementwise" in k.lower())
    cal_w = pick(write, lambda k: "copy" in k.lower() or "elementwise" in k.lower())
    avg = lambda v: sum(v) / len(v)

    def rel(path):
        # the command lines record where the counter runs wrote, relative to
        # the repository when inside it
        r = os.path.relpath(os.path.abspath(path), ROOT)
        return path if r.startswith("..") else r

    fdir, wdir = rel(os.path.dirname(fetch_csv) or "."), rel(os.path.dirname(write_csv) or ".")
    f_scale = max(fetch[cal_f]) / CAL_BYTES
    w_scale = max(write[cal_w]) / CAL_BYTES
    pflag = "" if prec == "mixed" else " --profile-prec fp64"
    rec = {
        "kernel": kernel,
        "workload": "c2: 20480-triangle sphere, 3-level FMM, tight quadrature, "
                    + ("complex-FP32" if prec == "mixed" else "FP64") + " near field",
        "fetch_bytes_per_launch_raw": avg(fetch[near_f]),
        "write_bytes_per_launch_raw": avg(write[near_w]),
        "launches": len(fetch[near_f]),
        "calibration": {"kernel": cal_f, "known_bytes": CAL_BYTES,
                        "fetch_bytes": max(fetch[cal_f]), "write_bytes": max(write[cal_w]),
                        "fetch_scale": f_scale, "write_scale": w_scale},
        "hbm_bytes_per_launch": avg(fetch[near_f]) / f_scale + avg(write[near_w]) / w_scale,
        "source_sha256": kernel_source_hash(),
        "commands": [
            f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fdir} -o f -- "
            f"python bench.py --profile-near-only --steps 3 --warmup 1{pflag}",
            f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {wdir} -o w -- "
            f"python bench.py --profile-near-only --steps 3 --warmup 1{pflag}",
            f"python bench.py --summarize-counters {rel(fetch_csv)} {rel(write_csv)}{pflag}",
        ],
    }
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def measured_traffic(prec="mixed", workload="c2"):
    """HBM bytes per near-field launch from the traffic record of the c2
    workload (None for other workloads, or once the kernel sources changed)."""
    if workload != "c2":
        return None
    try:
        with open(TRAFFIC_FILES[prec]) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def summarize_translate(fetch_csv, write_csv, out, prec="mixed"):
    """FETCH_SIZE / WRITE_SIZE per translation launch of precision prec,
    grouped by grid (one group per tree level), scaled by what the same
    counters read for the calibration copy of known size."""
    import csv

    def per_dispatch(path, counter):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], r.get("Grid_Size", r.get("Grid_Size_X", "")))
                acc.setdefault(key, []).append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    cal = lambda d: max(max(v) for k, v in d.items() if "copy" in k[0].lower() or "elementwise" in k[0].lower())
    f_scale, w_scale = cal(fetch) / CAL_BYTES, cal(write) / CAL_BYTES
    avg = lambda v: sum(v) / len(v)
    groups = []
    kname = "k_translate<double" if prec == "fp64" else "k_translate<float"
    for key in sorted(k for k in fetch if kname in k[0]):
        fb = avg(fetch[key]) / f_scale
        wb = avg(write.get(key, [0.0])) / w_scale
        groups.append({"kernel": key[0].replace("bem::(anonymous namespace)::", "").split("(")[0],
                       "grid": key[1], "launches": len(fetch[key]),
                       "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb})
    rel = lambda p: (lambda r: p if r.startswith("..") else r)(os.path.relpath(os.path.abspath(p), ROOT))
    pflag = " --profile-prec fp64" if prec == "fp64" else ""
    rec = {"workload": "c2: 20480-triangle sphere, 3-level FMM, tight preset, "
                       + ("FP64 far field" if prec == "fp64" else "complex-FP32 far field"),
           "calibration": {"known_bytes": CAL_BYTES, "fetch_scale": f_scale, "write_scale": w_scale},
           "groups": sorted(groups, key=lambda g: -g["fetch_bytes_per_launch"]),
           "commands": [
               f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {rel(os.path.dirname(fetch_csv) or '.')} -o f -- "
               f"python bench.py --profile-far-only --steps 3 --warmup 1{pflag}",
               f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {rel(os.path.dirname(write_csv) or '.')} -o w -- "
               f"python bench.py --profile-far-only --steps 3 --warmup 1{pflag}",
               f"python bench.py --summarize-translate {rel(fetch_csv)} {rel(write_csv)}{pflag}"
               + (f" --translate-out {rel(out)}" if prec == "fp64" else "")]}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def summarize_valu(pmc_csv, out_md):
    """Per kernel (name, grid): dispatches, average duration (the dispatch's
    timestamps; counter runs serialise dispatches, so each ran alone), and
    per-dispatch averages of SQ_INSTS_VALU (wavefront VALU instructions),
    SQ_ACTIVE_INST_VALU, SQ_WAVES and GRBM_GUI_ACTIVE.  GRBM_GUI_ACTIVE is
    summed over the 8 XCDs, so GRBM_GUI_ACTIVE / 8 / duration is the clock the
    dispatch ran at.  A wave64 VALU instruction occupies its 16-lane SIMD for
    4 cycles and the chip has 1024 SIMDs, so the share of SIMD cycles that
    full-rate issue of the counted instructions needs is
    4 SQ_INSTS_VALU / (1024 x clock x duration) (quarter-rate transcendentals
    count once: a lower bound of the VALU pipe's occupancy)."""
    import csv
    acc = {}
    with open(pmc_csv) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].replace("bem::(anonymous namespace)::", "").split("(")[0]
            key = (name, r.get("Grid_Size", r.get("Grid_Size_X", "")))
            d = acc.setdefault(key, {}).setdefault(r["Dispatch_Id"], {})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            d["dur"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    rows = []
    for (name, grid), ds in acc.items():
        n = len(ds)
        avg = lambda c: sum(v.get(c, 0.0) for v in ds.values()) / n
        dur, ins, gui = avg("dur"), avg("SQ_INSTS_VALU"), avg("GRBM_GUI_ACTIVE")
        if dur <= 0 or gui <= 0:
            continue
        clk = gui / 8.0 / dur
        rows.append((dur * n, name, grid, n, dur, ins, avg("SQ_ACTIVE_INST_VALU"), avg("SQ_WAVES"), clk,
                     4.0 * ins / (1024.0 * clk * dur)))
    rows.sort(reverse=True)
    rel = lambda p: (lambda r: p if r.startswith("..") else r)(os.path.relpath(os.path.abspath(p), ROOT))
    with open(out_md, "w") as fh:
        fh.write("# VALU instruction counts per kernel\n\n")
        fh.write(f"From `{rel(pmc_csv)}`; summary by `python bench.py --summarize-valu {rel(pmc_csv)} "
                 f"{rel(out_md)}`.  Dispatches ran one at a time (counter collection); clock = "
                 "GRBM_GUI_ACTIVE / 8 XCDs / duration; VALU share = 4 SQ_INSTS_VALU / (1024 SIMDs x clock x "
                 "duration), the fraction of SIMD cycles that full-rate issue of the counted VALU instructions "
                 "needs.  The largest 25 kernels by total time (the run includes the autotuner's launch-shape "
                 "candidates).\n\n")
        fh.write("| kernel | grid | dispatches | avg duration (us) | SQ_INSTS_VALU | SQ_ACTIVE_INST_VALU | SQ_WAVES "
                 "| clock (GHz) | VALU share |\n|---|---:|---:|---:|---:|---:|---:|---:|---:|\n")
        for _, name, grid, n, dur, ins, act, waves, clk, share in rows[:25]:
            fh.write(f"| `{name}` | {grid} | {n} | {dur * 1e6:.1f} | {ins:.4g} | {act:.4g} | {waves:.4g} | "
                     f"{clk / 1e9:.2f} | {share:.2f} |\n")
    print(open(out_md).read())


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.traffic_out,
                           args.profile_prec)
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu[0], args.summarize_valu[1])
        return
    if args.summarize_translate:
        summarize_translate(args.summarize_translate[0], args.summarize_translate[1], args.translate_out,
                            args.profile_prec)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(frequency sharding across GPUs is a design note only).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    from paper_2312_00005_amd import bemfmm

    wl = WORKLOADS[args.workload]
    if args.profile_far_direct:
        return profile_far_direct(args)
    if wl.get("sweep"):
        return run_sweep(args, wl)
    src = None
    if wl["mesh"][0] == "graded":
        nodes, tris, apex, apex_n = synth.graded_ellipsoid_bump()
        src = tuple(apex + 1e-3 * apex_n)
    else:
        nodes, tris = synth.icosphere(wl["mesh"][1])
    N = len(tris)
    if "k" in wl:
        k = wl["k"]
    else:
        k = 2 * math.pi / (wl["elems_per_wavelength"] * synth.mean_edge_length(nodes, tris))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    kw = dict(use_fmm=wl["use_fmm"])
    if wl["use_fmm"]:
        kw.update(levels=wl["levels"], leaf_size=wl["leaf_size"])
    mesh = bemfmm.Mesh(nodes, tris, wl["preset"], **kw)
    t_mesh = time.perf_counter() - t0
    log(f"mesh N={N} built in {t_mesh:.2f}s: {mesh.stats()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh.set_problem(k)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tune = mesh.autotune()
    log(f"launch shapes {tune}")
    stats = mesh.stats()
    x = torch.from_numpy(synth.complex_normal(N, seed=4)).to("cuda")
    y = torch.empty_like(x)
    if args.profile_near_only or args.profile_far_only:
        for _ in range(args.warmup + args.steps):
            mesh.apply_part(x, 2 if args.profile_far_only else 1, prec=args.profile_prec, out=y)
        src = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"profiled {args.warmup + args.steps} {'far' if args.profile_far_only else 'near'}-field "
            f"applications and one {CAL_BYTES} B copy")
        return

    # the stream every kernel of an application is enqueued on (near field,
    # permutations and the final sum; the far field forks from and joins it),
    # so events recorded on it bracket whole launches
    def timed(fn, steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / steps

    res = {}
    for prec in ("fp64", "mixed"):
        for _ in range(args.warmup):
            mesh.apply(x, prec=prec, out=y)
        t_full = timed(lambda: mesh.apply(x, prec=prec, out=y), args.steps)
        t_near = timed(lambda: mesh.apply_part(x, 1, prec=prec, out=y), args.steps)
        res[prec] = dict(t_full=t_full, t_near=t_near)
        log(f"{prec}: matvec {t_full * 1e3:.3f} ms, near part {t_near * 1e3:.3f} ms")
    golden = load_golden(args.workload, N, k)
    acc = {}
    if golden is not None:
        acc["operator_rel_l2"] = {}
        for prec in ("fp64", "mixed"):
            yv = mesh.apply(x, prec=prec).cpu().numpy()
            acc["operator_rel_l2"][prec] = rel_l2(yv, golden["y_ax"])
        log(f"operator vs oracle (dense, converged quadrature): {acc['operator_rel_l2']}")
    solves = {}
    if not args.no_solve:
        for prec in ("mixed", "fp64"):
            o = bemfmm.bem_options_default(wl["preset"])
            o.use_fmm = wl["use_fmm"]
            if wl["use_fmm"]:
                o.levels = wl["levels"]
                o.leaf_size = wl["leaf_size"]
            o.precision = bemfmm.BEM_PREC_MIXED if prec == "mixed" else bemfmm.BEM_PREC_FP64
            o.gmres_tol = SOLVE_TOL
            ms = bemfmm.Mesh(nodes, tris, o)
            # one problem at a nearby wavenumber first: the device buffers of the
            # per-frequency state are allocated once per mesh, as in a sweep;
            # the launch shapes are tuned once per mesh there too
            ms.set_problem(k * 1.01)
            ms.autotune()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ms.set_problem(k)
            if wl.get("source") == "point":
                rhs = ms.rhs_point_source(src)
            else:
                rhs = ms.rhs_plane_wave((0.0, 0.0, 1.0))
            p, _, info = ms.solve(rhs)
            torch.cuda.synchronize()
            solves[prec] = dict(seconds=time.perf_counter() - t0, iterations=info["iterations"],
                                refinements=info["refinements"], rel_residual=info["rel_residual"],
                                L=info["L"])
            if golden is not None:
                pv = p.cpu().numpy()
                ref = golden["p_lu"]
                solves[prec]["pressure_rel_l2_vs_oracle_lu"] = rel_l2(pv, ref)
                solves[prec]["pressure_max_rel_vs_oracle_lu"] = float(np.max(np.abs(pv - ref)) / np.max(np.abs(ref)))
            log(f"{prec}: solve {solves[prec]}")
            ms.close()
    if golden is not None and solves:
        acc["pressure_rel_l2"] = {p_: solves[p_]["pressure_rel_l2_vs_oracle_lu"] for p_ in solves}
        acc["pressure_max_rel"] = {p_: solves[p_]["pressure_max_rel_vs_oracle_lu"] for p_ in solves}
        acc["tolerance"] = {"fp64": 1e-5, "mixed": 1e-3}
        acc["oracle"] = ("dense N x N operator assembled by the CPU oracle with converged quadrature "
                         "(order tolerance 1e-11), LU solution (tests/golden/c2_sphere20480.npz, written by "
                         "tests/golden/make_c2_golden.py)")

    # headline: the FP64 (complex128) whole-operator application
    t_step = res["fp64"]["t_full"]
    value = N * N / t_step
    pts = stats["quad_points"]
    near_flops = pts * FLOPS_PER_POINT
    achieved64 = near_flops / res["fp64"]["t_near"] / 1e12
    achieved32 = near_flops / res["mixed"]["t_near"] / 1e12
    out = {
        "metric": "FMM matvec element-interactions/s and GMRES solve s/frequency, mixed vs FP64",
        "value": value,
        "unit": "element-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128",
        "data": "synthetic (seeded mesh and complex-normal vector)",
        "config": {"workload": f"{args.workload}: "
                   + ("graded ellipsoid with bump" if src is not None else "rigid sphere")
                   + f" N={N}, k={k:.4f}, "
                   + (f"{wl['levels']}-level FMM leaf~{wl['leaf_size']}" if wl["use_fmm"] else "all pairs direct")
                   + f", preset {wl['preset']} (coupling gamma = -i/k), FP64 operator",
                   "n_elements": N, "k": k, "preset": wl["preset"], "coupling": "-i/k"},
        "mixed": {"value": N * N / res["mixed"]["t_full"], "ms_per_step": res["mixed"]["t_full"] * 1e3,
                  "dtype": "complex64 operator (FP64 self terms, Krylov vectors and refinement)",
                  "roofline": {"bound": "alu", "kernel": NEAR_KERNEL, "achieved": achieved32,
                               "peak": PEAK_TFLOPS["fp32_packed"], "unit": "TFLOP/s",
                               "frac": achieved32 / PEAK_TFLOPS["fp32_packed"],
                               "peak_unpacked": PEAK_TFLOPS["fp32"],
                               "frac_unpacked": achieved32 / PEAK_TFLOPS["fp32"],
                               "traffic": measured_traffic("mixed", args.workload)}},
        "mixed_speedup_over_fp64": res["fp64"]["t_full"] / res["mixed"]["t_full"],
        "accuracy": acc,
        "near_ms": {p_: res[p_]["t_near"] * 1e3 for p_ in res},
        "near_quad_points": pts,
        "setup_s": {"mesh": t_mesh, "per_frequency": t_setup},
        "launch_shapes": tune,
        "solve_s_per_frequency": {p_: solves[p_]["seconds"] for p_ in solves},
        "solve": solves,
        "roofline": {"bound": "alu", "kernel": NEAR_KERNEL64, "achieved": achieved64,
                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s", "frac": achieved64 / PEAK_TFLOPS["fp64"],
                     "traffic": measured_traffic("fp64", args.workload),
                     "flops_per_launch": near_flops, "flops_per_point": FLOPS_PER_POINT,
                     "flops_per_point_direct": FLOPS_PER_POINT_DIRECT,
                     "frac_at_direct_count": achieved64 * FLOPS_PER_POINT_DIRECT / FLOPS_PER_POINT
                     / PEAK_TFLOPS["fp64"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nodes, tris, k, wl["preset"], args.cpu_seconds,
                                           mesh_spec=wl["mesh"])
    print(json.dumps(out), flush=True)


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


GOLDEN = {"c2": os.path.join(ROOT, "tests", "golden", "c2_sphere20480.npz")}


def load_golden(workload, N, k):
    """Stored oracle results for the workload (dense operator applied to the
    seed-4 vector, LU solution of the plane-wave problem), or None."""
    import numpy as np
    path = GOLDEN.get(workload)
    if path is None or not os.path.exists(path):
        return None
    z = np.load(path)
    if int(z["N"]) != N or abs(float(z["k"]) - k) > 1e-12 * k:
        raise SystemExit(f"{path} holds another workload (N={int(z['N'])}, k={float(z['k'])})")
    return {"y_ax": z["y_ax"], "p_lu": z["p_lu"]}


def profile_far_direct(args):
    """Direct far-field applications alone on the c4 mesh, for counter runs."""
    import torch
    import synth
    from paper_2312_00005_amd import bemfmm
    from paper_2312_00005_amd.sweep import wavenumbers

    nodes, tris = synth.geodesic_sphere(WORKLOADS["c4"]["mesh"][1])
    torch.cuda.set_device(0)
    m = bemfmm.Mesh(nodes, tris, WORKLOADS["c4"]["preset"], use_fmm=1, levels=4, leaf_size=32, far_direct=1,
                    far_rows=args.far_rows)
    m.set_problem(wavenumbers([9382.3])[0])
    x = torch.from_numpy(synth.complex_normal(len(tris), seed=4)).to("cuda")
    y = torch.empty_like(x)
    for _ in range(args.warmup + args.steps):
        m.apply_part(x, 2, prec=args.profile_prec, out=y)
    src = torch.ones(CAL_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"profiled {args.warmup + args.steps} direct far-field applications ({args.profile_prec}, far_rows "
        f"{args.far_rows}) and one {CAL_BYTES} B copy")
    m.close()


def run_sweep(args, wl):
    """One pass of the whole sweep: 64 frequencies, each set up and solved
    (mixed precision, GMRES tolerance 1e-6) with the method chosen for it."""
    import numpy as np
    import torch
    import synth
    from paper_2312_00005_amd import sweep

    nodes, tris = synth.geodesic_sphere(wl["mesh"][1])
    N = len(tris)
    freqs = [100.0 * 200.0 ** (i / 63.0) for i in range(64)]
    torch.cuda.set_device(0)
    S = sweep.FrequencySweep(nodes, tris, freqs, preset=wl["preset"], depths=(4, 3, 2), leaf_size=32,
                             streams=args.streams, memory_budget=48e9)
    log(f"sweep N={N}: methods {S.methods}")
    results, tot = S.run(keep_solutions=False)
    matvecs = sum(r["info"]["iterations"] + 2 * r["info"]["refinements"] + 1 for r in results)
    solve_time = tot["wall_s"] - tot["mesh_setup_s"]
    per = [{"f": round(r["f"], 1), "method": f"{r['method'][0]}{r['method'][1]}",
            "it": r["info"]["iterations"], "ref": r["info"]["refinements"], "res": r["info"]["rel_residual"],
            "s": round(r["seconds"], 4),
            "setup_s": round(r["setup_seconds"], 4)}
           for r in results]
    n_direct = sum(1 for r in results if r["method"][0] == "direct")
    n_fmm32 = sum(1 for r in results if r["method"][0] == "fmm32")
    out = {
        "metric": "FMM matvec element-interactions/s and GMRES solve s/frequency, mixed vs FP64",
        "value": N * N * matvecs / solve_time,
        "unit": "element-interactions/s",
        "n_gpus": 1, "steps": len(freqs), "warmup": 0,
        "ms_per_step": tot["wall_s"] / len(freqs) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (fp32 operator; fp64 diagonal, Krylov and refinement)",
        "data": "synthetic (seeded geodesic sphere mesh)",
        "config": {"workload": f"c4: frequency sweep, rigid sphere N={N}, 64 frequencies 100 Hz - 20 kHz, "
                               f"per-frequency FMM depth 2-4, FP32 FMM with FP64 direct far field, or direct "
                               f"far field, {args.streams} streams",
                   "n_elements": N, "frequencies": len(freqs)},
        "solve_s_per_frequency": tot["wall_s"] / len(freqs),
        "solve_s_per_frequency_excluding_plans": solve_time / len(freqs),
        "sweep": {"wall_s": tot["wall_s"], "mesh_setup_s": tot["mesh_setup_s"], "probe_s": tot["probe_s"],
                  "probes": S.probes,
                  "plan_choice_s": tot["plan_choice_s"], "operator_applications": matvecs,
                  "direct_far_field_frequencies": n_direct,
                  "fp32_fmm_fp64_direct_frequencies": n_fmm32, "per_frequency": per},
    }
    print(json.dumps(out), flush=True)


def _oracle_rows_worker(task):
    """Worker process of the CPU baseline: assemble dense oracle rows (one
    host thread per process) and return the time taken."""
    subdiv, kind, k, pre, rows = task
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    import numpy as np
    import synth
    from oracle import operator as op
    from oracle.geometry import element_geometry
    from oracle.presets import preset
    if kind == "icosphere":
        nodes, tris = synth.icosphere(subdiv)
    elif kind == "geodesic":
        nodes, tris = synth.geodesic_sphere(subdiv)
    else:
        nodes, tris = synth.graded_ellipsoid_bump()[:2]
    g = element_geometry(nodes, tris)
    x = synth.complex_normal(len(tris), seed=4)
    t0 = time.perf_counter()
    y = op.rows(g, np.asarray(rows), k, p=preset(pre)) @ x
    return time.perf_counter() - t0, len(rows), complex(y[0])


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nodes, tris, k, pre, budget, mesh_spec=None):
    """The oracle timed on the host's own cores:
    (1) dense operator rows assembled by direct quadrature, one worker
        process per core (the oracle's assembly rate, extrapolated to all N
        rows);
    (2) the dense matvec (zgemv, BLAS threads = cores) of an assembled-size
        row block, extrapolated to N rows: N^2 / t_zgemv is the oracle's
        element-interactions/s, the value reported;
    (3) LU factor + solve (zgetrf / zgetrs) of an n x n complex block,
        extrapolated to N as (N/n)^3.
    Every extrapolation is labelled as such."""
    import multiprocessing as mp
    import numpy as np
    import scipy.linalg
    from threadpoolctl import threadpool_info, threadpool_limits
    N = len(tris)
    ncpu = os.cpu_count() or 1
    cores = max(1, min(ncpu, int(os.environ.get("OMP_NUM_THREADS") or ncpu)))
    rng = np.random.default_rng(7)
    # (1) assembly: a one-row probe sizes the sample to about budget/2 seconds
    ctx = mp.get_context("spawn")
    spec = mesh_spec
    with ctx.Pool(cores) as pool:
        t1, _, _ = pool.apply(_oracle_rows_worker, ((spec[1], spec[0], k, pre, [0]),))
        per = max(1, int(0.5 * budget / max(t1, 1e-4)))
        rows = rng.choice(N, min(N, per * cores), replace=False)
        chunks = [(spec[1], spec[0], k, pre, list(map(int, c))) for c in np.array_split(rows, cores) if len(c)]
        t0 = time.perf_counter()
        outs = pool.map(_oracle_rows_worker, chunks)
        t_asm = time.perf_counter() - t0
    asm_rate = len(rows) * N / t_asm
    # (2) zgemv on a dense block with the BLAS on every core
    nb = min(N, 4096)
    with threadpool_limits(cores):
        blas = [{k_: i.get(k_) for k_ in ("internal_api", "num_threads", "version")} for i in threadpool_info()]
        M = (rng.standard_normal((nb, N)) + 1j * rng.standard_normal((nb, N))).astype(np.complex128)
        xv = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            M @ xv
            ts.append(time.perf_counter() - t0)
        t_gemv = float(np.median(ts)) * N / nb
        del M
        # (3) LU on an n x n block
        n = min(N, 3072)
        B = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) + n * np.eye(n)
        t0 = time.perf_counter()
        lu = scipy.linalg.lu_factor(B, overwrite_a=True, check_finite=False)
        scipy.linalg.lu_solve(lu, np.ones(n, dtype=np.complex128), check_finite=False)
        t_lu = (time.perf_counter() - t0) * (N / n) ** 3
        del B, lu
    return {"value": N * N / t_gemv, "unit": "element-interactions/s", "cores": cores, "kind": "oracle",
            "sample": (f"dense zgemv of a {nb} x {N} complex128 block (median of 5, {cores} BLAS threads), "
                       f"extrapolated to the {N} x {N} matrix; assembly: {len(rows)} random rows of the {pre} "
                       f"operator by the numpy oracle in {len(chunks)} processes, {t_asm:.1f} s"),
            "cpu_model": _cpu_model(), "os_cpu_count": ncpu, "blas": blas,
            "zgemv_s_extrapolated": t_gemv,
            "assembly_element_interactions_per_s": asm_rate,
            "assembly_s_extrapolated": N * N / asm_rate,
            "lu_s_extrapolated": t_lu,
            "lu_block": n,
            "solve_s_per_frequency_extrapolated": N * N / asm_rate + t_lu}


if __name__ == "__main__":
    main()
