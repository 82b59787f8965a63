#!/usr/bin/env python3
"""Benchmark of the local-FFT PSATD field push on one MI355X.

Workload (default): the 256^3 periodic grid cut into 4x4x4 subdomains of 64^3,
16 guard cells per side (local FFTs of 96^3), order p = 32, dt = 0.5, c = 1.
The FP32 precision path (FP32 state and FFT, FP64 coefficients and update) is
the headline; the FP64 plain path runs the same input for the "FP32 vs FP64
plain" comparison.  Both run K steps from the same initial state, replayed from
a captured HIP graph, inputs resident in HBM.  Prints ONE JSON line.

Synthetic input (seeded): one Gaussian current pulse (sigma = 8 cells), plus a
background of 8 vacuum plane waves (|m_u| <= 8, amplitude 0.1, polarisation
orthogonal to the grid wave vector).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PSATD cell-updates/s at 1 GPU (FP32/MFMA vs FP64 plain) at <=1e-5 rel L2; % HBM BW"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1707_08500_amd", "csrc")
PHASE_KERNEL = {"fft_xy_fwd": "k_fwd_xy", "z_update": "k_z_update", "fft_xy_inv": "k_inv_xy",
                "exchange_EB": "k_fill", "exchange_J": "k_fill"}
COPY_BYTES = 1 << 30  # the calibration copy: 2^28 floats read and written

WORKLOADS = {
    # name: grid, boxes per axis, guard, order p, dt
    "cfg2": dict(N=(256, 256, 256), nbox=(4, 4, 4), guard=16, p=32, dt=0.5,
                 desc="256^3 grid, 4x4x4 subdomains of 64^3, 16 guards (local FFT 96^3), p=32, dt=0.5, c=1"),
    "cfg4": dict(N=(512, 512, 256), nbox=None, guard=None, p=64, dt=0.5,
                 desc="512x512x256 grid cut into uneven subdomains (edges from {48,64,80,96}, guards from "
                      "{8,16,32}), p=64, dt=0.5, c=1"),
    "cfg5": dict(N=(1024, 1024, 512), nbox=(8, 8, 4), guard=24, p=100, dt=0.5,
                 desc="1024x1024x512 grid, 8x8x4 subdomains of 128^3, 24 guards (local FFT 176^3), p=100, dt=0.5, c=1"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(N, d, case):
    import numpy as np
    from paper_1707_08500_amd import synth
    J = synth.current_pulses(N, d, case=case, count=1, sigma=8.0)
    E = np.zeros_like(J)
    B = np.zeros_like(J)
    ms, amps, phases = synth.wave_parameters(case=case, count=8, mmax=8)
    for m, a, ph in zip(ms, amps, phases):
        k = 2 * np.pi * m / np.array(N, dtype=float)
        kh = k / np.linalg.norm(k)
        a = a - (a @ kh) * kh
        a = 0.1 * a / np.linalg.norm(a)
        E += synth.plane_wave(N, m, a, ph)
        B += synth.plane_wave(N, m, np.cross(kh, a), ph)
    return E, B, J


def algorithmic_bytes(plan, dec_lo, dec_n, dec_g, sb):
    """Bytes each phase must move at least once, per launch (one step).  The z
    pass reads 9 complex fields at every k-point and writes the 6 results on the
    interior z-planes only (all the inverse pass reads).  The FP32 forms add
    increments, so their inverse pass reads and writes the interior cells.  With
    the fused E,B exchange the inverse pass also writes every guard copy (no
    read), and the exchange phase moves nothing."""
    import numpy as np
    fused = bool(plan.tuning()["fuse_eb"])
    inc = plan.precision != "f64"
    out = dict(exchange_J=0, fft_xy_fwd=0, z_update=0, fft_xy_inv=0, exchange_EB=0)
    kpoints = 0
    for s in range(len(dec_lo)):
        (px, py, pz), _ = plan.layout(s)
        nx, ny, nz = (int(v) for v in dec_n[s])
        V = px * py * pz
        H = px // 2 + 1
        guard = V - nx * ny * nz
        out["exchange_J"] += guard * 3 * 2 * sb
        out["fft_xy_fwd"] += 9 * V * sb + 9 * pz * py * H * 2 * sb
        out["z_update"] += (9 * pz + 6 * nz) * py * H * 2 * sb
        out["fft_xy_inv"] += 6 * nz * py * H * 2 * sb + (2 if inc else 1) * 6 * nz * ny * nx * sb
        if fused:
            out["fft_xy_inv"] += guard * 6 * sb
        else:
            out["exchange_EB"] += guard * 6 * 2 * sb
        kpoints += pz * py * H
    return out, kpoints


def timed_run(plan, E, B, J, glob_init, steps, warmup):
    import torch
    for F, pad in zip(glob_init, (E, B, J)):
        plan.scatter(F, pad)
    if warmup:
        plan.run(E, B, J, warmup)
    for F, pad in zip(glob_init, (E, B, J)):  # reset to the initial state
        plan.scatter(F, pad)
    plan.run(E, B, J, steps)  # capture outside the timed region
    for F, pad in zip(glob_init, (E, B, J)):
        plan.scatter(F, pad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(E, B, J, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def source_digest():
    """sha256 over the kernel sources: HBM counters taken on other sources are stale."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp"))
                       + glob.glob(os.path.join(CSRC, "*.h"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_path(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")


def _pmc_rows(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter_collection.csv."""
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def summarize_pmc(fetch_csv, write_csv, workload, command):
    """HBM bytes per dispatch of every psatd kernel from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by the factor that makes the
    1 GiB calibration copy read and write exactly 1 GiB."""
    out = {}
    factors = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _pmc_rows(path, counter)
        # the calibration dispatches are the only ones outside the library that
        # move more than 256 MiB: the 1 GiB fill (writes) and the 1 GiB copies
        copies = [v for name, v in rows if "psatd" not in name and v > 0.25 * COPY_BYTES / 1024]
        if not copies:
            raise SystemExit(f"no 1 GiB calibration dispatch among the {counter} dispatches")
        factors[counter] = (COPY_BYTES / 1024) / (sum(copies) / len(copies))
        factors[counter + "_n"] = len(copies)
        per = {}
        for name, v in rows:
            short = name.split("(")[0].replace("void ", "").strip()
            base = short.split("<")[0].split("::")[-1]
            if base in PHASE_KERNEL.values() or base.startswith("k_"):
                per.setdefault(short, []).append(v)
        for short, vals in per.items():
            out.setdefault(short, {})[counter] = (sum(vals) / len(vals), len(vals))
    lines = [f"# HBM traffic per dispatch, workload {workload} (rocprofv3 --pmc, two passes)",
             f"# command: {command}",
             f"source_digest: {source_digest()}",
             f"copy_factor FETCH_SIZE: {factors['FETCH_SIZE']:.6f} "
             f"(from {factors['FETCH_SIZE_n']} calibration dispatches)",
             f"copy_factor WRITE_SIZE: {factors['WRITE_SIZE']:.6f} "
             f"(from {factors['WRITE_SIZE_n']} calibration dispatches)",
             "# kernel | dispatches | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | HBM bytes (scaled)"]
    for short, d in sorted(out.items()):
        fk, n = d.get("FETCH_SIZE", (0.0, 0))
        wk, _ = d.get("WRITE_SIZE", (0.0, 0))
        b = 1024 * (fk * factors["FETCH_SIZE"] + wk * factors["WRITE_SIZE"])
        lines.append(f"kernel {short} | {n} | {fk:.1f} | {wk:.1f} | {b:.0f}")
    return "\n".join(lines) + "\n"


def summarize_ktrace(stats_csv, bench_line, workload, command):
    """Per-kernel launch statistics from rocprofv3 --kernel-trace --stats, next to
    the per-phase times the same run measured with HIP events."""
    lines = [f"# rocprofv3 kernel statistics, workload {workload}",
             f"# command: {command}",
             f"source_digest: {source_digest()}",
             "# kernel | calls | average us | total ms | % of GPU time"]
    for r in csv.DictReader(open(stats_csv)):
        short = r["Name"].split("(")[0].replace("void ", "").strip()
        lines.append(f"{short} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {r['Percentage']}")
    if bench_line:
        d = json.loads(bench_line)
        lines.append("# the same run's bench line (FP32 path), per-phase ms from HIP events:")
        lines.append("phases_ms " + " ".join(f"{k}={v:.3f}" for k, v in d["phases_ms"].items()))
        lines.append(f"ms_per_step {d['ms_per_step']:.3f}")
    return "\n".join(lines) + "\n"


def summarize_mix(a_csv, b_csv, workload, command):
    """VALU instruction mix per dispatch of every psatd kernel from two
    rocprofv3 --pmc passes: SQ_INSTS_VALU, the F64 kinds, SQ_INSTS_LDS,
    SQ_INSTS_SALU and SQ_INSTS_VALU_INT32 in the first, the F32 kinds and
    SQ_INSTS_VALU_CVT in the second (wave instructions, mean over dispatches)."""
    per = {}
    for path in (a_csv, b_csv):
        for r in csv.DictReader(open(path)):
            if "psatd" not in r["Kernel_Name"]:
                continue
            short = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            per.setdefault(short, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    mean = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in per.items()}
    lines = [f"# VALU instruction mix per dispatch (wave instructions), workload {workload}, FP32 VALU form",
             f"# command: {command}",
             f"source_digest: {source_digest()}",
             "# kernel | VALU | INT32 | F32 (add+mul+fma) | F64 (add+mul+fma+trans) | CVT | other VALU | "
             "SALU | LDS"]
    for k in sorted(mean):
        d = mean[k]
        if "SQ_INSTS_VALU" not in d:
            continue
        v = d["SQ_INSTS_VALU"]
        i32 = d.get("SQ_INSTS_VALU_INT32", 0.0)
        f32 = sum(d.get(c, 0.0) for c in ("SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
                                           "SQ_INSTS_VALU_FMA_F32"))
        f64 = sum(d.get(c, 0.0) for c in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                                           "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64"))
        cvt = d.get("SQ_INSTS_VALU_CVT", 0.0)
        other = max(0.0, v - i32 - f32 - f64 - cvt)
        pct = (lambda x: f"{x:.3g} ({100 * x / v:.0f}%)") if v else (lambda x: f"{x:.3g}")
        lines.append(f"{k} | {v:.3g} | {pct(i32)} | {pct(f32)} | {pct(f64)} | {pct(cvt)} | {pct(other)} | "
                     f"{d.get('SQ_INSTS_SALU', 0.0):.3g} | {d.get('SQ_INSTS_LDS', 0.0):.3g}")
    return "\n".join(lines) + "\n"


SPL_OF = {"f32": 0, "bf16x3": 2, "bf16x6": 3}


def kernel_instance(phase, form, tuning):
    """The template instance (as the profiler prints it) that runs `phase` for
    the FP32 form `form` with launch shapes `tuning` (unsplit x/y passes)."""
    spl = SPL_OF[form]
    maxr = 16 if spl else tuning["max_radix"]
    if phase == "z_update":
        pb = tuning["z_pencils"]
        nt = 512 if pb == 4 else tuning["z_threads"]
        return f"psatd::k_z_update<float, {nt}, {pb}, true, {maxr}, {spl}>"
    if phase == "fft_xy_fwd":
        return f"psatd::k_fwd_xy<float, {tuning['xy_threads']}, {maxr}, {spl}>"
    if phase == "fft_xy_inv":
        return f"psatd::k_inv_xy<float, true, {tuning['xy_threads']}, {maxr}, {spl}>"
    return "psatd::k_fill<float>"


def read_traffic(workload, instance):
    """Scaled HBM bytes per dispatch of the kernel instance from the committed
    summary, or None when there is none or it was taken on other sources."""
    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    digest, found = None, None
    for line in open(path):
        if line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("kernel "):
            fields = [f.strip() for f in line[len("kernel "):].split("|")]
            if fields[0] == instance:
                found = float(fields[4])
    if digest != source_digest():
        return None
    return found


def cpu_baseline(N, d, lo, n, g, p, dt, E, B, J, budget_s=15.0):
    """The oracle as it stands, on a bounded sample of subdomains of the same
    workload (one local step each: local FFTs, update, inverse FFTs)."""
    import numpy as np
    from oracle import psatd_oracle as O
    dec = O.Decomposition(N, lo, n, g)

    def box(F, s):
        ix, iy, iz = dec.global_index(s)
        return F[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
    cells, t = 0, 0.0
    s = 0
    while t < budget_s and s < dec.nsub:
        e, b, j = box(E, s), box(B, s), box(J, s)
        t0 = time.perf_counter()
        O.step_global(e, b, j, d, p, 1.0, dt)
        t += time.perf_counter() - t0
        cells += int(np.prod(dec.n[s]))
        s += 1
    return dict(value=cells / t, unit="cell-updates/s", cores=O._WORKERS, kind="oracle",
                sample=f"{s} of {dec.nsub} subdomains, one local step each (FP64 scipy.fft, "
                       f"{O._WORKERS} workers), {t:.1f} s; the guard exchange is not timed")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-global", action="store_true", help="skip the PSATD-global comparison leg")
    ap.add_argument("--no-heat", action="store_true", help="skip the heat-equation leg")
    ap.add_argument("--precisions", default="f32,bf16x3,bf16x6",
                    help="FP32-state forms to time (comma list of f32, bf16x3, bf16x6)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--autotune", action="store_true",
                    help="time launch-shape candidates first (the defaults are the measured best for cfg2)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM-traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--pmc-command", default="", help="the profiled command, recorded in the summary")
    ap.add_argument("--summarize-ktrace", nargs=2, metavar=("KERNEL_STATS_CSV", "BENCH_LOG"),
                    help="print the kernel-statistics summary of a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-mix", nargs=2, metavar=("PASS_A_CSV", "PASS_B_CSV"),
                    help="print the VALU instruction-mix summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_pmc:
        text = summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload,
                             args.pmc_command)
        with open(traffic_path(args.workload), "w") as f:
            f.write(text)
        print(text, end="")
        return
    if args.summarize_ktrace:
        bench_line = ""
        for line in open(args.summarize_ktrace[1]):
            if line.startswith("{"):
                bench_line = line
        print(summarize_ktrace(args.summarize_ktrace[0], bench_line, args.workload, args.pmc_command),
              end="")
        return
    if args.summarize_mix:
        print(summarize_mix(args.summarize_mix[0], args.summarize_mix[1], args.workload, args.pmc_command),
              end="")
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the single-GPU kernel is the per-GPU share of a sharded run)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1707_08500_amd import psatd, synth

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] copy calibration: 3 x 1 GiB device copies")

    wl = WORKLOADS[args.workload]
    N, d = wl["N"], (1.0, 1.0, 1.0)
    if wl["nbox"] is None:
        lo, n, g = synth.uneven_decomposition(N, case=4)
    else:
        lo, n, g = synth.uniform_decomposition(N, wl["nbox"], wl["guard"])
    p, dt, c = wl["p"], wl["dt"], 1.0
    log(f"[bench] workload {args.workload}: {wl['desc']}")
    E0, B0, J0 = make_inputs(N, d, case=2)
    interior = N[0] * N[1] * N[2]

    FORMS = {"f32": "FP32 state, FP32 VALU radix FFT of increments, FP64 coefficients",
             "bf16x3": "FP32 state, radix-16 DFT stages as split-BF16 3-product MFMA GEMMs "
                       "(other stages VALU), FFT of increments, FP64 coefficients",
             "bf16x6": "FP32 state, radix-16 DFT stages as split-BF16 6-product MFMA GEMMs "
                       "(other stages VALU), FFT of increments, FP64 coefficients"}
    forms = [f.strip() for f in args.precisions.split(",") if f.strip()]
    for f in forms:
        if f not in FORMS:
            raise SystemExit(f"unknown FP32 form {f}")
    runs = forms + ([] if args.no_fp64 else ["f64"])
    results = {}
    finals = {}
    for prec in runs:
        dtype = torch.float64 if prec == "f64" else torch.float32
        plan = psatd.Plan(N, d, lo, n, g, p, dt, c, precision=prec)
        glob = [[torch.from_numpy(np.ascontiguousarray(F[a])).to("cuda", dtype).reshape(-1)
                 for a in range(3)] for F in (E0, B0, J0)]
        E, B, J = plan.empty_fields(), plan.empty_fields(), plan.empty_fields()
        if args.autotune:
            for F, pad in zip(glob, (E, B, J)):
                plan.scatter(F, pad)
            tuned_ms = plan.autotune(E, B, J, steps_per_trial=3)
            log(f"[bench] {prec}: autotuned {plan.tuning()} ({tuned_ms:.3f} ms/step in trials)")
        log(f"[bench] {prec}: {args.warmup} warmup + {args.steps} timed steps")
        t = timed_run(plan, E, B, J, glob, args.steps, args.warmup)
        padded = plan.field_elems
        results[prec] = dict(seconds=t, ms_per_step=1e3 * t / args.steps,
                             value=interior * args.steps / t,
                             padded_value=padded * args.steps / t, tuning=plan.tuning())
        outE = [torch.empty_like(x) for x in glob[0]]
        outB = [torch.empty_like(x) for x in glob[1]]
        plan.gather(E, outE)
        plan.gather(B, outB)
        torch.cuda.synchronize()
        finals[prec] = [x.double().cpu().numpy() for x in outE + outB]
        if prec != "f64":
            for F, pad in zip(glob, (E, B, J)):
                plan.scatter(F, pad)
            results[prec]["phases_ms"] = plan.run_profiled(E, B, J, args.profile_steps)
            results[prec]["algo_bytes"], _ = algorithmic_bytes(plan, lo, n, g, 4)
        log(f"[bench] {prec}: {results[prec]['ms_per_step']:.3f} ms/step, "
            f"{results[prec]['value'] / 1e9:.2f} G interior cell-updates/s")
        plan.close()
        del E, B, J, glob
        torch.cuda.empty_cache()

    # error of every FP32 form against the FP64 path after the same steps
    names = ["Ex", "Ey", "Ez", "Bx", "By", "Bz"]
    for prec in forms:
        if "f64" not in finals:
            break
        err = {}
        for i, name in enumerate(names):
            ref = finals["f64"][i]
            den = float(np.sqrt(np.sum(ref * ref)))
            err[name] = float(np.sqrt(np.sum((finals[prec][i] - ref) ** 2)) / (den if den else 1.0))
        results[prec]["rel_l2_vs_fp64"] = err
        results[prec]["rel_l2_vs_fp64_max"] = max(err.values())
    # headline: the fastest FP32 form within the 1e-5 gate (all forms when FP64 did not run)
    ok = [f for f in forms if results[f].get("rel_l2_vs_fp64_max", 0.0) <= 1e-5]
    head = max(ok or forms, key=lambda f: results[f]["value"])
    r32 = results[head]
    phases = r32["phases_ms"]
    dom = max(phases, key=phases.get)
    achieved = r32["algo_bytes"][dom] / (phases[dom] * 1e-3) / 1e9
    step_algo = sum(r32["algo_bytes"].values())
    bmin = 15 * 4 * sum(int(np.prod(n[s] + 2 * g[s])) for s in range(len(lo)))
    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"] + "; " + FORMS[head],
                   "global_batch": interior, "precision": head, "graph": True,
                   "tuning": r32["tuning"]},
        "padded_cell_updates_per_s": r32["padded_value"],
        "phases_ms": phases,
        "hbm_fraction_of_step": {
            "bmin_15_words": (bmin / (r32["ms_per_step"] * 1e-3)) / 1e9 / HBM_PEAK_GBS,
            "per_pass_algorithmic": (step_algo / (sum(phases.values()) * 1e-3)) / 1e9 / HBM_PEAK_GBS,
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "kernel_instance": kernel_instance(dom, head, r32["tuning"]),
                     "traffic": (read_traffic(args.workload, kernel_instance(dom, head, r32["tuning"]))
                                 if not r32["tuning"]["split_xy"] else None),
                     "algorithmic_bytes": r32["algo_bytes"][dom]},
        "fp32_forms": {f: {k: results[f][k] for k in ("value", "ms_per_step", "rel_l2_vs_fp64",
                                                      "rel_l2_vs_fp64_max", "phases_ms")
                           if k in results[f]} for f in forms},
    }
    if "f64" in results:
        r64 = results["f64"]
        out["fp64_plain"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                             "speedup_fp32_over_fp64": r32["value"] / r64["value"]}
        out["rel_l2_fp32_vs_fp64_gpu"] = r32["rel_l2_vs_fp64"]
        out["rel_l2_fp32_vs_fp64_gpu_max"] = r32["rel_l2_vs_fp64_max"]
    if not args.no_global:
        # PSATD-global: the same grid as one box without guards (one global 3D
        # FFT per step), same form, input and steps; the difference from the
        # local result is the method's truncation (a property, not a gate)
        log(f"[bench] PSATD-global {head}: {args.warmup} warmup + {args.steps} timed steps")
        plan = psatd.Plan(N, d, [[0, 0, 0]], [list(N)], [[0, 0, 0]], p, dt, c, precision=head)
        glob = [[torch.from_numpy(np.ascontiguousarray(F[a])).to("cuda", torch.float32).reshape(-1)
                 for a in range(3)] for F in (E0, B0, J0)]
        E, B, J = plan.empty_fields(), plan.empty_fields(), plan.empty_fields()
        t = timed_run(plan, E, B, J, glob, args.steps, args.warmup)
        outE = [torch.empty_like(x) for x in glob[0]]
        outB = [torch.empty_like(x) for x in glob[1]]
        plan.gather(E, outE)
        plan.gather(B, outB)
        torch.cuda.synchronize()
        gl = [x.double().cpu().numpy() for x in outE + outB]
        loc = finals[head]
        num = sum(float(np.sum((loc[i] - gl[i]) ** 2)) for i in range(6))
        den = sum(float(np.sum(gl[i] ** 2)) for i in range(6))
        out["psatd_global"] = {"ms_per_step": 1e3 * t / args.steps, "value": interior * args.steps / t,
                               "precision": head, "split_xy": plan.tuning()["split_xy"],
                               "rel_l2_local_vs_global": float(np.sqrt(num / den))}
        log(f"[bench] PSATD-global: {1e3 * t / args.steps:.3f} ms/step")
        plan.close()
        del E, B, J, glob
        torch.cuda.empty_cache()
    if not args.no_heat:
        # the same local-FFT push for the heat equation (one field, D = 0.1)
        log(f"[bench] heat equation {head}: {args.warmup} warmup + {args.steps} timed steps")
        plan = psatd.Plan(N, d, lo, n, g, p, dt, c, precision=head)
        glob = [torch.from_numpy(np.ascontiguousarray(E0[0])).to("cuda", torch.float32).reshape(-1)] * 3
        u = plan.empty_fields()
        plan.scatter(glob, u)
        plan.heat_run(u[0], 0.1, max(args.warmup, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.heat_run(u[0], 0.1, args.steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["heat_equation"] = {"ms_per_step": 1e3 * t / args.steps, "value": interior * args.steps / t,
                                "precision": head, "diffusivity": 0.1}
        log(f"[bench] heat equation: {1e3 * t / args.steps:.3f} ms/step")
        plan.close()
        del u, glob
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle, bounded sample)")
        out["cpu_baseline"] = cpu_baseline(N, d, lo, n, g, p, dt, E0, B0, J0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
