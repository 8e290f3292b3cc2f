"""Benchmark of the cooling source step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (default): 256^3 = 16,777,216 independent cells of the iid recipe
(paper_2505_08855_amd/workloads.py), tables 4 x 128^3 FP32 built on the GPU from
the closed forms, one backward-Euler (Newton) cooling step per timed step over
all cells with dt = 1e-3 r_g/c (M = 10 M_sun).  Inputs and outputs stay in HBM.
Prints one JSON line.

Roofline: algorithmic HBM bytes per step = 72 B per cell (read n_e, T_e, T_i,
B, H as FP64; write T_e', T_i', Q_rad, Q_cc as FP64) + one read of the four
tables; the status byte (1 B/cell) is counted too.  A step is one
rc_cool_step call (one launch).  Achieved = bytes / average step time from
HIP events on the launch stream; peak = 8 TB/s.
traffic: HBM bytes per step from rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
scaled by a plain 512 MiB copy's readings, taken from the committed counter
summary when it was measured on the current kernel sources (else null).

cpu_baseline: the oracle (oracle/, NumPy FP64, one process) timed on a seeded
sample of the same workload; the same run supplies the max relative error of
the GPU outputs on that sample.

precision: the storage-precision experiment on a sample of the spherical
workload with 64^3 tables: FP32 and bfloat16 residual storage, per-field
errors against the oracle's FP64 tables, and the throughput of each.

    python bench.py --counters FETCH_DIR WRITE_DIR
turns two rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE; each run
with --calibrate-copy) into the counter summary kept under profiles/.
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = 5 * 8 + 4 * 8 + 1      # state in, T', Q_rad, Q_cc out, status
COPY_BYTES = 64 << 23                   # the calibration copy: 512 MiB read and written
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "newton_iid256_t128_counters.md")
STEP_KERNELS = re.compile(r"k_step<0, rc::CellTab>")     # the Newton kernel (demangled name), FP32 tables


def source_hash():
    """Hash of the library sources and build flags (identifies the kernels)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2505_08855_amd", "csrc", "*.h*")))
    files += [os.path.join(ROOT, "include", "radcool.h"), os.path.join(ROOT, "paper_2505_08855_amd", "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counters(folder, counter):
    """{kernel name: [value per dispatch]} of one rocprofv3 --pmc output folder (KiB)."""
    out = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter:
                    out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def counters_summary(fetch_dir, write_dir):
    """Markdown summary of the FETCH_SIZE / WRITE_SIZE passes with the traffic record."""
    fetch = read_counters(fetch_dir, "FETCH_SIZE")
    write = read_counters(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the FETCH pass: run it with --calibrate-copy")
    # the 512 MiB copies are the largest copy dispatches (small uploads use the same kernel)
    f_copy = max(v for k in copy for v in fetch[k]) * 1024.0
    w_copy = max(v for k in copy if k in write for v in write[k]) * 1024.0
    f_scale, w_scale = COPY_BYTES / f_copy, COPY_BYTES / w_copy

    def per_step(table):
        first = [k for k in table if STEP_KERNELS.search(k)]
        steps = len(table[first[0]]) if first else 0
        total = sum(sum(v) for k, v in table.items() if STEP_KERNELS.search(k)) * 1024.0
        return total / max(steps, 1), steps

    f_step, nf = per_step(fetch)
    w_step, nw = per_step(write)
    rec = {"source_hash": source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "fetch_bytes_per_step": f_step * f_scale, "write_bytes_per_step": w_step * w_scale,
           "traffic_bytes_per_step": f_step * f_scale + w_step * w_scale, "steps_counted": [nf, nw]}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch |", "|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, []), write.get(k, [])
        lines.append("| %s | %d | %.6g | %.6g |" % (k[:90], max(len(fv), len(wv)), np.mean(fv) if fv else float("nan"),
                                                   np.mean(wv) if wv else float("nan")))
    print("\n".join(lines))
    print()
    print("Calibration (512 MiB device copy): FETCH_SIZE x %.4f, WRITE_SIZE x %.4f." % (f_scale, w_scale))
    print("Per Newton step (all its launches): FETCH %.4g B, WRITE %.4g B, traffic %.4g B." %
          (rec["fetch_bytes_per_step"], rec["write_bytes_per_step"], rec["traffic_bytes_per_step"]))
    print()
    print("traffic-record: " + json.dumps(rec))


def measured_traffic():
    """Traffic per step from the committed counter summary, if it matches these sources."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            m = re.search(r"^traffic-record: (\{.*\})$", fh.read(), re.M)
    except OSError:
        return None
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec["traffic_bytes_per_step"] if rec.get("source_hash") == source_hash() else None


def measured_valu():
    """(VALU instructions per wavefront, wavefronts) of the Newton kernel from the
    committed counter summary, if it matches these sources."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"^traffic-record: (\{.*\})$", text, re.M)
    if not m or json.loads(m.group(1)).get("source_hash") != source_hash():
        return None
    per = re.search(r"^\| SQ_INSTS_VALU per wave \| ([0-9,.]+) \|", text, re.M)
    waves = re.search(r"^\| SQ_WAVES \| ([0-9,]+) \|", text, re.M)
    if not per or not waves:
        return None
    return float(per.group(1).replace(",", "")), float(waves.group(1).replace(",", ""))


def valu_roofline(ms):
    got = measured_valu()
    if got is None:
        return None
    per_wave, waves = got
    achieved = per_wave * waves / (ms * 1e-3) / 1e9
    peak = 1024 * 2.4e9 / 4 / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "G wave64 VALU instructions/s",
            "frac": achieved / peak, "source": os.path.relpath(TRAFFIC_SUMMARY, ROOT)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", choices=("iid256", "iid32", "sphere128", "blocks"), default="iid256")
    p.add_argument("--table-n", type=int, default=128)
    p.add_argument("--variant", default="auto")
    p.add_argument("--scheme", default="newton")
    p.add_argument("--passes", type=int, default=0, help="Newton step passes (0 = library choice, 1, 2)")
    p.add_argument("--sample", type=int, default=131072, help="cells in the cpu_baseline sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="first run a plain 512 MiB device copy (known HBM traffic) for counter calibration")
    p.add_argument("--no-precision", action="store_true")
    p.add_argument("--counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="summarise two rocprofv3 --pmc folders instead of benchmarking")
    return p.parse_args()


def cells_for(name):
    from paper_2505_08855_amd import workloads as W
    if name == "iid256":
        return W.workload(1), "iid cells 256^3 (n_e, T_e, T_i, B, H FP64 SoA), tables 4x128^3 FP32 read through their cell-blocked copy"
    if name == "iid32":
        return W.workload(0), "iid cells 32^3, tables 4x64^3 FP32 (cell-blocked copy)"
    return W.workload(2), "spherical-polar MAD-like profile 128^3, tables 4x64^3 FP32 (cell-blocked copy)"


def time_steps(R, torch, tables, state, dt, opts, out, steps, warmup):
    for _ in range(warmup):
        R.cool_step(tables, state, dt, opts, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        R.cool_step(tables, state, dt, opts, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall


def cpu_baseline(cells, idx, table_n, dt, gpu_out, scheme):
    """Oracle on the sample; returns (baseline dict, error dict)."""
    from oracle import step as S
    from oracle import tables as T
    from paper_2505_08855_amd import workloads as W
    spec = T.TableSpec.default(table_n)
    t0 = time.perf_counter()
    tabs = T.build_tables(spec)
    t_build = time.perf_counter() - t0
    ts = S.TableSet(spec, tabs)
    sample = [cells[f][idx] for f in W.FIELDS]
    t0 = time.perf_counter()
    if scheme == "explicit16":
        ref = S.step_explicit16(ts, *sample, dt)
    else:
        ref = S.step_be(ts, *sample, dt)
    t_step = time.perf_counter() - t0
    err = {}
    for g, r in (("Q_rad", "q_rad"), ("Q_cc", "q_cc"), ("T_e_new", "T_e_new"), ("T_i_new", "T_i_new")):
        a = gpu_out[g][idx]
        b = ref[r]
        err[g] = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
    base = {"value": idx.size / t_step / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d seeded cells of the same workload, %s step with the oracle's own FP64 %d^3 tables "
                      "(table build %.1f s not included, step %.1f s)" % (idx.size, scheme, table_n, t_build, t_step)}
    return base, err


def bench_blocks(args, R, W, torch, dev):
    """Batched form: uneven AMR blocks x accretion states through one captured,
    autotuned persistent launch (rc_plan)."""
    cells, blocks, _ = W.amr_blocks()
    n_states = 8
    dts = np.full(n_states, W.DT_DEFAULT)
    n = cells["n_e"].size
    state = {k: torch.from_numpy(cells[k]).to(dev) for k in W.FIELDS}
    del cells
    tables = R.Tables.build(R.default_spec(64))
    bdev, nb = R.blocks_to_device(blocks, dev)
    plan = R.Plan(tables, state, bdev, nb, dts, R.default_opts(scheme=args.scheme))
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    algo = BYTES_PER_CELL * n + 16 * 64 ** 3
    st = plan.out["status"].cpu().numpy()
    res = {"metric": "cooling Gcell-updates/s, % HBM roofline, max rel err vs FP64 oracle",
           "value": n / (ms * 1e-3) / 1e9, "unit": "Gcell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "4096 AMR blocks (8^3..32^3, mixed) x 8 accretion states, tables 4x64^3 FP32 (cell-blocked copy), "
                                  "one captured persistent launch", "cells": n, "blocks": nb,
                      "scheme": args.scheme, "plan": plan.info()},
           "roofline": {"bound": "hbm", "achieved": algo / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None},
           "status_counts": {str(int(v)): int(c) for v, c in zip(*np.unique(st, return_counts=True))}}
    print(json.dumps(res), flush=True)


def precision_report(R, torch, dev, W, dt, sample=16384):
    """Storage-precision experiment: FP32 and bfloat16 residual storage of 64^3
    tables on the spherical workload.  Errors of the GPU outputs on a seeded
    sample against the oracle's FP64 tables (rates and the Newton step), and
    the Newton throughput over the whole workload with each storage form."""
    from oracle import step as S
    from oracle import tables as T
    cells = W.workload(2)
    n = cells["n_e"].size
    idx = np.sort(np.random.default_rng(W.SEED_BASE + 2).choice(n, size=sample, replace=False))
    sub = [cells[f][idx] for f in W.FIELDS]
    spec = T.TableSpec.default(64)
    ts = S.TableSet(spec, T.build_tables(spec))
    ref = S.table_rates(ts, *sub)
    ref.update({k: v for k, v in S.step_be(ts, *sub, dt).items() if k in ("T_e_new", "T_i_new")})
    full = {k: torch.from_numpy(np.ascontiguousarray(cells[k])).to(dev) for k in W.FIELDS}
    part = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in zip(W.FIELDS, sub)}
    rep = {"workload": "spherical-polar profile 128^3 (%d cells); errors on a %d-cell seeded sample vs the "
                       "oracle's FP64 64^3 tables" % (n, sample)}
    for vd in ("f32", "bf16"):
        gt = R.Tables.build(R.default_spec(64, vd))
        o = R.cool_step(gt, part, dt, diagnostics=True)
        errs = {}
        for g, rk in (("Q_rad", "q_rad"), ("Q_cc", "q_cc"), ("Q_brem", "q_brem"), ("Q_syn", "q_syn"),
                      ("eta", "eta"), ("T_e_new", "T_e_new"), ("T_i_new", "T_i_new")):
            e = np.abs(o[g].cpu().numpy() - ref[rk]) / np.maximum(np.abs(ref[rk]), 1e-300)
            errs[g] = {"max": float(e.max()), "median": float(np.median(e))}
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
        out["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
        ms, _ = time_steps(R, torch, gt, full, dt, R.default_opts(), out, 10, 2)
        rep[vd] = {"table_bytes": (8 if vd == "bf16" else 16) * 64 ** 3 + (2 if vd == "bf16" else 4) * 64 ** 3,
                   "newton_ms": ms, "Gcell_per_s": n / (ms * 1e-3) / 1e9, "rel_err": errs}
    return rep


def accuracy_report(R, torch, dev):
    """Model accuracy of the two time integrators over one step: backward Euler
    (Newton) and 16 explicit substeps on the GPU with 64^3 tables, against the
    stored tight-tolerance ODE solution of 256 seeded cells (tests/golden)."""
    path = os.path.join(ROOT, "tests", "golden", "ode_reference_iid2m_256.json")
    with open(path) as fh:
        d = json.load(fh)
    cols = np.array(d["cells"], dtype=np.float64)
    state = {f: torch.from_numpy(np.ascontiguousarray(cols[:, k])).to(dev) for k, f in enumerate(d["fields"])}
    te_ode = np.array(d["T_e_ode"])
    change = np.abs(te_ode - cols[:, 1]) / cols[:, 1]
    gt = R.Tables.build(R.default_spec(64))
    rep = {"reference": d["description"]}
    bands = ((0.0, 1e-4), (1e-4, 1e-2), (1e-2, 0.3), (0.3, np.inf))
    for scheme in ("newton", "explicit16"):
        o = R.cool_step(gt, state, d["dt"], R.default_opts(scheme=scheme))
        e = np.abs(o["T_e_new"].cpu().numpy() - te_ode) / te_ode
        by = {}
        for lo, hi in bands:
            m = (change >= lo) & (change < hi)
            if m.any():
                by["|dT_e/T_e| in [%g, %g)" % (lo, hi)] = {"cells": int(m.sum()), "median": float(np.median(e[m])),
                                                         "max": float(e[m].max())}
        rep[scheme] = {"T_e_rel_err_median": float(np.median(e)), "T_e_rel_err_max": float(e.max()),
                       "by_change": by}
    return rep


def main():
    args = parse()
    if args.counters:
        return counters_summary(*args.counters)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the cooling step shards trivially by cells; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2505_08855_amd import radcool as R
    from paper_2505_08855_amd import workloads as W
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.workload == "blocks":
        return bench_blocks(args, R, W, torch, dev)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)    # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cells, desc = cells_for(args.workload)
    table_n = args.table_n if args.workload == "iid256" else 64
    n = cells["n_e"].size
    state = {k: torch.from_numpy(np.ascontiguousarray(cells[k])).to(dev) for k in W.FIELDS}
    dt = W.DT_DEFAULT
    t0 = time.perf_counter()
    tables = R.Tables.build(R.default_spec(table_n))
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
    out["status"] = torch.empty(n, dtype=torch.uint8, device=dev)
    opts = R.default_opts(variant=args.variant, scheme=args.scheme, passes=args.passes)
    ms, wall = time_steps(R, torch, tables, state, dt, opts, out, args.steps, args.warmup)
    table_bytes = 4 * 4 * table_n ** 3
    algo_bytes = BYTES_PER_CELL * n + table_bytes
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    value = n / (ms * 1e-3) / 1e9
    status = out["status"].cpu().numpy()
    res = {
        "metric": "cooling Gcell-updates/s, % HBM roofline, max rel err vs FP64 oracle",
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": n, "scheme": args.scheme, "variant": args.variant,
                   "table_n": table_n, "dt_s": dt, "T_floor_K": opts.T_floor},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if (args.workload == "iid256" and table_n == 128 and
                                                       args.scheme == "newton" and args.variant == "auto") else None},
        "table_build_s": t_build,
        # the Newton kernel is bound by FP64 vector issue, not HBM: the VALU
        # issue rate against the chip's (1024 SIMDs, one wave64 instruction per
        # 4 cycles at 2.4 GHz), from the committed SQ counters of this kernel
        "roofline_valu": valu_roofline(ms) if (args.workload == "iid256" and table_n == 128 and
                                                args.scheme == "newton" and args.variant == "auto") else None,
        "status_counts": {str(int(v)): int(c) for v, c in zip(*np.unique(status, return_counts=True))},
    }
    if not args.no_variants:
        var = {}
        for name, kw, steps in (("newton_block256", dict(block=256), 3),
                                ("rates", dict(scheme="rates"), 5),
                                ("explicit16", dict(scheme="explicit16"), 3),
                                ("rates_direct", dict(scheme="rates", variant="direct"), 1),
                                ("newton_global", dict(variant="global"), 3),
                                ("rates_global", dict(scheme="rates", variant="global"), 5),
                                ("newton_lds", dict(variant="lds"), 3),
                                ("rates_lds", dict(scheme="rates", variant="lds"), 5)):
            o = R.default_opts(**kw)
            try:
                vms, _ = time_steps(R, torch, tables, state, dt, o, out, steps, 1)
                var[name] = {"ms": vms, "Gcell_per_s": n / (vms * 1e-3) / 1e9}
            except R.RadcoolError as e:
                var[name] = {"error": str(e)}
        # the upstream inputs and the radiation-pressure correction over the same
        # cell count: elementwise kernels, 48 and 33 algorithmic bytes per cell
        rng = torch.Generator(device=dev).manual_seed(W.SEED_BASE)
        prims = {"rho": torch.rand(n, dtype=torch.float64, device=dev, generator=rng) * 1e-8 + 1e-12,
                 "r": torch.rand(n, dtype=torch.float64, device=dev, generator=rng) * 998.0 + 2.0}
        prims["P"] = prims["rho"] * 1e17
        prims["u"] = 1.5 * prims["P"]
        for name, fn, nbytes in (
                ("disk_inputs", lambda: R.disk_inputs(prims), 48),
                ("rad_pressure_correction", lambda: R.rad_pressure_correction(state["n_e"], state["T_e"],
                                                                             state["H"]), 33)):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fn()
            e1.record()
            torch.cuda.synchronize()
            vms = e0.elapsed_time(e1) / 5
            var[name] = {"ms": vms, "Gcell_per_s": n / (vms * 1e-3) / 1e9,
                         "hbm_frac": nbytes * n / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del prims
        # downstream coupling: the step's cooling applied to the gas
        # energy-momentum in place; reads n_e, T_e, T_i, T_e', T_i', u_mu (4),
        # sqrt(-g), U_mu (4) and writes U_mu (4) and lambda: 152 B per cell
        R.cool_step(tables, state, dt, opts, out=out)
        z0 = torch.zeros(n, dtype=torch.float64, device=dev)
        u_cov = [-torch.ones(n, dtype=torch.float64, device=dev), z0, z0.clone(), z0.clone()]
        U_cons = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(4)]
        sqrt_g = torch.ones(n, dtype=torch.float64, device=dev)
        fwd = {"T_e_new": out["T_e_new"], "T_i_new": out["T_i_new"]}
        lam = R.apply_cooling(state, fwd, u_cov, U_cons, dt, sqrt_g=sqrt_g)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            R.apply_cooling(state, fwd, u_cov, U_cons, dt, sqrt_g=sqrt_g)
        e1.record()
        torch.cuda.synchronize()
        vms = e0.elapsed_time(e1) / 5
        var["apply_cooling"] = {"ms": vms, "Gcell_per_s": n / (vms * 1e-3) / 1e9,
                                "hbm_frac": 152 * n / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del z0, u_cov, U_cons, sqrt_g, lam, fwd
        # the paper's own layout: log2 Q_total on a 4-D grid of 100^4 nodes over
        # the paper's ranges, read by 4-D interpolation (16 corners); speed
        # against the rates kernel of the 3-D column tables (which also
        # produces Q_cc), and model error of both layouts against the closed
        # forms (DIRECT variant) on a sample of the same cells
        t4 = R.Table4D.build()
        q4, _ = R.rates4d(t4, state, opts.T_floor)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            q4, _ = R.rates4d(t4, state, opts.T_floor)
        e1.record()
        torch.cuda.synchronize()
        vms = e0.elapsed_time(e1) / 5
        m = min(n, 1 << 20)
        sub = {k: v[:m] for k, v in state.items()}
        qd = R.cool_step(tables, sub, dt, R.default_opts(scheme="rates", variant="direct"))["Q_rad"]
        q3 = R.cool_step(tables, sub, dt, R.default_opts(scheme="rates"))["Q_rad"]
        on = qd > 0
        err = {}
        for name, qq in (("table4d_100", q4[:m]), ("tables3d_%d" % table_n, q3)):
            e = ((qq[on] - qd[on]).abs() / qd[on]).cpu().numpy()
            err[name] = {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)), "max": float(e.max())}
        var["rates_table4d"] = {"ms": vms, "Gcell_per_s": n / (vms * 1e-3) / 1e9,
                                "table_bytes": 4 * int(np.prod(list(R.paper_axes4().n))),
                                "q_rad_rel_err_vs_closed_forms": err, "sample_cells": m}
        t4.destroy()
        del q4, qd, q3, sub
        # the same step reading bfloat16-stored tables (half the table bytes)
        t16 = R.Tables.build(R.default_spec(table_n, "bf16"))
        vms, _ = time_steps(R, torch, t16, state, dt, opts, out, 3, 1)
        var["newton_bf16_tables"] = {"ms": vms, "Gcell_per_s": n / (vms * 1e-3) / 1e9}
        t16.destroy()
        # differentiation form: adjoint of the Newton step (cotangents of the
        # radiated energy) with table-entry gradients
        R.cool_step(tables, state, dt, opts, out=out)
        c = 1.5 * state["n_e"] * 1.380649e-16
        cot = {"T_e_new": -c, "T_i_new": -c}
        _, nv = tables.info()
        tg = torch.zeros(nv, dtype=torch.float64, device=dev)
        fwd = {"T_e_new": out["T_e_new"], "T_i_new": out["T_i_new"], "status": out["status"]}
        R.cool_step_backward(tables, state, dt, fwd, cot, opts, table_grad=tg)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            R.cool_step_backward(tables, state, dt, fwd, cot, opts, table_grad=tg)
        e1.record()
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / 3
        var["backward_newton"] = {"ms": bms, "Gcell_per_s": n / (bms * 1e-3) / 1e9}
        del tg, c, cot
        res["variants"] = var
        # the timed configuration again, so that the outputs below are its own
        R.cool_step(tables, state, dt, opts, out=out)
        torch.cuda.synchronize()
    if not args.no_precision:
        res["precision"] = precision_report(R, torch, dev, W, dt)
        res["accuracy"] = accuracy_report(R, torch, dev)
    if not args.no_cpu_baseline:
        gpu_out = {k: out[k].cpu().numpy() for k in ("T_e_new", "T_i_new", "Q_rad", "Q_cc")}
        rng = np.random.default_rng(20250513)
        idx = np.sort(rng.choice(n, size=min(args.sample, n), replace=False))
        base, err = cpu_baseline(cells, idx, table_n, dt, gpu_out, args.scheme)
        res["cpu_baseline"] = base
        res["max_rel_err_vs_oracle"] = err
        res["max_rel_err_note"] = ("rates: GPU FP32-stored tables vs oracle FP64 tables (tolerance 1e-5); "
                                   "T': same, so FP32 table rounding is amplified by stiffness; the 1e-9 "
                                   "energy tier on identical tables is a GPU test")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
