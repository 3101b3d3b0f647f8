"""Throughput benchmark of the matrix-element hot path on one MI355X.

Workload (default): gg -> t t~ g g at sqrt(s) = 1.5 TeV, m_t = 173 GeV, alpha_s = 0.118,
524288 RAMBO events (seed 0) generated on the device and resident in HBM before timing;
one step = one me_sigma call over the whole batch (helicity-filtered amplitude kernel +
matrix-core colour sum + helicity sum, every event).  Reported: MEs/s in FP64 and in the
mixed form (with its relative error against FP64 on the full batch), the roofline of the
amplitude kernel from HIP-event timings of its launches inside the timed region, the
per-call latency p50/p99, the serving loop's p50/p99, and the CPU oracle timed on a
bounded sample of the same workload on the host cores.

Prints ONE JSON line on stdout.  `--gpus N` with N > 1 is refused: this build measures one
GPU (events are independent; the multi-GPU design is documented, not run).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# the paper's FP64 figure for this exact workload (Table 2: V100, gg->ttgg, grid 524288); context only
PAPER_FP64_MES = 4.20e5
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0           # HBM3E, published peak
FP32_VALU_PEAK_TFLOPS = 78.6   # same without packed FP32 (disabled in this build)
MFMA_F64_PEAK_TFLOPS = 78.6
MFMA_F16_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(proc, x, steps, warmup, torch):
    out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    for _ in range(warmup):
        proc.sigma(x, out=out)
    torch.cuda.synchronize()
    proc.profile(True)
    per_call = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        proc.sigma(x, out=out)
        b.record()
        per_call.append((a, b))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_amp, ms_cs, n_amp, n_cs = proc.profile(False)
    lat = sorted(a.elapsed_time(b) for a, b in per_call)
    return out, (t1 - t0) * 1e3 / steps, lat, ms_amp, ms_cs, n_amp, n_cs


def kernel_source_hash(process):
    """hash of the sources that define the amplitude kernel of `process` and its launch (the
    helper headers and the generated file up to the process descriptor)"""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2210_11122_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "generated", f"proc_{process}.hip"), "rb") as fh:
        gen = fh.read().split(b"const ProcessDesc* process_")[0]
    heads = ["helas.hpp"] + (["colorsum.hpp"] if b'#include "../colorsum.hpp"' in gen else [])
    for name in heads:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    h.update(gen)
    return h.hexdigest()[:16]


def measured_traffic(process):
    """HBM bytes per amplitude-kernel launch from the committed rocprofv3 counter summary, or
    None when the kernel changed since the counters were taken"""
    path = os.path.join(ROOT, "profiles", f"amp_kernel_{process}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_source_hash(process):
        return None
    return t


def quantile(v, q):
    import numpy as np
    return float(np.quantile(np.asarray(v), q)) if len(v) else None


def sweep(processes, precisions, log2_sizes, torch, min_ms=300.0):
    """batch-size sweep: median per-call time (HIP events) of me_sigma per process, precision
    and batch size, momenta resident on the device"""
    import numpy as np
    from paper_2210_11122_amd import Process
    from tests import workloads as W
    out = {}
    for name in processes:
        rows = []
        for prec in precisions:
            proc = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S, precision=prec)
            for k in log2_sizes(name):
                n = 1 << k
                x = proc.rambo(W.SEED, W.sqrt_s(name), n)
                y = torch.empty(n, dtype=torch.float64, device="cuda")
                for _ in range(2):
                    proc.sigma(x, out=y)
                torch.cuda.synchronize()
                times, spent = [], 0.0
                while len(times) < 5 or (spent < min_ms and len(times) < 200):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    proc.sigma(x, out=y)
                    b.record()
                    b.synchronize()
                    times.append(a.elapsed_time(b))
                    spent += times[-1]
                med = float(np.median(times))
                rows.append({"precision": prec, "n_evt": n, "ms_median": med, "MEs_per_s": n / med * 1e3,
                             "calls": len(times)})
                log(f"sweep {name} {prec} n=2^{k}: {med:.4f} ms, {n / med * 1e3:.4g} MEs/s")
                del x, y
            del proc
        out[name] = rows
    return out


def roofline_bound(bytes_per_me, flops_per_me):
    """'hbm' if moving an ME's bytes at the HBM peak takes longer than its algorithmic flops at
    the FP64 peak (fewer flops per byte than the machine balance), else 'alu'"""
    return "hbm" if bytes_per_me / (HBM_PEAK_GBS * 1e9) > flops_per_me / (FP64_VALU_PEAK_TFLOPS * 1e12) else "alu"


def sweep_markdown(res):
    """the sweep as a table: MEs/s per process and form (rows) and batch size (columns)"""
    sizes = sorted({r["n_evt"] for rows in res.values() for r in rows})
    L = ["| process | form | " + " | ".join(f"2^{n.bit_length() - 1}" for n in sizes) + " |",
         "|---|---|" + "---|" * len(sizes)]
    for name, rows in res.items():
        for prec in dict.fromkeys(r["precision"] for r in rows):
            by = {r["n_evt"]: r["MEs_per_s"] for r in rows if r["precision"] == prec}
            L.append(f"| {name} | {prec} | " + " | ".join(f"{by[n]:.3g}" if n in by else "-" for n in sizes) + " |")
    return "\n".join(L) + "\n"


def cpu_baseline(name, n_evt_total, params, budget_s, threads):
    """the oracle as it stands on a bounded sample: first events of the same RAMBO stream"""
    import numpy as np
    import oracle
    from tests import workloads as W
    n_probe = 8 * threads
    while True:
        probe = oracle.rambo(0, W.sqrt_s(name), W.final_masses(name), n_probe)
        t = time.perf_counter()
        oracle.me_batch(name, probe, params=params, threads=threads)
        dt = time.perf_counter() - t
        if dt > 0.5 or n_probe >= n_evt_total:
            break
        n_probe *= 4
    rate = n_probe / max(dt, 1e-6)
    n = int(min(n_evt_total, max(threads, rate * budget_s)))
    p = oracle.rambo(0, W.sqrt_s(name), W.final_masses(name), n)
    t = time.perf_counter()
    me = oracle.me_batch(name, p, params=params, threads=threads)
    dt = time.perf_counter() - t
    return p, me, n / dt, dt


# oracle subset per process for the table: enough events for the error statistics, a few
# seconds of the oracle on the host threads
TABLE_ORACLE_EVENTS = {"ee_mumu": 8192, "gg_tt": 65536, "gg_ttg": 16384, "gg_ttgg": 4096, "gg_ttggg": 1024}


def rel_stats(rel):
    import numpy as np
    return {"max": float(rel.max()), "median": float(np.median(rel)), "p99": float(np.quantile(rel, 0.99)),
            "p999": float(np.quantile(rel, 0.999)), "n": int(rel.size)}


def process_table(torch, min_ms=500.0, threads=None):
    """Per process at its configured size: MEs/s of the FP64 and the two mixed forms (median
    per-call time), the amplitude kernel's algorithmic rate against the VALU peak (HIP events
    around its launches), the end-to-end rate (MEs/s x algorithmic flops per ME), the mixed
    forms' relative error against the GPU FP64 result on the whole batch and against the FP64
    oracle on a subset, and the oracle's own MEs/s on all host threads and on one."""
    import numpy as np
    import oracle
    from paper_2210_11122_amd import Process
    from tests import hostinfo
    from tests import workloads as W
    threads = threads or hostinfo.host_threads()
    rows = []
    # every process at its configured size; ee_mumu also at 2^20, where its calls are long enough
    # to be set by HBM rather than by launches
    for name, n in [(nm, W.PROCESSES[nm][2]) for nm in W.ALL] + [("ee_mumu", 1 << 20)]:
        rs = W.sqrt_s(name)
        row = {"process": name, "n_events": n}
        ref = None
        nsub = min(n, TABLE_ORACLE_EVENTS[name])
        psub = oracle.rambo(W.SEED, rs, W.final_masses(name), nsub)
        t = time.perf_counter()
        me_or = oracle.me_batch(name, psub, params=W.PARAMS, threads=threads)
        dt = time.perf_counter() - t
        row["oracle"] = {"MEs_per_s": nsub / dt, "threads": threads, "events": nsub}
        n1 = max(1, min(nsub, int(nsub / dt / threads * 1.5)))
        t = time.perf_counter()
        oracle.me_batch(name, psub[:n1], params=W.PARAMS, threads=1)
        row["oracle"]["MEs_per_s_single_thread"] = n1 / (time.perf_counter() - t)
        xsub = torch.from_numpy(psub).cuda()
        for prec in ("fp64", "mixed_fp16", "mixed_bf16"):
            proc = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S, precision=prec)
            info = proc.info
            x = proc.rambo(W.SEED, rs, n)
            y = torch.empty(n, dtype=torch.float64, device="cuda")
            for _ in range(2):
                proc.sigma(x, out=y)
            torch.cuda.synchronize()
            # per-call times without the library's per-launch events (which add host work
            # before each launch, a visible share of the small processes' calls) ...
            times, spent = [], 0.0
            while len(times) < 5 or (spent < min_ms and len(times) < 200):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                proc.sigma(x, out=y)
                b.record()
                b.synchronize()
                times.append(a.elapsed_time(b))
                spent += times[-1]
            # ... then the amplitude kernel's own time over as many calls
            proc.profile(True)
            for _ in range(len(times)):
                proc.sigma(x, out=y)
            torch.cuda.synchronize()
            ms_amp, ms_cs, n_amp, _ = proc.profile(False)
            med = float(np.median(times))
            lanes = n * info["n_good_hel"]
            f_amp = info["flops_amp_lane"] + (info["flops_colour_lane"] if info["fused_colour"] else 0.0)
            f_me = info["n_good_hel"] * (info["flops_amp_lane"] + info["flops_colour_lane"])
            mes = n / med * 1e3
            bytes_me = x.shape[1] * 32 + 8   # momenta in, |M|^2 out
            r = {"MEs_per_s": mes, "ms_per_call": med, "calls": len(times),
                 "hbm_bytes_per_me": bytes_me, "hbm_frac": mes * bytes_me / (HBM_PEAK_GBS * 1e9),
                 "amp_kernel_tflops": f_amp * lanes * len(times) / (ms_amp / 1e3) / 1e12 if ms_amp > 0 else None,
                 "end_to_end_tflops": mes * f_me / 1e12,
                 "flops_per_me": f_me, "colour_sum_in_amp_kernel": bool(info["fused_colour"]),
                 "two_streams": bool(info["n_partial_slots"] > 0 and n > info["chunk_events"])}
            r["amp_kernel_frac"] = r["amp_kernel_tflops"] / FP64_VALU_PEAK_TFLOPS if r["amp_kernel_tflops"] else None
            r["end_to_end_frac"] = r["end_to_end_tflops"] / FP64_VALU_PEAK_TFLOPS
            got_sub = proc.sigma(xsub).cpu().numpy()
            rel_or = np.abs(got_sub / me_or - 1)
            r["rel_err_vs_oracle"] = rel_stats(rel_or)
            if prec == "fp64":
                ref = y.clone()
                r["n_over_1e-12_vs_oracle"] = int((rel_or > 1e-12).sum())
            else:
                r["rel_err_vs_gpu_fp64_full_batch"] = rel_stats((y / ref - 1).abs().cpu().numpy())
            row[prec] = r
            log(f"table {name} {prec}: {mes:.4g} MEs/s, amp kernel {r['amp_kernel_tflops'] or 0:.2f} TFLOP/s, "
                f"vs oracle max {rel_or.max():.2e} median {np.median(rel_or):.2e}")
            del proc, x, y
        rows.append(row)
    return rows


def table_markdown(rows):
    def f(v, k=3):
        return "-" if v is None else f"{v:.{k}g}"
    L = ["| process | events | form | MEs/s | amp. kernel TFLOP/s (frac of 78.6) | end-to-end frac | HBM frac | "
         "rel. err vs FP64 oracle (max / median / p99 / p99.9; n) | vs GPU FP64, full batch (max / median) |",
         "|---|---|---|---|---|---|---|---|---|"]
    for row in rows:
        for prec in ("fp64", "mixed_fp16", "mixed_bf16"):
            r = row[prec]
            e = r["rel_err_vs_oracle"]
            g = r.get("rel_err_vs_gpu_fp64_full_batch")
            L.append(f"| {row['process']} | {row['n_events']} | {prec} | {f(r['MEs_per_s'], 4)} | "
                     f"{f(r['amp_kernel_tflops'])} ({f(r['amp_kernel_frac'], 2)}) | {f(r['end_to_end_frac'], 2)} | "
                     f"{f(r['hbm_frac'], 2)} | "
                     f"{f(e['max'], 2)} / {f(e['median'], 2)} / {f(e['p99'], 2)} / {f(e['p999'], 2)}; {e['n']} | "
                     + (f"{f(g['max'], 2)} / {f(g['median'], 2)} |" if g else "- |"))
    L.append("")
    L.append("| process | oracle MEs/s (threads) | oracle MEs/s, 1 thread |")
    L.append("|---|---|---|")
    seen = set()
    for row in rows:
        if row["process"] in seen:
            continue
        seen.add(row["process"])
        o = row["oracle"]
        L.append(f"| {row['process']} | {f(o['MEs_per_s'], 4)} ({o['threads']}) | {f(o['MEs_per_s_single_thread'], 4)} |")
    return "\n".join(L) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--process", default="gg_ttgg")
    ap.add_argument("--n-evt", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sweep", action="store_true",
                    help="batch-size sweep 2^8..2^20 of every process instead of the benchmark line")
    ap.add_argument("--sweep-md", default=None, metavar="MD_PATH", help="with --sweep: also write it as markdown")
    ap.add_argument("--table", default=None, metavar="MD_PATH",
                    help="per-process table (FP64 and mixed MEs/s, roofline fractions, mixed errors, oracle "
                         "MEs/s) as one JSON line, and as markdown to MD_PATH, instead of the benchmark line")
    ap.add_argument("--serving-processes", default="gg_tt,gg_ttg,gg_ttgg")
    ap.add_argument("--serving-seconds", type=float, default=10.0)
    ap.add_argument("--serving-budget-mib", type=int, default=None,
                    help="device-memory budget of the serving loop (default: 256 MiB without gg_ttggg, 32 GiB with it)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one plain device copy of this size (for PMC byte calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the events are independent, so a run "
              "on N GPUs would give each GPU 1/N of the events; it is not measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2210_11122_amd import Process
    from tests import workloads as W

    name = args.process
    n_evt = args.n_evt or W.PROCESSES[name][2]
    rs = W.sqrt_s(name)
    torch.cuda.set_device(0)
    if args.sweep:
        sizes = lambda nm: range(8, (19 if nm == "gg_ttggg" else 21), 2)
        res = sweep(["ee_mumu", "gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"], ["fp64", "mixed_fp16"], sizes, torch)
        if args.sweep_md:
            with open(args.sweep_md, "w") as fh:
                fh.write(sweep_markdown(res))
        print(json.dumps({"metric": "batch-size sweep: matrix elements/sec at 1 GPU", "unit": "MEs/s",
                          "data": "synthetic (RAMBO phase space on device, seed 0)", "sweep": res}), flush=True)
        return
    if args.table:
        from tests import hostinfo
        rows = process_table(torch)
        with open(args.table, "w") as fh:
            fh.write(table_markdown(rows))
        print(json.dumps({"metric": "matrix elements/sec at 1 GPU per process: FP64 and mixed precision at stated "
                                    "rel. err", "unit": "MEs/s", "cpu_model": hostinfo.cpu_model(),
                          "data": "synthetic (RAMBO phase space, seed 0)", "table": rows}), flush=True)
        return
    log(f"bench: {name} n_evt={n_evt} steps={args.steps} warmup={args.warmup}")

    p64 = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S, precision="fp64")
    info = p64.info
    x = p64.rambo(W.SEED, rs, n_evt)
    torch.cuda.synchronize()

    if args.copy_calibration_mb:
        a = torch.ones(args.copy_calibration_mb << 17, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    out64, ms64, lat64, ms_amp, ms_cs, n_amp, n_cs = timed_steps(p64, x, args.steps, args.warmup, torch)
    mes64 = n_evt / (ms64 / 1e3)
    lanes = n_evt * info["n_good_hel"]
    flops_amp_step = info["flops_amp_lane"] * lanes
    flops_cs_step = info["flops_colour_lane"] * lanes
    fused = bool(info["fused_colour"])
    # with the fused colour sum the amplitude kernel also does the colour contraction
    flops_kernel_step = flops_amp_step + (flops_cs_step if fused else 0.0)
    amp_launches_per_step = n_amp / args.steps
    achieved_tflops = flops_kernel_step * args.steps / (ms_amp / 1e3) / 1e12
    log(f"fp64: {ms64:.3f} ms/step, {mes64:.4g} MEs/s; amplitude kernel{' (+ colour sum)' if fused else ''} "
        f"{ms_amp / args.steps:.3f} ms/step ({achieved_tflops:.2f} TFLOP/s), "
        f"{'helicity sum' if fused else 'colour sum'} {ms_cs / args.steps:.3f} ms/step")

    result = {
        "metric": "matrix elements/sec at 1 GPU (FP64; mixed precision at its stated rel. err)",
        "value": mes64,
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": mes64 / PAPER_FP64_MES if name == "gg_ttgg" and n_evt == 524288 else None,
        "dtype": "f64",
        "data": "synthetic (RAMBO phase space on device, seed 0)",
        "config": {"workload": f"{name} LO, {n_evt} RAMBO events at sqrt(s)={rs:g} GeV, m_t={W.M_TOP:g}, "
                               f"alpha_s={W.ALPHA_S}, helicity-filtered ({info['n_good_hel']}/{info['n_hel']})",
                   "process": name, "n_events": n_evt, "parallelism": "single GPU, one lane per (event, helicity)"},
        "latency_ms": {"p50": quantile(lat64, 0.5), "p99": quantile(lat64, 0.99), "unit": "ms per me_sigma call"},
        "roofline": {
            "bound": "alu",
            "kernel": ("amplitude kernel with the colour sum (FP64 VALU, FP64 MFMA)" if fused
                       else "amplitude kernel (FP64 VALU)"),
            "achieved": achieved_tflops,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP64_VALU_PEAK_TFLOPS,
            "traffic": None,  # filled below from the committed counter profile
            "flops_per_launch": flops_kernel_step / max(amp_launches_per_step, 1),
            "avg_launch_ms": ms_amp / max(n_amp, 1),
            "launches_per_step": amp_launches_per_step,
        },
        "colour_sum": ({"fused_into_amplitude_kernel": True, "helicity_sum_ms_per_step": ms_cs / args.steps}
                       if fused else {
            "bound": "mfma",
            "achieved": flops_cs_step * args.steps / (ms_cs / 1e3) / 1e12 if ms_cs > 0 else None,
            "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "ms_per_step": ms_cs / args.steps,
        }),
    }

    # bytes the path must move per ME: the event's momenta in, |M|^2 out
    bytes_me = x.shape[1] * 32 + 8
    amp_bytes_launch = bytes_me * n_evt / max(amp_launches_per_step, 1)
    hbm_launch = amp_bytes_launch / (result["roofline"]["avg_launch_ms"] / 1e3) / 1e9
    result["hbm"] = {"bytes_per_me": bytes_me,
                     "per_call_GBs": mes64 * bytes_me / 1e9, "per_call_frac": mes64 * bytes_me / (HBM_PEAK_GBS * 1e9),
                     "amp_kernel_GBs": hbm_launch, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    flops_me = info["n_good_hel"] * (info["flops_amp_lane"] + info["flops_colour_lane"])
    if roofline_bound(bytes_me, flops_me) == "hbm":
        # fewer flops per byte than the machine balance (ee_mumu): HBM sets the roofline
        rf = result["roofline"]
        rf.update({"bound": "hbm", "kernel": rf["kernel"] + "; algorithmic bytes: momenta in, |M|^2 out",
                   "achieved": hbm_launch, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": hbm_launch / HBM_PEAK_GBS, "bytes_per_launch": amp_bytes_launch,
                   "alu_TFLOPs": achieved_tflops})
        del rf["flops_per_launch"]

    if info["n_partial_slots"] > 0 and n_evt > info["chunk_events"]:
        # chunks alternate between two streams, so two amplitude launches share the GPU and each
        # takes longer: the per-launch rate above is halved; the step-time rate is a lower bound
        # on the throughput of the amplitude work (the step also holds the colour sum)
        result["roofline"]["concurrent_streams"] = 2
        result["roofline"]["achieved_per_step_time"] = flops_kernel_step / (ms64 / 1e3) / 1e12
    tr = measured_traffic(name)
    mean_launch = n_evt / max(amp_launches_per_step, 1)
    if tr is not None and abs(tr.get("events_per_launch", 0) / mean_launch - 1) > 0.05:
        tr = None   # counters taken at another launch size (the last launch of a batch may be short)
    if tr is not None:
        result["roofline"]["traffic"] = tr["hbm_bytes_per_launch"]
        result["roofline"]["traffic_source"] = tr["source"]
        result["roofline"]["traffic_events_per_launch"] = tr["events_per_launch"]

    if not args.no_mixed:
        for prec, dt_name in [("mixed_fp16", "f32 amplitudes, f16 MFMA colour sum"),
                              ("mixed_bf16", "f32 amplitudes, bf16 MFMA colour sum")]:
            pm = Process(name, m_top=W.M_TOP, alpha_em=W.ALPHA_EM, alpha_s=W.ALPHA_S, precision=prec)
            outm, msm, latm, ms_amp_m, ms_cs_m, n_amp_m, _ = timed_steps(pm, x, args.steps, args.warmup, torch)
            rel = (outm / out64 - 1).abs().cpu().numpy()
            mesm = n_evt / (msm / 1e3)
            ach_m = flops_amp_step * args.steps / (ms_amp_m / 1e3) / 1e12
            result[prec] = {
                "value": mesm, "unit": "MEs/s", "ms_per_step": msm, "dtype": dt_name,
                "rel_err_vs_fp64": {"max": float(rel.max()), "median": float(np.median(rel)),
                                    "p99": float(np.quantile(rel, 0.99)), "p999": float(np.quantile(rel, 0.999))},
                "latency_ms": {"p50": quantile(latm, 0.5), "p99": quantile(latm, 0.99)},
                "amplitude_kernel_tflops": ach_m, "amplitude_kernel_frac_fp32_peak": ach_m / FP32_VALU_PEAK_TFLOPS,
                "colour_sum_in_amplitude_kernel": bool(pm.info["fused_colour"]),
                # with the colour sum in the amplitude kernel: the helicity-sum kernel's time
                "colour_sum_ms_per_step": ms_cs_m / args.steps,
            }
            if pm.info["n_partial_slots"] > 0 and n_evt > pm.info["chunk_events"]:
                # two streams: per-launch times overlap (as for FP64 above)
                result[prec]["amplitude_kernel_tflops_per_step_time"] = flops_amp_step / (msm / 1e3) / 1e12
            log(f"{prec}: {msm:.3f} ms/step, {mesm:.4g} MEs/s, rel err max {rel.max():.2e} "
                f"median {np.median(rel):.2e}, colour sum {ms_cs_m / args.steps:.3f} ms/step")
            del pm

    if not args.no_serving:
        try:
            from paper_2210_11122_amd import serve
            budget = args.serving_budget_mib << 20 if args.serving_budget_mib else None
            result["serving"] = serve.bench_serving(duration_s=args.serving_seconds,
                                                    processes=tuple(args.serving_processes.split(",")),
                                                    hbm_budget=budget, log=log)
        except ImportError:
            result["serving"] = None

    if not args.no_cpu:
        from tests import hostinfo
        threads = hostinfo.host_threads()
        p, me_cpu, rate, dt = cpu_baseline(name, n_evt, W.PARAMS, args.cpu_seconds, threads)
        from tests import referee
        got = p64.sigma(torch.from_numpy(p).cuda()).cpu().numpy()
        rel = np.abs(got / me_cpu - 1)
        # events beyond the FP64 tolerance go to the referee (long double + FP64 spread)
        over = np.where(rel > 1e-12)[0]
        referee_ok, worst, detail = 0, [], []
        for i in over:
            ok, r, spread = referee.judge(name, p[i], got[i], W.PARAMS)
            referee_ok += ok
            worst.append((r, spread, int(i)))
            detail.append({"event": int(i), "gpu": float(got[i]), "oracle": float(me_cpu[i]),
                           "rel_vs_long_double": r, "fp64_spread": spread, "accepted": bool(ok)})
        worst.sort(reverse=True)
        import oracle
        n1 = max(1, min(len(p), int(rate / threads * 2.0)))
        t1 = time.perf_counter()
        oracle.me_batch(name, p[:n1], params=W.PARAMS, threads=1)
        rate1 = n1 / (time.perf_counter() - t1)
        result["cpu_baseline"] = {"value": rate, "unit": "MEs/s", "cores": threads, "kind": "oracle",
                                  "cpu_model": hostinfo.cpu_model(),
                                  "sample": f"first {len(p)} events of the same RAMBO stream, {dt:.1f} s",
                                  "single_thread_value": rate1, "single_thread_sample": f"first {n1} events"}
        result["parity_sample"] = {"n": int(len(p)), "max_rel_err": float(rel.max()),
                                   "median_rel_err": float(np.median(rel)), "tolerance": 1e-12,
                                   "n_over_tolerance": int(len(over)),
                                   "n_over_tolerance_within_fp64_conditioning": int(referee_ok),
                                   "worst_rel_vs_long_double_and_fp64_spread": worst[:3],
                                   "over_tolerance": detail[:64]}
        log(f"cpu oracle: {rate:.4g} MEs/s on {threads} threads ({len(p)} events); GPU vs oracle max rel {rel.max():.2e}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
