#!/usr/bin/env python
"""Benchmark: Gauss-Newton Hessian-vector products per second on one MI355X.

Workload (default): the image-transport variant of band-limited PDE-LDDMM
(original BL PDE-LDDMM, Section 2.3.1 of the paper) on a 128^3 grid with a
32^3 x 3 band-limited velocity, Nt = 10 SL-RK2 steps, alpha = 0.0025, s = 2,
sigma^2 = 1, FP32 fields with FP64 reductions.  One step = one full Hessian
matvec (incremental state sweep, t = 1 coupling, incremental adjoint sweep
with the Hessian time integral, L~ term), after a state solve at a fixed
velocity (not timed).  Inputs are synthetic: a brain-like phantom pair and a
random band-limited velocity of 8 voxels maximum displacement per unit time,
resident on the GPU before timing starts.

Prints one JSON line with the throughput, the roofline figures of the
dominant kernel (per-launch algorithmic bytes over its event-timed average
duration) and the CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3     # MI355X dense FP32 (matrix and vector)

# variant-1 Hessian matvec kernels that move data (HBM roofline); DFT kernels also report MFMA use
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_matvec_kernels_128.json")
WEIGHTS_FILE = os.path.join(ROOT, "paper_2006_06823_amd", "weights", "warmstart_v1_128.npz")


VARIANT_NAMES = {1: "image-transport", 2: "state-equation", 3: "deformation-state"}

# library profile names of the DFT-stage kernels (MFMA figures in "extra")
DFT_KERNELS = ("k_expand", "k_reduce", "k_axis0", "dft_", "k_iota", "k_pi")

# library profile name (trailing field count and row-set suffix dropped) -> (pattern of the compiled kernel
# name as a profiler lists it, spaces removed; the source files its code comes from)
KERNEL_SOURCES = {
    "k_brick<k_bl_adjoint_step>": (r"k_brick<[\w:()]*EpiBLAdjoint<", ("brick.hip", "common.h")),
    "k_brick<k_interp>": (r"k_brick<[\w:()]*EpiInterp<", ("brick.hip", "common.h")),
    "k_brick<k_interp_diff>": (r"k_brick<[\w:()]*EpiInterpDiff<", ("brick.hip", "common.h")),
    "k_expand": (r"k_expand<", ("dft_planes.hip",)),
    "k_reduce": (r"k_reduce<0,", ("dft_planes.hip",)),
    "k_reduce_products": (r"k_reduce<[1-4],", ("dft_planes.hip",)),
}


def _base_name(name):
    import re
    return re.sub(r"(\[.*\])?\d*$", "", name)


def _source_digest(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_2006_06823_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, N, K, variant, alg_bytes):
    """HBM bytes per launch of `kernel`: the stored ratio of measured (profiler FETCH_SIZE + WRITE_SIZE, scaled
    by a plain copy of known size) over algorithmic bytes, times this run's algorithmic bytes per launch.  None
    when no ratio was stored for this kernel and workload, or when the kernel's source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no stored counter ratio"
    tr = json.load(open(TRAFFIC_FILE))
    ent = tr.get("kernels", {}).get(kernel)
    if tr.get("workload") != list(N) + list(K) + [variant] or ent is None:
        return None, "no stored counter ratio for this kernel and workload"
    src = KERNEL_SOURCES.get(_base_name(kernel))
    if src is None or _source_digest(src[1]) != ent.get("source_digest"):
        return None, "kernel source changed since the counters were taken"
    return (round(ent["traffic_over_algorithmic"] * alg_bytes),
            f"stored ratio {ent['traffic_over_algorithmic']} (profiles/{os.path.basename(TRAFFIC_FILE)}) "
            f"x this run's algorithmic bytes per launch")


def write_traffic(d):
    """Post-process four counter runs (no GPU): `d`/fetch and `d`/write hold FETCH_SIZE and WRITE_SIZE runs of
    `bench.py --steps 2 --warmup 1 --no-cpu-baseline --learned-pairs 0`, `d`/cal_fetch and `d`/cal_write the
    same counters over `bench.py --calibrate-copy 256`, `d`/bench.json the JSON line of an unprofiled run of
    the same workload (it names the dominant kernel and its algorithmic bytes per launch; under the counters
    the kernels run serialised and another kernel may lead).  Writes the stored ratio of the dominant kernel
    (the profiler's most frequent launch shape of it) and prints a markdown table of every dispatch group."""
    import collections
    import csv
    import re

    def load(sub):
        rows = list(csv.DictReader(open(os.path.join(d, sub, "run_counter_collection.csv"))))
        per = collections.defaultdict(float)
        meta = {}
        for r in rows:
            key = int(r["Dispatch_Id"])
            per[key] += float(r["Counter_Value"])
            # the brick tile (an autotuner choice, which may differ between the runs) is dropped from the
            # name: every tile writes the same fields and differs only in its halo re-reads
            name = re.sub(r",?lddmm::\(anonymousnamespace\)::Tile<[^>]*>", "", r["Kernel_Name"].replace(" ", ""))
            meta[key] = (name, int(r["Grid_Size"]))
        return per, meta

    bench = json.loads(open(os.path.join(d, "bench.json")).read().strip().splitlines()[-1])
    scale = {}
    for c in ("fetch", "write"):
        per, meta = load("cal_" + c)
        vals = [per[k] for k in per if "copyBuffer" in meta[k][0]]
        n_kib = 256 * 1024
        scale[c] = n_kib / (sum(vals) / len(vals))
    groups = collections.defaultdict(lambda: [0, 0.0, 0.0])
    fetch, fmeta = load("fetch")
    write, wmeta = load("write")
    for c, per, meta in (("fetch", fetch, fmeta), ("write", write, wmeta)):
        for k, v in per.items():
            g = groups[meta[k]]
            if c == "fetch":
                g[0] += 1
                g[1] += v * scale[c]
            else:
                g[2] += v * scale[c]
    rf = bench["roofline"]
    dom = rf["kernel"]
    pat, files = KERNEL_SOURCES[_base_name(dom)]
    cand = {key: g for key, g in groups.items() if re.search(pat, key[0]) and g[0] > 0}
    if not cand:
        raise SystemExit(f"no dispatch of {dom} in the counter runs")
    key = max(cand, key=lambda k: cand[k][0])       # the most frequent (name, grid): the matvec's launches
    n, rd, wr = cand[key]
    ratio = round((rd + wr) / n * 1024.0 / rf["algorithmic_bytes_per_launch"], 4)
    cfg = bench["config"]
    out = {"workload": list(cfg["grid"]) + list(cfg["band"]) + [cfg["variant"]],
           "fetch_scale": round(scale["fetch"], 5), "write_scale": round(scale["write"], 5),
           "kernels": {dom: {"traffic_over_algorithmic": ratio, "dispatches": n, "source_digest": _source_digest(files),
                             "read_KiB": round(rd / n, 1), "write_KiB": round(wr / n, 1),
                             "algorithmic_KiB": round(rf["algorithmic_bytes_per_launch"] / 1024.0, 1)}}}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"FETCH_SIZE x {scale['fetch']:.5f}, WRITE_SIZE x {scale['write']:.5f} (plain 256 MiB copy)\n")
    print("| kernel | grid | dispatches | read KiB | write KiB |\n|---|---|---|---|---|")
    for (name, grid), (n_, rd_, wr_) in sorted(groups.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        if n_ == 0:
            continue
        short = re.sub(r"\(.*", "", name.replace("void", "").replace("lddmm::", "").replace("(anonymousnamespace)::", ""))
        print(f"| {short[:60]} | {grid} | {n_} | {rd_ / n_:.1f} | {wr_ / n_:.1f} |")
    print(f"\n{dom}: {key[0][:60]} grid {key[1]}, {n} dispatches, measured/algorithmic = {ratio}")
    if os.path.isdir(os.path.join(d, "sq")):
        sq_table(d)


def sq_table(d):
    """Per-kernel averages of the SQ counter runs `d`/sq (SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY
    SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY) and `d`/mfma (SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CU_CYCLES SQ_WAVES)."""
    import collections
    import csv
    import re

    def load(sub):
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        cnt = collections.defaultdict(set)
        for r in csv.DictReader(open(os.path.join(d, sub, "run_counter_collection.csv"))):
            name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("void ", "").replace("lddmm::", "")
                          .replace("(anonymous namespace)::", ""))
            name = re.sub(r",\s*Tile<.*", ">", name)
            agg[name][r["Counter_Name"]] += float(r["Counter_Value"])
            cnt[name].add(r["Dispatch_Id"])
        return agg, cnt

    sq, n_sq = load("sq")
    mf, _ = load("mfma") if os.path.isdir(os.path.join(d, "mfma")) else ({}, {})
    print("\n| kernel | dispatches | waves / dispatch | wave lifetime (cycles) | waiting | issuing | MFMA busy |")
    print("|---|---|---|---|---|---|---|")
    order = sorted(sq, key=lambda k: -sq[k].get("SQ_WAVE_CYCLES", 0))
    for k in order[:16]:
        a, n = sq[k], len(n_sq[k])
        w = a.get("SQ_WAVES", 0)
        if w == 0:
            continue
        life = a.get("SQ_WAVE_CYCLES", 0)
        mb = None
        if k in mf and mf[k].get("SQ_BUSY_CU_CYCLES", 0) > 0:
            mb = mf[k].get("SQ_VALU_MFMA_BUSY_CYCLES", 0) / (4.0 * mf[k]["SQ_BUSY_CU_CYCLES"])
        print(f"| {k[:58]} | {n} | {w / n:.0f} | {4 * life / w:.0f} | {a.get('SQ_WAIT_ANY', 0) / life:.0%} | "
              f"{a.get('SQ_ACTIVE_INST_ANY', 0) / life:.0%} | {'' if mb is None else f'{mb:.1%}'} |")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", type=int, default=1, choices=(1, 2, 3),
                    help="1 image transport (default), 2 state equation, 3 deformation state")
    ap.add_argument("--rk4", action="store_true",
                    help="deformation-state variant integrated by the explicit RK4 comparator (Eulerian form) "
                         "instead of SL-RK2; use with --variant 3 and its nt (25-50)")
    ap.add_argument("--nonstationary", action="store_true",
                    help="a velocity per time node (variants 1 and 3): the matvec of the (nt + 1)-node parameter")
    ap.add_argument("--size", type=int, nargs=3, default=(128, 128, 128))
    ap.add_argument("--band", type=int, nargs=3, default=(32, 32, 32))
    ap.add_argument("--nt", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", type=int, default=0,
                    help="instead of the matvec benchmark: register this many uneven subjects (96^3..192^3, "
                         "deformation-state variant, split-bf16 DFT) to one template in one batched GN-Krylov call")
    ap.add_argument("--batched-gn", type=int, default=2)
    ap.add_argument("--batched-pcg", type=int, default=5)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="instead of the benchmark: 5 plain device copies of MB megabytes (float32), the reference "
                         "for scaling the HBM byte counters of a profiler run")
    ap.add_argument("--write-traffic", default=None, metavar="DIR",
                    help="instead of the benchmark (no GPU): turn four counter runs under DIR into the stored "
                         "HBM-traffic ratio of the dominant kernel and print their table")
    ap.add_argument("--learned-pairs", type=int, default=8,
                    help="held-out pairs registered plain and with the trained warm start (0: skip)")
    ap.add_argument("--tune-save", default=None, metavar="FILE",
                    help="write the autotuner's choices of this run ({key: choice} JSON) to FILE at the end")
    ap.add_argument("--tune-load", default=None, metavar="FILE",
                    help="fix the autotuner's choices from FILE before the run (so that a profiled run, whose "
                         "timings the profiler perturbs, launches the kernels an unprofiled run chose)")
    return ap.parse_args()


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the library runs one "
              f"registration context per GPU; independent registrations would shard one per GPU).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_06823_amd import lddmm_bl as L
    from paper_2006_06823_amd import synthetic as syn

    if args.tune_load:
        for key, choice in json.load(open(args.tune_load)).items():
            L.tune_set(key, int(choice))
    if args.batched > 0:
        print(json.dumps(batched_leg(args)), flush=True)
        return
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.rand(n, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 5}), flush=True)
        return

    N, K, Nt = tuple(args.size), tuple(args.band), args.nt
    variant = {1: L.IMAGE_TRANSPORT, 2: L.STATE_EQUATION, 3: L.DEFORMATION_STATE}[args.variant]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    I0, I1 = syn.phantom_pair_3d(N, seed=1, max_disp_vox=8.0)
    integ = L.EULER_RK4 if args.rk4 else L.SL_RK2
    ctx = L.Context(L.Problem(N, K, nt=Nt, variant=variant, precision=L.FP32, integrator=integ,
                              nonstationary=args.nonstationary))
    g = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)
    ctx.set_images(g(I0), g(I1))
    # random band-limited velocity scaled to 8 voxels maximum displacement per unit time
    vc = syn.random_bl_coefficients(3, K, seed=2)
    vg = ctx.include(g(vc), 3).double()
    scale = torch.tensor([float(n) for n in N], dtype=torch.float64, device=dev).reshape(3, 1, 1, 1)
    vmax = float((vg * scale).abs().max())
    v = g(vc * (8.0 / vmax))
    dv = g(syn.random_bl_coefficients(3, K, seed=3))
    if args.nonstationary:   # the same fields at every node: a time-constant velocity in the (nt + 1)-node form
        v = v.unsqueeze(0).repeat(Nt + 1, 1, 1, 1, 1).contiguous()
        dv = dv.unsqueeze(0).repeat(Nt + 1, 1, 1, 1, 1).contiguous()
    E, _ = ctx.state_solve(v)
    out = torch.empty_like(dv)
    # the matvecs are enqueued on the context's own stream (the library's calls only enqueue them), so no
    # cross-stream event waits sit between two of them
    stream = ctx.stream
    torch.cuda.synchronize()

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            ctx.hess_matvec(dv, out)
    torch.cuda.synchronize()

    # timed region: K matvecs
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    with torch.cuda.stream(stream):
        t_start.record(stream)
        for _ in range(args.steps):
            ctx.hess_matvec(dv, out)
        t_stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_stop)
    ms_per_step = ms_total / args.steps
    value = 1000.0 / ms_per_step

    # same region again with per-kernel HIP events inside the library (roofline of the dominant kernel)
    L.profile_enable(True)
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            ctx.hess_matvec(dv, out)
    torch.cuda.synchronize()
    stats = L.profile_read()
    L.profile_enable(False)
    dom_name, dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    kernel_ms = sum(s["ms"] for s in stats.values())
    avg_ms = dom["ms"] / dom["count"]
    bytes_per_launch = dom["bytes"] / dom["count"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic, traffic_note = stored_traffic(dom_name, N, K, args.variant, bytes_per_launch)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_note,
        "kernel": dom_name, "launches_per_step": dom["count"] / args.steps,
        "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": bytes_per_launch,
    }
    dft = [s for n, s in stats.items() if n.startswith(DFT_KERNELS)]
    dft_flops = sum(s["flops"] for s in dft)
    dft_ms = sum(s["ms"] for s in dft)
    kernels = {n: {"launches_per_step": s["count"] / args.steps, "ms_per_step": round(s["ms"] / args.steps, 4),
                   "GBps": round(s["bytes"] / (s["ms"] * 1e-3) / 1e9, 1) if s["ms"] > 0 else None}
               for n, s in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])}

    # extra timings of the other solves at this velocity (not the metric)
    t0 = time.perf_counter()
    ctx.state_solve(v)
    state_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ctx.adjoint_solve()
    adjoint_ms = (time.perf_counter() - t0) * 1e3

    learned = None
    if args.learned_pairs > 0 and args.variant == 1 and N == (128, 128, 128) and K == (32, 32, 32):
        learned = learned_leg(args.learned_pairs)

    cpu = None
    if not args.no_cpu_baseline and not args.nonstationary:
        cpu = cpu_baseline(variant, N, K, Nt, I0, I1, (vc * (8.0 / vmax)), syn.random_bl_coefficients(3, K, seed=3),
                           rk4=args.rk4)

    line = {
        "metric": "Hessian-matvecs/s at 128^3" if N == (128, 128, 128) else f"Hessian-matvecs/s at {N}",
        "value": round(value, 2), "unit": "matvec/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{VARIANT_NAMES[args.variant]} BL PDE-LDDMM "
                               f"Gauss-Newton Hessian matvec, grid {N[0]}x{N[1]}x{N[2]}, band {K[0]}x{K[1]}x{K[2]}x3, "
                               f"Nt={Nt}, {'explicit RK4 (Eulerian)' if args.rk4 else 'SL-RK2'}, "
                               f"{'non-stationary velocity, ' if args.nonstationary else ''}"
                               f"FP32 with FP64 reductions",
                   "grid": list(N), "band": list(K), "nt": Nt, "variant": args.variant,
                   "integrator": "rk4" if args.rk4 else "sl-rk2", "nonstationary": bool(args.nonstationary),
                   "alpha": 0.0025, "s": 2, "sigma2": 1.0},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": {"wall_s_timed": round(wall, 4), "kernel_ms_per_step": round(kernel_ms / args.steps, 4),
                  "dft_mfma_tflops": round(dft_flops / (dft_ms * 1e-3) / 1e12, 2) if dft_ms > 0 else None,
                  "dft_mfma_frac_fp32": round(dft_flops / (dft_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4)
                  if dft_ms > 0 else None,
                  "state_solve_ms": round(state_ms, 3), "adjoint_solve_ms": round(adjoint_ms, 3),
                  "objective": E, "kernels": kernels, "registrations": learned},
    }
    print(json.dumps(line), flush=True)
    if args.tune_save:
        with open(args.tune_save, "w") as fh:
            json.dump(L.tune_table(), fh, indent=1, sort_keys=True)


def _render_subject(i):
    from paper_2006_06823_amd import synthetic as syn
    import numpy as np
    n = 96 + 16 * int(np.random.default_rng(1000 + i).integers(0, 7))
    I0, I1 = syn.phantom_pair_3d((n, n, n), 1000 + i, max_disp_vox=8.0, template_seed=999)
    return n, I0, I1


def batched_leg(args):
    """Uneven subjects (N_i in {96, 112, ..., 192}, K_i = clamp(8 ceil(N_i / 32), 32, 48)) registered to one
    template in one batched Gauss-Newton-Krylov call with a fixed iteration budget."""
    import multiprocessing as mp
    import numpy as np
    import torch
    from paper_2006_06823_amd import lddmm_bl as L
    B = args.batched
    with mp.get_context("fork").Pool(min(16, B)) as pool:
        subj = pool.map(_render_subject, range(B))
    dev = torch.device("cuda", 0)
    probs, I0s, I1s, vs = [], [], [], []
    for n, I0, I1 in subj:
        k = min(48, max(32, 8 * -(-n // 32)))
        probs.append(L.Problem((n, n, n), (k, k, k), nt=args.nt, variant=L.DEFORMATION_STATE, precision=L.BF16_DFT))
        I0s.append(torch.from_numpy(I0).to(dev))
        I1s.append(torch.from_numpy(I1).to(dev))
        vs.append(torch.zeros((3, k, k, k), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, reps = L.gn_solve_batched(probs, I0s, I1s, vs, max_gn=args.batched_gn, max_pcg=args.batched_pcg,
                                  fixed_iters=True, device=dev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mv = sum(r["hess_matvecs"] for r in reps)
    vox = sum(n ** 3 for n, _, _ in subj)
    # reference bytes of a deformation-state matvec: (27 + 59 Nt) grid fields of 4 N^3 bytes each, the
    # per-matvec dataflow in which every kernel reads its grid inputs once
    ref_bytes = sum(r["hess_matvecs"] * (27 + 59 * args.nt) * 4.0 * n ** 3 for r, (n, _, _) in zip(reps, subj))
    achieved = ref_bytes / wall / 1e9
    return {"metric": "batched subject Hessian-matvecs/s", "value": round(mv / wall, 2), "unit": "matvec/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": "bf16-split DFT, f32 fields, f64 reductions",
            "data": "synthetic",
            "config": {"workload": f"{B} subjects 96^3..192^3 to one template, deformation-state, Nt={args.nt}, "
                                   f"{args.batched_gn} GN x {args.batched_pcg} PCG fixed",
                       "subject_sizes": [n for n, _, _ in subj]},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(achieved / 8000.0, 4), "traffic": None,
                         "basis": "reference bytes of every subject's matvecs over the whole batch's wall time, "
                                  "which also holds the state, adjoint and line-search solves"},
            "extra": {"wall_s": round(wall, 3), "status": st, "matvecs": mv,
                      "voxel_matvecs_per_s": round(mv / wall * vox / B, 1),
                      "mse_rel_mean": round(float(np.mean([r["mse_rel"] for r in reps])), 4)}}


def learned_leg(npairs):
    """Registrations/s on held-out pairs: plain GN-Krylov vs the trained warm start (if its weights exist)."""
    if not os.path.exists(WEIGHTS_FILE):
        return {"skipped": "no trained weights"}
    from paper_2006_06823_amd import learned as LW
    seeds = list(range(20000, 20000 + npairs))
    pairs = [LW.render_pair(sd) for sd in seeds]
    reg = LW.Registrar(variant=1)
    net = LW.load_weights(WEIGHTS_FILE, device=reg.device)

    class _List:
        def pairs(self, sds):
            for sd, (a, b) in zip(sds, pairs):
                yield sd, a, b
    rows = LW.compare(net, reg, seeds, _List(), LW.SolveOpts(), log=lambda *a, **k: None, with_Z=True, ml_inner=5)
    summ = LW.summarize(rows, with_Z=True)
    out = {"pairs": npairs, "seeds": f"{seeds[0]}..{seeds[-1]}", "tolerance": "rel grad 1e-3 of |g(0)|_inf",
           "caps": "20 GN x 10 PCG"}
    for k in ("plain", "learned", "learned_E", "learned_Z", "plain_ml"):
        out[k] = {m: round(summ[k][m], 4) for m in ("registrations_per_s", "gn_iters_mean", "hess_matvecs_mean",
                                                    "seconds_mean", "reached_tol", "reached_plain_E",
                                                    "gn_iter_ratio", "time_ratio") if m in summ[k]}
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(variant, N, K, Nt, I0, I1, v, dv, rk4=False):
    """The FP64 CPU oracle on the host cores: full Hessian matvecs at the same workload, with torch's default
    thread count (the reported value) and with one thread, plus one matvec of the other variant."""
    import numpy as np
    import torch

    from oracle.problem import Problem as OP
    from oracle.eulerian_rk import Variant3RK
    from oracle.variant1 import Variant1
    from oracle.variant2 import Variant2
    from oracle.variant3 import Variant3

    def timed(var, reps):
        cls = Variant3RK if (rk4 and var == 3) else {1: Variant1, 2: Variant2, 3: Variant3}[var]
        model = cls(OP(N, K, Nt=Nt), I0.astype(np.float64), I1.astype(np.float64))
        model.setup(v)
        model.state()
        t0 = time.perf_counter()
        for _ in range(reps):
            model.hess_matvec(dv)
        return (time.perf_counter() - t0) / reps

    threads = torch.get_num_threads()
    dt = timed(variant, 2)
    other = timed(3 if variant == 1 else 1, 1)
    torch.set_num_threads(1)
    try:
        dt1 = timed(variant, 1)
    finally:
        torch.set_num_threads(threads)
    return {"value": round(1.0 / dt, 5), "unit": "matvec/s", "cores": threads, "kind": "oracle",
            "sample": f"2 full Hessian matvecs of the same workload in the FP64 oracle (torch CPU, {threads} "
                      f"threads), {dt:.1f} s each; set-up and state solve excluded",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": round(1.0 / dt1, 5), "cores": 1, "sample": f"1 matvec, {dt1:.1f} s"},
            "other_variant": {"variant": 3 if variant == 1 else 1, "value": round(1.0 / other, 5), "cores": threads,
                              "sample": f"1 matvec of the {VARIANT_NAMES[3 if variant == 1 else 1]}"
                                        f" variant at the same sizes, {other:.1f} s"}}


if __name__ == "__main__":
    main()
