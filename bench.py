#!/usr/bin/env python3
"""Benchmark of the TAPT hot path on one MI355X.

Workload: 64 synthetic 3D Edwards-Anderson +-J instances, L = 8 periodic
(512 int8 spins), 32 replicas on a geometric beta ladder 0.2..3.0, Metropolis,
one sweep per swap stage, proposals every 100 sweeps on the 30 hottest slots
from per-slot banks of 256 configurations produced by plain-PT runs of the same
instance. One step = 10^4 sweeps of the whole batch (every step of
Algorithm 1: sweeps, proposal stages, swap stages, best tracking); the default
10 timed steps are the 10^5-sweep run.

Prints one JSON line: batched attempts/ns (value), the plain
one-instance-per-launch path on the same chain (bit-identical final state),
the LDS roofline of the chunk kernel (with the ALU one beside it) from HIP
events, and the CPU oracle baseline on every core of this host. Beside it:
the mixed-size workload (40 EA instances, L = 6..16, R = 24..48, 10^5
sweeps, autotuned tiling), the factorization workload (64 8x8-bit
multipliers, R = 32, 10^4 sweeps, then time to the ground energy) and the
continuous-batching server under Poisson arrivals.
"""
import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/ns (batched vs plain) + p50/p99 time-to-target per request"
# algorithmic integer VALU issue slots per single-spin attempt on the +-J cubic
# lattice: 6 multiply-accumulates for the local field, 2 for dE/2 = m I and the
# table index, 10 for one eighth of a Philox4x32-10 call (10 rounds of two
# 32x32->64 multiplies, each at half rate so two slots, and four XORs; the key
# schedule is uniform and runs on the scalar unit; 8 uniforms per call) and 3
# for compare, flip and energy.
OPS_PER_ATTEMPT = 6 + 2 + 10 + 3
# int32 VALU lane slots/s: 128 lanes/clk/CU (two wave64 instructions per clock
# per CU, the rate of the fp32 vector peak, 157.3 TFLOP/s = 2 x 128 x 256 x 2.4
# GHz) x 256 CUs x 2.4 GHz. The probe issues 1.66 v_xor_b32 and 0.91
# v_mul_hi_u32 / 0.87 v_mad_u64_u32 wave instructions per clock per CU.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
VALU_PEAK_SOURCE = ("128 int32 lanes/clk/CU x 256 CUs x 2.4 GHz (32-bit multiplies issue at half rate and "
                    "count two slots); the VALU probe (bench.py --workload probe) issues 1.66 v_xor_b32 "
                    "wave instructions per clock per CU of the 2.0 this assumes")
LDS_BYTES_PER_ATTEMPT = 14                       # 6 neighbour spins + 6 couplings + own spin read + write
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12          # 256 B/clk/CU x 256 CUs x 2.4 GHz
LDS_PEAK_SOURCE = ("256 B/clk/CU (CDNA4 LDS reads, twice CDNA3's 128) x 256 CUs x 2.4 GHz; the LDS probe "
                   "(bench.py --workload probe) reads 137 TB/s with ds_read_b128, above the 78.6 TB/s "
                   "a 128 B/clk LDS could give")
HBM_PEAK_TBS = 8.0


def csr_bytes_per_attempt(problem):
    """Algorithmic LDS bytes of one attempt on a general sparse graph: per
    bond the neighbour spin (1 B), the coupling (1 B) and its int16 index
    (2 B), plus the own spin read and write, averaged over the free sites."""
    rp = np.asarray(problem["row_ptr"])
    free = np.asarray(problem["clamp"]) == 0
    deg = np.diff(rp)[free]
    return float(4 * deg.mean() + 2)


def csr_ops_per_attempt(problem):
    """Algorithmic VALU issue slots of one attempt on a general sparse graph:
    one multiply-accumulate per bond (mean degree of the free sites), the
    field term, and the 2 + 10 + 3 of the lattice count (dE and table index,
    an eighth of a Philox call, compare / flip / energy)."""
    rp = np.asarray(problem["row_ptr"])
    free = np.asarray(problem["clamp"]) == 0
    return float(np.diff(rp)[free].mean() + 1 + 2 + 10 + 3)


def rooflines(attempts_per_launch, avg_ms, lds_bytes, ops=OPS_PER_ATTEMPT, traffic=None, kernel=None):
    """LDS roofline (the target bound) with the ALU one beside it, for one
    kernel: algorithmic bytes / ops per launch over the measured launch time."""
    sec = avg_ms * 1e-3
    lds = lds_bytes * attempts_per_launch / sec / 1e12
    alu = ops * attempts_per_launch / sec / 1e12
    fr = dict(lds=lds / LDS_PEAK_TBS, alu=alu / VALU_PEAK_TOPS)
    if traffic is not None:
        fr["hbm"] = traffic / sec / 1e12 / HBM_PEAK_TBS
    return dict(bound="lds", achieved=round(lds, 3), peak=round(LDS_PEAK_TBS, 1), unit="TB/s",
                frac=round(lds / LDS_PEAK_TBS, 4), traffic=traffic, kernel=kernel, avg_launch_ms=round(avg_ms, 4),
                bytes_per_attempt=round(lds_bytes, 2), peak_source=LDS_PEAK_SOURCE,
                alu=dict(achieved=round(alu, 3), peak=round(VALU_PEAK_TOPS, 1), unit="TOP/s",
                         frac=round(alu / VALU_PEAK_TOPS, 4), ops_per_attempt=ops,
                         peak_source=VALU_PEAK_SOURCE),
                measured_binding=max(fr, key=fr.get),
                fractions={k: round(v, 4) for k, v in fr.items()})


SWEEP_KERNELS = ("chunk_kernel", "pm_kernel", "pml_kernel", "csrw_kernel", "plain_", "wave_kernel")


def rocprof_summary(d):
    """Markdown tables of a rocprofv3 ``-f csv`` output directory: the kernel
    statistics, the sweep-kernel dispatches grouped by (kernel, grid, block,
    LDS, VGPRs), and each counter's mean per dispatch grouped by (kernel,
    grid)."""
    import collections
    import csv
    import glob

    def files(pat):
        return sorted(glob.glob(os.path.join(d, "**", pat), recursive=True))

    def col(r, *names):
        return next((r[n] for n in names if n in r), "")

    def sweep(name):
        return any(k in name for k in SWEEP_KERNELS)

    out = []
    for f in files("*kernel_stats.csv"):
        out += ["### kernel stats\n", "| kernel | calls | total ms | avg ms | min ms | max ms | % |",
                "|---|---|---|---|---|---|---|"]
        for r in list(csv.DictReader(open(f)))[:12]:
            out.append(f"| `{r['Name'][:100]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                       f"{float(r['AverageNs']) / 1e6:.4f} | {float(r['MinNs']) / 1e6:.4f} | "
                       f"{float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f} |")
    for f in files("*kernel_trace.csv"):
        g = collections.defaultdict(list)
        for r in csv.DictReader(open(f)):
            if not sweep(r["Kernel_Name"]):
                continue
            key = (r["Kernel_Name"][:100], col(r, "Grid_Size", "Grid_Size_X"),
                   col(r, "Workgroup_Size", "Workgroup_Size_X"), col(r, "LDS_Block_Size", "Lds_Size"),
                   col(r, "VGPR_Count", "Arch_VGPR_Count"))
            g[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
        out += ["\n### sweep-kernel dispatches by launch shape\n",
                "| kernel | grid | block | LDS B | VGPRs | dispatches | mean ms | min ms | max ms |",
                "|---|---|---|---|---|---|---|---|---|"]
        for k, v in sorted(g.items(), key=lambda kv: -sum(kv[1]))[:12]:
            out.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {k[3]} | {k[4]} | {len(v)} | {sum(v) / len(v):.4f} | "
                       f"{min(v):.4f} | {max(v):.4f} |")
    for f in files("*counter_collection.csv"):
        g = collections.defaultdict(lambda: collections.defaultdict(float))
        ids = collections.defaultdict(set)
        for r in csv.DictReader(open(f)):
            if not sweep(r["Kernel_Name"]):
                continue
            key = (r["Kernel_Name"][:100], col(r, "Grid_Size", "Grid_Size_X"))
            did = col(r, "Dispatch_Id", "Correlation_Id")
            g[key][(did, r["Counter_Name"])] += float(r["Counter_Value"])
            ids[key].add(did)
        out += ["\n### counters per dispatch (mean over the dispatches of each launch shape)\n",
                "| kernel | grid | dispatches | counter | mean per dispatch |", "|---|---|---|---|---|"]
        for key in sorted(g, key=lambda k: -len(ids[k]))[:6]:
            per = collections.defaultdict(list)
            for (_, cname), v in g[key].items():
                per[cname].append(v)
            for cname in sorted(per):
                vals = per[cname]
                out.append(f"| `{key[0]}` | {key[1]} | {len(ids[key])} | {cname} | {sum(vals) / len(vals):.4g} |")
    return "\n".join(out)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps-per-step", type=int, default=10_000)
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--L", type=int, default=8)
    ap.add_argument("--R", type=int, default=32)
    ap.add_argument("--bank", type=int, default=256)
    ap.add_argument("--workload", default="pt",
                    choices=("pt", "mixed", "fact", "plain", "probe", "bankgen-sg", "bankgen-fact", "tts",
                             "context"),
                    help="pt: the batched PT benchmark (default); mixed / fact / plain: only the mixed-size, "
                         "the factorization or the plain-path leg (for profiling); probe: LDS read "
                         "bandwidth and VALU issue rates of the device; "
                         "bankgen-*: the long-run MCMC bank "
                         "generation of Supp. Table S3 (3D spin glass L=10, or 16-bit factorization); "
                         "tts: the factorization TTS study; context: the proposal-context ablation")
    ap.add_argument("--ctx-instances", type=int, default=16, help="context: spin-glass instances")
    ap.add_argument("--ctx-runs", type=int, default=16, help="context: independent runs per instance and variant")
    ap.add_argument("--ctx-sweeps", type=int, default=5000, help="context: sweeps per run")
    ap.add_argument("--ctx-completion", type=int, default=20, help="context: completion sweeps per proposal")
    ap.add_argument("--bank-samples", type=int, default=100_000, help="bankgen: chains (samples) per bank")
    ap.add_argument("--tts-bits", default="16,18,20", help="tts: product bit lengths (even)")
    ap.add_argument("--tts-instances", type=int, default=8, help="tts: semiprimes per size")
    ap.add_argument("--tts-runs", type=int, default=100, help="tts: independent runs per instance and method")
    ap.add_argument("--tts-tmax", type=int, default=20_000, help="tts: longest run length, sweeps")
    ap.add_argument("--tts-bank", type=int, default=1024, help="tts: MCMC bank samples per proposal slot")
    ap.add_argument("--tts-bank-burn-in", type=int, default=10_000, help="tts: burn-in of each bank sample")
    ap.add_argument("--tts-ladder", default="adaptive", choices=("adaptive", "geometric"),
                    help="tts: adaptive (uniform swap acceptance, fitted per size on the first instance) "
                         "or geometric 0.2..3.0")
    ap.add_argument("--bank-burn-in", type=int, default=0, help="bankgen: burn-in sweeps (0: the paper's)")
    ap.add_argument("--sweeps-per-swap", type=int, default=1,
                    help="M, sweeps per swap stage (the workload's value is 1; must divide 100)")
    ap.add_argument("--tiling", default="auto", help="'auto' or G,rpt[,kernel] (slots per workgroup, per thread; "
                                                     "kernel auto|block|wave)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=1500)
    ap.add_argument("--calib-copy", action="store_true", help="also run a 256 MiB device copy (PMC scaling)")
    ap.add_argument("--rocprof-summary", default=None, metavar="DIR",
                    help="print markdown tables of a rocprofv3 csv output directory (kernel stats, sweep-kernel "
                         "dispatches by launch shape, counters per dispatch) and exit; uses no GPU")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-size workload")
    ap.add_argument("--no-fact", action="store_true", help="skip the factorization workload")
    ap.add_argument("--mixed-sweeps", type=int, default=100_000, help="mixed: timed sweeps")
    ap.add_argument("--plain-sweeps", type=int, default=2000, help="plain: sweeps of the plain-path leg")
    ap.add_argument("--leg-tiling", default=None,
                    help="mixed / fact legs: G,rpt,kernel instead of the autotuner's choice (for profiling)")
    ap.add_argument("--leg-bank", type=int, default=256,
                    help="mixed / fact legs: bank entries per slot (the workloads' 256; fewer for profiling)")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000", help="Poisson arrival rates, req/s")
    ap.add_argument("--serve-requests", default="1000,1000,1000,1000,1000", help="requests per rate")
    ap.add_argument("--serve-pipeline", action="store_true",
                    help="serving: enqueue each round before retiring the last (one more round before a request joins)")
    ap.add_argument("--serve-cap", type=int, default=100_000, help="sweep cap per request")
    ap.add_argument("--serve-ref-runs", type=int, default=8,
                    help="independent PT runs per spin-glass instance that set its reference energy")
    ap.add_argument("--serve-ref-sweeps", type=int, default=50_000, help="sweeps of each reference run")
    ap.add_argument("--serve-chunk", type=int, default=250, help="sweeps per serving round")
    ap.add_argument("--bank-cache", default=None,
                    help="file to save the generated banks to, or load them from when it exists")
    return ap.parse_args()


def problems(n_inst, L, R):
    from paper_2509_23043_amd import inputs
    probs = [inputs.ea_lattice(L, 2000 + i) for i in range(n_inst)]
    betas = inputs.geometric_ladder(R)
    return probs, betas


def make_banks(probs, betas, B, n_prop_slots, log):
    """Per-slot banks from plain-PT runs (no proposals) of each instance:
    10^4 burn-in sweeps, then one sample of every slot every 100 sweeps."""
    import torch
    from paper_2509_23043_amd import binding
    n = probs[0]["n"]
    R = len(betas)
    gens = [binding.Context(p, betas, seed=1_000_000 + i) for i, p in enumerate(probs)]
    bt = binding.Batch(gens, chunk_sweeps=2000)
    bt.sweep(10_000)
    bank = torch.empty((len(probs), n_prop_slots, B, n), dtype=torch.int8, device="cuda")
    tmp = torch.empty((R, n), dtype=torch.int8, device="cuda")
    for k in range(B):
        bt.sweep(100)
        for i, g in enumerate(gens):
            g.state_device(tmp.data_ptr())
            bank[i, :, k, :] = tmp[:n_prop_slots]
        if (k + 1) % 64 == 0:
            log(f"bank samples {k + 1}/{B}")
    torch.cuda.synchronize()
    log(f"banks: {len(probs)} x {n_prop_slots} slots x {B} configs")
    bt.close()
    for g in gens:
        g.close()
    return bank


def build_contexts(probs, betas, bank, seeds, M=1):
    from paper_2509_23043_amd import binding, workloads
    ctxs = []
    for i, p in enumerate(probs):
        c = binding.Context(p, betas, seed=seeds[i], M=M, prop_start=100, prop_period=100,
                            target=workloads.ea_target(p["n"]))
        for r in range(bank.shape[1]):
            c.propose_device(r, bank[i, r].data_ptr(), bank.shape[2])
        ctxs.append(c)
    return ctxs


def tune_tiling(probs, betas, bank, log, M=1):
    """The autotuner's choice of tiling on scratch contexts of the same batch
    (M is fixed by the workload: one sweep per swap stage unless asked)."""
    from paper_2509_23043_amd import autotune

    def make(m):
        return build_contexts(probs, betas, bank, [7 + i for i in range(len(probs))], M=m)

    res = autotune.tune(make, Ms=(M,), warm=300, timed=1500, log=log)
    return res


def _cpu_worker(args):
    idx, L, R, seed, bank, sweeps = args
    import oracle
    from paper_2509_23043_amd import inputs
    p = inputs.ea_lattice(L, 2000 + idx)
    betas = inputs.geometric_ladder(R)
    banks = {r: bank[r] for r in range(bank.shape[0])}
    run = oracle.Run(p, betas, seed=seed, banks=banks, prop_start=100, prop_period=100, check_energy=False)
    t0 = time.perf_counter()
    run.run(sweeps)
    return time.perf_counter() - t0, sweeps * R * L ** 3


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(bank_host, L, R, sweeps, log):
    """The oracle on every core this process may use: one process per core,
    each running one instance of the workload (instance i % 64 with its bank),
    timed from the first start to the last finish."""
    cores = len(os.sched_getaffinity(0))
    jobs = [(i % len(bank_host), L, R, 3000 + i, bank_host[i % len(bank_host)], sweeps) for i in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        out = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    attempts = sum(a for _, a in out)
    single = np.mean([a / t for t, a in out]) / 1e9
    rate = attempts / max(t for t, _ in out) / 1e9
    log(f"cpu oracle: {cores} processes on {cores} cores ({cpu_model()}), {attempts:.3g} attempts, "
        f"{wall:.1f} s wall, {rate:.4f} attempts/ns ({single:.4f} per core)")
    return dict(value=round(rate, 5), unit="attempts/ns", cores=cores, processes=cores, cpu_model=cpu_model(),
                kind="oracle", single_core_value=round(single, 5),
                cpu_seconds=round(sum(t for t, _ in out), 1),
                sample=f"{cores} instances (one oracle process per core), {sweeps} sweeps each of the same "
                       f"workload with proposals every 100 sweeps and the GPU run's banks")


KERNEL_SOURCES = {"pm": "kernels_pm.hip", "pm1": "kernels_pm.hip", "wave": "kernels_wave.hip", "block": "kernels.hip"}


def kernel_source_hash(kern="pm"):
    """Hash of the device sources that make up one kernel (a counter file
    taken on another version of that kernel does not apply)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_23043_amd", "csrc")
    for f in ("tapt_dev.h", "sweep.h", KERNEL_SOURCES[kern]):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


KERNEL_NAMES = {"pm": "pm_kernel<2>", "pm1": "pm_kernel<1>", "wave": "wave_kernel<8>", "block": "chunk_kernel<LatSweep<8,*>>"}


def traffic_from_profiles(launch_sweeps, kern_hash, kern):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on these sources with this launch length."""
    tag = {"pm": "pm_kernel", "pm1": "pm_kernel_spw1", "wave": "wave_kernel", "block": "chunk_kernel"}[kern]
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}_ea_l8_r32_x64.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kern_hash or d.get("sweeps_per_launch") != launch_sweeps:
        return None
    return d.get("hbm_bytes_per_launch")


def pt_banks(cases, B, log, seed0, burn=10_000, every=100):
    """Banks [n_prop, B, n] (device tensors, one per case) from plain-PT runs
    of each instance with no proposals: ``burn`` sweeps, then one sample of
    every banked slot every ``every`` sweeps. One batch for all the cases."""
    import torch
    from paper_2509_23043_amd import binding
    gens = [binding.Context(c["g"], c["betas"], seed=seed0 + c["k"]) for c in cases]
    bt = binding.Batch(gens, chunk_sweeps=2000)
    bt.sweep(burn)
    banks = [torch.empty((c["n_prop"], B, c["g"]["n"]), dtype=torch.int8, device="cuda") for c in cases]
    tmp = [torch.empty((len(c["betas"]), c["g"]["n"]), dtype=torch.int8, device="cuda") for c in cases]
    for k in range(B):
        bt.sweep(every)
        for c, g, t, b in zip(cases, gens, tmp, banks):
            g.state_device(t.data_ptr())
            b[:, k, :] = t[:c["n_prop"]]
    torch.cuda.synchronize()
    bt.close()
    for g in gens:
        g.close()
    log(f"banks: {len(cases)} instances x {B} configs per banked slot")
    return banks


def case_contexts(cases, cfg, banks, M=1, target=True):
    from paper_2509_23043_amd import binding, workloads
    ctxs = []
    for c, b in zip(cases, banks if banks is not None else [None] * len(cases)):
        kw = workloads.run_kwargs(cfg, c)
        kw["M"] = M
        if not target:
            kw.pop("target")
        ctx = binding.Context(c["g"], c["betas"], seed=c["seed"], **kw)
        if b is not None:
            for r in range(b.shape[0]):
                ctx.propose_device(r, b[r].data_ptr(), b.shape[1])
        ctxs.append(ctx)
    return ctxs


def timed_batch(ctxs, tiling, sweeps, chunk, warm_chunks=1):
    """attempts/ns of a batch over ``sweeps`` sweeps after a warm-up, with the
    chunk kernel's average launch time from its HIP events."""
    import torch
    from paper_2509_23043_amd import binding
    G, rpt, kern = tiling
    bt = binding.Batch(ctxs, replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=chunk, kernel=kern)
    for _ in range(warm_chunks):
        bt.sweep(chunk)
    torch.cuda.synchronize()
    bt.kernel_time()
    t0 = time.perf_counter()
    bt.sweep(sweeps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, launches = bt.kernel_time()
    bt.close()
    att = sweeps * sum(c.R * c.nfree for c in ctxs)
    return dict(value=att / dt / 1e9, seconds=dt, attempts=att, avg_ms=ms / max(launches, 1), launches=launches)


def tuned_tiling(cases, cfg, log, fixed=None):
    """The autotuner's tiling, or a fixed G,rpt,kernel string (profiling)."""
    from paper_2509_23043_amd import autotune
    if fixed:
        G, rpt, kern = fixed.split(",")
        return (int(G), int(rpt), kern), []
    res = autotune.tune(lambda M: case_contexts(cases, cfg, None, M=M), Ms=(1,), warm=200, timed=1000, log=log)
    return (res["replicas_per_wg"], res["replicas_per_thread"], res["kernel"]), res["scan"]


def mixed_leg(args, log):
    """The mixed-size workload: 40 EA +-J instances (8 each of L = 6, 8, 10,
    12, 16 with ladders of 24..48 slots) in one persistent launch sequence,
    10^5 sweeps, proposals every 50 sweeps from 256-entry plain-PT banks on
    all but the two coldest slots, tiling from the autotuner (M = 1)."""
    from paper_2509_23043_amd import workloads
    cfg = workloads.EA_MIXED
    cases = workloads.ea_cases(cfg)
    t0 = time.perf_counter()
    banks = pt_banks(cases, args.leg_bank, log, seed0=1_300_000)
    log(f"mixed: banks in {time.perf_counter() - t0:.1f} s")
    tiling, scan = tuned_tiling(cases, cfg, log, args.leg_tiling)
    ctxs = case_contexts(cases, cfg, banks)
    r = timed_batch(ctxs, tiling, args.mixed_sweeps, cfg["chunk"])
    for c in ctxs:
        c.close()
    log(f"mixed: {r['value']:.1f} attempts/ns over {args.mixed_sweeps} sweeps, tiling {tiling}, "
        f"chunk kernel {r['avg_ms']:.3f} ms avg")
    roof = rooflines(r["attempts"] / max(r["launches"], 1), r["avg_ms"], LDS_BYTES_PER_ATTEMPT,
                     kernel={"pml": "pml_kernel", "auto": "chunk_kernel_mixed", "block": "chunk_kernel_mixed"}.get(
                         tiling[2], tiling[2]))
    return dict(value=round(r["value"], 2), unit="attempts/ns", sweeps=args.mixed_sweeps,
                seconds=round(r["seconds"], 3), attempts_per_sweep=sum(len(c["betas"]) * c["g"]["n"] for c in cases),
                instances=len(cases), sizes=[list(x) for x in cfg["sizes"]], sweeps_per_swap=1,
                tiling=dict(replicas_per_wg=tiling[0], replicas_per_thread=tiling[1], kernel=tiling[2]),
                tiling_scan=[dict(G=d["replicas_per_wg"], rpt=d["replicas_per_thread"], kernel=d["kernel"],
                                  attempts_per_ns=d["attempts_per_ns"]) for d in scan],
                roofline=roof,
                workload="3D EA +-J L in {6,8,10,12,16} x 8 instances, R = 24/30/36/42/48 beta 0.2..3.0 "
                         f"geometric, Metropolis, M=1, proposals every 50 sweeps from {args.leg_bank}-entry plain-PT "
                         "banks on all but the 2 coldest slots; one persistent launch sequence of 10^4-sweep launches")


def factorization_leg(args, log):
    """The factorization workload: 64 distinct products of two primes in
    [128, 256) as 8x8-bit multipliers (200 spins, 176 free), R = 32,
    proposals every 100 sweeps from 256-entry plain-PT banks on the 23
    hottest slots. Throughput over 10^4 sweeps; then fresh runs until every
    product reaches its ground energy (cap 10^5 sweeps): sweeps to solve per
    product and their device time within the 64-product batch."""
    import torch
    from paper_2509_23043_amd import binding, workloads
    cfg = workloads.MULT8
    cases = workloads.fact_cases(cfg)
    t0 = time.perf_counter()
    banks = pt_banks(cases, args.leg_bank, log, seed0=1_400_000)
    log(f"factorization: banks in {time.perf_counter() - t0:.1f} s")
    tiling, scan = tuned_tiling(cases, cfg, log, args.leg_tiling)
    ctxs = case_contexts(cases, cfg, banks)
    r = timed_batch(ctxs, tiling, cfg["sweeps"], 2000)
    for c in ctxs:
        c.close()
    bpa = csr_bytes_per_attempt(cases[0]["g"])
    log(f"factorization: {r['value']:.1f} attempts/ns over {cfg['sweeps']} sweeps, tiling {tiling}, "
        f"chunk kernel {r['avg_ms']:.3f} ms avg")
    roof = rooflines(r["attempts"] / max(r["launches"], 1), r["avg_ms"], bpa, ops=csr_ops_per_attempt(cases[0]["g"]),
                     kernel={"csrw": "csrw_kernel", "row": "chunk_kernel<CsrRowSweep>",
                             "row4": "chunk_kernel<CsrRowQuadSweep>"}.get(tiling[2], "chunk_kernel<CsrSweep>"))
    # time to solution: fresh contexts, chunks of 1000 sweeps until every
    # product has hit its ground energy or the cap
    ctxs = case_contexts(cases, cfg, banks)
    G, rpt, kern = tiling
    bt = binding.Batch(ctxs, replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=1000, kernel=kern)
    bt.kernel_time()
    done, hits = 0, [-1] * len(ctxs)
    while done < cfg["solve_cap"] and min(hits) < 0:
        bt.sweep(1000)
        done += 1000
        hits = [c.summary()["first_hit"] for c in ctxs]
    ms, _ = bt.kernel_time()
    bt.close()
    best = [c.summary() for c in ctxs]
    solved = [h for h in hits if h >= 0]
    ok = all(inputs_factor(cases[k], best[k]["best_spins"]) for k in range(len(cases)) if hits[k] >= 0)
    for c in ctxs:
        c.close()
    ms_per_sweep = ms / done
    sw = np.array([h if h >= 0 else np.inf for h in hits], float)
    med = float(np.median(sw))
    log(f"factorization: {len(solved)}/{len(hits)} solved within {done} sweeps, median {med:g} sweeps "
        f"({med * ms_per_sweep:.1f} ms of the batch), factors checked: {ok}")
    torch.cuda.synchronize()
    return dict(value=round(r["value"], 2), unit="attempts/ns", sweeps=cfg["sweeps"], seconds=round(r["seconds"], 3),
                products=len(cases), replicas=cfg["R"], banked_slots=cfg["n_prop"], lds_bytes_per_attempt=round(bpa, 2),
                tiling=dict(replicas_per_wg=G, replicas_per_thread=rpt, kernel=kern),
                tiling_scan=[dict(G=d["replicas_per_wg"], rpt=d["replicas_per_thread"], kernel=d["kernel"],
                                  attempts_per_ns=d["attempts_per_ns"]) for d in scan],
                roofline=roof,
                solve=dict(cap=cfg["solve_cap"], sweeps_run=done, solved=len(solved), products=len(hits),
                           median_sweeps=None if not math.isfinite(med) else med,
                           p90_sweeps=None if not math.isfinite(float(np.percentile(sw, 90)))
                           else float(np.percentile(sw, 90)),
                           batch_ms_per_sweep=round(ms_per_sweep, 5),
                           median_seconds=None if not math.isfinite(med) else round(med * ms_per_sweep / 1e3, 5),
                           factors_checked=ok,
                           note="seconds = sweeps to the ground energy x device time per sweep of the "
                                "64-product batch"),
                workload="8x8-bit array multipliers (200 spins, 176 free) of 64 distinct semiprimes, R=32 beta "
                         "0.2..3.0 geometric, Metropolis, M=1, DSATUR colors, proposals every 100 sweeps from "
                         f"{args.leg_bank}-entry plain-PT banks on the 23 hottest slots")


def inputs_factor(case, spins):
    """The factor bits of a ground state multiply to the product."""
    from paper_2509_23043_amd import inputs
    A = inputs.bits_to_int(spins, case["g"]["a_idx"])
    B = inputs.bits_to_int(spins, case["g"]["b_idx"])
    return A * B == case["C"]


def serving_pool(args, log):
    """Problems of the mixed serving workload, each a registered context with
    proposal banks and a residual-energy target.

    Spin glasses: 3D EA +-J, L in {6, 8, 10, 12, 16}, 8 instances per size,
    ladders of 24/30/36/42/48 slots (beta 0.2..3.0 geometric), proposals every
    50 sweeps on all but the two coldest slots. Factorization: m x m-bit
    multipliers, m = 8..12, 4 semiprimes per size, 32 slots, proposals on the
    23 hottest. Banks: 64 configurations per slot from a plain-PT run of the
    instance (10^4 burn-in sweeps, then one sample every 100 sweeps). The EA
    reference energy E_ref is the lowest energy of ``--serve-ref-runs``
    independent plain-PT runs of ``--serve-ref-sweeps`` sweeps (seeds apart
    from the bank run and from every request), and the target is E_ref plus
    1% of N rounded up to the energy grid (multiples of 4); the factorization
    target is the ground energy -3m^2 - 4m(m-1), reached exactly by the
    factor pairs."""
    import torch
    from paper_2509_23043_amd import banks as bankmod
    from paper_2509_23043_amd import binding, inputs
    B, burn, every = 64, 10_000, 100
    specs = []
    for L, R in ((6, 24), (8, 30), (10, 36), (12, 42), (16, 48)):
        for i in range(8):
            specs.append(dict(kind="ea", size=L, g=inputs.ea_lattice(L, 5100 + 10 * L + i),
                              betas=inputs.geometric_ladder(R), slots=R - 2, period=50))
    for m in range(8, 13):
        for i, (C, _p, _q) in enumerate(inputs.semiprimes(m, 4, seed=5200 + m)):
            specs.append(dict(kind="fact", size=m, g=inputs.multiplier(m, C),
                              betas=inputs.geometric_ladder(32), slots=round(13 * 32 / 18), period=50,
                              target=-3 * m * m - 4 * m * (m - 1)))
    # plain-PT bank runs, one batch per shape (each fits the co-resident limit)
    t0 = time.perf_counter()
    groups = {}
    for k, sp in enumerate(specs):
        groups.setdefault((sp["kind"], sp["size"]), []).append(k)
    for key, idx in groups.items():
        gens = [binding.Context(specs[k]["g"], specs[k]["betas"], seed=2_000_000 + k) for k in idx]
        bt = binding.Batch(gens, chunk_sweeps=2000)
        bt.sweep(burn)
        banks = [torch.empty((specs[k]["slots"], B, specs[k]["g"]["n"]), dtype=torch.int8, device="cuda")
                 for k in idx]
        tmp = [torch.empty((len(specs[k]["betas"]), specs[k]["g"]["n"]), dtype=torch.int8, device="cuda")
               for k in idx]
        for j in range(B):
            bt.sweep(every)
            for q, g in enumerate(gens):
                g.state_device(tmp[q].data_ptr())
                banks[q][:, j, :] = tmp[q][:specs[idx[q]]["slots"]]
        torch.cuda.synchronize()
        for q, k in enumerate(idx):
            specs[k]["bank"] = banks[q]
        bt.close()
        for g in gens:
            g.close()
    log(f"serving pool: {len(specs)} problems, banks in {time.perf_counter() - t0:.1f} s")
    # reference energies of the spin glasses from independent long runs
    t0 = time.perf_counter()
    ea = [k for k, sp in enumerate(specs) if sp["kind"] == "ea"]
    refs = [binding.Context(specs[k]["g"], specs[k]["betas"], seed=3_000_000 + 100 * k + j)
            for k in ea for j in range(args.serve_ref_runs)]
    owner = [k for k in ea for _ in range(args.serve_ref_runs)]
    for group, bt in bankmod._batches(refs, lambda grp: binding.Batch(grp, chunk_sweeps=5000)):
        bt.sweep(args.serve_ref_sweeps)
        bt.close()
    eref = {}
    for k, c in zip(owner, refs):
        eref[k] = min(eref.get(k, 1 << 30), int(c.summary()["best"]))
        c.close()
    for k in ea:
        n = specs[k]["g"]["n"]
        slack = -(-((n + 99) // 100) // 4) * 4
        specs[k]["eref"] = eref[k]
        specs[k]["target"] = eref[k] + slack
    log(f"serving pool: reference energies from {args.serve_ref_runs} x {args.serve_ref_sweeps}-sweep runs per "
        f"spin glass in {time.perf_counter() - t0:.1f} s")
    ctxs = []
    for sp in specs:
        c = binding.Context(sp["g"], sp["betas"], seed=0, prop_start=sp["period"], prop_period=sp["period"])
        for r in range(sp["slots"]):
            c.propose_device(r, sp["bank"][r].data_ptr(), B)
        ctxs.append(c)
    return specs, ctxs


def serving_leg(args, log):
    """Poisson arrivals of mixed requests (70% spin glass with L uniform over
    the five sizes, 30% factorization with m uniform over 8..12) into the
    continuous-batching server; time-to-target per request = completion seen
    by the host minus arrival."""
    from paper_2509_23043_amd import binding
    specs, ctxs = serving_pool(args, log)
    ea = {}
    fa = {}
    for k, sp in enumerate(specs):
        (ea if sp["kind"] == "ea" else fa).setdefault(sp["size"], []).append(k)
    rates = [float(x) for x in args.serve_rates.split(",")]
    counts = [int(x) for x in args.serve_requests.split(",")]
    out = []
    srv = binding.Server(chunk_sweeps=args.serve_chunk, mem_budget=8 << 30, pipeline=args.serve_pipeline)
    pids = [srv.register(c) for c in ctxs]
    seed_base = 5000
    for lam, nreq in zip(rates, counts):
        rng = np.random.Generator(np.random.PCG64(5000 + int(lam)))
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=nreq))
        picks = []
        for _ in range(nreq):
            if rng.random() < 0.7:
                size = sorted(ea)[rng.integers(len(ea))]
                picks.append(ea[size][rng.integers(len(ea[size]))])
            else:
                size = sorted(fa)[rng.integers(len(fa))]
                picks.append(fa[size][rng.integers(len(fa[size]))])
        st0 = srv.stats()
        t_start = srv.clock()
        results = []
        i = 0
        while len(results) < nreq:
            now = srv.clock() - t_start
            while i < nreq and arrivals[i] <= now:
                k = picks[i]
                srv.submit(pids[k], seed_base + i, args.serve_cap, target=specs[k]["target"],
                           want_best=False, user_tag=k)
                i += 1
            wait = 1 if i < nreq else 50
            if i < nreq:
                wait = max(0, min(50, int((arrivals[i] - (srv.clock() - t_start)) * 1000)))
            results += srv.poll(256, wait_ms=wait)
        seed_base += nreq
        st1 = srv.stats()
        wall = max(r["t_done"] for r in results) - t_start
        ok = [r for r in results if r["status"] == 0]
        hits = [r for r in ok if r["hit"]]
        pct = lambda v, q: round(float(np.percentile(v, q)), 4) if len(v) else None
        done_t = [r["t_done"] - r["t_submit"] for r in ok]
        hit_t = [r["t_done"] - r["t_submit"] for r in hits]
        by_kind = {}
        for kind in ("ea", "fact"):
            mine = [r for r in ok if specs[r["user_tag"]]["kind"] == kind]
            h = [r["t_done"] - r["t_submit"] for r in mine if r["hit"]]
            dn = [r["t_done"] - r["t_submit"] for r in mine]
            by_kind[kind] = dict(n=len(mine), hit_frac=round(len(h) / max(len(mine), 1), 4),
                                 p50_time_to_done_s=pct(dn, 50), p99_time_to_done_s=pct(dn, 99),
                                 p50_time_to_target_s=pct(h, 50), p99_time_to_target_s=pct(h, 99))
        busy = (st1["busy_s"] - st0["busy_s"]) / max(wall, 1e-9)
        gpu_busy = (st1["gpu_busy_s"] - st0["gpu_busy_s"]) / max(wall, 1e-9)
        d = dict(rate_req_per_s=lam, requests=nreq, completed=len(ok), rejected=nreq - len(ok),
                 hit_frac=round(len(hits) / max(len(ok), 1), 4), cap_frac=round(1 - len(hits) / max(len(ok), 1), 4),
                 p50_time_to_done_s=pct(done_t, 50), p99_time_to_done_s=pct(done_t, 99),
                 p50_time_to_target_s=pct(hit_t, 50), p99_time_to_target_s=pct(hit_t, 99),
                 completed_req_per_s=round(len(ok) / wall, 2),
                 attempts_per_ns=round((st1["attempts"] - st0["attempts"]) / (wall * 1e9), 2),
                 round_busy_frac=round(busy, 4), gpu_busy_frac=round(gpu_busy, 4),
                 rounds=st1["rounds"] - st0["rounds"],
                 peak_active=st1["peak_active"], peak_lanes=st1["peak_lanes"], by_kind=by_kind)
        log(f"serving lambda={lam:g}: done p50 {d['p50_time_to_done_s']} s p99 {d['p99_time_to_done_s']} s; "
            f"target p50 {d['p50_time_to_target_s']} s p99 {d['p99_time_to_target_s']} s; "
            f"{d['completed_req_per_s']} req/s, hit {d['hit_frac']} (ea {by_kind['ea']['hit_frac']}, "
            f"fact {by_kind['fact']['hit_frac']}), {d['attempts_per_ns']} attempts/ns, "
            f"round busy {d['round_busy_frac']}, GPU busy {d['gpu_busy_frac']}, peak active {d['peak_active']}")
        out.append(d)
    srv.stop()
    for c in ctxs:
        c.close()
    return dict(rates=out, sweep_cap=args.serve_cap, chunk_sweeps=args.serve_chunk, pipelined=bool(args.serve_pipeline),
                pool="40 EA +-J (L=6..16, 8 each, R=24..48) + 20 multipliers (m=8..12, 4 each, R=32); "
                     "banks 64/slot from plain-PT runs; EA target = E_ref + 1% N on the grid of 4, E_ref the "
                     f"best of {args.serve_ref_runs} independent {args.serve_ref_sweeps}-sweep plain-PT runs; "
                     "factorization target = ground energy",
                mix="70% EA (L uniform), 30% factorization (m uniform)",
                latency="time to done = host sees the result minus arrival, over every completed request "
                        "(hits and capped ones); time to target over the hits only",
                reference_energies={str(sp["size"]) + "_" + str(k): sp["eref"] for k, sp in enumerate(specs)
                                    if sp["kind"] == "ea"})


# Supp. Table S3: one complete 10^5-sample bank for one (instance, beta), with
# the burn-in per sample, the spin count and the total time the paper
# reports; the update rate is derived as samples x burn-in x spins / time.
PAPER_BANKGEN = {
    "bankgen-sg": dict(spins=999, burn_in=10_000, samples=100_000, seconds=16.23),
    "bankgen-fact": dict(spins=200, burn_in=100_000, samples=100_000, seconds=38.24),
}


def bankgen(args, log):
    """Long-run MCMC bank generation (Supp. Table S3): independent chains at
    one beta, each from its own random start, one configuration kept after
    the burn-in. Timed end to end (contexts, sweeps, state read-back)."""
    import torch
    from paper_2509_23043_amd import banks, binding, inputs
    torch.cuda.set_device(0)
    binding.lib()
    ref = PAPER_BANKGEN[args.workload]
    burn = args.bank_burn_in or ref["burn_in"]
    if args.workload == "bankgen-sg":
        g = inputs.ea_lattice(10, 5100)
        beta = 1.0
        what = f"3D EA +-J L=10 (1000 spins), beta {beta}"
    else:
        ps = inputs.primes_in(128, 256)
        g = inputs.multiplier(8, ps[3] * ps[17])
        beta = 1.0
        what = f"8x8-bit multiplier (16-bit product, {g['n']} spins), beta {beta}"
    timing = {}
    # warm-up: one small bank (kernel load, first-touch allocations)
    banks.generate_bank(g, beta, 2048, 10, seed=1)
    # the runtime's own choice: the +-J row kernel for the lattice, the
    # workgroup-synchronous sparse kernel at 32 chains per workgroup for the
    # multiplier (independent chains)
    cfg, E = banks.generate_bank(g, beta, args.bank_samples, burn, seed=77, timing=timing)
    value = timing["attempts"] / timing["wall_s"] / 1e9
    paper_rate = ref["samples"] * ref["burn_in"] * ref["spins"] / ref["seconds"] / 1e9
    log(f"{args.workload}: {args.bank_samples} chains x {burn} sweeps in {timing['wall_s']:.2f} s "
        f"({timing['sweep_s']:.2f} s of sweep kernels): {value:.1f} attempts/ns; paper {paper_rate:.1f}")
    out = dict(metric="single-spin update attempts/ns, long-run MCMC bank generation (Supp. Table S3)",
               value=round(value, 2), unit="attempts/ns", n_gpus=1, steps=1, warmup=1,
               ms_per_step=round(timing["wall_s"] * 1e3, 1), higher_is_better=True, scaling="weak",
               vs_baseline=round(value / paper_rate, 3), dtype="int8", data="synthetic",
               config=dict(workload=f"{what}: {args.bank_samples} independent chains, each from its own "
                                    f"random start, {burn} burn-in sweeps, one sample kept per chain",
                           samples=args.bank_samples, burn_in=burn, spins=g["n"],
                           sweep_kernel_s=round(timing["sweep_s"], 3), wall_s=round(timing["wall_s"], 3),
                           mean_energy=float(np.mean(E))),
               paper=dict(total_s=ref["seconds"], samples=ref["samples"], burn_in=ref["burn_in"],
                          spins=ref["spins"], derived_attempts_per_ns=round(paper_rate, 1),
                          hardware="NVIDIA RTX 6000 Ada (context only, not the target)"))
    print(json.dumps(out), flush=True)


def tts_study(args, log):
    """Reduced TTS scaling study on factorization (Supp. TTS methodology):
    PT vs TAPT with long-run MCMC proposal banks on the 13 hottest of 18
    slots, proposals every sweep; median TTS per size with bootstrap CIs and
    the fitted exponent k of TTS(n) = A exp(k n)."""
    import torch
    from paper_2509_23043_amd import banks, binding, inputs, ladder, tts
    torch.cuda.set_device(0)
    binding.lib()
    R, NPROP = 18, 13
    betas0 = inputs.geometric_ladder(R)
    grid = [t for t in (250, 500, 1000, 2000, 5000, 10_000, 20_000, 50_000, 100_000) if t <= args.tts_tmax]
    sizes = [int(b) for b in args.tts_bits.split(",")]
    res = {"pt": {}, "tapt": {}}
    ladders = {}
    t0 = time.perf_counter()
    for n_bits in sizes:
        m = n_bits // 2
        egnd = -3 * m * m - 4 * m * (m - 1)
        insts = inputs.semiprimes(m, args.tts_instances, seed=9100 + m)
        betas = betas0
        if args.tts_ladder == "adaptive":
            # one ladder per size, fitted on the first instance and fixed for every run
            betas, hist = ladder.adapt(inputs.multiplier(m, insts[0][0]), betas0, rounds=8, sweeps=4000,
                                       runs=4, seed=m)
            log(f"tts {n_bits}-bit ladder: swap acceptance spread {hist[0][1].std():.3f} -> "
                f"{hist[-1][1].std():.3f} (mean {hist[-1][1].mean():.3f})")
            ladders[n_bits] = [round(float(x), 5) for x in betas]
        per = {"pt": [], "tapt": []}
        succ = {"pt": [], "tapt": []}
        for i, (C, p, q) in enumerate(insts):
            g = inputs.multiplier(m, C)
            bank = {r: banks.generate_bank(g, betas[r], args.tts_bank, args.tts_bank_burn_in,
                                           seed=500_000 + 1000 * i + 37 * r)[0] for r in range(NPROP)}
            for method, bk in (("pt", None), ("tapt", bank)):
                hits, dt = tts.run_instance(g, betas, args.tts_runs, args.tts_tmax, seed=10_000 * i + 7,
                                            target=egnd, banks=bk)
                star, t_a = tts.tts_star(hits, grid)
                per[method].append(star * dt)
                succ[method].append(tts.success_probability(hits, args.tts_tmax))
                log(f"tts {n_bits}-bit instance {i} {method}: success at t_max {succ[method][-1]:.2f}, "
                    f"TTS {star * dt:.3g} s")
        for method in ("pt", "tapt"):
            v = np.array(per[method])
            lo, hi = tts.bootstrap_median_ci(v, seed=n_bits)
            med = float(np.median(v))
            res[method][n_bits] = dict(median_tts_s=med, ci95=[lo, hi],
                                       mean_success_at_tmax=round(float(np.mean(succ[method])), 3),
                                       solved_instances=int(np.sum(np.isfinite(v))))
            log(f"tts {n_bits}-bit {method}: median {med:.3g} s [{lo:.3g}, {hi:.3g}], "
                f"success at t_max {np.mean(succ[method]):.2f}")
    fits = {}
    for method in ("pt", "tapt"):
        ns = [n for n in sizes if math.isfinite(res[method][n]["median_tts_s"])]
        fits[method] = None
        if len(ns) >= 3:                  # two points fit any exponent exactly
            A, k = tts.fit_exponential(ns, [res[method][n]["median_tts_s"] for n in ns])
            fits[method] = dict(A=A, k=round(k, 4), sizes=ns)
    k_tapt = fits["tapt"]["k"] if fits["tapt"] else None
    fin = lambda x: None if isinstance(x, float) and not math.isfinite(x) else x
    clean = lambda d: {str(k): {kk: ([fin(x) for x in vv] if isinstance(vv, list) else fin(vv))
                                for kk, vv in v.items()} for k, v in d.items()}
    out = dict(metric="fitted TTS scaling exponent k, TTS(n) = A exp(k n), factorization, TAPT with MCMC banks",
               value=k_tapt, unit="1/bit", n_gpus=1, steps=1, warmup=0,
               ms_per_step=round((time.perf_counter() - t0) * 1e3, 1), higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="int8", data="synthetic",
               config=dict(workload=f"semiprimes of two m-bit primes, product bits {sizes}, {args.tts_instances} "
                                    f"instances per size, {args.tts_runs} runs each, t_a in {grid}, R={R} "
                                    f"{args.tts_ladder} ladder on 0.2..3.0, proposals every sweep on the {NPROP} "
                                    f"hottest slots from "
                                    f"{args.tts_bank}-sample MCMC banks ({args.tts_bank_burn_in} burn-in sweeps)"),
               fits=fits, pt=clean(res["pt"]), tapt=clean(res["tapt"]), ladders=ladders,
               paper=dict(k_pt=0.846, k_tapt=0.564, sizes=[16, 18, 20, 22, 24], instances=440, runs=400,
                          note="Supp. TTS scaling; adaptive ladders and 10^5-sample banks; context only"))
    print(json.dumps(out), flush=True)


def context_study(args, log):
    """Proposal-context ablation (Supp., Fig. S4b) on 3D spin glasses: PT,
    TAPT with long-run MCMC bank proposals (no context), and contextual
    proposals that clamp 12.5%, 25% or 50% of the slot's current spins and
    complete the rest by MCMC from the bank entry. Residual energy per spin
    of each run's best energy at checkpoints, against the lowest energy any
    run found on the instance, and the chain's sweep throughput."""
    import torch
    from paper_2509_23043_amd import banks, binding, inputs
    torch.cuda.set_device(0)
    binding.lib()
    L, R, NPROP, B, PERIOD = 10, 22, 20, 128, 10
    n = L ** 3
    betas = inputs.geometric_ladder(R)
    T = args.ctx_sweeps
    checkpoints = [t for t in (100, 250, 500, 1000, 2000, 5000, 10_000) if t < T] + [T]
    variants = [("pt", None), ("bank", 0.0), ("ctx12.5", 0.125), ("ctx25", 0.25), ("ctx50", 0.5)]
    t0 = time.perf_counter()
    insts = [inputs.ea_lattice(L, 7000 + i) for i in range(args.ctx_instances)]
    bank_sets = []
    for i, g in enumerate(insts):
        bank_sets.append({r: banks.generate_bank(g, betas[r], B, 10_000, seed=800_000 + 1000 * i + 37 * r)[0]
                          for r in range(NPROP)})
    log(f"context: {len(insts)} instances, {NPROP} banks of {B} samples each in {time.perf_counter() - t0:.1f} s")
    best = {}
    rate = {}
    for name, frac in variants:
        ctxs = []
        for i, g in enumerate(insts):
            for k in range(args.ctx_runs):
                kw = {} if frac is None else dict(prop_start=PERIOD, prop_period=PERIOD)
                c = binding.Context(g, betas, seed=90_000 + 100 * i + k, **kw)
                if frac is not None:
                    for r, b in bank_sets[i].items():
                        c.propose(r, b)
                    if frac > 0:
                        c.set_context(frac, args.ctx_completion)
                ctxs.append(c)
        traj = np.zeros((len(ctxs), len(checkpoints)), np.int64)
        make = lambda group: binding.Batch(group, chunk_sweeps=min(250, checkpoints[0]))
        ms = 0.0
        at = 0
        # batches of as many runs as stay co-resident, one after the other
        for group, bt in banks._batches(ctxs, make):
            bt.kernel_time()
            done = 0
            for j, t in enumerate(checkpoints):
                bt.sweep(t - done)
                done = t
                traj[at:at + len(group), j] = [c.summary()["best"] for c in group]
            ms += bt.kernel_time()[0]
            at += len(group)
            bt.close()
        rate[name] = len(ctxs) * R * n * T / (ms * 1e6)
        best[name] = traj.reshape(len(insts), args.ctx_runs, len(checkpoints))
        for c in ctxs:
            c.close()
        log(f"context {name}: {rate[name]:.1f} attempts/ns of chain sweeps")
    eref = np.min([best[v][:, :, -1].min(axis=1) for v, _ in variants], axis=0)     # per instance
    rho = {v: [(best[v][:, :, j] - eref[:, None]).mean() / n for j in range(len(checkpoints))] for v, _ in variants}
    for v, _ in variants:
        log(f"context {v}: rho_E " + ", ".join(f"t={t}: {r:.5f}" for t, r in zip(checkpoints, rho[v])))
    out = dict(metric="residual energy per spin at t_max, TAPT with MCMC bank proposals (no context)",
               value=round(float(rho["bank"][-1]), 6), unit="energy/spin", n_gpus=1, steps=1, warmup=0,
               ms_per_step=round((time.perf_counter() - t0) * 1e3, 1), higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="int8", data="synthetic",
               config=dict(workload=f"3D EA +-J L={L}, {len(insts)} instances x {args.ctx_runs} runs per variant, "
                                    f"R={R} geometric 0.2..3.0, proposals every {PERIOD} sweeps on the {NPROP} "
                                    f"hottest slots from {B}-sample MCMC banks (10^4 burn-in), contextual "
                                    f"completion {args.ctx_completion} sweeps, {T} sweeps; rho_E against the "
                                    f"lowest energy any run found per instance"),
               checkpoints=checkpoints,
               rho_E={v: [round(float(x), 6) for x in rho[v]] for v, _ in variants},
               attempts_per_ns={v: round(float(x), 2) for v, x in rate.items()})
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.rocprof_summary:
        print(rocprof_summary(args.rocprof_summary))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); instances would shard "
              f"across GPUs with no communication between them", file=sys.stderr)
        sys.exit(2)
    if args.workload == "tts":
        tts_study(args, lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True))
        return
    if args.workload == "context":
        context_study(args, lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True))
        return
    if args.workload == "probe":
        import torch
        from paper_2509_23043_amd import binding
        torch.cuda.set_device(0)
        binding.lib()
        rows = []
        for nbytes in (16, 8):
            for bpc in (1, 2, 3, 4, 5):
                tb, ms = binding.probe_lds(nbytes, bpc, 4096)
                rows.append(dict(read=f"ds_read_b{8 * nbytes}", workgroups_per_cu=bpc, threads=256,
                                 TBps=round(tb, 2), ms=round(ms, 3)))
                print(f"[bench] ds_read_b{8 * nbytes}, {bpc} workgroups of 256 per CU: {tb:.2f} TB/s", file=sys.stderr,
                      flush=True)
        valu = {}
        for op, name in ((0, "v_xor_b32"), (1, "v_mul_hi_u32"), (2, "v_mul_lo_u32"), (3, "v_mad_u64_u32")):
            rate, ms = binding.probe_valu(op, 4096)
            valu[name] = round(rate, 4)
            print(f"[bench] {name}: {rate:.3f} wave-instructions per clock per CU", file=sys.stderr, flush=True)
        best = max(r["TBps"] for r in rows)
        print(json.dumps(dict(metric="LDS read bandwidth", value=best, unit="TB/s", peak=round(LDS_PEAK_TBS, 1),
                              frac=round(best / LDS_PEAK_TBS, 4), rows=rows,
                              valu_wave_instr_per_clk_per_cu=valu)), flush=True)
        return
    if args.workload == "plain":
        import torch
        from paper_2509_23043_amd import binding
        torch.cuda.set_device(0)
        binding.lib()
        log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
        probs, betas = problems(1, args.L, args.R)
        bank = make_banks(probs, betas, args.bank, args.R - 2, log)
        ctx = build_contexts(probs, betas, bank, [3000], M=args.sweeps_per_swap)[0]
        ctx.sweep(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.sweep(args.plain_sweeps)
        dt = time.perf_counter() - t0
        v = args.plain_sweeps * args.R * args.L ** 3 / dt / 1e9
        log(f"plain: {v:.4f} attempts/ns over {args.plain_sweeps} sweeps")
        print(json.dumps(dict(metric="plain path attempts/ns", value=round(v, 4), unit="attempts/ns",
                              sweeps=args.plain_sweeps)), flush=True)
        return
    if args.workload in ("mixed", "fact"):
        import torch
        from paper_2509_23043_amd import binding
        torch.cuda.set_device(0)
        binding.lib()
        log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)
        leg = mixed_leg(args, log) if args.workload == "mixed" else factorization_leg(args, log)
        print(json.dumps(leg), flush=True)
        return
    if args.workload != "pt":
        bankgen(args, lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True))
        return
    import torch
    from paper_2509_23043_amd import binding

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    binding.lib()
    L, R, NI, S = args.L, args.R, args.instances, args.sweeps_per_step
    M = args.sweeps_per_swap
    if M < 1 or 100 % M:
        sys.exit("--sweeps-per-swap must divide the proposal period (100)")
    n = L ** 3
    n_prop = R - 2
    probs, betas = problems(NI, L, R)
    t0 = time.perf_counter()
    if args.bank_cache and os.path.exists(args.bank_cache):
        bank = torch.load(args.bank_cache, weights_only=True).cuda()
        assert tuple(bank.shape) == (NI, n_prop, args.bank, n), bank.shape
        log(f"banks loaded from {args.bank_cache}")
    else:
        bank = make_banks(probs, betas, args.bank, n_prop, log)
        log(f"bank generation {time.perf_counter() - t0:.1f} s")
        if args.bank_cache:
            torch.save(bank.cpu(), args.bank_cache)

    if args.tiling == "auto":
        tuned = tune_tiling(probs, betas, bank, log, M=M)
        G, rpt, kern = tuned["replicas_per_wg"], tuned["replicas_per_thread"], tuned["kernel"]
        scan = tuned["scan"]
    else:
        parts = args.tiling.split(",")
        G, rpt = int(parts[0]), int(parts[1])
        kern = parts[2] if len(parts) > 2 else "auto"
        scan = []
    log(f"tiling: {G} slots per workgroup, {rpt} per thread, kernel {kern}")

    seeds = [3000 + i for i in range(NI)]
    ctxs = build_contexts(probs, betas, bank, seeds, M=M)
    bt = binding.Batch(ctxs, replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=S, kernel=kern)
    for _ in range(args.warmup):
        bt.sweep(S)
    torch.cuda.synchronize()
    bt.kernel_time()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.sweep(S)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = bt.kernel_time()
    attempts = args.steps * S * NI * R * n
    value = attempts / dt / 1e9
    ms_step = dt * 1e3 / args.steps
    log(f"batched: {value:.1f} attempts/ns, {ms_step:.2f} ms/step, chunk kernel {kern_ms / max(launches, 1):.3f} ms avg")

    # the plain path on instance 0, same seed and bank: same chain, compared bit for bit
    plain = None
    if not args.no_plain:
        p_ctx = build_contexts(probs[:1], betas, bank[:1], seeds[:1], M=M)[0]
        total = (args.warmup + args.steps) * S
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_ctx.sweep(total)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        p_att = total * R * n
        s_plain, _ = p_ctx.state()
        s_batch, _ = ctxs[0].state()
        same = bool(np.array_equal(s_plain, s_batch) and np.array_equal(p_ctx.energies(), ctxs[0].energies()))
        res_b = ctxs[0].summary()["best"]
        plain = dict(value=round(p_att / pdt / 1e9, 4), unit="attempts/ns", sweeps=total,
                     instances=1, identical_final_state=same, best_energy=int(p_ctx.summary()["best"]),
                     best_energy_batched=int(res_b))
        log(f"plain: {plain['value']} attempts/ns over {total} sweeps, identical={same}")
        if not same:
            log("ERROR: plain and batched chains differ")
            sys.exit(1)
        plain["speedup"] = round(value / plain["value"], 1)

    if args.calib_copy:
        a = torch.ones(1 << 28, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # rooflines of the chunk kernel from its own HIP events
    avg_ms = kern_ms / max(launches, 1)
    att_launch = attempts / max(launches, 1)
    ran = kern if kern != "auto" else ("pm" if ctxs[0].pm else "wave")
    kern_hash = kernel_source_hash(ran)
    roof = rooflines(att_launch, avg_ms, LDS_BYTES_PER_ATTEMPT, traffic=traffic_from_profiles(S, kern_hash, ran),
                     kernel=KERNEL_NAMES[ran])
    roof["launches"] = launches

    mixed = fact = None
    if not args.no_mixed or not args.no_fact:
        for c in ctxs:
            c.close()
        bt.close()
        ctxs = []
    if not args.no_mixed:
        mixed = mixed_leg(args, log)
    if not args.no_fact:
        fact = factorization_leg(args, log)

    serving = None
    if not args.no_serve:
        for c in ctxs:
            c.close()
        if ctxs:
            bt.close()
        serving = serving_leg(args, log)

    cpu = None
    if not args.no_cpu:
        bank_host = bank[:16].cpu().numpy()
        cpu = cpu_baseline(bank_host, L, R, args.cpu_sweeps, log)

    out = dict(metric=METRIC, value=round(value, 2), unit="attempts/ns", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="int8", data="synthetic",
               config=dict(workload=f"3D EA +-J L={L} ({n} spins) x {NI} instances, {R} replicas beta 0.2..3.0 "
                                    f"geometric, Metropolis, M={M}, proposals every 100 sweeps from {args.bank}-entry "
                                    f"plain-PT banks on {n_prop} slots (bank energies computed once when the banks "
                                    f"are installed, before the timed region); {S} sweeps per step",
                           instances=NI, L=L, replicas=R, sweeps_per_step=S, sweeps_per_swap=M, bank=args.bank,
                           tiling=dict(replicas_per_wg=G, replicas_per_thread=rpt, kernel=kern)),
               plain=plain, roofline=roof, cpu_baseline=cpu, mixed=mixed, factorization=fact,
               tiling_scan=[dict(G=d["replicas_per_wg"], rpt=d["replicas_per_thread"], kernel=d["kernel"],
                                 attempts_per_ns=d["attempts_per_ns"]) for d in scan],
               serving=serving)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
