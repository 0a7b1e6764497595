"""Autotuner of the batched path.

Picks the tiling of a batch and, where the caller allows it, the sweeps per
swap stage M. The tiling is the number of beta slots each workgroup holds
(which fixes the workgroups per ladder) and the slots each thread sweeps. The
tuner times short runs of every feasible candidate on scratch contexts and
caches the winner as JSON, keyed by the batch's shape and the GPU
architecture.

Every tiling realises the same chain bit for bit, because random numbers are
keyed by site, sweep, slot and seed and never by thread or workgroup. So the
tiling is chosen on speed alone. M is different: it changes the Markov chain
(Algorithm 1 runs M sweeps between swap stages), so a faster M is no gain if
it samples worse. The caller's first M is the reference; another M is taken
only if it is faster and, on held-out runs of the same batch (other seeds,
the same number of sweeps), its mean best energy is no higher than the
reference's. A tuned M is returned to the caller, who must run every path
that is compared with the batch (the oracle, the plain path) with the same M.

Timing uses the chunk-kernel HIP events of the batch (pt_batch_kernel_time)
and is argument marshalling plus arithmetic on the host only.
"""
from __future__ import annotations

import json
import os
import time

from . import binding

G_CANDIDATES = (1, 2, 4, 8, 16, 32, 64)
RPT_CANDIDATES = (1, 2, 4)


def arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def batch_key(contexts, extra=""):
    """Cache key: the multiset of (kind, L or n, R) of the batch plus arch."""
    shapes = {}
    for c in contexts:
        k = (c.kind, c.L if c.kind == "lattice" else c.n, c.R)
        shapes[k] = shapes.get(k, 0) + 1
    parts = [f"{kind}:{size}:R{R}x{cnt}" for (kind, size, R), cnt in sorted(shapes.items())]
    return f"{arch()}|" + ",".join(parts) + (f"|{extra}" if extra else "")


def candidates(contexts):
    """(replicas_per_wg, replicas_per_thread, kernel) triples worth timing:
    every cap on the slots per workgroup up to the longest ladder, with 1, 2
    or 4 slots per thread in the workgroup-synchronous kernel (the runtime
    lowers the cap per context until it fits; general graphs sweep one slot
    per thread, from the LDS graph or from either packed-row layout), the
    wave-per-replica kernel where every context is an 8^3 lattice, the +-J
    8^3 kernel (two slots or one slot per wavefront) where every coupling is
    +-1 and every ladder has even length, and the +-J row kernel (one slot
    per wavefront, any even L in 6..16, sizes mixed) where every coupling is
    +-1, and the one-slot-per-wavefront sparse kernel for general graphs."""
    rmax = max(c.R for c in contexts)
    wave_ok = all(c.kind == "lattice" and c.L == 8 for c in contexts)
    pm_ok = all(getattr(c, "pm", False) for c in contexts)
    csr_ok = all(c.kind != "lattice" for c in contexts)
    pml_ok = all(getattr(c, "pml", False) for c in contexts)
    out = []
    for G in G_CANDIDATES:
        if G > 2 * rmax:
            continue
        for rpt in RPT_CANDIDATES:
            if rpt <= G and (rpt == 1 or not csr_ok):
                out.append((G, rpt, "block"))
        if csr_ok:
            out.append((G, 1, "row"))
            out.append((G, 1, "row4"))
        if wave_ok and G <= 8:
            out.append((G, 1, "wave"))
        if pm_ok and 2 <= G <= 16:
            out.append((G, 1, "pm"))
        if pm_ok and G <= 8:
            out.append((G, 1, "pm1"))

    if pml_ok:   # one slot per wavefront: every workgroup size up to 8 wavefronts, or the runtime's per size
        out += [(G, 1, "pml") for G in range(0, 9) if G <= rmax]
    if csr_ok:   # the same for general graphs
        out += [(G, 1, "csrw") for G in range(1, 9) if G <= rmax]
    return out


def _attempts_per_sweep(contexts):
    return sum(c.R * c.nfree for c in contexts)


def time_tiling(contexts, G, rpt, kernel="auto", warm=200, timed=600, chunk=None):
    """attempts/ns of the chunk kernel for one tiling, or None if infeasible."""
    try:
        bt = binding.Batch(contexts, replicas_per_wg=G, replicas_per_thread=rpt,
                           chunk_sweeps=chunk or timed, kernel=kernel)
    except binding.TaptError:
        return None
    try:
        bt.sweep(warm)
        bt.kernel_time()
        bt.sweep(timed)
        ms, launches = bt.kernel_time()
    finally:
        bt.close()
    if launches == 0 or ms <= 0:
        return None
    return _attempts_per_sweep(contexts) * timed / (ms * 1e6)


def mean_best_energy(make_contexts, M, tiling, sweeps, seed_offset=1_000_003):
    """Mean best energy over the batch after ``sweeps`` sweeps with M sweeps
    per cycle, on scratch contexts whose seeds are shifted by seed_offset
    (runs held out from the timing)."""
    ctxs = make_contexts(M, seed_offset=seed_offset)
    try:
        bt = binding.Batch(ctxs, replicas_per_wg=tiling["replicas_per_wg"],
                           replicas_per_thread=tiling["replicas_per_thread"], chunk_sweeps=min(sweeps, 1000),
                           kernel=tiling["kernel"])
        bt.sweep(sweeps)
        bt.close()
        return float(sum(c.summary()["best"] for c in ctxs)) / len(ctxs)
    finally:
        for c in ctxs:
            c.close()


def tune(make_contexts, Ms=(1,), cache=None, key_extra="", warm=200, timed=600, log=None, quality_sweeps=2000):
    """Choose (M, replicas_per_wg, replicas_per_thread) for a batch.

    make_contexts(M) returns fresh scratch binding.Context objects of the
    batch's shape with M sweeps per cycle (they are run and discarded); with
    several Ms it must also accept ``seed_offset`` (held-out runs for the
    quality check of a faster M).
    cache: JSON file path or None. Returns a dict with the choice, its rate
    and the timed scan.
    """
    Ms = tuple(int(m) for m in Ms)
    probe = make_contexts(Ms[0])
    key = batch_key(probe, f"M{'/'.join(map(str, Ms))}" + (f"|{key_extra}" if key_extra else ""))
    table = {}
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except ValueError:
            table = {}
        if key in table:
            for c in probe:
                c.close()
            return dict(table[key], cached=True, key=key)
    scan = []
    for i, M in enumerate(Ms):
        ctxs = probe if i == 0 else make_contexts(M)
        for G, rpt, kern in candidates(ctxs):
            t0 = time.perf_counter()
            rate = time_tiling(ctxs, G, rpt, kern, warm, timed)
            if log:
                log(f"autotune M={M} G={G} rpt={rpt} {kern}: "
                    f"{'infeasible' if rate is None else f'{rate:.1f} attempts/ns'} ({time.perf_counter() - t0:.2f} s)")
            if rate is not None:
                scan.append(dict(M=M, replicas_per_wg=G, replicas_per_thread=rpt, kernel=kern,
                                 attempts_per_ns=round(rate, 2)))
        for c in ctxs:
            c.close()
    if not scan:
        raise binding.TaptError(binding.PT_EUNSUPPORTED, "no feasible tiling for this batch")
    best = max(scan, key=lambda d: d["attempts_per_ns"])
    quality = {}
    if len(Ms) > 1 and best["M"] != Ms[0]:
        # a faster M must sample no worse than the reference M on held-out runs
        ref = max((d for d in scan if d["M"] == Ms[0]), key=lambda d: d["attempts_per_ns"], default=None)
        quality = {Ms[0]: mean_best_energy(make_contexts, Ms[0], ref, quality_sweeps) if ref else None,
                   best["M"]: mean_best_energy(make_contexts, best["M"], best, quality_sweeps)}
        if log:
            log(f"autotune quality check over {quality_sweeps} sweeps: mean best energy {quality}")
        if ref is not None and quality[best["M"]] > quality[Ms[0]]:
            best = ref
    res = dict(M=best["M"], replicas_per_wg=best["replicas_per_wg"],
               replicas_per_thread=best["replicas_per_thread"], kernel=best["kernel"],
               attempts_per_ns=best["attempts_per_ns"], scan=scan,
               quality={str(k): v for k, v in quality.items()})
    if cache:
        table[key] = res
        tmp = cache + ".tmp"
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(res, cached=False, key=key)
