#!/usr/bin/env python3
"""SU(3) x SU(3) streaming benchmark on one MI355X.

A step is one evaluation of z(x) = x(x) * y(x) over a 48^4 lattice of SU(3)
matrices stored in double precision, structure-of-arrays layout (the
streaming test of Section 4, Listing 3).  Inputs are seeded synthetic
Haar-random SU(3) fields already resident in HBM; the timed region is K
back-to-back launches bracketed by device synchronisation.

Prints ONE JSON line on stdout (progress and launch settings go to stderr):
  value        achieved GB/s = 432 B/site * V / (time per step)
  roofline     the dominant kernel against the 8 TB/s HBM peak, timed with
               HIP events on the launch stream; traffic from the committed
               PMC summary (null if the kernel changed since)
  cpu_baseline the FP64 oracle on the host cores, on a bounded sample
  variants     every other configuration, each in GB/s of its own
               algorithmic bytes and % of 8 TB/s, with the oracle's rate on
               the same inputs beside it ("cpu": [all threads, one thread],
               GB/s of the same byte accounting): the tuned bandwidth
               ceilings (triad, read-only, write-only, copy), the precision
               forms at 48^4 (with their error against the FP64 product),
               the layouts, the volume sweep (hot and cold), the t-slab
               shard, the precision forms at 32^4, the shifted operands,
               the Wilson hopping term, Grid's virtual-node layout,
               expression programs, fused vs chained expressions at 32^4
               (hot and cold) and the 64-lattice batch (persistent and
               one-shot grids, graph replays; 64 small lattices batched
               against separate launches); each variant time is the
               median over --repeats blocks of K launches (default 5)

`--only a,b` runs just those sections (precision, fused, ceiling, dslash,
batch, shift, programs) with the tuned or cached launches, for profiler
runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
MALL_BYTES = 268435456  # the 256 MiB Infinity Cache
METRIC = ("SU(3)×SU(3) achieved HBM GB/s (% of peak) at 48^4, "
          "FP64 vs FP32/compressed")

# algorithmic bytes per site: every operand read once, the result written
# once, in its stored format
BYTES_PER_SITE = {0: 432, 1: 216, 2: 108, 3: 144}   # MUL by precision
FLOPS_PER_SITE = {0: 198, 1: 396, 2: 414, 3: 18, 4: 234}
REAL_BYTES = {0: 8, 1: 4, 2: 2, 3: 4}
# Wilson hopping term, keyed (spinor precision, link precision): four link
# matrices + input and output spinors once each; the customary 1320 flops
# per site (8 hops of 12 projection + 132 colour + 24 accumulation flops,
# less the first accumulation)
DSLASH_BYTES_PER_SITE = {(0, 0): 960, (1, 1): 480, (1, 3): 384}
DSLASH_FLOPS_PER_SITE = 1320
PREC_NAME = {0: "f64", 1: "f32", 2: "f16_f32acc", 3: "c12_f32"}
SECTIONS = ("precision", "fused", "ceiling", "dslash", "batch", "shift", "programs",
            "vnode")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def expr_bytes_per_site(prec, expr):
    E = 6 if prec == 3 else 9
    site = E * 2 * REAL_BYTES[prec]
    nops = {0: 2, 1: 3, 2: 4, 3: 2, 4: 2}[expr]
    return site * (nops + 1)


def gbps(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9


def entry(ms, nbytes, **extra):
    """Compact record of one timing: microseconds, GB/s, % of 8 TB/s."""
    g = gbps(nbytes, ms)
    out = {"us": round(ms * 1e3, 1), "gbps": round(g), "pct": round(100 * g / HBM_PEAK_GBPS, 1)}
    out.update(extra)
    return out


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="blocks of K launches per variant measurement; the "
                         "median is reported (the headline is one block)")
    ap.add_argument("--seed", type=int, default=1710)
    ap.add_argument("--no-variants", action="store_true",
                    help="headline only (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="no autotuning: the library's default launch, or the "
                         "one cached in the file SU3_TUNE_CACHE names")
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run alone (%s), without "
                         "the headline (for profiler runs)" % ", ".join(SECTIONS))
    ap.add_argument("--layout", default="both", choices=("soa", "aosoa64", "both"),
                    help="layouts of the precision, fused and dslash sections")
    ap.add_argument("--lean", action="store_true",
                    help="sections time only their configured kernels (no chained, "
                         "cold or alternative-grid runs), for profiler runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain copies of known size (PMC scaling)")
    return ap.parse_args()


class Timer:
    """Blocks of K launches between two events on `stream`, plus host wall
    time between synchronisations.  A measurement is the median over
    `repeats` blocks (the headline times a single block of exactly K)."""

    def __init__(self, torch, stream, repeats=5):
        self.torch, self.stream, self.repeats = torch, stream, repeats

    def run(self, launch, steps, warmup, repeats=None):
        torch = self.torch
        for _ in range(warmup):
            launch()
        torch.cuda.synchronize()
        per_launch, host_s = [], 0.0
        for _ in range(self.repeats if repeats is None else repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(self.stream)
            for _ in range(steps):
                launch()
            e1.record(self.stream)
            torch.cuda.synchronize()
            host_s += time.perf_counter() - t0
            per_launch.append(e0.elapsed_time(e1) / steps)
        return statistics.median(per_launch), host_s  # ms per launch (events)


# the sources that define the headline kernel (k_site and what it inlines)
HEADLINE_KERNEL_SOURCES = ("su3_device.h", "su3_internal.h", "su3_kprec.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1710_09409_amd", "csrc")
    for name in HEADLINE_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def committed_traffic():
    """Counter-derived HBM bytes per launch of the headline kernel, from the
    committed PMC summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "su3_mult_f64_soa_48x48x48x48_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class CpuLeg:
    """The oracle timed on the host cores beside each configuration.  Jobs
    are queued while the GPU runs and executed after it, so that host work
    never overlaps a GPU measurement.  Each job fills target[key] with
    [GB/s on all the oracle's threads, GB/s on one thread] of the same byte
    accounting as the GPU figure."""

    def __init__(self, enabled):
        self.enabled = enabled
        self.jobs = []
        self.checks = []
        self.orc = None

    def add(self, target, key, fn, nbytes, min_s=0.4):
        if self.enabled:
            self.jobs.append((target, key, fn, nbytes, min_s))

    def check(self, target, key, fn):
        """A post-run comparison of a GPU result with the oracle."""
        if self.enabled:
            self.checks.append((target, key, fn))

    def oracle(self):
        if self.orc is None:
            import oracle
            self.orc = oracle.get()
        return self.orc

    @staticmethod
    def _timed(fn, min_s):
        passes, t0 = 0, time.perf_counter()
        while True:
            fn()
            passes += 1
            el = time.perf_counter() - t0
            if el >= min_s:
                return passes, el

    def rate(self, fn, nbytes, min_s):
        orc = self.oracle()
        threads = orc.threads()
        p, el = self._timed(fn, min_s)
        orc.set_threads(1)
        try:
            p1, el1 = self._timed(fn, min_s)
        finally:
            orc.set_threads(threads)
        return [round(nbytes * p / el / 1e9, 2), round(nbytes * p1 / el1 / 1e9, 3)]

    def run(self):
        if not self.enabled:
            return
        orc = self.oracle()
        t0 = time.perf_counter()
        for target, key, fn, nbytes, min_s in self.jobs:
            target[key] = self.rate(lambda: fn(orc), nbytes, min_s)
        for target, key, fn in self.checks:
            target[key] = fn(orc)
        log(f"cpu leg: {len(self.jobs)} oracle timings and {len(self.checks)} checks "
            f"in {time.perf_counter() - t0:.1f} s on {orc.threads()} threads")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): every "
              "site is independent, so a multi-GPU run would shard the lattice "
              "into t-slabs with no exchange step (the hopping term would add "
              "a t-face halo)", file=sys.stderr)
        sys.exit(2)
    only = [s for s in args.only.split(",") if s]
    for s in only:
        if s not in SECTIONS:
            sys.exit(f"unknown section {s!r}; sections: {', '.join(SECTIONS)}")

    import numpy as np
    import torch

    import testgen
    import paper_1710_09409_amd as su3

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    props = torch.cuda.get_device_properties(0)
    log(f"device: {props.name} ({getattr(props, 'gcnArchName', '?')}), "
        f"{props.multi_processor_count} CUs")

    host_cache = {}

    def host_field(V, fid):
        key = (V, fid)
        if key not in host_cache:
            host_cache[key] = testgen.su3_field(V, seed=args.seed, field_id=fid)
        return host_cache[key]

    def make(dims, prec, layout, lanes, fid):
        f = su3.field_tensor(dims, prec, layout, lanes)
        su3.su3_field_upload(f, host_field(testgen.volume(dims), fid), stream)
        return f

    def tune(expr, prec, layout, lanes, dims, label=None):
        if args.no_tune:
            cfg = su3.su3_launch_get(expr, prec, layout, lanes, dims).as_dict()
        else:
            cfg = su3.su3_autotune(expr, prec, layout, lanes, dims, stream).as_dict()
        if label:
            log(f"launch {label}: {cfg}")
        return cfg

    ctx = dict(args=args, su3=su3, torch=torch, np=np, testgen=testgen,
               stream=stream, timer=Timer(torch, stream, args.repeats), make=make, tune=tune,
               host_field=host_field, cpu=CpuLeg(not args.no_cpu_baseline))

    if only:
        out = {}
        for s in only:
            out[s] = SECTION_FUNCS[s](ctx)
        ctx["cpu"].run()
        print(json.dumps(out, separators=(",", ":")), flush=True)
        return

    timer = ctx["timer"]
    # ------------------------------------------------------------ headline
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    F64, SOA = su3.SU3_F64, su3.SU3_LAYOUT_SOA
    log(f"headline: z = x*y, {V} sites, FP64 SoA; generating inputs")
    x = make(dims, F64, SOA, 0, testgen.FID_X)
    y = make(dims, F64, SOA, 0, testgen.FID_Y)
    z = su3.field_tensor(dims, F64, SOA, 0)
    cfg = tune(su3.SU3_EXPR_MUL, F64, SOA, 0, dims, "headline")
    step_bytes = BYTES_PER_SITE[0] * V
    ms_ev, host_s = timer.run(lambda: su3.su3_mult(z, x, y, stream),
                              args.steps, args.warmup, repeats=1)
    ms_per_step = host_s * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = gbps(step_bytes, ms_ev)
    log(f"headline: {ms_ev * 1e3:.1f} us/launch (events), {achieved:.0f} GB/s "
        f"= {100 * achieved / HBM_PEAK_GBPS:.1f}% of 8 TB/s")
    traffic = committed_traffic()
    if args.calibrate_copy:
        nbytes = 1 << 30
        cs = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cd = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        for _ in range(5):
            su3.su3_copy(cd.data_ptr(), cs.data_ptr(), nbytes, stream)
        torch.cuda.synchronize()
        del cs, cd

    ctx.update(x64=x, y64=y, z64=z, ms_f64=ms_ev, headline_bytes=step_bytes)
    variants = {}
    if not args.no_variants:
        variants["ceiling"] = section_ceiling(ctx)
        variants["ceiling"]["headline_of_triad"] = round(
            variants["ceiling"]["triad"]["us"] / (ms_ev * 1e3), 4)
        variants["ceiling"]["headline_of_sum"] = round(
            variants["ceiling"]["sum_48^4"]["us"] / (ms_ev * 1e3), 4)
        run_variants(ctx, variants)

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        ctx["cpu"].run()
        cpu = cpu_baseline(ctx["cpu"], host_field(V, testgen.FID_X),
                           host_field(V, testgen.FID_Y))
        cpu["gpu_over_cpu"] = round(value / cpu["value"], 1)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Haar-random SU(3), seed %d)" % args.seed,
        "config": {
            "workload": "su3_mult z=x*y, 48^4 lattice (5,308,416 sites), FP64 "
                        "storage and arithmetic, SoA layout, 432 B/site",
            "sites": V, "bytes_per_step": step_bytes,
            "flops_per_step": FLOPS_PER_SITE[0] * V,
            "gflops": round(FLOPS_PER_SITE[0] * V / (ms_ev * 1e-3) / 1e9, 1),
            "launch": "block %d, occupancy %d, schedule %d, nontemporal %d, "
                      "sites/lane %d" % (cfg["block"], cfg["occupancy"], cfg["schedule"],
                                         cfg["nontemporal"], cfg["sites_per_lane"]),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": "k_site<MUL> FP64 SoA",
            "avg_launch_us": round(ms_ev * 1e3, 2),
            "bytes_per_launch": step_bytes,
        },
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out, separators=(",", ":")), flush=True)


# ------------------------------------------------------------- sections

def section_ceiling(ctx):
    """The STREAM-style yardsticks over the headline's bytes (arrays of a
    third of 2.29 GB each), each tuned over block, occupancy and store
    policy: triad (2:1 read:write, the product's mix), read-only,
    write-only, copy (1:1); and the tuned sum z = x + y of two 48^4 FP64
    SoA fields, which moves the product's bytes in the product's 27 entry
    planes."""
    su3, torch, stream, timer = ctx["su3"], ctx["torch"], ctx["stream"], ctx["timer"]
    args = ctx["args"]
    nb = 2293235712 // 3  # 764,411,904 bytes per array (the headline's)
    arrs = [torch.ones(nb // 8, dtype=torch.float64, device="cuda") for _ in range(3)]
    a, b, c = (t.data_ptr() for t in arrs)
    steps = max(10, min(args.steps, 50))
    out = {}
    for kind, name, traffic in ((su3.SU3_STREAM_TRIAD, "triad", 3 * nb),
                                (su3.SU3_STREAM_READ, "read", 2 * nb),
                                (su3.SU3_STREAM_WRITE, "write", nb),
                                (su3.SU3_STREAM_COPY, "copy", 2 * nb)):
        if args.no_tune:
            best = None
        else:
            best, _ = su3.su3_stream_autotune(kind, a, b, c, nb, stream)
        ms, _ = timer.run(lambda: su3.su3_stream(kind, a, b, c, 3.0, nb, best, stream),
                          steps, 3)
        cfg = best.as_dict() if best is not None else {}
        out[name] = entry(ms, traffic, block=cfg.get("block"), occ=cfg.get("occupancy"),
                          nt=cfg.get("nontemporal"))
        log(f"ceiling {name}: {out[name]} {cfg}")
    del arrs
    torch.cuda.synchronize()
    # the sum z = x + y of the same fields: the product's bytes and its 27
    # entry planes per wave (18 read, 9 written), without the products
    dims = (48, 48, 48, 48)
    V = ctx["testgen"].volume(dims)
    F64, SOA = su3.SU3_F64, su3.SU3_LAYOUT_SOA
    if "x64" in ctx:
        x, y, z = ctx["x64"], ctx["y64"], ctx["z64"]
    else:
        x = ctx["make"](dims, F64, SOA, 0, ctx["testgen"].FID_X)
        y = ctx["make"](dims, F64, SOA, 0, ctx["testgen"].FID_Y)
        z = su3.field_tensor(dims, F64, SOA, 0)
    cfg = ctx["tune"](su3.SU3_EXPR_ADD, F64, SOA, 0, dims, "ceiling sum")
    ms, _ = timer.run(lambda: su3.su3_fused_eval(z, su3.SU3_EXPR_ADD, [x, y], stream), steps, 3)
    out["sum_48^4"] = entry(ms, 432 * V, block=cfg.get("block"), occ=cfg.get("occupancy"),
                            nt=cfg.get("nontemporal"))
    log(f"ceiling sum z = x + y: {out['sum_48^4']}")
    return out


def section_precision(ctx):
    """z = x*y at 48^4 in FP32, FP16 (FP32 arithmetic) and two-row
    compressed FP32, SoA and AoSoA(64): speed-up over the FP64 product, and
    (SoA) the end-to-end error against the FP64 oracle product."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args, cpu, host_field = ctx["args"], ctx["cpu"], ctx["host_field"]
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    SOA, AOSOA = su3.SU3_LAYOUT_SOA, su3.SU3_LAYOUT_AOSOA
    lays = [("soa", SOA, 0), ("aosoa64", AOSOA, 64)]
    if args.layout != "both":
        lays = [l for l in lays if l[0] == args.layout]
    hx, hy = host_field(V, testgen.FID_X), host_field(V, testgen.FID_Y)
    out = {}
    z64_ref = {}

    def f64_product(orc):
        if "z" not in z64_ref:
            z64_ref["z"] = orc.mult(hx, hy)
        return z64_ref["z"]

    for prec in (su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        for lname, lay, lanes in lays:
            x = make(dims, prec, lay, lanes, testgen.FID_X)
            y = make(dims, prec, lay, lanes, testgen.FID_Y)
            z = su3.field_tensor(dims, prec, lay, lanes)
            tune(su3.SU3_EXPR_MUL, prec, lay, lanes, dims, f"precision {prec} {lname}")
            ms, _ = timer.run(lambda: su3.su3_mult(z, x, y, stream), steps, 3)
            b = BYTES_PER_SITE[prec] * V
            key = f"{PREC_NAME[prec]}_{lname}"
            e = entry(ms, b)
            if "ms_f64" in ctx:
                e["x_f64"] = round(ctx["ms_f64"] / ms, 2)
            out[key] = e
            if lname == "soa" and cpu.enabled:
                zh = su3.su3_field_download(z, stream)

                def err(orc, zh=zh):
                    m = orc.metrics(zh, f64_product(orc))
                    return [float("%.2e" % m["e_max"]), float("%.2e" % m["d_u"])]
                cpu.check(e, "err", err)
                cpu.add(e, "cpu", lambda orc, p=prec: orc.reference(0, p, [hx, hy]), b,
                        min_s=0.3)
            log(f"precision {key}: {e}")
            del x, y, z
    return out


def hot_and_cold(ctx, d, prec, fid_x, fid_y, cpu_rate=True):
    """z = x*y at lattice d (SoA): hot (the same buffers every launch) and
    cold (rotating through k buffer sets of >= 1 GiB in all, so the 256 MiB
    Infinity Cache never holds the next launch's operands)."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args, cpu, host_field = ctx["args"], ctx["cpu"], ctx["host_field"]
    SOA = su3.SU3_LAYOUT_SOA
    steps = max(10, min(args.steps, 50))
    Vd = testgen.volume(d)
    ws = BYTES_PER_SITE[prec] * Vd
    x = make(d, prec, SOA, 0, fid_x)
    y = make(d, prec, SOA, 0, fid_y)
    z = su3.field_tensor(d, prec, SOA, 0)
    tune(su3.SU3_EXPR_MUL, prec, SOA, 0, d, f"{d} prec {prec}")
    ms, _ = timer.run(lambda: su3.su3_mult(z, x, y, stream), steps, 3)
    k = max(2, -(-(1 << 30) // ws))
    sets = [(x, y, z)]
    for _ in range(k - 1):
        xi = su3.field_tensor(d, prec, SOA, 0)
        yi = su3.field_tensor(d, prec, SOA, 0)
        xi.owner.copy_(x.owner)
        yi.owner.copy_(y.owner)
        sets.append((xi, yi, su3.field_tensor(d, prec, SOA, 0)))
    turn = [0]

    def rotating():
        xs, ys, zs = sets[turn[0] % k]
        turn[0] += 1
        su3.su3_mult(zs, xs, ys, stream)

    ms_cold, _ = timer.run(rotating, max(steps, 2 * k), k)
    del sets
    e = entry(ms, ws)
    c = entry(ms_cold, ws)
    e.update(cold_us=c["us"], cold_gbps=c["gbps"], cold_pct=c["pct"], sets=k,
             cached=ws < 2 * MALL_BYTES)
    if cpu_rate:
        hx, hy = host_field(Vd, fid_x), host_field(Vd, fid_y)
        if prec == su3.SU3_F64:
            cpu.add(e, "cpu", lambda orc: orc.mult(hx, hy), ws)
        else:
            cpu.add(e, "cpu", lambda orc: orc.reference(0, prec, [hx, hy]), ws)
    return e


def section_fused(ctx):
    """Fused MUL3 / MULADD on four link fields at 32^4 against chained
    su3_mult (+ ADD) calls, hot and cold (rotating operand sets of >= 1 GiB)."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args, cpu, host_field = ctx["args"], ctx["cpu"], ctx["host_field"]
    SOA, AOSOA = su3.SU3_LAYOUT_SOA, su3.SU3_LAYOUT_AOSOA
    steps = max(10, min(args.steps, 50))
    d = (32, 32, 32, 32)
    Vf = testgen.volume(d)
    hU = [host_field(Vf, testgen.FID_U0 + mu) for mu in range(4)]
    out = {}
    for prec, lname, lay, lanes in ((su3.SU3_F64, "soa", SOA, 0), (su3.SU3_F32, "soa", SOA, 0),
                                    (su3.SU3_F64, "aosoa64", AOSOA, 64),
                                    (su3.SU3_F32, "aosoa64", AOSOA, 64)):
        if args.layout != "both" and lname != args.layout:
            continue
        U = [make(d, prec, lay, lanes, testgen.FID_U0 + mu) for mu in range(4)]
        z = su3.field_tensor(d, prec, lay, lanes)
        t1 = su3.field_tensor(d, prec, lay, lanes)
        t2 = su3.field_tensor(d, prec, lay, lanes)
        for expr, name in ((su3.SU3_EXPR_MUL3, "mul3"), (su3.SU3_EXPR_MULADD, "muladd")):
            nops = 3 if expr == su3.SU3_EXPR_MUL3 else 4
            tune(expr, prec, lay, lanes, d, f"fused {PREC_NAME[prec]} {lname} {name}")
            tune(su3.SU3_EXPR_MUL, prec, lay, lanes, d)
            tune(su3.SU3_EXPR_ADD, prec, lay, lanes, d)
            ms_f, _ = timer.run(lambda: su3.su3_fused_eval(z, expr, U[:nops], stream),
                                steps, 3)
            b = expr_bytes_per_site(prec, expr) * Vf
            key = f"{PREC_NAME[prec]}_{lname}_{name}"
            if args.lean:
                out[key] = entry(ms_f, b)
                continue
            if expr == su3.SU3_EXPR_MUL3:
                def chained():
                    su3.su3_mult(t1, U[0], U[1], stream)
                    su3.su3_mult(z, t1, U[2], stream)
            else:
                def chained():
                    su3.su3_mult(t1, U[0], U[1], stream)
                    su3.su3_mult(t2, U[2], U[3], stream)
                    su3.su3_fused_eval(z, su3.SU3_EXPR_ADD, [t1, t2], stream)
            ms_c, _ = timer.run(chained, steps, 3)
            # cold: operand sets rotating through >= 1 GiB
            k = max(2, -(-(1 << 30) // b))
            sets = [(U[:nops], z)]
            for _ in range(k - 1):
                ops = []
                for u in U[:nops]:
                    f = su3.field_tensor(d, prec, lay, lanes)
                    f.owner.copy_(u.owner)
                    ops.append(f)
                sets.append((ops, su3.field_tensor(d, prec, lay, lanes)))
            turn = [0]

            def rotating():
                ops, zz = sets[turn[0] % k]
                turn[0] += 1
                su3.su3_fused_eval(zz, expr, ops, stream)
            ms_cold, _ = timer.run(rotating, max(steps, 2 * k), k)
            del sets
            e = entry(ms_f, b)
            c = entry(ms_cold, b)
            e.update(chained_us=round(ms_c * 1e3, 1), x_chained=round(ms_c / ms_f, 2),
                     cold_us=c["us"], cold_gbps=c["gbps"], cold_pct=c["pct"], sets=k,
                     cached=b < 2 * MALL_BYTES)
            if lname == "soa":
                if prec == su3.SU3_F64:
                    cpu.add(e, "cpu", lambda orc, x=expr, n=nops: orc.fused(x, hU[:n]), b)
                else:
                    cpu.add(e, "cpu",
                            lambda orc, x=expr, n=nops: orc.reference(x, prec, hU[:n]), b)
            out[key] = e
            log(f"fused {key}: {e}")
        del U, z, t1, t2
    return out


def section_dslash(ctx):
    """The Wilson hopping term at 48^4 (four link fields + input and output
    spinors moved once each)."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args = ctx["args"]
    SOA, AOSOA = su3.SU3_LAYOUT_SOA, su3.SU3_LAYOUT_AOSOA
    steps = max(10, min(args.steps, 50))
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    host_psi = testgen.spinor_field(V, seed=args.seed, field_id=200)
    out = {}
    lays = (("soa", SOA, 0), ("aosoa64", AOSOA, 64))
    if args.layout != "both":
        lays = [l for l in lays if l[0] == args.layout]
    for sp, lp, name in ((su3.SU3_F64, su3.SU3_F64, "f64"), (su3.SU3_F32, su3.SU3_F32, "f32"),
                         (su3.SU3_F32, su3.SU3_C12_F32, "f32_c12")):
        for lname, lay, lanes in lays:
            U = [make(dims, lp, lay, lanes, testgen.FID_U0 + mu) for mu in range(4)]
            fin = su3.spinor_tensor(dims, sp, lay, lanes)
            su3.su3_field_upload(fin, host_psi, stream)
            fout = su3.spinor_tensor(dims, sp, lay, lanes)
            tune(su3.SU3_EXPR_DSLASH, lp, lay, lanes, dims, f"dslash {name} {lname}")
            ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
            b = DSLASH_BYTES_PER_SITE[(sp, lp)] * V
            key = f"{name}_{lname}"
            out[key] = entry(ms, b, tflops=round(DSLASH_FLOPS_PER_SITE * V / ms / 1e9, 2))
            log(f"dslash {key}: {out[key]}")
            del U, fin, fout
    return out


def section_batch(ctx):
    """64 uneven lattices, mixed FP64 and compressed FP32, replayed from one
    HIP graph: the tuned launch, the best persistent grid (k workgroups per
    compute unit looping over the tiles), and 64 separate launches."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args, cpu, host_field = ctx["args"], ctx["cpu"], ctx["host_field"]
    AOSOA = su3.SU3_LAYOUT_AOSOA
    lat = testgen.batch_lattices(64, seed=args.seed)
    # each item's storage: the layout the library recommends for the
    # product at that lattice and precision (AoSoA(64) without tuning)
    rec = {}
    for d, comp in lat:
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        if (d, prec) not in rec:
            if args.no_tune:
                rec[(d, prec)] = (AOSOA, 64)
            else:
                lay, lanes, _, _ = su3.su3_layout_recommend(su3.SU3_EXPR_MUL, prec, d, stream)
                rec[(d, prec)] = (lay, lanes)
    lay_names = {su3.SU3_LAYOUT_SOA: "soa", AOSOA: "aosoa"}
    rec_text = ["%s %s %s%s" % ("x".join(map(str, d)), PREC_NAME[p], lay_names[l], L or "")
                for (d, p), (l, L) in sorted(rec.items())]
    log(f"batch layouts: {rec_text}")
    zs, ops, exprs = [], [], []
    total_bytes = 0
    log("batch: generating 64 lattices")
    for i, (d, comp) in enumerate(lat):
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        lay, lanes = rec[(d, prec)]
        ops.append([make(d, prec, lay, lanes, testgen.FID_BATCH_BASE + 4 * i + k)
                    for k in range(2)])
        zs.append(su3.field_tensor(d, prec, lay, lanes))
        exprs.append(su3.SU3_EXPR_MUL)
        total_bytes += BYTES_PER_SITE[prec] * testgen.volume(d)
    total_sites = sum(testgen.volume(d) for d, _ in lat)
    key = su3.SU3_EXPR_BATCH + su3.SU3_EXPR_MUL
    kprec = su3.SU3_C12_F32 if lat[0][1] else su3.SU3_F64
    klay, klanes = rec[(lat[0][0], kprec)]
    kdims = (total_sites, 1, 1, 1)
    if args.no_tune:
        bcfg = su3.su3_launch_get(key, kprec, klay, klanes, kdims)
    else:
        bcfg = su3.su3_batch_autotune(exprs, zs, ops, stream)
    log(f"batch tune: {bcfg.as_dict()}")

    def replay(cfg, repeats=None):
        su3.su3_launch_set(key, kprec, klay, klanes, kdims, cfg)
        b = su3.su3_batch_create(exprs, zs, ops, stream)
        ms, _ = timer.run(lambda: su3.su3_batch_launch(b, stream), 100, 3, repeats)
        su3.su3_batch_destroy(b)
        return ms

    ms_b = replay(bcfg)
    out = entry(ms_b, total_bytes, lattices=64, layouts=rec_text, sites=total_sites,
                bytes=total_bytes, n_c12=sum(1 for _, c in lat if c), replays=100,
                persistent=bcfg.persistent, tile=bcfg.tile_sites)
    # the best persistent grid (and the best one-shot grid when the tuned
    # launch is persistent), from the tuned setting's other knobs
    alt = []
    if bcfg.persistent == 0:
        # persistent grids drawing tiles from the ticket counter: blocks of
        # 64-256 lanes, 4-16 waves per compute unit, tiles of 256-8192 sites
        shapes = [(64, 4), (64, 8), (64, 16), (128, 2), (128, 4), (128, 8),
                  (256, 1), (256, 2), (256, 4)]
        tiles = (256, 512, 2048, 8192)
    else:
        shapes, tiles = [(bcfg.block, 0)], (bcfg.tile_sites,)
    for block, pers in shapes:
        for tile in tiles:
            c = su3.su3_launch(**bcfg.as_dict())
            c.block, c.persistent, c.tile_sites, c.occupancy = block, pers, tile, 0
            if pers:
                c.nontemporal = 7
            alt.append((replay(c, repeats=1), pers, tile, block, c))
    _, pers_a, tile_a, block_a, c_a = min(alt, key=lambda r: r[0])
    ms_a = replay(c_a)  # the search's winner, timed like the others
    a = entry(ms_a, total_bytes)
    pre = "oneshot" if bcfg.persistent else "persistent"
    out.update({f"{pre}_us": a["us"], f"{pre}_gbps": a["gbps"], f"{pre}_pct": a["pct"],
                f"{pre}_k": pers_a, f"{pre}_tile": tile_a, f"{pre}_block": block_a})
    su3.su3_launch_set(key, kprec, klay, klanes, kdims, bcfg)

    # the same 64 products as 64 back-to-back launches (each shape's tuned
    # launch, kept by the layout recommendation)

    def unbatched():
        for i in range(64):
            su3.su3_mult(zs[i], ops[i][0], ops[i][1], stream)
    ms_u, _ = timer.run(unbatched, 20, 2)
    out["unbatched_us"] = round(ms_u * 1e3, 1)
    hosts = [(testgen.volume(d), comp, [host_field(testgen.volume(d),
                                                   testgen.FID_BATCH_BASE + 4 * i + k)
                                        for k in range(2)])
             for i, (d, comp) in enumerate(lat)]

    def all_items(orc):
        for Vi, comp, (hx, hy) in hosts:
            if comp:
                orc.reference(0, 3, [hx, hy])
            else:
                orc.mult(hx, hy)
    cpu.add(out, "cpu", all_items, total_bytes, min_s=0.2)
    del zs, ops

    # the remedy for launch-bound small lattices: 64 separate 16^4 FP64
    # products (1.8 GB in all, so no launch finds its operands cached) as
    # one batched launch, against the same products as 64 tuned launches
    F64, SOA = su3.SU3_F64, su3.SU3_LAYOUT_SOA
    d16 = (16, 16, 16, 16)
    szs, sops = [], []
    for i in range(64):
        sops.append([make(d16, F64, SOA, 0, testgen.FID_BATCH_BASE + 4 * i + k)
                     for k in range(2)])
        szs.append(su3.field_tensor(d16, F64, SOA, 0))
    sexprs = [su3.SU3_EXPR_MUL] * 64
    sbytes = 64 * BYTES_PER_SITE[F64] * testgen.volume(d16)
    tune(su3.SU3_EXPR_MUL, F64, SOA, 0, d16, "small lattice")
    scfg = None if args.no_tune else su3.su3_batch_autotune(sexprs, szs, sops, stream)
    sb = su3.su3_batch_create(sexprs, szs, sops, stream)
    ms_sb, _ = timer.run(lambda: su3.su3_batch_launch(sb, stream), 100, 3)
    su3.su3_batch_destroy(sb)

    def small_unbatched():
        for i in range(64):
            su3.su3_mult(szs[i], sops[i][0], sops[i][1], stream)
    ms_su, _ = timer.run(small_unbatched, 20, 2)
    su = entry(ms_su, sbytes)
    small = entry(ms_sb, sbytes, lattices=64, dims="16^4", bytes=sbytes,
                  separate_us=su["us"], separate_gbps=su["gbps"], separate_pct=su["pct"])
    if scfg is not None:
        small["persistent"], small["tile"] = scfg.persistent, scfg.tile_sites
    out["small_16^4_x64"] = small
    log(f"batch: {out}")
    del szs, sops
    return out


def section_shift(ctx):
    """Cshift and the product with a shifted operand at 48^4, FP64 SoA, in
    each direction (288 and 432 B/site)."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args = ctx["args"]
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    SOA = su3.SU3_LAYOUT_SOA
    if "x64" in ctx:
        x64, y64, z64 = ctx["x64"], ctx["y64"], ctx["z64"]
    else:
        x64 = make(dims, su3.SU3_F64, SOA, 0, testgen.FID_X)
        y64 = make(dims, su3.SU3_F64, SOA, 0, testgen.FID_Y)
        z64 = su3.field_tensor(dims, su3.SU3_F64, SOA, 0)
    shift = {}
    tune(su3.SU3_EXPR_CSHIFT, su3.SU3_F64, SOA, 0, dims, "cshift")
    tune(su3.SU3_EXPR_MUL_SHIFTED, su3.SU3_F64, SOA, 0, dims, "mult_shifted")
    for mu in range(4):
        ms_c, _ = timer.run(lambda: su3.su3_cshift(z64, y64, mu, 1, stream), steps, 3)
        ms_m, _ = timer.run(lambda: su3.su3_mult_shifted(z64, x64, y64, mu, 1, stream),
                            steps, 3)
        shift[f"mu{mu}"] = {"cshift": entry(ms_c, 288 * V), "mult": entry(ms_m, 432 * V)}
        log(f"shift mu {mu}: {shift[f'mu{mu}']}")
    return shift


def section_programs(ctx):
    """Expression programs at 48^4, SoA, in double and single arithmetic."""
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args = ctx["args"]
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    SOA = su3.SU3_LAYOUT_SOA
    # expression programs at 48^4 (one precompiled kernel interpreting the
    # host-compiled expression): the sum plus the product of two real
    # fields, a+b+a*b (the real-valued composite example of Section 3,
    # Listing 2; two real inputs, one real output: 24 B/site), the streaming product,
    # the MULADD shape and a trace into a complex field, each against its
    # algorithmic bytes; the fixed-expression kernels beside them
    progs = {}
    M, R, C = su3.SU3_KIND_MATRIX, su3.SU3_KIND_REAL, su3.SU3_KIND_COMPLEX
    for prec, pname in ((su3.SU3_F64, "f64"), (su3.SU3_F32, "f32")):
        tune(su3.SU3_EXPR_PROGRAM, prec, SOA, 0, dims, f"program {pname}")
        tune(su3.SU3_EXPR_PROGRAM_SCALAR, prec, SOA, 0, dims, f"program {pname} scalar result")
        rb = REAL_BYTES[prec]
        ra = su3.scalar_tensor(dims, prec, SOA, R)
        rb_ = su3.scalar_tensor(dims, prec, SOA, R)
        rz = su3.scalar_tensor(dims, prec, SOA, R)
        su3.su3_program_eval(su3.Program("1.0", []), ra, [], stream)
        su3.su3_program_eval(su3.Program("2.0", []), rb_, [], stream)
        mats = [make(dims, prec, SOA, 0, testgen.FID_U0 + k) for k in range(4)]
        zm = su3.field_tensor(dims, prec, SOA, 0)
        zc = su3.scalar_tensor(dims, prec, SOA, C)
        cases = [("apb_ab_real", "a+b+a*b", [R, R], rz, [ra, rb_], 3 * rb),
                 ("mul", "a*b", [M, M], zm, mats[:2], 54 * rb),
                 ("muladd", "a*b+c*d", [M, M, M, M], zm, mats, 90 * rb),
                 ("trace", "trace(a*adj(b))", [M, M], zc, mats[:2], 38 * rb),
                 # seven matrix registers: the 8-register kernel (in double
                 # one wave per SIMD, part of its registers in AGPRs)
                 ("deep", "(a*b+c*d)*(a*c+b*d)+(a-b)*(c-d)", [M, M, M, M], zm, mats,
                  90 * rb)]
        for name, text, kinds, z, ops, bps in cases:
            prog = su3.Program(text, kinds)
            ms, _ = timer.run(lambda: su3.su3_program_eval(prog, z, ops, stream), steps, 3)
            key = f"{pname}_{name}"
            progs[key] = entry(ms, bps * V)
            if name == "mul":
                tune(su3.SU3_EXPR_MUL, prec, SOA, 0, dims)
                mf, _ = timer.run(lambda: su3.su3_mult(zm, mats[0], mats[1], stream), steps, 3)
                progs[key]["fixed_us"] = round(mf * 1e3, 1)
            if name == "muladd":
                # the fixed kernel in its own tuned launch at this size
                tune(su3.SU3_EXPR_MULADD, prec, SOA, 0, dims, f"muladd {pname}")
                mf, _ = timer.run(lambda: su3.su3_fused_eval(zm, su3.SU3_EXPR_MULADD, mats,
                                                             stream), steps, 3)
                progs[key]["fixed_us"] = round(mf * 1e3, 1)
            log(f"program {key} ({text}): {progs[key]}")
        del ra, rb_, rz, mats, zm, zc
    return progs


def section_vnode(ctx):
    """Grid's virtual-node layout used in place at 48^4: the streaming
    product (FP64) and the hopping term (FP64 and FP32) for N_sub = 4 and
    16."""
    su3, testgen, stream, timer, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "tune"))
    args, host_field = ctx["args"], ctx["host_field"]
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    # Grid's virtual-node layout used in place (N_sub sites per outer site,
    # one per virtual node): the streaming product and the hopping term in
    # FP64 on the same inputs, for N_sub = 4 (t and z split in two, Grid's
    # usual split) and 16 (every direction split in two)
    vn = {}
    host_psi = testgen.spinor_field(V, seed=args.seed, field_id=200)
    for nsub, simd in ((4, (1, 1, 2, 2)), (16, (2, 2, 2, 2))):
        F64, VN = su3.SU3_F64, su3.SU3_LAYOUT_VNODE

        def vfield(host, kind=su3.SU3_KIND_MATRIX, prec=F64):
            f = su3.vnode_tensor(dims, prec, simd, kind)
            su3.su3_field_upload(f, host, stream)
            return f

        fx, fy = vfield(host_field(V, testgen.FID_X)), vfield(host_field(V, testgen.FID_Y))
        fz = su3.vnode_tensor(dims, F64, simd)
        tune(su3.SU3_EXPR_MUL, F64, VN, nsub, dims, f"vnode mul {nsub}")
        ms, _ = timer.run(lambda: su3.su3_mult(fz, fx, fy, stream), steps, 3)
        vn[f"mul_nsub{nsub}"] = entry(ms, BYTES_PER_SITE[F64] * V)
        del fx, fy, fz
        U = [vfield(host_field(V, testgen.FID_U0 + mu)) for mu in range(4)]
        fin = vfield(host_psi, su3.SU3_KIND_SPINOR)
        fout = su3.vnode_tensor(dims, F64, simd, su3.SU3_KIND_SPINOR)
        tune(su3.SU3_EXPR_DSLASH, F64, VN, nsub, dims, f"vnode dslash {nsub}")
        ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
        vn[f"dslash_nsub{nsub}"] = entry(ms, DSLASH_BYTES_PER_SITE[(F64, F64)] * V)
        log(f"vnode nsub {nsub}: {vn[f'mul_nsub{nsub}']} {vn[f'dslash_nsub{nsub}']}")
        del U, fin, fout
        # the same hopping term with single-precision spinors and links
        F32 = su3.SU3_F32
        U = [vfield(host_field(V, testgen.FID_U0 + mu), prec=F32) for mu in range(4)]
        fin = vfield(host_psi, su3.SU3_KIND_SPINOR, prec=F32)
        fout = su3.vnode_tensor(dims, F32, simd, su3.SU3_KIND_SPINOR)
        tune(su3.SU3_EXPR_DSLASH, F32, VN, nsub, dims, f"vnode dslash f32 {nsub}")
        ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
        vn[f"dslash_f32_nsub{nsub}"] = entry(ms, DSLASH_BYTES_PER_SITE[(F32, F32)] * V)
        log(f"vnode nsub {nsub} f32 dslash: {vn[f'dslash_f32_nsub{nsub}']}")
        del U, fin, fout
    del host_psi
    return vn


SECTION_FUNCS = {"precision": section_precision, "fused": section_fused,
                 "ceiling": section_ceiling, "dslash": section_dslash,
                 "batch": section_batch, "shift": section_shift,
                 "programs": section_programs, "vnode": section_vnode}


def run_variants(ctx, out):
    su3, testgen, stream, timer, make, tune = (ctx[k] for k in (
        "su3", "testgen", "stream", "timer", "make", "tune"))
    args, cpu, host_field = ctx["args"], ctx["cpu"], ctx["host_field"]
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    SOA, AOS, AOSOA = su3.SU3_LAYOUT_SOA, su3.SU3_LAYOUT_AOS, su3.SU3_LAYOUT_AOSOA
    x64, y64, z64, ms_f64 = ctx["x64"], ctx["y64"], ctx["z64"], ctx["ms_f64"]

    out["precision_48^4"] = section_precision(ctx)

    # layouts at 48^4 (FP64)
    lay_out = {}
    cases = [("aos", AOS, 0, 0), ("aos_lds", AOS, 0, 1)] + \
        [(f"aosoa{L}", AOSOA, L, 0) for L in (8, 16, 32, 64)]
    for name, lay, lanes, lds in cases:
        x = make(dims, su3.SU3_F64, lay, lanes, testgen.FID_X)
        y = make(dims, su3.SU3_F64, lay, lanes, testgen.FID_Y)
        z = su3.field_tensor(dims, su3.SU3_F64, lay, lanes)
        if lay == AOS:
            cfg = su3.su3_launch_get(0, 0, lay, lanes, dims).as_dict()
            cfg.update(lds_stage=lds, block=64)
            su3.su3_launch_set(0, 0, lay, lanes, dims, cfg)
        else:
            tune(su3.SU3_EXPR_MUL, su3.SU3_F64, lay, lanes, dims, f"layout {name}")
        ms, _ = timer.run(lambda: su3.su3_mult(z, x, y, stream), steps, 3)
        lay_out[name] = entry(ms, 432 * V)
        log(f"layout {name}: {lay_out[name]}")
        del x, y, z
    out["layouts_f64_48^4"] = lay_out

    # volume sweep (FP64 SoA); sizes below 2x the 256 MiB Infinity Cache
    # are cache-resident when hot, not HBM figures: the cold figures are
    sweep = {}
    d8 = (8, 8, 8, 8)
    sweep["8^4"] = hot_and_cold(ctx, d8, su3.SU3_F64, 18, 19)
    for L in (16, 24, 32):
        d = (L, L, L, L)
        sweep[f"{L}^4"] = hot_and_cold(ctx, d, su3.SU3_F64, 10 + L, 11 + L)
        log(f"sweep {L}^4: {sweep[f'{L}^4']}")
    e48 = entry(ms_f64, 432 * V, cached=False)
    hx, hy = host_field(V, testgen.FID_X), host_field(V, testgen.FID_Y)
    cpu.add(e48, "cpu", lambda orc: orc.mult(hx, hy), 432 * V)
    sweep["48^4"] = e48
    out["sweep_f64_soa"] = sweep

    # one GPU's share of a 48^4 lattice cut into 8 t-slabs: 48^3 x 6 sites,
    # 287 MB of operands, just above the Infinity Cache, so the cold figure
    # is the HBM one
    shard = hot_and_cold(ctx, (48, 48, 48, 6), su3.SU3_F64, 60, 61, cpu_rate=False)
    log(f"shard 48^3x6: {shard}")
    out["shard_f64_soa_48^3x6"] = shard

    # storage precisions at 32^4 (SoA): every working set fits the Infinity
    # Cache, so the cold figures are the HBM ones
    p32 = {}
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        p32[PREC_NAME[prec]] = hot_and_cold(ctx, (32, 32, 32, 32), prec, 40, 41)
        log(f"precision 32^4 {PREC_NAME[prec]}: {p32[PREC_NAME[prec]]}")
    out["precision_32^4"] = p32

    # shifted operands at 48^4 (FP64 SoA): Cshift moves 288 B/site, the
    # product with a shifted operand 432 B/site
    out["shift_f64_48^4"] = section_shift(ctx)

    out["dslash_48^4"] = section_dslash(ctx)

    # the hopping term at the same t-slab's shape (periodic in t over its 6
    # slices: the traffic and work of a slab without its halo exchange);
    # 637 MB of operands, more than twice the Infinity Cache
    ds = (48, 48, 48, 6)
    Vs = testgen.volume(ds)
    U = [make(ds, su3.SU3_F64, SOA, 0, 60 + mu) for mu in range(4)]
    fin = su3.spinor_tensor(ds, su3.SU3_F64, SOA, 0)
    su3.su3_field_upload(fin, testgen.spinor_field(Vs, seed=args.seed, field_id=201),
                         stream)
    fout = su3.spinor_tensor(ds, su3.SU3_F64, SOA, 0)
    tune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, SOA, 0, ds, "dslash shard")
    ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
    out["dslash_shard_f64_soa_48^3x6"] = entry(ms, DSLASH_BYTES_PER_SITE[(0, 0)] * Vs)
    log(f"dslash shard 48^3x6: {out['dslash_shard_f64_soa_48^3x6']}")
    del U, fin, fout

    out["vnode_f64_48^4"] = section_vnode(ctx)

    out["programs_48^4"] = section_programs(ctx)

    out["fused_32^4"] = section_fused(ctx)
    out["batch_64"] = section_batch(ctx)
    return out


def cpu_baseline(leg, x, y):
    """The FP64 oracle, as it stands, on the host cores: full 48^4 products
    repeated until at least 8 s have passed on all the process's threads,
    then for at least 4 s on one thread."""
    orc = leg.oracle()
    V = x.shape[0]
    threads = orc.threads()
    passes, el = leg._timed(lambda: orc.mult(x, y), 8.0)
    g = 432 * V * passes / el / 1e9
    orc.set_threads(1)
    try:
        p1, el1 = leg._timed(lambda: orc.mult(x, y), 4.0)
    finally:
        orc.set_threads(threads)
    g1 = 432 * V * p1 / el1 / 1e9
    log(f"cpu baseline: {passes} passes in {el:.1f} s, {g:.2f} GB/s, "
        f"{threads} threads; 1 thread: {p1} passes in {el1:.1f} s, {g1:.3f} GB/s")
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(g, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} full z=x*y passes over the 48^4 lattice "
                      f"({V} sites, same seeded inputs), {el:.1f} s wall",
            "gflops": round(198 * V * passes / el / 1e9, 2),
            "value_1core": round(g1, 4),
            "sample_1core": f"{p1} passes on one thread, {el1:.1f} s wall",
            "cpu_model": model}


if __name__ == "__main__":
    main()
