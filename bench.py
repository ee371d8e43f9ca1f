#!/usr/bin/env python3
"""SU(3) x SU(3) streaming benchmark on one MI355X.

A step is one evaluation of z(x) = x(x) * y(x) over a 48^4 lattice of SU(3)
matrices stored in double precision, structure-of-arrays layout (the
streaming test of Section 4, Listing 3).  Inputs are seeded synthetic
Haar-random SU(3) fields already resident in HBM; the timed region is K
back-to-back launches bracketed by device synchronisation.

Prints ONE JSON line on stdout (progress goes to stderr):
  value        achieved GB/s = 432 B/site * V / (time per step)
  roofline     the dominant kernel against the 8 TB/s HBM peak, timed with
               HIP events on the launch stream; traffic from the committed
               PMC summary (null if the kernel changed since)
  cpu_baseline the FP64 oracle on the host cores, on a bounded sample
  variants     the precision forms (F32, F16 with F32 arithmetic, two-row
               compressed F32) at 48^4, the layouts (AoS, AoS+LDS, AoSoA),
               the volume sweep, the shifted operands, the Wilson hopping
               term at 48^4, expression programs at 48^4, fused vs
               chained expressions at 32^4, the
               64-lattice batch replayed from a HIP graph, and the triad
               ceiling -- each in GB/s of its own algorithmic bytes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def expr_bytes_per_site(prec, expr):
    E = 6 if prec == 3 else 9
    site = E * 2 * REAL_BYTES[prec]
    nops = {0: 2, 1: 3, 2: 4, 3: 2, 4: 2}[expr]
    return site * (nops + 1)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1710)
    ap.add_argument("--no-variants", action="store_true",
                    help="headline only (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="no autotuning: the library's default launch, or the "
                         "one cached in the file SU3_TUNE_CACHE names")
    ap.add_argument("--only-dslash", action="store_true",
                    help="time only the Wilson hopping term (48^4, FP64, "
                         "SoA) and print its line (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain copies of known size (PMC scaling)")
    return ap.parse_args()


class Timer:
    """K launches between two events on `stream`, plus host wall time
    between synchronisations."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def run(self, launch, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(self.stream)
        for _ in range(steps):
            launch()
        e1.record(self.stream)
        torch.cuda.synchronize()
        host_s = time.perf_counter() - t0
        return e0.elapsed_time(e1) / steps, host_s  # ms per launch (events)


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): every "
              "site is independent, so a multi-GPU run would shard the lattice "
              "into t-slabs with no exchange step (the hopping term would add "
              "a t-face halo)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import testgen
    import paper_1710_09409_amd as su3

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    timer = Timer(torch, stream)
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

    def tune(expr, prec, layout, lanes, dims):
        if args.no_tune:
            return su3.su3_launch_get(expr, prec, layout, lanes, dims).as_dict()
        return su3.su3_autotune(expr, prec, layout, lanes, dims, stream).as_dict()

    if args.only_dslash:
        dslash_only(args, su3, torch, testgen, stream, timer, make, tune)
        return

    # ------------------------------------------------------------ headline
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    F64, SOA = su3.SU3_F64, su3.SU3_LAYOUT_SOA
    log(f"headline: z = x*y, {V} sites, FP64 SoA; generating inputs")
    x = make(dims, F64, SOA, 0, testgen.FID_X)
    y = make(dims, F64, SOA, 0, testgen.FID_Y)
    z = su3.field_tensor(dims, F64, SOA, 0)
    cfg = tune(su3.SU3_EXPR_MUL, F64, SOA, 0, dims)
    log(f"launch: {cfg}")
    step_bytes = BYTES_PER_SITE[0] * V
    ms_ev, host_s = timer.run(lambda: su3.su3_mult(z, x, y, stream),
                              args.steps, args.warmup)
    ms_per_step = host_s * 1e3 / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = step_bytes / (ms_ev * 1e-3) / 1e9
    log(f"headline: {ms_ev * 1e3:.1f} us/launch (events), {achieved:.0f} GB/s "
        f"= {100 * achieved / HBM_PEAK_GBPS:.1f}% of 8 TB/s")
    traffic = committed_traffic()

    # triad ceiling over the same bytes (2 read streams + 1 write stream)
    n = step_bytes // 24
    ta = torch.empty(n, dtype=torch.float64, device="cuda")
    tb = torch.ones(n, dtype=torch.float64, device="cuda")
    tc = torch.ones(n, dtype=torch.float64, device="cuda")
    ms_tr, _ = timer.run(lambda: su3.su3_triad(ta.data_ptr(), tb.data_ptr(),
                                               tc.data_ptr(), 3.0, n, stream),
                         args.steps, args.warmup)
    triad = 24 * n / (ms_tr * 1e-3) / 1e9
    log(f"triad: {triad:.0f} GB/s")
    if args.calibrate_copy:
        nbytes = 1 << 30
        cs = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cd = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        for _ in range(5):
            su3.su3_copy(cd.data_ptr(), cs.data_ptr(), nbytes, stream)
        torch.cuda.synchronize()
        del cs, cd
    del ta, tb, tc

    variants = {"triad_gbps": round(triad, 1),
                "headline_frac_of_triad": round(achieved / triad, 4)}

    if not args.no_variants:
        variants.update(run_variants(args, su3, torch, testgen, np, stream,
                                     timer, make, tune, x, y, z, dims, ms_ev))

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(host_field(V, testgen.FID_X),
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
            "dims": list(dims), "sites": V, "bytes_per_step": step_bytes,
            "flops_per_step": FLOPS_PER_SITE[0] * V,
            "gflops": round(FLOPS_PER_SITE[0] * V / (ms_ev * 1e-3) / 1e9, 1),
            "launch": cfg,
            "input_sha256": {"x": testgen.buffer_sha256(host_field(V, testgen.FID_X))[:16],
                             "y": testgen.buffer_sha256(host_field(V, testgen.FID_Y))[:16]},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "kernel": "k_site<MUL, 1 site/lane> (FP64 SoA)",
            "avg_launch_us": round(ms_ev * 1e3, 2),
            "bytes_per_launch": step_bytes,
        },
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


def dslash_only(args, su3, torch, testgen, stream, timer, make, tune):
    dims = (48, 48, 48, 48)
    V = testgen.volume(dims)
    F64, SOA = su3.SU3_F64, su3.SU3_LAYOUT_SOA
    log(f"Dslash: {V} sites, FP64 SoA; generating inputs")
    U = [make(dims, F64, SOA, 0, testgen.FID_U0 + mu) for mu in range(4)]
    fin = su3.spinor_tensor(dims, F64, SOA)
    su3.su3_field_upload(fin, testgen.spinor_field(V, seed=args.seed, field_id=200), stream)
    fout = su3.spinor_tensor(dims, F64, SOA)
    cfg = tune(su3.SU3_EXPR_DSLASH, F64, SOA, 0, dims)
    ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), args.steps, args.warmup)
    b = DSLASH_BYTES_PER_SITE[(0, 0)] * V
    print(json.dumps({"kernel": "k_dslash (FP64 SoA 48^4)", "us": round(ms * 1e3, 2),
                      "gbps": round(b / (ms * 1e-3) / 1e9, 1),
                      "bytes_per_launch": b, "launch": cfg}), flush=True)


def run_variants(args, su3, torch, testgen, np, stream, timer, make, tune,
                 x64, y64, z64, dims, ms_f64):
    out = {}
    V = testgen.volume(dims)
    steps = max(10, min(args.steps, 50))
    SOA, AOS, AOSOA = su3.SU3_LAYOUT_SOA, su3.SU3_LAYOUT_AOS, su3.SU3_LAYOUT_AOSOA

    # precision forms at 48^4 (SoA)
    prec_out = {}
    for prec in (su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        for lname, lay, lanes in (("soa", SOA, 0), ("aosoa64", AOSOA, 64)):
            x = make(dims, prec, lay, lanes, testgen.FID_X)
            y = make(dims, prec, lay, lanes, testgen.FID_Y)
            z = su3.field_tensor(dims, prec, lay, lanes)
            cfg = tune(su3.SU3_EXPR_MUL, prec, lay, lanes, dims)
            ms, _ = timer.run(lambda: su3.su3_mult(z, x, y, stream), steps, 3)
            b = BYTES_PER_SITE[prec] * V
            key = f"{PREC_NAME[prec]}_{lname}"
            prec_out[key] = {
                "us": round(ms * 1e3, 2), "gbps": round(b / (ms * 1e-3) / 1e9, 1),
                "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "speedup_vs_f64_soa": round(ms_f64 / ms, 3), "launch": cfg}
            log(f"precision {key}: {prec_out[key]}")
            del x, y, z
    out["precision_48^4"] = prec_out

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
            cfg = tune(su3.SU3_EXPR_MUL, su3.SU3_F64, lay, lanes, dims)
        ms, _ = timer.run(lambda: su3.su3_mult(z, x, y, stream), steps, 3)
        lay_out[name] = {"us": round(ms * 1e3, 2),
                         "gbps": round(432 * V / (ms * 1e-3) / 1e9, 1),
                         "launch": cfg}
        log(f"layout {name}: {lay_out[name]}")
        del x, y, z
    out["layouts_f64_48^4"] = lay_out

    def hot_and_cold(d, prec, fid_x, fid_y):
        """z = x*y at lattice d (SoA): hot (the same buffers every launch)
        and cold (rotating through k buffer sets of >= 1 GiB in all, so the
        256 MiB Infinity Cache never holds the next launch's operands)."""
        Vd = testgen.volume(d)
        ws = BYTES_PER_SITE[prec] * Vd
        x = make(d, prec, SOA, 0, fid_x)
        y = make(d, prec, SOA, 0, fid_y)
        z = su3.field_tensor(d, prec, SOA, 0)
        cfg = tune(su3.SU3_EXPR_MUL, prec, SOA, 0, d)
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
        return {"us": round(ms * 1e3, 2), "gbps": round(ws / (ms * 1e-3) / 1e9, 1),
                "cold_us": round(ms_cold * 1e3, 2),
                "cold_gbps": round(ws / (ms_cold * 1e-3) / 1e9, 1),
                "cold_frac_of_peak": round(ws / (ms_cold * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "cold_sets": k, "working_set_bytes": ws,
                "cache_resident": ws < 2 * 268435456, "launch": cfg}

    # volume sweep (FP64 SoA); sizes below 2x the 256 MiB Infinity Cache
    # are cache-resident when hot, not HBM figures: the cold figures are
    sweep = {}
    for L in (16, 24, 32):
        d = (L, L, L, L)
        sweep[f"{L}^4"] = hot_and_cold(d, su3.SU3_F64, 10 + L, 11 + L)
        log(f"sweep {L}^4: {sweep[f'{L}^4']}")
    sweep["48^4"] = {"us": round(ms_f64 * 1e3, 2),
                     "gbps": round(432 * V / (ms_f64 * 1e-3) / 1e9, 1),
                     "working_set_bytes": 432 * V, "cache_resident": False}
    out["sweep_f64_soa"] = sweep

    # one GPU's share of a 48^4 lattice cut into 8 t-slabs: 48^3 x 6 sites,
    # 287 MB of operands, just above the Infinity Cache, so the cold figure
    # is the HBM one
    shard = hot_and_cold((48, 48, 48, 6), su3.SU3_F64, 60, 61)
    log(f"shard 48^3x6: {shard}")
    out["shard_f64_soa_48^3x6"] = shard

    # storage precisions at 32^4 (SoA): every working set fits the Infinity
    # Cache, so the cold figures are the HBM ones
    p32 = {}
    for prec in (su3.SU3_F64, su3.SU3_F32, su3.SU3_F16_F32ACC, su3.SU3_C12_F32):
        p32[PREC_NAME[prec]] = hot_and_cold((32, 32, 32, 32), prec, 40, 41)
        log(f"precision 32^4 {PREC_NAME[prec]}: {p32[PREC_NAME[prec]]}")
    out["precision_32^4"] = p32

    # shifted operands at 48^4 (FP64 SoA): Cshift moves 288 B/site, the
    # product with a shifted operand 432 B/site
    shift = {}
    tune(su3.SU3_EXPR_CSHIFT, su3.SU3_F64, SOA, 0, dims)
    tune(su3.SU3_EXPR_MUL_SHIFTED, su3.SU3_F64, SOA, 0, dims)
    for mu in range(4):
        ms_c, _ = timer.run(lambda: su3.su3_cshift(z64, y64, mu, 1, stream), steps, 3)
        ms_m, _ = timer.run(lambda: su3.su3_mult_shifted(z64, x64, y64, mu, 1, stream),
                            steps, 3)
        shift[f"mu{mu}"] = {
            "cshift_us": round(ms_c * 1e3, 2),
            "cshift_gbps": round(288 * V / (ms_c * 1e-3) / 1e9, 1),
            "mult_shifted_us": round(ms_m * 1e3, 2),
            "mult_shifted_gbps": round(432 * V / (ms_m * 1e-3) / 1e9, 1)}
        log(f"shift mu {mu}: {shift[f'mu{mu}']}")
    out["shift_f64_48^4"] = shift

    # Wilson hopping term at 48^4: algorithmic bytes per site = four link
    # matrices + one input spinor + one output spinor, each moved once
    # (F64: 4*144 + 192 + 192 = 960; F32: 480; F32 with compressed links:
    # 4*48 + 96 + 96 = 384); 1320 flops per site
    dsl = {}
    host_psi = testgen.spinor_field(V, seed=args.seed, field_id=200)
    for sp, lp, name in ((su3.SU3_F64, su3.SU3_F64, "f64"), (su3.SU3_F32, su3.SU3_F32, "f32"),
                         (su3.SU3_F32, su3.SU3_C12_F32, "f32_c12")):
        for lname, lay, lanes in (("soa", SOA, 0), ("aosoa64", AOSOA, 64)):
            U = [make(dims, lp, lay, lanes, testgen.FID_U0 + mu) for mu in range(4)]
            fin = su3.spinor_tensor(dims, sp, lay, lanes)
            su3.su3_field_upload(fin, host_psi, stream)
            fout = su3.spinor_tensor(dims, sp, lay, lanes)
            cfg = tune(su3.SU3_EXPR_DSLASH, lp, lay, lanes, dims)
            ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
            b = DSLASH_BYTES_PER_SITE[(sp, lp)] * V
            key = f"{name}_{lname}"
            dsl[key] = {"us": round(ms * 1e3, 2),
                        "gbps": round(b / (ms * 1e-3) / 1e9, 1),
                        "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                        "gflops": round(DSLASH_FLOPS_PER_SITE * V / (ms * 1e-3) / 1e9, 1),
                        "bytes_per_site": DSLASH_BYTES_PER_SITE[(sp, lp)],
                        "launch": cfg}
            log(f"dslash {key}: {dsl[key]}")
            del U, fin, fout
    out["dslash_48^4"] = dsl

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
    cfg = tune(su3.SU3_EXPR_DSLASH, su3.SU3_F64, SOA, 0, ds)
    ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
    b = DSLASH_BYTES_PER_SITE[(su3.SU3_F64, su3.SU3_F64)] * Vs
    out["dslash_shard_f64_soa_48^3x6"] = {
        "us": round(ms * 1e3, 2), "gbps": round(b / (ms * 1e-3) / 1e9, 1),
        "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "launch": cfg}
    log(f"dslash shard 48^3x6: {out['dslash_shard_f64_soa_48^3x6']}")
    del U, fin, fout

    # Grid's virtual-node layout used in place (N_sub sites per outer site,
    # one per virtual node): the streaming product and the hopping term in
    # FP64 on the same inputs, for N_sub = 4 (t and z split in two, Grid's
    # usual split) and 16 (every direction split in two)
    vn = {}
    hosts = {fid: testgen.su3_field(V, seed=args.seed, field_id=fid)
             for fid in (testgen.FID_X, testgen.FID_Y) +
             tuple(testgen.FID_U0 + mu for mu in range(4))}
    host_x, host_y = hosts[testgen.FID_X], hosts[testgen.FID_Y]
    for nsub, simd in ((4, (1, 1, 2, 2)), (16, (2, 2, 2, 2))):
        F64, VN = su3.SU3_F64, su3.SU3_LAYOUT_VNODE

        def vfield(host, kind=su3.SU3_KIND_MATRIX):
            f = su3.vnode_tensor(dims, F64, simd, kind)
            su3.su3_field_upload(f, host, stream)
            return f

        fx, fy = vfield(host_x), vfield(host_y)
        fz = su3.vnode_tensor(dims, F64, simd)
        cfg = tune(su3.SU3_EXPR_MUL, F64, VN, nsub, dims)
        ms, _ = timer.run(lambda: su3.su3_mult(fz, fx, fy, stream), steps, 3)
        b = BYTES_PER_SITE[F64] * V
        vn[f"mul_nsub{nsub}"] = {"us": round(ms * 1e3, 2),
                                 "gbps": round(b / (ms * 1e-3) / 1e9, 1),
                                 "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                 "simd": list(simd), "launch": cfg}
        log(f"vnode mul nsub {nsub}: {vn[f'mul_nsub{nsub}']}")
        del fx, fy, fz
        U = [vfield(hosts[testgen.FID_U0 + mu]) for mu in range(4)]
        fin = vfield(host_psi, su3.SU3_KIND_SPINOR)
        fout = su3.vnode_tensor(dims, F64, simd, su3.SU3_KIND_SPINOR)
        cfg = tune(su3.SU3_EXPR_DSLASH, F64, VN, nsub, dims)
        ms, _ = timer.run(lambda: su3.su3_dslash(fout, U, fin, stream), steps, 3)
        b = DSLASH_BYTES_PER_SITE[(F64, F64)] * V
        vn[f"dslash_nsub{nsub}"] = {"us": round(ms * 1e3, 2),
                                    "gbps": round(b / (ms * 1e-3) / 1e9, 1),
                                    "frac_of_peak": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                    "simd": list(simd), "launch": cfg}
        log(f"vnode dslash nsub {nsub}: {vn[f'dslash_nsub{nsub}']}")
        del U, fin, fout
    del host_psi, host_x, host_y, hosts
    out["vnode_f64_48^4"] = vn

    # expression programs at 48^4 (one precompiled kernel interpreting the
    # host-compiled expression): Listing 2 on double fields (two real
    # inputs, one real output: 24 B/site), the streaming product, the
    # MULADD shape and a trace into a complex field, each against its
    # algorithmic bytes; the fixed-expression kernels beside them
    progs = {}
    M, R, C = su3.SU3_KIND_MATRIX, su3.SU3_KIND_REAL, su3.SU3_KIND_COMPLEX
    for prec, pname in ((su3.SU3_F64, "f64"), (su3.SU3_F32, "f32")):
        tune(su3.SU3_EXPR_PROGRAM, prec, SOA, 0, dims)
        rb = REAL_BYTES[prec]
        v1 = su3.scalar_tensor(dims, prec, SOA, R)
        v2 = su3.scalar_tensor(dims, prec, SOA, R)
        v3 = su3.scalar_tensor(dims, prec, SOA, R)
        su3.su3_program_eval(su3.Program("1.0", []), v1, [], stream)
        su3.su3_program_eval(su3.Program("2.0", []), v2, [], stream)
        mats = [make(dims, prec, SOA, 0, testgen.FID_U0 + k) for k in range(4)]
        zm = su3.field_tensor(dims, prec, SOA, 0)
        zc = su3.scalar_tensor(dims, prec, SOA, C)
        cases = [("listing2", "a+b+a*b", [R, R], v3, [v1, v2], 3 * rb),
                 ("mul", "a*b", [M, M], zm, mats[:2], 54 * rb),
                 ("muladd", "a*b+c*d", [M, M, M, M], zm, mats, 90 * rb),
                 ("trace", "trace(a*adj(b))", [M, M], zc, mats[:2], 38 * rb)]
        for name, text, kinds, z, ops, bps in cases:
            prog = su3.Program(text, kinds)
            ms, _ = timer.run(lambda: su3.su3_program_eval(prog, z, ops, stream), steps, 3)
            key = f"{pname}_{name}"
            progs[key] = {"expr": text, "us": round(ms * 1e3, 2),
                          "gbps": round(bps * V / (ms * 1e-3) / 1e9, 1),
                          "bytes_per_site": bps}
            if name == "mul":
                mf, _ = timer.run(lambda: su3.su3_mult(zm, mats[0], mats[1], stream), steps, 3)
                progs[key]["fixed_kernel_us"] = round(mf * 1e3, 2)
            if name == "muladd":
                mf, _ = timer.run(lambda: su3.su3_fused_eval(zm, su3.SU3_EXPR_MULADD, mats,
                                                             stream), steps, 3)
                progs[key]["fixed_kernel_us"] = round(mf * 1e3, 2)
            log(f"program {key}: {progs[key]}")
        del v1, v2, v3, mats, zm, zc
    out["programs_48^4"] = progs

    # fused vs chained at 32^4 with four link fields
    d = (32, 32, 32, 32)
    Vf = testgen.volume(d)
    fused = {}
    for prec, lname, lay, lanes in ((su3.SU3_F64, "soa", SOA, 0), (su3.SU3_F32, "soa", SOA, 0),
                                    (su3.SU3_F64, "aosoa64", AOSOA, 64),
                                    (su3.SU3_F32, "aosoa64", AOSOA, 64)):
        U = [make(d, prec, lay, lanes, testgen.FID_U0 + mu) for mu in range(4)]
        z = su3.field_tensor(d, prec, lay, lanes)
        t1 = su3.field_tensor(d, prec, lay, lanes)
        t2 = su3.field_tensor(d, prec, lay, lanes)
        for expr, name in ((su3.SU3_EXPR_MUL3, "mul3"), (su3.SU3_EXPR_MULADD, "muladd")):
            nops = 3 if expr == su3.SU3_EXPR_MUL3 else 4
            cfg = tune(expr, prec, lay, lanes, d)
            tune(su3.SU3_EXPR_MUL, prec, lay, lanes, d)
            tune(su3.SU3_EXPR_ADD, prec, lay, lanes, d)
            ms_f, _ = timer.run(lambda: su3.su3_fused_eval(z, expr, U[:nops], stream),
                                steps, 3)
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
            b = expr_bytes_per_site(prec, expr) * Vf
            fused[f"{PREC_NAME[prec]}_{lname}_{name}"] = {
                "fused_us": round(ms_f * 1e3, 2), "chained_us": round(ms_c * 1e3, 2),
                "fused_gbps": round(b / (ms_f * 1e-3) / 1e9, 1),
                "speedup": round(ms_c / ms_f, 3), "launch": cfg}
            log(f"fused {PREC_NAME[prec]} {lname} {name}: {fused[f'{PREC_NAME[prec]}_{lname}_{name}']}")
        del U, z, t1, t2
    out["fused_32^4"] = fused

    # 64 uneven lattices, mixed FP64 and compressed FP32, one graph replay;
    # AoSoA(64) storage: most of these volumes are powers of two, whose SoA
    # entry planes sit at power-of-two strides
    lat = testgen.batch_lattices(64, seed=args.seed)
    zs, ops, exprs = [], [], []
    total_bytes = 0
    log("batch: generating 64 lattices")
    for i, (d, comp) in enumerate(lat):
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        Vi = testgen.volume(d)
        ops.append([make(d, prec, AOSOA, 64, testgen.FID_BATCH_BASE + 4 * i + k)
                    for k in range(2)])
        zs.append(su3.field_tensor(d, prec, AOSOA, 64))
        exprs.append(su3.SU3_EXPR_MUL)
        total_bytes += BYTES_PER_SITE[prec] * Vi
    total_sites = sum(testgen.volume(d) for d, _ in lat)
    bcfg = None
    if not args.no_tune:
        bcfg = su3.su3_batch_autotune(exprs, zs, ops, stream).as_dict()
        log(f"batch tune: {bcfg}")
    b = su3.su3_batch_create(exprs, zs, ops, stream)
    ms_b, _ = timer.run(lambda: su3.su3_batch_launch(b, stream), 100, 3)

    # the same 64 products as 64 back-to-back launches (tuned per shape)
    for i, (d, comp) in enumerate(lat):
        prec = su3.SU3_C12_F32 if comp else su3.SU3_F64
        tune(su3.SU3_EXPR_MUL, prec, AOSOA, 64, d)

    def unbatched():
        for i in range(64):
            su3.su3_mult(zs[i], ops[i][0], ops[i][1], stream)
    ms_u, _ = timer.run(unbatched, 20, 2)
    out["batch_64"] = {
        "lattices": 64, "layout": "aosoa64", "sites": total_sites, "bytes": total_bytes,
        "n_c12": sum(1 for _, c in lat if c),
        "us": round(ms_b * 1e3, 2),
        "gbps": round(total_bytes / (ms_b * 1e-3) / 1e9, 1),
        "unbatched_us": round(ms_u * 1e3, 2),
        "unbatched_gbps": round(total_bytes / (ms_u * 1e-3) / 1e9, 1),
        "replays": 100, "launch": bcfg}
    log(f"batch: {out['batch_64']}")
    su3.su3_batch_destroy(b)
    del zs, ops
    return out


def cpu_baseline(x, y):
    """The FP64 oracle, as it stands, on the host cores: full 48^4 products
    repeated until at least 10 s have passed on all the process's threads,
    then for at least 5 s on one thread."""
    import oracle
    orc = oracle.get()
    V = x.shape[0]

    def timed(min_s):
        passes, t0 = 0, time.perf_counter()
        while True:
            orc.mult(x, y)
            passes += 1
            el = time.perf_counter() - t0
            if el >= min_s or passes >= 5000:
                return passes, el

    threads = orc.threads()
    passes, el = timed(10.0)
    gbps = 432 * V * passes / el / 1e9
    orc.set_threads(1)
    p1, el1 = timed(5.0)
    orc.set_threads(threads)
    gbps1 = 432 * V * p1 / el1 / 1e9
    log(f"cpu baseline: {passes} passes in {el:.1f} s, {gbps:.2f} GB/s, "
        f"{threads} threads; 1 thread: {p1} passes in {el1:.1f} s, {gbps1:.3f} GB/s")
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(gbps, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} full z=x*y passes over the 48^4 lattice "
                      f"({V} sites, same seeded inputs), {el:.1f} s wall",
            "gflops": round(198 * V * passes / el / 1e9, 2),
            "value_1core": round(gbps1, 4),
            "sample_1core": f"{p1} passes on one thread, {el1:.1f} s wall",
            "cpu_model": model}


if __name__ == "__main__":
    main()
