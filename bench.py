#!/usr/bin/env python3
"""Benchmark of the scattering self-energy kernel on one MI355X.

One step = one sse_compute of the device-scale problem (NA=1024, NB=4,
Norb=10, Nkz=Nqz=7, NE=1000, Nw=30; Sigma [7, 1000, 1024, 10, 10]) for both
components (lesser and greater) in binary64, inputs resident in HBM.  Prints
one JSON line.  Algorithmic flops per launch: 8 N3D^2 Norb^2 per (k, e, q, w,
a, b) for the tap correlation plus 48 Norb^3 per (k, e, a, b) for the dH
sandwich, 4.4730e13 at this size.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 fp64 FMA lanes/clk x 2
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0}  # dense MFMA peak of the operand type


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32,bf16x3,fp64c64,fp64ah",
                    help="precision forms timed after the binary64 headline ('' = none); "
                         "fp64c64 = binary64 arithmetic on complex64 storage; fp64ah = "
                         "binary64 with the anti-Hermitian D~ mode (half the tap work)")
    ap.add_argument("--shard-gpus", type=int, default=8,
                    help="time one GPU's energy shard of the device-scale problem split over "
                         "this many GPUs (0 = skip)")
    ap.add_argument("--aux-steps", type=int, default=5,
                    help="timed steps of the D -> D~ and retarded passes at device scale "
                         "(0 = skip)")
    ap.add_argument("--only", default="",
                    help="time only this part, e.g. for profiling: a precision form (fp64, "
                         "fp32, bf16x3, fp64c64, fp64ah) or a section (pi, ablation, aux, "
                         "serving, batch, shard)")
    ap.add_argument("--pi-steps", type=int, default=2,
                    help="timed steps of the phonon self-energy (Eqs. (4)-(5)) at device "
                         "scale, both components (0 = skip)")
    ap.add_argument("--ablation-steps", type=int, default=1,
                    help="timed steps of the paper's own final form of Eq. (3) (dH G and "
                         "dH D precomputed, Norb x Norb Nw x Norb GEMMs on the matrix cores) "
                         "at device scale, both components (0 = skip)")
    ap.add_argument("--batch", default="fp64,bf16x3",
                    help="precisions of the 48-instance batched run ('' = skip)")
    ap.add_argument("--batch-budget-gb", type=float, default=200.0)
    ap.add_argument("--batch-small", type=int, default=48,
                    help="instances of each small-instance batch (tiny and small mixes), "
                         "one persistent launch against one submission each (0 = skip)")
    ap.add_argument("--serving-jobs", type=int, default=24,
                    help="jobs of the saturated serving run (0 = skip the serving section)")
    ap.add_argument("--serving-half-jobs", type=int, default=8,
                    help="jobs of the run at half the measured capacity (service latency; "
                         "0 = skip)")
    ap.add_argument("--serving-small-jobs", type=int, default=48,
                    help="jobs of each of the small-job and tiny-job mixes, served "
                         "concurrently and one at a time (0 = skip)")
    ap.add_argument("--serving-plain-jobs", type=int, default=4,
                    help="jobs (the first of the saturated run's) timed on the plain per-job "
                         "path")
    ap.add_argument("--profile-steps", action="store_true",
                    help="print a progress line per step (for profiler runs)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="after the timed steps, copy a buffer of this many GiB once "
                         "(reference kernel of known traffic for HBM byte counters)")
    return ap.parse_args()


# HBM traffic of the binary64 kernel, from the FETCH_SIZE / WRITE_SIZE counter
# passes summarised under profiles/.  The summary records a hash of the kernel's
# sources and of the build script (its compile flags); once they change, the
# counters no longer describe the kernel and the traffic is reported as null.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_sse_fp64_device_scale_traffic.json")
KERNEL_SOURCES = ["paper_1912_08810_amd/csrc/sse_fp64.hip",
                  "paper_1912_08810_amd/csrc/sse_internal.h",
                  "paper_1912_08810_amd/csrc/sse_copy.h",
                  "paper_1912_08810_amd/build.py"]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch (read + written) if the counters describe the
    current sources, else None."""
    try:
        with open(TRAFFIC_SUMMARY) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != kernel_sources_sha256():
        return None
    return t["read_bytes_per_launch"] + t["write_bytes_per_launch"]


def ci95(xs):
    if len(xs) < 2:
        return 0.0
    return 1.96 * statistics.stdev(xs) / math.sqrt(len(xs))


def progress(msg):
    """Progress lines go to stderr; stdout carries only the JSON result."""
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(prob, seed, target_s):
    """The oracle (unchanged) on a bounded sample of output blocks of the same
    workload: all k, sampled energies (incl. the edges) and atoms."""
    import numpy as np
    import oracle
    import ssegen
    from tests import gpu_util as gu
    cores = len(os.sched_getaffinity(0))
    blocks_all = gu.sample_blocks(prob, 11, n_e=16, n_a=64)
    neigh = ssegen.neigh(seed, prob.NA, prob.NB)
    dH = ssegen.dH(seed, prob.NA, prob.NB, prob.Norb)
    D = ssegen.D(seed, 0, prob.Nqz, prob.Nw, prob.NA, prob.NB)

    need = oracle.needed_g_blocks(neigh, prob.shifts(), prob.Nkz, prob.Nqz, prob.NE, prob.NA,
                                  blocks_all)
    Gb = ssegen.G_flat_blocks(seed, 0, prob.Norb, need)
    gslot = np.full(prob.Nkz * prob.NE * prob.NA, -1, dtype=np.int64)
    gslot[need] = np.arange(need.size)

    # the oracle over the whole sample, repeated until about target_s of work
    reps, t = 0, 0.0
    while reps == 0 or t < target_s:
        t0 = time.perf_counter()
        oracle.sigma(neigh, dH, Gb, D, prob.shifts(), prob.Nkz, prob.NE, blocks=blocks_all,
                     gslot=gslot, nthreads=cores)
        t += time.perf_counter() - t0
        reps += 1
    n = reps * len(blocks_all)
    per_block_alg = prob.flops() / (prob.Nkz * prob.NE * prob.NA)
    per_block_plain = prob.flops_plain() / (prob.Nkz * prob.NE * prob.NA)
    # one core on a sixteenth of the sample, for the per-core rate
    sub = blocks_all[::16]
    t1 = time.perf_counter()
    oracle.sigma(neigh, dH, Gb, D, prob.shifts(), prob.Nkz, prob.NE, blocks=sub, gslot=gslot,
                 nthreads=1)
    t1 = time.perf_counter() - t1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": round(per_block_alg * n / t / 1e9, 3),
        "unit": "GFLOP/s (algorithmic-equivalent)",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(blocks_all)} output blocks of one component (all 7 k x 16 energies "
                  f"incl. edges x 64 atoms), computed {reps} times: {n} blocks in {t:.1f} s",
        "blocks_per_s": round(n / t, 2),
        "plain_gflops": round(per_block_plain * n / t / 1e9, 3),
        "extrapolated_full_job_s": round(t / n * prob.Nkz * prob.NE * prob.NA * 2, 1),
        "one_core": {"value": round(per_block_alg * len(sub) / t1 / 1e9, 3),
                     "blocks": len(sub), "s": round(t1, 2)},
        "cpu_model": cpu_model,
    }


def pi_section(args, torch, sse, prob, seed, DeviceProblem, log):
    """The phonon self-energy of the device-scale problem, both components,
    binary64: one step = one sse_pi_compute.  Its algorithmic flops per
    component equal the electron self-energy's (9 (i, j) complex multiply-adds
    per orbital pair and (k, e, q, w, a, b); 48 Norb^3 per (k, e, a, b) for the
    two dH products)."""
    dp = DeviceProblem(prob, seed, ncomp=2)
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         ncomp=2, prec=sse.FP64)
    plan = sse.sse_plan(desc, prob.shifts())
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    Pi = torch.empty(2, sse.pi_elems(desc) * 2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    sse.sse_pi_compute(plan, dp.neigh, dp.dH, dp.G, Pi, ws, stream)
    torch.cuda.synchronize()
    times = []
    for i in range(args.pi_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sse.sse_pi_compute(plan, dp.neigh, dp.dH, dp.G, Pi, ws, stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        log(f"pi step {i}: {times[-1] * 1e3:.1f} ms")
    del dp, Pi, ws
    torch.cuda.empty_cache()
    med = statistics.median(times)
    tf = prob.flops() / (med / 2) / 1e12
    return {"value": round(2 * prob.flops() / med / 1e9, 1), "unit": "GFLOP/s",
            "ms_per_step": round(med * 1e3, 3), "steps": len(times), "storage": "complex128",
            "workload": "Pi lesser+greater [7, 30, 1024, 5, 3, 3] from G [2, 7, 1000, 1024, "
                        "10, 10], NB=4, s_w=w+1",
            "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4),
                         "kernel": "k_pi_fp64"}}


def ablation_section(args, torch, sse, prob, seed, DeviceProblem, log, headline_ms):
    """The paper's own final form of Eq. (3) on the same problem and inputs
    (sse_ablation_compute), against the reassociated binary64 kernel of the
    headline: time to the same Sigma, and its rate in the paper form's own
    flop count (8 N3D Norb^3 per (k, e, q, w, a, b) plus the dH G products)."""
    dp = DeviceProblem(prob, seed, ncomp=2)
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         ncomp=2)
    plan = sse.sse_plan(desc, prob.shifts())
    atoms = 256  # transients of 256 atoms at a time: ~35 GB of workspace
    ws = torch.empty(sse.ablation_workspace_bytes(desc, atoms), dtype=torch.uint8,
                     device="cuda")
    stream = torch.cuda.current_stream()
    times = []
    for i in range(args.ablation_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sse.sse_ablation_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        log(f"ablation step {i}: {times[-1] * 1e3:.1f} ms")
    del dp, ws
    torch.cuda.empty_cache()
    med = statistics.median(times)
    fp = prob.flops_paper_form()
    tf = fp / (med / 2) / 1e12
    return {"ms_per_step": round(med * 1e3, 3), "steps": len(times),
            "time_vs_reassociated": round(med / (headline_ms / 1e3), 2),
            "flops_per_component": fp,
            "value_paper_flops": round(2 * fp / med / 1e9, 1), "unit": "GFLOP/s",
            "value_algorithmic": round(2 * prob.flops() / med / 1e9, 1),
            "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4),
                         "kernel": "k_abl_gemm (+ k_abl_dhg, k_abl_dhd)"}}


def shard_section(args, torch, sse, prob, seed, DeviceProblem, log):
    """One GPU's share of the device-scale problem split over args.shard_gpus GPUs
    by energy (the paper's energy decomposition, Sec. 4.1): the shard's NE / n
    output energies plus the halo of shift-spread rows it reads, binary64, both
    components, every atom and momentum on the GPU.  The halo rows' own outputs
    are computed too (the library computes every energy of its G), so the timed
    work is NE / n + spread energies per component."""
    import dataclasses
    s = prob.shifts()
    spread = int(s.max() - s.min())
    ne = -(-prob.NE // args.shard_gpus) + spread
    sp = dataclasses.replace(prob, NE=ne)
    dp = DeviceProblem(sp, seed, ncomp=2)
    desc = sse.make_desc(sp.NA, sp.NB, sp.Norb, sp.Nkz, sp.Nqz, sp.NE, sp.Nw, ncomp=2,
                         prec=sse.FP64)
    plan = sse.sse_plan(desc, sp.shifts())
    ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    t = statistics.median(times)
    out_flops = 2 * prob.flops() / args.shard_gpus
    log(f"shard of {args.shard_gpus}: NE {ne} ({prob.NE // args.shard_gpus} + halo {spread}), "
        f"{t * 1e3:.1f} ms/step")
    del dp, ws
    torch.cuda.empty_cache()
    return {"gpus": args.shard_gpus, "NE_computed": ne, "halo_energies": spread,
            "ms_per_step": round(t * 1e3, 3),
            "output_tflops": round(out_flops / t / 1e12, 3),
            "computed_tflops": round(2 * sp.flops() / t / 1e12, 3),
            "note": "binary64, both components; energies of one shard plus its halo"}


def aux_section(args, torch, sse, prob, log):
    """The memory-bound passes either side of the kernels at device scale, both
    components, complex128: D [2, 7, 30, 1024, 5, 3, 3] -> D~ (reverse neighbour
    map on a symmetric table) and Sigma< / Sigma> -> Sigma^R.  Roofline: HBM,
    algorithmic bytes = read each input once, write each output once."""
    import numpy as np
    import ssegen
    nqw = prob.Nqz * prob.Nw
    d_in = nqw * prob.NA * (prob.NB + 1) * 9
    d_out = nqw * prob.NA * prob.NB * 9
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         ncomp=2)
    plan = sse.sse_plan(desc, prob.shifts())
    neigh = torch.from_numpy(ssegen.neigh_symmetric(configs_seed(), prob.NA, prob.NB)).cuda()
    D = torch.randn(2, 2 * d_in, dtype=torch.float64, device="cuda")
    Dt = torch.empty(2, 2 * d_out, dtype=torch.float64, device="cuda")
    ws = torch.empty(sse.dtilde_workspace_bytes(desc), dtype=torch.uint8, device="cuda")
    S = torch.randn(2, 2 * prob.g_elems(), dtype=torch.float64, device="cuda")
    SR = torch.empty(2 * prob.g_elems(), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.aux_steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return statistics.median(ts)

    t_dt = timed(lambda: sse.sse_wait(sse.sse_dtilde_submit(plan, neigh, D, Dt, ws, stream)))
    t_r = timed(lambda: sse.sse_retarded(plan, 0, S, SR, stream))
    b_dt = 2 * 16 * (d_in + d_out) + prob.NA * prob.NB * 4
    b_r = 3 * 16 * prob.g_elems()
    log(f"aux: D~ {t_dt*1e3:.3f} ms, Sigma^R {t_r*1e3:.3f} ms")
    del D, Dt, S, SR, ws
    torch.cuda.empty_cache()

    def roof(b, t, kern):
        gbs = b / t / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "kernel": kern}

    return {"dtilde": {"ms": round(t_dt * 1e3, 4), "bytes": b_dt,
                       "roofline": roof(b_dt, t_dt, "k_reverse_map + k_dtilde")},
            "retarded_sigma": {"ms": round(t_r * 1e3, 4), "bytes": b_r,
                               "roofline": roof(b_r, t_r, "k_retarded")}}


def configs_seed():
    from paper_1912_08810_amd import configs
    return configs.SEED


def batch_section(args, torch, sse, configs, DeviceProblem, log):
    """48 uneven instances (one component each) in HBM-budgeted waves; each wave
    is one persistent launch; tile shapes and tap chunks from the autotuner's cache."""
    from paper_1912_08810_amd import autotune
    cache = autotune.load_cache()
    insts = configs.batch_instances(configs.SEED, 48)
    out = {}
    for name in [x for x in args.batch.split(",") if x]:
        prec = {"fp64": sse.FP64, "fp32": sse.FP32, "bf16x3": sse.BF16X3}[name]
        esz = 16 if prec == sse.FP64 else 8
        tuned = {i: autotune.params_for(prec, p.Norb, p.NE, p.Nw, cache)
                 for i, p in enumerate(insts)}
        descs_all = {i: sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, prec=prec,
                                      tile_e=tuned[i][0], chunk_taps=tuned[i][1])
                     for i, p in enumerate(insts)}
        # resident bytes of one instance: G, Sigma, D~, dH and its plan workspace
        # (A fragments and the split copy of G on the MFMA paths)
        per = lambda i: ((2 * insts[i].g_elems() + insts[i].d_elems()) * esz
                         + insts[i].NA * insts[i].NB * insts[i].NN * 3 * 8
                         + sse.sse_plan(descs_all[i], insts[i].shifts()).workspace_bytes)
        order = sorted(range(len(insts)), key=lambda i: -insts[i].flops())
        waves, cur, used = [], [], 0
        for i in order:
            need = per(i)
            if cur and (used + need > args.batch_budget_gb * 1e9 or len(cur) == 64):
                waves.append(cur)
                cur, used = [], 0
            cur.append(i)
            used += need
        waves.append(cur)
        wave_s, flops = [], 0.0
        one_by_one = None
        for wi, wave in enumerate(waves):
            dps = [DeviceProblem(insts[i], 5000 + i, ncomp=1, fp32=prec != sse.FP64)
                   for i in wave]
            descs = [descs_all[i] for i in wave]
            plan = sse.sse_plan_batch(descs, [insts[i].shifts() for i in wave])
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
            stream = torch.cuda.current_stream()
            items = [(d.neigh, d.dH, d.G, d.D, d.Sigma) for d in dps]
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            t = sse.sse_submit(plan, items, ws, stream)
            e1.record(stream)
            sse.sse_wait(t)
            e1.synchronize()
            wave_s.append(e0.elapsed_time(e1) / 1e3)
            flops += sum(insts[i].flops() for i in wave)
            log(f"batch {name} wave {wi}: {len(wave)} instances, {wave_s[-1]:.3f} s")
            if wi == 0:
                # the same wave, one instance after the other (one-shot launches)
                e0.record(stream)
                for i, d in zip(wave, dps):
                    p = insts[i]
                    sp = sse.sse_plan(descs[wave.index(i)], p.shifts())
                    w1 = torch.empty(max(sp.workspace_bytes, 256), dtype=torch.uint8,
                                     device="cuda")
                    sse.sse_compute(sp, d.neigh, d.dH, d.G, d.D, d.Sigma, w1, stream)
                e1.record(stream)
                e1.synchronize()
                one_by_one = e0.elapsed_time(e1) / 1e3
                log(f"batch {name} wave 0 one-by-one: {one_by_one:.3f} s")
            del dps, ws, items
            torch.cuda.empty_cache()
        total = sum(wave_s)
        out[name] = {"instances": len(insts), "waves": len(waves),
                     "wave_s": [round(x, 3) for x in wave_s], "total_s": round(total, 3),
                     "value": round(flops / total / 1e9, 1), "unit": "GFLOP/s",
                     "storage": "complex128" if prec == sse.FP64 else "complex64",
                     "budget_gb": args.batch_budget_gb,
                     "tile_e_tuned": bool(cache)}
        if one_by_one is not None:
            out[name]["wave0_one_by_one_s"] = round(one_by_one, 3)
            out[name]["wave0_persistent_speedup"] = round(one_by_one / wave_s[0], 3)
    if args.batch_small > 0:
        out["small_instances"] = small_batch_section(args, torch, sse, configs, DeviceProblem,
                                                     log)
    return out


def small_batch_section(args, torch, sse, configs, DeviceProblem, log):
    """Batches of instances too small to fill the GPU alone: one persistent
    launch for the whole batch against one submission per instance, all
    enqueued back to back on one stream (plans and workspaces made beforehand,
    one untimed pass of each first)."""
    mixes = {
        "tiny": (configs.tiny_instances(configs.SEED + 5, args.batch_small),
                 "NA ~ U{8..16}, NE ~ U{30..60}, Nw ~ U{4..10}, Nkz = Nqz = 3: fewer output "
                 "tiles per instance than the GPU has compute units"),
        "small": (configs.small_instances(configs.SEED + 3, args.batch_small),
                  "NA ~ U{64..160}, NE ~ U{200..320}, Nw ~ U{10..20}, Nkz = Nqz = 5"),
    }
    out = {}
    stream = torch.cuda.current_stream()
    for mix, (insts, sizes) in mixes.items():
        out[mix] = {"instances": len(insts), "sizes": sizes}
        for name in [x for x in args.batch.split(",") if x]:
            prec = {"fp64": sse.FP64, "fp32": sse.FP32, "bf16x3": sse.BF16X3}[name]
            dps = [DeviceProblem(p, 7000 + i, ncomp=1, fp32=prec != sse.FP64)
                   for i, p in enumerate(insts)]
            descs = [sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, prec=prec)
                     for p in insts]
            items = [(d.neigh, d.dH, d.G, d.D, d.Sigma) for d in dps]
            plan = sse.sse_plan_batch(descs, [p.shifts() for p in insts])
            ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
            plans = [sse.sse_plan(d, p.shifts()) for d, p in zip(descs, insts)]
            wss = [torch.empty(max(pl.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
                   for pl in plans]

            def persistent():
                return [sse.sse_submit(plan, items, ws, stream)]

            def one_by_one():
                return [sse.sse_submit(pl, [it], w, stream)
                        for pl, it, w in zip(plans, items, wss)]

            res = {}
            for key, run in (("persistent", persistent), ("one_by_one", one_by_one)):
                for t in run():  # untimed pass
                    sse.sse_wait(t)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                tickets = run()
                e1.record(stream)
                for t in tickets:
                    sse.sse_wait(t)
                e1.synchronize()
                res[key] = e0.elapsed_time(e1)
            flops = sum(p.flops() for p in insts)
            out[mix][name] = {"persistent_ms": round(res["persistent"], 3),
                              "one_by_one_ms": round(res["one_by_one"], 3),
                              "persistent_gflops": round(flops / res["persistent"] / 1e6, 1),
                              "speedup": round(res["one_by_one"] / res["persistent"], 2)}
            log(f"batch {mix} {name}: persistent {res['persistent']:.2f} ms, one by one "
                f"{res['one_by_one']:.2f} ms")
            del dps, ws, wss, items, plans, plan
            torch.cuda.empty_cache()
    return out


def serving_section(args, torch, sse, configs, log):
    """Jobs from the batch size distribution, Poisson arrivals at 200 jobs/s,
    10 SCBA iterations each, complex64 (bf16 hi/lo MFMA) at the fp32 tolerance
    with binary64 fallback; then the same mix at half the measured capacity
    (service latency); compared with the plain per-job path (binary64, one job
    at a time, inputs copied in and results out every iteration) and with the
    same resident loop serving one job at a time.  A mix of small jobs that do
    not fill the GPU is served both ways too."""
    from paper_1912_08810_amd import serving
    from ssegen.device_problem import DeviceProblem
    probs = configs.batch_instances(configs.SEED + 1, args.serving_jobs)
    jobs = serving.make_jobs(probs, rate=200.0, seed=configs.SEED)
    srv = serving.Server(budget_bytes=200e9, slots=4, prec=sse.BF16X3, tol=1e-5)
    res = srv.run(jobs, log=log)
    sat = serving.summarize(res)
    out = {"saturated": dict(sat, arrival_rate=200.0, label="saturated (offered load far above "
                             "capacity; latency is queueing-dominated)")}
    del srv
    torch.cuda.empty_cache()
    if args.serving_half_jobs > 0:
        # service latency: the first jobs of the mix offered at half the capacity
        # just measured (Poisson, seeded)
        rate = 0.5 * sat["jobs_per_s"]
        jobs2 = serving.make_jobs(probs[:args.serving_half_jobs], rate=rate,
                                  seed=configs.SEED + 7)
        r2 = serving.Server(budget_bytes=200e9, slots=4, prec=sse.BF16X3, tol=1e-5).run(
            jobs2, log=log)
        out["half_capacity"] = dict(serving.summarize(r2), arrival_rate=round(rate, 4),
                                    label="half the measured capacity (service latency)")
        torch.cuda.empty_cache()
    # plain per-job path over the first jobs (each iteration costs the same, so two
    # iterations per job): host -> device copies of G and D~ (complex128),
    # binary64 compute, Sigma back to the host, every iteration, one job at a time
    plain_iters = 2
    t_plain, flops_plain = 0.0, 0.0
    # host data in ordinary memory, moved through two fixed pinned staging
    # buffers: the host copy into one overlaps the DMA out of the other
    CH = 1 << 25  # float64 elements per staging buffer (256 MiB)
    stage = [torch.empty(CH, dtype=torch.float64, pin_memory=True) for _ in range(2)]
    done = [torch.cuda.Event(), torch.cuda.Event()]

    def h2d(dev, host):
        dev, host = dev.view(-1), host.view(-1)
        for k, i in enumerate(range(0, host.numel(), CH)):
            m = min(CH, host.numel() - i)
            st = stage[k & 1]
            done[k & 1].synchronize()
            st[:m].copy_(host[i:i + m])
            dev[i:i + m].copy_(st[:m], non_blocking=True)
            done[k & 1].record()

    def d2h(host, dev):
        host, dev = host.view(-1), dev.view(-1)
        chunks = list(range(0, dev.numel(), CH))
        for k, i in enumerate(chunks):
            m = min(CH, dev.numel() - i)
            stage[k & 1][:m].copy_(dev[i:i + m], non_blocking=True)
            done[k & 1].record()
            if k > 0:
                j = chunks[k - 1]
                done[(k - 1) & 1].synchronize()
                host[j:j + min(CH, dev.numel() - j)].copy_(stage[(k - 1) & 1][:min(CH, dev.numel() - j)])
        j = chunks[-1]
        done[(len(chunks) - 1) & 1].synchronize()
        host[j:j + min(CH, dev.numel() - j)].copy_(stage[(len(chunks) - 1) & 1][:min(CH, dev.numel() - j)])

    plain_probs = probs[:args.serving_plain_jobs]
    for p in plain_probs:
        dp = DeviceProblem(p, 77, ncomp=2)
        hG, hD, hS = dp.G.cpu(), dp.D.cpu(), torch.empty(dp.Sigma.shape, dtype=dp.Sigma.dtype)
        desc = sse.make_desc(p.NA, p.NB, p.Norb, p.Nkz, p.Nqz, p.NE, p.Nw, ncomp=2,
                             prec=sse.FP64)
        plan = sse.sse_plan(desc, p.shifts())
        ws = torch.empty(max(plan.workspace_bytes, 256), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(plain_iters):
            h2d(dp.G, hG)
            h2d(dp.D, hD)
            sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws,
                            torch.cuda.current_stream())
            d2h(hS, dp.Sigma)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        flops_plain += 2 * p.flops() * plain_iters
        log(f"plain per-job: job NA={p.NA} NE={p.NE} Nw={p.Nw} done")
        del dp, ws, plan, hG, hS, hD
        torch.cuda.empty_cache()
    del stage
    plain_tflops = flops_plain / t_plain / 1e12
    log(f"plain per-job: {plain_tflops:.2f} TFLOP/s over {len(plain_probs)} jobs")
    # the same resident complex64 loop with one slot over the same jobs: isolates
    # the gain of overlapping jobs
    serial = serving.Server(budget_bytes=200e9, slots=1, prec=sse.BF16X3, tol=1e-5)
    j0 = serving.make_jobs(probs, rate=1e9, seed=configs.SEED, iterations=plain_iters)
    rs = serial.run(j0, log=log)
    ser = serving.summarize(rs)
    out["plain_per_job"] = {"tflops": round(plain_tflops, 3), "s": round(t_plain, 3),
                            "jobs": len(plain_probs), "iterations_per_job": plain_iters,
                            "path": "fp64, one job at a time; G, D~ in and Sigma out every "
                                    "iteration through two 256 MiB pinned staging buffers"}
    out["serial_resident_c64"] = {"tflops": ser["tflops"], "jobs": ser["jobs"],
                                  "iterations_per_job": plain_iters}
    out["speedup_vs_plain"] = round(sat["tflops"] / plain_tflops, 2)
    out["speedup_vs_serial_resident"] = round(sat["tflops"] / ser["tflops"], 2)
    if args.serving_small_jobs > 0:
        # small jobs (each launch still has thousands of output tiles, but lasts a
        # millisecond or less) and tiny jobs (fewer output tiles than compute
        # units: one job alone leaves most of the GPU idle); all present at the
        # start, served with 4 slots and with one, 10 iterations each
        mixes = {
            "small_jobs": (configs.small_instances(configs.SEED + 3, args.serving_small_jobs),
                           "NA ~ U{64..160}, NE ~ U{200..320}, Nw ~ U{10..20}, Nkz = Nqz = 5"),
            "tiny_jobs": (configs.tiny_instances(configs.SEED + 5, args.serving_small_jobs),
                          "NA ~ U{8..16}, NE ~ U{30..60}, Nw ~ U{4..10}, Nkz = Nqz = 3"),
        }
        for key, (sp, sizes) in mixes.items():
            # untimed warm-up over the first jobs (plans, allocator, first launches)
            serving.Server(budget_bytes=200e9, slots=4, prec=sse.BF16X3, tol=1e-5).run(
                serving.make_jobs(sp[:8], rate=1e9, seed=configs.SEED + 4, iterations=2))
            mix = {}
            for slots in (4, 1):
                js = serving.make_jobs(sp, rate=1e9, seed=configs.SEED + 3)
                r = serving.Server(budget_bytes=200e9, slots=slots, prec=sse.BF16X3,
                                   tol=1e-5).run(js)
                mix[slots] = serving.summarize(r)
                log(f"{key}, {slots} slot(s): {mix[slots]['makespan_s']:.3f} s, "
                    f"{mix[slots]['tflops']:.2f} TFLOP/s")
            out[key] = {
                "jobs": len(sp), "iterations_per_job": 10, "sizes": sizes,
                "concurrent_4_slots": mix[4], "serial_1_slot": mix[1],
                "speedup_vs_serial_resident": round(mix[4]["tflops"] / mix[1]["tflops"], 2)}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only; --gpus above 1 is not supported (every output "
              "block is independent, so a multi-GPU run would split the atoms across GPUs).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1912_08810_amd import configs, sse
    from ssegen.device_problem import DeviceProblem

    prob = configs.DEVICE
    seed = configs.SEED
    ncomp = 2

    def time_form(prec, fp32, scaled, antiherm=0):
        dp = DeviceProblem(prob, seed, ncomp=ncomp, fp32=fp32, scaled=scaled)
        desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                             ncomp=ncomp, prec=prec, dt_antiherm=antiherm)
        plan = sse.sse_plan(desc, prob.shifts())
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream()

        def step():
            sse.sse_compute(plan, dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma, ws, stream)

        for i in range(args.warmup):
            step()
            if args.profile_steps:
                progress(f"prec {prec} warmup {i} done")
        torch.cuda.synchronize()
        times = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            step()
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
            if args.profile_steps:
                progress(f"prec {prec} step {i}: {times[-1]*1e3:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        del dp, ws
        torch.cuda.empty_cache()
        return times, wall

    if args.calib_copy_gib > 0:
        n = int(args.calib_copy_gib * 2**30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        progress(f"calibration copy: {n * 8} bytes read, {n * 8} bytes written")
        del src, dst
        torch.cuda.empty_cache()
    if args.only in ("pi", "ablation", "aux", "serving", "batch", "shard"):
        # one section alone (profiling runs); the ablation compares with the
        # headline, so that case times one binary64 step first
        out = {}
        if args.only == "pi":
            out["phonon"] = pi_section(args, torch, sse, prob, seed, DeviceProblem, progress)
        elif args.only == "aux":
            out["aux"] = aux_section(args, torch, sse, prob, progress)
        elif args.only == "shard":
            out["shard"] = shard_section(args, torch, sse, prob, seed, DeviceProblem, progress)
        elif args.only == "serving":
            out["serving"] = serving_section(args, torch, sse, configs, progress)
        elif args.only == "batch":
            out["batch"] = batch_section(args, torch, sse, configs, DeviceProblem, progress)
        else:
            ht, _ = time_form(sse.FP64, False, False)
            out["ablation_paper_form"] = ablation_section(args, torch, sse, prob, seed,
                                                          DeviceProblem, progress,
                                                          statistics.median(ht) * 1e3)
        print(json.dumps(out), flush=True)
        return
    forms = [f for f in args.forms.split(",") if f]
    if args.only:
        forms = [args.only] if args.only != "fp64" else []
    form_out = {}
    for name in forms:
        if name == "fp64ah":
            # binary64, complex128 inputs of the headline; D~ is anti-Hermitian per block
            ft, _ = time_form(sse.FP64, False, False, antiherm=1)
            fm = statistics.median(ft)
            fl = prob.flops(antiherm=True)
            tf = fl / (fm / ncomp) / 1e12
            form_out[name] = {
                "value": round(fl * ncomp / fm / 1e9, 1), "unit": "GFLOP/s",
                "ms_per_step": round(fm * 1e3, 3), "ms_per_step_ci95": round(ci95(ft) * 1e3, 3),
                "storage": "complex128", "flops_per_component": fl,
                "inputs": "D~ anti-Hermitian per 3x3 block (dt_antiherm=1: tap work halved)",
                "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4),
                             "kernel": "k_sse_fp64<complex128, antiherm>"},
                "speedup_vs_fp64": None}
            progress(f"form {name}: {fm*1e3:.1f} ms/step")
            continue
        prec = {"fp32": sse.FP32, "bf16x3": sse.BF16X3, "fp64c64": sse.FP64C64}[name]
        ft, _ = time_form(prec, True, True)
        fm = statistics.median(ft)
        tf = prob.flops() / (fm / ncomp) / 1e12
        if name == "fp64c64":
            # the binary64 kernel on complex64 inputs and outputs (VALU)
            roof = {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4),
                    "kernel": "k_sse_fp64<complex64>"}
        else:
            roof = {"bound": "mfma", "achieved": round(tf, 3),
                    "peak": PEAK_MFMA_TFLOPS[name], "unit": "TFLOP/s",
                    "frac": round(tf / PEAK_MFMA_TFLOPS[name], 4),
                    "kernel": f"k_sse_mfma<{name}>"}
        form_out[name] = {
            "value": round(prob.flops() * ncomp / fm / 1e9, 1), "unit": "GFLOP/s",
            "ms_per_step": round(fm * 1e3, 3), "ms_per_step_ci95": round(ci95(ft) * 1e3, 3),
            "storage": "complex64", "inputs": "G magnitudes spread over ~8 decades",
            "roofline": roof, "speedup_vs_fp64": None}
        progress(f"form {name}: {fm*1e3:.1f} ms/step")
    if args.only and args.only != "fp64":
        print(json.dumps({"forms": form_out}), flush=True)
        return
    times, wall = time_form(sse.FP64, False, False)

    med = statistics.median(times)
    flops_step = prob.flops() * ncomp
    launches_per_step = ncomp
    t_launch = med / launches_per_step
    achieved_tf = prob.flops() / t_launch / 1e12
    out = {
        "metric": "SSE complex GFLOP/s (algorithmic, binary64) at device scale",
        "value": round(flops_step / med / 1e9, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med * 1e3, 3),
        "ms_per_step_ci95": round(ci95(times) * 1e3, 3),
        "wall_s_timed": round(wall, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Philox inputs: anti-Hermitian G and D~, N(0,1) dH, "
                "random neighbour table without self)",
        "config": {"workload": "Sigma lesser+greater, NA=1024 NB=4 Norb=10 Nkz=Nqz=7 NE=1000 "
                               "Nw=30 (s_w=w+1), complex128",
                   "ncomp": ncomp, "output_blocks_per_s": round(
                       prob.Nkz * prob.NE * prob.NA * ncomp / med, 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved_tf, 3),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tf / PEAK_FP64_TFLOPS, 4), "traffic": measured_traffic(),
                     "kernel": "k_sse_fp64", "launch_ms": round(t_launch * 1e3, 3)},
        "forms": form_out,
    }
    for f in form_out.values():
        f["speedup_vs_fp64"] = round(med / (f["ms_per_step"] / 1e3), 2)
    progress(f"fp64: {med*1e3:.1f} ms/step")
    log = progress
    if args.only:
        args.batch, args.serving_jobs, args.pi_steps = "", 0, 0
    if args.pi_steps > 0:
        out["phonon"] = pi_section(args, torch, sse, prob, seed, DeviceProblem, log)
    if args.shard_gpus > 0 and not args.only:
        out["shard"] = shard_section(args, torch, sse, prob, seed, DeviceProblem, log)
    if args.aux_steps > 0 and not args.only:
        out["aux"] = aux_section(args, torch, sse, prob, log)
    if args.ablation_steps > 0 and not args.only:
        out["ablation_paper_form"] = ablation_section(args, torch, sse, prob, seed,
                                                      DeviceProblem, log, med * 1e3)
    if args.batch:
        out["batch"] = batch_section(args, torch, sse, configs, DeviceProblem, log)
    if args.serving_jobs > 0:
        out["serving"] = serving_section(args, torch, sse, configs, log)
    if not args.no_cpu_baseline:
        progress(f"cpu baseline: the oracle on a sample, about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(prob, seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
