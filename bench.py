"""Benchmark: BN254-Fr NTT throughput on one MI355X.

A step is one forward NTT of N = 2^20 seeded uniform field elements (the
2^20 four-step configuration), timed on the GPU with HIP events on the
stream the kernels run on, inputs already resident in HBM. The headline
``value`` is the int8-MFMA limb-matmul form in Melem/s (= N / time); the
butterfly form, the 2^24 coset round trip, the uneven batch and the oracle
on host cores are reported beside it. Before any timed region both forms run
alternately, untimed, for ``--settle-s`` seconds so that neither is timed
while the GPU clock is still ramping up from idle.

Prints one JSON line (see the keys below). ``--gpus`` above 1 exits: frntt
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s (published)
INT8_PEAK_TOPS = 5000.0        # MI355X dense int8 MFMA, TOP/s (published)
# The VALU peak for the 32x32+64-bit multiply-add (v_mad_u64_u32) is not a
# published figure: it is measured live by the saturating kernel of
# libfrntt_peaks.so (256 workgroups, 1..4 waves per SIMD, the best rate).
MADS_PER_PRODUCT = 162         # Montgomery product on nine 29-bit limbs (9 rows x 18)
MADS_PER_SHOUP = 154           # inter-level Shoup product: 64 quotient + 45 + 45 low columns
MADS_PER_MERGE = 32            # carry merge: 24 for the word groups + 8 for the quotient step
MADS_PER_MERGE_UNREDUCED = 24  # a merge feeding a Shoup product skips the quotient step
PASS_TABLE_MAX_LOG = 25        # the library keeps a twiddle table for non-last passes up to 2^25 entries
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mfma_fwd_2e20.txt")
# sources of the profiled kernel: the field arithmetic, the level engine and the
# translation unit instantiating the <3,4,3> plan kernel of the 2^20 passes
KERNEL_SOURCES = ["fr.hpp", "ntt_device.hpp", "ntt_levels.hpp", "ntt_plan_h.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_transform(ctx, torch, ptr, log_n, batch, kind, algo, steps, warmup, stream):
    """Warm up, then time exactly `steps` back-to-back transforms between two
    events on the launch stream, synchronised on both sides. Returns the
    mean milliseconds per transform."""
    for _ in range(warmup):
        ctx.transform_checked(ptr, log_n, batch, kind, stream, algo)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.transform_checked(ptr, log_n, batch, kind, stream, algo)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def settle_clocks(ctx, torch, fr, ptr, log_n, stream, seconds):
    """Untimed: alternate both forms' transforms for `seconds` of wall time so
    that the GPU clock has left its idle state before anything is timed.
    Without it the form timed first runs partly at a lower clock."""
    if seconds <= 0:
        return
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for algo in (fr.ALGO_FOURSTEP_MFMA, fr.ALGO_BUTTERFLY):
            for _ in range(100):
                ctx.transform_checked(ptr, log_n, 1, fr.FWD, stream, algo)
        torch.cuda.synchronize()


def level_split(l, max_m=4):
    """Radices (log2) of the MFMA levels of a pass of radix 2^l with a
    4096-element tile: fewest levels of at most 2^max_m, as even as possible,
    larger first except that a three-level split starts with its smallest
    (the library's default split)."""
    n = max(1, -(-l // max_m))
    base, extra = divmod(l, n)
    levs = [base + (1 if i < extra else 0) for i in range(n)]
    return levs[-1:] + levs[:-1] if n == 3 else levs


def algorithmic_work(plan, kind=0):
    """Per-element multiply-adds and int8 MFMA operations of each pass of a
    transform (forward: kind 0) with HBM passes `plan`."""
    out = []
    # the first pass keeps a twiddle table: an inverse transform takes N^-1
    # from it (otherwise the last pass multiplies by it), a coset transform
    # the per-line part of its pre-scale
    folded = len(plan) > 1 and sum(plan) <= PASS_TABLE_MAX_LOG
    for p, l in enumerate(plan):
        levs = level_split(l)
        # every level merges; all but the last feed an inter-level Shoup product
        # with their unreduced sum
        mads = MADS_PER_MERGE + (MADS_PER_MERGE_UNREDUCED + MADS_PER_SHOUP) * (len(levs) - 1)
        if p + 1 < len(plan):
            # pass twiddle: read from the pass table (one product), or formed
            # from the split tables (two products) above the table size limit
            mads += MADS_PER_PRODUCT * (1 if l + sum(plan[p + 1:]) <= PASS_TABLE_MAX_LOG else 2)
        if p == 0 and kind == 2:
            # coset pre-scale: one product when the first pass's table carries
            # the per-line factor (and holds the per-element one), else two
            mads += (1 if folded else 2) * MADS_PER_PRODUCT
        if p + 1 == len(plan) and kind == 1 and not folded:
            mads += MADS_PER_PRODUCT              # N^-1
        if p + 1 == len(plan) and kind == 3:
            # g^-K: one product from the first pass's table tail (two passes),
            # two from the split tables, three with N^-1
            mads += (1 if folded and len(plan) == 2 else 2 if folded else 3) * MADS_PER_PRODUCT
        rest = sum(plan[p + 1:])
        # HBM: read and write every element; a non-last pass also reads its
        # twiddle table (one 32-byte entry per element) when the library keeps one
        hbm = 64 + (32 if p + 1 < len(plan) and l + rest <= PASS_TABLE_MAX_LOG else 0)
        # int8 operations: a radix-rho level takes rho/2 MFMAs of 32x32x32 per
        # 32 vectors and output pair (even/odd split), i.e. 1024 rho per element
        out.append({"levels": levs, "mads": mads, "mfma_ops": 1024 * sum(1 << m for m in levs), "hbm_bytes": hbm})
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_17808_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the MFMA pass kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None if the kernel sources
    changed since the counters were taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def measure_peaks(table=None):
    """Sustained v_mad_u64_u32 and int8 MFMA rates of this GPU (libfrntt_peaks.so):
    the best of 1..4 waves per SIMD on one workgroup per CU. Each run's rate
    is appended to `table` if given."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2604_17808_amd", "libfrntt_peaks.so"))
    lib.frntt_peaks_run.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)] * 2
    out = {}
    for kind, name, iters in ((0, "mad_tps", 4000), (1, "mfma_tops", 4000)):
        best = 0.0
        for w in (1, 2, 3, 4):
            ms, work = ctypes.c_double(), ctypes.c_double()
            rc = lib.frntt_peaks_run(0, kind, 256, w, iters, ctypes.byref(ms), ctypes.byref(work))
            if rc != 0:
                raise RuntimeError(f"frntt_peaks_run failed with hipError {rc}")
            rate = work.value / (ms.value * 1e-3) / 1e12
            if table is not None:
                table.append({"kernel": name, "waves_per_simd": w, "ms": round(ms.value, 4),
                              "work": work.value, "rate_t_per_s": round(rate, 3)})
            best = max(best, rate)
        out[name] = round(best, 2)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(log_n_sample=20, budget_s=20.0):
    """The C oracle (radix-2, OpenMP) on this host's cores, on 2^20 forward
    transforms repeated for about `budget_s` seconds."""
    import numpy as np

    import seeded_inputs as si
    from oracle import cref
    x = si.polynomial(2, log_n_sample)
    threads = cref.max_threads()
    t0 = time.perf_counter()
    reps = 0
    while True:
        cref.transform(x, log_n_sample, 0, threads=threads)
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": round((1 << log_n_sample) / dt / 1e6, 3), "unit": "Melem/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{reps} forward NTTs of 2^{log_n_sample} (seed 2) with the plain C radix-2 "
                      f"oracle, OpenMP over {threads} threads, {dt * 1e3:.1f} ms each"}


def plan_kernel_name(ctx, algo, log_n):
    """Name of the tile kernel the first pass of 2^log_n runs (ntt_plan_kernel_abc
    for in-tile levels of 2^a, 2^b, 2^c)."""
    levs = ctx.get_plan_levels(algo, log_n, 0)
    return "ntt_plan_kernel_" + "".join(str(v) for v in (levs + [0, 0, 0])[:3])


def bench_f1(ctx, torch, fr, stream, steps):
    """Two HBM passes against three (the recursive five-step split) at 2^22 and
    2^24, both forms, forward: time per transform and the pass-twiddle table
    memory each plan adds; and the two-pass plan with the split tables only
    (no pass table)."""
    out = {}
    for log_n, plans in ((22, ([11, 11], [8, 7, 7])), (24, ([12, 12], [8, 8, 8]))):
        n = 1 << log_n
        buf = torch.empty((n, 4), dtype=torch.int64, device="cuda:0")
        ctx.generate(buf.data_ptr(), 6, 0, 0, n, stream)
        row = {}
        for name, algo in (("mfma", fr.ALGO_FOURSTEP_MFMA), ("butterfly", fr.ALGO_BUTTERFLY)):
            for plan in plans:
                log(f"f1: 2^{log_n} {name} plan {plan}")
                ctx.set_plan(algo, log_n, plan)
                before = ctx.table_bytes()
                ctx.transform_checked(buf.data_ptr(), log_n, 1, fr.FWD, stream, algo)   # builds its tables
                torch.cuda.synchronize()
                table = ctx.table_bytes() - before
                t = time_transform(ctx, torch, buf.data_ptr(), log_n, 1, fr.FWD, algo, steps, 2, stream)
                row[f"{name}_{'x'.join(map(str, plan))}"] = {
                    "ms": round(t, 4), "melem_s": round(n / (t * 1e-3) / 1e6, 1),
                    "table_mib_added": round(table / 2**20, 1)}
            ctx.set_plan(algo, log_n, [])
        # the same two-pass plan with the split tables instead of a pass table
        # (FRNTT_SPLIT_TWIDDLES: every pass twiddle is one more product)
        sctx = fr.Context(0, max_log_n=log_n, flags=fr.frntt.SPLIT_TWIDDLES)
        for name, algo in (("mfma", fr.ALGO_FOURSTEP_MFMA), ("butterfly", fr.ALGO_BUTTERFLY)):
            plan = plans[0]
            log(f"f1: 2^{log_n} {name} plan {plan}, split tables")
            sctx.set_plan(algo, log_n, plan)
            t = time_transform(sctx, torch, buf.data_ptr(), log_n, 1, fr.FWD, algo, steps, 2, stream)
            row[f"{name}_{'x'.join(map(str, plan))}_split_tables"] = {
                "ms": round(t, 4), "melem_s": round(n / (t * 1e-3) / 1e6, 1),
                "table_mib_total": round(sctx.table_bytes() / 2**20, 2)}
        torch.cuda.synchronize()
        sctx.close()
        out[f"2e{log_n}"] = row
        del buf
    return out


def time_op(torch, fn, steps, warmup):
    """Mean milliseconds of `fn` (which enqueues on the current stream) over
    `steps` back-to-back calls between two events, after `warmup` calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# RNS lazy product (Alg. 1): per element, the int8 MFMA work of Main (2 row
# blocks x 3 K steps of 32x32x32 per 32 elements) and the HBM bytes of each
# call (base Q: 20 words, base P: 12 words, canonical: 8 words)
RNS_MUL_OPS = 2 * 3 * 2 * 32 * 32 * 32 // 32
RNS_BYTES = {"encode": 32 + 80, "mul": 2 * 80 + 48, "decode": 48 + 32, "mont_mul": 3 * 32}


def bench_f2(ctx, torch, fr, stream, steps):
    """The RNS lazy modular product against the radix Montgomery product on the
    VALUs (the paper's arithmetic ablation) at batch sizes 2^20, 2^22, 2^24:
    elements per second of each call and of the whole canonical-to-canonical
    pipeline (two encodes, the product, one decode), with the HBM bandwidth
    each call reaches and the int8 MFMA rate of the product."""
    out = {}
    for log_n in (20, 22, 24):
        n = 1 << log_n
        a = torch.empty((n, 4), dtype=torch.int64, device="cuda:0")
        b = torch.empty_like(a)
        ctx.generate(a.data_ptr(), 8, 0, 0, n, stream)
        ctx.generate(b.data_ptr(), 8, 1, 0, n, stream)
        xa = torch.empty((n * fr.RNS_Q_WORDS,), dtype=torch.int32, device="cuda:0")
        xb = torch.empty_like(xa)
        xp = torch.empty((n * fr.RNS_P_WORDS,), dtype=torch.int32, device="cuda:0")
        o = torch.empty_like(a)
        ops = {
            "encode": lambda: ctx.rns_encode(a.data_ptr(), xa.data_ptr(), n, stream),
            "mul": lambda: ctx.rns_mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, stream),
            "decode": lambda: ctx.rns_decode(xp.data_ptr(), o.data_ptr(), n, stream),
            "mont_mul": lambda: ctx.mont_mul(a.data_ptr(), b.data_ptr(), o.data_ptr(), n, stream),
        }
        ctx.rns_encode(b.data_ptr(), xb.data_ptr(), n, stream)
        row = {}
        for name, fn in ops.items():
            log(f"f2: 2^{log_n} {name}")
            t = time_op(torch, fn, steps, 2) * 1e-3
            row[name] = {"us": round(t * 1e6, 2), "melem_s": round(n / t / 1e6, 1),
                         "hbm_gbs": round(n * RNS_BYTES[name] / t / 1e9, 1)}
        row["mul"]["mfma_tops"] = round(n * RNS_MUL_OPS / (row["mul"]["us"] * 1e-6) / 1e12, 2)

        def pipeline():
            ops["encode"]()
            ctx.rns_encode(b.data_ptr(), xb.data_ptr(), n, stream)
            ops["mul"]()
            ops["decode"]()
        t = time_op(torch, pipeline, steps, 2) * 1e-3
        row["pipeline"] = {"us": round(t * 1e6, 2), "melem_s": round(n / t / 1e6, 1)}
        row["mul_over_mont"] = round(row["mont_mul"]["us"] / row["mul"]["us"], 3)
        out[f"2e{log_n}"] = row
        del a, b, xa, xb, xp, o
        torch.cuda.empty_cache()
    return out


# Baby Jubjub's published generator of the prime-order subgroup; the MSM
# workload's points are k_i times it (k_i uniform field elements)
MSM_BASE = (5299619240641551281634865583518297030282874472190772894086521144482721001553,
            16950150798460657717958625567821834550301663161624707787222815936182638968203)
MONT_MADS = 162   # 32x32+64-bit multiply-adds of one 9-limb Montgomery product


def msm_products(n, c):
    """Montgomery products of one MSM of n points with c-bit windows, in the
    a = -1 model the kernels use: the point preparation (4 per point), the
    bucket accumulation (7 per added point), the tree reduction (two
    additions into W, one addition and one doubling into B per bucket pair
    and level: 9 + 9 + 9 + 8), and the window merging (c doublings and one
    addition per window)."""
    K = -(-256 // c)
    prep = 4 * n
    accum = 7 * n * K
    reduce_ = K * ((1 << c) - 1) * (9 + 9 + 9 + 8)
    merge = K * (8 * c + 9 + 1) + 6
    return prep + accum + reduce_ + merge


def bench_f4(ctx, torch, fr, stream, steps):
    """Multi-scalar multiplication (Alg. 2, LS-PPG) on the twisted Edwards
    curve over Fr at 2^20, 2^22, 2^24 and 2^26 points (the paper's 256-bit
    MSM runs 2^22 to 2^26): milliseconds per MSM, points per second, the rate of
    Montgomery-product multiply-adds the whole MSM sustains, and the time of
    the Presort-PPG baseline (the paper's dataflow baseline) beside it up to
    2^24, and a batch of four MSMs in one call (frntt_msm_batch) against
    four single calls at 2^20 and 2^22. Points are k_i G
    from the batch scalar multiplication, scalars uniform field elements."""
    out = {}
    for log_n in (20, 22, 24, 26):
        n = 1 << log_n
        k = torch.empty((n, 4), dtype=torch.int64, device="cuda:0")
        sc = torch.empty_like(k)
        ctx.generate(k.data_ptr(), 21, 0, 0, n, stream)
        ctx.generate(sc.data_ptr(), 21, 1, 0, n, stream)
        g = torch.tensor([[(v >> (32 * i)) & 0xFFFFFFFF for v in MSM_BASE for i in range(8)]],
                         dtype=torch.int64).to(torch.int32).to("cuda:0")
        g = g.expand(n, 16).contiguous()
        pts = torch.empty((n, 16), dtype=torch.int32, device="cuda:0")
        ctx.ec_mul(k.data_ptr(), g.data_ptr(), n, pts.data_ptr(), stream)
        del g, k
        o = torch.empty(16, dtype=torch.int32, device="cuda:0")
        c = fr.msm_window(n)
        log(f"f4: msm 2^{log_n} window {c}")
        t = time_op(torch, lambda: ctx.msm(sc.data_ptr(), pts.data_ptr(), n, o.data_ptr(), 0, stream),
                    steps, 1) * 1e-3
        mads = msm_products(n, c) * MONT_MADS
        row = {"window": c, "ms": round(t * 1e3, 3), "mpoints_s": round(n / t / 1e6, 2),
               "tmad_s": round(mads / t / 1e12, 3)}
        if log_n <= 22:
            # four independent MSMs in one batched call (side streams) against
            # the same four one after another
            outs = [torch.empty(16, dtype=torch.int32, device="cuda:0") for _ in range(4)]
            log(f"f4: msm 2^{log_n} batch of 4")
            tq = time_op(torch, lambda: ctx.msm_batch([sc.data_ptr()] * 4, [pts.data_ptr()] * 4, [n] * 4,
                                                      [q.data_ptr() for q in outs], 0, stream), steps, 1) * 1e-3
            row["batch4_ms"] = round(tq * 1e3, 3)
            row["batch4_speedup"] = round(4 * t / tq, 3)
            del outs
        if log_n <= 24:  # the baseline's presorted copy is K n 96 bytes (80 GB at 2^26)
            log(f"f4: msm 2^{log_n} Presort-PPG baseline")
            tb = time_op(torch, lambda: ctx.msm_presort(sc.data_ptr(), pts.data_ptr(), n, o.data_ptr(), 0, stream),
                         steps, 1) * 1e-3
            row["presort_ms"] = round(tb * 1e3, 3)
            row["ls_over_presort"] = round(tb / t, 3)
        out[f"2e{log_n}"] = row
        del sc, pts, o
        torch.cuda.empty_cache()
    return out


def bench_f3(ctx, torch, fr, stream, steps):
    """The RNS lazy product against the radix Montgomery product at the wider
    widths the paper evaluates (the largest primes below 2^377 and 2^753), at
    2^20 and 2^22 elements: elements per second of each call and of the whole
    pipeline, the HBM bandwidth of each call, the product's int8 MFMA rate.
    Inputs are uniform below 2^bits (values of M or above, probability
    about 2^-369, are not excluded)."""
    out = {}
    for bits, modulus in ((377, fr.FIELD_377), (753, fr.FIELD_753)):
        f = fr.RnsField(ctx, modulus)
        mw, qw, pw = f.words, f.q_words, f.p_words
        # int8 operations of Main per element: row blocks x K steps of 32x32x32 per 32 elements
        rbm, ksq = (4 * f.n_p + 3 + 31) // 32, (f.n_q + 7) // 8
        ops = rbm * ksq * 2 * 32 * 32 * 32 // 32
        nbytes = {"encode": 4 * (mw + qw), "mul": 4 * (2 * qw + pw), "decode": 4 * (pw + mw), "mont_mul": 12 * mw}
        row_w = {}
        for log_n in (20, 22):
            n = 1 << log_n
            gen = torch.Generator(device="cuda:0")
            gen.manual_seed(bits + log_n)
            a = torch.randint(-2**31, 2**31, (n, mw), dtype=torch.int64, device="cuda:0", generator=gen)
            a = a.to(torch.int32)
            top_bits = bits - 32 * (mw - 1)
            a[:, mw - 1] &= (1 << top_bits) - 1
            b = torch.randint(-2**31, 2**31, (n, mw), dtype=torch.int64, device="cuda:0", generator=gen).to(torch.int32)
            b[:, mw - 1] &= (1 << top_bits) - 1
            xa = torch.empty((n * qw,), dtype=torch.int32, device="cuda:0")
            xb = torch.empty_like(xa)
            xp = torch.empty((n * pw,), dtype=torch.int32, device="cuda:0")
            o = torch.empty_like(a)
            f.encode(b.data_ptr(), xb.data_ptr(), n, stream)
            calls = {
                "encode": lambda: f.encode(a.data_ptr(), xa.data_ptr(), n, stream),
                "mul": lambda: f.mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, stream),
                "decode": lambda: f.decode(xp.data_ptr(), o.data_ptr(), n, stream),
                "mont_mul": lambda: f.mont_mul(a.data_ptr(), b.data_ptr(), o.data_ptr(), n, stream),
            }
            row = {}
            for name, fn in calls.items():
                log(f"f3: {bits} bits 2^{log_n} {name}")
                t = time_op(torch, fn, steps, 2) * 1e-3
                row[name] = {"us": round(t * 1e6, 2), "melem_s": round(n / t / 1e6, 1),
                             "hbm_gbs": round(n * nbytes[name] / t / 1e9, 1)}
            row["mul"]["mfma_tops"] = round(n * ops / (row["mul"]["us"] * 1e-6) / 1e12, 2)

            def pipeline():
                calls["encode"]()
                f.encode(b.data_ptr(), xb.data_ptr(), n, stream)
                calls["mul"]()
                calls["decode"]()
            t = time_op(torch, pipeline, steps, 2) * 1e-3
            row["pipeline"] = {"us": round(t * 1e6, 2), "melem_s": round(n / t / 1e6, 1)}
            row["mul_over_mont"] = round(row["mont_mul"]["us"] / row["mul"]["us"], 3)
            row_w[f"2e{log_n}"] = row
            del a, b, xa, xb, xp, o
            torch.cuda.empty_cache()
        torch.cuda.synchronize()
        f.close()
        out[f"{bits}bit"] = row_w
    return out


def bench_c4(ctx, torch, fr, stream, replays):
    """256 forward NTTs, sizes uniform over 2^12..2^20 (seed 4): tune every
    size, capture the persistent batch launch in a hipGraph, time replays."""
    import seeded_inputs as si
    sizes = si.uneven_batch_sizes(4, 256, 12, 20)
    tuned = {}
    for l in sorted(set(sizes)):
        log(f"c4: tuning 2^{l}")
        algo, npass, ms = ctx.tune(l, 1, stream)
        tuned[l] = {"algo": "mfma" if algo == fr.ALGO_FOURSTEP_MFMA else "butterfly",
                    "passes": ctx.get_plan(fr.ALGO_AUTO, l), "ms": round(ms, 4)}
    bufs = []
    for j, l in enumerate(sizes):
        t = torch.empty((1 << l, 4), dtype=torch.int64, device="cuda:0")
        ctx.generate(t.data_ptr(), 4, j, 0, 1 << l, stream)
        bufs.append(t)
    jobs = [(b.data_ptr(), l, 0) for b, l in zip(bufs, sizes)]
    log(f"c4: {replays} graph replays")
    ctx.batch(jobs, stream, graph=True)                    # capture
    torch.cuda.synchronize()
    times = []
    for _ in range(replays):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.batch(jobs, stream, graph=True)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    total = sum(1 << l for l in sizes)
    p50 = times[len(times) // 2]
    p99 = times[min(len(times) - 1, int(round(0.99 * (len(times) - 1))))]
    del bufs
    return {"jobs": 256, "elements": total, "replays": replays, "p50_ms": round(p50, 4),
            "p99_ms": round(p99, 4), "melem_s_at_p50": round(total / (p50 * 1e-3) / 1e6, 1),
            "tuned": tuned}


def bench_c5(ctx, fr, n_requests):
    """Poisson arrivals of NTT/INTT/coset-NTT (40/40/20), sizes uniform over
    2^14..2^22, 64 GiB budget, at 0.5/0.8/0.95 of the measured saturation rate."""
    import seeded_inputs as si
    srv = fr.Server(ctx, 64 << 30, slots=4)
    srv.set_release_on_done(True)            # results stay on the device; only latency is read
    try:
        # saturation: a burst of requests with the same size/kind mix
        burst = si.request_stream(1005, min(2000, n_requests), 14, 22, rate_per_s=1.0)
        log("c5: warm-up + saturation burst")
        warm = [srv.submit(r["kind"], r["log_n"], 5) for r in burst[:200]]
        srv.drain(600)
        t0 = time.perf_counter()
        tks = [srv.submit(r["kind"], r["log_n"], 5) for r in burst]
        srv.drain(600)
        sat = len(burst) / (time.perf_counter() - t0)
        res = {"saturation_req_s": round(sat, 1), "requests": n_requests, "budget_gib": 64, "slots": 4}
        for frac in (0.5, 0.8, 0.95):
            rate = frac * sat
            reqs = si.request_stream(5, n_requests, 14, 22, rate_per_s=rate)
            log(f"c5: {n_requests} requests at {rate:.0f}/s")
            t0 = time.perf_counter()
            tks = []
            for r in reqs:
                while time.perf_counter() - t0 < r["t_arrive_s"]:
                    pass
                tks.append(srv.submit(r["kind"], r["log_n"], 5))
            srv.drain(600)
            wall = time.perf_counter() - t0
            lats = []
            for tk in tks:
                done, lat = srv.poll(tk)
                lats.append(lat)
            lats.sort()
            elems = sum(1 << r["log_n"] for r in reqs)
            res[f"lambda_{frac}"] = {
                "rate_req_s": round(rate, 1), "p50_ms": round(lats[len(lats) // 2], 3),
                "p99_ms": round(lats[int(0.99 * (len(lats) - 1))], 3),
                "throughput_req_s": round(len(reqs) / wall, 1),
                "throughput_melem_s": round(elems / wall / 1e6, 1)}
        st = srv.stats()
        res["batches"] = st["batches"]
        res["peak_gib"] = round(st["peak_bytes"] / 2**30, 2)
        res["peak_inflight_batches"] = st["peak_inflight_batches"]
        res["peak_inflight_requests"] = st["peak_inflight_requests"]
        res["generation"] = c5_generation_time(ctx, reqs)
        return res
    finally:
        srv.close()


def c5_generation_time(ctx, reqs):
    """Device time of generating the request data alone (the server does it on
    the device at admission, inside each request's latency): every request of
    the stream generated back to back into one buffer, between two events."""
    import torch
    biggest = max(r["log_n"] for r in reqs)
    buf = torch.empty(((1 << biggest), 4), dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i, r in enumerate(reqs):
        ctx.generate(buf.data_ptr(), 5, i + 1, 0, 1 << r["log_n"], stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del buf
    return {"total_ms": round(ms, 2), "mean_ms_per_request": round(ms / len(reqs), 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing on host cores")
    ap.add_argument("--quick", action="store_true", help="headline config only")
    ap.add_argument("--only", default="c3,c4,c5,f1,f2,f3,f4",
                    help="comma list of the other configurations to run (c3, c4, c5, f1, f2, f3, f4)")
    ap.add_argument("--c4-replays", type=int, default=200)
    ap.add_argument("--calib", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="untimed seconds of alternating transforms before the first timed region")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the multiply-add and int8 MFMA rate microbenchmarks and print their table")
    args = ap.parse_args()
    extra = set() if args.quick else {c.strip() for c in args.only.split(",") if c.strip()}
    if args.gpus != 1:
        print("bench.py: frntt runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_17808_amd as fr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.peaks:
        table = []
        best = measure_peaks(table)
        print(json.dumps({"peaks": best, "runs": table}), flush=True)
        return
    ctx = fr.Context(0, max_log_n=24)
    stream = torch.cuda.current_stream().cuda_stream
    out = {}

    if args.calib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale factor for the transform kernels' counters
        a = torch.zeros(256 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---- headline: 2^20 forward, MFMA vs butterfly
    log_n = 20
    n = 1 << log_n
    buf = torch.empty((n, 4), dtype=torch.int64, device="cuda:0")
    ctx.generate(buf.data_ptr(), 2, 0, 0, n, stream)
    log(f"settling clocks for {args.settle_s} s")
    settle_clocks(ctx, torch, fr, buf.data_ptr(), log_n, stream, args.settle_s)
    res = {}
    for name, algo in (("mfma", fr.ALGO_FOURSTEP_MFMA), ("butterfly", fr.ALGO_BUTTERFLY)):
        log(f"timing 2^20 forward {name}")
        t = time_transform(ctx, torch, buf.data_ptr(), log_n, 1, fr.FWD, algo, args.steps, args.warmup,
                           stream)
        res[name] = {"ms": t, "melem_s": n / (t * 1e-3) / 1e6, "plan": ctx.get_plan(algo, log_n)}
    mf = res["mfma"]
    out["c2"] = res
    # the tile kernel the timed passes ran (the autotuner of the batch may
    # change the plan of 2^20 later)
    headline_kernel = plan_kernel_name(ctx, fr.ALGO_FOURSTEP_MFMA, log_n)

    # ---- C1: 2^10 forward + inverse, butterfly form, microseconds per call
    b10 = torch.empty((1024, 4), dtype=torch.int64, device="cuda:0")
    ctx.generate(b10.data_ptr(), 1, 0, 0, 1024, stream)
    c1 = {}
    for kind_name, kind in (("fwd", fr.FWD), ("inv", fr.INV)):
        c1[kind_name + "_us"] = round(1e3 * time_transform(ctx, torch, b10.data_ptr(), 10, 1, kind,
                                                          fr.ALGO_BUTTERFLY, 200, 5, stream), 3)
    out["c1"] = c1
    del b10

    if "c3" in extra:
        # ---- 2^24 coset NTT then coset INTT, both forms, per transform
        log(f"timing 2^24 coset round trip")
        n24 = 1 << 24
        b24 = torch.empty((n24, 4), dtype=torch.int64, device="cuda:0")
        ctx.generate(b24.data_ptr(), 3, 0, 0, n24, stream)
        c3 = {}
        for name, algo in (("mfma", fr.ALGO_FOURSTEP_MFMA), ("butterfly", fr.ALGO_BUTTERFLY)):
            steps = max(3, args.steps // 5)
            t_f = time_transform(ctx, torch, b24.data_ptr(), 24, 1, fr.COSET, algo, steps, 2, stream)
            t_i = time_transform(ctx, torch, b24.data_ptr(), 24, 1, fr.COSET_INV, algo, steps, 2, stream)
            c3[name] = {"coset_ms": t_f, "coset_inv_ms": t_i, "melem_s": n24 / (t_f * 1e-3) / 1e6,
                        "roundtrip_melem_s": n24 / ((t_f + t_i) * 1e-3) / 1e6,
                        "plan": ctx.get_plan(algo, 24)}
        out["c3"] = c3
        del b24

    if "f1" in extra:
        out["f1"] = bench_f1(ctx, torch, fr, stream, max(3, args.steps // 10))
    if "f2" in extra:
        out["f2"] = bench_f2(ctx, torch, fr, stream, max(5, args.steps // 4))
    if "f3" in extra:
        out["f3"] = bench_f3(ctx, torch, fr, stream, max(5, args.steps // 4))
    if "f4" in extra:
        out["f4"] = bench_f4(ctx, torch, fr, stream, 3)
    if "c4" in extra:
        out["c4"] = bench_c4(ctx, torch, fr, stream, args.c4_replays)
    if "c5" in extra:
        out["c5"] = bench_c5(ctx, fr, args.serve_requests)

    # ---- roofline of the dominant kernel (the MFMA pass kernel) on the
    # headline workload: algorithmic work per launch / average launch time,
    # for each unit (Big-T): int8 MFMA, VALU multiply-adds, HBM bytes. The
    # bound is the unit with the largest fraction of its peak.
    log("measuring the VALU multiply-add and int8 MFMA rates")
    peaks = measure_peaks()
    for row in out.get("f4", {}).values():
        row["alu_frac"] = round(row["tmad_s"] / peaks["mad_tps"], 4)
    work = algorithmic_work(mf["plan"])
    launches = len(mf["plan"])
    per_launch_ms = mf["ms"] / launches
    t = per_launch_ms * 1e-3
    mads = n * sum(w["mads"] for w in work) / launches
    ops = n * sum(w["mfma_ops"] for w in work) / launches
    hbm = n * sum(w["hbm_bytes"] for w in work) / launches
    terms = {
        "mfma": {"achieved": ops / t / 1e12, "peak": INT8_PEAK_TOPS, "unit": "TOP/s", "work_per_launch": ops,
                 "peak_source": "published dense int8"},
        "alu": {"achieved": mads / t / 1e12, "peak": peaks["mad_tps"], "unit": "Tmad/s", "work_per_launch": mads,
                "peak_source": "measured v_mad_u64_u32 rate (libfrntt_peaks)"},
        "hbm": {"achieved": hbm / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "work_per_launch": hbm,
                "peak_source": "published HBM3E"},
    }
    for v in terms.values():
        v["frac"] = round(v["achieved"] / v["peak"], 4)
        v["achieved"] = round(v["achieved"], 3)
    bound = max(terms, key=lambda k: terms[k]["frac"])
    roofline = {"bound": bound, "achieved": terms[bound]["achieved"], "peak": terms[bound]["peak"],
                "unit": terms[bound]["unit"], "frac": terms[bound]["frac"], "traffic": measured_traffic(),
                "kernel": headline_kernel, "launch_ms": round(per_launch_ms, 5),
                "terms": terms, "measured_peaks": peaks}
    if "c3" in out:
        # C3 (2^24 coset NTT, MFMA form): achieved HBM bandwidth and int8 MFMA
        # utilisation from the algorithmic bytes and operations of the transform
        w3 = algorithmic_work(out["c3"]["mfma"]["plan"], kind=2)
        n24 = 1 << 24
        t3 = out["c3"]["mfma"]["coset_ms"] * 1e-3
        out["c3"]["mfma"]["hbm_gbs"] = round(n24 * sum(w["hbm_bytes"] for w in w3) / t3 / 1e9, 1)
        out["c3"]["mfma"]["mfma_util"] = round(n24 * sum(w["mfma_ops"] for w in w3) / t3 / 1e12 / INT8_PEAK_TOPS, 4)
        out["c3"]["mfma"]["valu_mad_frac"] = round(n24 * sum(w["mads"] for w in w3) / t3 / 1e12 / peaks["mad_tps"], 4)

    cpu = None if args.no_cpu else cpu_baseline()

    line = {
        "metric": "BN254-Fr NTT Melem/s at N=2^20 (int8-MFMA limb-matmul form)",
        "value": round(mf["melem_s"], 2),
        "unit": "Melem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": args.settle_s,
        "ms_per_step": round(mf["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "single forward NTT, N=2^20, BN254 Fr, uniform seeded coefficients "
                               "(seed 2), four-step int8-MFMA form, batch 1",
                   "log_n": 20, "batch": 1, "plan_passes": mf["plan"]},
        "butterfly_melem_s": round(res["butterfly"]["melem_s"], 2),
        "mfma_over_butterfly": round(mf["melem_s"] / res["butterfly"]["melem_s"], 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": out,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
