"""Benchmark: Radic subdeterminants per second on one MI355X.

Workload: the 8 x 32 float64 matrix with iid N(0, 1) entries (seed 150801328),
C(32, 8) = 10,518,300 column minors of size 8 x 8.  One step evaluates its Radic
determinant twice through the C ABI, once in FP64 and once in FP32-bulk (float
LU on power-of-two row-scaled minors, double refactorisation of flagged minors,
double-double accumulation).  Inputs are resident in device memory before the
timed region; nothing is skipped inside it.

Printed: one JSON line.  `value` is minors evaluated per second over the whole
step (both forms); the per-form rates (whole library call, events on the launch
stream), errors against the oracle (normalised by sum |det(A_J)|), the roofline
of the dominant kernel (HIP events recorded by the library around each
enumeration launch inside the timed region) and the CPU oracle's rate on the
host cores are reported beside it.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

TIME_EVERY = 4   # timed steps whose dominant kernel the library times with events: 1 in TIME_EVERY
METRIC = "Radic subdeterminants/sec, m=8 n=32: FP64 vs FP32-bulk at stated error"
UNIT = "subdeterminants/s"
PEAK_FP64_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, one FP64 FMA per lane per clock
PEAK_FP32_TFLOPS = 157.3   # published vector FP32 peak (packed FP32); unpacked issue gives 78.6


# HBM bytes per launch of the enumeration kernels on this workload, from
# rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a 256 MiB reference copy (the
# summary and commands are in profiles/k_radic_shared_8x32.md).  They hold for
# the kernel sources they were taken on: `traffic` is reported only while the
# sources hash to the same value.
KERNEL_SOURCES = ["kernels_shared.hip", "shared_lu.h", "prefix.h", "stage.h", "lu_float.h", "enumerate.h", "radic_internal.h",
                  "radic_api.cpp"]
PROFILED_TRAFFIC = {"sources_sha256": "1226dd564bd723c5bd1272d29263b48351485b3b00fcf4852925a85167193319", "fp64": 671184, "fp32_bulk": 3524917}


def kernel_sources_sha256():
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1508_01326_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(base, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_flops_per_minor(m):
    return 2.0 * m ** 3 / 3.0


def gepp_flops(rows, cols, steps):
    """Floating-point operations of `steps` steps of LU with partial pivoting on
    a rows x cols block: per step k the multipliers (one multiply each), the
    updates of the block's columns right of k (one FMA = 2 flops each) and one
    reciprocal of the pivot."""
    f = 0
    for k in range(steps):
        below = rows - 1 - k
        f += below + 2 * below * (cols - 1 - k) + 1
    return f


def executed_flops(m, n, enumeration):
    """Floating-point operations one launch performs on the whole C(n, m) rank
    space.  Per minor: GEPP of the m x m minor (m - 1 steps; 2 sum t^2 + sum t +
    (m - 1) = 315 for m = 8) plus the m - 1 multiplications of the pivot
    product.  Prefix-shared (m >= 3, P = m - 2): per prefix the P steps on the
    m x P block, the 2 x P row solve for W, and the product of its pivots; per
    later column W x (2P FMAs); per minor the 2 x 2 determinant and the product
    with the prefix's signed pivot product (4 flops).  Group-shared (m >= 4,
    P = m - 3): per group the P steps, the 3 x P row solve and the pivot
    product; per later column 3P FMAs; per pair of later columns a cross product
    (9 flops); per minor the dot product and the pivot product (6 flops)."""
    total = math.comb(n, m)
    if enumeration == "per_minor" or m < 3:
        return (gepp_flops(m, m, m - 1) + (m - 1)) * total
    kt = 3 if enumeration == "group_shared" and m >= 4 else 2
    P = m - kt
    per_prefix = gepp_flops(m, P, P) + kt * P * (P - 1) + P
    flops = 0
    for v in range(P - 1, n - kt):           # last prefix column (0-based)
        k = math.comb(v, P - 1)              # prefixes ending at v
        r = n - 1 - v                        # columns after it
        if kt == 2:
            flops += k * (per_prefix + 4 * P * r + 4 * math.comb(r, 2))
        else:
            flops += k * (per_prefix + 6 * P * r + 9 * math.comb(r, 2) + 6 * math.comb(r, 3))
    return flops


def cpu_baseline(A, threads, max_seconds=20.0):
    """The oracle (FP64 GEPP enumeration) timed on the host: the whole workload,
    repeated while under the time budget; median rate."""
    import oracle
    m, n = A.shape
    total = math.comb(n, m)
    rates, values = [], []
    t_start = time.perf_counter()
    for _ in range(3):
        t0 = time.perf_counter()
        r = oracle.radic_f64(A, nthreads=threads)
        dt = time.perf_counter() - t0
        rates.append(total / dt)
        values.append(r)
        if time.perf_counter() - t_start > max_seconds:
            break
    rates.sort()
    return rates[len(rates) // 2], values[0], len(rates)


def other_workloads(radic, binding, workloads, torch, dev, args):
    """Secondary figures (not the headline): the exact-integer 6x40 workload and
    the batched 4096-matrix workload, each timed with events around K calls
    after warm-up, checked against the oracle (exact) or sampled oracle values."""
    import numpy as np
    import oracle
    out = {}
    # exact integer path: synchronous per call (the result comes back to the host)
    A = workloads.single_matrix(3)
    m, n = A.shape
    total = math.comb(n, m)
    dA = torch.from_numpy(A).to(dev)
    work = binding.workspace(radic.RADIC_WS_INT, m, n, device=dev)
    for _ in range(max(1, args.warmup)):
        got = radic.radic_det_int_exact(dA, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        got = radic.radic_det_int_exact(dA, work=work)
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    out["exact_int_6x40"] = {"minors": total, "ms_per_call": ms, "subdet_per_s": total / (ms * 1e-3),
                             "bit_exact_vs_oracle": got == oracle.radic_int(A),
                             "note": "host-synchronous call including the 2 x 4-byte result copy"}
    # batched: one graph launch over the 4096 matrices
    mats = [M for _, M in workloads.batch_matrices()]
    batch = radic.Batch(mats, device=dev)
    g = radic.BatchGraph(batch, precision="fp32_bulk")
    for _ in range(max(1, args.warmup)):
        g.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    res = batch.results()
    minors = sum(math.comb(M.shape[1], M.shape[0]) for M in mats)
    bad = 0
    for b in range(0, len(mats), 97):                 # sampled check against the oracle
        M = mats[b]
        if M.dtype == np.int32:
            bad += res[b]["exact"] != oracle.radic_int(M)
        else:
            ref = oracle.radic_f64(M)
            bad += abs(res[b]["value"] - ref["value"]) > 1e-5 * max(ref["abs_sum"], 1e-300)
    out["batched_4096"] = {"minors": minors, "ms_per_launch": ms, "subdet_per_s": minors / (ms * 1e-3),
                           "float_precision": "fp32_bulk", "sampled_mismatches": int(bad),
                           "note": "one HIP-graph replay per launch; ints exact, floats FP32-bulk"}
    return out


def traffic_for(form, enumeration):
    if enumeration not in ("auto", "prefix_shared") or kernel_sources_sha256() != PROFILED_TRAFFIC["sources_sha256"]:
        return None
    return PROFILED_TRAFFIC[form]


def kernel_name(enumeration, form):
    if enumeration == "per_minor":
        return "k_radic_float<8,true,false,true>" if form == "fp32_bulk" else "k_radic_float<8,false,false,false>"
    if enumeration == "group_shared":
        return "k_radic_shared3<8,true>" if form == "fp32_bulk" else "k_radic_shared3<8,false>"
    return "k_radic_shared<8,true>" if form == "fp32_bulk" else "k_radic_shared<8,false>"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--enumeration", default="auto", choices=["auto", "per_minor", "prefix_shared", "group_shared"],
                    help="enumeration used by the library (default: auto, prefix-shared where supported)")
    ap.add_argument("--other", action="store_true",
                    help="also time the exact-integer workload (6x40 int32) and the batched workload "
                         "(4096 mixed matrices, one HIP-graph launch); reported under other_workloads")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="before the steps, run one plain device-to-device copy of this many bytes (a "
                         "known-size reference for the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the rank-space split across "
              "GPUs is described in DESIGN.md but not run here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1508_01326_amd as radic
    import workloads
    from paper_1508_01326_amd import binding

    A_host = workloads.single_matrix(2)
    m, n = A_host.shape
    total = math.comb(n, m)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A = torch.from_numpy(A_host).to(dev)
    radic.set_enumeration(args.enumeration)
    outs = {p: binding.new_f64_result(dev) for p in ("fp64", "fp32_bulk")}
    work = {p: binding.workspace(radic.RADIC_WS_DET, m, n, device=dev) for p in ("fp64", "fp32_bulk")}
    stream = torch.cuda.current_stream()
    print(f"[bench] workload 8x32, {total} minors, steps={args.steps} warmup={args.warmup}", file=sys.stderr,
          flush=True)

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] reference copy of {src.numel() * 4} bytes done", file=sys.stderr, flush=True)
        del src, dst

    # per form, the whole call (enumeration, refactorisation, finalisation),
    # from events on the stream the library launches on (torch's current
    # stream); these steps run after the timed ones, since each recorded event
    # is a packet of its own on the stream
    form_events = []

    def step(record=False):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if record else None
        if record:
            ev[0].record(stream)
        for i, p in enumerate(("fp64", "fp32_bulk")):
            radic.radic_det(A, precision=p, out=outs[p], work=work[p], sync=False)
            if record:
                ev[i + 1].record(stream)
        if record:
            form_events.append(ev)

    # warm-up, with the library timing both enumeration kernels: the longer
    # one is the dominant kernel of the roofline
    radic.profile_read_launches()
    radic.profile_enable(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    radic.profile_enable(False)
    warm = radic.profile_read_launches()
    dom = None
    if len(warm) >= 2:
        dom = "fp64" if sum(warm[0::2]) >= sum(warm[1::2]) else "fp32_bulk"

    def timed_step(i):
        # inside the timed region the library times the dominant kernel (with
        # events bound to its dispatch) on every TIME_EVERY-th step: a timed
        # launch lengthens its step by about 13 us (0.164 against 0.151 ms per
        # step untimed), so timing every launch would slow the steps measured
        for p in ("fp64", "fp32_bulk"):
            on = (dom is None or p == dom) and i % TIME_EVERY == 0
            if on:
                radic.profile_enable(True)
            radic.radic_det(A, precision=p, out=outs[p], work=work[p], sync=False)
            if on:
                radic.profile_enable(False)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        timed_step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = radic.profile_read_launches()
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.4f} ms/step", file=sys.stderr, flush=True)
    # per-form figures from extra steps: both kernels, and the whole calls
    radic.profile_enable(True)
    for _ in range(min(args.steps, 10)):
        step(record=True)
    torch.cuda.synchronize()
    radic.profile_enable(False)
    launches = radic.profile_read_launches()
    if dom is None:
        dom = "fp64" if sum(launches[0::2]) >= sum(launches[1::2]) else "fp32_bulk"
        dom_ms = sum(timed[(0 if dom == "fp64" else 1)::2]) / max(1, len(timed) // 2)
    else:
        dom_ms = sum(timed) / max(1, len(timed))

    k64 = launches[0::2]
    k32 = launches[1::2]
    avg64 = sum(k64) / len(k64)
    avg32 = sum(k32) / len(k32)
    call_ms = {"fp64": sum(e[0].elapsed_time(e[1]) for e in form_events) / len(form_events),
               "fp32_bulk": sum(e[1].elapsed_time(e[2]) for e in form_events) / len(form_events)}
    res = {p: binding.read_f64_result(outs[p]) for p in outs}

    # CPU oracle: baseline rate and the reference value for the error figures
    threads = min(os.cpu_count() or 1, 16)
    cpu = None
    if not args.no_cpu:
        rate, ref, reps = cpu_baseline(A_host, threads)
        cpu = {"value": rate, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"whole workload (all {total} minors, FP64 GEPP + compensated sum), "
                         f"median of {reps} run(s) on {threads} threads"}
    else:
        import oracle
        ref = oracle.radic_f64(A_host, nthreads=threads)

    S = ref["abs_sum"]
    flop = counted_flops_per_minor(m) * total
    xflop = executed_flops(m, n, args.enumeration)
    per_form = {}
    for p, avg, peak in (("fp64", avg64, PEAK_FP64_TFLOPS), ("fp32_bulk", avg32, PEAK_FP32_TFLOPS)):
        r = res[p]
        per_form[p] = {
            "subdet_per_s": total / (call_ms[p] * 1e-3),
            "call_ms": call_ms[p],
            "kernel_ms": avg,
            "value": r["value"],
            "err_over_sum_abs": abs(r["value"] - ref["value"]) / S,
            "tol": 1e-12 if p == "fp64" else 1e-5,
            "n_fallback": r["n_fallback"],
            "kernel_executed_tflops": xflop / (avg * 1e-3) / 1e12,
            "kernel_counted_tflops": flop / (avg * 1e-3) / 1e12,
            "peak_tflops": peak,
        }
    # algorithmic work: the counted (2/3) m^3 FLOP of one minor's elimination;
    # the prefix-shared kernels execute far fewer, stated beside it
    achieved = flop / (dom_ms * 1e-3) / 1e12
    peak = per_form[dom]["peak_tflops"]
    line = {
        "metric": METRIC,
        "value": 2 * total / (ms_step * 1e-3),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32bulk",
        "data": "synthetic",
        "config": {"workload": "Radic determinant of one 8x32 float64 matrix, iid N(0,1), seed 150801328; "
                               "C(32,8)=10518300 minors per form; one step = FP64 form + FP32-bulk form",
                   "m": m, "n": n, "minors_per_form": total, "forms": ["fp64", "fp32_bulk"],
                   "enumeration": args.enumeration},
        "roofline": {"bound": "alu", "kernel": kernel_name(args.enumeration, dom),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic_for(dom, args.enumeration),
                     "per_unit": f"counted (2/3) m^3 = {counted_flops_per_minor(m):.2f} FLOP per minor x {total} "
                                 f"minors per launch = {flop:.4g} FLOP; the kernel executes "
                                 f"{xflop / total:.2f} FLOP per minor (averaged over the launch; "
                                 f"{args.enumeration} enumeration), {xflop:.4g} FLOP, "
                                 f"{xflop / (dom_ms * 1e-3) / 1e12:.2f} TFLOP/s",
                     "kernel_ms": dom_ms, "launches_timed": len(timed),
                     "timed_launches": f"the dominant kernel of 1 in {TIME_EVERY} timed steps"},
        "cpu_baseline": cpu,
        "forms": per_form,
    }
    if args.other:
        line["other_workloads"] = other_workloads(radic, binding, workloads, torch, dev, args)
    for p in per_form:
        if per_form[p]["err_over_sum_abs"] > per_form[p]["tol"]:
            print(f"[bench] ERROR: {p} error {per_form[p]['err_over_sum_abs']:.3e} above tolerance",
                  file=sys.stderr)
            print(json.dumps(line))
            sys.exit(1)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
