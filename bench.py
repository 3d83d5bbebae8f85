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
# the kernel sources and the launch shape (subsets per lane, "spl") they were
# taken on: `traffic` is reported only while the sources hash to the same value
# and the run uses the same shape.
KERNEL_SOURCES = ["kernels_shared.hip", "shared_round.h", "shared_lu.h", "prefix.h", "split.h", "stage.h", "lu_float.h", "enumerate.h",
                  "radic_internal.h", "radic_api.cpp"]
PROFILED_TRAFFIC = {"sources_sha256": "0587ed8f1ed234ec4c0fadc60ee478cd891222b0653a10aedb933b55ebdee406", "spl": {"fp64": 48, "fp32_bulk": 80}, "fp64": 415463, "fp32_bulk": 1022437}
# the library's default subsets per lane for the prefix-shared float kernels
DEFAULT_SPL_SHARED = 64
# launch shapes written by the library's autotuner (paper_1508_01326_amd/tune_shapes.py)
TUNED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1508_01326_amd", "tuned_gfx950.txt")
ENUM_CODES = {"auto": 0, "per_minor": 1, "prefix_shared": 2, "group_shared": 3}


def table_shapes(path, m, n, enumeration):
    """Subsets per lane per float precision that a launch-shape table gives an
    m x n matrix under the enumeration (rows: kind prec m n_bucket enumeration
    spl block; kind 0 is a single float matrix)."""
    nb = n if n <= 16 else ((n + 7) // 8 * 8 if n <= 64 else (n + 31) // 32 * 32)
    out = {}
    with open(path) as f:
        for line in f:
            v = line.split()
            if (len(v) == 7 and v[0] == "0" and v[1] in ("0", "1") and int(v[2]) == m and int(v[3]) == nb
                    and int(v[4]) == ENUM_CODES[enumeration]):
                out["fp64" if v[1] == "0" else "fp32_bulk"] = int(v[5])
    return out
# FLOPs per launch counted by SQ_INSTS_VALU_FLOPS_FP32/FP64 (x 64 lanes) on the same sources
PROFILED_FLOPS = {"fp64": {"fp32": 1600000, "fp64": 247332032}, "fp32_bulk": {"fp32": 204090112, "fp64": 87046528}}
# VALU wave instructions per launch (SQ_INSTS_VALU) on the same sources
PROFILED_VALU = {"fp64": 13410005, "fp32_bulk": 16581212}
# wave-instruction issue rate of the VALUs: 256 CU x 4 SIMD x 2.4 GHz, one
# 64-lane instruction per SIMD every 4 clocks (16 lanes per clock)
PEAK_VALU_ISSUE = 256 * 4 * 2.4e9 / 4


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
        r = n - 1 - v                        # columns after it
        if kt == 2:
            # two-sided blocks: the prefixes ending at v on either side
            k = split_prefix_count(P, n, 0, v) + split_prefix_count(P, n, 1, v)
            flops += k * (per_prefix + 4 * P * r + 4 * math.comb(r, 2))
        else:
            k = math.comb(v, P - 1)          # prefixes ending at v
            flops += k * (per_prefix + 6 * P * r + 9 * math.comb(r, 2) + 6 * math.comb(r, 3))
    return flops


def split_prefix_count(P, n, side, v):
    """Prefixes of P = m - 2 columns ending at column v on one side of the
    prefix-shared kernels' two-sided blocks over a whole rank space: a minor is
    shared through its first m - 2 columns (side 0) when at least as many
    columns follow them as precede its last m - 2 (side 1, the same in the
    column-reversed matrix), so a side-s prefix c is taken when c_2 <= r - s,
    r = n - 1 - v; below m = 5 every prefix is on side 0."""
    if P <= 2:
        return math.comb(v, P - 1) if side == 0 else 0
    L = n - 1 - v - side
    if P == 3:
        return math.comb(v, 2) if v <= L else 0
    a = min(L + 1, v)
    return sum(math.comb(a, i) * math.comb(v - a, P - 1 - i) for i in range(3, P))


def host_info():
    """Host CPU: logical cores the process may use and the model name."""
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return nproc, model


def cpu_baseline(A, threads, max_seconds=20.0):
    """The oracle (FP64 GEPP enumeration, compensated sum) timed on the host: the
    whole workload on `threads` threads, repeated while under the time budget
    (median rate), then once on one thread."""
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
    t0 = time.perf_counter()
    oracle.radic_f64(A, nthreads=1)
    rate1 = total / (time.perf_counter() - t0)
    return rates[len(rates) // 2], values[0], len(rates), rate1


def read_golden(name):
    """Stored expected values written by tests/golden/make_golden.py (oracle only)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def timed_calls(fn, steps, torch):
    """Mean wall time of `steps` calls of fn() (each waits for its result), ms."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def kernel_ms(radic, fn, reps):
    """Mean duration of the main enumeration kernel of fn() (library timing hook)."""
    radic.profile_read_launches()
    radic.profile_enable(True)
    for _ in range(reps):
        fn()
    radic.profile_enable(False)
    ms = radic.profile_read_launches()
    return sum(ms) / len(ms) if ms else None


def other_workloads(radic, binding, workloads, torch, dev, args):
    """The other configurations, each checked against the oracle or the stored
    oracle values: the 5x14 latency case, the exact 6x40 int32 matrix, the 12x36
    precision stress in both precisions and the 4096-matrix batch."""
    import numpy as np
    from fractions import Fraction
    from oracle import exact
    out = {}

    # 5 x 14, 2002 minors: end-to-end latency of one synchronous call through
    # the C ABI (enqueue, kernels, wait; the finalize kernel writes the 56-byte
    # result into the binding's pinned host buffer)
    A = workloads.single_matrix(1)
    dA = torch.from_numpy(A).to(dev)
    ex = float(exact.radic_subset_dp(A))
    res = {}
    for p in ("fp64", "fp32_bulk"):
        w = binding.workspace(radic.RADIC_WS_DET, 5, 14, device=dev)
        call = lambda: radic.radic_det(dA, precision=p, work=w)   # noqa: E731
        for _ in range(10):
            r = call()
        ms = timed_calls(call, 200, torch)
        S = r["abs_sum"]
        res[p] = {"latency_us": ms * 1e3, "err_over_sum_abs_vs_exact": abs(r["value"] - ex) / S,
                  "kernel_us": kernel_ms(radic, call, 20) * 1e3}
    out["w1_5x14"] = {"minors": 2002, "forms": res,
                      "note": "latency = one synchronous call, result read from pinned host memory, mean of 200"}

    # 6 x 40 int32, exact: synchronous call (the CRT kernel writes the result
    # into pinned host memory)
    A = workloads.single_matrix(3)
    m, n = A.shape
    total = math.comb(n, m)
    dA = torch.from_numpy(A).to(dev)
    work = binding.workspace(radic.RADIC_WS_INT, m, n, device=dev)
    call = lambda: radic.radic_det_int_exact(dA, work=work)   # noqa: E731
    for _ in range(5):
        got = call()
    ms = timed_calls(call, 50, torch)
    kms = kernel_ms(radic, call, 10)
    out["w3_6x40_exact"] = {"minors": total, "ms_per_call": ms, "subdet_per_s": total / (ms * 1e-3),
                            "kernel": "k_radic_int_shared<6>", "kernel_ms": kms, "primes": 2,
                            "minor_primes_per_s_kernel": 2 * total / (kms * 1e-3),
                            "bit_exact_vs_oracle": got == exact.radic_subset_dp(A)}

    # 12 x 36 precision stress: 1,251,677,700 minors per form
    A = workloads.single_matrix(4)
    g = {r[0]: r[1] for r in read_golden("workload4_12x36.txt")}
    ex = float(Fraction(int(g["exact_num"]), int(g["exact_den"])))
    S = float(g["oracle_abs_sum"])
    total = math.comb(36, 12)
    dA = torch.from_numpy(A).to(dev)
    res = {}
    for p in ("fp64", "fp32_bulk"):
        o = binding.new_f64_result(dev)
        w = binding.workspace(radic.RADIC_WS_DET, 12, 36, device=dev)
        call = lambda: radic.radic_det(dA, precision=p, out=o, work=w)   # noqa: E731
        r = call()
        ms = timed_calls(call, 3, torch)
        kms = kernel_ms(radic, call, 2)
        enum = "auto"
        xf = executed_flops(12, 36, enum)
        peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
        res[p] = {"ms_per_call": ms, "subdet_per_s": total / (ms * 1e-3),
                  "err_over_sum_abs_vs_exact": abs(r["value"] - ex) / S, "tol": 1e-12 if p == "fp64" else 1e-5,
                  "n_fallback": r["n_fallback"], "fallback_fraction": r["n_fallback"] / total,
                  "kernel": "k_radic_shared<12,%s>" % ("false" if p == "fp64" else "true"),
                  "kernel_ms": kms,
                  "roofline": {"bound": "alu", "achieved": xf / (kms * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                               "frac": xf / (kms * 1e-3) / 1e12 / peak,
                               "per_unit": f"executed {xf / total:.1f} FLOP per minor ({enum} enumeration)"}}
    out["w4_12x36"] = {"minors": total, "forms": res}

    # 4096 matrices in one HIP-graph launch, every result against the stored values
    batch_list = workloads.batch_matrices()
    mats = [M for _, M in batch_list]
    gold = read_golden("workload5_batch4096.txt")
    batch = radic.Batch(mats, device=dev)
    res = {}
    tuned = {}
    for p in ("fp32_bulk", "fp64"):
        # the persistent kernels' chunk size from the library's autotuner, timed
        # on this batch; the graph is captured with the tuned shape
        tuned[p] = radic.autotune_batched(batch, precision=p)[0]
        gph = radic.BatchGraph(batch, precision=p)
        for _ in range(3):
            gph.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            gph.launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rr = batch.results()
        gph.destroy()
        bad = 0
        tol = 1e-12 if p == "fp64" else 1e-5
        for b, (kind, M) in enumerate(batch_list):
            gr = gold[b]
            if rr[b]["status"] != 0:
                bad += 1
            elif kind == "i32":
                bad += rr[b]["exact"] != int(gr[4])
            else:
                Sg = float(gr[5])
                if Sg <= 1e-9 * exact.hadamard_sum(M):
                    Sg = exact.hadamard_sum(M)
                bad += not abs(rr[b]["value"] - float(gr[4])) <= tol * Sg
        minors = sum(r["n_subsets"] for r in rr)
        res[p] = {"ms_per_launch": ms, "subdet_per_s": minors / (ms * 1e-3), "mismatches_vs_oracle": int(bad),
                  "checked": len(batch_list)}
    out["w5_batch4096"] = {"minors": 342865835, "float_forms": res,
                           "tuned_subsets_per_lane": tuned,
                           "note": "one HIP-graph replay per launch; int32 matrices exact (bit-exact check), "
                                   "float64 matrices in the named precision; chunk sizes (64 x subsets per "
                                   "lane ranks) chosen by radic_autotune_batched on this batch beforehand"}
    return out


def per_minor_roofline(radic, A, outs, work, torch):
    """The per-minor kernels (every minor unranked or advanced and factored on
    its own, Sections 4-6) on the same matrix, on the counted (2/3) m^3 FLOP per
    minor, outside the timed steps."""
    m, n = A.shape
    total = math.comb(n, m)
    radic.set_enumeration("per_minor")
    res = {}
    try:
        for p, peak in (("fp64", PEAK_FP64_TFLOPS), ("fp32_bulk", PEAK_FP32_TFLOPS)):
            call = lambda: radic.radic_det(A, precision=p, out=outs[p], work=work[p], sync=False)   # noqa: E731
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            kms = kernel_ms(radic, call, 10)
            torch.cuda.synchronize()
            flop = counted_flops_per_minor(m) * total
            res[p] = {"kernel": kernel_name("per_minor", p), "bound": "alu", "kernel_ms": kms,
                      "achieved": flop / (kms * 1e-3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                      "frac": flop / (kms * 1e-3) / 1e12 / peak,
                      "per_unit": f"counted (2/3) m^3 = {counted_flops_per_minor(m):.2f} FLOP per minor x {total} "
                                  f"minors (executed {executed_flops(m, n, 'per_minor') / total:.0f})"}
    finally:
        radic.set_enumeration("auto")
    return res


def profiled(form, enumeration, spl):
    """The profiled figures hold for this run: the same kernel sources, the
    prefix-shared enumeration and the same subsets per lane (block size)."""
    return (enumeration in ("auto", "prefix_shared") and spl == PROFILED_TRAFFIC["spl"][form]
            and kernel_sources_sha256() == PROFILED_TRAFFIC["sources_sha256"])


def traffic_for(form, enumeration, spl):
    if not profiled(form, enumeration, spl):
        return None
    return PROFILED_TRAFFIC[form]


def rocprof_flops(form, enumeration, spl, kernel_ms):
    """FLOPs per launch of the prefix-shared kernel from its rocprofv3 counters
    (SQ_INSTS_VALU_FLOPS_FP32/FP64 x 64), over this run's kernel time; None
    once the kernel sources or the launch shape differ from those profiled."""
    if not profiled(form, enumeration, spl):
        return None
    f = PROFILED_FLOPS[form]
    peak = PEAK_FP32_TFLOPS if form == "fp32_bulk" else PEAK_FP64_TFLOPS
    t32 = f["fp32"] / (kernel_ms * 1e-3) / 1e12
    t64 = f["fp64"] / (kernel_ms * 1e-3) / 1e12
    return {"fp32_flop": f["fp32"], "fp64_flop": f["fp64"], "fp32_tflops": t32, "fp64_tflops": t64,
            "frac_of_form_peak": (t32 if form == "fp32_bulk" else t64) / peak,
            "source": "rocprofv3 counters per launch (profiles/k_radic_shared_8x32.md)"}


def valu_issue(form, enumeration, spl, kernel_ms):
    """VALU wave instructions per launch of the prefix-shared kernel from its
    rocprofv3 counter (SQ_INSTS_VALU), over this run's kernel time, against the
    chip's issue rate: the bound these kernels meet, since most of their
    instructions are not floating point; None once the kernel sources or the
    launch shape differ from those profiled."""
    if not profiled(form, enumeration, spl):
        return None
    v = PROFILED_VALU[form]
    rate = v / (kernel_ms * 1e-3)
    return {"valu_instructions": v, "achieved": rate, "peak": PEAK_VALU_ISSUE, "unit": "wave instructions/s",
            "frac": rate / PEAK_VALU_ISSUE,
            "source": "rocprofv3 SQ_INSTS_VALU per launch (profiles/k_radic_shared_8x32.md)"}


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
    ap.add_argument("--no-other", action="store_true",
                    help="skip the other workloads (5x14 latency, exact 6x40 int32, 12x36 precision stress, "
                         "4096-matrix batch) and the per-minor kernels' roofline")
    ap.add_argument("--tune", choices=["table", "live", "none"], default="table",
                    help="launch shapes for the 8x32 shape: the committed table written by the library's "
                         "autotuner (paper_1508_01326_amd/tuned_gfx950.txt, default), radic_autotune in this "
                         "run, or the library's defaults")
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
    # launch shapes for this shape in each precision, chosen by the library's
    # autotuner: from the table it wrote on this architecture (the same shapes
    # in every run, profiler runs included), or timed in this run
    tuned = {}
    if args.tune == "table" and os.path.exists(TUNED_TABLE):
        radic.tune_load(TUNED_TABLE)
        tuned = table_shapes(TUNED_TABLE, m, n, args.enumeration)
    elif args.tune == "live":
        for p in ("fp64", "fp32_bulk"):
            tuned[p] = radic.autotune(radic.RADIC_WS_DET, m, n, p)[0]
    spl_used = {p: tuned.get(p, DEFAULT_SPL_SHARED) for p in ("fp64", "fp32_bulk")}
    shape_source = {p: (args.tune if p in tuned else "default") for p in ("fp64", "fp32_bulk")}
    print(f"[bench] subsets per lane: {spl_used} ({shape_source})", file=sys.stderr, flush=True)

    if args.copy_bytes > 0:
        # a copy kernel that reads and writes copy_bytes each (an element-wise
        # multiply by one: a same-device copy_ may go to a DMA engine, which the
        # kernel counters do not see)
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
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
        dom_times = timed[(0 if dom == "fp64" else 1)::2]
    else:
        dom_times = list(timed)
    dom_ms = sum(dom_times) / max(1, len(dom_times))
    dom_sorted = sorted(dom_times)
    dom_median = dom_sorted[len(dom_sorted) // 2] if dom_sorted else None
    dom_min = dom_sorted[0] if dom_sorted else None

    k64 = launches[0::2]
    k32 = launches[1::2]
    avg64 = sum(k64) / len(k64)
    avg32 = sum(k32) / len(k32)
    call_ms = {"fp64": sum(e[0].elapsed_time(e[1]) for e in form_events) / len(form_events),
               "fp32_bulk": sum(e[1].elapsed_time(e[2]) for e in form_events) / len(form_events)}
    res = {p: binding.read_f64_result(outs[p]) for p in outs}

    # CPU oracle: baseline rate and the reference value for the error figures
    nproc, cpu_model = host_info()
    threads = min(nproc or 1, 16)
    cpu = None
    if not args.no_cpu:
        rate, ref, reps, rate1 = cpu_baseline(A_host, threads)
        cpu = {"value": rate, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"whole workload (all {total} minors, FP64 GEPP + compensated sum), "
                         f"median of {reps} run(s) on {threads} threads; once more on 1 thread",
               "value_1_thread": rate1, "host_nproc": nproc, "host_cpu": cpu_model}
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
            "launch_shape": {"subsets_per_lane": spl_used[p], "source": shape_source[p]},
            "kernel_executed_tflops": xflop / (avg * 1e-3) / 1e12,
            "kernel_counted_tflops": flop / (avg * 1e-3) / 1e12,
            "peak_tflops": peak,
        }
    # roofline of the dominant kernel on the floating-point operations it
    # executes (prefix sharing removes most of the counted (2/3) m^3 per minor:
    # a different method, so the counted figure is reported beside it, labelled)
    achieved = xflop / (dom_ms * 1e-3) / 1e12
    counted = flop / (dom_ms * 1e-3) / 1e12
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
                     "traffic": traffic_for(dom, args.enumeration, spl_used[dom]),
                     "per_unit": f"executed {xflop / total:.2f} FLOP per minor (averaged over the launch; "
                                 f"{args.enumeration} enumeration) x {total} minors = {xflop:.4g} FLOP per launch",
                     "counted_equivalent": {"tflops": counted, "frac": counted / peak,
                                            "per_unit": f"counted (2/3) m^3 = {counted_flops_per_minor(m):.2f} "
                                                        f"FLOP per minor x {total} minors = {flop:.4g} FLOP, "
                                                        f"a different method's work"},
                     "rocprof_flops": rocprof_flops(dom, args.enumeration, spl_used[dom], dom_ms),
                     "valu_issue": valu_issue(dom, args.enumeration, spl_used[dom], dom_ms),
                     "launch_shape": {"subsets_per_lane": spl_used[dom], "source": shape_source[dom]},
                     "kernel_ms": dom_ms, "kernel_ms_median": dom_median, "kernel_ms_min": dom_min,
                     "launches_timed": len(dom_times),
                     "timed_launches": f"the dominant kernel of 1 in {TIME_EVERY} timed steps"},
        "cpu_baseline": cpu,
        "forms": per_form,
    }
    if not args.no_other:
        print("[bench] per-minor kernels", file=sys.stderr, flush=True)
        line["roofline_per_minor"] = per_minor_roofline(radic, A, outs, work, torch)
        print("[bench] other workloads", file=sys.stderr, flush=True)
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
