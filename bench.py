#!/usr/bin/env python3
"""Benchmark of the MI355X MRRR tridiagonal eigensolver (FP64, one GPU).

Step = one pass of the whole solver over the single-tridiagonal workload: the
full spectrum (all eigenvalues and eigenvectors) of three order-20000
tridiagonals -- random U(-1,1) entries (seed 2001), the "1-2-1" Toeplitz matrix,
and a spectrum geometrically spaced in [1e-8, 1] (seed 2003) -- each solved by
its own single-problem call (mrrr_step).  Metric: FP64 eigenpairs per second
(60000 eigenpairs per step), inputs resident in HBM, outputs from the caching
allocator, stream synchronized around the timed region.  Every call is also
timed on its own (each call synchronizes its stream); the median per type is
reported beside the value.

Also reported on the same JSON line:
  roofline      the dominant kernel's achieved rate from HIP events recorded by
                the library on the launch stream over the timed region
                (algorithmic work / event time) against the MI355X peak
  cpu_baseline  the CPU oracle (single thread, pinned to one host core) on a
                bounded sample of the workload, with the host CPU model
  three_in_one_call  the same three problems solved together by one call of the
                batched entry point (launch shapes from its autotuner)
  batched       solves/s of the batched entry point on 4096 mixed problems (sizes
                log-uniform in [32, 2048]) and of a loop of single-problem calls
  backward      the differentiation workload: 256 problems of order 512
                (batched) and one of order 8192, forward and hand-written FP64
                MFMA backward, against a loop of single-problem calls
  backtransform the Stage 5 back-transformation Y = Q Z (FP64 MFMA, compact-WY
                blocks of 64 reflectors) at n = m = 20000, against the FP64
                matrix peak
  reduce        the Stage 3 reduction of a dense symmetric order-20000 matrix
                to tridiagonal form (panels of 64 reflectors), against HBM
                bandwidth for the matrix-vector products that bound it
  fp32          the three order-20000 matrices rounded to FP32 through the FP32
                interface (FP64 inside, relaxed classification threshold),
                against the FP64 calls on the same data
  ghep          the generalized eigenproblem A x = lambda B x of order 20000
                (the paper's dense workload), every stage on the GPU, each
                stage timed
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz
PEAK_FP64_MATRIX_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(n):
    from paper_1205_2107_amd import workloads as W
    return [("random", *W.random_uniform(n, W.SEEDS["c2_random"])),
            ("toeplitz_121", *W.toeplitz(n)),
            ("geometric_1e-8", *W.geometric(n, W.SEEDS["c2_geometric"]))]


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(n):
    """Oracle (single-threaded C, as it stands) on a bounded sample: the 1500
    smallest eigenpairs of the random n = 20000 matrix, the process pinned to
    one host core while it runs."""
    import oracle
    from paper_1205_2107_amd import workloads as W
    d, e = W.random_uniform(n, W.SEEDS["c2_random"])
    k = 1500
    model, logical, usable = host_cpu()
    keep = None
    pinned = None
    try:
        keep = os.sched_getaffinity(0)
        pinned = min(keep)
        os.sched_setaffinity(0, {pinned})
    except (AttributeError, OSError):
        pinned = None
    try:
        t0 = time.perf_counter()
        w, Z, st = oracle.mrrr(d, e, kind=oracle.RANGE_INDEX, il=1, iu=k)
        dt = time.perf_counter() - t0
    finally:
        if keep is not None:
            os.sched_setaffinity(0, keep)
    return {"value": k / dt, "unit": "eigenpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"random n={n} (seed 2001), eigenpairs 1..{k} (il..iu), {dt:.1f} s on 1 host thread",
            "host_cpu": model, "host_logical_cpus": logical, "host_cpus_usable": usable,
            "pinned_core": pinned}


KERNEL_SOURCE = os.path.join(ROOT, "paper_1205_2107_amd", "csrc", "mrrr_kernels.hip")
# kernel symbol per profiled category (the traffic summary under profiles/ is
# named for the symbol and the workload)
KERNEL_SYMBOL = {"grid": "k_grid", "refine": "k_refine", "child": "k_child", "vectors": "k_vectors_stored",
                 "vectors_ckpt": "k_vectors"}


def traffic_summary(kernel):
    return os.path.join(ROOT, "profiles", f"{KERNEL_SYMBOL.get(kernel, kernel)}_traffic_n20000.md")


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    when there is none or the kernel source changed since it was taken."""
    path = traffic_summary(kernel)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k.strip("`")] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_issue(kernel):
    """Issued FP64 fraction, instruction-mix ceiling and VALU occupancy of
    `kernel` from the committed SQ-counter summary (profiles/valu_counters_n20000.md),
    or None when the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "valu_counters_n20000.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k.strip("`")] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    sym = KERNEL_SYMBOL.get(kernel, kernel)
    try:
        return {"issued_frac": float(fields[f"{sym}.issued_frac"]), "mix_ceiling": float(fields[f"{sym}.mix_ceiling"]),
                "valu_busy": float(fields[f"{sym}.valu_busy"])}
    except (KeyError, ValueError):
        return None


def roofline(prof):
    """dominant kernel by event time; ALU-bound kernels against the FP64 vector
    peak, the eigenvector kernels (whose algorithmic bytes are the Z entries
    they write) against HBM bandwidth"""
    name = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[name]
    out = {"kernel": name, "symbol": KERNEL_SYMBOL.get(name, name), "launches": p["launches"],
           "avg_ms": p["ms"] / max(p["launches"], 1), "traffic": measured_traffic(name)}
    if name in ("vectors", "vectors_ckpt"):
        ach = p["bytes"] / (p["ms"] * 1e-3) / 1e9
        out.update({"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS})
    else:
        ach = p["work"] / (p["ms"] * 1e-3) / 1e12
        out.update({"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                    "frac": ach / PEAK_FP64_VECTOR_TFLOPS})
    # the issued measure beside the algorithmic one: FP64 VALU flops from SQ
    # counters, the ceiling the instruction mix sets, the SIMD share issuing VALU
    out["issue"] = measured_issue(name)
    return out


def batched_leg(torch, M, count, loop_count, mark=False):
    from paper_1205_2107_amd import workloads as W
    flag = torch.empty(1, dtype=torch.uint8, device="cuda")
    probs = W.batched_mix(count, W.SEEDS["c4"])
    d, e, ns, off = W.pack(probs)
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e, device="cuda")
    # launch shapes for this size mix (untimed: a coordinate search over about
    # ten solves; the choice is cached for batches with the same size histogram)
    tuning = M.autotune_batched(dt, et, ns)
    M.eigh_tridiagonal_batched(dt, et, ns)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    if mark:
        flag.fill_(1)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        M.eigh_tridiagonal_batched(dt, et, ns)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    if mark:
        flag.fill_(2)
        torch.cuda.synchronize()
    # loop of single-problem calls over the first loop_count problems of the same mix
    singles = [(torch.tensor(p[0], device="cuda"), torch.tensor(p[1], device="cuda")) for p in probs[:loop_count]]
    for a, b in singles[:8]:
        M.eigh_tridiagonal(a, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in singles:
        M.eigh_tridiagonal(a, b)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    return {"problems": count, "sum_n": int(ns.sum()), "seconds": tb, "solves_per_s": count / tb, "tuning": tuning,
            "looped_problems": loop_count, "looped_solves_per_s": loop_count / tl,
            "speedup_vs_looped": (count / tb) / (loop_count / tl)}


def median(xs):
    xs = sorted(xs)
    k = len(xs)
    return 0.5 * (xs[(k - 1) // 2] + xs[k // 2]) if k else 0.0


def backward_leg(torch, M, reps=5, loop_count=64):
    """Differentiation workload: 256 problems of order 512 (separated spectra)
    through the batched forward and the batched FP64-MFMA backward, one problem
    of order 8192; a loop of single-problem forward + backward calls over the
    first loop_count problems of the batch as the looped baseline.  The
    backward work is 4 n^3 flops per problem (two n x n x n products)."""
    from paper_1205_2107_amd import workloads as W
    out = {}
    nb, count = 512, 256
    probs = [W.separated(nb, W.SEEDS["c5"] + k) for k in range(count)]
    d, e, ns, off = W.pack(probs)
    dt = torch.tensor(d, device="cuda")
    et = torch.tensor(e, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(W.SEEDS["c5"])
    gw = torch.randn(count * nb, generator=g, dtype=torch.float64).cuda()
    gZ = torch.randn(count * nb * nb, generator=g, dtype=torch.float64).cuda()
    wb, Zb, zoff = M.eigh_tridiagonal_batched(dt, et, ns)
    M.eigh_tridiagonal_backward_batched(wb, Zb, ns, gw, gZ)
    torch.cuda.synchronize()
    tf, tbw = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        wb, Zb, zoff = M.eigh_tridiagonal_batched(dt, et, ns)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        M.eigh_tridiagonal_backward_batched(wb, Zb, ns, gw, gZ)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        tbw.append(t2 - t1)
    flops = 4.0 * nb ** 3 * count
    out["batched_256x512"] = {"forward_s": median(tf), "backward_s": median(tbw),
                              "backward_tflops": flops / median(tbw) / 1e12,
                              "backward_frac_of_fp64_mfma_peak": flops / median(tbw) / 1e12 / PEAK_FP64_MATRIX_TFLOPS,
                              "solves_per_s": count / (median(tf) + median(tbw))}
    # looped: single forward + single backward per problem
    singles = []
    for k in range(loop_count):
        singles.append((torch.tensor(probs[k][0], device="cuda"), torch.tensor(probs[k][1], device="cuda"),
                        gw[k * nb:(k + 1) * nb], gZ[k * nb * nb:(k + 1) * nb * nb].reshape(nb, nb).t()))
    for a, b, c, G in singles[:4]:
        w1, Z1 = M.eigh_tridiagonal(a, b)
        M.eigh_tridiagonal_backward(w1, Z1, c, G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b, c, G in singles:
        w1, Z1 = M.eigh_tridiagonal(a, b)
        M.eigh_tridiagonal_backward(w1, Z1, c, G)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    out["batched_256x512"]["looped_solves_per_s"] = loop_count / tl
    out["batched_256x512"]["speedup_vs_looped"] = out["batched_256x512"]["solves_per_s"] / (loop_count / tl)
    # one problem of order 8192
    n8 = 8192
    d8, e8 = W.separated(n8, W.SEEDS["c5"])
    d8t, e8t = torch.tensor(d8, device="cuda"), torch.tensor(e8, device="cuda")
    gw8 = torch.randn(n8, generator=g, dtype=torch.float64).cuda()
    gZ8 = torch.randn(n8, n8, generator=g, dtype=torch.float64).cuda()
    w8, Z8 = M.eigh_tridiagonal(d8t, e8t)
    M.eigh_tridiagonal_backward(w8, Z8, gw8, gZ8)
    torch.cuda.synchronize()
    tf8, tb8 = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        w8, Z8 = M.eigh_tridiagonal(d8t, e8t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        M.eigh_tridiagonal_backward(w8, Z8, gw8, gZ8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf8.append(t1 - t0)
        tb8.append(t2 - t1)
    f8 = 4.0 * n8 ** 3
    out["single_8192"] = {"forward_s": median(tf8), "backward_s": median(tb8),
                          "backward_tflops": f8 / median(tb8) / 1e12,
                          "backward_frac_of_fp64_mfma_peak": f8 / median(tb8) / 1e12 / PEAK_FP64_MATRIX_TFLOPS}
    return out


def backtransform_leg(torch, M, n, reps=3):
    """Stage 5 back-transformation Y = Q Z at n = m (the eigenvectors of one
    order-n problem): synthetic reflectors of a lower tridiagonal reduction
    (seeded; the reduction itself is not built), Z normal random, resident on
    the device.  Algorithmic work 2 n^2 m flops (reflector application)."""
    from paper_1205_2107_amd import workloads as W
    V, tau = W.reflectors(n, W.SEEDS["c2_random"])
    Vd = torch.tensor(V.T, device="cuda").t()  # column-major on the device
    del V
    g = torch.Generator(device="cpu").manual_seed(W.SEEDS["c2_random"])
    Z = torch.randn((n, n), generator=g, dtype=torch.float64).cuda().t()
    M.backtransform(Vd, tau, Z)  # warm-up (in place; the values stay finite and orthogonally transformed)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        M.backtransform(Vd, tau, Z)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t = median(ts)
    flops = 2.0 * n * n * n
    return {"n": n, "m": n, "seconds": t, "tflops": flops / t / 1e12,
            "frac_of_fp64_mfma_peak": flops / t / 1e12 / PEAK_FP64_MATRIX_TFLOPS, "reps": reps}


def reduce_leg(torch, M, n, reps=2):
    """Stage 3 reduction T = Q^T M Q of a dense symmetric order-n matrix
    (lower triangle U(-1, 1), seeded, drawn on the device).  Each call
    overwrites its input, so every repetition reduces a fresh device copy made
    outside the timed region.  Work 4 n^3 / 3 flops; HBM bytes of the
    matrix-vector products (one read of the trailing lower triangle per
    reflector, sum over m = 1 .. n-1 of 8 m (m + 1) / 2) bound it."""
    from paper_1205_2107_amd import workloads as W
    lower, full = W.dense_symmetric_device(n, W.SEEDS["c2_random"], "cuda")
    del full
    work = torch.empty_like(lower)
    ts = []
    prof = []
    for r in range(reps + 1):
        work.copy_(lower)
        torch.cuda.synchronize()
        if r > 0:
            M.profile(True)
        t0 = time.perf_counter()
        M.tridiagonalize(work)
        torch.cuda.synchronize()
        if r > 0:
            ts.append(time.perf_counter() - t0)
            prof.append(M.profile_read()["tridiag"])
            M.profile(False)
    del work, lower
    t = median(ts)
    nn = float(n)
    flops = 4.0 / 3.0 * nn ** 3
    symv_bytes = 8.0 * (nn - 1.0) * nn * (nn + 1.0) / 6.0
    return {"n": n, "seconds": t, "gflops": flops / t / 1e9,
            "symv_bytes": symv_bytes, "symv_gbs_over_call": symv_bytes / t / 1e9,
            "frac_of_hbm_peak_over_call": symv_bytes / t / 1e9 / PEAK_HBM_GBS,
            "launches": prof[-1]["launches"] if prof else None, "reps": reps}


def fp32_leg(torch, M, n, reps=3):
    """The bench matrices rounded to FP32 (so both interfaces solve the same
    tridiagonal): median call time of mrrr_step_f32 and of mrrr_step on the
    widened data, and the representation-tree sizes of both."""
    import numpy as np
    from paper_1205_2107_amd import workloads as W
    out = {}
    for kind, (d, e) in (("random", W.random_uniform(n, W.SEEDS["c2_random"])), ("toeplitz_121", W.toeplitz(n)),
                         ("geometric_1e-8", W.geometric(n, W.SEEDS["c2_geometric"]))):
        d32 = torch.tensor(np.asarray(d, dtype=np.float32), device="cuda")
        e32 = torch.tensor(np.asarray(e, dtype=np.float32), device="cuda")
        d64, e64 = d32.double(), e32.double()
        row = {}
        for name, call in (("fp32", lambda: M.eigh_tridiagonal_f32(d32, e32, return_info=True)),
                           ("fp64", lambda: M.eigh_tridiagonal(d64, e64, return_info=True))):
            w, Z, info = call()
            del w, Z
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                w, Z, info = call()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                del w, Z
            row[name + "_ms"] = median(ts) * 1e3
            row[name + "_nodes"] = info["nodes"]
        out[kind] = row
        torch.cuda.empty_cache()
    return out


def ghep_leg(torch, M, n):
    """A x = lambda B x of order n, all eigenpairs: A symmetric (lower
    triangle U(-1, 1)), B = G G^T / n + I, both seeded and drawn on the device.
    Each of the six stages is timed on its own (stream synchronized around
    it); the total is their sum.  Work of the dense stages: Cholesky n^3/3,
    reduction to standard form 2 n^3 (two triangular solves with n right-hand
    sides), tridiagonal reduction 4 n^3/3, first back-transformation 2 n^3,
    second back-transformation n^3 flops."""
    from paper_1205_2107_amd import workloads as W
    lower, full = W.dense_symmetric_device(n, W.SEEDS["c2_random"], "cuda")
    del full
    B = W.dense_spd_device(n, W.SEEDS["c2_random"] + 1, "cuda")
    torch.cuda.empty_cache()
    t = {}

    def timed(name, f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        t[name] = time.perf_counter() - t0
        return r

    L = timed("cholesky", lambda: M.cholesky(B))
    Ms = timed("standard_form", lambda: M.sygst(lower, L))
    d, e, tau, V = timed("tridiagonal_reduction", lambda: M.tridiagonalize(Ms))
    w, Z = timed("tridiagonal_eigensolver", lambda: M.eigh_tridiagonal(d, e))
    Y = timed("back_transformation_q", lambda: M.backtransform(V, tau, Z))
    X = timed("back_transformation_l", lambda: M.trsm_lt(L, Y))
    ok = bool(torch.isfinite(w).all()) and bool(torch.isfinite(X[:, :4]).all())
    nn = float(n)
    flops = {"cholesky": nn ** 3 / 3.0, "standard_form": 2.0 * nn ** 3, "tridiagonal_reduction": 4.0 * nn ** 3 / 3.0,
             "back_transformation_q": 2.0 * nn ** 3, "back_transformation_l": nn ** 3}
    del lower, B, L, Ms, V, Z, Y, X
    total = sum(t.values())
    return {"n": n, "seconds_total": total, "seconds": t, "eigenpairs_per_s": n / total,
            "tflops": {k: flops[k] / t[k] / 1e12 for k in flops}, "finite": ok}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-backtransform", action="store_true")
    ap.add_argument("--no-reduce", action="store_true")
    ap.add_argument("--no-ghep", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--only-fp32", action="store_true", help="only the FP32-interface leg; prints its JSON")
    ap.add_argument("--only-ghep", action="store_true",
                    help="only the generalized-problem leg (for a profiler run); prints its JSON")
    ap.add_argument("--only-reduce", action="store_true",
                    help="only the reduction leg (for a profiler run); prints its JSON")
    ap.add_argument("--only-backtransform", action="store_true",
                    help="only the back-transformation leg (for a profiler run); prints its JSON")
    ap.add_argument("--only-batched", action="store_true",
                    help="only the batched leg, its timed calls between two one-byte fill kernels "
                         "that mark them in a kernel trace; prints its JSON")
    ap.add_argument("--batched-count", type=int, default=4096)
    ap.add_argument("--looped-count", type=int, default=512)
    ap.add_argument("--profile-once", action="store_true",
                    help="the step twice after one warm-up step (for a profiler run); no JSON")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="copy BYTES between two device buffers (counter calibration); no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1205_2107_amd as M
    if not torch.cuda.is_available():
        print("bench.py: no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    n = args.n
    if args.only_fp32:
        log("[bench] FP32-interface leg only")
        print(json.dumps({"fp32": fp32_leg(torch, M, n)}), flush=True)
        return
    if args.only_ghep:
        log("[bench] generalized-problem leg only")
        print(json.dumps({"ghep": ghep_leg(torch, M, n)}), flush=True)
        return
    if args.only_reduce:
        log("[bench] reduction leg only")
        print(json.dumps({"reduce": reduce_leg(torch, M, n)}), flush=True)
        return
    if args.only_backtransform:
        log("[bench] back-transformation leg only")
        print(json.dumps({"backtransform": backtransform_leg(torch, M, n)}), flush=True)
        return
    if args.only_batched:
        log("[bench] batched leg only")
        print(json.dumps({"batched": batched_leg(torch, M, args.batched_count, args.looped_count, mark=True)}),
              flush=True)
        return
    if args.copy_calib:
        src = torch.ones(args.copy_calib // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {src.numel() * 8} bytes")
        return
    from paper_1205_2107_amd import workloads as W
    log(f"[bench] generating inputs n={n}")
    inputs = make_inputs(n)
    names = [name for name, _, _ in inputs]
    dev = [(torch.tensor(d, device="cuda"), torch.tensor(e, device="cuda")) for _, d, e in inputs]
    torch.cuda.synchronize()

    def step(times=None):
        infos = []
        for k, (dd, ee) in enumerate(dev):
            t0 = time.perf_counter()
            w, Z, info = M.eigh_tridiagonal(dd, ee, return_info=True)  # synchronizes its stream
            if times is not None:
                times[k].append((time.perf_counter() - t0) * 1e3)
            infos.append(info)
            del w, Z
        return infos

    if args.profile_once:
        step()
        torch.cuda.synchronize()
        step()
        step()
        torch.cuda.synchronize()
        log("[bench] profiled the step twice (after one warm-up step)")
        return
    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    M.profile(True)
    times = [[] for _ in dev]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        infos = step(times)
        log(f"[bench] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = M.profile_read()
    M.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    pairs_per_step = n * len(dev)
    value = pairs_per_step / (ms_per_step * 1e-3)
    per_type = {name: median(times[k]) for k, name in enumerate(names)}
    out = {
        "metric": "FP64 eigenpairs/s at n=20k full spectrum (random, 1-2-1, geometric types)",
        "value": value,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"STEP full spectrum, three single tridiagonals of order {n} per step "
                               "(one mrrr_step call each)",
                   "n": n, "types": names,
                   "median_call_ms_per_type": per_type,
                   "calls_per_type": args.steps,
                   "tree": {name: {"levels": infos[k]["levels"], "nodes": infos[k]["nodes"],
                                   "max_depth": infos[k]["max_depth"]} for k, name in enumerate(names)}},
        "roofline": roofline(prof),
        "kernels": {k: {"ms_per_step": v["ms"] / args.steps, "launches": v["launches"],
                        "tflops": (v["work"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else 0.0}
                    for k, v in prof.items()},
    }
    # the same three problems in one batched call
    log("[bench] three problems in one batched call")
    d_all, e_all, ns, _ = W.pack([(d, e) for _, d, e in inputs])
    d_dev = torch.tensor(d_all, device="cuda")
    e_dev = torch.tensor(e_all, device="cuda")
    tuning = M.autotune_batched(d_dev, e_dev, ns)
    tb = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.eigh_tridiagonal_batched(d_dev, e_dev, ns)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    out["three_in_one_call"] = {"ms": median(tb) * 1e3, "eigenpairs_per_s": pairs_per_step / median(tb),
                                "tuning": tuning}
    del d_dev, e_dev
    torch.cuda.empty_cache()
    if not args.no_batched:
        log("[bench] batched leg")
        out["batched"] = batched_leg(torch, M, args.batched_count, args.looped_count)
        torch.cuda.empty_cache()
    if not args.no_backward:
        log("[bench] backward leg")
        out["backward"] = backward_leg(torch, M)
        torch.cuda.empty_cache()
    if not args.no_backtransform:
        log("[bench] back-transformation leg")
        out["backtransform"] = backtransform_leg(torch, M, n)
        torch.cuda.empty_cache()
    if not args.no_reduce:
        log("[bench] reduction leg")
        out["reduce"] = reduce_leg(torch, M, n)
        torch.cuda.empty_cache()
    if not args.no_fp32:
        log("[bench] FP32-interface leg")
        out["fp32"] = fp32_leg(torch, M, n)
        torch.cuda.empty_cache()
    if not args.no_ghep:
        log("[bench] generalized-problem leg")
        out["ghep"] = ghep_leg(torch, M, n)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
