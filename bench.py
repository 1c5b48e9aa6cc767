"""Benchmark: effective TFLOP/s (2mnk/t) of Strassen-fused GEMM at one and two
levels against the plain MFMA GEMM of the same kernels (levels = 0), fp32,
m = n = k = 16384, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--levels L]

A step is one strassen_gemm call (C := A*B + C) on device-resident seeded
inputs (A, B, C ~ U[-1, 1]).  Every level 0, 1, 2 is timed: W untimed calls,
then K calls between two synchronisations and device events.  `value` is the
effective rate of the headline level (--levels, default 1); all three levels
are reported under "levels".  The roofline object describes the dominant
kernel of the headline level, timed per launch with HIP events recorded by
the library itself on the launch stream.  The CPU oracle is timed on a
bounded sample of rows of the same product (cpu_baseline); it is used
nowhere else here: the sampled error checks compare against fp64 dot
products computed in this script.  Secondary sections: the compensated
bf16x3 mode at 8192^3 and 16384^3 (plain as stored and on pre-split copies,
fused and formed one- and two-level products timed in interleaved rounds,
the Strassen speedups taken against the faster plain product), bf16 / fp16 / bf16x3 at
4096-16384 (N(0,1) and rows/columns scaled over six decades), the fp32
square and rank-k sweep and the awkward padded shapes, differentiation, and
small sizes by schedule.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_MFMA_PEAK = 157.3  # TFLOP/s, MI355X dense fp32 matrix peak
BF16_MFMA_PEAK = 2516.6  # TFLOP/s, MI355X dense bf16/fp16 matrix peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--levels", type=int, default=1, choices=[0, 1, 2])
    p.add_argument("--size", type=int, default=16384)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-precision", action="store_true",
                   help="skip the bf16 / fp16 / bf16x3 section")
    p.add_argument("--no-autograd", action="store_true",
                   help="skip the forward + backward section")
    p.add_argument("--no-sweep", action="store_true",
                   help="skip the fp32 square / rank-k sweep and the awkward shapes (their "
                        "rank-k launches share kernel and grid with the headline's, so per-kernel "
                        "profiles of the headline are taken without them)")
    p.add_argument("--no-compensated", action="store_true",
                   help="skip the bf16x3 plain / fused / formed comparison")
    p.add_argument("--no-small", action="store_true",
                   help="skip the small-size schedule section")
    p.add_argument("--mfma-probe", action="store_true",
                   help="only measure the matrix cores' attainable rate (register-operand MFMA loops, "
                        "bf16 / fp16 / fp32, constant and random operands) and print one JSON line")
    p.add_argument("--launch-table", metavar="PATH",
                   help="only time every launch of squares m=n=k in 1024..16384 at levels 0/1/2 "
                        "(fp32, bf16, bf16x3; plus the formed one-level calls) with library "
                        "events and write them to PATH as JSON (for the performance model)")
    return p.parse_args()


def host_cpu():
    """Model name and core / thread counts of the host CPU."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = set()
    try:
        with open("/proc/cpuinfo") as f:
            phys = core = None
            for ln in f:
                if ln.startswith("physical id"):
                    phys = ln.split(":", 1)[1].strip()
                elif ln.startswith("core id"):
                    core = ln.split(":", 1)[1].strip()
                    cores.add((phys, core))
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "physical_cores": len(cores) or None,
            "affinity_threads": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _omp_set_threads(n):
    """Sets the OpenMP thread count of the oracle library (libgomp, shared
    with this process) and returns the previous count."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    prev = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return prev


def cpu_baseline(A, B, C, target_s):
    """The oracle on the GPU host's cores: its classical fp64 GEMM on the
    first rows of the headline product (about target_s seconds; the `value`),
    and, on bounded samples (leading rows, about a second each), the other
    workload shapes: the small square, the square and rank-k sweep, the
    awkward shapes; its fp64 Strassen recursion at one and two levels; and
    the classical GEMM on one core.  Rates in TFLOP/s = 2 * rows * n * k / t."""
    import numpy as np
    import oracle

    lib = oracle._load()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))

    def classical(Ad, Bd, rows):
        m, k = Ad.shape
        n = Bd.shape[1]
        Cd = np.zeros((rows, n))
        t0 = time.perf_counter()
        lib.oracle_gemm_f64(rows, n, k, oracle._ptr(Ad), k, oracle._ptr(Bd), n, oracle._ptr(Cd), n,
                            1.0, 0.0)
        return time.perf_counter() - t0

    def bounded(Ad, Bd, seconds, align):
        """Times the first rows of Ad @ Bd, rows sized for `seconds`."""
        m = Ad.shape[0]
        probe = min(m, max(align, 4))
        t = classical(Ad, Bd, probe)
        rows = int(min(m, max(probe, probe * seconds / max(t, 1e-6))))
        rows = min(m, max(align, (rows // align) * align))
        t = classical(Ad, Bd, rows)
        return rows, t

    n, k = B.shape[1], A.shape[1]
    Bd = oracle._f64(B)
    # headline: the first rows of the 16384^3 product
    rows, t = bounded(oracle._f64(A), Bd, target_s, threads)
    main = {"value": 2.0 * rows * n * k / t / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "classical fp64 oracle_gemm_f64 on the first %d of %d rows of C = A*B "
                      "(n = k = %d), %.1f s" % (rows, A.shape[0], n, t)}
    samples = []
    rng = np.random.default_rng(7)

    def shape_sample(name, m_, n_, k_, seconds=1.0):
        Ad_ = rng.random((min(m_, 4096), k_)) * 2 - 1
        Bd_ = Bd[:k_, :n_] if (k_ <= Bd.shape[0] and n_ <= Bd.shape[1]) else rng.random((k_, n_)) * 2 - 1
        Bd_ = np.ascontiguousarray(Bd_)
        r, tt = bounded(Ad_, Bd_, seconds, threads)
        samples.append({"workload": name, "m": m_, "n": n_, "k": k_, "rows_timed": r, "seconds": round(tt, 3),
                        "tflops": round(2.0 * r * n_ * k_ / tt / 1e12, 4), "kind": "classical fp64"})

    shape_sample("small square", 1024, 1024, 1024)
    for N in (2048, 4096, 8192, 12288):
        shape_sample("square sweep", N, N, N)
    for kk in (512, 1024, 2048, 4096):
        shape_sample("rank-k sweep", 16384, 16384, kk, 0.5)
    shape_sample("awkward", 15001, 17003, 9007)
    shape_sample("awkward", 3000, 20000, 5000)
    # the fp64 Strassen recursion (explicit zero-padded quadrant copies) on
    # the small square
    for N in (1024,):
        A2 = rng.random((N, N)) * 2 - 1
        B2 = rng.random((N, N)) * 2 - 1
        for L in (0, 1, 2):
            C2 = np.zeros((N, N))
            t0 = time.perf_counter()
            rc = lib.oracle_strassen(N, N, N, oracle._ptr(A2), N, oracle._ptr(B2), N, oracle._ptr(C2), N,
                                     1.0, 0.0, L, 0)
            tt = time.perf_counter() - t0
            if rc:
                raise SystemExit("oracle_strassen failed (%d)" % rc)
            samples.append({"workload": "square, oracle_strassen fp64", "m": N, "n": N, "k": N,
                            "levels": L, "seconds": round(tt, 3),
                            "tflops": round(2.0 * N ** 3 / tt / 1e12, 4), "kind": "strassen fp64"})
    # one core
    try:
        prev = _omp_set_threads(1)
    except OSError:
        prev = None
    if prev is not None:
        A2 = rng.random((2048, 2048)) * 2 - 1
        B2 = rng.random((2048, 2048)) * 2 - 1
        r, tt = bounded(A2, B2, 2.0, 1)
        _omp_set_threads(prev)
        samples.append({"workload": "square, one core", "m": 2048, "n": 2048, "k": 2048, "rows_timed": r,
                        "seconds": round(tt, 3), "tflops": round(2.0 * r * 2048 * 2048 / tt / 1e12, 5),
                        "kind": "classical fp64", "threads": 1})
    main["host"] = host_cpu()
    main["samples"] = samples
    return main


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "strassen_f32_16384_traffic.md")


def kernel_source_text(path):
    """The code of a C++ source without comments or whitespace: the part of
    a kernel source that can change the kernel."""
    import re
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "".join(src.split())


def measured_traffic(kernel, workgroups):
    """HBM bytes per launch of `kernel` launched with `workgroups` workgroups,
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when
    there is no row for it or the kernel sources changed since the counters
    were taken (the summary records a sha256 of those sources)."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"kernel-source-sha256: ([0-9a-f]{64}) \(sha256 over (.*?), concatenated, "
                  r"comments and whitespace removed\)", text)
    if not m:
        return None
    h = hashlib.sha256()
    for f in m.group(2).split(", "):
        try:
            h.update(kernel_source_text(os.path.join(ROOT, f)).encode())
        except OSError:
            return None
    if h.hexdigest() != m.group(1):
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 8 and cells[0] == "`%s`" % kernel and cells[1] == str(workgroups):
            return float(cells[7])
    return None


def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def sampled_reference(A, B, C, rows, cols, alpha, beta):
    """fp64 alpha * sum_l A[i,l] B[l,j] + beta * C[i,j] at the sampled (i, j),
    one dot product per entry on the host, and the componentwise scale
    |alpha| sum_l |A[i,l] B[l,j]| + |beta C[i,j]| of each entry.  A, B, C are
    host or device tensors (only the sampled rows and columns are copied)."""
    import torch
    ri = torch.as_tensor(rows, device=A.device)
    ci = torch.as_tensor(cols, device=B.device)
    a = A[ri].double().cpu()
    b = B[:, ci].double().cpu().t()
    prod = a * b
    val = alpha * prod.sum(dim=1)
    mag = abs(alpha) * prod.abs().sum(dim=1)
    if beta != 0.0:
        c = C[torch.as_tensor(rows, device=C.device), torch.as_tensor(cols, device=C.device)]
        c = c.double().cpu()
        val = val + beta * c
        mag = mag + abs(beta) * c.abs()
    return val.numpy(), mag.numpy()


def sampled_got(C, rows, cols):
    import torch
    return C[torch.as_tensor(rows, device=C.device),
             torch.as_tensor(cols, device=C.device)].double().cpu().numpy()


def precision_section(sizes, steps, dev, stream, log):
    """bf16 and fp16 operands and the compensated bf16x3 mode at m=n=k in
    `sizes`, beta = 0.  N(0,1) inputs: effective TFLOP/s per level and the
    sampled errors.  Scaled inputs (rows of A and columns of B with 2-norms
    spread over 1e-3..1e3): sampled errors only.  Errors against fp64 dot
    products on the stored (rounded) operands, on 256 sampled entries:
    e_norm (max |err| / (eps k max|A| max|B|)), relative Frobenius error of
    the sample, and the componentwise maximum |err| / (eps sum_l |A_il B_lj|).
    The inputs of the smaller sizes are the leading blocks of the largest."""
    import numpy as np
    import torch
    import paper_1808_07984_amd as sg
    from paper_1808_07984_amd import inputs

    Nmax = max(sizes)
    gens = {"normal": (inputs.normal(Nmax, Nmax, inputs.SEED_A), inputs.normal(Nmax, Nmax, inputs.SEED_B)),
            "scaled": (inputs.scaled(Nmax, Nmax, inputs.SEED_A, axis=0),
                       inputs.scaled(Nmax, Nmax, inputs.SEED_B, axis=1))}
    out = {}
    for name, tdt, mode, eps_gate in (("bf16", torch.bfloat16, "plain", 2.0 ** -7),
                                      ("f16", torch.float16, "plain", 2.0 ** -10),
                                      ("bf16x3", torch.float32, "bf16x3", 2.0 ** -16)):
        res = {}
        for N in sizes:
            rng = np.random.default_rng(N)
            rows, cols = rng.integers(0, N, 256), rng.integers(0, N, 256)
            for dist in ("normal", "scaled"):
                Ah = gens[dist][0][:N, :N].contiguous().to(tdt)
                Bh = gens[dist][1][:N, :N].contiguous().to(tdt)
                want, mag = sampled_reference(Ah, Bh, None, rows, cols, 1.0, 0.0)
                scale = N * float(Ah.float().abs().max()) * float(Bh.float().abs().max())
                A, B = Ah.to(dev), Bh.to(dev)
                C = torch.zeros(N, N, device=dev)
                ws = torch.empty(max(sg.api.formed_workspace_bytes(N, N, N, tdt, mode, lv_) for lv_ in (1, 2)),
                                 dtype=torch.uint8, device=dev)
                for L in (0, 1, "1_formed", 2, "2_formed"):
                    if L in ("1_formed", "2_formed"):
                        lv = int(L[0])
                        call = (lambda lv=lv: sg.gemm_formed(A, B, C, 1.0, 0.0, mode=mode, workspace=ws,
                                                             levels=lv))
                    else:
                        call = (lambda L=L: sg.gemm(A, B, C, 1.0, 0.0, levels=L, mode=mode))
                        lv = L
                    call()
                    torch.cuda.synchronize()
                    err = np.abs(sampled_got(C, rows, cols) - want)
                    row = {"e_norm_gate": round(float(err.max()) / (eps_gate * scale), 5),
                           "rel_frobenius": float(np.sqrt((err ** 2).sum() / (want ** 2).sum())),
                           "componentwise_gate": round(float((err / (eps_gate * mag)).max()), 4),
                           "gate_eps": eps_gate, "tolerance": 2.0 ** (lv + 1)}
                    if mode == "bf16x3":
                        # the same error in units of fp32's eps (reported, not gated)
                        row["e_norm_2m23"] = round(float(err.max()) / (2.0 ** -23 * scale), 4)
                        row["componentwise_2m23"] = round(float((err / (2.0 ** -23 * mag)).max()), 3)
                    if dist == "normal":
                        ms = time_calls(call, steps, 1, stream)
                        info = sg.plan_info(N, N, N, lv, tdt, mode)
                        mult = 3.0 if mode == "bf16x3" else 1.0
                        exe = mult * info.executed_flops / (ms * 1e-3) / 1e12
                        row.update({"ms_per_step": round(ms, 4),
                                    "effective_tflops": round(2.0 * N ** 3 / (ms * 1e-3) / 1e12, 2),
                                    "executed_mfma_tflops": round(exe, 2),
                                    "mfma_frac_executed": round(exe / BF16_MFMA_PEAK, 4)})
                        log("%s N=%d L%s: %.3f ms  effective %.1f TFLOP/s  e_norm %.4f%s  rel_F %.2e"
                            % (name, N, L, ms, row["effective_tflops"], row["e_norm_gate"],
                               (" (%.3f at 2^-23)" % row["e_norm_2m23"]) if "e_norm_2m23" in row else "",
                               row["rel_frobenius"]))
                    else:
                        log("%s N=%d L%s scaled: e_norm %.4f  rel_F %.2e  componentwise %.3f"
                            % (name, N, L, row["e_norm_gate"], row["rel_frobenius"],
                               row["componentwise_gate"]))
                    res.setdefault(str(N), {}).setdefault(dist, {})["L%s" % L] = row
                del A, B, C, ws
                torch.cuda.empty_cache()
        out[name] = res
    return out


def compensated_section(sizes, steps, rounds, dev, stream, log):
    """The compensated bf16x3 mode on fp32 N(0,1) operands, C := A*B (the
    precision workload) at m=n=k in `sizes`: the plain product (as stored,
    and on pre-split copies of A and B: the formed call at level 0, the
    operand path of the formed products), the fused
    one-level call, the formed one-level call (two-term sums formed into
    workspace first, bit-identical to the fused one) and the fused and formed
    two-level calls; the Strassen calls' speedups are against the faster of
    the two plain products.  Timed in `rounds` interleaved rounds of `steps` calls each (the
    16-bit matrix cores run power-limited, so the variants are timed in
    turn under the same conditions); the median round of each is reported.
    Also: the formed call's form and product launch times (library events),
    its equality with the fused call on the blocks the chained products do
    not touch, and sampled errors at 2^-16 (the gate) and 2^-23 (fp32's
    eps)."""
    import numpy as np
    import torch
    import paper_1808_07984_amd as sg
    from paper_1808_07984_amd import inputs

    out = {}
    for N in sizes:
        A = inputs.normal(N, N, inputs.SEED_A).to(dev)
        B = inputs.normal(N, N, inputs.SEED_B).to(dev)
        C = torch.zeros(N, N, device=dev)
        ws = torch.empty(max(sg.api.formed_workspace_bytes(N, N, N, torch.float32, "bf16x3", lv) for lv in (0, 1, 2)),
                         dtype=torch.uint8, device=dev)
        variants = {
            "L0": lambda: sg.gemm(A, B, C, 1.0, 0.0, levels=0, mode="bf16x3"),
            "L0_formed": lambda: sg.gemm_formed(A, B, C, 1.0, 0.0, mode="bf16x3", workspace=ws, levels=0),
            "L1_fused": lambda: sg.gemm(A, B, C, 1.0, 0.0, levels=1, mode="bf16x3"),
            "L1_formed": lambda: sg.gemm_formed(A, B, C, 1.0, 0.0, mode="bf16x3", workspace=ws),
            "L2_fused": lambda: sg.gemm(A, B, C, 1.0, 0.0, levels=2, mode="bf16x3"),
            "L2_formed": lambda: sg.gemm_formed(A, B, C, 1.0, 0.0, mode="bf16x3", workspace=ws, levels=2),
        }
        # correctness first: formed == fused, sampled errors vs fp64
        rng = np.random.default_rng(N + 1)
        rows, cols = rng.integers(0, N, 256), rng.integers(0, N, 256)
        want, _ = sampled_reference(A, B, None, rows, cols, 1.0, 0.0)
        scale = N * float(A.abs().max()) * float(B.abs().max())
        errs = {}
        ref0 = ref1 = ref2 = None
        for name, fn in variants.items():
            fn()
            torch.cuda.synchronize()
            err = float(np.abs(sampled_got(C, rows, cols) - want).max())
            errs[name] = {"e_norm_2m16": round(err / (2.0 ** -16 * scale), 5),
                          "e_norm_2m23": round(err / (2.0 ** -23 * scale), 4)}
            if name == "L0":
                ref0 = C.clone()
            if name == "L0_formed" and not torch.equal(C, ref0):
                raise SystemExit("pre-split plain result differs from the plain one at N=%d" % N)
            if name == "L1_fused":
                ref1 = C.clone()
            if name == "L2_fused":
                ref2 = C.clone()
            if name == "L2_formed" and not torch.equal(C, ref2):
                raise SystemExit("formed two-level result differs from the fused one at N=%d" % N)
            if name == "L1_formed":
                # C1 and C2 equal the fused call bit for bit; C0 and C3 take the
                # chained products (added together with their partners)
                h = N // 2
                if not (torch.equal(C[:h, h:], ref1[:h, h:]) and torch.equal(C[h:, :h], ref1[h:, :h])
                        and errs[name]["e_norm_2m16"] <= 4.0):
                    raise SystemExit("formed one-level result check failed at N=%d" % N)
        del ref0, ref1, ref2
        times = {name: [] for name in variants}
        for _ in range(rounds):
            for name, fn in variants.items():
                times[name].append(time_calls(fn, steps, 1, stream))
        # the formed call's launches
        sg.strassen_profile_start()
        variants["L1_formed"]()
        rc, recs = sg.strassen_profile_stop()
        forms = sum(r.ms for r in recs if r.kernel.decode().startswith("form_sums"))
        prods = sum(r.ms for r in recs if not r.kernel.decode().startswith("form_sums"))
        row = {}
        for name, ts in times.items():
            ms = float(np.median(ts))
            row[name] = {"ms_per_step": round(ms, 4), "rounds_ms": [round(t, 4) for t in ts],
                         "effective_tflops": round(2.0 * N ** 3 / (ms * 1e-3) / 1e12, 2), **errs[name]}
        row["L1_formed"]["form_ms"] = round(forms, 4)
        row["L1_formed"]["product_ms"] = round(prods, 4)
        row["L1_formed"]["workspace_bytes"] = int(ws.numel())
        # speedups against the faster plain product
        plain = min(row["L0"]["ms_per_step"], row["L0_formed"]["ms_per_step"])
        row["plain_ms"] = plain
        row["L1_formed_vs_L0"] = round(plain / row["L1_formed"]["ms_per_step"], 4)
        row["L1_fused_vs_L0"] = round(plain / row["L1_fused"]["ms_per_step"], 4)
        row["L2_formed_vs_L0"] = round(plain / row["L2_formed"]["ms_per_step"], 4)
        out[str(N)] = row
        log("bf16x3 N=%d (median of %d rounds): L0 %.3f  L0 pre-split %.3f  L1 fused %.3f  L1 formed %.3f (forms %.3f)  "
            "L2 fused %.3f  L2 formed %.3f ms;  formed speedup over the faster plain %.3fx (L1) %.3fx (L2), fused %.3fx"
            % (N, rounds, row["L0"]["ms_per_step"], row["L0_formed"]["ms_per_step"], row["L1_fused"]["ms_per_step"],
               row["L1_formed"]["ms_per_step"], forms, row["L2_fused"]["ms_per_step"],
               row["L2_formed"]["ms_per_step"], row["L1_formed_vs_L0"], row["L2_formed_vs_L0"],
               row["L1_fused_vs_L0"]))
        del A, B, C, ws
        torch.cuda.empty_cache()
    return out


def sweep_section(A, B, C0, steps, dev, stream, log):
    """fp32 square sizes 2048-12288 and rank-k shapes m = n = 16384,
    k = 512-4096, C := A*B + C at levels 0/1/2: effective TFLOP/s.  Operands
    are copies (squares) or views (rank-k, leading dimension 16384) of the
    seeded 16384 x 16384 benchmark inputs."""
    import torch
    import paper_1808_07984_amd as sg

    out = {"square": {}, "rank_k": {}}
    for N in (2048, 4096, 8192, 12288):
        a, b = A[:N, :N].contiguous(), B[:N, :N].contiguous()
        c0 = C0[:N, :N].contiguous()
        c = c0.clone()
        row = {}
        for L in (0, 1, 2):
            ms = time_calls(lambda: sg.gemm(a, b, c, 1.0, 1.0, levels=L), steps, 1, stream)
            row["L%d" % L] = round(2.0 * N ** 3 / (ms * 1e-3) / 1e12, 2)
        out["square"][str(N)] = row
        log("sweep square %d: %s" % (N, row))
        del a, b, c, c0
    M = A.shape[0]
    c = C0.clone()
    for kk in (512, 1024, 2048, 4096):
        a, b = A[:, :kk], B[:kk, :]
        row = {}
        for L in (0, 1, 2):
            ms = time_calls(lambda: sg.gemm(a, b, c, 1.0, 1.0, levels=L), steps, 1, stream)
            row["L%d" % L] = round(2.0 * M * M * kk / (ms * 1e-3) / 1e12, 2)
        out["rank_k"][str(kk)] = row
        log("sweep rank-k k=%d: %s" % (kk, row))
    del c
    torch.cuda.empty_cache()
    return out


def awkward_section(A, B, C0, steps, dev, stream, log):
    """The padded awkward shapes (15001 x 17003 x 9007 with lda 9024,
    ldb = ldc = 17024; 3000 x 20000 x 5000 with lda 5056, ldb = ldc = 20032;
    padding holds NaN), alpha 1.5, beta 0.5, levels 0/1/2: effective TFLOP/s
    and the sampled e_norm (fp32 eps, 256 entries).  Operands are the leading
    blocks of the seeded benchmark inputs; B and C are continued along n past
    their 16384 columns by repeating their leading columns."""
    import numpy as np
    import torch
    import paper_1808_07984_amd as sg

    out = {}
    for (m, n, k, lda, ldb) in ((15001, 17003, 9007, 9024, 17024), (3000, 20000, 5000, 5056, 20032)):
        Ap = torch.full((m, lda), float("nan"), device=dev)
        Ap[:, :k] = A[:m, :k]
        Bp = torch.full((k, ldb), float("nan"), device=dev)
        w = min(n, B.shape[1])
        Bp[:, :w] = B[:k, :w]
        if n > w:
            Bp[:, w:n] = B[:k, :n - w]
        Cp = torch.full((m, ldb), float("nan"), device=dev)
        Cp[:, :n] = C0[:m, :n] if n <= C0.shape[1] else torch.cat([C0[:m], C0[:m, :n - C0.shape[1]]], 1)
        a, b, cin = Ap[:, :k], Bp[:, :n], Cp[:, :n].clone()
        rng = np.random.default_rng(m)
        rows, cols = rng.integers(0, m, 256), rng.integers(0, n, 256)
        want, _ = sampled_reference(a, b, cin, rows, cols, 1.5, 0.5)
        scale = 1.5 * k * float(a.abs().max()) * float(b.abs().max()) + 0.5 * float(cin.abs().max())
        row = {}
        for L in (0, 1, 2):
            Cp[:, :n] = cin
            sg.gemm(a, b, Cp[:, :n], 1.5, 0.5, levels=L)
            torch.cuda.synchronize()
            en = float(np.abs(sampled_got(Cp[:, :n], rows, cols) - want).max()) / (2.0 ** -23 * scale)
            if not (en <= 2.0 ** (L + 1) and bool(torch.isfinite(Cp[:, :n]).all())):
                raise SystemExit("parity failure: awkward %dx%dx%d levels=%d" % (m, n, k, L))
            ms = time_calls(lambda: sg.gemm(a, b, Cp[:, :n], 1.5, 0.5, levels=L), steps, 1, stream)
            row["L%d" % L] = {"effective_tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2),
                              "ms_per_step": round(ms, 4), "sampled_e_norm": round(en, 4)}
        key = "%dx%dx%d" % (m, n, k)
        out[key] = row
        log("awkward %s: %s" % (key, {L: v["effective_tflops"] for L, v in row.items()}))
        del Ap, Bp, Cp, a, b, cin
        torch.cuda.empty_cache()
    return out


def differentiation_section(steps, dev, stream, log):
    """StrassenMatmul forward + backward (dA = dC B^T, dB = A^T dC) at the two
    differentiation shapes, fp32, levels 1 and 2: effective TFLOP/s of the
    three products (6mnk / t)."""
    import torch
    import paper_1808_07984_amd as sg
    from paper_1808_07984_amd import inputs

    out = {}
    for (m, n, k) in ((4096, 4096, 4096), (8192, 2048, 6144)):
        A = inputs.uniform(m, k, inputs.SEED_A).to(dev).requires_grad_(True)
        B = inputs.uniform(k, n, inputs.SEED_B).to(dev).requires_grad_(True)
        dC = inputs.normal(m, n, inputs.SEED_DC).to(dev)
        for L in (0, 1, 2):
            def step():
                A.grad = None
                B.grad = None
                sg.strassen_matmul(A, B, L).backward(dC)
            ms = time_calls(step, steps, 1, stream)
            eff = 6.0 * m * n * k / (ms * 1e-3) / 1e12
            out["%dx%dx%d_L%d" % (m, n, k, L)] = {"ms_per_step": round(ms, 4),
                                                  "effective_tflops": round(eff, 2)}
            log("autograd %dx%dx%d L%d: %.3f ms fwd+bwd  effective %.1f TFLOP/s" % (m, n, k, L, ms, eff))
        del A, B, dC
    return out


def small_sizes_section(steps, dev, stream, log):
    """Small and medium squares (the regime where the paper launches products
    concurrently): effective TFLOP/s of the batched, the concurrent (atomic
    updates) and, at one level, the stream-by-stage schedules, and of the
    plain GEMM."""
    import torch
    import paper_1808_07984_amd as sg
    from paper_1808_07984_amd import inputs

    out = {}
    for N in (1024, 2048, 4096, 8192):
        A = inputs.uniform(N, N, inputs.SEED_A).to(dev)
        B = inputs.uniform(N, N, inputs.SEED_B).to(dev)
        C = torch.zeros(N, N, device=dev)
        row = {}
        for name, L, sched in (("L0", 0, sg.STRASSEN_SCHEDULE_BATCHED),
                               ("L1_batched", 1, sg.STRASSEN_SCHEDULE_BATCHED),
                               ("L1_concurrent", 1, sg.STRASSEN_SCHEDULE_CONCURRENT),
                               ("L1_streams", 1, sg.STRASSEN_SCHEDULE_STREAMS),
                               ("L2_batched", 2, sg.STRASSEN_SCHEDULE_BATCHED),
                               ("L2_concurrent", 2, sg.STRASSEN_SCHEDULE_CONCURRENT)):
            sg.strassen_set_schedule(sched)
            ms = time_calls(lambda: sg.gemm(A, B, C, 1.0, 0.0, levels=L), steps, 2, stream)
            row[name] = round(2.0 * N ** 3 / (ms * 1e-3) / 1e12, 2)
        sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_BATCHED)
        out["%d" % N] = row
        log("small N=%d: %s" % (N, row))
        del A, B, C
    return out


def mfma_probe(dev, stream, log, reps=5):
    """The matrix cores' attainable rate (strassen_probe_mfma): two
    workgroups of four waves per CU, each wave a long run of independent
    MFMAs on register operands, constant or random values; median of `reps`
    timed launches after one warm-up, TFLOP/s against the dense peaks."""
    import numpy as np
    import torch
    import paper_1808_07984_amd as sg

    wgs = 512
    out = torch.empty(wgs * 256, device=dev)
    res = {}
    for op, name, iters, per, peak in ((0, "bf16", 400000, 32768.0, 2516.6), (1, "fp16", 400000, 32768.0, 2516.6),
                                       (2, "fp32", 100000, 4096.0, FP32_MFMA_PEAK)):
        for random in (0, 1):
            def run():
                rc = sg.strassen_probe_mfma(op, random, iters, wgs, out.data_ptr(), stream.cuda_stream)
                if rc != 0:
                    raise SystemExit("strassen_probe_mfma failed: %d" % rc)
            ts = [time_calls(run, 1, 1 if r == 0 else 0, stream) for r in range(reps)]
            ms = float(np.median(ts))
            tf = wgs * 4 * iters * 4 * per / (ms * 1e-3) / 1e12
            key = "%s_%s" % (name, "random" if random else "constant")
            res[key] = {"ms": round(ms, 3), "tflops": round(tf, 1), "frac_of_peak": round(tf / peak, 4),
                        "peak": peak}
            log("mfma probe %s: %.3f ms  %.1f TFLOP/s  (%.3f of %.1f)" % (key, ms, tf, tf / peak, peak))
    return res


def launch_table(path, dev, stream, log, sizes=(1024, 2048, 4096, 8192, 16384), reps=3):
    """Every launch of C := A*B at m=n=k in `sizes`, levels 0/1/2, for fp32,
    bf16 and bf16x3 (N(0,1) operands, drawn on the device: the 16-bit
    matrix cores' power-limited clock depends on operand values), plus the
    formed one-level calls of bf16 and bf16x3: per launch the median over
    `reps` recorded calls of its library-event time, and the median call
    time.  Written to `path` as JSON records."""
    import json
    import numpy as np
    import torch
    import paper_1808_07984_amd as sg

    g = torch.Generator(device=dev)
    out = []
    for N in sizes:
        g.manual_seed(N)
        Af = torch.randn(N, N, device=dev, generator=g)
        Bf = torch.randn(N, N, device=dev, generator=g)
        C = torch.zeros(N, N, device=dev)
        operands = {"f32": (Af, Bf, "plain"), "bf16": (Af.bfloat16(), Bf.bfloat16(), "plain"),
                    "x3": (Af, Bf, "bf16x3")}
        cases = [(kind, L, "fused") for kind in ("f32", "bf16", "x3") for L in (0, 1, 2)]
        cases += [("bf16", 1, "formed"), ("x3", 1, "formed"), ("f32", 2, "formed"), ("bf16", 2, "formed"),
                  ("x3", 2, "formed")]
        for kind, L, sched in cases:
            A, B, mode = operands[kind]
            if sched == "formed":
                ws = torch.empty(sg.api.formed_workspace_bytes(N, N, N, A.dtype, mode, L),
                                 dtype=torch.uint8, device=dev)
                fn = lambda: sg.gemm_formed(A, B, C, 1.0, 0.0, mode=mode, workspace=ws, levels=L)
            else:
                fn = lambda: sg.gemm(A, B, C, 1.0, 0.0, levels=L, mode=mode)
            call_ms = [time_calls(fn, 1, 1 if r == 0 else 0, stream) for r in range(reps)]
            per = {}
            for _ in range(reps):
                sg.strassen_profile_start()
                fn()
                rc, recs = sg.strassen_profile_stop(capacity=256)
                if rc < 0:
                    raise SystemExit("strassen_profile_stop failed: %d" % rc)
                for i, r in enumerate(recs):
                    per.setdefault(i, (r, []))[1].append(r.ms)
            launches = [{"kernel": r.kernel.decode(), "launch": int(r.launch), "batch": int(r.batch),
                         "workgroups": int(r.workgroups), "ms": round(float(np.median(ms)), 4)}
                        for i, (r, ms) in sorted(per.items())]
            out.append({"kind": kind, "N": N, "levels": L, "schedule": sched,
                        "call_ms": round(float(np.median(call_ms)), 4), "launches": launches})
            log("%s N=%d L%d %s: %.3f ms, %d launches" % (kind, N, L, sched, out[-1]["call_ms"],
                                                         len(launches)))
            if sched == "formed":
                del ws
        del Af, Bf, C, operands
        torch.cuda.empty_cache()
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1808_07984_amd as sg
    from paper_1808_07984_amd import inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.launch_table:
        launch_table(args.launch_table, dev, torch.cuda.current_stream(dev), log)
        return
    if args.mfma_probe:
        print(json.dumps({"mfma_probe": mfma_probe(dev, torch.cuda.current_stream(dev), log),
                          "workload": "register-operand MFMA loops, 512 workgroups of 4 waves, "
                                      "4 independent accumulators per wave"}), flush=True)
        return
    N = args.size
    m = n = k = N
    log("generating inputs %dx%d fp32" % (N, N))
    A_h = inputs.uniform(m, k, inputs.SEED_A)
    B_h = inputs.uniform(k, n, inputs.SEED_B)
    C_h = inputs.uniform(m, n, inputs.SEED_C)
    A, B, C0 = A_h.to(dev), B_h.to(dev), C_h.to(dev)
    C = C0.clone()
    stream = torch.cuda.current_stream(dev)

    # Sampled correctness check of each level on the benchmark inputs.
    import numpy as np
    rng = np.random.default_rng(0)
    rows, cols = rng.integers(0, m, 256), rng.integers(0, n, 256)
    want, _ = sampled_reference(A_h, B_h, C_h, rows, cols, 1.0, 1.0)
    scale = k * float(A_h.abs().max()) * float(B_h.abs().max()) + float(C_h.abs().max())
    parity = {}
    for L in (0, 1, 2):
        C.copy_(C0)
        sg.gemm(A, B, C, 1.0, 1.0, levels=L)
        torch.cuda.synchronize()
        got = C[torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)].double().cpu().numpy()
        en = float(np.abs(got - want).max()) / (2.0 ** -23 * scale)
        parity["L%d" % L] = round(en, 4)
        log("parity L%d sampled e_norm %.4f (tolerance %g)" % (L, en, 2.0 ** (L + 1)))
        if not en <= 2.0 ** (L + 1):
            raise SystemExit("parity failure at levels=%d" % L)

    per_level = {}
    headline_records = None
    for L in (0, 1, 2):
        info = sg.plan_info(m, n, k, L)
        for _ in range(args.warmup):
            sg.gemm(A, B, C, 1.0, 1.0, levels=L)
        torch.cuda.synchronize()
        if L == args.levels:
            sg.strassen_profile_start()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            sg.gemm(A, B, C, 1.0, 1.0, levels=L)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / args.steps
        if L == args.levels:
            rc, headline_records = sg.strassen_profile_stop(capacity=1 << 14)
            if rc < 0:
                raise SystemExit("strassen_profile_stop failed: %d" % rc)
        eff = 2.0 * m * n * k / (ms * 1e-3) / 1e12
        exe = info.executed_flops / (ms * 1e-3) / 1e12
        per_level["L%d" % L] = {"ms_per_step": round(ms, 4), "effective_tflops": round(eff, 2),
                                "executed_tflops": round(exe, 2),
                                "mfma_frac_executed": round(exe / FP32_MFMA_PEAK, 4),
                                "launches_per_step": info.n_launches}
        log("L%d: %.3f ms/step  effective %.1f TFLOP/s  executed %.1f TFLOP/s  (wall %.2f s)"
            % (L, ms, eff, exe, wall))

    # Hybrid two-level scheme (workspace for the top-level operand sums,
    # allocated here, outside the timed region; the library allocates nothing)
    ws = torch.empty(sg.strassen_hybrid_workspace_size(m, n, k), dtype=torch.uint8, device=dev)
    C.copy_(C0)
    sg.gemm_hybrid(A, B, C, 1.0, 1.0, workspace=ws)
    torch.cuda.synchronize()
    got = C[torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)].double().cpu().numpy()
    en = float(np.abs(got - want).max()) / (2.0 ** -23 * scale)
    parity["L2_hybrid"] = round(en, 4)
    if not en <= 8.0:
        raise SystemExit("parity failure (hybrid)")
    ms = time_calls(lambda: sg.gemm_hybrid(A, B, C, 1.0, 1.0, workspace=ws), args.steps,
                    args.warmup, stream)
    info2 = sg.plan_info(m, n, k, 2)
    per_level["L2_hybrid"] = {"ms_per_step": round(ms, 4),
                              "effective_tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2),
                              "executed_tflops": round(info2.executed_flops / (ms * 1e-3) / 1e12, 2),
                              "workspace_bytes": int(ws.numel())}
    log("L2 hybrid: %.3f ms/step  effective %.1f TFLOP/s  (sampled e_norm %.4f)"
        % (ms, per_level["L2_hybrid"]["effective_tflops"], en))
    del ws

    # Formed two-level schedule (every multi-term operand sum formed into
    # caller workspace first, then 49 single-term products): bit-identical to
    # the fused two-level call
    ws = torch.empty(sg.api.formed_workspace_bytes(m, n, k, torch.float32, "plain", 2), dtype=torch.uint8,
                     device=dev)
    C.copy_(C0)
    sg.gemm(A, B, C, 1.0, 1.0, levels=2)
    ref2 = C.clone()
    C.copy_(C0)
    sg.gemm_formed(A, B, C, 1.0, 1.0, workspace=ws, levels=2)
    torch.cuda.synchronize()
    if not torch.equal(C, ref2):
        raise SystemExit("formed two-level result differs from the fused one")
    del ref2
    ms = time_calls(lambda: sg.gemm_formed(A, B, C, 1.0, 1.0, workspace=ws, levels=2), args.steps,
                    args.warmup, stream)
    per_level["L2_formed"] = {"ms_per_step": round(ms, 4),
                              "effective_tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2),
                              "executed_tflops": round(info2.executed_flops / (ms * 1e-3) / 1e12, 2),
                              "workspace_bytes": int(ws.numel())}
    log("L2 formed: %.3f ms/step  effective %.1f TFLOP/s  (equal to the fused two-level result)"
        % (ms, per_level["L2_formed"]["effective_tflops"]))
    del ws

    # Dominant kernel of the headline level: the instantiation with the most
    # device time; achieved = its executed flops / its launch time.
    by_kernel = {}
    for r in headline_records:
        key = (r.kernel.decode(), r.workgroups)
        t = by_kernel.setdefault(key, [0.0, 0.0, 0])
        t[0] += r.ms
        t[1] += r.flops
        t[2] += 1
    dom = max(by_kernel.items(), key=lambda kv: kv[1][0])
    (dom_name, dom_wg), (dom_ms, dom_flops, dom_n) = dom
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_MFMA_PEAK, 4),
                "traffic": measured_traffic(dom_name, dom_wg),
                "kernel": dom_name, "workgroups": dom_wg, "launches": dom_n,
                "avg_launch_ms": round(dom_ms / dom_n, 4),
                "flops_per_launch": dom_flops / dom_n}

    sweep = awkward = None
    if not args.no_sweep:
        sweep = sweep_section(A, B, C0, max(1, min(args.steps, 3)), dev, stream, log)
        awkward = awkward_section(A, B, C0, max(1, min(args.steps, 3)), dev, stream, log)

    compensated = None
    if not args.no_compensated:
        log("compensated section: bf16x3 plain / fused / formed at m=n=k in (8192, %d)" % N)
        compensated = compensated_section(tuple(s_ for s_ in (8192, N) if s_ <= N),
                                          max(2, min(args.steps, 5)), 3, dev, stream, log)

    precision = None
    if not args.no_precision:
        sizes = tuple(s_ for s_ in (4096, 8192, N) if s_ <= N)
        log("precision section: bf16, fp16, bf16x3 at m=n=k in %s" % (sizes,))
        del C0
        torch.cuda.empty_cache()
        precision = precision_section(sizes, max(1, min(args.steps, 5)), dev, stream, log)

    small = None
    if not args.no_small:
        small = small_sizes_section(max(3, args.steps), dev, stream, log)

    autograd = None
    if not args.no_autograd:
        autograd = differentiation_section(max(1, min(args.steps, 5)), dev, stream, log)

    head = per_level["L%d" % args.levels]
    result = {
        "metric": "effective TFLOP/s (2mnk/t) Strassen 1L/2L vs plain GEMM, m=n=k=16384",
        "value": head["effective_tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fp32 C = A*B + C, m=n=k=%d, row-major, A,B,C ~ U[-1,1] seeded, "
                               "%d-level Strassen (levels 0/1/2 all timed)" % (N, args.levels),
                   "m": m, "n": n, "k": k, "levels": args.levels, "alpha": 1.0, "beta": 1.0},
        "levels": per_level,
        "parity_sampled_e_norm": parity,
        "roofline": roofline,
    }
    if small is not None:
        result["small_sizes"] = {"workload": "fp32 C := A*B, A,B ~ U[-1,1], m=n=k=N; effective "
                                             "TFLOP/s per schedule", **small}
    if autograd is not None:
        result["differentiation"] = {"workload": "StrassenMatmul forward + backward, fp32, "
                                                 "A,B ~ U[-1,1], dC ~ N(0,1); 6mnk flops per step",
                                     **autograd}
    if sweep is not None:
        result["sweep"] = {"workload": "fp32 C = A*B + C, A,B,C ~ U[-1,1] seeded; squares m=n=k=N "
                                       "and rank-k m=n=16384; effective TFLOP/s per level", **sweep}
    if awkward is not None:
        result["awkward"] = {"workload": "fp32 C = 1.5*A*B + 0.5*C, NaN in the leading-dimension "
                                         "padding, A,B,C ~ U[-1,1] seeded", **awkward}
    if compensated is not None:
        result["compensated"] = {"workload": "bf16x3 mode, fp32 A,B ~ N(0,1) seeded, C := A*B, "
                                             "m=n=k=N; plain (L0, operands as stored), plain on "
                                             "pre-split copies (L0_formed), fused and formed one-level "
                                             "(sums in workspace), fused and formed two-level; "
                                             "*_vs_L0 against the faster plain (plain_ms); median of "
                                             "interleaved rounds; errors on 256 sampled entries vs "
                                             "fp64 in units of N*max|A|*max|B|*eps", **compensated}
    if precision is not None:
        result["precision"] = {"workload": "C := A*B (beta 0), m=n=k in {4096, 8192, %d}; A,B ~ N(0,1) "
                                           "seeded (timed) and rows of A / columns of B scaled to "
                                           "2-norms over 1e-3..1e3 (errors only); errors on 256 "
                                           "sampled entries vs fp64 dot products of the stored "
                                           "operands" % N,
                               **precision}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(A_h, B_h, C_h, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
