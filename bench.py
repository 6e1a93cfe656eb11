"""Benchmark: KKT Newton-step solves/s of the parallel Riccati solver on one
MI355X in FP64 and in mixed precision, plus single-instance p50/p99 latency,
the roofline position of the dominant kernel and the serial FP64 oracle timed
on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--Ns 16]
                    [--branch 4] [--precision both|fp64|mixed]
                    [--latency-reps R] [--cpu-seconds S]

Workload: the UFTOC Newton system with n_x = 32, n_u = 16, N = 1024 (G2
generator: time-varying A_t, dense Q_t, diagonal R_t, cross term S_t), a batch
of B independent instances resident in HBM, drawn on the device with a seeded
generator.  One step = one rs_batch_solve over the batch: in FP64 the fused
solve (leaf reduction, tree up, top solve, tree down, leaf solve); in mixed
precision the FP32-leaf factorization, the solve and the FP64 residual /
refinement passes until every instance meets the 1e-10 target.  Prints one
JSON line; `value` is the faster of the two precisions (both are reported).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT Newton solves/s at n_x=32,N=1024 (FP64 vs mixed) + p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector (and FP64 matrix) peak
FP32_PEAK_TFLOPS = 157.3         # MI355X FP32 vector / FP32 matrix (dense) peak
BF16_PEAK_TFLOPS = 2500.0        # MI355X BF16 matrix (dense) peak
HBM_PEAK_GBS = 8000.0
# shapes with register/LDS-resident matrix-core kernels; the others run the
# large-block kernels (matrices in a per-workgroup global workspace)
MATRIX_CORE_SHAPES = {(16, 16), (32, 16), (32, 32)}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ------------------------------------------------ algorithmic work per stage
def flops_reduce(n, m):
    """Alg. 4 stage as executed by the leaf reduction, dense products counted
    in full, including K, k and L = -G^{-1} B'V that it stores for the leaf
    solve: 6n^3 + 12n^2 m + 6n m^2 + m^3/3 + 6n^2 + 6nm + 3m^2."""
    return 6 * n ** 3 + 12 * n * n * m + 6 * n * m * m + m ** 3 / 3 + 6 * n * n + 6 * n * m + 3 * m * m


def flops_elim(n, m):
    """Alg. 1-2 stage (last leaf, with K and k stored):
    4n^3 + 6n^2 m + 4n m^2 + m^3/3 + 4n^2 + 4nm + 3m^2."""
    return 4 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3 + 4 * n * n + 4 * n * m + 3 * m * m


def flops_solve(n, m):
    """Alg. 1-3 stage (whole-problem leaf): 4n^3 + 6n^2 m + 4n m^2 + m^3/3 + 8n^2 + 8nm + 2m^2."""
    return 4 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3 + 8 * n * n + 8 * n * m + 2 * m * m


def flops_forward(n, m):
    """Leaf solve as a forward sweep on the stored preliminary solution:
    K x, L lam_N, P x, V lam_N, A x, B w: 6n^2 + 6nm."""
    return 6 * n * n + 6 * n * m


def flops_serial(n, m):
    """Serial Riccati (Alg. 1-3) per stage, the reference count."""
    return flops_solve(n, m)


def flops_factor_reduce(n, m):
    """Matrix lines of an Alg. 4 stage (stored factorization): 6n^3 + 12n^2 m + 4n m^2 + m^3/3."""
    return 6 * n ** 3 + 12 * n * n * m + 4 * n * m * m + m ** 3 / 3


def flops_factor_elim(n, m):
    """Matrix lines of an Alg. 1 stage with K: 4n^3 + 6n^2 m + 4n m^2 + m^3/3."""
    return 4 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3


def input_bytes_stage(n, m):
    return 8 * (2 * n * n + 2 * n * m + m * m + 2 * n + m + 1)


def residual_bytes_stage(n, m):
    """FP64 residual pass per stage: reads Qx, Qw, Qxw, A, B, x, w, lam,
    x+, lam+, lx, lw, a, c; writes lx', lw', a'."""
    return 8 * (2 * n * n + 2 * n * m + m * m + (4 * n + m) + (2 * n + m + 1) + (2 * n + m))


def csrc_hash():
    """Hash of the device sources (.hip, .hpp): the kernels the counters
    describe; host-only changes of the library leave it unchanged."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1510_03110_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if not f.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for r in rec.get("records", []):
        if r.get("kernel") == kernel and r.get("workload") == workload and r.get("csrc_hash") == csrc_hash():
            return r.get("bytes_per_launch")
    return None


# ------------------------------------------------------------- CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host_probs, seconds):
    """The serial FP64 oracle on the host cores: instances are solved one per
    thread (ctypes releases the GIL) until `seconds` of wall time are used.
    The oracle is built here with -O3 -march=native for this host (same
    source and summation order as the portable build the tests use)."""
    from concurrent.futures import ThreadPoolExecutor, wait, FIRST_COMPLETED
    import tempfile
    from oracle import build as obuild, riccati
    threads = max(1, min(16, os.cpu_count() or 1))
    try:
        path = obuild.build(path=os.path.join(tempfile.gettempdir(), "rs_oracle_native_%d" % os.getpid(),
                                              "liboracle.so"), native=True)
        riccati.use_library(path)
        flags = "-O3 -march=native"
    except Exception as e:          # no compiler: the portable build
        log("native oracle build failed (%s); using the portable build" % e)
        flags = "-O3"
    riccati.solve(host_probs[0])              # load/build outside the timing
    done = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        pending = set()
        i = 0
        while True:
            while len(pending) < threads and time.perf_counter() - t0 < seconds:
                pending.add(ex.submit(riccati.solve, host_probs[i % len(host_probs)]))
                i += 1
            if not pending:
                break
            fin, pending = wait(pending, return_when=FIRST_COMPLETED)
            done += len(fin)
    el = time.perf_counter() - t0
    return done, el, threads, flags


def leaf_work(leaves, n, m, up_fn, elim_fn, down_fn, top_fn=None):
    """Per-launch algorithmic FLOPs of the leaf kernels from the plan's leaf
    table: up = reduction (or elimination for the last leaf), down = solve
    (top_fn for a leaf that is a whole instance)."""
    up = down = 0.0
    for lf in leaves:
        ln, fl = int(lf[2]), int(lf[3])
        down += ln * ((top_fn or down_fn)(n, m) if fl & 2 else down_fn(n, m))
        if fl & 2:
            continue
        up += ln * (elim_fn(n, m) if fl & 1 else up_fn(n, m))
    return up, down


def run_precision(prec, args, data, dev):
    import numpy as np
    import torch
    from paper_1510_03110_amd import rs
    from paper_1510_03110_amd import workloads as W
    from oracle import kkt, riccati

    n, m, N, B = args.nx, args.nu, args.N, args.batch
    mixed = prec != "fp64"
    pc = {"fp64": rs.RS_FP64, "mixed": rs.RS_MIXED_FP32, "bf16": rs.RS_MIXED_BF16}[prec]
    batch = rs.Batch(data, precision=pc, Ns=args.Ns, branch=args.branch, device=dev, rank_reveal=args.rank_reveal)
    log("[%s] workspace %.2f GB, leaves %d, tree items %d, depth %d" % (
        prec, batch.work_bytes / 1e9, rs.rs_plan_query(batch.plan, 0), rs.rs_plan_query(batch.plan, 1),
        rs.rs_plan_query(batch.plan, 2)))
    for _ in range(args.warmup):
        batch.solve()
    torch.cuda.synchronize()
    bad = int((batch.status()[:, 0] != 0).sum())
    log("[%s] warmup done, instances with nonzero status: %d" % (prec, bad))

    # ------------------------------------------------------ timed region
    rs.rs_plan_kernel_times(batch.plan, reset=True)
    rs.rs_plan_set_timing(batch.plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rs.rs_plan_set_timing(batch.plan, False)
    kt = rs.rs_plan_kernel_times(batch.plan, reset=True)
    ms_per_step = 1e3 * el / args.steps
    value = B * args.steps / el
    st = batch.status()
    bad = int((st[:, 0] != 0).sum())
    log("[%s] %d steps: %.3f ms/step, %.1f solves/s, nonzero status %d" % (prec, args.steps, ms_per_step,
                                                                        value, bad))
    per_step = {k: v[0] / args.steps for k, v in kt.items() if v[1]}
    launches = {k: v[1] // args.steps for k, v in kt.items() if v[1]}
    log("[%s] kernel ms per step:" % prec, {k: round(v, 3) for k, v in per_step.items()})

    # ------------------------------------------------ roofline (dominant)
    leaves = rs.rs_plan_export(batch.plan, 0)
    fused = "leaf_up" in per_step          # otherwise the solve runs on the stored factorization
    matrix_core = (n, m) in MATRIX_CORE_SHAPES
    if fused:
        up, down = leaf_work(leaves, n, m, flops_reduce, flops_elim, flops_forward, flops_solve)
        work = {"leaf_up": ("alu", up, FP64_PEAK_TFLOPS, "km_leaf_up"),
                "leaf_down": ("alu", down, FP64_PEAK_TFLOPS, "kv_leaf_fwd")}
    else:
        # the factorization's leaf-down kernel serves whole-problem leaves only
        up, down = leaf_work(leaves, n, m, flops_factor_reduce, flops_factor_elim, lambda a, b: 0.0,
                             flops_factor_elim)
        # BF16 plans: the dominant products run on BF16 matrix cores
        peak = BF16_PEAK_TFLOPS if prec == "bf16" else FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
        pre = "kf_" if matrix_core else "kl_"
        # kernels launched once per step (the refinement kernels skip
        # converged instances, so their per-launch work is not fixed)
        work = {"factor_leaf_up": ("alu", up, peak, pre + "leaf_up"),
                "factor_leaf_down": ("alu", down, peak, pre + "leaf_down")}
    avg = {k: kt[k][0] / max(kt[k][1], 1) for k in work if k in kt}
    dom = max(avg, key=lambda k: per_step.get(k, 0.0))
    bound, amount, peak, kname = work[dom]
    if bound == "hbm":
        achieved = amount / (avg[dom] * 1e-3) / 1e9
        unit = "GB/s"
    else:
        achieved = amount / (avg[dom] * 1e-3) / 1e12
        unit = "TFLOP/s"
    workload = "uftoc_g2_nx%d_nu%d_N%d_batch%d" % (n, m, N, B) + ("_rr" if args.rank_reveal else "")
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": load_traffic(kname, workload + "_" + prec),
                "kernel": kname, "avg_launch_ms": round(avg[dom], 4),
                ("bytes_per_launch" if bound == "hbm" else "flops_per_launch"): amount}

    # -------------------------------------------------- B = 1 latency
    lat = None
    if args.latency_reps > 0:
        one = rs.Batch({k: v[:1] for k, v in data.items()}, precision=pc, Ns=args.latency_Ns or args.Ns,
                       branch=args.latency_branch or args.branch, device=dev, rank_reveal=args.rank_reveal)
        for _ in range(5):
            one.solve()
        torch.cuda.synchronize()
        samples = []
        for _ in range(args.latency_reps):
            s0 = time.perf_counter()
            one.solve()
            torch.cuda.synchronize()
            samples.append(1e3 * (time.perf_counter() - s0))
        samples = np.array(samples)
        lat = {"batch": 1, "p50_ms": round(float(np.percentile(samples, 50)), 4),
               "p99_ms": round(float(np.percentile(samples, 99)), 4), "reps": args.latency_reps,
               "Ns": args.latency_Ns or args.Ns, "branch": args.latency_branch or args.branch}
        # the same call captured once as a HIP graph and replayed (no host
        # launch work per kernel); replays must reproduce the eager result
        eager = one.result(0)
        graph = one.capture(0)
        for _ in range(5):
            one.replay(graph)
        torch.cuda.synchronize()
        gsamples = []
        for _ in range(args.latency_reps):
            s0 = time.perf_counter()
            one.replay(graph)
            torch.cuda.synchronize()
            gsamples.append(1e3 * (time.perf_counter() - s0))
        rep = one.result(0)
        lat["graph_p50_ms"] = round(float(np.percentile(gsamples, 50)), 4)
        lat["graph_p99_ms"] = round(float(np.percentile(gsamples, 99)), 4)
        lat["graph_equals_eager"] = bool(all(np.array_equal(rep[k], eager[k]) for k in ("x", "w", "lam"))
                                         and int(one.status()[0, 0]) == 0)
        log("[%s] latency B=1:" % prec, lat)
        one.close()

    # -------------------------------------------- sampled parity check
    errs, host = [], []
    rng = np.random.default_rng(0)
    idx = sorted(set([0, B - 1] + list(rng.integers(0, B, size=max(0, args.verify - 2)))))[:max(args.verify, 1)]
    for i in idx:
        p = W.instance_to_numpy(data, i)
        host.append(p)
        if args.verify > 0:
            errs.append(kkt.rel_error(batch.result(i), riccati.solve(p)))
    log("[%s] sampled rel err vs oracle:" % prec, ["%.2e" % e for e in errs])
    res = {"value": round(value, 2), "ms_per_step": round(ms_per_step, 4), "nonzero_status": bad,
           "max_rel_err_sampled": max(errs) if errs else None, "sampled_instances": idx,
           "kernels_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
           "launches_per_step": launches, "latency": lat, "roofline": roofline}
    if mixed:
        stt = batch.refine_stats()
        res["refinement"] = {"corrections_min": float(stt[:, 2].min()), "corrections_max": float(stt[:, 2].max()),
                             "rel_residual_max": float(stt[:, 0].max()),
                             "est_forward_error_max": float(stt[:, 1].max()),
                             "converged": int(stt[:, 3].sum())}
        log("[%s] refinement:" % prec, res["refinement"])
    batch.close()
    del batch
    torch.cuda.empty_cache()
    return res, host


def ingest_counters(fetch_csv, write_csv, copy_bytes, workload):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of this script
    (FETCH_SIZE, then WRITE_SIZE, both with --copy-calibration-mib): HBM bytes
    per dispatch of each solver kernel's first full-batch launch, scaled by the
    factor that the plain device copy of `copy_bytes` shows on the same
    counter."""
    import csv

    def rows(path, counter):
        out = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]),
                                float(r["Counter_Value"])))
        return sorted(out)

    names = ("km_leaf_up", "km_leaf_down", "km_tree", "kv_leaf_fwd", "kf_leaf_up", "kf_leaf_down", "kf_tree",
             "kv_leaf_up", "kv_leaf_down", "kv_tree", "kr_residual")
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rr = rows(path, counter)
        copies = [v for _, k, _, v in rr if "copyBuffer" in k]
        if not copies:
            raise SystemExit("no device copy dispatch in %s" % path)
        scale = copy_bytes / (max(copies) * 1024.0)
        for name in names:
            mine = [(g, v) for _, k, g, v in rr if name + "<" in k]
            if not mine:
                continue
            gmax = max(g for g, _ in mine)
            first = next(v for g, v in mine if g == gmax)
            per.setdefault(name, {})[counter] = (first, scale)
    records = []
    for name, c in sorted(per.items()):
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        (fk, fs), (wk, ws) = c["FETCH_SIZE"], c["WRITE_SIZE"]
        fp64 = name.startswith("km_") or name == "kv_leaf_fwd"      # the fused FP64 solve's kernels
        records.append({"kernel": name, "workload": workload + ("_fp64" if fp64 else "_mixed"),
                        "csrc_hash": csrc_hash(), "fetch_kib_raw": fk, "write_kib_raw": wk,
                        "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                        "bytes_per_launch": fk * 1024.0 * fs + wk * 1024.0 * ws})
    rec = {"note": "HBM bytes per dispatch from rocprofv3 FETCH_SIZE / WRITE_SIZE (first full-batch dispatch "
                   "of each kernel), each scaled by the factor that a plain device copy of %d bytes shows on "
                   "the same counter" % copy_bytes, "records": records}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    for r in records:
        log("%-14s %-45s %.3f GB/launch" % (r["kernel"], r["workload"], r["bytes_per_launch"] / 1e9))


def run_ip(args):
    """Interior-point mode: one problem of the workload's shape (G2) with
    bounds on every input at +-0.3 of the largest |w| of its unconstrained
    solution (solved on the GPU first), solved by the Mehrotra iteration on the
    factor / solve split (one rs_factor and two rs_solve per iteration) with
    the single-instance tree (--latency-Ns, --latency-branch).  Prints one
    JSON line: solves/s, iterations, ms per iteration, active bounds."""
    import numpy as np
    import torch
    from paper_1510_03110_amd import ip, rs
    from paper_1510_03110_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n, m, N = args.nx, args.nu, args.N
    prec = "mixed" if args.precision == "mixed" else "fp64"
    pc = rs.RS_MIXED_FP32 if prec == "mixed" else rs.RS_FP64
    Ns, br = args.latency_Ns or args.Ns, args.latency_branch or args.branch
    prob = W.g2(n, m, N, seed=W.seed_for(6))
    one = rs.Batch({k: [prob[k]] for k in prob}, precision=pc, Ns=Ns, branch=br)
    one.solve()
    torch.cuda.synchronize()
    scale = float(np.abs(one.result(0)["w"]).max())
    one.close()
    lo, hi = np.full((N, m), -0.3 * scale), np.full((N, m), 0.3 * scale)
    box = ip.BoxIP(prob, lo, hi, precision=pc, Ns=Ns, branch=br)
    for _ in range(args.warmup):
        box.solve(tol=1e-9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    for _ in range(args.steps):
        r = box.solve(tol=1e-9)
        its += r["iterations"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    box.close()
    act = int((np.isclose(r["w"], lo, atol=1e-7) | np.isclose(r["w"], hi, atol=1e-7)).sum())
    out = {"metric": "box-constrained P(N) solves/s by the interior-point method", "value": round(args.steps / el, 3),
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * el / args.steps, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32+f64",
           "data": "synthetic: seeded G2 generator, bounds +-0.3 max |w| of the unconstrained solution",
           "config": {"workload": "uftoc_g2_box_nx%d_nu%d_N%d" % (n, m, N), "Ns": Ns, "branch": br,
                      "precision": prec},
           "iterations_per_solve": its / args.steps, "ms_per_iteration": round(1e3 * el / max(its, 1), 4),
           "active_bounds": act, "final_residual": r["history"][-1][0], "final_mu": r["history"][-1][1],
           "status": r["status"]}
    print(json.dumps(out), flush=True)


def run_batching(args):
    """Batching mode: 4096 instances of n_x = 16, n_u = 8 with horizons drawn
    uniformly in [32, 2048] (G1 with time-invariant A and B given once), one
    rs_batch_solve per step over all of them, FP64 and mixed precision.  The
    leaf length and branch of every instance come from the autotuner (with
    --tune: measured on this GPU first, one key per power-of-two horizon range
    and precision; else its cache or defaults).  Prints one JSON line."""
    import numpy as np
    import torch
    from paper_1510_03110_amd import autotune, rs
    from paper_1510_03110_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nx, nu, count = 16, 8, 4096
    rng = np.random.default_rng(W.seed_for(2))
    Ns_all = rng.integers(32, 2049, size=count)
    t0 = time.perf_counter()
    probs = [W.g1_invariant(nx, nu, int(n), seed=W.seed_for(2, i)) for i, n in enumerate(Ns_all)]
    data = {k: [p[k] for p in probs] for k in probs[0]}
    dims = [(nx, nu, int(n)) for n in Ns_all]
    stages = int(Ns_all.sum())
    log("batching: %d instances, %d stages, generated in %.1fs" % (count, stages, time.perf_counter() - t0))
    tuner = autotune.Tuner(args.tune_cache or None)
    precs = {"both": ("fp64", "mixed"), "all": ("fp64", "mixed")}.get(args.precision, (args.precision,))
    out_prec = {}
    for prec in precs:
        pc = rs.RS_MIXED_FP32 if prec == "mixed" else rs.RS_FP64
        if args.tune:
            for b in sorted({autotune.n_bucket(N) for _, _, N in dims}):
                tuner.tune(nx, nu, b, pc, log=log)
        per = tuner.per_instance(dims, pc)
        bt = rs.Batch(data, precision=pc, per_instance=per, flags=tuner.plan_flags(dims, pc))
        for _ in range(args.warmup):
            bt.solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            bt.solve()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t1) / args.steps
        bad = int((bt.status()[:, 0] != 0).sum())
        rec = {"value": round(count / el, 2), "ms_per_step": round(1e3 * el, 4),
               "stages_per_s": round(stages / el, 1), "nonzero_status": bad,
               "tree_shapes": sorted({"%d/%d" % tuple(p) for p in per})}
        if pc == rs.RS_MIXED_FP32:
            st = bt.refine_stats()
            rec["converged"] = int((st[:, 3] == 1.0).sum())
            rec["rel_residual_max"] = float(st[:, 0].max())
        bt.close()
        out_prec[prec] = rec
        log("[%s]" % prec, rec)
    head = max(out_prec, key=lambda k: out_prec[k]["value"])
    out = {"metric": "KKT Newton solves/s, 4096 instances of n_x=16, n_u=8, N in [32, 2048]",
           "value": out_prec[head]["value"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": out_prec[head]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if head == "fp64" else "f32+f64",
           "data": "synthetic: seeded G1 generator (time-invariant A, B), horizons uniform in [32, 2048]",
           "config": {"workload": "uftoc_g1_nx16_nu8_N32to2048_batch4096", "precision": head,
                      "autotuned": bool(args.tune)},
           "precisions": out_prec}
    print(json.dumps(out), flush=True)


def _timed_solves(batch, reps, warmup=1):
    """ms per rs_batch_solve (host clock around `reps` calls, synchronized)."""
    import torch
    for _ in range(warmup):
        batch.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.solve()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def run_extras(args, dev):
    """The other configurations, each small enough to add seconds to the run:
    single-instance latency across leaf lengths at n_x = 20, n_u = 10,
    N = 1024 (FP64); 4096 instances of n_x = 16, n_u = 8 with horizons in
    [32, 2048], leaf length and branch chosen by the autotuner measured here
    (FP64 and mixed); the large-block configuration's single instance
    (n_x = 128, n_u = 64, N = 16384; FP64, mixed, BF16 products) and its batch
    of 64 (FP64, leaf factorization kept for 1024 leaves at a time).  Sampled
    instances are checked against the oracle where it finishes in seconds."""
    import tempfile
    import numpy as np
    import torch
    from oracle import kkt, riccati
    from paper_1510_03110_amd import autotune, rs
    from paper_1510_03110_amd import workloads as W
    out = {}
    # ----------------------------------------- C2: latency across N_s
    prob = W.g2(20, 10, 1024, seed=W.seed_for(1))
    ref = riccati.solve(prob)
    lat = {}
    for Ns in (4, 8, 16, 32, 64):
        one = rs.Batch({k: [prob[k]] for k in prob}, precision=rs.RS_FP64, Ns=Ns, branch=4, device=dev)
        for _ in range(5):
            one.solve()
        torch.cuda.synchronize()
        smp = []
        for _ in range(50):
            s0 = time.perf_counter()
            one.solve()
            torch.cuda.synchronize()
            smp.append(1e3 * (time.perf_counter() - s0))
        err = kkt.rel_error(one.result(0), ref)
        lat[str(Ns)] = {"p50_ms": round(float(np.percentile(smp, 50)), 4),
                        "p99_ms": round(float(np.percentile(smp, 99)), 4), "rel_err": float(err),
                        "status": int(one.status()[0, 0])}
        one.close()
    out["c2_latency_nx20_nu10_N1024_branch4_by_Ns"] = lat
    log("extras c2:", lat)
    # ------------------------------------- C3: 4096 uneven, autotuned
    rng = np.random.default_rng(W.seed_for(2))
    horizons = rng.integers(32, 2049, size=4096)
    data = W.g1_invariant_torch(16, 8, horizons, seed=W.seed_for(2, 1), device=dev)
    dims = [(16, 8, int(n)) for n in horizons]
    tuner = autotune.Tuner(os.path.join(tempfile.gettempdir(), "rs_tune_%d.json" % os.getpid()))
    c3 = {}
    for prec, pc in (("fp64", rs.RS_FP64), ("mixed", rs.RS_MIXED_FP32)):
        for b in sorted({autotune.n_bucket(N) for _, _, N in dims}):
            tuner.tune(16, 8, b, pc, reps=2)
        per = tuner.per_instance(dims, pc)
        flags = tuner.plan_flags(dims, pc)
        bt = rs.Batch(data, precision=pc, per_instance=per, device=dev, flags=flags)
        ms = _timed_solves(bt, 3)
        st = bt.status()
        errs = [kkt.rel_error(bt.result(i), riccati.solve(W.materialize(W.instance_to_numpy(data, i))))
                for i in (0, 2047, 4095)]
        c3[prec] = {"solves_per_s": round(4096 / (ms * 1e-3), 1), "ms_per_batch": round(ms, 3),
                    "nonzero_status": int((st[:, 0] != 0).sum()), "max_rel_err_sampled": float(max(errs)),
                    "tree_shapes": sorted({"%d/%d" % tuple(p) for p in per}),
                    "tiles": "native" if flags else "mfma16"}
        bt.close()
    del data
    torch.cuda.empty_cache()
    out["c3_batching_4096_nx16_nu8_N32to2048_autotuned"] = c3
    log("extras c3:", c3)
    # --------------------------------------- C5: single and batch of 64
    data = W.c5_torch(128, 64, 16384, 1, seed=W.seed_for(5), device=dev)
    c5 = {}
    for prec, pc in (("fp64", rs.RS_FP64), ("mixed", rs.RS_MIXED_FP32), ("bf16", rs.RS_MIXED_BF16)):
        bt = rs.Batch(data, precision=pc, Ns=64, branch=8, device=dev)
        ms = _timed_solves(bt, 3)
        c5[prec] = {"ms_per_solve": round(ms, 3), "status": int(bt.status()[0, 0])}
        if pc != rs.RS_FP64:
            c5[prec]["corrections"] = float(bt.refine_stats()[0, 2])
        bt.close()
    del data
    torch.cuda.empty_cache()
    out["c5_single_nx128_nu64_N16384"] = c5
    log("extras c5 single:", c5)
    data = W.c5_torch(128, 64, 16384, 64, seed=W.seed_for(5, 64), device=dev)
    bt = rs.Batch(data, precision=rs.RS_FP64, Ns=64, branch=8, leaf_chunk=1024, device=dev)
    ms = _timed_solves(bt, 1)
    out["c5_batch64_nx128_nu64_N16384_fp64"] = {
        "solves_per_s": round(64 / (ms * 1e-3), 3), "ms_per_batch": round(ms, 1),
        "nonzero_status": int((bt.status()[:, 0] != 0).sum()), "leaf_chunk": 1024,
        "workspace_gb": round(bt.work_bytes / 1e9, 1)}
    bt.close()
    del data
    torch.cuda.empty_cache()
    log("extras c5 batch:", out["c5_batch64_nx128_nu64_N16384_fp64"])
    return out


def run_large(args):
    """Large-block mode: the large-block configuration's single instance
    (n_x = 128, n_u = 64, N = 16384, A_t per stage, B, Q, R given once) in
    one precision (--precision fp64|mixed|bf16), K timed solves after W
    warm-up solves, leaf length 64, branch 8; one JSON line with ms per solve
    and the per-kernel device times (for profiling runs)."""
    import torch
    from paper_1510_03110_amd import rs
    from paper_1510_03110_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prec = args.precision if args.precision in ("fp64", "mixed", "bf16") else "fp64"
    pc = {"fp64": rs.RS_FP64, "mixed": rs.RS_MIXED_FP32, "bf16": rs.RS_MIXED_BF16}[prec]
    data = W.c5_torch(128, 64, 16384, 1, seed=W.seed_for(5), device="cuda")
    flags = rs.RS_PLAN_REFACTOR_DOWN if args.refactor_down else 0
    bt = rs.Batch(data, precision=pc, Ns=64, branch=8, flags=flags)
    for _ in range(args.warmup):
        bt.solve()
    torch.cuda.synchronize()
    rs.rs_plan_kernel_times(bt.plan, reset=True)
    rs.rs_plan_set_timing(bt.plan, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rs.rs_plan_set_timing(bt.plan, False)
    kt = rs.rs_plan_kernel_times(bt.plan, reset=True)
    out = {"metric": "KKT Newton solve time, n_x=128, n_u=64, N=16384, one instance", "value": round(1e3 * el / args.steps, 3),
           "unit": "ms/solve", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
           "dtype": {"fp64": "f64", "mixed": "f32+f64", "bf16": "bf16+f32+f64"}[prec],
           "data": "synthetic: seeded, A_t per stage, B, Q, R given once (drawn on the device)",
           "config": {"workload": "uftoc_c5_nx128_nu64_N16384_batch1", "precision": prec, "Ns": 64, "branch": 8,
                      "master_down": "refactor" if args.refactor_down else "superposition"},
           "status": int(bt.status()[0, 0]),
           "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items() if v[1]}}
    bt.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--nx", type=int, default=32)
    ap.add_argument("--nu", type=int, default=16)
    ap.add_argument("--N", type=int, default=1024)
    # Throughput tree shape, measured at this shape and batch: two leaves of
    # 512 stages per instance (leaf lengths 128 / 256 / 512 / 1024 give
    # 30.3k / 30.8k / 31.4k / 28.7k solves/s in FP64: the leaf reduction's
    # rate per stage is the same, fewer leaves mean a smaller tree and forward
    # sweep, and a whole-problem leaf per instance leaves half the GPU idle in
    # its second round).  The B = 1 latency plan keeps short leaves (16,
    # branch 4), where the O(log N) tree is what lowers the latency.
    ap.add_argument("--Ns", type=int, default=512)
    ap.add_argument("--branch", type=int, default=8)
    ap.add_argument("--precision", choices=("both", "fp64", "mixed", "bf16", "all"), default="both",
                    help="both = fp64 and mixed; all adds bf16 (large-block shapes only)")
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--latency-Ns", type=int, default=16, help="leaf length of the B=1 latency plan")
    ap.add_argument("--latency-branch", type=int, default=4, help="branch of the B=1 latency plan")
    ap.add_argument("--verify", type=int, default=4, help="sampled instances checked against the oracle")
    ap.add_argument("--batching", action="store_true",
                    help="batching mode: 4096 instances of 16 x 8, N in [32, 2048] (see run_batching)")
    ap.add_argument("--tune", action="store_true", help="batching mode: autotune leaf length and branch first")
    ap.add_argument("--tune-cache", default="", help="autotuner cache file (default: the tuner's)")
    ap.add_argument("--ip", action="store_true",
                    help="interior-point mode: one problem with input bounds (see run_ip)")
    ap.add_argument("--refactor-down", action="store_true",
                    help="large-block mode: factor the master levels again on the way down (RS_PLAN_REFACTOR_DOWN) "
                         "instead of the superposition sweep")
    ap.add_argument("--large", action="store_true",
                    help="large-block mode: the n_x=128, n_u=64, N=16384 single instance (see run_large)")
    ap.add_argument("--rank-reveal", action="store_true",
                    help="rank-revealing master stages (allows Ns * nu < nx)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the other configurations (single-instance latency across leaf lengths, the "
                         "4096-instance batching configuration, the large-block single and batch-64 runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 counter collections of this "
                         "script (run with --copy-calibration-mib) and exit")
    args = ap.parse_args()

    if args.ingest_counters:
        ingest_counters(args.ingest_counters[0], args.ingest_counters[1], args.copy_calibration_mib << 20,
                        "uftoc_g2_nx%d_nu%d_N%d_batch%d" % (args.nx, args.nu, args.N, args.batch))
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: sharding instances or a horizon across GPUs is designed "
              "but not built; --gpus %d is not supported." % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.ip:
        run_ip(args)
        return
    if args.batching:
        run_batching(args)
        return
    if args.large:
        run_large(args)
        return

    import torch
    from paper_1510_03110_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    n, m, N, B = args.nx, args.nu, args.N, args.batch
    workload = "uftoc_g2_nx%d_nu%d_N%d_batch%d" % (n, m, N, B) + ("_rr" if args.rank_reveal else "")
    log("workload", workload, "Ns", args.Ns, "branch", args.branch)
    t0 = time.perf_counter()
    data = W.g2_torch(n, m, N, B, seed=W.seed_for(5), device=dev)
    torch.cuda.synchronize()
    log("generated inputs in %.1fs (%.1f GB)" % (time.perf_counter() - t0,
                                                 sum(v.numel() * 8 for v in data.values()) / 1e9))
    precs = {"both": ("fp64", "mixed"), "all": ("fp64", "mixed", "bf16")}.get(args.precision, (args.precision,))
    results, host = {}, None
    for prec in precs:
        results[prec], host = run_precision(prec, args, data, dev)

    head = max(precs, key=lambda k: results[k]["value"])
    r = results[head]
    extras = run_extras(args, dev) if args.extras else None

    # --------------------------------------------------- CPU oracle baseline
    cpu = None
    if args.cpu_seconds > 0:
        done, cel, threads, flags = cpu_baseline(host, args.cpu_seconds)
        cpu = {"value": round(done / cel, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(), "build": "gcc %s" % flags,
               "sample": "%d solves of instances %s of the same workload (serial FP64 Riccati, C, gcc %s) "
                         "in %.1fs on %d host threads" % (done, [int(i) for i in r["sampled_instances"]], flags,
                                                          cel, threads)}
        log("cpu baseline:", cpu)

    out = {
        "metric": METRIC, "value": r["value"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "bf16": "bf16+f32+f64"}[head],
        "data": "synthetic: seeded G2 generator drawn on the device",
        "config": {"workload": workload, "nx": n, "nu": m, "N": N, "batch": B, "Ns": args.Ns,
                   "branch": args.branch, "precision": head, "rank_reveal": bool(args.rank_reveal)},
        "latency": r["latency"],
        "max_rel_err_sampled": r["max_rel_err_sampled"],
        "roofline": r["roofline"],
        "cpu_baseline": cpu,
        "precisions": {k: {kk: vv for kk, vv in v.items() if kk != "sampled_instances"}
                       for k, v in results.items()},
        "extras": extras,
    }
    if args.copy_calibration_mib > 0:
        # a plain copy kernel of known size, for scaling FETCH_SIZE/WRITE_SIZE
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
        log("copy calibration: 3 copies of %d bytes" % nbytes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
