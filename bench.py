"""Benchmark: KKT Newton-step solves/s of the parallel Riccati solver on one
MI355X, plus single-instance latency, per-kernel roofline and the serial FP64
oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--Ns 16]
                    [--branch 4] [--latency-reps R] [--cpu-seconds S]

Workload: the UFTOC Newton system with n_x = 32, n_u = 16, N = 1024 (G2
generator: time-varying A_t, dense Q_t, diagonal R_t, cross term S_t), a batch
of B independent instances resident in HBM, drawn on the device with a seeded
generator.  One step = one rs_batch_solve over the batch (leaf reduction,
tree up, top solve, tree down, leaf solve).  Prints one JSON line.
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
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ------------------------------------------------ algorithmic work per stage
def flops_reduce(n, m):
    """Alg. 4 stage as executed by the leaf reduction (dense products counted
    in full): 6n^3 + 12n^2 m + 4n m^2 + m^3/3 + 6n^2 + 6nm + m^2."""
    return 6 * n ** 3 + 12 * n * n * m + 4 * n * m * m + m ** 3 / 3 + 6 * n * n + 6 * n * m + m * m


def flops_elim(n, m):
    """Alg. 1-2 stage (last leaf): 4n^3 + 6n^2 m + 3n m^2 + m^3/3 + 4n^2 + 4nm + m^2."""
    return 4 * n ** 3 + 6 * n * n * m + 3 * n * m * m + m ** 3 / 3 + 4 * n * n + 4 * n * m + m * m


def flops_solve(n, m):
    """Alg. 1-3 stage (leaf solve): 4n^3 + 6n^2 m + 4n m^2 + m^3/3 + 8n^2 + 8nm + 2m^2."""
    return 4 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3 + 8 * n * n + 8 * n * m + 2 * m * m


def flops_serial(n, m):
    """Serial Riccati (Alg. 1-3) per stage, the reference count."""
    return flops_solve(n, m)


def input_bytes_stage(n, m):
    return 8 * (2 * n * n + 2 * n * m + m * m + 2 * n + m + 1)


def csrc_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1510_03110_amd", "csrc")
    for f in sorted(os.listdir(d)):
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
def cpu_baseline(host_probs, seconds):
    """The serial FP64 oracle on the host cores: instances are solved one per
    thread (ctypes releases the GIL) until `seconds` of wall time are used."""
    from concurrent.futures import ThreadPoolExecutor, wait, FIRST_COMPLETED
    from oracle import riccati
    threads = max(1, min(16, os.cpu_count() or 1))
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
    return done, el, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--nx", type=int, default=32)
    ap.add_argument("--nu", type=int, default=16)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--branch", type=int, default=4)
    ap.add_argument("--latency-reps", type=int, default=200)
    ap.add_argument("--latency-Ns", type=int, default=0, help="leaf length of the B=1 latency plan (0: --Ns)")
    ap.add_argument("--verify", type=int, default=4, help="sampled instances checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver shards instances or horizons across GPUs "
              "only by design (see DESIGN.md); --gpus %d is not supported." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1510_03110_amd import rs
    from paper_1510_03110_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    n, m, N, B = args.nx, args.nu, args.N, args.batch
    workload = "uftoc_g2_nx%d_nu%d_N%d_batch%d" % (n, m, N, B)
    log("workload", workload, "Ns", args.Ns, "branch", args.branch)
    t0 = time.perf_counter()
    data = W.g2_torch(n, m, N, B, seed=W.seed_for(5), device=dev)
    torch.cuda.synchronize()
    log("generated inputs in %.1fs (%.1f GB)" % (time.perf_counter() - t0,
                                                 sum(v.numel() * 8 for v in data.values()) / 1e9))

    batch = rs.Batch(data, Ns=args.Ns, branch=args.branch, device=dev)
    stream = torch.cuda.current_stream()
    log("workspace %.2f GB, leaves %d, tree items %d, depth %d" % (
        batch.work_bytes / 1e9, rs.rs_plan_query(batch.plan, 0), rs.rs_plan_query(batch.plan, 1),
        rs.rs_plan_query(batch.plan, 2)))

    for _ in range(args.warmup):
        batch.solve()
    torch.cuda.synchronize()
    st = batch.status()
    bad = int((st[:, 0] != 0).sum())
    log("warmup done, instances with nonzero status: %d" % bad)

    # ---------------------------------------------------------- timed region
    rs.rs_plan_kernel_times(batch.plan, reset=True)
    rs.rs_plan_set_timing(batch.plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rs.rs_plan_set_timing(batch.plan, False)
    ktimes = rs.rs_plan_kernel_times(batch.plan, reset=True)
    ms_per_step = 1e3 * el / args.steps
    value = B * args.steps / el
    log("timed %d steps: %.3f ms/step, %.1f solves/s" % (args.steps, ms_per_step, value))
    log("kernel ms per launch:", {k: round(v[0] / max(v[1], 1), 4) for k, v in ktimes.items()})

    # ---------------------------------------------------- roofline (dominant)
    leaves = rs.rs_plan_export(batch.plan, 0)
    up_flops = 0.0
    for lf in leaves:
        ln, fl = int(lf[2]), int(lf[3])
        if fl & 2:
            continue
        up_flops += ln * (flops_elim(n, m) if fl & 1 else flops_reduce(n, m))
    down_flops = float(leaves[:, 2].sum()) * flops_solve(n, m)
    per_launch = {"leaf_up": up_flops, "leaf_down": down_flops}
    avg_ms = {k: ktimes[k][0] / max(ktimes[k][1], 1) for k in ("leaf_up", "leaf_down", "tree")}
    dom = max(("leaf_up", "leaf_down"), key=lambda k: avg_ms[k])
    achieved = per_launch[dom] / (avg_ms[dom] * 1e-3) / 1e12
    traffic = load_traffic("k_" + dom, workload)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_" + dom, "avg_launch_ms": round(avg_ms[dom], 4),
                "flops_per_launch": per_launch[dom]}

    # ----------------------------------------------------- B = 1 latency
    lat = None
    if args.latency_reps > 0:
        one = rs.Batch({k: v[:1] for k, v in data.items()}, Ns=args.latency_Ns or args.Ns,
                       branch=args.branch, device=dev)
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
               "Ns": args.latency_Ns or args.Ns}
        log("latency B=1:", lat)
        one.close()

    # ------------------------------------------------ sampled parity check
    from oracle import kkt, riccati
    host = []
    errs = []
    rng = np.random.default_rng(0)
    idx = sorted(set([0, B - 1] + list(rng.integers(0, B, size=max(0, args.verify - 2)))))[:max(args.verify, 1)]
    for i in idx:
        p = W.instance_to_numpy(data, i)
        host.append(p)
        if args.verify > 0:
            ref = riccati.solve(p)
            errs.append(kkt.rel_error(batch.result(i), ref))
    max_err = max(errs) if errs else None
    log("sampled rel err vs oracle:", ["%.2e" % e for e in errs])

    # --------------------------------------------------- CPU oracle baseline
    cpu = None
    if args.cpu_seconds > 0:
        done, cel, threads = cpu_baseline(host, args.cpu_seconds)
        cpu = {"value": round(done / cel, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": "%d solves of instances %s of the same workload (serial FP64 Riccati, C) "
                         "in %.1fs on %d host threads" % (done, idx, cel, threads)}
        log("cpu baseline:", cpu)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded G2 generator drawn on the device",
        "config": {"workload": workload, "nx": n, "nu": m, "N": N, "batch": B, "Ns": args.Ns,
                   "branch": args.branch, "precision": "fp64"},
        "latency": lat,
        "max_rel_err_sampled": max_err,
        "kernels_ms_per_launch": {k: round(v, 4) for k, v in avg_ms.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    batch.close()
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
