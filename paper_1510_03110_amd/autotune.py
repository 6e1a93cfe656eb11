"""Autotuner for the tree shape and tile shape of the parallel Riccati solve.

The leaf length N_s (Sec. 4.1: the horizon is split into subintervals of
N_s stages) and the branch b of the master tree (Alg. 5: b master stages per
master subproblem) trade leaf work against tree depth: long leaves mean few
master stages but long sequential leaf sweeps; short leaves mean many
parallel leaves but a deeper tree of FP64 master problems.  The best pair
depends on (n_x, n_u), the horizon and the precision, so it is measured.

For shapes with n_x = 16 or 32 and n_u < 16 it also chooses the tile shape:
the 16 x 16 matrix-core tile kernels on inputs padded to n_u = 16, or the
kernels for the shape itself (RS_PLAN_NATIVE_TILES).

A choice is stored per key (n_x, n_u, N range, precision), where the N range
is the power-of-two bucket [2^(k-1), 2^k).  It never depends on the batch an
instance is solved in (the plan of an instance is a function of its own
key), so an instance gives the same result alone and in any batch.  Choices
persist in a JSON cache: $RS_TUNE_CACHE, else
~/.cache/paper_1510_03110_amd/tune.json.

Timing runs the library's own HIP-graph replay of rs_batch_solve on a
synthetic batch of the key's shape (G1 stages, about 2^20 of them, so the
GPU is full), three replays per candidate after one warm-up.
"""
import json
import os
import time

NS_CANDIDATES = (4, 8, 16, 32, 64)
BRANCH_CANDIDATES = (2, 4, 8)
# Tile shape: shapes with n_x = 16 or 32 and n_u < 16 run on the 16 x 16
# matrix-core tiles with padded inputs ("mfma16") or on the kernels for their
# own shape ("native", RS_PLAN_NATIVE_TILES).
TILE_CANDIDATES = ("mfma16", "native")
NATIVE_TILES_FLAG = 16
DEFAULT_NS, DEFAULT_BRANCH = 16, 4
PRECISIONS = {0: "fp64", 1: "mixed"}


def n_bucket(N):
    """Upper end of the power-of-two range holding N (1, 2, 4, ..., 2^k >= N)."""
    b = 1
    while b < N:
        b <<= 1
    return b


def key(nx, nu, N, precision):
    return "nx%d_nu%d_N%d_%s" % (nx, nu, n_bucket(N), PRECISIONS.get(precision, str(precision)))


def valid(nx, nu, N, Ns, branch):
    """A tree shape the plan accepts: several leaves need Ns*nu >= nx (the
    reduced input weight of a leaf is singular otherwise, Sec. 4.2)."""
    if Ns < 1 or branch < 2:
        return False
    return N <= Ns or Ns * nu >= nx


def tile_choices(nx, nu):
    """Tile shapes that differ for this shape."""
    return TILE_CANDIDATES if (nx in (16, 32) and nu < 16) else TILE_CANDIDATES[:1]


def default_choice(nx, nu, N):
    """Untuned choice: the smallest of 16, 32, 64, ... that the shape allows."""
    Ns = DEFAULT_NS
    while not valid(nx, nu, N, Ns, DEFAULT_BRANCH):
        Ns *= 2
    return Ns, DEFAULT_BRANCH


def cache_path():
    p = os.environ.get("RS_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1510_03110_amd", "tune.json")


class Tuner:
    """Per-key (Ns, branch) choices with a persistent JSON cache."""

    def __init__(self, path=None):
        self.path = path or cache_path()
        self.table = {}
        try:
            with open(self.path) as f:
                self.table = json.load(f)
        except (OSError, ValueError):
            self.table = {}

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def choose(self, nx, nu, N, precision=0):
        rec = self.table.get(key(nx, nu, N, precision))
        if rec and valid(nx, nu, N, rec["Ns"], rec["branch"]):
            return rec["Ns"], rec["branch"]
        return default_choice(nx, nu, N)

    def per_instance(self, dims, precision=0):
        """(Ns, branch) for each (nx, nu, N) of a batch (rs_plan_create_ex)."""
        return [self.choose(nx, nu, N, precision) for nx, nu, N in dims]

    def tile(self, nx, nu, N, precision=0):
        rec = self.table.get(key(nx, nu, N, precision))
        return rec.get("tile", TILE_CANDIDATES[0]) if rec else TILE_CANDIDATES[0]

    def plan_flags(self, dims, precision=0):
        """Plan-wide flags of the tuned tile shape: native tiles only if every
        instance's key chose them (the flag applies to the whole plan)."""
        tiles = {self.tile(nx, nu, N, precision) for nx, nu, N in dims if len(tile_choices(nx, nu)) > 1}
        return NATIVE_TILES_FLAG if tiles == {"native"} else 0

    def tune(self, nx, nu, N, precision=0, batch=None, ns_candidates=NS_CANDIDATES,
             branch_candidates=BRANCH_CANDIDATES, reps=3, device="cuda", log=None, tiles=None):
        """Measure every valid candidate (leaf length, branch and, where it
        matters, tile shape) on a synthetic batch of the key's shape (horizon
        = the bucket's upper end) and store the fastest."""
        import torch
        from . import rs
        from . import workloads as W
        Nt = n_bucket(N)
        B = batch or max(1, min(1024, (1 << 20) // Nt))
        # the timing depends on the shape only: G1 stages drawn in a few
        # device calls (A, B given once per instance)
        data = W.g1_invariant_torch(nx, nu, [Nt] * B, seed=W.seed_for(2, 0), device=device)
        results = {}
        for tile in (tiles or tile_choices(nx, nu)):
            flags = NATIVE_TILES_FLAG if tile == "native" else 0
            for Ns in ns_candidates:
                for br in branch_candidates:
                    if not valid(nx, nu, Nt, Ns, br) or (Ns >= Nt and br != branch_candidates[0]):
                        continue
                    try:
                        bt = rs.Batch(data, precision=precision, Ns=Ns, branch=br, device=device, flags=flags)
                    except rs.RsError:      # no kernel for this tile shape and precision
                        continue
                    try:
                        g = bt.capture(0)
                        bt.replay(g)
                        torch.cuda.synchronize()
                        if (bt.status()[:, 0] != 0).any():
                            continue
                        t0 = time.perf_counter()
                        for _ in range(reps):
                            bt.replay(g)
                        torch.cuda.synchronize()
                        ms = 1e3 * (time.perf_counter() - t0) / reps
                    finally:
                        bt.close()
                    results["%d/%d/%s" % (Ns, br, tile)] = round(ms, 4)
                    if log:
                        log("tune %s Ns=%d branch=%d tile=%s: %.3f ms" % (key(nx, nu, N, precision), Ns, br,
                                                                          tile, ms))
        if not results:
            return default_choice(nx, nu, N)
        best = min(results, key=results.get)
        Ns, br, tile = best.split("/")
        Ns, br = int(Ns), int(br)
        self.table[key(nx, nu, N, precision)] = {"Ns": Ns, "branch": br, "tile": tile, "ms": results[best],
                                                 "batch": B, "horizon": Nt, "tried": results}
        self.save()
        return Ns, br
