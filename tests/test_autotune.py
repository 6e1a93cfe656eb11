"""Autotuner: keys, validity of the choices, persistence (host), and a small
measured tuning run whose choice solves correctly (GPU)."""
import json

import numpy as np
import pytest

from paper_1510_03110_amd import autotune as T


def test_bucket_and_key():
    assert [T.n_bucket(n) for n in (1, 2, 3, 64, 65, 1024, 1040)] == [1, 2, 4, 64, 128, 1024, 2048]
    assert T.key(32, 16, 1000, 0) == T.key(32, 16, 1024, 0) == "nx32_nu16_N1024_fp64"
    assert T.key(32, 16, 1025, 1) == "nx32_nu16_N2048_mixed"


@pytest.mark.parametrize("nx,nu,N", [(32, 16, 1024), (64, 2, 1000), (4, 2, 3), (32, 32, 50), (128, 1, 4096)])
def test_default_choice_is_a_valid_plan(nx, nu, N):
    Ns, b = T.default_choice(nx, nu, N)
    assert T.valid(nx, nu, N, Ns, b)
    assert N <= Ns or Ns * nu >= nx


def test_cache_round_trip_and_fallback(tmp_path):
    path = tmp_path / "tune.json"
    t = T.Tuner(str(path))
    assert t.choose(32, 16, 1024) == (16, 4)
    t.table[T.key(32, 16, 1024, 0)] = {"Ns": 32, "branch": 8}
    t.table[T.key(64, 2, 512, 0)] = {"Ns": 4, "branch": 2}      # invalid (4*2 < 64): ignored
    t.save()
    t2 = T.Tuner(str(path))
    assert t2.choose(32, 16, 700) == (32, 8)                    # same bucket
    assert t2.choose(32, 16, 700, precision=1) == (16, 4)       # other precision: default
    assert t2.choose(64, 2, 512) == T.default_choice(64, 2, 512)
    assert t2.per_instance([(32, 16, 600), (32, 16, 2000)]) == [(32, 8), (16, 4)]
    json.loads(path.read_text())


@pytest.mark.gpu
def test_tune_small_and_solve_with_choice(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import kkt, riccati
    from paper_1510_03110_amd import rs
    from paper_1510_03110_amd import workloads as W
    t = T.Tuner(str(tmp_path / "tune.json"))
    Ns, b = t.tune(16, 16, 200, precision=0, batch=8, ns_candidates=(4, 16), branch_candidates=(2, 4))
    assert (Ns, b) in {(4, 2), (4, 4), (16, 2), (16, 4)}
    rec = T.Tuner(str(tmp_path / "tune.json")).table[T.key(16, 16, 200, 0)]
    assert rec["Ns"] == Ns and len(rec["tried"]) == 4 and rec["tile"] == "mfma16"
    probs = [W.g2(16, 16, n, seed=n) for n in (150, 200, 256)]
    per = t.per_instance([(16, 16, n) for n in (150, 200, 256)])
    bt = rs.Batch({k: [p[k] for p in probs] for k in probs[0]}, per_instance=per)
    bt.solve()
    torch.cuda.synchronize()
    assert np.all(bt.status()[:, 0] == 0)
    for i, p in enumerate(probs):
        assert kkt.rel_error(bt.result(i), riccati.solve(p)) <= 1e-10
    bt.close()


def test_tile_choices_and_plan_flags(tmp_path):
    assert T.tile_choices(16, 8) == ("mfma16", "native")
    assert T.tile_choices(32, 16) == ("mfma16",) and T.tile_choices(20, 10) == ("mfma16",)
    t = T.Tuner(str(tmp_path / "tune.json"))
    dims = [(16, 8, 100), (16, 8, 1000)]
    assert t.plan_flags(dims) == 0
    t.table[T.key(16, 8, 100, 0)] = {"Ns": 16, "branch": 4, "tile": "native"}
    assert t.plan_flags(dims) == 0                      # the other key keeps the default tiles
    t.table[T.key(16, 8, 1000, 0)] = {"Ns": 16, "branch": 4, "tile": "native"}
    assert t.plan_flags(dims) == T.NATIVE_TILES_FLAG
    assert t.plan_flags([(32, 16, 100)]) == 0


@pytest.mark.gpu
def test_tune_tile_axis_and_solve(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import kkt, riccati
    from paper_1510_03110_amd import rs
    from paper_1510_03110_amd import workloads as W
    t = T.Tuner(str(tmp_path / "tune.json"))
    t.tune(16, 8, 200, precision=0, batch=16, ns_candidates=(16,), branch_candidates=(4,))
    rec = t.table[T.key(16, 8, 200, 0)]
    assert set(rec["tried"]) == {"16/4/mfma16", "16/4/native"} and rec["tile"] in ("mfma16", "native")
    probs = [W.g2(16, 8, n, seed=n) for n in (150, 200)]
    dims = [(16, 8, n) for n in (150, 200)]
    for flags in (0, T.NATIVE_TILES_FLAG):
        bt = rs.Batch({k: [p[k] for p in probs] for k in probs[0]}, per_instance=t.per_instance(dims),
                      flags=flags)
        bt.solve()
        torch.cuda.synchronize()
        assert np.all(bt.status()[:, 0] == 0)
        for i, p in enumerate(probs):
            assert kkt.rel_error(bt.result(i), riccati.solve(p)) <= 1e-10
        bt.close()
