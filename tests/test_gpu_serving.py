"""Serving loop: receding-horizon sessions with continuous batching.

Each served request is checked against the oracle on the window it solved,
the receding-horizon semantics are checked (the window's initial state is
the previous solution's x_1, the stages shift by one), and every session's
results in the mix are bit-identical to serving that session alone."""
import numpy as np
import pytest

from oracle import kkt, riccati
from paper_1510_03110_amd import workloads as W

pytestmark = pytest.mark.gpu


def _engine(precision, record=True):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import serving
    from paper_1510_03110_amd.autotune import Tuner
    return torch, serving, serving.ServingEngine(precision=precision, lanes=2, record=True,
                                                 tuner=Tuner("/nonexistent/tune.json"))


@pytest.mark.parametrize("precision,shapes", [(0, [(4, 2), (8, 4), (32, 16), (16, 16)]),
                                              (1, [(32, 16), (16, 16)]),
                                              (1, [(8, 4), (32, 16), (64, 32)]),
                                              (0, [(64, 32), (8, 4)])])
def test_serving_mix_equals_alone_and_oracle(precision, shapes):
    torch, serving, eng = _engine(precision)
    probs = [W.g2(nx, nu, 40 + 23 * i, seed=300 + i) for i, (nx, nu) in enumerate(shapes)]
    for p in probs:
        assert eng.add_session(p) is not None
    pools = {sh: serving.stage_pool(sh[0], sh[1], 8, seed=sh[0]) for sh in set(shapes)}
    trace = serving.poisson_trace(3000.0, 0.02, len(shapes), pools, shapes, seed=1)
    assert len(trace) >= 20
    stats = eng.run(trace)
    assert stats["completed"] == len(trace)
    # every result: status ok, matches the oracle on its window; shift semantics
    for sid, res in eng.results.items():
        prev = None
        for r in res:
            assert r["status"] == 0
            win = r["window"]
            assert kkt.rel_error(r, riccati.solve(win)) <= 1e-10
            if prev is not None:
                np.testing.assert_array_equal(win["x0"], prev["x"][1])
                for k in ("A", "Qx", "lx"):
                    np.testing.assert_array_equal(win[k][:-1], prev["window"][k][1:])
            prev = r
    # alone: the same session with the same request sequence
    sid = max(eng.results, key=lambda s: len(eng.results[s]))
    mine = [t for t in trace if t[1] == sid]
    eng.close()
    _, _, one = _engine(precision)
    one.add_session(probs[sid])
    one.run([(t[0], 0, t[2]) for t in mine])
    assert len(one.results[0]) == len(eng.results[sid])
    for a, b in zip(one.results[0], eng.results[sid]):
        for k in ("x", "w", "lam"):
            np.testing.assert_array_equal(a[k], b[k])
    one.close()


def test_admission_rejects_beyond_budget():
    torch, serving, eng = _engine(0)
    eng.budget = eng.used + 1_000_000          # about 1 MB of room
    small = W.g2(4, 2, 16, seed=1)
    big = W.g2(32, 16, 2048, seed=2)
    assert eng.add_session(small) is not None
    assert eng.add_session(big) is None
    assert eng.rejected == 1
    eng.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", [0, 1])
def test_serving_c4_range_sampled_parity(precision):
    """The serving configuration's ranges: sessions with n_x in {8, 32, 64},
    n_u = n_x / 2 and horizons across [64, 4096] (both ends included), served
    from a Poisson stream with receding-horizon shifts; every 10th served
    request (10 %) is recorded with its window and checked against the serial
    oracle at 1e-10, and every request must succeed."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03110_amd import serving
    from paper_1510_03110_amd.autotune import Tuner
    eng = serving.ServingEngine(precision=precision, lanes=2, record_every=10,
                                tuner=Tuner("/nonexistent/tune.json"))
    shapes = [(8, 4, 4096), (32, 16, 3000), (64, 32, 4096), (8, 4, 64), (32, 16, 700), (64, 32, 1500)]
    for i, (nx, nu, N) in enumerate(shapes):
        assert eng.add_session(W.g2(nx, nu, N, seed=1300 + i)) is not None
    sh = [(nx, nu) for nx, nu, _ in shapes]
    pools = {s: serving.stage_pool(s[0], s[1], 8, seed=s[0]) for s in set(sh)}
    trace = serving.poisson_trace(3000.0, 0.05, len(shapes), pools, sh, seed=3)
    assert len(trace) >= 100
    stats = eng.run(trace)
    assert stats["completed"] == len(trace) and stats["failed"] == 0
    checked = 0
    for sid, res in eng.results.items():
        for r in res:
            assert r["status"] == 0
            err = kkt.rel_error(r, riccati.solve(r["window"]))
            assert err <= 1e-10, (sid, shapes[sid], err)
            checked += 1
    assert checked >= max(1, len(trace) // 100)
    eng.close()


def test_serving_failure_is_isolated():
    """A session whose window holds a stage with a G that cannot be positive
    definite reports a failure for every request while its window holds that
    stage; the other sessions' requests are served and match the oracle, and
    the failed requests are counted apart from the completed ones (no latency
    sample, no reuse of the failed factors or x_1)."""
    torch, serving, eng = _engine(0)
    good = W.g2(32, 16, 90, seed=41)
    bad = W.g2(32, 16, 90, seed=42)
    bad["Qw"] = np.array(bad["Qw"])
    bad["Qw"][70] = -1e6 * np.eye(16)
    assert eng.add_session(good) == 0 and eng.add_session(bad) == 1
    pools = {(32, 16): serving.stage_pool(32, 16, 8, seed=5)}
    trace = serving.poisson_trace(3000.0, 0.02, 2, pools, [(32, 16), (32, 16)], seed=7)
    nbad = sum(1 for t in trace if t[1] == 1)
    assert nbad >= 3 and nbad < 60           # the bad stage stays inside the window
    stats = eng.run(trace)
    assert stats["failed"] == nbad and stats["completed"] == len(trace) - nbad
    for r in eng.results[1]:
        assert r["status"] == 2
    x0 = eng.results[1][0]["window"]["x0"]
    for r in eng.results[1]:
        np.testing.assert_array_equal(r["window"]["x0"], x0)     # x0 never taken from a failed solve
    for r in eng.results[0]:
        assert r["status"] == 0 and kkt.rel_error(r, riccati.solve(r["window"])) <= 1e-10
    eng.close()
