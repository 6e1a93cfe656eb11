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
