"""Host logic of the tree plan (Sec. 4.1 batches, Alg. 5/6 levels).

The plan is built by the C library on the host (no GPU needed).  Its tables
are checked structurally and then executed on the CPU with the oracle's
closed-form reductions and serial Riccati solves, following exactly the slot
indices and work order of the plan.  Reassembling the leaf solutions must give
the oracle's solution of the whole problem: this pins the plan semantics
(ragged last leaf, terminal elimination, message indexing) independently of
the GPU kernels."""
import numpy as np
import pytest

from oracle import kkt, reduction, riccati
from paper_1510_03110_amd import rs
from paper_1510_03110_amd import workloads as W

UP, UP_LAST, TOP, DOWN = 0, 1, 2, 3
LAST, ISTOP = 1, 2


def _tables(dims, Ns, branch):
    plan = rs.rs_plan_create(dims, Ns=Ns, branch=branch)
    try:
        return rs.rs_plan_export(plan, 0), rs.rs_plan_export(plan, 1), \
            [rs.rs_plan_query(plan, k) for k in range(5)]
    finally:
        rs.rs_plan_destroy(plan)


@pytest.mark.parametrize("N,Ns,b", [(1024, 16, 4), (37, 4, 3), (100, 8, 2), (5, 8, 4),
                                    (64, 1, 2), (65, 4, 4), (16, 4, 4), (17, 4, 4)])
def test_plan_structure(N, Ns, b):
    leaves, items, q = _tables([(4, 4, N)], Ns, b)
    # leaves cover 0..N-1 once, in order, the last one ragged and terminal
    t = 0
    for lf in leaves:
        assert lf[1] == t and 1 <= lf[2] <= Ns
        t += lf[2]
    assert t == N
    assert leaves[-1][3] & LAST
    nleaf = len(leaves)
    assert nleaf == -(-N // Ns)
    if nleaf == 1:
        assert leaves[0][3] & ISTOP and len(items) == 0
        return
    # every dependency precedes its item
    for i, it in enumerate(items):
        assert it[8] + it[9] <= i
    tops = [it for it in items if it[0] == TOP]
    assert len(tops) == 1 and tops[0][5] == 1
    n_up = sum(1 for it in items if it[0] in (UP, UP_LAST))
    n_down = sum(1 for it in items if it[0] == DOWN)
    assert n_up == n_down
    # depth is logarithmic in the number of leaves
    assert q[2] <= 1 + int(np.ceil(np.log(max(nleaf, 2)) / np.log(b)))


def _stage_dict(slots, first, count, nx):
    st = [slots[first + s] for s in range(count)]
    z = lambda shp: np.zeros((count,) + shp)
    return dict(
        Qx=np.array([s["Qx"] for s in st]).reshape(count, nx, nx),
        Qw=np.array([s["Qw"] for s in st]).reshape(count, nx, nx),
        Qxw=z((nx, nx)),
        A=np.array([s["A"] for s in st]).reshape(count, nx, nx),
        B=np.array([s["Qw"] for s in st]).reshape(count, nx, nx),
        a=np.array([s["a"] for s in st]).reshape(count, nx),
        lx=np.array([s["lx"] for s in st]).reshape(count, nx),
        lw=z((nx,)), c=np.array([s["c"] for s in st]).reshape(count))


def _emulate(prob, leaves, items):
    """Run the plan on the CPU with oracle arithmetic."""
    nx = prob["QxN"].shape[0]
    N = prob["Qx"].shape[0]
    slots = {}
    real_term = (prob["QxN"], -prob["lN"], float(prob["cN"]))
    for lf in leaves:
        _, t0, ln, fl, slot = lf[:5]
        if fl & ISTOP:
            continue
        if fl & LAST:
            QxN, lN, cN = reduction.eliminate_last(reduction.sub_problem(prob, t0, t0 + ln, real_term))
            slots[slot] = dict(Qx=QxN, lx=lN, c=cN)
        else:
            slots[slot] = reduction.reduce_closed_form(reduction.sub_problem(prob, t0, t0 + ln))
    for it in items:
        kind, _, _, first, count, last, term, out = it[:8]
        sub = _stage_dict(slots, first, count, nx)
        if kind in (UP, UP_LAST):
            if kind == UP:
                sub.update(QxN=np.zeros((nx, nx)), lN=np.zeros(nx), cN=0.0, x0=np.zeros(nx))
                slots[out] = reduction.reduce_closed_form(sub)
            else:
                t = slots[term]
                sub.update(QxN=t["Qx"], lN=t["lx"], cN=t["c"], x0=np.zeros(nx))
                QxN, lN, cN = reduction.eliminate_last(sub)
                slots[out] = dict(Qx=QxN, lx=lN, c=cN)
        else:
            if kind == TOP:
                x0 = prob["x0"]
            else:
                x0 = slots[out]["xh"]
            if last:
                t = slots[term]
                sub.update(QxN=t["Qx"], lN=t["lx"], cN=t["c"])
            else:
                m = slots[out]
                sub.update(QxN=m["P"], lN=-m["Psi"], cN=m["cb"])
            sub["x0"] = x0
            sol = riccati.solve(sub, want_factors=True)
            for s in range(count):
                slots[first + s].update(xh=sol["x"][s], P=sol["P"][s + 1], Psi=sol["Psi"][s + 1],
                                        cb=sol["cbar"][s + 1])
            if last:
                slots[term]["xh"] = sol["x"][count]
    x = np.zeros((N + 1, prob["QxN"].shape[0]))
    w = np.zeros((N, prob["Qw"].shape[1]))
    lam = np.zeros_like(x)
    for lf in leaves:
        _, t0, ln, fl, slot = lf[:5]
        if fl & (LAST | ISTOP):
            term = real_term
        else:
            m = slots[slot]
            term = (m["P"], m["Psi"], m["cb"])
        sub = reduction.sub_problem(prob, t0, t0 + ln, term)
        sub["x0"] = prob["x0"] if fl & ISTOP else slots[slot]["xh"]
        sol = riccati.solve(sub)
        x[t0:t0 + ln + 1] = sol["x"]
        w[t0:t0 + ln] = sol["w"]
        lam[t0:t0 + ln + 1] = sol["lam"]
    return dict(x=x, w=w, lam=lam)


@pytest.mark.parametrize("nx,nu,N,Ns,b", [(3, 2, 37, 4, 3), (4, 2, 64, 4, 4), (2, 2, 23, 2, 2),
                                          (4, 4, 17, 4, 4), (4, 4, 9, 8, 2), (2, 1, 40, 2, 3)])
def test_plan_emulated_with_oracle_matches_serial(nx, nu, N, Ns, b):
    prob = W.g2(nx, nu, N, seed=N + 13 * nx)
    leaves, items, _ = _tables([(nx, nu, N)], Ns, b)
    emu = _emulate(prob, leaves, items)
    ref = riccati.solve(prob)
    assert kkt.rel_error(emu, ref) < 1e-9


def test_plan_batch_groups_and_offsets():
    dims = [(4, 2, 64), (3, 2, 10), (4, 2, 7), (4, 2, 130)]
    leaves, items, q = _tables(dims, 8, 4)
    assert q[0] == sum(-(-N // 8) for _, _, N in dims)
    # scratch offsets of a group increase with the stages they cover
    for g in np.unique(leaves[:, 6]):
        L = leaves[leaves[:, 6] == g]
        assert np.all(np.diff(L[:, 5]) > 0)


def test_plan_rejects_bad_arguments():
    with pytest.raises(rs.RsError):
        rs.rs_plan_create([(4, 1, 64)], Ns=2)          # Ns*nu < nx: singular Q_w_hat
    with pytest.raises(rs.RsError):
        rs.rs_plan_create([(0, 1, 64)])
    with pytest.raises(rs.RsError):
        rs.rs_plan_create([(130, 65, 64)])             # no kernel for this shape
    with pytest.raises(rs.RsError):
        rs.rs_plan_create([(4, 2, 3)], Ns=1)           # Ns*nu < nx on a multi-leaf problem
    p = rs.rs_plan_create([(4, 2, 1)], Ns=1)           # a single leaf needs no reduction
    rs.rs_plan_destroy(p)


def test_rank_revealing_plan_allows_short_leaves():
    """With RS_PLAN_RANK_REVEAL the master stages take a rank-revealing
    factor of the reduced input weight, so Ns * nu < nx is allowed (down to
    Ns = 1); the plan adds one nx x nx identity per shape group (the master
    input weight) to the uploaded tables."""
    for dims, Ns in (([(4, 1, 64)], 2), ([(4, 2, 3)], 1), ([(32, 16, 100), (128, 64, 40)], 1)):
        with pytest.raises(rs.RsError):
            rs.rs_plan_create(dims, Ns=Ns)
        p = rs.rs_plan_create(dims, Ns=Ns, flags=rs.RS_PLAN_RANK_REVEAL)
        rs.rs_plan_destroy(p)
    dims = [(32, 16, 256), (20, 10, 100)]
    p0 = rs.rs_plan_create(dims, Ns=8, branch=4)
    p1 = rs.rs_plan_create(dims, Ns=8, branch=4, flags=rs.RS_PLAN_RANK_REVEAL)
    try:
        extra = rs.rs_plan_workspace_size(p1) - rs.rs_plan_workspace_size(p0)
        assert 8 * (32 * 32 + 20 * 20) <= extra <= 8 * (32 * 32 + 20 * 20) + 2 * 256
    finally:
        rs.rs_plan_destroy(p0)
        rs.rs_plan_destroy(p1)
    r = rs.rs_plan_create_ring([(32, 16, 64, 1, 4, 0, 0, 0)], flags=rs.RS_PLAN_RANK_REVEAL)
    rs.rs_plan_destroy(r)


def test_factored_plan_workspace_and_shape_support():
    """The stored factorization adds LeafRec doubles per leaf stage."""
    dims = [(32, 16, 1024)]
    p0 = rs.rs_plan_create(dims, Ns=16, branch=4)
    p1 = rs.rs_plan_create(dims, Ns=16, branch=4, flags=rs.RS_PLAN_FACTORED)
    try:
        extra = rs.rs_plan_workspace_size(p1) - rs.rs_plan_workspace_size(p0)
        nx, nu = 32, 16
        per_stage = (2 * nx * nx + 2 * nu * nu + 2 * nu * nx) + (nx * nx + 2 * nu * nu + nu * nx) + nx + nu
        assert 0 <= extra - 8 * 1024 * per_stage < 4096
    finally:
        rs.rs_plan_destroy(p0)
        rs.rs_plan_destroy(p1)
    # shapes without a matrix-core form store their factorization with the
    # large-block kernels
    p2 = rs.rs_plan_create([(4, 2, 64)], flags=rs.RS_PLAN_FACTORED)
    rs.rs_plan_destroy(p2)


def test_factor_needs_factored_plan():
    """rs_factor / rs_solve on a plan without the stored factorization is an
    argument error, reported before anything is launched."""
    plan = rs.rs_plan_create([(16, 16, 64)], Ns=8)
    try:
        probs = (rs.rs_problem * 1)()
        p = probs[0]
        p.nx, p.nu, p.N = 16, 16, 64
        fake = 1 << 20          # never dereferenced: the call fails its checks first
        for k in ("Qx", "Qw", "A", "B", "QxN", "x0", "x", "w", "lam"):
            setattr(p, k, fake)
        for name in ("rs_factor", "rs_solve"):
            st = getattr(rs.library(), name)(plan, probs, fake, rs.rs_plan_workspace_size(plan), None, None)
            assert st == rs.RS_ERR_ARG
    finally:
        rs.rs_plan_destroy(plan)


def test_per_instance_leaf_length_and_branch():
    """rs_plan_create_ex: each instance's tree follows its own (Ns, branch)."""
    dims = [(4, 2, 100, 8, 2), (4, 2, 100, 4, 3), (4, 2, 37, 0, 0)]
    plan = rs.rs_plan_create(dims, Ns=16, branch=4)
    try:
        leaves = rs.rs_plan_export(plan, 0)
        for inst, (ns, n) in enumerate(((8, 100), (4, 100), (16, 37))):
            L = leaves[leaves[:, 0] == inst]
            assert len(L) == -(-n // ns)
            assert L[0, 2] == min(ns, n)
        # the same instance alone gets the same tree
        alone = rs.rs_plan_create([dims[1]], Ns=16, branch=4)
        try:
            a_items = rs.rs_plan_export(alone, 1)
        finally:
            rs.rs_plan_destroy(alone)
        items = rs.rs_plan_export(plan, 1)
        mine = items[items[:, 1] == 1]
        assert len(mine) == len(a_items)
        assert np.array_equal(np.sort(mine[:, 2]), np.sort(a_items[:, 2]))
    finally:
        rs.rs_plan_destroy(plan)
    with pytest.raises(rs.RsError):
        rs.rs_plan_create([(4, 2, 100, 8, 1)])       # branch 1 is invalid


def test_large_block_shapes_plan_factored():
    """Shapes up to 128 beyond the register-resident ones are planned with the
    stored factorization, on which their FP64 solve runs, and a per-workgroup
    matrix workspace; larger shapes stay unsupported."""
    nx, nu, N = 64, 32, 256
    p0 = rs.rs_plan_create([(nx, nu, N)], Ns=8, branch=4)
    p1 = rs.rs_plan_create([(nx, nu, N)], Ns=8, branch=4, flags=rs.RS_PLAN_FACTORED)
    try:
        ws = rs.rs_plan_workspace_size(p0)
        assert ws == rs.rs_plan_workspace_size(p1)
        records = 8 * N * ((2 * nx * nx + 2 * nu * nu + 2 * nu * nx) + (nx * nx + 2 * nu * nu + nu * nx) + nx + nu)
        unit = 8 * (5 * nx * nx + 2 * nx * 2 * nx + 4 * nx * nx + 4 * nx * nx + 512 + 16 * nx)   # master blocks m = n
        assert ws >= records + (N // 8) * unit
    finally:
        rs.rs_plan_destroy(p0)
        rs.rs_plan_destroy(p1)
    for dims in [(144, 16, 64), (64, 136, 64), (129, 64, 64)]:
        with pytest.raises(rs.RsError) as e:
            rs.rs_plan_create([dims], Ns=16)
        assert e.value.status == rs.RS_ERR_UNSUPPORTED


@pytest.mark.parametrize("rr", [False, True])
@pytest.mark.parametrize("N,Ns", [(200, 16), (37, 8), (64, 16), (20, 16)])
def test_receding_horizon_plan_layout(N, Ns, rr):
    """Receding-horizon plans: leaves on absolute multiples of Ns (first leaf
    at least Ns stages, or, with rank-revealing master stages, ending at the
    first boundary; last leaf ends with the window), the reuse range marks
    exactly the interior leaves an earlier window left current, each interior
    leaf keeps its record offset across windows, and the workspace size does
    not depend on the window position."""
    nx, nu = 32, 16
    flags = rs.RS_PLAN_RANK_REVEAL if rr else 0
    sizes, where = set(), {}
    prev = (0, 0)
    for start in list(range(0, 40)) + [1000, 1001]:
        lo, hi = prev
        p = rs.rs_plan_create_ring([(nx, nu, N, Ns, 4, start, lo, hi)], flags=flags)
        try:
            sizes.add(rs.rs_plan_workspace_size(p))
            leaves = rs.rs_plan_export(p, 0)      # inst, t0, len, flags, slot, scratch, group
        finally:
            rs.rs_plan_destroy(p)
        assert int(leaves[:, 2].sum()) == N and leaves[0, 1] == 0
        assert np.all(leaves[1:, 1] == np.cumsum(leaves[:-1, 2]))
        if len(leaves) == 1:
            assert leaves[0, 3] == 3                       # LEAF_LAST | LEAF_TOP
        elif rr:
            assert 1 <= leaves[0, 2] <= Ns and (start + leaves[0, 2]) % Ns == 0 and leaves[0, 3] == 0
        else:
            assert Ns <= leaves[0, 2] < 2 * Ns and leaves[0, 3] == 0
            assert leaves[-1, 3] == 1 and (start + leaves[-1, 1]) % Ns == 0 and 1 <= leaves[-1, 2] <= Ns
            for lf in leaves[1:-1]:
                a = (start + int(lf[1])) // Ns
                assert (start + int(lf[1])) % Ns == 0 and lf[2] == Ns
                assert bool(lf[3] & 4) == (lo <= a < hi)
                if a in where:
                    assert where[a] == lf[5]                  # same record offset
                where[a] = lf[5]
            cur = rs.ring_current_leaves(start, N, Ns, rank_reveal=rr)
            assert cur == ((start + int(leaves[1, 1])) // Ns, (start + int(leaves[-1, 1])) // Ns)
        prev = rs.ring_current_leaves(start, N, Ns, rank_reveal=rr)
        if start == 39:
            prev = (0, 0)                                  # a jump: nothing current
    assert len(sizes) == 1


def test_receding_horizon_plan_update_checks_layout():
    """rs_plan_ring_update moves a receding-horizon plan to new window
    positions; rows with another horizon or leaf length, or a plan of
    another kind, are argument errors."""
    rows = [(32, 16, 100, 8, 4, 0, 0, 0), (16, 8, 60, 8, 4, 3, 0, 0)]
    p = rs.rs_plan_create_ring(rows)
    q = rs.rs_plan_create([(32, 16, 100)])
    try:
        size = rs.rs_plan_workspace_size(p)
        rs.rs_plan_ring_update(p, [(32, 16, 100, 8, 4, 7, 1, 5), (16, 8, 60, 8, 4, 9, 0, 0)])
        assert rs.rs_plan_workspace_size(p) == size
        leaves = rs.rs_plan_export(p, 0)
        assert leaves[0, 2] == 9                        # first leaf of the window at 7: [7, 16)
        for bad in ([(32, 16, 101, 8, 4, 7, 0, 0), (16, 8, 60, 8, 4, 9, 0, 0)],
                    [(32, 16, 100, 16, 4, 7, 0, 0), (16, 8, 60, 8, 4, 9, 0, 0)]):
            with pytest.raises(rs.RsError) as e:
                rs.rs_plan_ring_update(p, bad)
            assert e.value.status == rs.RS_ERR_ARG
        with pytest.raises(rs.RsError) as e:
            rs.rs_plan_ring_update(q, rows)
        assert e.value.status == rs.RS_ERR_ARG
    finally:
        rs.rs_plan_destroy(p)
        rs.rs_plan_destroy(q)


def test_bf16_precision_only_for_large_block_shapes():
    """RS_MIXED_BF16 runs on the large-block kernels; shapes served by the
    register-resident matrix-core kernels report RS_ERR_UNSUPPORTED."""
    p = rs.rs_plan_create([(128, 64, 256)], precision=rs.RS_MIXED_BF16, Ns=16)
    rs.rs_plan_destroy(p)
    with pytest.raises(rs.RsError) as e:
        rs.rs_plan_create([(32, 16, 256)], precision=rs.RS_MIXED_BF16, Ns=16)
    assert e.value.status == rs.RS_ERR_UNSUPPORTED


def _split_tables(dims, lens, brs, flags=0):
    plan = rs.rs_plan_create_split(dims, lens, brs, flags=flags)
    try:
        return rs.rs_plan_export(plan, 0), rs.rs_plan_export(plan, 1)
    finally:
        rs.rs_plan_destroy(plan)


@pytest.mark.parametrize("nx,nu,lens,brs", [
    (3, 2, [5, 2, 9, 3, 4, 2, 7, 6], [3, 2]),
    (4, 2, [2, 2, 11, 2, 3, 8, 2, 2, 5, 3, 7], [2, 4, 3]),
    (2, 1, [3, 4, 2, 6, 2, 5], [5]),
    (4, 4, [1, 1, 1, 1, 1, 1, 1], [2]),
    (3, 2, [4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 1], [2, 6]),
])
def test_split_plan_emulated_with_oracle_matches_serial(nx, nu, lens, brs):
    """rs_plan_create_split: leaves of the given lengths in order and master
    levels grouped by the given per-level sizes; executed on the CPU with the
    oracle's reductions, the plan reproduces the serial solution."""
    N = sum(lens)
    prob = W.g2(nx, nu, N, seed=N + 7 * nx)
    leaves, items = _split_tables([(nx, nu, N)], [lens], [brs])
    assert [int(lf[2]) for lf in leaves] == lens
    assert [int(lf[1]) for lf in leaves] == list(np.cumsum([0] + lens[:-1]))
    for i, it in enumerate(items):
        assert it[8] + it[9] <= i
    # the first level groups master stages by brs[0]
    lev1 = [it for it in items if it[2] == 1 and it[0] in (UP, UP_LAST)]
    if lev1:
        assert max(int(it[4]) for it in lev1) <= brs[0]
    emu = _emulate(prob, leaves, items)
    ref = riccati.solve(prob)
    assert kkt.rel_error(emu, ref) < 1e-9


@pytest.mark.parametrize("N,Ns,b", [(1024, 16, 4), (37, 4, 3), (100, 8, 2), (17, 4, 4)])
def test_split_plan_with_uniform_lengths_equals_uniform_plan(N, Ns, b):
    lens = [Ns] * (N // Ns) + ([N % Ns] if N % Ns else [])
    l1, i1 = _split_tables([(4, 4, N)], [lens], [[b]])
    l0, i0, _ = _tables([(4, 4, N)], Ns, b)
    np.testing.assert_array_equal(l1, l0)
    np.testing.assert_array_equal(i1, i0)


def test_split_plan_rejects_bad_arguments():
    with pytest.raises(rs.RsError):
        rs.rs_plan_create_split([(4, 2, 10)], [[4, 5]], [[2]])        # lengths sum to 9
    with pytest.raises(rs.RsError):
        rs.rs_plan_create_split([(4, 2, 10)], [[0, 10]], [[2]])       # empty leaf
    with pytest.raises(rs.RsError):
        rs.rs_plan_create_split([(4, 2, 10)], [[5, 5]], [[1]])        # group size 1
    with pytest.raises(rs.RsError):
        rs.rs_plan_create_split([(4, 2, 10)], [[1, 9]], [[2]])        # 1 * nu < nx, plain form
    p = rs.rs_plan_create_split([(4, 2, 10)], [[1, 9]], [[2]], flags=rs.RS_PLAN_RANK_REVEAL)
    rs.rs_plan_destroy(p)
    p = rs.rs_plan_create_split([(4, 2, 10)], [[9, 1]], [[2]])        # a short last leaf is fine
    rs.rs_plan_destroy(p)
