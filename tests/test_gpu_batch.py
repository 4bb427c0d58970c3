"""Batched TWED (one persistent launch over many pairs) against the CPU oracle.

Bars as for single pairs: FP64 within 1e-12 relative, FP32 within 1e-5 of the
FP64 oracle on the same rounded inputs; structural properties (symmetry, zero
diagonal, equality with the single-pair call) exactly.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2007_16135_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2007_16135_amd as tw  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(col, precision):
    dt = torch.float64 if precision == "f64" else torch.float32
    npdt = np.float64 if precision == "f64" else np.float32
    X = torch.as_tensor(np.ascontiguousarray(col.X.astype(npdt)), device="cuda")
    T = torch.as_tensor(np.ascontiguousarray(col.T.astype(npdt)), device="cuda")
    assert X.dtype == dt
    return X, T


def ref_inputs(col, precision):
    if precision == "f64":
        return col.X, col.T
    return col.X.astype(np.float32).astype(np.float64), col.T.astype(np.float32).astype(np.float64)


def max_rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


TOL = {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-6}


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_acc64"])
def test_symmetric_small(precision):
    col = synth.batch_collection(40, 1, 300, seed=11)
    X, T = to_dev(col, precision)
    say(f"batch symmetric 40 {precision}")
    D = tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision=precision)
    torch.cuda.synchronize()
    D = D.cpu().numpy().astype(np.float64)
    Xr, Tr = ref_inputs(col, precision)
    ref = oracle.get().all_pairs(Xr, Tr, col.off, 1e-3, 1.0, 1.0)
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 0)
    assert max_rel(D, ref) <= TOL[precision]


@pytest.mark.parametrize("dim,p", [(2, 1.0), (3, 2.0), (5, 3.0), (8, 2.0)])
def test_symmetric_multidim(dim, p):
    rng_cols = []
    for k in range(24):
        r = np.random.default_rng([77, k])
        L = int(r.integers(1, 200))
        rng_cols.append((synth.walk(r, L, dim), synth.irregular_times(r, L)))
    col = synth.pack([x for x, _ in rng_cols], [t for _, t in rng_cols])
    X, T = to_dev(col, "f64")
    say(f"batch multidim dim{dim} p{p}")
    D = tw.twed_batch(X, T, col.off, nu=0.05, lam=0.5, p=p, precision="f64")
    torch.cuda.synchronize()
    ref = oracle.get().all_pairs(col.X, col.T, col.off, 0.05, 0.5, p)
    assert max_rel(D.cpu().numpy(), ref) <= 1e-12


def test_rectangular_and_pair_list():
    cx = synth.batch_collection(17, 1, 400, seed=21)
    cy = synth.batch_collection(13, 1, 400, seed=22)
    X, TX = to_dev(cx, "f64")
    Y, TY = to_dev(cy, "f64")
    say("batch rectangular 17x13")
    D = tw.twed_batch(X, TX, cx.off, Y, TY, cy.off, nu=0.01, lam=0.3, p=1.0, precision="f64")
    torch.cuda.synchronize()
    prs = np.array([(i, j) for i in range(17) for j in range(13)], np.int64)
    ref = oracle.get().pairs(cx.X, cx.T, cx.off, cy.X, cy.T, cy.off, prs, 0.01, 0.3, 1.0)
    assert max_rel(D.cpu().numpy().reshape(-1), ref) <= 1e-12

    rng = np.random.default_rng(3)
    pl = np.stack([rng.integers(0, 17, 300), rng.integers(0, 13, 300)], axis=1).astype(np.int64)
    say("batch pair list 300")
    Dp = tw.twed_batch(X, TX, cx.off, Y, TY, cy.off, pairs=torch.as_tensor(pl, device="cuda"),
                       nu=0.01, lam=0.3, p=1.0, precision="f64")
    torch.cuda.synchronize()
    Dm = D.cpu().numpy()
    assert np.array_equal(Dp.cpu().numpy(), Dm[pl[:, 0], pl[:, 1]])


def test_entries_equal_single_pair_call():
    col = synth.batch_collection(12, 1, 700, seed=31)
    X, T = to_dev(col, "f64")
    D = tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision="f64").cpu().numpy()
    for (i, j) in [(0, 1), (3, 7), (11, 2), (5, 9)]:
        a0, a1 = col.off[i], col.off[i + 1]
        b0, b1 = col.off[j], col.off[j + 1]
        say(f"pair call {i},{j}")
        v = tw.twed_pair(X[a0:a1], T[a0:a1], X[b0:b1], T[b0:b1], 1e-3, 1.0, 1.0, "f64")
        torch.cuda.synchronize()
        assert float(v.item()) == D[i, j]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_width_classes_bitwise(prec):
    # A symmetric batch whose pairs fall in every width class: K <= 8 (the
    # shorter series at most 512 samples), K = 9..16 (both longer than 512)
    # and the single-pair sweep (both longer than 1024).  The wide pairs run
    # in one launch, the narrow ones in another; every entry equals twed_pair
    # bit for bit, and the pair-list and rectangular forms give the same.
    rng = np.random.default_rng(61)
    lens = [30, 200, 511, 512, 513, 700, 1000, 1024, 1025, 1500, 64, 577]
    col = synth.pack([synth.walk(rng, L, 1) for L in lens], [synth.irregular_times(rng, L) for L in lens])
    X, T = to_dev(col, prec)
    say(f"width classes {prec}: {len(lens)} series")
    D = tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision=prec).cpu().numpy()
    n = len(lens)
    for i in range(n):
        for j in range(i + 1, n):
            a = slice(col.off[i], col.off[i + 1])
            b = slice(col.off[j], col.off[j + 1])
            v = tw.twed_pair(X[a], T[a], X[b], T[b], 1e-3, 1.0, 1.0, prec).item()
            assert D[i, j] == v and D[j, i] == v, (lens[i], lens[j], D[i, j], v)
    prs = np.array([(i, j) for i in range(n) for j in range(n) if i != j], dtype=np.int64)
    Dp = tw.twed_batch(X, T, col.off, X, T, col.off, pairs=torch.as_tensor(prs, device="cuda"), nu=1e-3,
                       lam=1.0, p=1.0, precision=prec).cpu().numpy()
    assert np.array_equal(Dp, D[prs[:, 0], prs[:, 1]])
    Dr = tw.twed_batch(X, T, col.off, X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision=prec).cpu().numpy()
    off = ~np.eye(n, dtype=bool)
    assert np.array_equal(Dr[off], D[off])


def test_empty_pair_list_and_single_series():
    col = synth.batch_collection(1, 5, 50, seed=41)
    X, T = to_dev(col, "f32")
    D = tw.twed_batch(X, T, col.off, precision="f32")
    torch.cuda.synchronize()
    assert D.shape == (1, 1) and float(D[0, 0]) == 0.0
    Dp = tw.twed_batch(X, T, col.off, X, T, col.off, pairs=torch.zeros((0, 2), dtype=torch.int64, device="cuda"),
                       precision="f32")
    assert Dp.numel() == 0


def test_all_pairs_2048_sampled():
    """2,048 1-D FP32 walks, lengths U[64,1024], in the benchmark's launch
    configuration; 1,500 sampled entries checked against the FP64 oracle."""
    col = synth.batch_collection(2048, 64, 1024)
    X, T = to_dev(col, "f32")
    say("batch 2048 all pairs f32")
    D = tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision="f32")
    torch.cuda.synchronize()
    D = D.cpu().numpy()
    assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0)
    rng = np.random.default_rng(5)
    i = rng.integers(0, 2048, 1500)
    j = rng.integers(0, 2048, 1500)
    keep = i != j
    prs = np.stack([i[keep], j[keep]], axis=1).astype(np.int64)
    Xr, Tr = ref_inputs(col, "f32")
    say("oracle on sampled entries")
    ref = oracle.get().pairs(Xr, Tr, col.off, Xr, Tr, col.off, prs, 1e-3, 1.0, 1.0)
    err = max_rel(D[prs[:, 0], prs[:, 1]], ref)
    say(f"max relative error of sampled entries: {err:.3e}")
    assert err <= 1e-5


def test_paper_shaped_rn_query_vs_oracle():
    """One query against many 28-step series in R^28 (the shape of the paper's
    R^N experiment) in the rectangular batch mode, FP64, against the oracle."""
    col = synth.paper_shaped_rn(count=300, length=28, dim=28, seed=29)
    q = col.subset([0])
    X, T = to_dev(q, "f64")
    Y, TY = to_dev(col, "f64")
    say("batch R^28 1 x 300 f64")
    D = tw.twed_batch(X.reshape(-1, 28), T, q.off, Y.reshape(-1, 28), TY, col.off, nu=1e-3, lam=1.0, p=2.0,
                      precision="f64")
    torch.cuda.synchronize()
    D = D.cpu().numpy().reshape(-1)
    pairs = np.array([(0, j) for j in range(col.count)], dtype=np.int64)
    ref = oracle.get().pairs(q.X, q.T, q.off, col.X, col.T, col.off, pairs, 1e-3, 1.0, 2.0, threads=8)
    assert max_rel(D, ref) <= 1e-12
    assert D[0] == 0.0


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_acc64"])
def test_short_query_lane_mode_bitwise(prec):
    """One query of at most 32 samples against a collection runs one lane per
    pair; every entry must be bitwise what twed_pair gives for that pair
    (ragged collection lengths, some shorter and some much longer than the
    query, a count that is not a multiple of 64), and within the precision's
    bar of the oracle."""
    rng = np.random.default_rng(17)
    for nq, dim, p in ((1, 1, 1.0), (5, 3, 2.0), (32, 8, 2.0), (28, 28, 2.0), (17, 2, 3.0)):
        col = synth.batch_collection(131, 1, 90, seed=100 + nq)
        Y = rng.standard_normal((len(col.T), dim)).cumsum(0)
        q = rng.standard_normal((nq, dim)).cumsum(0)
        tq = np.cumsum(rng.exponential(1.0, nq))
        dt = torch.float64 if prec == "f64" else torch.float32
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
        say(f"lane mode {prec} query {nq} dim {dim}")
        D = tw.twed_batch(f(q), f(tq), np.array([0, nq]), f(Y), f(col.T), col.off, nu=0.05, lam=0.7, p=p,
                          precision=prec)
        torch.cuda.synchronize()
        D = D.cpu().numpy().reshape(-1)
        for j in range(col.count):
            yj = Y[col.off[j]:col.off[j + 1]]
            tj = col.T[col.off[j]:col.off[j + 1]]
            v = float(tw.twed_pair(f(q), f(tq), f(yj), f(tj), 0.05, 0.7, p, prec).item())
            assert D[j] == v, (j, D[j], v)
        rounded = (lambda a: a) if prec == "f64" else (lambda a: np.asarray(a, np.float32).astype(np.float64))
        ref = oracle.get().pairs(rounded(q), rounded(tq), np.array([0, nq]), rounded(Y), rounded(col.T), col.off,
                                 np.array([(0, j) for j in range(col.count)]), 0.05, 0.7, p)
        assert max_rel(D, ref) <= {"f64": 1e-12, "f32": 1e-5, "f32_acc64": 1e-6}[prec]


def _walks(rng, lens, dim):
    xs = [rng.standard_normal((n, dim)).cumsum(0) for n in lens]
    ts = [np.cumsum(rng.exponential(1.0, n)) for n in lens]
    return np.concatenate(xs), np.concatenate(ts), np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


@pytest.mark.parametrize("case", ["sym_long_f32", "query_lane_f64", "pairs_acc64"])
def test_batch_plan_graph_replay(case):
    """A batch plan runs kernels only, so its run can be captured in a graph:
    every replay, on fresh input values copied into the captured tensors and
    with other library work and host synchronisation between replays, is
    bitwise the eager twed_batch result on the same values."""
    rng = np.random.default_rng({"sym_long_f32": 5, "query_lane_f64": 6, "pairs_acc64": 7}[case])
    prec, dim = {"sym_long_f32": ("f32", 1), "query_lane_f64": ("f64", 3), "pairs_acc64": ("f32_acc64", 2)}[case]
    dt = torch.float64 if prec == "f64" else torch.float32
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    kw = dict(nu=0.02, lam=0.6, p=2.0 if dim > 1 else 1.0, precision=prec)
    if case == "sym_long_f32":
        # two series longer than one wave's strip: the single-pair sweeps
        lens_x = list(rng.integers(20, 300, 30)) + [1500, 1300]
        lens_y, n_pairs = None, 0
    elif case == "query_lane_f64":
        lens_x, lens_y, n_pairs = [23], list(rng.integers(5, 200, 150)), 0
    else:
        lens_x, lens_y, n_pairs = list(rng.integers(10, 120, 19)), list(rng.integers(10, 300, 11)), 257
    variants = []
    for _ in range(4):
        X, TX, offX = _walks(rng, lens_x, dim)
        Y, TY, offY = _walks(rng, lens_y, dim) if lens_y is not None else (None, None, None)
        variants.append((X, TX, Y, TY))
    pl = None
    if n_pairs:
        pl = torch.as_tensor(np.stack([rng.integers(0, len(lens_x), n_pairs), rng.integers(0, len(lens_y), n_pairs)],
                                      axis=1).astype(np.int64), device="cuda")

    def eager(v):
        X, TX, Y, TY = v
        return tw.twed_batch(f(X), f(TX), offX, None if Y is None else f(Y), None if TY is None else f(TY),
                             offY, pairs=pl, **kw)

    say(f"batch plan {case}: eager results")
    want = [eager(v).cpu().numpy() for v in variants]
    other = synth.batch_collection(9, 5, 200, seed=77)
    oX, oT = to_dev(other, prec if prec == "f64" else "f32")
    other_want = tw.twed_batch(oX, oT, other.off, precision=prec).cpu().numpy()

    plan = tw.BatchPlan(offX, offY, n_pairs=n_pairs, dim=dim, nu=kw["nu"], lam=kw["lam"], p=kw["p"],
                        precision=prec)
    X0, TX0, Y0, TY0 = variants[0]
    bX, bTX = f(X0), f(TX0)
    bY, bTY = (f(Y0), f(TY0)) if Y0 is not None else (None, None)
    D = plan.output()
    say(f"batch plan {case}: eager run")
    plan.run(bX, bTX, bY, bTY, pairs=pl, D=D)
    torch.cuda.synchronize()
    assert np.array_equal(D.cpu().numpy(), want[0])
    g = torch.cuda.CUDAGraph()
    say(f"batch plan {case}: capture")
    with torch.cuda.graph(g):
        plan.run(bX, bTX, bY, bTY, pairs=pl, D=D)
    for i in range(1, 4):
        X, TX, Y, TY = variants[i]
        bX.copy_(f(X)); bTX.copy_(f(TX))
        if Y is not None:
            bY.copy_(f(Y)); bTY.copy_(f(TY))
        D.fill_(-1.0)
        say(f"batch plan {case}: replay {i}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(D.cpu().numpy(), want[i]), (case, i)
        o = tw.twed_batch(oX, oT, other.off, precision=prec).cpu().numpy()
        assert np.array_equal(o, other_want)
    plan.close()


@pytest.mark.parametrize("prec,dim,nq", [("f64", 28, 28), ("f32", 3, 150)])
def test_batch_plan_staged_collection(prec, dim, nq):
    """A collection staged once by the plan serves many queries: runs without
    Y (eager and replayed from a graph, with new query values each time) are
    bitwise the eager twed_batch result with Y passed; a run without Y before
    staging is refused on the host.  nq = 28: one short query (lane per pair);
    nq = 150: longer than a lane-mode query (wave per pair)."""
    rng = np.random.default_rng(90 + dim)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    lens_y = list(rng.integers(10, 60, 97))
    Y, TY, offY = _walks(rng, lens_y, dim)
    offX = np.array([0, nq], np.int64)
    queries = [_walks(rng, [nq], dim)[:2] for _ in range(4)]
    kw = dict(nu=0.01, lam=0.4, p=2.0, precision=prec)
    want = [tw.twed_batch(f(q), f(t), offX, f(Y), f(TY), offY, **kw).cpu().numpy() for q, t in queries]
    plan = tw.BatchPlan(offX, offY, dim=dim, nu=0.01, lam=0.4, p=2.0, precision=prec)
    bX, bTX = f(queries[0][0]), f(queries[0][1])
    D = plan.output()
    with pytest.raises(tw.TwedError):
        plan.run(bX, bTX, D=D)
    say(f"staged collection {prec} dim {dim}: stage and eager run")
    plan.stage_y(f(Y), f(TY))
    plan.run(bX, bTX, D=D)
    torch.cuda.synchronize()
    assert np.array_equal(D.cpu().numpy(), want[0])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(bX, bTX, D=D)
    for i in range(1, 4):
        bX.copy_(f(queries[i][0])); bTX.copy_(f(queries[i][1]))
        D.fill_(-1.0)
        say(f"staged collection {prec} dim {dim}: replay {i}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(D.cpu().numpy(), want[i]), i
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pair_list_with_long_series(prec):
    # Pair lists whose pairs hold two series longer than one wave's strip run
    # those pairs through the single-pair sweep: every entry equals twed_pair
    # bit for bit, short pairs stay in the batch kernel, invalid entries are NaN.
    rng = np.random.default_rng(21)
    lx, ly = [50, 1100, 2000, 700], [1500, 70, 1030, 4000]
    cx = synth.pack([synth.walk(rng, L, 1) for L in lx], [synth.irregular_times(rng, L) for L in lx])
    cy = synth.pack([synth.walk(rng, L, 1) for L in ly], [synth.irregular_times(rng, L) for L in ly])
    Xd, TXd = to_dev(cx, prec)
    Yd, TYd = to_dev(cy, prec)
    prs = [(1, 0), (2, 3), (0, 1), (3, 2), (1, 2), (-1, 0), (2, 0), (0, 3), (3, 9)]
    P = torch.as_tensor(np.array(prs, dtype=np.int64), device="cuda")
    say(f"pair list with long series {prec}: {len(prs)} pairs")
    D = tw.twed_batch(Xd, TXd, cx.off, Yd, TYd, cy.off, pairs=P, nu=1e-3, lam=1.0, p=1.0,
                      precision=prec).cpu().numpy()
    Xr, TXr = ref_inputs(cx, prec)
    Yr, TYr = ref_inputs(cy, prec)
    for k, (i, j) in enumerate(prs):
        if not (0 <= i < len(lx) and 0 <= j < len(ly)):
            assert np.isnan(D[k]), k
            continue
        a = slice(cx.off[i], cx.off[i + 1])
        b = slice(cy.off[j], cy.off[j + 1])
        one = tw.twed_pair(Xd[a], TXd[a], Yd[b], TYd[b], 1e-3, 1.0, 1.0, prec).item()
        assert D[k] == one, (k, D[k], one)
        ref = oracle.get().twed(Xr[a], TXr[a], Yr[b], TYr[b], 1e-3, 1.0, 1.0, rows=True)
        assert abs(D[k] - ref) <= TOL[prec] * ref, k


def test_batch_plan_tune_bitwise(tmp_path):
    # The autotuner's runs and the tuned plan's runs give the untuned matrix
    # bit for bit; the choice is cached under the plan's size class (a new plan
    # of that class picks it up) and survives a save / clear / load cycle.
    col = synth.batch_collection(300, 64, 1024, seed=31)
    X, T = to_dev(col, "f32")
    tw.twed_tune_clear()
    plan = tw.BatchPlan(col.off, precision="f32")
    assert plan.config() == (0, 0, -1)
    D0 = plan.run(X, T).clone()
    say("batch plan tune: 300 series")
    Dt = plan.output()
    choice = plan.tune(X, T, D=Dt)
    say(f"  tuned (chunk, waves/CU, lane mode) = {choice}")
    torch.cuda.synchronize()
    assert torch.equal(Dt, D0)
    assert plan.config() == choice
    D1 = plan.run(X, T)
    assert torch.equal(D1, D0)
    plan2 = tw.BatchPlan(col.off, precision="f32")
    assert plan2.config() == choice
    path = tmp_path / "tune.txt"
    tw.twed_tune_save(path)
    tw.twed_tune_clear()
    assert tw.BatchPlan(col.off, precision="f32").config() == (0, 0, -1)
    tw.twed_tune_load(path)
    plan3 = tw.BatchPlan(col.off, precision="f32")
    assert plan3.config() == choice
    assert torch.equal(plan3.run(X, T), D0)
    # a single short query: the lane mode is one of the candidates
    q = col.subset([5])
    qs = synth.pack([q.X[:20]], [q.T[:20]])
    Q, TQ = to_dev(qs, "f32")
    qplan = tw.BatchPlan(qs.off, col.off, precision="f32")
    R0 = qplan.run(Q, TQ, X, T).clone()
    qplan.tune(Q, TQ, X, T)
    assert torch.equal(qplan.run(Q, TQ, X, T), R0)
    for p in (plan, plan2, plan3, qplan):
        p.close()
    tw.twed_tune_clear()
