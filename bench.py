#!/usr/bin/env python3
"""Benchmark: TWED cell updates per second on one MI355X.

Headline workload: one pair of 8-D Gaussian random walks, n = m = 1,000,000
(regular timestamps, nu = 1e-3, lambda = 1, L2 point cost), FP32 inputs and
costs with FP64 accumulators, inputs resident in device memory.  One step is
one full twed_pair call (staging + the wavefront sweep, 10^12 cells).

Also reported (secondary, not the headline value): the same pair in FP64;
the 3-D n = 1e5 pair (FP64 and FP32); the batched all-pairs distance matrix
of 2,048 1-D FP32 walks with lengths uniform in [64, 1024]; one column shard,
an alignment path, LCS and DTW on the band sweep; one R^28 query against
60,000 series; the paper's own shapes; the learned k-NN search (1e5-series
database, 1e4 queries: recall@10 against exhaustive TWED, queries/s).

Printed: ONE JSON line with metric, value (GCUPS), timing, the roofline of the
dominant kernel (VALU-bound: the cell-rate ceiling of its operation mix at the
published FP32 / FP64 vector rates, with the fraction against the rates probed
on the device beside it) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Published vector rates of MI355X (256 CUs at 2.4 GHz): FP32 vector 157.3
# TFLOP/s and FP64 vector 78.6 TFLOP/s, i.e. 78.6 T and 39.3 T lane operations
# per second (an FMA is one lane operation, two flops).  Transcendentals (the
# FP32 square root) run at a quarter of the FP32 rate.  The FP64 square root
# (a reciprocal-root seed and refinement steps, thirteen instructions) is
# priced as one quarter-rate FP64 operation.  Every HIP file is compiled without
# packed FP32 instructions.
RATES_PUBLISHED = {"f32": 157.3 / 2, "f32_trans": 157.3 / 8, "f64": 78.6 / 2, "f64_sqrt": 78.6 / 8}

# Algorithmic VALU lane operations per DP cell, by rate class:
#   8-D L2 distance in f32: 8 sub + 1 mul + 7 fma, then the root (f32_trans);
#   time term: sub + fma (|.| is a free source modifier); f32 -> f64 convert;
#   f64 accumulators: match add, up + del_A, left + del_B, X add, two min
#   (there is no three-way f64 min).
MIX_8D_L2_ACC64 = {"f32": 18, "f32_trans": 1, "f64": 7}
#   1-D L1 in f32: value sub, time sub, fma, match add, two deletion adds,
#   one three-way min (v_min3_f32), X add.
MIX_1D_L1_F32 = {"f32": 8}
#   3-D L2 in f64: 3 sub + 1 mul + 2 fma, root, time sub + fma, 6 accumulator ops.
MIX_3D_L2_F64 = {"f64": 14, "f64_sqrt": 1}
#   3-D L2 in f32: 3 sub + 1 mul + 2 fma, root, time sub + fma, match add, two
#   deletion adds, one three-way min, X add.
MIX_3D_L2_F32 = {"f32": 13, "f32_trans": 1}
#   1-D L1 in f64: value sub, time sub, fma, 6 accumulator ops.
MIX_1D_L1_F64 = {"f64": 9}
#   28-D L2 in f64: 28 sub + 1 mul + 27 fma, root, time sub + fma, 6 accumulator ops.
MIX_28D_L2_F64 = {"f64": 64, "f64_sqrt": 1}


def mix_ops(mix):
    return sum(mix.values())


def ceiling_gcups(mix, rates):
    """Cell-rate ceiling (GCUPS) of a cell with this operation mix when every
    class issues at its rate (T lane-op/s) and the classes share the SIMDs."""
    ps_per_cell = sum(n / rates[k] for k, n in mix.items())  # chip-wide picoseconds per cell
    return 1e3 / ps_per_cell


def measured_rates(peaks):
    """Rates by class from the on-device probes (add / minimum chains for the
    plain classes, the square-root chain for f32_trans)."""
    return {"f32": peaks["f32_add_T_lane_op_s"], "f32_trans": peaks["f32_sqrt_T_lane_op_s"],
            "f64": peaks["f64_add_T_lane_op_s"], "f64_sqrt": peaks["f64_add_T_lane_op_s"] / 4}


def roofline_of(mix, gcups, peaks=None):
    """Roofline fields of a VALU-bound sweep measured at `gcups`."""
    ceil = ceiling_gcups(mix, RATES_PUBLISHED)
    ops = mix_ops(mix)
    out = {"bound": "alu", "achieved": round(ops * gcups / 1e3, 3), "peak": round(ops * ceil / 1e3, 3),
           "unit": "T VALU lane-op/s", "frac": round(gcups / ceil, 4), "ops_per_cell": dict(mix),
           "cell_rate_ceiling_GCUPS": round(ceil, 1)}
    if peaks:
        mceil = ceiling_gcups(mix, measured_rates(peaks))
        out["frac_of_measured_peak"] = round(gcups / mceil, 4)
        out["measured_cell_rate_ceiling_GCUPS"] = round(mceil, 1)
    return out


# The paper's single-pair timings (table "Raw Time to Solution", 1-D FP64,
# most likely a P100; cuTWED_dev = device-resident inputs), seconds by N.
PAPER_CUTWED_DEV_S = {1048576: 211.51, 524288: 54.084, 262144: 13.827, 131072: 3.6344, 65536: 0.8571,
                      32768: 0.2851, 16384: 0.1140, 8192: 0.0499, 4096: 0.0243, 2048: 0.0118, 1024: 0.0059}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(n, strip_k, kernel):
    """HBM-side bytes per launch of the headline sweep from the committed
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a copy of known size),
    or None when the sweep's sources changed since the counters were taken or
    the workload or kernel differs from the one profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wavefront_8d_n1e6_hbm_counters.md")
    if n != 1_000_000 or strip_k not in (0, 8) or not os.path.exists(path):
        return None
    traffic, ok = None, True
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1])
        elif line.startswith("kernel:"):
            ok &= line.split(":", 1)[1].strip() == kernel
        elif line.startswith("source_sha256 "):
            name, digest = line[len("source_sha256 "):].split(":", 1)
            src = os.path.join(ROOT, "paper_2007_16135_amd", "csrc", name.strip())
            ok &= os.path.exists(src) and hashlib.sha256(open(src, "rb").read()).hexdigest() == digest.strip()
    return traffic if ok else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000, help="series length of the headline pair")
    ap.add_argument("--strip-k", type=int, default=0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched all-pairs measurement")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--cpu-n", type=int, default=30000, help="prefix length of the CPU oracle sample")
    ap.add_argument("--no-rn", action="store_true", help="skip the R^28 single-query measurement")
    ap.add_argument("--no-tiles", action="store_true", help="skip the column-shard and alignment-path measurements")
    ap.add_argument("--rn-all", action="store_true", help="also time the 60000 x 60000 R^28 all-pairs matrix")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--no-knn", action="store_true", help="skip the learned k-NN measurement")
    ap.add_argument("--no-peaks", action="store_true", help="skip the on-device VALU / HBM rate probes")
    ap.add_argument("--no-c2", action="store_true", help="skip the 3-D n=1e5 pair")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run of the headline pair")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-shaped workloads")
    ap.add_argument("--cpu-pairs", type=int, default=20000,
                    help="pairs of the all-pairs batch timed on all host cores with the oracle")
    ap.add_argument("--knn-db", type=int, default=100_000, help="k-NN database size")
    ap.add_argument("--knn-queries", type=int, default=10_000, help="k-NN queries timed")
    ap.add_argument("--knn-truth", type=int, default=1000,
                    help="queries given exhaustive ground truth (recall sample)")
    ap.add_argument("--knn-train-steps", type=int, default=80000, help="training steps (2,048 pairs each)")
    ap.add_argument("--knn-schedule", choices=("cosine", "constant"), default="cosine",
                    help="learning-rate schedule of the embedding training")
    ap.add_argument("--knn-anchors", type=int, default=4096,
                    help="database series whose exact neighbours are mined for training")
    return ap.parse_args()


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) / 1e3 for a, b in ev]
    return wall, per


def measure_peaks(torch, dev):
    """Achievable VALU lane-operation rates (twed_probe_valu: eight independent
    chains per lane, FP32 / FP64 FMA and add+min) and the HBM rate of a plain
    device copy, measured on this GPU."""
    import ctypes
    from paper_2007_16135_amd import binding as Bd
    L = Bd.load_library()
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    waves = cus * 4 * 8  # eight waves per SIMD
    sink = torch.empty(waves * 64, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    out = {"compute_units": cus}
    names = {0: "f32_fma", 1: "f32_add_min", 2: "f64_fma", 3: "f64_add_min", 4: "f32_sqrt", 5: "f32_add",
             6: "f64_add", 7: "f32_min3"}
    for kind, name in names.items():
        iters = 30000 if kind in (1, 3) else 60000
        ops = ctypes.c_double()
        best = None
        for _ in range(4):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            Bd._check(L.twed_probe_valu(kind, waves, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ops),
                                         ctypes.c_void_p(stream.cuda_stream)))
            b.record(stream)
            b.synchronize()
            t = a.elapsed_time(b) / 1e3
            best = t if best is None else min(best, t)
        out[name + "_T_lane_op_s"] = round(ops.value / best / 1e12, 3)
    n = 1 << 30  # 4 GiB copy: read 4 GiB + write 4 GiB
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    out["hbm_copy_GB_s"] = round(2 * 4 * n / best / 1e9, 1)
    del src, dst, sink
    torch.cuda.empty_cache()
    out["published_T_lane_op_s"] = {k: round(v, 3) for k, v in RATES_PUBLISHED.items()}
    return out


def knn_bench(args, torch, tw, synth, dev, time_steps):
    from paper_2007_16135_amd import knn
    from paper_2007_16135_amd import binding as B
    nu, lam, k = 1e-3, 1.0, 10
    log(f"knn: generating database {args.knn_db} and {args.knn_queries} queries")
    db = synth.knn_collection(args.knn_db, 3)
    qs = synth.knn_collection(args.knn_queries, 4)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a.reshape(-1), dtype=np.float32), device=dev)
    DB, TDB, Q, TQ = f32(db.X), f32(db.T), f32(qs.X), f32(qs.T)
    dbc = knn.Collection(DB, TDB, db.off)

    tr = knn.Trainer(dbc, nu, lam, seed=0, batch_series=256, pairs_per_step=2048, n_anchors=args.knn_anchors)
    log(f"knn: exact neighbours of {args.knn_anchors} anchors mined in {tr.mine_s:.1f} s")
    train_s = tr.train(args.knn_train_steps, log_every=5000, log=log, schedule=args.knn_schedule)
    params = tr.params.clone()
    t0 = time.perf_counter()
    index = B.KnnIndex(DB, TDB, db.off, params, nu, lam)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"knn: trained {tr.pairs_seen} pairs in {train_s:.1f} s, index built in {build_s:.2f} s")

    # exhaustive ground truth on a sample of queries: FP32 TWED to every database series
    nt = min(args.knn_truth, args.knn_queries)
    qoff_t = qs.off[:nt + 1]
    Qt, TQt = Q[:qoff_t[-1]], TQ[:qoff_t[-1]]
    D = torch.empty((nt, args.knn_db), dtype=torch.float32, device=dev)
    ws = torch.empty(max(B.twed_batch_workspace_size(qoff_t, db.off, B.make_params(nu, lam, 1.0, 1, "f32")), 256),
                     dtype=torch.uint8, device=dev)
    exh_wall, _ = time_steps(lambda: B.twed_batch(Qt, TQt, qoff_t, DB, TDB, db.off, nu=nu, lam=lam, p=1.0,
                                                   precision="f32", D=D, workspace=ws), 1, 0, torch)
    Dn = D.cpu().numpy()
    del D, ws
    truth = np.argsort(Dn, axis=1, kind="stable")[:, :k]
    exh_qps = nt / exh_wall
    log(f"knn: exhaustive TWED for {nt} queries in {exh_wall:.2f} s ({exh_qps:.1f} q/s)")

    def recall(n_cand, net=params):
        ix = index if net is params else B.KnnIndex(DB, TDB, db.off, net, nu, lam)
        ids, _ = ix.query(Qt, TQt, qoff_t, k=k, n_cand=n_cand)
        r = knn.recall_at(ids.cpu().numpy(), truth)
        if ix is not index:
            ix.close()
        return r

    curve = {}
    chosen = None
    for c in (200, 400, 800, 1600, 3200, 4000, 4400, 4800, 5200, 5600, 6000, 6400, 7200, 8000, 9600, 11200, 12800, 16000,
              19200, 25600, 38400, 51200):
        c = min(c, args.knn_db)
        curve[c] = recall(c)
        log(f"knn: recall@10 with {c} candidates: {curve[c]:.4f}")
        if curve[c] >= 0.99 and chosen is None:
            chosen = c
            break
        if c == args.knn_db:
            break
    ablation = {"untrained_at_200": recall(200, torch.as_tensor(knn.init_params(0), device=dev)),
                "network_only": recall(k)}
    log(f"knn: ablations {ablation}")

    def qps(n_cand):
        ids = torch.empty((args.knn_queries, k), dtype=torch.int64, device=dev)
        dist = torch.empty((args.knn_queries, k), dtype=torch.float32, device=dev)
        wsq = torch.empty(max(index.workspace_size(qs.off, k, n_cand), 256), dtype=torch.uint8, device=dev)
        wall, _ = time_steps(lambda: index.query(Q, TQ, qs.off, k=k, n_cand=n_cand, ids=ids, dist=dist,
                                                 workspace=wsq), 2, 1, torch)
        return args.knn_queries * 2 / wall

    q200 = qps(200)
    out = {"workload": f"{args.knn_db} database / {args.knn_queries} query 1-D FP32 series, lengths U[128,512], "
                       f"half random walks, half noisy sinusoids of 8 classes; nu=1e-3, lambda=1, L1; k=10",
           "train_pairs_labelled": tr.pairs_seen, "train_steps": args.knn_train_steps,
           "mined_anchors": args.knn_anchors, "lr_schedule": args.knn_schedule,
           "mine_s": round(tr.mine_s, 2), "train_s": round(train_s, 2), "index_build_s": round(build_s, 3),
           "recall_sample_queries": nt, "recall_curve": {str(c): round(r, 4) for c, r in curve.items()},
           "recall@10_at_200": round(curve[200], 4), "queries_per_s_at_200": round(q200, 1),
           "exhaustive_queries_per_s": round(exh_qps, 1), "ablation_recall@10": {
               a: round(v, 4) for a, v in ablation.items()}}
    if chosen is not None:
        qc = q200 if chosen == 200 else qps(chosen)
        out.update({"n_cand_for_recall_0.99": chosen, "recall@10": round(curve[chosen], 4),
                    "queries_per_s": round(qc, 1), "speedup_vs_exhaustive": round(qc / exh_qps, 1)})
    else:
        out.update({"n_cand_for_recall_0.99": None, "recall@10": None, "queries_per_s": None})
    index.close()
    log(f"knn: {out}")
    return out


def c2_bench(torch, tw, synth, dev, peaks):
    """3-D walks n = m = 1e5 (seeds 2/3, irregular times, nu = 0.01,
    lambda = 0.5, L2): FP64 and FP32 runs, each against the FP64 oracle value
    of the same inputs (tests/golden/oracle_values.json, written by the oracle
    alone)."""
    gold = {c["name"]: c["value"] for c in json.load(open(os.path.join(ROOT, "tests", "golden",
                                                                       "oracle_values.json")))["cases"]}
    c = synth.single_pair_3d(100_000)
    n = 100_000
    cells = float(n) * n
    out = {"workload": "single pair, 3-D random walks n=m=100000, irregular Exp(1) timestamps, nu=0.01, "
                       "lambda=0.5, L2", "cells_per_step": cells}
    for prec, key, mix, gname in (("f64", "fp64", MIX_3D_L2_F64, "walk3d_n100000"),
                                  ("f32", "fp32", MIX_3D_L2_F32, "walk3d_n100000_f32")):
        dt = torch.float64 if prec == "f64" else torch.float32
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        A, TA, B, TB = t(c.A), t(c.TA), t(c.B), t(c.TB)
        prm = tw.make_params(c.nu, c.lam, c.p, 3, prec)
        ws = torch.empty(max(tw.twed_pair_workspace_size(n, n, prm), 256), dtype=torch.uint8, device=dev)
        res = torch.empty(1, dtype=torch.float64 if prec == "f64" else torch.float32, device=dev)
        wall, per = time_steps(lambda: tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, prec, out=res, workspace=ws),
                               5, 2, torch)
        k = float(np.median(per))
        v = float(res.item())
        entry = {"ms": round(k * 1e3, 3), "GCUPS": round(cells / k / 1e9, 3), "result": v,
                 "oracle": gold[gname], "rel_err_vs_oracle": abs(v - gold[gname]) / gold[gname],
                 "roofline": roofline_of(mix, cells / k / 1e9, peaks)}
        out[key] = entry
        del A, TA, B, TB, ws
    log(f"pair 3d n=1e5: {out}")
    return out


def batch_checks(torch, tw, col, X, T, D, dev, samples=256):
    """The timed FP32 matrix against the FP64 oracle on sampled entries, and
    an FP64 GPU run of the same batch (inputs: the FP32 values widened)
    against which every FP32 entry's error is stated."""
    import oracle
    n = col.count
    Dh = D.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(99)
    i = rng.integers(0, n, samples)
    j = rng.integers(0, n - 1, samples)
    j = j + (j >= i)
    X64 = col.X.astype(np.float32).astype(np.float64)
    T64 = col.T.astype(np.float32).astype(np.float64)
    ref = oracle.get().pairs(X64, T64, col.off, X64, T64, col.off, np.stack([i, j], 1), 1e-3, 1.0, 1.0)
    got = Dh[i, j]
    X64d = torch.as_tensor(X64, device=dev)
    T64d = torch.as_tensor(T64, device=dev)
    D64 = tw.twed_batch(X64d, T64d, col.off, nu=1e-3, lam=1.0, p=1.0, precision="f64")
    torch.cuda.synchronize()
    D64h = D64.cpu().numpy()
    off_diag = ~np.eye(n, dtype=bool)
    rel = np.abs(Dh - D64h)[off_diag] / np.abs(D64h)[off_diag]
    out = {"timed_output_vs_oracle": {"samples": samples, "max_rel_err": float(np.max(np.abs(got - ref) / ref))},
           "fp64_gpu_vs_oracle_max_rel_err": float(np.max(np.abs(D64h[i, j] - ref) / ref)),
           "fp32_vs_fp64_gpu_rel_err": {"max": float(rel.max()), "mean": float(rel.mean())}}
    del D64, X64d, T64d
    return out


def paper_shapes(torch, tw, synth, dev, peaks=None):
    """1-D FP64 workloads of the paper's tables: single pairs of random walks
    N = 2^10 .. 2^20 (the C1 generator, seeds 0/1, t = 0..N-1, nu = 1e-3,
    lambda = 1, L1) next to the paper's device-resident timings (table "Raw
    Time to Solution", other hardware); all-pairs of 600 series of 60 and of
    10 series of 1e5 (table "Timings From Validation Exercises" shapes, seeded
    walks standing in for the UCI data)."""
    out = {"single_pairs": {}}
    f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    big = synth.single_pair_1d(1 << 20)
    for e in range(10, 21):
        N = 1 << e
        A, TA, B, TB = f64(big.A[:N]), f64(big.TA[:N]), f64(big.B[:N]), f64(big.TB[:N])
        res = torch.empty(1, dtype=torch.float64, device=dev)
        ws = torch.empty(max(tw.twed_pair_workspace_size(N, N, tw.make_params(1e-3, 1.0, 1.0, 1, "f64")), 256),
                         dtype=torch.uint8, device=dev)
        reps = 5 if N <= (1 << 16) else 2
        _, per = time_steps(lambda: tw.twed_pair(A, TA, B, TB, 1e-3, 1.0, 1.0, "f64", out=res, workspace=ws),
                            reps, 1, torch)
        k = float(np.median(per))
        out["single_pairs"][str(N)] = {"ms": round(k * 1e3, 4), "GCUPS": round(float(N) * N / k / 1e9, 3),
                                       "paper_gpu_s": PAPER_CUTWED_DEV_S[N],
                                       "speedup_vs_paper_gpu": round(PAPER_CUTWED_DEV_S[N] / k, 1)}
    # (N = 2^20 also gives the 1-D FP64 roofline fraction)
    k20 = out["single_pairs"][str(1 << 20)]["ms"] / 1e3
    out["single_pairs_2^20_roofline"] = roofline_of(MIX_1D_L1_F64, float(1 << 40) / k20 / 1e9, peaks)
    for count, length, paper_s, name in ((600, 60, 1.0, "600x60"), (10, 100_000, 147.0, "10x100k")):
        col = synth.paper_shaped_collection(count, length)
        X, T = f64(col.X), f64(col.T)
        D = torch.empty((count, count), dtype=torch.float64, device=dev)
        ws = torch.empty(max(tw.twed_batch_workspace_size(col.off, None, tw.make_params(1e-3, 1.0, 1.0, 1, "f64")),
                             256), dtype=torch.uint8, device=dev)
        _, per = time_steps(lambda: tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision="f64", D=D,
                                                  workspace=ws), 3, 1, torch)
        k = float(np.median(per))
        cells = float(length) * length * count * (count - 1) / 2
        out[name] = {"ms": round(k * 1e3, 4), "GCUPS": round(cells / k / 1e9, 3),
                     "paper_gpu_s": paper_s, "speedup_vs_paper_gpu": round(paper_s / k, 1),
                     "note": "upper triangle swept; the paper's GPU run filled the full matrix"}
    log(f"paper shapes: {out}")
    return out


def cpu_all_cores(pairs, synth):
    """The oracle (FP64, one thread per pair) on a sample of the 2048-series
    all-pairs batch, spread over every host core."""
    import oracle
    col = synth.batch_collection(2048, 64, 1024)
    rng = np.random.default_rng(5)
    i = rng.integers(0, 2048, pairs)
    j = rng.integers(0, 2047, pairs)
    j = j + (j >= i)
    X64 = col.X.astype(np.float32).astype(np.float64)
    T64 = col.T.astype(np.float32).astype(np.float64)
    L = col.lengths
    cells = float(np.sum(L[i].astype(np.float64) * L[j]))
    cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    oracle.get().pairs(X64, T64, col.off, X64, T64, col.off, np.stack([i, j], 1), 1e-3, 1.0, 1.0, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "sample": f"{pairs} random pairs of the 2048-series all-pairs batch ({cells:.3g} cells, {dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the library has no "
                                   "multi-GPU path (column shards are swept one GPU at a time)", "n_gpus": args.gpus}))
        return 2

    import torch
    import paper_2007_16135_amd as tw
    from paper_2007_16135_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    tw.load_library()
    if args.calib_bytes > 0:
        # a plain copy of known size: rocprofv3's FETCH_SIZE / WRITE_SIZE for
        # this dispatch calibrate the counters read for the sweep kernel
        src = torch.ones(args.calib_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    peaks = None
    if not args.no_peaks:
        peaks = measure_peaks(torch, dev)
        log(f"peaks: {peaks}")

    # ---- headline: one 8-D pair, n = m = 1e6, FP32 costs + FP64 accumulators
    n = args.n
    log(f"generating 8-D walks n={n}")
    c = synth.single_pair_8d(n)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
    A, TA, B, TB = f32(c.A), f32(c.TA), f32(c.B), f32(c.TB)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    prm = tw.make_params(c.nu, c.lam, c.p, 8, "f32_acc64", strip_k=args.strip_k)
    ws = torch.empty(max(tw.twed_pair_workspace_size(n, n, prm), 256), dtype=torch.uint8, device=dev)

    def step():
        tw.twed_pair(A, TA, B, TB, c.nu, c.lam, c.p, "f32_acc64", strip_k=args.strip_k, out=out,
                     workspace=ws)

    log(f"headline: warmup {args.warmup}, steps {args.steps}")
    wall, per = time_steps(step, args.steps, args.warmup, torch)
    value = float(out.item())
    cells = float(n) * float(n)
    ms_step = wall / args.steps * 1e3
    gcups = cells * args.steps / wall / 1e9
    kern_s = float(np.mean(per))
    log(f"headline: {ms_step:.1f} ms/step, {gcups:.1f} GCUPS, value {value!r}")

    result = {
        "metric": "TWED GCUPS (1 pair n=1e6; batched all-pairs) + k-NN queries/s at recall@10>=0.99",
        "value": round(gcups, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 costs / f64 accumulators",
        "data": "synthetic (seeded Gaussian random walks)",
        "config": {"workload": f"single pair, 8-D random walks n=m={n}, regular timestamps, nu=1e-3, "
                               f"lambda=1, L2, FP32 costs + FP64 accumulators",
                   "cells_per_step": cells, "result": value},
        "roofline": roofline_of(MIX_8D_L2_ACC64, cells / kern_s / 1e9, peaks),
    }
    plan = tw.twed_pair_config(n, n, 8, c.nu, c.lam, c.p, "f32_acc64", strip_k=args.strip_k)
    if plan["wide_strips"] > 0:
        kname = "wavefront_mixed_kernel<float,double,8,L2,%d,%d,%d>" % (plan["strip_k"], plan["strip_k"] - 1,
                                                                          plan["group"])
    else:
        kname = "wavefront_kernel<float,double,8,L2,%d,%d>" % (plan["strip_k"], plan["group"])
    result["config"]["strips"] = plan
    result["roofline"].update({"traffic": counter_traffic(n, args.strip_k, kname),
                               "kernel": kname, "kernel_avg_s": kern_s})
    if peaks:
        result["measured_peaks"] = peaks

    # ---- the same pair in FP64 on the GPU (inputs: the FP32 values widened),
    # and the mixed-precision result's error against it
    if not args.no_fp64:
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32), dtype=np.float64), device=dev)
        A64, TA64, B64, TB64 = f64(c.A), f64(c.TA), f64(c.B), f64(c.TB)
        out64 = torch.empty(1, dtype=torch.float64, device=dev)
        ws64 = torch.empty(max(tw.twed_pair_workspace_size(n, n, tw.make_params(c.nu, c.lam, c.p, 8, "f64")), 256),
                           dtype=torch.uint8, device=dev)
        w64, p64 = time_steps(lambda: tw.twed_pair(A64, TA64, B64, TB64, c.nu, c.lam, c.p, "f64", out=out64,
                                                   workspace=ws64), 1, 0, torch)
        v64 = float(out64.item())
        result["headline_fp64"] = {
            "workload": "the headline pair in FP64 (inputs, costs and accumulators; the FP32 inputs widened)",
            "result": v64, "ms": round(p64[0] * 1e3, 3), "GCUPS": round(cells / p64[0] / 1e9, 3),
            "mixed_vs_fp64_rel_err": abs(value - v64) / abs(v64)}
        log(f"headline fp64: {result['headline_fp64']}")
        del A64, TA64, B64, TB64, ws64

    # ---- the 3-D pair n = m = 1e5 (irregular times, L2), FP64 and FP32,
    # against the stored oracle values
    if not args.no_c2:
        result["pair_3d_n1e5"] = c2_bench(torch, tw, synth, dev, peaks)

    # ---- secondary: batched all-pairs, 2048 1-D FP32 series
    if not args.no_batch:
        log("generating batch collection 2048 x [64, 1024]")
        col = synth.batch_collection(2048, 64, 1024)
        X = torch.as_tensor(col.X.astype(np.float32), device=dev)
        T = torch.as_tensor(col.T.astype(np.float32), device=dev)
        L = col.lengths.astype(np.float64)
        bcells = float((L.sum() ** 2 - (L ** 2).sum()) / 2)
        D = torch.empty((2048, 2048), dtype=torch.float32, device=dev)
        bprm = tw.make_params(1e-3, 1.0, 1.0, 1, "f32")
        bws = torch.empty(max(tw.twed_batch_workspace_size(col.off, None, bprm), 256), dtype=torch.uint8,
                          device=dev)

        def bstep():
            tw.twed_batch(X, T, col.off, nu=1e-3, lam=1.0, p=1.0, precision="f32", D=D, workspace=bws)

        bwall, bper = time_steps(bstep, max(args.steps, 3), 1, torch)
        bk = float(np.mean(bper))
        result["batched_all_pairs"] = {
            "workload": "2048 1-D FP32 walks, lengths U[64,1024], irregular Exp(1) times, nu=1e-3, "
                        "lambda=1, L1; symmetric matrix (upper triangle swept)",
            "cells_per_step": bcells, "ms_per_step": round(bwall / max(args.steps, 3) * 1e3, 3),
            "GCUPS": round(bcells / bk / 1e9, 3),
            "roofline": roofline_of(MIX_1D_L1_F32, bcells / bk / 1e9, peaks),
        }
        result["batched_all_pairs"].update(batch_checks(torch, tw, col, X, T, D, dev))
        # the same batch as a plan, before and after the autotuner
        plan = tw.BatchPlan(col.off, precision="f32", device=dev)
        _, dper = time_steps(lambda: plan.run(X, T, D=D), 3, 1, torch)
        choice = plan.tune(X, T, D=D)
        _, tper = time_steps(lambda: plan.run(X, T, D=D), 3, 1, torch)
        plan.close()
        result["batched_all_pairs"]["autotuned"] = {
            "choice_chunk_waves_per_cu_lane_mode": list(choice),
            "plan_default_ms": round(float(np.median(dper)) * 1e3, 3),
            "plan_tuned_ms": round(float(np.median(tper)) * 1e3, 3),
            "tuned_GCUPS": round(bcells / float(np.median(tper)) / 1e9, 3)}
        log(f"batch: {result['batched_all_pairs']}")
        del D, bws

    # ---- one GPU's share of a column-sharded sweep, and the alignment path
    if not args.no_tiles:
        shard = 125_000
        if n >= 2 * shard:
            def tstep(c0):
                left = None if c0 == 0 else shard_right
                return tw.twed_pair_tile(A, TA, B, TB, 0, n, c0, c0 + shard, None, left, c.nu, c.lam, c.p,
                                         "f32_acc64", bottom=False)
            _, _, shard_right = tstep(0)
            twall, tper = time_steps(lambda: tstep(shard), max(args.steps, 3), 1, torch)
            tk = float(np.mean(tper))
            result["column_shard"] = {
                "workload": f"rows 1..{n} x columns {shard + 1}..{2 * shard} of the headline pair (one of eight "
                            f"column shards): left boundary column in, right boundary column out",
                "ms_per_step": round(tk * 1e3, 3), "GCUPS": round(float(n) * shard / tk / 1e9, 3)}
            log(f"column shard: {result['column_shard']}")
        pn = min(n, 100_000)
        pc = c.prefix(pn)
        pA, pTA, pB, pTB = f32(pc.A), f32(pc.TA), f32(pc.B), f32(pc.TB)
        pprm = tw.make_params(c.nu, c.lam, c.p, 8, "f32_acc64")
        pws = torch.empty(max(tw.binding.twed_pair_path_workspace_size(pn, pn, pprm), 256), dtype=torch.uint8,
                          device=dev)
        _, path = tw.twed_pair_path(pA, pTA, pB, pTB, c.nu, c.lam, c.p, "f32_acc64", workspace=pws)
        pwall, _ = time_steps(lambda: tw.twed_pair_path(pA, pTA, pB, pTB, c.nu, c.lam, c.p, "f32_acc64",
                                                        workspace=pws), 2, 0, torch)
        result["alignment_path"] = {
            "workload": f"8-D pair n=m={pn} (prefix of the headline pair), FP32 costs + FP64 accumulators, "
                        f"blocks of 4096",
            "s_per_path": round(pwall / 2, 4), "path_cells": int(path.shape[0]),
            "forward_GCUPS_equiv": round(float(pn) * pn / (pwall / 2) / 1e9, 3)}
        log(f"path: {result['alignment_path']}")

    # ---- sibling programs on the band sweep: LCS of 1e6-token sequences, 8-D DTW
    if not args.no_tiles:
        rng = np.random.default_rng(7)
        la = torch.as_tensor(rng.integers(0, 4, n).astype(np.float32), device=dev)
        lb = torch.as_tensor(rng.integers(0, 4, n).astype(np.float32), device=dev)
        lws = torch.empty(max(tw.binding.twed_dp_workspace_size("lcs", n, n,
                                                               tw.make_params(0.0, 0.0, 1.0, 1, "f32_acc64")), 256),
                          dtype=torch.uint8, device=dev)
        lwall, lper = time_steps(lambda: tw.twed_dp("lcs", la, lb, precision="f32_acc64", workspace=lws), 2, 1,
                                 torch)
        lk = float(np.mean(lper))
        dn = min(n, 250_000)
        dA, dB = A[:dn].contiguous(), B[:dn].contiguous()
        dwall, dper = time_steps(lambda: tw.twed_dp("dtw", dA, dB, p=2.0, precision="f32_acc64"), 2, 1, torch)
        dk = float(np.mean(dper))
        result["siblings"] = {
            "lcs": {"workload": f"LCS length of two {n}-token sequences (alphabet of 4, seed 7), FP32 tokens, "
                                f"FP64 accumulators", "ms": round(lk * 1e3, 3),
                    "GCUPS": round(float(n) * n / lk / 1e9, 3)},
            "dtw": {"workload": f"DTW of the first {dn} samples of the headline pair (8-D, L2), FP32 costs, "
                                f"FP64 accumulators", "ms": round(dk * 1e3, 3),
                    "GCUPS": round(float(dn) * dn / dk / 1e9, 3)},
        }
        log(f"siblings: {result['siblings']}")

    # ---- R^28: one query against 60,000 series of 28 samples in R^28 (FP64, L2)
    if not args.no_rn:
        log("generating 60000 x 28 series in R^28")
        rcol = synth.paper_shaped_rn(60000, 28, 28)
        rq = rcol.subset([0])
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
        QX, QT, RX, RT = f64(rq.X), f64(rq.T), f64(rcol.X), f64(rcol.T)
        rprm = tw.make_params(1e-3, 1.0, 2.0, 28, "f64")
        rD = torch.empty((1, rcol.count), dtype=torch.float64, device=dev)
        rws = torch.empty(max(tw.twed_batch_workspace_size(rq.off, rcol.off, rprm), 256), dtype=torch.uint8,
                          device=dev)

        def rstep():
            tw.twed_batch(QX, QT, rq.off, RX, RT, rcol.off, nu=1e-3, lam=1.0, p=2.0, precision="f64", D=rD,
                          workspace=rws)

        rsteps = max(args.steps, 10)
        rwall, rper = time_steps(rstep, rsteps, 2, torch)
        rcells = 28.0 * 28.0 * rcol.count
        # the same query through a batch plan whose collection was packed once
        # (a fixed collection queried repeatedly): per query, the query's
        # staging and the sweep
        rplan = tw.BatchPlan(rq.off, rcol.off, dim=28, nu=1e-3, lam=1.0, p=2.0, precision="f64", device=dev)
        rplan.stage_y(RX, RT)
        pwall, pper = time_steps(lambda: rplan.run(QX, QT, D=rD), rsteps, 2, torch)
        rplan.close()
        result["rn_query"] = {
            "workload": "1 query x 60000 series, 28 samples in R^28 each (seeded Gaussian walks standing in "
                        "for unravelled 28x28 images), regular times, nu=1e-3, lambda=1, L2, FP64",
            "ms_per_query": round(rwall / rsteps * 1e3, 4),
            "kernel_ms": round(float(np.mean(rper)) * 1e3, 4),
            "GCUPS": round(rcells / float(np.mean(rper)) / 1e9, 3),
            "ms_per_query_collection_staged_once": round(float(np.mean(pper)) * 1e3, 4),
            "GCUPS_collection_staged_once": round(rcells / float(np.mean(pper)) / 1e9, 3),
            "paper_gpu_s": 0.20,
            "roofline_staged_once": roofline_of(MIX_28D_L2_F64, rcells / float(np.mean(pper)) / 1e9, peaks),
        }
        log(f"rn query: {result['rn_query']}")
        if args.rn_all:
            # the full 60000 x 60000 symmetric matrix (28.8 GB of FP64 output)
            aD = torch.empty((rcol.count, rcol.count), dtype=torch.float64, device=dev)
            aws = torch.empty(max(tw.twed_batch_workspace_size(rcol.off, None, rprm), 256),
                              dtype=torch.uint8, device=dev)
            log("rn all-pairs 60000 x 60000")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tw.twed_batch(RX, RT, rcol.off, nu=1e-3, lam=1.0, p=2.0, precision="f64", D=aD, workspace=aws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            acells = 28.0 * 28.0 * rcol.count * (rcol.count - 1) / 2
            result["rn_all_pairs"] = {"workload": "60000 x 60000 symmetric matrix of the same collection "
                                                  "(upper triangle swept)",
                                      "seconds": round(dt, 3), "GCUPS": round(acells / dt / 1e9, 3)}
            log(f"rn all-pairs: {result['rn_all_pairs']}")
            del aD, aws

    # ---- the paper's own shapes (1-D FP64): single pairs N = 2^10 .. 2^20,
    # 600 x 60 and 10 x 100k all-pairs
    if not args.no_paper:
        result["paper_shapes"] = paper_shapes(torch, tw, synth, dev, peaks)

    # ---- learned k-NN: train, index, query; recall against exhaustive TWED
    if not args.no_knn:
        result["knn"] = knn_bench(args, torch, tw, synth, dev, time_steps)

    # ---- CPU oracle on a bounded sample (prefix of the headline pair)
    if not args.no_cpu:
        import oracle
        m = min(args.cpu_n, n)
        pc = c.prefix(m).astype(np.float32).astype(np.float64)
        log(f"cpu oracle on the {m}x{m} prefix")
        t0 = time.perf_counter()
        oracle.get().twed(pc.A, pc.TA, pc.B, pc.TB, pc.nu, pc.lam, pc.p, rows=True)
        dt = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(m * m / dt / 1e9, 5), "unit": "GCUPS", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"{m}x{m} prefix of the headline pair (FP64 oracle, two-row "
                                            f"form, one thread; {dt:.1f} s)"}
        if args.cpu_pairs > 0:
            result["cpu_all_cores"] = cpu_all_cores(args.cpu_pairs, synth)
            log(f"cpu all cores: {result['cpu_all_cores']}")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
