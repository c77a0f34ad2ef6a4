"""Benchmark: symmetric ACT top-l search of a query batch against a resident
text-shaped histogram database on one MI355X.

One step = one lcemd_topl call on the whole batch (query staging, phase-1
distance GEMM + ordered extraction, phase-2 transfers, Q2D for the pruned
candidates, symmetric max, top-l), with the database and the query batch
already resident in HBM.

Workload (synthetic, seeded; stands in for 20 Newsgroups with 300-d word
vectors, which is not available here): vocabulary 70,000 x 300 unit-norm
Gaussian embeddings, 18,000 database histograms and 1,000 queries of 50-300
distinct Zipf(1.0) words (log-normal lengths, mean ~120), tf weights.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {"fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--method", default="act")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--ell", type=int, default=16)
    ap.add_argument("--direction", default="sym")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--workload", default="text")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--B", type=int, default=None)
    ap.add_argument("--cpu-queries", type=int, default=2, help="queries in the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the bf16-path comparison")
    ap.add_argument("--no-big", action="store_true", help="skip the 1M-word precision and serving section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--big-queries", type=int, default=4096, help="queries of the 1M-word precision run")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="offered load, queries/s")
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--serve-sat", type=int, default=256, help="queries in the saturation sample")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-budget", type=int, default=8, help="GiB of device memory for lanes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def phase1_kernel(method, k, precision, m):
    """The phase-1 kernel the library picks for the table (D2Q) pass of
    queries against m-dimensional embeddings."""
    depth = {"rwmd": 1, "omr": 2, "act": k, "ict": 64}[method]
    margin = 0 if precision == "fp32" or depth + 8 > 32 else 8
    kl = 2
    while kl < depth + margin:
        kl *= 2
    prec = 0 if margin == 0 else 1
    if prec == 0 and (m + 3) // 4 <= 7 and depth <= 64 and method != "ict":  # float32, at most 28 dims: 64-row kernel
        return f"k_phase1_fast<0, {kl}, 0>"
    if depth + margin <= 32:
        return f"k_phase1_wide<0, {kl}, {prec}, false>"
    return "k_phase1_fast<0, 64, 0>" if depth <= 64 else "k_phase1_f32"


def measured_traffic(kernel, a):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary of this workload, if it was taken on the current kernel source
    (its sha256 is recorded with it); otherwise None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1812_02091_amd", "csrc", "phase1_wide.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    key = f"{a.workload}:{a.method}:{a.k}:{a.direction}:{a.precision}"
    e = rec.get(key)
    if not e or e.get("source_sha256") != digest or e.get("kernel") != kernel:
        return None
    return e["bytes_per_launch"]


def copy_calibration():
    """A plain device-to-device copy of known size: its FETCH_SIZE and
    WRITE_SIZE counters convert the counters of the real kernels to bytes."""
    import torch

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": nbytes, "launches": 3}))


_ORC = None


def _oracle_init(V, ptr, col, val):
    global _ORC
    from oracle import emd_oracle as O

    _ORC = O.Oracle(V, ptr, col, val)


def _oracle_task(args):
    """One query of the CPU baseline: the oracle's symmetric distances to every
    database row, then its top-l (what one GPU step computes per query)."""
    qc, qw, method, k, ell = args
    t0 = time.time()
    row = _ORC.row_distances(qc, qw, method, k, "sym")
    _ORC.top_l(row, ell)
    return row.shape[0], time.time() - t0, row


def cpu_baseline(w, method, k, ell, nq):
    import multiprocessing as mp

    cores = max(1, min(16, os.cpu_count() or 1, nq))
    tasks = [(*w.queries.row(b), method, k, ell) for b in range(nq)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_oracle_init,
                  initargs=(w.V, w.db.rowptr, w.db.col, w.db.val)) as pool:
        res = pool.map(_oracle_task, tasks, chunksize=1)
    pairs = sum(r[0] for r in res)
    # per-worker compute time (excludes process start-up); queries run in parallel
    dt = max(sum(r[1] for r in res) / cores, max(r[1] for r in res))
    rec = {"value": pairs / dt, "unit": "distances/s", "cores": cores, "kind": "oracle",
           "sample": f"{nq} queries x all {w.db.n} database rows, {method.upper()} k={k} symmetric "
                     f"+ top-{ell}, float64 numpy/scipy, {cores} worker processes, {dt:.1f} s of oracle time per worker"}
    return rec, [r[2] for r in res]


def oracle_error(ctx, w, nq, rows, method, k, precision):
    """Relative error of the library's symmetric distances (first nq
    queries, every database row) against the float64 oracle rows."""
    import numpy as np

    q = w.queries.take(list(range(nq)))
    g = ctx.distances(q.rowptr, q.col, q.val, method=method, k=k, direction="sym", precision=precision)
    o = np.stack(rows)
    rel = np.abs(g.astype(np.float64) - o) / np.maximum(np.abs(o), 1e-30)
    rel[o == 0] = np.where(g[o == 0] == 0, 0.0, np.inf)
    return {"max_rel_err_vs_fp64_oracle": float(rel.max()), "median_rel_err_vs_fp64_oracle": float(np.median(rel)),
            "pairs": int(rel.size)}


def image_section(a, lcemd):
    """Image-shaped dense histograms (28x28 grid, 60,000 database and 10,000
    query blobs; m = 2): symmetric ACT top-16 for the whole query batch."""
    import numpy as np

    from synth import make_workload

    w = make_workload("image")
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
    B, n = w.queries.n, w.db.n
    q = w.queries
    small = q.take(list(range(8)))
    res = {"workload": f"image: 784 pixels x 2 coordinates, {n} database and {B} query histograms "
                       f"({w.db.nnz} database non-zeros), symmetric top-16",
           "paper_context": {"distances_per_s": 1.8e7, "hardware": "GTX 1080Ti (top-l on an 8-core CPU)",
                             "workload": "MNIST 60,000 x 60,000 all pairs, ACT with one phase-2 iteration "
                                         "(k=2 here), symmetric (Sec. 5)"}}
    for k in (2, 16):
        ctx.topl(small.rowptr, small.col, small.val, 16, method="act", k=k, direction="sym")
        ctx.profile(True)
        t1 = time.perf_counter()
        ctx.topl(q.rowptr, q.col, q.val, 16, method="act", k=k, direction="sym")
        dt = time.perf_counter() - t1
        ph = {p["name"]: p for p in ctx.profile_get()}
        ctx.profile(False)
        rec = {"distances_per_s": B * n / dt, "s_per_batch": dt,
               "phase_ms": {k2: v["ms"] for k2, v in ph.items()}}
        if "phase2" in ph and ph["phase2"]["ms"] > 0:
            gbs = ph["phase2"]["work"] / (ph["phase2"]["ms"] * 1e-3) / 1e9
            rec["phase2_algorithmic_GBps"] = gbs
            rec["phase2_hbm_frac"] = gbs * 1e9 / HBM_PEAK
        res[f"act{k}"] = rec
        print(f"[bench] image ACT k={k}: {dt:.3f} s", file=sys.stderr, flush=True)
    # the full symmetric matrix (the reverse direction by the swapped-role
    # linear method), device-resident queries and output
    import torch

    dev = torch.device("cuda:0")
    qd = [torch.from_numpy(x).to(dev) for x in (q.rowptr, q.col, q.val)]
    D = ctx.distances(*qd, method="act", k=2, direction="sym")  # scratch and output allocated once
    ctx.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.distances(*qd, method="act", k=2, direction="sym", out=D)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    ph = {p["name"]: p["ms"] for p in ctx.profile_get()}
    ctx.profile(False)
    res["full_sym_matrix_act2"] = {"shape": list(D.shape), "seconds": dt, "distances_per_s": B * n / dt,
                                   "phase_ms": ph}
    del D
    print(f"[bench] image full SYM matrix ACT k=2: {dt:.3f} s", file=sys.stderr, flush=True)
    ctx.close()
    return res


def measures_section(a, lcemd):
    """The paper's other measures on the text and image workloads (symmetric
    top-16 over the whole query batch, device-resident queries): RWMD, OMR
    (Alg. 1), ACT k=4 and ICT (Alg. 2), next to the headline ACT k=16."""
    import torch

    from synth import make_workload

    dev = torch.device("cuda:0")
    res = {}
    for name in ("text", "image"):
        w = make_workload(name)
        ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
        qs = w.queries
        q = [torch.from_numpy(x).to(dev) for x in (qs.rowptr, qs.col, qs.val)]
        small = qs.take([0, 1])
        out = {}
        for method, k in (("rwmd", 1), ("omr", 1), ("act", 4), ("ict", 1)):
            ctx.topl(small.rowptr, small.col, small.val, 16, method=method, k=k, direction="sym")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.topl(*q, 16, method=method, k=k, direction="sym")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            out[f"{method}{k}" if method == "act" else method] = {"seconds": dt,
                                                                   "distances_per_s": qs.n * w.db.n / dt}
            print(f"[bench] {name} {method} k={k}: {dt:.3f} s", file=sys.stderr, flush=True)
        # one direction (D2Q), RWMD against ACT with one phase-2 iteration
        # (k=2): Sec. 5 compares their costs (phase 1 dominates at m = 300,
        # phase 2 at m = 2)
        d2q = {}
        for method, k in (("rwmd", 1), ("act", 2)):
            ctx.topl(small.rowptr, small.col, small.val, 16, method=method, k=k, direction="d2q")
            ctx.profile(True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.topl(*q, 16, method=method, k=k, direction="d2q")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            ph = {p["name"]: p["ms"] for p in ctx.profile_get()}
            ctx.profile(False)
            d2q[f"{method}{k}" if method == "act" else method] = {"seconds": dt, "phase_ms": ph}
        d2q["act2_over_rwmd"] = d2q["act2"]["seconds"] / d2q["rwmd"]["seconds"]
        res[name] = {"queries": qs.n, "database": w.db.n, "sym_top16": out, "d2q_top16": d2q}
        ctx.close()
    return res


def selfjoin_section(a, lcemd):
    """All-pairs protocol of Sec. 5 at the MNIST training-set shape: every one
    of 60,000 image histograms against all 60,000 (itself excluded), ACT
    k=2 symmetric, top-16 neighbours per histogram, one lcemd_selfjoin_topl."""
    from synth import make_workload

    w = make_workload("image", B=8)
    n = w.db.n
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
    res = {"workload": f"image self-join: {n} histograms on the 28x28 grid ({w.db.nnz} non-zeros), "
                       f"all {n}x{n} pairs, ACT k=2 symmetric, top-16 per histogram",
           "paper_context": {"seconds": 3.3 * 60, "distances_per_s": 3.6e9 / (3.3 * 60),
                             "hardware": "GTX 1080Ti",
                             "workload": "MNIST 60,000 training images, all pairs, ACT-1 (Sec. 5)"}}
    small = lcemd.open_context(w.V, w.db.rowptr[:65], w.db.col[:w.db.rowptr[64]], w.db.val[:w.db.rowptr[64]],
                               device=0)
    small.selfjoin_topl(16, method="act", k=2, direction="sym")  # loads kernels
    small.close()
    ctx.selfjoin_topl(16, method="act", k=2, direction="sym")  # workspace
    ctx.profile(True)
    t1 = time.perf_counter()
    ctx.selfjoin_topl(16, method="act", k=2, direction="sym")
    dt = time.perf_counter() - t1
    ph = {p["name"]: p["ms"] for p in ctx.profile_get()}
    ctx.profile(False)
    ctx.close()
    res.update({"seconds": dt, "distances_per_s": n * n / dt, "phase_ms": ph,
                "speedup_vs_paper": (3.3 * 60) / dt})
    print(f"[bench] image self-join {n}x{n}: {dt:.3f} s", file=sys.stderr, flush=True)
    return res


def dense_section(a, lcemd):
    """Images with their background (every one of the 784 pixels a
    coordinate, Sec. 5): 60,000 database histograms of 784 words, symmetric
    top-16 for RWMD, OMR, ACT k=2, k=16 and ICT.  RWMD is 0 for every pair
    here; the ACT family separates the images."""
    import torch

    from synth import make_workload

    w = make_workload("image-bg", B=1000)
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
    n = w.db.n
    dev = torch.device("cuda:0")
    res = {"workload": f"image-bg: 784 pixels x 2 coordinates, {n} database histograms of 784 words "
                       f"({w.db.nnz} non-zeros), symmetric top-16"}
    for method, k, B in (("rwmd", 1, 1000), ("omr", 1, 1000), ("act", 2, 1000), ("act", 16, 1000),
                         ("ict", 1, 100)):
        qs = w.queries.take(list(range(B)))
        q = [torch.from_numpy(x).to(dev) for x in (qs.rowptr, qs.col, qs.val)]
        small = w.queries.take([0, 1])
        ctx.topl(small.rowptr, small.col, small.val, 16, method=method, k=k, direction="sym")
        ctx.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        idx, dist = ctx.topl(*q, 16, method=method, k=k, direction="sym")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ph = {p["name"]: p["ms"] for p in ctx.profile_get()}
        ctx.profile(False)
        rec = {"queries": B, "seconds": dt, "distances_per_s": B * n / dt, "phase_ms": ph}
        if method == "rwmd":
            rec["all_zero"] = bool((dist == 0).all())
        res[f"{method}{k}" if method == "act" else method] = rec
        print(f"[bench] dense {method} k={k}: {dt:.3f} s for {B} queries", file=sys.stderr, flush=True)
    ctx.close()
    return res


def big_workload(a, lcemd):
    """The 1M-word / 1M-document workload: (1) the precision variant -- one
    symmetric ACT k=8 top-16 call over the whole query batch with float32,
    bf16 and fp8 phase-1 keys: rates, top-16 agreement with float32, and the
    error of returned distances against the float64 oracle on sampled
    (query, neighbour) pairs; (2) serving (see serve_path)."""
    import numpy as np

    from synth import make_workload

    t0 = time.time()
    w = make_workload("text-1M", B=a.big_queries)
    print(f"[bench] 1M-word workload built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
    v, n, B = w.V.shape[0], w.db.n, w.queries.n
    res = {"workload": f"text-1M: vocab {v} x {w.V.shape[1]}, {n} database histograms "
                       f"({w.db.nnz} non-zeros), {B} queries, ACT k=8 symmetric, top-16"}
    prec = {}
    qs = w.queries
    ref = None
    rng = np.random.default_rng(77)
    sample = [(int(b), int(j)) for b, j in zip(rng.integers(0, B, 24), rng.integers(0, 16, 24))]
    small = qs.take(list(range(8)))
    for p in ("fp32", "bf16", "fp8"):
        ctx.topl(small.rowptr, small.col, small.val, 16, method="act", k=8, direction="sym", precision=p)
        t1 = time.perf_counter()
        idx, dist = ctx.topl(qs.rowptr, qs.col, qs.val, 16, method="act", k=8, direction="sym", precision=p)
        dt = time.perf_counter() - t1
        rec = {"distances_per_s": B * n / dt, "s_per_batch": dt}
        if ref is None:
            ref = (idx, dist)
        else:
            rec["top16_agreement_vs_fp32"] = float(np.mean([len(set(ref[0][i]) & set(idx[i])) / 16 for i in range(B)]))
        rec["_pairs"] = [(b, int(idx[b, j]), float(dist[b, j])) for b, j in sample]
        prec[p] = rec
        print(f"[bench] 1M-word {p}: {dt:.2f} s", file=sys.stderr, flush=True)
    # float64 oracle on the sampled (query, returned neighbour) pairs
    from oracle import emd_oracle as O

    docs = sorted({u for p in prec.values() for (_, u, _) in p["_pairs"]})
    sub = w.db.take(docs)
    pos = {u: i for i, u in enumerate(docs)}
    orc = O.Oracle(w.V, sub.rowptr, sub.col, sub.val)
    for p, rec in prec.items():
        errs = []
        for b, u, d in rec.pop("_pairs"):
            qc, qw = qs.row(b)
            o = orc.pair(qc, qw, pos[u], "act", 8, "sym")
            errs.append(abs(d - o) / max(abs(o), 1e-30))
        rec["max_rel_err_vs_fp64_oracle"] = float(np.max(errs))
        rec["median_rel_err_vs_fp64_oracle"] = float(np.median(errs))
        rec["oracle_pairs"] = len(errs)
    res["precision"] = prec
    fb, fixed = ctx.counters()
    res["fallback_tiles"], res["rows_redone_exactly"] = fb, fixed
    del w, qs, sub, orc
    if not a.no_serving:
        res["serving"] = serve_path(a, lcemd, ctx, v, n)
    ctx.close()
    return res


def serve_path(a, lcemd, ctx, v, n):
    """Serving on the resident 1M-word database: a Poisson query stream
    (open loop; 10-500 words per query), ACT k=8, symmetric top-16.  Two
    paths: bf16 phase 1 on two graph-captured lanes with continuous
    admission, and float32 phase 1 on one lane with kernels launched per
    batch and a batch admitted only when the previous one is done.
    Latency = completion - scheduled arrival."""
    import threading

    import numpy as np

    from synth import arrival_trace

    _, qs = arrival_trace(a.serve_rate, a.serve_queries + a.serve_sat, v, lmin=10, lmax=500)
    rows = [qs.row(b) for b in range(qs.n)]
    res = {}
    for prec, graph in (("bf16", True), ("fp32", False)):
        srv = lcemd.Server(ctx, method="act", k=8, precision=prec, l=16, max_slots=a.serve_slots,
                           memory_budget=a.serve_budget << 30, use_graph=graph)
        for b in range(4):  # warm-up
            srv.wait(srv.submit(*rows[b]))
        # saturation throughput: the whole sample submitted at once
        sat = rows[a.serve_queries:]
        t1 = time.perf_counter()
        tk = [srv.submit(c, x) for c, x in sat]
        for t in tk:
            srv.wait(t)
        sat_qps = len(sat) / (time.perf_counter() - t1)
        # open loop at the stated rate
        rate = a.serve_rate
        arr = np.cumsum(np.random.default_rng(55).exponential(1.0 / rate, a.serve_queries))
        lag = np.zeros(a.serve_queries)
        tickets = [0] * a.serve_queries
        start = time.perf_counter() + 0.05

        def feed():
            for i in range(a.serve_queries):
                d = start + arr[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                lag[i] = time.perf_counter() - (start + arr[i])
                tickets[i] = srv.submit(*rows[i])

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        lat = np.empty(a.serve_queries)
        for i in range(a.serve_queries):
            lat[i] = srv.wait(tickets[i])[2] + lag[i]
        span = time.perf_counter() - start
        srv.stop()
        res[prec] = {"path": ("bf16 keys, 2 graph-captured lanes, continuous admission" if graph else
                              "float32 keys, 1 lane, per-batch launches, static FIFO batches"),
                     "offered_qps": rate, "queries": a.serve_queries,
                     "p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "achieved_qps": a.serve_queries / span,
                     "saturation_qps": sat_qps,
                     "saturation_distances_per_s": sat_qps * n}
        print(f"[bench] serving {prec}: {res[prec]}", file=sys.stderr, flush=True)
    res["setup"] = (f"Poisson arrivals at {a.serve_rate:g} qps, 10-500 words per query, up to "
                    f"{a.serve_slots} queries per batch; saturation = {a.serve_sat} queries submitted at once")
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "lcemd runs on one GPU (sharding over several is designed, not implemented); --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch

    from paper_1812_02091_amd import lcemd
    from synth import make_workload

    kw = {}
    if a.n:
        kw["n"] = a.n
    if a.B:
        kw["B"] = a.B
    w = make_workload(a.workload, **kw)
    dev = torch.device("cuda:0")
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0)
    qp, qc, qv = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    idx = torch.empty((w.queries.n, a.ell), dtype=torch.int64, device=dev)
    dist = torch.empty((w.queries.n, a.ell), dtype=torch.float32, device=dev)

    def step():
        ctx.topl(qp, qc, qv, a.ell, method=a.method, k=a.k, direction=a.direction,
                 precision=a.precision, out=(idx, dist))

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    phases = {}
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
        for p in ctx.profile_get():
            d = phases.setdefault(p["name"], {"ms": 0.0, "launches": 0, "work": 0.0})
            d["ms"] += p["ms"]
            d["launches"] += p["launches"]
            d["work"] += p["work"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ctx.profile(False)
    B, n = w.queries.n, w.db.n
    value = B * n / dt

    # roofline of the dominant kernel: phase-1 distance contraction (MFMA)
    p1 = phases.get("phase1_table", {"ms": 0.0, "launches": 1, "work": 0.0})
    per_launch_ms = p1["ms"] / max(1, p1["launches"])
    per_launch_flops = p1["work"] / max(1, p1["launches"])
    achieved = per_launch_flops / (per_launch_ms * 1e-3) if per_launch_ms > 0 else 0.0
    peak = PEAKS.get(a.precision, PEAKS["fp32"])
    kernel = phase1_kernel(a.method, a.k, a.precision, w.V.shape[1])
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(kernel, a),
                "kernel": kernel,
                "avg_launch_ms": per_launch_ms,
                "flops_per_launch": per_launch_flops}
    p2 = phases.get("phase2")
    phase_report = {k: {"ms_per_step": v["ms"] / a.steps, "launches_per_step": v["launches"] / a.steps}
                    for k, v in phases.items()}
    if p2:
        p2_ms = p2["ms"] / max(1, p2["launches"])
        p2_bytes = p2["work"] / max(1, p2["launches"])
        phase_report["phase2"]["algorithmic_GBps"] = p2_bytes / (p2_ms * 1e-3) / 1e9
        phase_report["phase2"]["hbm_frac"] = p2_bytes / (p2_ms * 1e-3) / HBM_PEAK

    cpu, orows = None, None
    if not a.no_cpu:
        cpu, orows = cpu_baseline(w, a.method, a.k, a.ell, min(a.cpu_queries, B))

    # the other phase-1 arithmetics on the same batch, against this run's
    # path (top-l agreement) and against the float64 oracle (sampled rows)
    precisions = {}
    if orows is not None:
        precisions[a.precision] = oracle_error(ctx, w, len(orows), orows, a.method, a.k, a.precision)
    if not a.no_compare:
        ref_idx = idx.cpu().numpy()
        ref_dist = dist.cpu().numpy().astype(np.float64)
        for other in ("fp32", "bf16", "fp8"):
            if other == a.precision:
                continue
            oi = torch.empty_like(idx)
            od = torch.empty_like(dist)

            def ostep():
                ctx.topl(qp, qc, qv, a.ell, method=a.method, k=a.k, direction=a.direction,
                         precision=other, out=(oi, od))

            ostep()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(max(1, a.steps // 2)):
                ostep()
            torch.cuda.synchronize()
            odt = (time.perf_counter() - t1) / max(1, a.steps // 2)
            oidx = oi.cpu().numpy()
            agree = float(np.mean([len(set(ref_idx[i]) & set(oidx[i])) / a.ell for i in range(B)]))
            maxrel = float(np.max(np.abs(od.cpu().numpy().astype(np.float64) - ref_dist)
                                  / np.maximum(ref_dist, 1e-30)))
            rec = {"value": B * n / odt, "ms_per_step": odt * 1e3,
                   f"top{a.ell}_agreement_vs_{a.precision}": agree,
                   f"max_rel_diff_of_returned_distances_vs_{a.precision}": maxrel}
            if orows is not None:
                rec.update(oracle_error(ctx, w, len(orows), orows, a.method, a.k, other))
            precisions[other] = rec
    fb, fixed = ctx.counters()
    counters = {"fallback_tiles": fb, "rows_redone_exactly": fixed}
    ctx.close()
    image = None if a.no_big else image_section(a, lcemd)
    selfjoin = None if a.no_big else selfjoin_section(a, lcemd)
    measures = None if a.no_big else measures_section(a, lcemd)
    dense = None if a.no_big else dense_section(a, lcemd)
    big = None if a.no_big else big_workload(a, lcemd)

    out = {
        "metric": "query-doc ACT distances/sec + p50/p99 query latency, BF16 vs FP32 path",
        "value": value,
        "unit": "distances/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32"}.get(a.precision, a.precision),
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: vocab {w.V.shape[0]} x {w.V.shape[1]}, {n} database "
                               f"histograms ({w.db.nnz} non-zeros), {B} queries, "
                               f"{a.method.upper()} k={a.k} {a.direction}, top-{a.ell}",
                   "global_batch": B, "database": n, "k": a.k, "ell": a.ell,
                   "method": a.method, "direction": a.direction, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phase_report,
        "precisions": precisions,
        "counters": counters,
        "image": image,
        "selfjoin": selfjoin,
        "measures": measures,
        "image_bg": dense,
        "text_1M": big,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
