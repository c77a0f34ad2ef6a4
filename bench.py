"""Benchmark: symmetric ACT top-l search of a query batch against a resident
1M-word / 1M-document histogram database on one MI355X.

One step = one lcemd_topl call on the whole batch (query staging, phase-1
distance contraction + ordered extraction + float32 recompute, phase-2
transfers, Q2D for the pruned candidates, symmetric max, top-l), with the
database and the query batch already resident in HBM.

Workload (synthetic, seeded; stands in for word2vec-embedded text, which is
not available here): vocabulary 1,000,000 x 300 unit-norm Gaussian
embeddings, 1,000,000 database histograms and 4,096 queries of 50-300
distinct Zipf(1.0) words (log-normal lengths, mean ~120), tf weights; ACT
k=8, symmetric, top-16.  The headline value is the bf16 path (bf16 phase-1
keys, float32 recompute of the selected candidates); the float32 and fp8
paths run the same batch beside it.  Serving: open-loop Poisson streams of
10-500-word queries against the same resident database.

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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="act")
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--ell", type=int, default=16)
    ap.add_argument("--direction", default="sym")
    ap.add_argument("--precision", default="bf16", help="phase-1 keys of the headline path")
    ap.add_argument("--workload", default="text-1M")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--B", type=int, default=None)
    ap.add_argument("--other-steps", type=int, default=1, help="timed steps of each other precision")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle worker processes (the box's CPU share)")
    ap.add_argument("--no-compare", action="store_true", help="skip the other precisions")
    ap.add_argument("--no-big", action="store_true", help="skip the image and self-join sections")
    ap.add_argument("--all-sections", action="store_true", help="also the measure and dense-image sections")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement (no batch steps)")
    ap.add_argument("--serve-rates", default="200,500,1000,2000,5000", help="offered loads, queries/s")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival span per rate")
    ap.add_argument("--serve-sat", type=int, default=512, help="queries in the saturation burst")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-budget", type=int, default=16, help="GiB of device memory for lanes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def phase1_kernel(method, k, precision, m):
    """The phase-1 kernel the library picks for the table (D2Q) pass of
    queries against m-dimensional embeddings."""
    depth = {"rwmd": 1, "omr": 2, "act": k, "ict": 64}[method]
    mb = (m + 6 + 63) // 64 * 64
    if precision == "bf16" and depth + 8 <= 32 and mb <= 384:  # its own kernel: P1_TABLE, list size, K steps
        return f"k_phase1_bf16<0, {16 if depth + 8 <= 16 else 32}, {mb // 16}>"
    margin = 0 if precision == "fp32" or depth + 8 > 32 else 8
    kl = 2
    while kl < depth + margin:
        kl *= 2
    prec = 0 if margin == 0 else {"bf16": 1, "fp8": 2}[precision]
    if prec == 0 and (m + 3) // 4 <= 7 and depth <= 64 and method != "ict":  # float32, at most 28 dims: 64-row kernel
        return f"k_phase1_fast<0, {kl}, 0>"
    if depth + margin <= 32:
        return f"k_phase1_wide<0, {kl}, {prec}, false>"
    return "k_phase1_fast<0, 64, 0>" if depth <= 64 else "k_phase1_f32"


KERNEL_SOURCES = {"k_phase1_bf16": "phase1_bf16.hip", "k_phase2_persistent": "phase2.hip",
                  "k_p2_word_costs": "phase2.hip", "k_p2_doc_sums": "phase2.hip"}


def traffic_record(kernel, a, precision):
    """The committed rocprofv3 --pmc record of `kernel` on this workload
    (profiles/traffic.json: HBM bytes per launch, launches per step), if it
    was taken on the current kernel source (its sha256 is recorded with it);
    otherwise None."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1812_02091_amd", "csrc", KERNEL_SOURCES.get(kernel.split("<")[0], "phase1_wide.hip"))
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    key = f"{a.workload}:{a.method}:{a.k}:{a.direction}:{precision}:{kernel}"
    e = rec.get(key)
    if not e or e.get("source_sha256") != digest:
        return None
    return e


def measured_traffic(kernel, a, precision):
    e = traffic_record(kernel, a, precision)
    return None if e is None else e["bytes_per_launch"]


def phase2_roofline(phases, steps, a, precision):
    """Phase 2 against HBM: the counted bytes of its kernels per step (the
    word-major pair on the 1M-word workload, from profiles/traffic.json) over
    its HIP-event time; beside it the A2 figure (a full pass over the
    database charged to every query, which the kernels share across 64
    queries: not a fraction of anything)."""
    p2 = phases.get("phase2")
    if not p2 or p2["ms"] <= 0:
        return None
    ms = p2["ms"] / steps
    kt = {"rwmd": 1, "omr": 2, "act": a.k}.get(a.method, 64)
    recs = [traffic_record(k, a, precision) for k in (f"k_p2_word_costs<{4 if (kt + 1) // 2 <= 4 else 8}>",
                                                      "k_p2_doc_sums")]
    out = {"bound": "hbm", "ms_per_step": ms, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
           "a2_algorithmic_GBps": p2["work"] / (p2["ms"] * 1e-3) / 1e9}
    if all(recs):
        byt = sum(r["bytes_per_launch"] * r["launches_per_step"] for r in recs)
        out.update({"kernels": "k_p2_word_costs + k_p2_doc_sums", "counted_bytes_per_step": byt,
                    "achieved": byt / (ms * 1e-3) / 1e9, "frac": byt / (ms * 1e-3) / HBM_PEAK})
    else:
        out.update({"achieved": None, "frac": None, "counted_bytes_per_step": None})
    return out


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


_ORC = {}


def _host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"os_cpu_count": os.cpu_count(), "nproc": nproc, "cpu_model": model}


def _oracle_task(args):
    """One oracle task: the float64 symmetric distances of one query to a
    range of database rows (a fresh Oracle over those rows), in a forked
    worker that inherited the workloads."""
    name, b, lo, hi, method, k = args
    from oracle import emd_oracle as O

    w = _ORC[name]
    sub = w.db.take(range(lo, hi))
    t0 = time.perf_counter()
    orc = O.Oracle(w.V, sub.rowptr, sub.col, sub.val)
    qc, qw = w.queries.row(b)
    row = orc.row_distances(qc, qw, method, k, "sym")
    return name, b, lo, hi - lo, time.perf_counter() - t0, row


def cpu_baseline(workers, method, k, big):
    """The float64 oracle timed on the host's cores, before any GPU work
    (forked workers inherit the workloads; one thread each).  Samples: the
    tiny workload whole (8 x 200); 8 text queries x all 18,000 rows; 8 image
    queries x all 60,000 rows; 1 query of the 1M-word workload x all
    1,000,000 rows (`big`, the headline's workload: its rate is `value`).
    Returns the record and the 1M-word oracle row (for the error check)."""
    import multiprocessing as mp

    import numpy as np

    from synth import make_workload

    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    _ORC["tiny"] = make_workload("tiny")
    _ORC["text"] = make_workload("text", B=8)
    _ORC["image"] = make_workload("image", B=8)
    _ORC["text-1M"] = big
    plan = (("text", 8, 18000, 2250), ("image", 8, 60000, 7500), ("text-1M", 1, big.db.n, 31250))
    tasks = [("tiny", b, 0, 200, method, min(k, 3)) for b in range(8)]
    for name, nq, n, chunk in plan:
        for b in range(nq):
            for lo in range(0, n, chunk):
                tasks.append((name, b, lo, min(n, lo + chunk), method, k))
    # the long 1M-word chunks first, so that the pool ends together
    tasks.sort(key=lambda t: -(t[3] - t[2]) * (3 if t[0] == "text-1M" else 1))
    workers = max(1, min(workers, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    res = []
    with ctx.Pool(workers) as pool:
        for i, r in enumerate(pool.imap_unordered(_oracle_task, tasks, chunksize=1)):
            res.append(r)
            if (i + 1) % 32 == 0 or i + 1 == len(tasks):
                print(f"[bench] oracle baseline: {i + 1}/{len(tasks)} tasks, {time.perf_counter() - t0:.0f} s",
                      file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    per = {}
    big_row = {}
    for name, b, lo, npairs, dt, row in res:
        d = per.setdefault(name, {"pairs": 0, "cpu_s": 0.0})
        d["pairs"] += npairs
        d["cpu_s"] += dt
        if name == "text-1M":
            big_row[lo] = row
    big_row = np.concatenate([big_row[lo] for lo in sorted(big_row)])
    total_cpu = sum(d["cpu_s"] for d in per.values())
    for name, d in per.items():
        d["single_core_pairs_per_s"] = d["pairs"] / d["cpu_s"]
        # all cores: the sample's share of the pool's wall time
        d["all_core_pairs_per_s"] = d["pairs"] / (wall * d["cpu_s"] / total_cpu)
    per["tiny"]["sample"] = "the whole 8 x 200 workload (ACT k=min(k,3))"
    per["text"]["sample"] = "8 queries x all 18,000 rows"
    per["image"]["sample"] = "8 queries x all 60,000 rows"
    per["text-1M"]["sample"] = f"query 0 x all {big.db.n:,} rows"
    bigrec = per["text-1M"]
    host = _host_info()
    full_h = big.queries.n * big.db.n / bigrec["all_core_pairs_per_s"] / 3600
    rec = {"value": bigrec["all_core_pairs_per_s"], "unit": "distances/s", "cores": workers, "kind": "oracle",
           "sample": (f"query 0 of the 1M-word workload x all {big.db.n:,} database rows, {method.upper()} k={k} "
                      f"symmetric, float64 numpy/scipy oracle, {workers} worker processes of one thread "
                      f"({wall:.1f} s wall for all samples, {total_cpu:.0f} s of CPU); the full "
                      f"{big.queries.n:,} x {big.db.n:,} batch would take {full_h:.0f} h at this rate "
                      f"(extrapolation)"),
           "host": host, "samples": per, "wall_s": wall, "cpu_s": total_cpu}
    return rec, big_row


def oracle_pairs_error(w, idx, dist, picks, method, k):
    """Relative error of returned (query, neighbour) distances against the
    float64 oracle, pair by pair."""
    import numpy as np

    from oracle import emd_oracle as O

    docs = sorted({int(idx[b, j]) for b, j in picks})
    sub = w.db.take(docs)
    pos = {u: i for i, u in enumerate(docs)}
    orc = O.Oracle(w.V, sub.rowptr, sub.col, sub.val)
    errs = []
    for b, j in picks:
        qc, qw = w.queries.row(int(b))
        o = orc.pair(qc, qw, pos[int(idx[b, j])], method, k, "sym")
        errs.append(abs(float(dist[b, j]) - o) / max(abs(o), 1e-30))
    return {"max_rel_err_vs_fp64_oracle": float(np.max(errs)), "median_rel_err_vs_fp64_oracle": float(np.median(errs)),
            "oracle_pairs": len(errs)}


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
            # A2 charges every query a full pass over the database; the kernel
            # shares each record read across up to 64 queries, so this rate can
            # pass the HBM peak and is not an HBM fraction
            rec["phase2_algorithmic_GBps_A2"] = ph["phase2"]["work"] / (ph["phase2"]["ms"] * 1e-3) / 1e9
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
                "paper_time_over_this_time_context_only": (3.3 * 60) / dt})
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


def serve_sweep(a, lcemd, ctx, v, n):
    """Serving on the resident 1M-word database: open-loop Poisson streams of
    10-500-word queries (ACT k=8, symmetric top-16), each offered rate for
    about --serve-seconds, rising until the path saturates (achieved rate
    below 90 % of the offered one), plus a saturation burst.  Three paths:
    bf16 keys on one launch lane (the default: the next batch starts the
    moment the previous one ends, with every query that arrived meanwhile),
    bf16 keys on four lanes (up to four batches side by side), and float32
    keys on one lane -- precision and lane count each change alone between
    two of them.  Latency = completion - scheduled arrival."""
    import threading

    import numpy as np

    from synth import arrival_trace

    rates = [float(x) for x in a.serve_rates.split(",") if x]
    need = a.serve_sat + sum(int(min(3000, max(200, r * a.serve_seconds))) for r in rates) + 8
    _, qs = arrival_trace(1000.0, need, v, lmin=10, lmax=500)
    rows = [qs.row(b) for b in range(qs.n)]
    out = {"setup": (f"Poisson arrivals, 10-500 words per query, up to {a.serve_slots} queries per batch; each "
                     f"rate offered for ~{a.serve_seconds:g} s (200-3,000 queries) until saturation; saturation = "
                     f"{a.serve_sat} queries submitted at once")}
    for name, prec, graph, lanes in (("bf16", "bf16", True, 1), ("bf16_4lanes", "bf16", True, 4),
                                     ("fp32", "fp32", False, 1)):
        srv = lcemd.Server(ctx, method="act", k=8, precision=prec, l=16, max_slots=a.serve_slots,
                           memory_budget=a.serve_budget << 30, use_graph=graph, lanes=lanes)
        cur = 0

        def take(m):
            nonlocal cur
            r = rows[cur:cur + m]
            cur += m
            return r

        for q in take(8):  # warm-up
            srv.wait(srv.submit(*q))
        sat = take(a.serve_sat)
        t1 = time.perf_counter()
        tk = [srv.submit(c, x) for c, x in sat]
        for t in tk:
            srv.wait(t)
        sat_qps = len(sat) / (time.perf_counter() - t1)
        sweep = []
        for rate in rates:
            nq = int(min(3000, max(200, rate * a.serve_seconds)))
            batch = take(nq)
            arr = np.cumsum(np.random.default_rng(55 + int(rate)).exponential(1.0 / rate, nq))
            lag = np.zeros(nq)
            tickets = [0] * nq
            start = time.perf_counter() + 0.05

            def feed():
                for i in range(nq):
                    d = start + arr[i] - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    lag[i] = time.perf_counter() - (start + arr[i])
                    tickets[i] = srv.submit(*batch[i])

            th = threading.Thread(target=feed)
            th.start()
            th.join()
            lat = np.empty(nq)
            for i in range(nq):
                lat[i] = srv.wait(tickets[i])[2] + lag[i]
            span = time.perf_counter() - start
            rec = {"offered_qps": rate, "queries": nq, "achieved_qps": nq / span,
                   "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}
            rec["saturated"] = rec["achieved_qps"] < 0.9 * rate
            sweep.append(rec)
            print(f"[bench] serving {name} {rate:g} qps: {rec}", file=sys.stderr, flush=True)
            if rec["saturated"]:
                break
        srv.stop()
        out[name] = {"path": (f"{prec} keys, {lanes} launch lane{'s' if lanes > 1 else ''} (a free lane takes the "
                              f"waiting queries at once), {'graph-captured' if graph else 'eagerly launched'} "
                              f"batches"),
                     "lanes": lanes,
                     "saturation_qps": sat_qps, "saturation_distances_per_s": sat_qps * n, "sweep": sweep}
    return out


def run_batch(ctx, q, out, a, precision, steps, warmup):
    """Warm-up and timed whole-batch steps of one precision: (s per step,
    per-phase record summed over the timed steps)."""
    import torch

    def step():
        ctx.topl(*q, a.ell, method=a.method, k=a.k, direction=a.direction, precision=precision, out=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    phases = {}
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        for p in ctx.profile_get():
            d = phases.setdefault(p["name"], {"ms": 0.0, "launches": 0, "work": 0.0})
            d["ms"] += p["ms"]
            d["launches"] += p["launches"]
            d["work"] += p["work"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ctx.profile(False)
    return dt, phases


def phase_report(phases, steps):
    rep = {}
    for k, v in phases.items():
        r = {"ms_per_step": v["ms"] / steps, "launches_per_step": v["launches"] / steps}
        if k == "phase1_table" and v["ms"] > 0:
            r["algorithmic_TFLOPs"] = v["work"] / (v["ms"] * 1e-3) / 1e12
        if k == "phase2" and v["ms"] > 0:
            # A2 model: every query streams the database and reads its tables once
            r["algorithmic_GBps_A2"] = v["work"] / (v["ms"] * 1e-3) / 1e9
        rep[k] = r
    return rep


def roofline_of(phases, precision, a):
    """Roofline of the dominant kernel: the phase-1 table pass (MFMA-bound,
    algorithmic flops 2 v_used H m per launch against the key precision's
    dense peak) or phase 2 (A2 bytes per launch against HBM)."""
    p1 = phases.get("phase1_table", {"ms": 0.0, "launches": 1, "work": 0.0})
    p2 = phases.get("phase2", {"ms": 0.0, "launches": 1, "work": 0.0})
    if p1["ms"] >= p2["ms"]:
        ms = p1["ms"] / max(1, p1["launches"])
        flops = p1["work"] / max(1, p1["launches"])
        ach = flops / (ms * 1e-3) if ms > 0 else 0.0
        peak = PEAKS.get(precision, PEAKS["fp32"])
        kernel = phase1_kernel(a.method, a.k, precision, a.m)
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": measured_traffic(kernel, a, precision), "kernel": kernel, "avg_launch_ms": ms,
                "flops_per_launch": flops}
    ms = p2["ms"] / max(1, p2["launches"])
    byt = p2["work"] / max(1, p2["launches"])
    ach = byt / (ms * 1e-3) if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": ach / HBM_PEAK,
            "traffic": measured_traffic("k_phase2_persistent", a, precision), "kernel": "k_phase2_persistent",
            "avg_launch_ms": ms, "bytes_per_launch": byt}


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

    from synth import make_workload

    kw = {}
    if a.n:
        kw["n"] = a.n
    if a.B:
        kw["B"] = a.B
    t0 = time.time()
    w = make_workload(a.workload, **kw)
    a.m = int(w.V.shape[1])
    print(f"[bench] {a.workload} workload built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    # the CPU baseline runs first, in forked workers, before any GPU work
    full = a.workload == "text-1M" and not kw
    cpu, orow = (None, None)
    if not a.no_cpu:
        cpu, orow = cpu_baseline(a.cpu_workers, a.method, a.k, w if full else make_workload("text-1M"))
        print(f"[bench] oracle baseline: {cpu['value']:.0f} distances/s on {cpu['cores']} workers",
              file=sys.stderr, flush=True)
        if not full:
            orow = None

    import torch

    from paper_1812_02091_amd import lcemd

    dev = torch.device("cuda:0")
    ctx = lcemd.open_context(w.V, w.db.rowptr, w.db.col, w.db.val, device=0, precisions=("bf16", "fp8"))
    q = [torch.from_numpy(x).to(dev) for x in (w.queries.rowptr, w.queries.col, w.queries.val)]
    B, n = w.queries.n, w.db.n
    out = (torch.empty((B, a.ell), dtype=torch.int64, device=dev), torch.empty((B, a.ell), dtype=torch.float32, device=dev))

    if a.serve_only:
        print(json.dumps({"serving": serve_sweep(a, lcemd, ctx, w.V.shape[0], n)}))
        ctx.close()
        return
    dt, phases = run_batch(ctx, q, out, a, a.precision, a.steps, a.warmup)
    value = B * n / dt
    print(f"[bench] {a.precision}: {dt:.3f} s per step", file=sys.stderr, flush=True)
    roofline = roofline_of(phases, a.precision, a)
    ref_idx, ref_dist = out[0].cpu().numpy(), out[1].cpu().numpy()
    rng = np.random.default_rng(77)
    picks = [(int(b), int(j)) for b, j in zip(rng.integers(0, B, 24), rng.integers(0, a.ell, 24))]
    precisions = {a.precision: {"distances_per_s": value, "s_per_step": dt, "phases": phase_report(phases, a.steps)}}
    precisions[a.precision].update(oracle_pairs_error(w, ref_idx, ref_dist, picks, a.method, a.k))
    results = {a.precision: (ref_idx, ref_dist)}
    if not a.no_compare:
        for other in ("fp32", "bf16", "fp8"):
            if other == a.precision:
                continue
            odt, oph = run_batch(ctx, q, out, a, other, a.other_steps, 1)
            oi, od = out[0].cpu().numpy(), out[1].cpu().numpy()
            results[other] = (oi, od)
            rec = {"distances_per_s": B * n / odt, "s_per_step": odt, "phases": phase_report(oph, a.other_steps),
                   "roofline_of_dominant_kernel": roofline_of(oph, other, a)}
            rec.update(oracle_pairs_error(w, oi, od, picks, a.method, a.k))
            precisions[other] = rec
            print(f"[bench] {other}: {odt:.3f} s per step", file=sys.stderr, flush=True)
        if "fp32" in results:
            fi = results["fp32"][0]
            for p, (ii, _) in results.items():
                if p != "fp32":
                    precisions[p][f"top{a.ell}_agreement_vs_fp32"] = float(
                        np.mean([len(set(fi[i]) & set(ii[i])) / a.ell for i in range(B)]))
    if orow is not None:
        # the whole oracle row of query 0 (all 1M documents): the GPU's
        # symmetric distances of the same query, and its top-l list against
        # the oracle's
        sub_q = w.queries.take([0])
        g = ctx.distances(sub_q.rowptr, sub_q.col, sub_q.val, method=a.method, k=a.k, direction="sym",
                          precision=a.precision)[0].astype(np.float64)
        rel = np.abs(g - orow) / np.maximum(np.abs(orow), 1e-30)
        o_top = np.lexsort((np.arange(orow.shape[0]), orow))[:a.ell]
        precisions[a.precision].update({"oracle_row_max_rel_err": float(rel.max()),
                                        "oracle_row_pairs": int(rel.size),
                                        "oracle_row_topl_overlap": len(set(o_top.tolist()) &
                                                                       set(ref_idx[0].tolist())) / a.ell})
    fb, fixed = ctx.counters()
    counters = {"fallback_tiles": fb, "rows_redone_exactly": fixed}
    serving = None if a.no_serving else serve_sweep(a, lcemd, ctx, w.V.shape[0], n)
    ctx.close()
    del q, out
    image = None if a.no_big else image_section(a, lcemd)
    selfjoin = None if a.no_big else selfjoin_section(a, lcemd)
    measures = measures_section(a, lcemd) if a.all_sections else None
    dense = dense_section(a, lcemd) if a.all_sections else None

    res = {
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
                               f"{a.method.upper()} k={a.k} {a.direction}, top-{a.ell}, {a.precision} phase-1 keys",
                   "global_batch": B, "database": n, "k": a.k, "ell": a.ell,
                   "method": a.method, "direction": a.direction, "parallelism": "single GPU"},
        "roofline": roofline,
        "phase2_roofline": phase2_roofline(phases, a.steps, a, a.precision),
        "cpu_baseline": cpu,
        "phases": precisions[a.precision]["phases"],
        "precisions": precisions,
        "counters": counters,
        "serving": serving,
        "image": image,
        "selfjoin": selfjoin,
        "measures": measures,
        "image_bg": dense,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
