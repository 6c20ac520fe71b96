"""Benchmark: the block Wiedemann sequence mod p on one MI355X.

Workload (the default, one "step"): 512 applications of B = D_c A^T D_r A D_c
(513 sequence terms S_k = U^T B^k V mod p, projections included) on the
planted 2 000 000 x 1 000 000 integer matrix (planted rank 900 000, 37.2 M
non-zeros, 85 % +-1), block size 16, p = 65521, the paper-scale shape.  The
matrix is encoded once on the device (bwr_matrix_create_dev) and the
autotuner has picked the launch plan before the timed region; every step is one
bwr_matrix_sequence_dev call from the same U, V and diagonals, inputs resident
in HBM.  After the timed steps the whole rank of the same matrix is computed
once (bwr_rank_modp_dev: encoding, 2 + 2n/16 + 4 terms, sigma-basis, read-out)
and checked against the planted rank, then once more with early termination
(bwr_set_early_termination; --no-early-rank skips it).

value = whole-job throughput in Gnnz.vec/s: the sparse multiply-adds of the
two products of every application of B (2 nnz s per application), summed over
the timed steps, divided by their wall time.

roofline: the kernel with the most device time per step (of the first product
A X with the row scale, and the second product A^T Y with the column scale and
the fused U^T projection); its average duration comes from HIP events around
back-to-back launches on the stream the kernel runs on
(bwr_time_step_kernels_dev), its algorithmic bytes per launch from the plain
encoding (4 B index + 1 B value per non-zero, 4 B row pointers, 4 B residues):
B_launch = 4 (rows + 1) + 5 nnz + 4 s (n + m).  traffic is the measured memory
traffic per launch from the committed counter summary (profiles/traffic.json),
null when that summary belongs to another revision of the kernel source.

cpu_baseline: the oracle's plain sequence (scipy CSR products and numpy
reductions mod p) on a bounded number of applications of B of the same
matrix, on all host cores (the block's columns split over threads, as the
paper splits them over processes) and on one core; plus the oracle's plain-C
elimination rank of the 2000 x 1500 and 200000 x 150000 planted matrices.

Other modes: --rank-c2 (ranks of the 200000 x 150000 matrix at p = 65521 and
2^31 - 1), --paper-rank (the whole rank only), --batch, --serve, and
--profile-kernels / --traffic-from for the counter summaries.  --early turns
early termination on for --paper-rank, --batch and --serve; --batch-retry n
applies the batched agreement retry to both passes of --batch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "GF(p) SpMM Gnnz·vec/s + % HBM roofline; rank solves/sec batched vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_info():
    """CPU model (from /proc/cpuinfo) and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    return model, threads


def cpu_baseline(A, p, s, target_s=12.0, ge_mats=()):
    """The oracle's sequence loop on a bounded number of applications of B of A: on all host threads (the
    block's columns split over a thread pool, each thread running the oracle's apply on its columns; scipy's
    sparse products release the interpreter lock) and on one thread; plus the oracle's plain-C elimination rank
    of each matrix in ge_mats (name, CSR)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import native
    from oracle import sequence as oseq

    model, threads = cpu_info()
    rng = np.random.default_rng(0)
    U = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    V = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    orc = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, dr, dc)

    def run(nthreads):
        groups = [list(range(c, s, nthreads)) for c in range(min(nthreads, s))]
        W = V % p
        steps = 0
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=len(groups)) as ex:
            while True:
                parts = list(ex.map(lambda g: orc.apply(W[:, g]), groups))
                for g, part in zip(groups, parts):
                    W[:, g] = part
                oseq.project(U, W, p)
                steps += 1
                el = time.perf_counter() - t0
                if el >= target_s or steps >= 400:
                    break
        return 2.0 * A.nnz * s * steps / el / 1e9, steps, el

    use = max(1, min(threads, s))
    log(f"cpu baseline: oracle sequence on {use} threads")
    rate_all, st_all, el_all = run(use)
    log("cpu baseline: oracle sequence on 1 thread")
    rate_one, st_one, el_one = run(1)
    ge = {}
    for name, M in ge_mats:
        log(f"cpu baseline: elimination rank of {name}")
        t0 = time.perf_counter()
        r = native.rank_csr_c(M, p)
        ge[name] = {"rank": int(r), "seconds": round(time.perf_counter() - t0, 3), "p": p}
    return {"value": round(rate_all, 4), "unit": "Gnnz·vec/s", "cores": use, "kind": "oracle",
            "sample": f"{st_all} applications of B = D_c A^T D_r A D_c to the n x {s} block (then U^T W mod {p}) "
                      f"of the same {A.m} x {A.n} matrix by the oracle's plain sequence, the block's columns split "
                      f"over {use} threads, {el_all:.1f} s",
            "one_core": {"value": round(rate_one, 4), "cores": 1,
                         "sample": f"{st_one} applications on one thread, {el_one:.1f} s"},
            "cpu_model": model, "host_threads": threads,
            "elimination_rank": ge}


def _source_digest(rel):
    import hashlib

    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def kernel_traffic(name):
    """Memory traffic per launch (bytes) of the kernel instantiation `name` (as rocprofv3 prints it, without
    the namespace; "ACC" stands for any accumulator digit) from the committed counter summary, or None when
    the summary is missing, was taken on another revision of the kernel's source, or does not hold exactly
    one matching instantiation."""
    import re

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        pat = re.compile(re.escape(name).replace("ACC", r"\d"))
        hits = [v for k, v in rec["kernels"].items() if pat.fullmatch(k)]
        if len(hits) != 1:
            return None
        ent = hits[0]
        src = ent["source"]
        if rec["sources"][src] != _source_digest(src):
            return None
    except (OSError, KeyError, ValueError, TypeError):
        return None
    return ent.get("bytes_per_launch")


def product_kernel(plan, which, s, p):
    """rocprofv3 name (without namespace) and source of the kernel that runs product `which` (1 or 2)."""
    esize = plan["esize"]
    etype = "unsigned short" if esize == 2 else "unsigned int"
    W = plan["W"]
    split = "true" if p > 65536 else "false"
    if plan[f"T{which}R"] > 0:
        proj = "1" if which == 2 else "0"
        return (f"k_spmm_tiled<{W}, {etype}, {split}, {proj}>", "paper_0704_2351_amd/csrc/spmm_tiled.hip",
                f"tiled: row blocks of {plan[f'T{which}R']} rows, slabs of 2^{plan[f'T{which}cb']} block rows, "
                f"{plan[f'T{which}grid']} workgroups, {plan.get(f'T{which}un', 4)} entries per lane per pass")
    G = plan[f"G{which}"]
    fused = "true" if (which == 2 and plan["fused"]) else "false"
    return (f"k_spmm_split<{W}, {G}, ACC, {'true' if p <= 65536 else 'false'}, {fused}, {etype}, 0>",
            "paper_0704_2351_amd/csrc/spmm.hip", f"row split G = {G}")


def roofline_entry(A, s, p, us, plan):
    """Roofline of the kernel with the most device time per step: algorithmic bytes per launch with the plain
    encoding (4 B row pointers, 4 B index + 1 B value per non-zero, 4 B per residue read and written; U and
    the diagonals are regenerable and not counted) over its average launch time."""
    m, n, nnz = A.m, A.n, A.nnz
    b = {1: 4 * (m + 1) + 5 * nnz + 4 * s * (n + m), 2: 4 * (n + 1) + 5 * nnz + 4 * s * (m + n)}
    t = {1: float(us[0]), 2: float(us[1]) + float(us[2])}
    dom = 1 if t[1] > t[2] else 2
    other = 3 - dom
    ach = b[dom] / (t[dom] * 1e-6) / 1e9
    ach_o = b[other] / (t[other] * 1e-6) / 1e9
    name, src, how = product_kernel(plan, dom, s, p)
    oname, _, ohow = product_kernel(plan, other, s, p)
    what = {1: "first product: A X, row scale", 2: "second product: A^T Y, column scale, fused U^T projection"}
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": kernel_traffic(name),
            "kernel": f"{name} ({what[dom]}; {how}; {plan['esize']}-byte residues), p = {p}",
            "avg_launch_us": round(t[dom], 3), "bytes_per_launch": int(b[dom]),
            "other_product": {"kernel": f"{oname} ({what[other]}; {ohow})", "achieved": round(ach_o, 1),
                              "frac": round(ach_o / PEAK_HBM_GBS, 4), "avg_launch_us": round(t[other], 3),
                              "bytes_per_launch": int(b[other]), "traffic": kernel_traffic(oname)},
            "step": {"achieved": round((b[1] + b[2]) / ((t[1] + t[2]) * 1e-6) / 1e9, 1),
                     "frac": round((b[1] + b[2]) / ((t[1] + t[2]) * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                     "kernel_us": round(t[1] + t[2], 3), "bytes": int(b[1] + b[2])}}


def batch_mode(args):
    """Batched ranks against one-at-a-time ranks on the same matrices and primes."""
    import paper_0704_2351_amd as bw
    from workloads import CONFIG4_PRIMES, config4_matrix, config4_shapes

    shapes = config4_shapes()
    order = sorted(range(len(shapes)), key=lambda j: shapes[j][1])
    step = max(1, len(order) // max(1, args.batch_count))
    pick = order[::step][: args.batch_count]
    log(f"generating {len(pick)} planted matrices (n from {shapes[pick[0]][1]} to {shapes[pick[-1]][1]})")
    mats = [config4_matrix(j, shapes) for j in pick]
    primes = CONFIG4_PRIMES
    nsolves = len(mats) * len(primes)
    work = sum(2.0 * A.nnz * 8 * (bw.sequence_length(min(A.m, A.n), 8) + 3) for A in mats) * len(primes)
    retry = int(args.batch_retry)
    bw.set_batch_retry(retry)
    log("batched: warmup on the smallest matrix")
    bw.rank_modp_batch(mats[:1], primes, 8, 1)
    t0 = time.perf_counter()
    ranks, info = bw.rank_modp_batch(mats, primes, 8, 1)
    tb = time.perf_counter() - t0
    short = [[int(j), int(primes[t]), int(ranks[j, t]), int(A.planted_rank)] for j, A in enumerate(mats)
             for t in range(len(primes)) if ranks[j, t] != A.planted_rank]
    ok_b = not short
    log(f"batched {tb:.2f} s, ranks ok: {ok_b}")
    t0 = time.perf_counter()
    plain_ok = True
    trials = bw.get_trials()
    for j, A in enumerate(mats):
        rj = [bw.rank_modp(A, p, 8, 1)[0] for p in primes]
        # the same agreement retry as the batched call: further draws where the primes disagree
        for t, p in enumerate(primes):
            k = 0
            while k < retry and rj[t] < max(rj):
                rj[t] = max(rj[t], bw.rank_modp(A, p, 8, 1 + trials + k)[0])
                k += 1
        plain_ok &= all(rj[t] == ranks[j, t] for t in range(len(primes)))
        log(f"plain: matrix {j + 1}/{len(mats)} done")
    tp = time.perf_counter() - t0
    log(f"plain {tp:.2f} s, identical ranks: {plain_ok}")
    print(json.dumps({
        "metric": METRIC, "mode": "batched", "value": round(nsolves / tb, 4), "unit": "solves/s",
        "plain_solves_per_s": round(nsolves / tp, 4), "speedup_vs_plain": round(tp / tb, 3),
        "batched_gnnzvec_per_s": round(work / tb / 1e9, 3), "plain_gnnzvec_per_s": round(work / tp / 1e9, 3),
        "ranks_equal_planted": bool(ok_b), "ranks_equal_plain": bool(plain_ok), "solves": nsolves,
        "ranks_short_of_planted": short,  # [matrix index, p, rank, planted rank]
        # with early termination the Gnnz.vec/s figures still count every sequence at its full length
        "early_termination": bool(bw.get_early_termination()), "batch_retry": retry,
        "batch_info": info, "higher_is_better": True, "n_gpus": 1, "dtype": "u32",
        "data": "synthetic planted-rank matrices (seeded)",
        "config": {"workload": f"{len(mats)} of the 64 batched-configuration matrices (n log-uniform 5e3..2e5, "
                               f"m = 1.2-2.0 n, rank 70-95 % of n) x primes {list(primes)}, block 8",
                   "matrices": [[A.m, A.n, A.nnz] for A in mats]}}), flush=True)


def draws(p, s, m, n, torch):
    """U, V (n x s) and the diagonals D_r (m), D_c (n) from the library's counter-based generator, on cuda:0."""
    import numpy as np

    import paper_0704_2351_amd as bw

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    return (t(bw.random_block(11, 1, n, s, p)), t(bw.random_block(11, 0, n, s, p)),
            t(bw.random_block(11, 2, m, 1, p, True).reshape(m)), t(bw.random_block(11, 3, n, 1, p, True).reshape(n)))


def sequence_mode(args):
    """The default workload: blocks of sequence terms of the 2 000 000 x 1 000 000 matrix (see the module
    docstring), then the whole rank once."""
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config1, config2, config3

    s, p = 16, 65521
    log("generating the planted 2000000 x 1000000 matrix")
    A = config3()
    m, n, nnz = A.m, A.n, A.nnz
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    log("kernel timing (the autotuner picks the launch plan on its first call)")
    us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
    log(f"plan {plan}, kernels {[round(x, 1) for x in us]} us")
    t0 = time.perf_counter()
    M = bw.Matrix(Ad, p)
    torch.cuda.synchronize()
    t_encode = time.perf_counter() - t0
    U, V, dr, dc = draws(p, s, m, n, torch)
    terms = args.terms
    for w in range(args.warmup):
        M.sequence_dev(U, V, p, terms, dr, dc)
        log(f"warmup {w + 1}/{args.warmup}")
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps of {terms - 1} applications of B")
    t0 = time.perf_counter()
    for k in range(args.steps):
        S = M.sequence_dev(U, V, p, terms, dr, dc)
        if (k + 1) % 5 == 0 or k + 1 == args.steps:
            log(f"step {k + 1}/{args.steps} queued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    work = 2.0 * nnz * s * (terms - 1) * args.steps
    # live kernel timing for the roofline (HIP events on the stream the kernels run on), with the plan the
    # timed steps used
    us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
    M.close()
    out = {
        "metric": METRIC,
        "value": round(work / elapsed / 1e9, 3),
        "unit": "Gnnz·vec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16" if plan["esize"] == 2 else "u32",
        "data": "synthetic planted-rank matrix (seeded); no dataset",
        "config": {"workload": f"block Wiedemann sequence mod {p} of a planted {m} x {n} sparse integer matrix "
                               f"(rank {A.planted_rank}, {nnz / 1e6:.1f} M non-zeros), block {s}, "
                               f"{terms - 1} applications of B per step",
                   "m": m, "n": n, "nnz": nnz, "block": s, "p": p, "applications_per_step": terms - 1,
                   "parallelism": "single GPU"},
        "us_per_application": round(1e6 * elapsed / ((terms - 1) * args.steps), 2),
        "encode_s": round(t_encode, 3),
        "step_kernel_us": [round(float(x), 3) for x in us],
        "step_plan": plan,
        "roofline": roofline_entry(A, s, p, us, plan),
    }
    if not args.no_rank:
        log(f"rank mod {p} of the same matrix, block {s} ({bw.sequence_length(n, s) + 4} terms)")
        t0 = time.perf_counter()
        r, info = bw.rank_modp_dev(Ad, p, s, 1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["rank"] = {"rank": int(r), "planted_rank": int(A.planted_rank), "equals_planted": bool(r == A.planted_rank),
                       "seconds": round(el, 2), "t_sequence": round(info["t_sequence"], 2),
                       "t_sigma_after_sequence": round(info["t_sigma"], 3), "t_encode": round(info["t_encode"], 3),
                       "gnnzvec_per_s": round(2.0 * nnz * info["s"] * (info["terms"] - 1) / el / 1e9,
                                              3)}
        if not args.no_early_rank:
            # the same rank with early termination (a library option, off by default): the sequence stops
            # once the sigma-basis beside it shows that the generator has stopped growing
            log("the same rank with early termination")
            try:
                bw.set_early_termination(True)
                t0 = time.perf_counter()
                r2, info2 = bw.rank_modp_dev(Ad, p, s, 1)
                torch.cuda.synchronize()
                el2 = time.perf_counter() - t0
                out["rank_early_termination"] = {
                    "rank": int(r2), "equals_planted": bool(r2 == A.planted_rank), "seconds": round(el2, 2),
                    "terms_computed": int(info2["terms"]), "full_length": int(info["terms"]),
                    "generator_order": int(info2["len"]), "t_sequence": round(info2["t_sequence"], 2)}
            except Exception as ex:  # reported, not fatal: the line above is the benchmark
                out["rank_early_termination"] = {"error": str(ex)}
            finally:
                bw.set_early_termination(False)
    del Ad
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, p, s, ge_mats=(("2000x1500", config1()), ("200000x150000", config2())))
    print(json.dumps(out), flush=True)


def gram_mode(args):
    """The symmetric projection U = V (Section 2.3) in Gram form at the default workload's size: two sequence terms
    per application of B (S_2k = W_k^T W_k, S_2k+1 = (A D_c W_k)^T D_r (A D_c W_k), W_k = B^k V; identities the paper
    does not use).  Steps of --terms terms from a kept matrix, then the whole rank with this projection."""
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config3

    s, p = 16, 65521
    log("generating the planted 2000000 x 1000000 matrix")
    A = config3()
    m, n, nnz = A.m, A.n, A.nnz
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    bw.time_step_kernels_dev(Ad, p, s, False, 5, with_plan=True)  # the autotuner's plan, cached
    M = bw.Matrix(Ad, p)
    U, V, dr, dc = draws(p, s, m, n, torch)
    terms = args.terms
    apps = (terms - 1 + 1) // 2
    for w in range(args.warmup):
        M.sequence_sym_dev(V, p, terms, dr, dc, gram=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        M.sequence_sym_dev(V, p, terms, dr, dc, gram=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    M.close()
    out = {"metric": METRIC, "mode": "symmetric_gram", "unit": "Gnnz·vec/s",
           "value": round(2.0 * nnz * s * apps * args.steps / el / 1e9, 3),
           "terms_per_s": round((terms - 1) * args.steps / el, 1), "ms_per_step": round(1000 * el / args.steps, 3),
           "applications_per_step": apps, "terms_per_step": terms, "steps": args.steps,
           "note": "two terms per application of B (Gram identities, not in the paper); value counts the sparse "
                   "products' multiply-adds",
           "config": {"workload": f"symmetric sequence (U = V) mod {p} of the planted {m} x {n} matrix "
                                  f"({nnz / 1e6:.1f} M non-zeros), block {s}"}}
    if not args.no_rank:
        log("rank with the symmetric projection in Gram form")
        t0 = time.perf_counter()
        r, info = bw.rank_modp_sym_dev(Ad, p, s, 1, gram=True)
        torch.cuda.synchronize()
        out["rank"] = {"rank": int(r), "planted_rank": int(A.planted_rank), "equals_planted": bool(r == A.planted_rank),
                       "seconds": round(time.perf_counter() - t0, 2), "t_sequence": round(info["t_sequence"], 2),
                       "t_sigma_after_sequence": round(info["t_sigma"], 3)}
    print(json.dumps(out), flush=True)


def profile_kernels_mode(args):
    """The kernels of one step of the default workload launched back to back (bwr_time_step_kernels_dev, after
    the autotuner), then a 256 MiB device copy: the command the counter summaries are taken on (the copy
    calibrates FETCH_SIZE and WRITE_SIZE)."""
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config3

    s, p = 16, 65521
    A = config3()
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
    src = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernels_us": [round(x, 3) for x in us], "plan": plan, "copy_bytes": 256 << 20,
                      "first": product_kernel(plan, 1, s, p)[0], "second": product_kernel(plan, 2, s, p)[0]}),
          flush=True)


def traffic_from(fetch_dir, write_dir, out_path, last=None):
    """profiles/traffic.json from two rocprofv3 --pmc runs of --profile-kernels (FETCH_SIZE, then WRITE_SIZE):
    per dispatch KiB of every sparse-product kernel, scaled by what the same counter reads for the 256 MiB
    device copy of that run (reads 256 MiB, writes 256 MiB).  With `last`, only the last `last` dispatches of
    each kernel count (the timing loop of the plan the autotuner chose, after its trials)."""
    import csv
    import glob

    def load(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                if row.get("Counter_Name") != counter:
                    continue
                k = row["Kernel_Name"]
                vals.setdefault(k, []).append((int(row.get("Dispatch_Id") or 0), float(row["Counter_Value"])))
        for k in vals:
            v = [x for _, x in sorted(vals[k])]
            vals[k] = v[-last:] if last else v
        return vals

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    big = 256 << 10  # KiB
    cf = max((v for k in copy for v in fetch[k]), default=0.0)
    cw = max((v for k in copy for v in write.get(k, [])), default=0.0)
    ff = big / cf if cf > 0 else 1.0
    fw = big / cw if cw > 0 else 1.0
    srcs = {"k_spmm_tiled": "paper_0704_2351_amd/csrc/spmm_tiled.hip",
            "k_spmm_split": "paper_0704_2351_amd/csrc/spmm.hip"}
    kernels = {}
    for k, v in fetch.items():
        short = k.replace("(anonymous namespace)::", "")
        short = short[5:] if short.startswith("void ") else short
        short = short.split("(")[0].split("::")[-1].strip()
        src = next((srcs[x] for x in srcs if short.startswith(x)), None)
        if src is None or k not in write:
            continue
        fk = sum(v) / len(v)
        wk = sum(write[k]) / len(write[k])
        kernels[short] = {"source": src, "dispatches": len(v), "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                          "bytes_per_launch": int(round(1024 * (fk * ff + wk * fw)))}
    rec = {"sources": {s: _source_digest(s) for s in sorted(set(srcs.values()))},
           "workload": "2000000 x 1000000 planted (37.2 M non-zeros), block 16, p = 65521",
           "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python3 bench.py --profile-kernels",
           "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
           "note": (f"average over the last {last} dispatches of each kernel (the chosen plan's timing loop)" if last
                    else "average over every dispatch of the kernel in the run (autotuner trials and timing loop)"),
           "kernels": dict(sorted(kernels.items()))}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def paper_rank_mode(args):
    """The whole rank of the 2 000 000 x 1 000 000 matrix (37 M non-zeros, block 16, p = 65521) from a CSR in
    device memory: encoding, all 2 + 2n/16 + 4 terms, the device sigma-basis beside the sequence, read-out."""
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config3

    s, p = 16, 65521
    log("generating the planted 2000000 x 1000000 matrix")
    A = config3()
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    log(f"rank mod {p}, block {s}: up to {bw.sequence_length(min(A.m, A.n), s) + 4} terms (one call, about "
        f"75 s), early termination {'on' if bw.get_early_termination() else 'off'}")
    t0 = time.perf_counter()
    r, info = bw.rank_modp_dev(Ad, p, s, 1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    work = 2.0 * A.nnz * info["s"] * (info["terms"] - 1)
    print(json.dumps({
        "metric": METRIC, "mode": "paper_rank", "unit": "Gnnz·vec/s", "value": round(work / el / 1e9, 3),
        "rank": int(r), "planted_rank": int(A.planted_rank), "rank_equals_planted": bool(r == A.planted_rank),
        "seconds": round(el, 2), "early_termination": bool(bw.get_early_termination()),
        "terms_computed": int(info["terms"]),
        "full_length": int(bw.sequence_length(min(A.m, A.n), s) + 4), "info": info, "higher_is_better": True, "n_gpus": 1, "dtype": "u16",
        "data": "synthetic planted-rank matrix (seeded)",
        "config": {"workload": f"planted {A.m} x {A.n}, rank {A.planted_rank}, {A.nnz / 1e6:.1f} M non-zeros, "
                               f"block {s}, p = {p}", "m": A.m, "n": A.n, "nnz": A.nnz}}), flush=True)


def serve_mode(args):
    """Seeded Poisson trace of rank requests through the continuous-batching server, then the same trace
    answered one request at a time by the single-matrix path (solves/s and latencies of both)."""
    import math

    import numpy as np

    import paper_0704_2351_amd as bw
    from workloads import CONFIG4_PRIMES, config_seed, planted

    rng = np.random.default_rng(config_seed(5, 999_999))
    trace = []
    t = 0.0
    for j in range(args.serve_count):
        t += rng.exponential(1.0 / args.serve_rate)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(args.serve_nmax)))))
        m = int(round(1.5 * n))
        r = int(round(n * rng.uniform(0.70, 0.95)))
        p = int(CONFIG4_PRIMES[rng.integers(0, 4)])
        trace.append((t, m, n, r, p, config_seed(5, j)))
    if args.serve_trials:
        bw.set_trials(args.serve_trials)
    log(f"generating {len(trace)} request matrices (n up to {max(x[2] for x in trace)})")
    mats = [planted(m, n, r, 9, sd) for (_, m, n, r, _, sd) in trace]
    srv = bw.Server(64 << 30, 128, 8)
    warm = srv.submit(mats[0], trace[0][4], 1)
    srv.wait(warm)
    srv.close()
    srv = bw.Server(64 << 30, 128, 8)
    tickets = []
    t0 = time.perf_counter()
    for (at, m, n, r, p, sd), A in zip(trace, mats):
        delay = at - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(A, p, 1))
    ranks, last = [], time.perf_counter()
    for i, tk in enumerate(tickets):
        ranks.append(srv.wait(tk))
        if time.perf_counter() - last > 20.0:  # progress of a long trace
            last = time.perf_counter()
            log(f"served {i + 1} of {len(tickets)} requests after {last - t0:.0f} s")
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    ok = all(rk == A.planted_rank for rk, A in zip(ranks, mats))
    # requests answered below their planted rank (the method's error is one-sided)
    short = [{"n": n, "p": p, "rank": rk, "planted": A.planted_rank}
             for (_, m, n, r, p, sd), A, rk in zip(trace, mats, ranks) if rk != A.planted_rank]
    log(f"served {st['completed']} requests: {st['solves_per_s']:.2f} solves/s, p50 {st['p50_ms']:.0f} ms")
    plain = {"plain_solves_per_s": None, "plain_p50_ms": None, "plain_p99_ms": None, "speedup_vs_plain": None,
             "ranks_equal_plain": None}
    if not args.serve_no_plain:
        # the same trace answered one request at a time by the single-matrix path, in arrival order: a request
        # waits for its arrival and for the one before it; rate and latencies are taken as the server takes them
        bw.rank_modp(mats[0], trace[0][4], 8, 1)
        plain_ranks, lat = [], []
        t0 = last = time.perf_counter()
        for (at, m, n, r, p, sd), A in zip(trace, mats):
            delay = at - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            plain_ranks.append(bw.rank_modp(A, p, 8, 1)[0])
            lat.append(time.perf_counter() - t0 - at)
            if time.perf_counter() - last > 20.0:
                last = time.perf_counter()
                log(f"plain: {len(lat)} of {len(trace)} requests after {last - t0:.0f} s")
        plain_span = (time.perf_counter() - t0) - trace[0][0]
        lat.sort()
        q = lambda f: 1000.0 * lat[min(len(lat) - 1, int(f * len(lat)))]
        plain_rate = len(trace) / plain_span
        log(f"plain: {plain_rate:.2f} solves/s, p50 {q(0.5):.0f} ms")
        plain = {"plain_solves_per_s": round(plain_rate, 4), "plain_p50_ms": round(q(0.5), 2),
                 "plain_p99_ms": round(q(0.99), 2), "speedup_vs_plain": round(st["solves_per_s"] / plain_rate, 3),
                 "ranks_equal_plain": plain_ranks == ranks}
    print(json.dumps({
        "metric": METRIC, "mode": "serving", "value": round(st["solves_per_s"], 4), "unit": "solves/s",
        "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2), "wall_s": round(wall, 2),
        "completed": st["completed"], "max_queue": st["max_queue"], "max_active": st["max_active"],
        **plain, "trials": bw.get_trials(), "short_ranks": short,
        "ranks_equal_planted": bool(ok), "higher_is_better": True, "n_gpus": 1, "dtype": "u32",
        "data": "synthetic planted-rank matrices (seeded), seeded Poisson arrivals",
        "config": {"workload": f"{args.serve_count} requests, Poisson {args.serve_rate}/s, n log-uniform "
                               f"1e3..{args.serve_nmax:g}, m = 1.5 n, rank 70-95 % of n, prime from {list(CONFIG4_PRIMES)}, "
                               f"block 8"}}), flush=True)


def rank_c2_mode(args):
    """Ranks of the 200 000 x 150 000 matrix (planted rank 140 000, block 8) at p = 65521 and p = 2^31 - 1 from a
    CSR in device memory, the two primes from two host threads; one step = both ranks."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import paper_0704_2351_amd as bw
    from workloads import config2

    s = 8
    primes = (65521, 2**31 - 1)
    log("generating the planted 200000 x 150000 matrix")
    A = config2()
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    pool = ThreadPoolExecutor(max_workers=len(primes))

    def solve(p):
        r, info = bw.rank_modp_dev(Ad, p, s, 1)
        if r != A.planted_rank:
            raise RuntimeError(f"rank {r} != planted {A.planted_rank} at p = {p}")
        return info

    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        list(pool.map(solve, primes))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        infos += list(pool.map(solve, primes))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    work = sum(2.0 * A.nnz * i["s"] * (i["terms"] - 1) for i in infos)
    rl = {}
    for p in primes:
        us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
        rl[str(p)] = roofline_entry(A, s, p, us, plan)
    print(json.dumps({"metric": METRIC, "mode": "rank_c2", "value": round(work / elapsed / 1e9, 3),
                      "unit": "Gnnz·vec/s", "solves_per_s": round(len(infos) / elapsed, 4), "steps": args.steps,
                      "ms_per_step": round(1000.0 * elapsed / args.steps, 2), "roofline": rl,
                      "config": {"workload": f"ranks of a planted {A.m} x {A.n} matrix (rank {A.planted_rank}, "
                                             f"{A.nnz / 1e6:.1f} M non-zeros), block {s}, p = 65521 and 2^31 - 1"}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--terms", type=int, default=513,
                    help="sequence terms per step of the default workload (terms - 1 applications of B)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rank", action="store_true", help="default workload: skip the whole rank after the steps")
    ap.add_argument("--no-early-rank", action="store_true",
                    help="default workload: skip the second whole rank, with early termination")
    ap.add_argument("--kernel-iters", type=int, default=50)
    ap.add_argument("--batch", action="store_true",
                    help="batched workload: planted matrices of the batched configuration, 4 primes, block 8; "
                         "solves/s of one batched call against the same ranks one call at a time")
    ap.add_argument("--batch-count", type=int, default=16, help="matrices of the batched configuration to use")
    ap.add_argument("--batch-retry", type=int, default=0,
                    help="agreement retry: up to this many further draws for a (matrix, prime) whose rank is below "
                         "the matrix's largest rank at the other primes (batched and one-at-a-time alike)")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: a seeded Poisson trace of rank requests through the server, and the "
                         "same trace one request at a time through the single-matrix path")
    ap.add_argument("--serve-count", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-nmax", type=float, default=2e4)
    ap.add_argument("--serve-trials", type=int, default=0,
                    help="independent draws per request (the largest rank kept); 0 keeps the library's setting")
    ap.add_argument("--serve-no-plain", action="store_true",
                    help="skip the one-request-at-a-time pass over the same trace")
    ap.add_argument("--paper-rank", action="store_true",
                    help="only the whole rank of the 2000000 x 1000000 matrix")
    ap.add_argument("--early", action="store_true",
                    help="early termination of the single-matrix ranks (--paper-rank, and the single-matrix "
                         "lanes of --batch and --serve): the sequence stops once the sigma-basis beside it "
                         "has converged")
    ap.add_argument("--rank-c2", action="store_true",
                    help="ranks of the 200000 x 150000 matrix at p = 65521 and 2^31 - 1 (one step = both)")
    ap.add_argument("--gram", action="store_true",
                    help="the symmetric projection in Gram form (two terms per application of B) at the default "
                         "workload's size, then its rank")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="the default workload's step kernels back to back, then a 256 MiB device copy (the "
                         "command the counter summaries are taken on)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc output folders of --profile-kernels "
                         "(FETCH_SIZE, then WRITE_SIZE), counting the last --kernel-iters dispatches of each "
                         "kernel (give the counter runs' value); needs no GPU")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is described, "
              f"not built", file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        rec = traffic_from(args.traffic_from[0], args.traffic_from[1], os.path.join(ROOT, "profiles", "traffic.json"),
                           last=args.kernel_iters)
        print(json.dumps({k: v for k, v in rec.items() if k != "kernels"}), flush=True)
        return

    import torch

    torch.cuda.set_device(0)
    if args.early:
        import paper_0704_2351_amd as bw

        bw.set_early_termination(True)
    if args.batch:
        return batch_mode(args)
    if args.serve:
        return serve_mode(args)
    if args.paper_rank:
        return paper_rank_mode(args)
    if args.rank_c2:
        return rank_c2_mode(args)
    if args.profile_kernels:
        return profile_kernels_mode(args)
    if args.gram:
        return gram_mode(args)
    return sequence_mode(args)


if __name__ == "__main__":
    main()
