"""Benchmark: block Wiedemann rank mod p on one MI355X.

Workload (one "step"): the rank of the planted 200 000 x 150 000 integer matrix
(planted rank 140 000, ~2.6 M non-zeros) with block size 8, once at
p = 65521 and once at p = 2^31 - 1, from a CSR already resident in device
memory: encoding of A and A^T, the 2 + ceil(2n/s) + 4 sequence terms on the
GPU, the sigma-basis and the read-out on the host.  Every rank is checked
against the planted rank.

value = whole-job throughput in Gnnz.vec/s: the sparse multiply-adds of the
two products of every sequence step (2 nnz s per step), summed over the step's
solves, divided by the step's wall time.  The two primes are solved from two
host threads (one library stream each), so one prime's sigma-basis overlaps
the other prime's sequence on the device.

roofline: the dominant kernel is the second sparse product of a step (A^T
times the block, column scale and the fused U^T projection); its average
device time comes from HIP events around back-to-back launches on the stream
the kernel runs on (bwr_time_step_kernels_dev), its algorithmic bytes per
launch from the plain encoding (4 B index + 1 B value per non-zero, 4 B row
pointers, 4 B residues): B_launch = 4(n+1) + 5 nnz + 4 s (n + m).  traffic is
the measured memory traffic per launch from the committed counter summary
(profiles/traffic.json), null when that summary belongs to another revision
of the kernel source.

cpu_baseline: the oracle's plain sequence (scipy CSR products and numpy
reductions mod p) for a bounded number of steps of the same workload.
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


def cpu_baseline(A, p, s, target_s=15.0):
    """The oracle's sequence loop, timed on a bounded number of steps."""
    import numpy as np

    from oracle import sequence as oseq

    rng = np.random.default_rng(0)
    U = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    V = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    orc = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, dr, dc)
    W = V % p
    steps = 0
    t0 = time.perf_counter()
    while True:
        W = orc.apply(W)
        oseq.project(U, W, p)
        steps += 1
        el = time.perf_counter() - t0
        if el >= target_s or steps >= 400:
            break
    rate = 2.0 * A.nnz * s * steps / el / 1e9
    return {"value": rate, "unit": "Gnnz·vec/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the oracle's plain sequence (B = D_c A^T D_r A D_c applied to an n x {s} "
                      f"block, then U^T W mod {p}) on the same matrix, {el:.1f} s single-threaded"}


def kernel_traffic(W, G, esize, fused, kpass=0):
    """HBM bytes per launch of the row-split kernel instantiation <W, G, *, esize == 2, fused, residue
    type, kpass> from the committed counter summary, or None when the summary is missing, was taken on
    another revision of the kernel source, or does not hold that instantiation."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256") != digest:
        return None
    etype = "unsigned short" if esize == 2 else "unsigned int"
    pat = re.compile(rf"k_spmm_split<{W}, {G}, \d, {str(esize == 2).lower()}, {str(bool(fused)).lower()}, "
                     rf"{etype}, {kpass}>$")
    hits = [v for k, v in rec.get("kernels", {}).items() if pat.match(k)]
    return hits[0].get("bytes_per_launch") if len(hits) == 1 else None


def roofline_entry(A, s, p, us, plan):
    """Roofline of the dominant kernel of a step: the second sparse product (A^T times the
    n_outer x s block, column scale, fused U^T projection).  Algorithmic bytes per launch with the
    plain encoding: 4 B row pointers, 4 B index + 1 B value per non-zero, 4 B per residue read and
    written (U and the diagonals are regenerable and not counted)."""
    m, n, nnz = A.m, A.n, A.nnz
    bytes_second = 4 * (n + 1) + 5 * nnz + 4 * s * (m + n)
    bytes_first = 4 * (m + 1) + 5 * nnz + 4 * s * (n + m)
    ach = bytes_second / (us[1] * 1e-6) / 1e9
    ach1 = bytes_first / (us[0] * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": kernel_traffic(plan["W"], plan["G2"], plan["esize"], plan["fused"]),
            "kernel": f"k_spmm_split (second product: A^T Y, column scale, projection fused={bool(plan['fused'])}, "
                      f"W={plan['W']}, G={plan['G2']}, {plan['esize']}-byte residues), p = {p}",
            "avg_launch_us": round(us[1], 3), "bytes_per_launch": int(bytes_second),
            "first_product": {"achieved": round(ach1, 1), "frac": round(ach1 / PEAK_HBM_GBS, 4),
                              "avg_launch_us": round(us[0], 3), "bytes_per_launch": int(bytes_first),
                              "G": plan["G1"]}}


def result_line(A, s, primes, steps, warmup, elapsed, infos, us, plans):
    """The JSON record of a timed run: `infos` are the rank_modp infos of the timed solves, `us` and
    `plans` the per-prime kernel timings and launch plans."""
    nnz = A.nnz
    work = sum(2.0 * nnz * i["s"] * (i["len"] + i["check_terms"] - 1) for i in infos)
    seq_time = sum(i["t_sequence"] for i in infos)
    sigma_time = sum(i["t_sigma"] for i in infos)
    return {
        "metric": METRIC,
        "value": round(work / elapsed / 1e9, 3),
        "unit": "Gnnz·vec/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(1000.0 * elapsed / steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic planted-rank matrix (seeded); no dataset",
        "config": {"workload": f"rank mod p of a planted {A.m} x {A.n} sparse integer matrix "
                               f"(rank {A.planted_rank}, {nnz / 1e6:.1f} M non-zeros), block {s}, "
                               f"p = {' and '.join(str(p) for p in primes)}",
                   "m": A.m, "n": A.n, "nnz": nnz, "block": s, "primes": list(primes), "parallelism": "single GPU"},
        "solves_per_s": round(len(infos) / elapsed, 4),
        "sequence_gnnzvec_per_s": round(work / seq_time / 1e9, 3),
        "sequence_s_per_solve": round(seq_time / len(infos), 4),
        "sigma_basis_s_per_solve": round(sigma_time / len(infos), 4),
        "sigma_threads": infos[0]["sigma_threads"],
        "step_kernel_us": {str(p): [round(float(x), 3) for x in us[p]] for p in primes},
        "step_plan": {str(p): plans[p] for p in primes},
        "roofline": roofline_entry(A, s, primes[0], us[primes[0]], plans[primes[0]]),
    }


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
    log("batched: warmup on the smallest matrix")
    bw.rank_modp_batch(mats[:1], primes, 8, 1)
    t0 = time.perf_counter()
    ranks, info = bw.rank_modp_batch(mats, primes, 8, 1)
    tb = time.perf_counter() - t0
    ok_b = all(ranks[j, t] == A.planted_rank for j, A in enumerate(mats) for t in range(len(primes)))
    log(f"batched {tb:.2f} s, ranks ok: {ok_b}")
    t0 = time.perf_counter()
    plain_ok = True
    for j, A in enumerate(mats):
        for t, p in enumerate(primes):
            r, _ = bw.rank_modp(A, p, 8, 1)
            plain_ok &= (r == ranks[j, t])
        log(f"plain: matrix {j + 1}/{len(mats)} done")
    tp = time.perf_counter() - t0
    log(f"plain {tp:.2f} s, identical ranks: {plain_ok}")
    print(json.dumps({
        "metric": METRIC, "mode": "batched", "value": round(nsolves / tb, 4), "unit": "solves/s",
        "plain_solves_per_s": round(nsolves / tp, 4), "speedup_vs_plain": round(tp / tb, 3),
        "batched_gnnzvec_per_s": round(work / tb / 1e9, 3), "plain_gnnzvec_per_s": round(work / tp / 1e9, 3),
        "ranks_equal_planted": bool(ok_b), "ranks_equal_plain": bool(plain_ok), "solves": nsolves,
        "batch_info": info, "higher_is_better": True, "n_gpus": 1, "dtype": "u32",
        "data": "synthetic planted-rank matrices (seeded)",
        "config": {"workload": f"{len(mats)} of the 64 batched-configuration matrices (n log-uniform 5e3..2e5, "
                               f"m = 1.2-2.0 n, rank 70-95 % of n) x primes {list(primes)}, block 8",
                   "matrices": [[A.m, A.n, A.nnz] for A in mats]}}), flush=True)


def paper_scale_mode(args):
    """The 2 000 000 x 1 000 000 matrix (37 M non-zeros, block 16, p = 65521): kernel timings and roofline at a
    size far beyond the caches, the sequence rate over a bounded number of steps, and the device sigma-basis
    time at the full sequence length (on a random sequence of that length and block size)."""
    import numpy as np
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config3

    s, p = 16, 65521
    log("generating the planted 2000000 x 1000000 matrix")
    A = config3()
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    m, n, nnz = A.m, A.n, A.nnz
    log("kernel timing")
    us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
    bytes_second = 4 * (n + 1) + 5 * nnz + 4 * s * (m + n)
    bytes_first = 4 * (m + 1) + 5 * nnz + 4 * s * (n + m)
    L = bw.sequence_length(n, s)
    steps = args.paper_steps
    log(f"sequence of {steps} terms")
    rng = np.random.default_rng(0)
    U = torch.from_numpy(rng.integers(0, p, size=(n, s), dtype=np.int64).astype(np.int32)).cuda()
    V = torch.from_numpy(rng.integers(0, p, size=(n, s), dtype=np.int64).astype(np.int32)).cuda()
    dr = torch.from_numpy(rng.integers(1, p, size=m, dtype=np.int64).astype(np.int32)).cuda()
    dc = torch.from_numpy(rng.integers(1, p, size=n, dtype=np.int64).astype(np.int32)).cuda()
    bw.sequence_dev(Ad, U, V, p, 600, dr, dc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bw.sequence_dev(Ad, U, V, p, steps, dr, dc)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    per_step = ts / (steps - 1)
    log(f"device sigma-basis at L = {L}, s = {s} (random sequence)")
    S = torch.from_numpy(rng.integers(0, p, size=(L, s, s), dtype=np.int64).astype(np.int32)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bw.min_generator_dev(S, p)
    tsig = time.perf_counter() - t0
    work_step = 2.0 * nnz * s
    print(json.dumps({
        "metric": METRIC, "mode": "paper_scale", "unit": "Gnnz·vec/s",
        "value": round(work_step / per_step / 1e9, 3), "steps": steps, "per_step_us": round(per_step * 1e6, 2),
        "projected_sequence_s": round(per_step * (L + 3), 2), "sigma_basis_s": round(tsig, 2),
        "projected_rank_s": round(per_step * (L + 3) + tsig, 2),
        "step_kernel_us": [round(float(x), 3) for x in us], "step_plan": plan,
        "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                     "second_product": {"achieved": round(bytes_second / (us[1] * 1e-6) / 1e9, 1),
                                        "frac": round(bytes_second / (us[1] * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                                        "avg_launch_us": round(float(us[1]), 3), "bytes_per_launch": int(bytes_second)},
                     "first_product": {"achieved": round(bytes_first / (us[0] * 1e-6) / 1e9, 1),
                                       "frac": round(bytes_first / (us[0] * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
                                       "avg_launch_us": round(float(us[0]), 3), "bytes_per_launch": int(bytes_first)}},
        "higher_is_better": True, "n_gpus": 1, "dtype": "u16" if plan["esize"] == 2 else "u32",
        "data": "synthetic planted-rank matrix (seeded); random sequence for the sigma-basis timing",
        "config": {"workload": f"planted {m} x {n}, rank {A.planted_rank}, {nnz / 1e6:.1f} M non-zeros, block {s}, "
                               f"p = {p}", "m": m, "n": n, "nnz": nnz, "sequence_length": L}}), flush=True)


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
    log(f"rank mod {p}, block {s}: {bw.sequence_length(min(A.m, A.n), s) + 4} terms (one call, about 2.5 min)")
    t0 = time.perf_counter()
    r, info = bw.rank_modp_dev(Ad, p, s, 1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    work = 2.0 * A.nnz * info["s"] * (info["len"] + info["check_terms"] - 1)
    print(json.dumps({
        "metric": METRIC, "mode": "paper_rank", "unit": "Gnnz·vec/s", "value": round(work / el / 1e9, 3),
        "rank": int(r), "planted_rank": int(A.planted_rank), "rank_equals_planted": bool(r == A.planted_rank),
        "seconds": round(el, 2), "info": info, "higher_is_better": True, "n_gpus": 1, "dtype": "u16",
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
    ranks = [srv.wait(tk) for tk in tickets]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    ok = all(rk == A.planted_rank for rk, A in zip(ranks, mats))
    log(f"served {st['completed']} requests: {st['solves_per_s']:.2f} solves/s, p50 {st['p50_ms']:.0f} ms")
    # the same trace answered one request at a time by the single-matrix path, in arrival order: a request
    # waits for its arrival and for the one before it; rate and latencies are taken as the server takes them
    bw.rank_modp(mats[0], trace[0][4], 8, 1)
    plain_ranks, lat = [], []
    t0 = time.perf_counter()
    for (at, m, n, r, p, sd), A in zip(trace, mats):
        delay = at - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        plain_ranks.append(bw.rank_modp(A, p, 8, 1)[0])
        lat.append(time.perf_counter() - t0 - at)
    plain_span = (time.perf_counter() - t0) - trace[0][0]
    lat.sort()
    q = lambda f: 1000.0 * lat[min(len(lat) - 1, int(f * len(lat)))]
    plain_rate = len(trace) / plain_span
    log(f"plain: {plain_rate:.2f} solves/s, p50 {q(0.5):.0f} ms")
    print(json.dumps({
        "metric": METRIC, "mode": "serving", "value": round(st["solves_per_s"], 4), "unit": "solves/s",
        "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2), "wall_s": round(wall, 2),
        "completed": st["completed"], "max_queue": st["max_queue"], "max_active": st["max_active"],
        "plain_solves_per_s": round(plain_rate, 4), "plain_p50_ms": round(q(0.5), 2),
        "plain_p99_ms": round(q(0.99), 2), "speedup_vs_plain": round(st["solves_per_s"] / plain_rate, 3),
        "ranks_equal_plain": plain_ranks == ranks,
        "ranks_equal_planted": bool(ok), "higher_is_better": True, "n_gpus": 1, "dtype": "u32",
        "data": "synthetic planted-rank matrices (seeded), seeded Poisson arrivals",
        "config": {"workload": f"{args.serve_count} requests, Poisson {args.serve_rate}/s, n log-uniform "
                               f"1e3..{args.serve_nmax:g}, m = 1.5 n, rank 70-95 % of n, prime from {list(CONFIG4_PRIMES)}, "
                               f"block 8"}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=50)
    ap.add_argument("--batch", action="store_true",
                    help="batched workload: planted matrices of the batched configuration, 4 primes, block 8; "
                         "solves/s of one batched call against the same ranks one call at a time")
    ap.add_argument("--batch-count", type=int, default=16, help="matrices of the batched configuration to use")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: a seeded Poisson trace of rank requests through the server, and the "
                         "same trace one request at a time through the single-matrix path")
    ap.add_argument("--serve-count", type=int, default=40)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-nmax", type=float, default=2e4)
    ap.add_argument("--paper-scale", action="store_true",
                    help="the 2000000 x 1000000 matrix (37 M non-zeros), block 16: kernel roofline, sequence rate "
                         "over --paper-steps terms, device sigma-basis time at the full length")
    ap.add_argument("--paper-steps", type=int, default=3000)
    ap.add_argument("--paper-rank", action="store_true",
                    help="the whole rank of the 2000000 x 1000000 matrix (about 2.5 minutes of GPU time)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel timing loop at p = 65521 plus a 256 MiB device copy "
                         "(a plain copy kernel of known size, for calibrating memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is described, "
              f"not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0704_2351_amd as bw
    from workloads import config2

    torch.cuda.set_device(0)
    if args.batch:
        return batch_mode(args)
    if args.serve:
        return serve_mode(args)
    if args.paper_rank:
        return paper_rank_mode(args)
    if args.paper_scale:
        return paper_scale_mode(args)
    s = 8
    primes = (65521, 2**31 - 1)
    log("generating the planted 200000 x 150000 matrix")
    A = config2()
    nnz = A.nnz
    Ad = bw.csr_to_device(A, "cuda:0")
    torch.cuda.synchronize()
    planted = A.planted_rank

    if args.kernels_only:
        out = {}
        for p in primes:
            us, plan = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
            out[str(p)] = {"kernels_us": [round(x, 3) for x in us], "plan": plan}
        src = torch.empty(64 << 20, dtype=torch.int32, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_bytes"] = 256 << 20
        print(json.dumps(out), flush=True)
        return

    from concurrent.futures import ThreadPoolExecutor

    pool = ThreadPoolExecutor(max_workers=len(primes))

    def solve(p):
        r, info = bw.rank_modp_dev(Ad, p, s, 1)
        if r != planted:
            raise RuntimeError(f"rank {r} != planted {planted} at p = {p}")
        return info

    def one_step():
        # one host thread per prime: each runs on its own library stream, so one prime's
        # sigma-basis overlaps the other prime's sequence on the device
        return list(pool.map(solve, primes))

    for w in range(args.warmup):
        log(f"warmup {w + 1}/{args.warmup}")
        one_step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    all_infos = []
    for k in range(args.steps):
        all_infos += one_step()
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # live kernel timing for the roofline (HIP events on the stream the kernels run on)
    us, plans = {}, {}
    for p in primes:
        us[p], plans[p] = bw.time_step_kernels_dev(Ad, p, s, False, args.kernel_iters, with_plan=True)
    torch.cuda.synchronize()
    out = result_line(A, s, primes, args.steps, args.warmup, elapsed, all_infos, us, plans)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sequence)")
        out["cpu_baseline"] = cpu_baseline(A, primes[0], s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
