#!/usr/bin/env python
"""Throughput of the tournament-pivoted FP64 LU on one MI355X.

One step = cfx_getrf + cfx_getrs (1 right-hand side) on a seeded N x N matrix
with N(0,1) entries, panel width v = 256 and L = 8 tournament leaves (the
plain FP64 blocked LU + solve workload at N = 32768).  The matrix is
restored from a pristine device copy before each step, outside the timed
interval; each step is timed with HIP events on the stream the library runs
on.  Flops are counted as 2N^3/3 (LU) + 2N^2 (the solve).

Printed: one JSON line with the metric, a roofline entry for the dominant
kernel (the FP64 MFMA Schur update, timed by the library's own per-phase
events) and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def hbm_report(n, v, L, launches):
    """Measured HBM bytes of the Schur launches (committed counter runs,
    per launch times the launches of one factorisation) against the
    Sec. 6 lower bound with P and M set for the XCD level and the compute
    unit level of the MI355X."""
    per = committed_traffic(n, v, L, launches=launches)
    xcd = lu_io_lower_bound_bytes(n, M_XCD)
    cu = lu_io_lower_bound_bytes(n, M_CU)
    out = {"bound_xcd_level_gb": round(xcd / 1e9, 2), "M_xcd_elements": M_XCD, "P_xcd": 8,
           "bound_cu_level_gb": round(cu / 1e9, 2), "M_cu_elements": M_CU, "P_cu": 256,
           "right_looking_c_traffic_gb": round(16.0 * sum((n - k - min(v, n - k)) ** 2
                                                          for k in range(0, n, v)) / 1e9, 2)}
    if per is not None:
        tot = per * launches
        out.update({"schur_measured_gb": round(tot / 1e9, 2),
                    "ratio_to_xcd_bound": round(tot / xcd, 3), "ratio_to_cu_bound": round(tot / cu, 3)})
    return out


def lu_flops_of_columns(n, k0, k1):
    """Exact LU flops of eliminating columns k0..k1-1: for column j,
    (n-j-1) divisions and 2 (n-j-1)^2 for the multiply-subtracts."""
    j = np.arange(k0, k1, dtype=np.float64)
    r = n - j - 1
    return float(np.sum(2.0 * r * r + r))


def committed_traffic(n, v, L, field="traffic_bytes_per_launch", launches=None, delay=1):
    """HBM bytes per launch of the FP64 Schur kernel from the committed
    rocprofv3 PMC summary of this workload (FETCH_SIZE and WRITE_SIZE runs
    on the Schur-only replay of the factorisation's launches, each counter
    calibrated by a plain copy), or None if there is none, the kernel's
    source changed since the counters were taken, or the factorisation now
    issues a different number of Schur launches."""
    import hashlib
    tag = "" if delay == 1 else f"_delay{delay}"
    path = os.path.join(ROOT, "profiles", f"schur_f64_kernel_traffic_n{n}_v{v}_L{L}{tag}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            key, _, val = line.partition(":")
            fields[key.strip()] = val.split()[0] if val.split() else ""
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_2010_05975_amd", "csrc", "schur_f64.hip"), "rb").read())
    if fields.get("kernel_source_sha256_16") != h.hexdigest()[:16] or field not in fields:
        return None
    if launches is not None and fields.get("launches") != str(launches):
        return None
    return float(fields[field])


# Fast memory of one processor at the two levels of the MI355X hierarchy
# (FP64 elements): an XCD (4 MiB L2 + 32 compute units x (160 KiB LDS +
# 512 KiB registers)) and a compute unit (LDS + registers).
# leaves of at least this many rows in every factorisation of the bench
# (cfx_lu_opts.min_leaf_rows; set from --min-leaf-rows)
MIN_LEAF = 0

M_XCD = (4 * 2**20 + 32 * (160 + 512) * 2**10) // 8
M_CU = ((160 + 512) * 2**10) // 8


def lu_io_lower_bound_bytes(n, M):
    """The parallel I/O lower bound of LU (Sec. 6), summed over the P
    processors of one level: P Q_{P,LU} >= (2N^3 - 6N^2 + 4N) / (3 sqrt(M))
    + N (N - 1) / 2 elements, 8 bytes each (P cancels)."""
    return 8.0 * ((2.0 * n ** 3 - 6.0 * n ** 2 + 4.0 * n) / (3.0 * np.sqrt(M)) + n * (n - 1) / 2.0)


def schur_replay(cfx, torch, n, v, chunk, seed, delay=1):
    """Only the Schur-complement launches of one lookahead factorisation at
    (n, v), in the library's order and shapes, on one stream: for each panel
    k, C = A[k+vb:, k+vb:] is updated from L21 = P[k+vb:, k:k+vb] and
    U12 = P[k:k+vb, k+vb:] (the strides and offsets of the factorisation;
    P is a second matrix that stays unchanged), first the next panel's
    columns, then the rest in `chunk`-column launches.  With delay d > 1
    the launches of the tile-stationary schedule instead: inside each batch
    of d panels the thin updates of panel k's columns and of its pivot rows
    (K = k - K0), and at the batch end the update of the trailing matrix
    with K = d v (the next panel's columns, then chunks).  No tournament
    kernels run, so a counter run sees these launches alone.  Returns
    (launches, algorithmic flops, seconds)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    P = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g) / 16.0
    stream = torch.cuda.current_stream()
    launches, flops = 0, 0.0

    def upd(r, c, m, nc, k0, K):
        nonlocal launches, flops
        if m <= 0 or nc <= 0 or K <= 0:
            return
        cfx.schur_update(P[r:r + m, k0:k0 + K], P[k0:k0 + K, c:c + nc], A[r:r + m, c:c + nc], stream=stream)
        launches += 1
        flops += 2.0 * m * nc * K

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for K0 in range(0, n, delay * v):
        kE = min(n, K0 + delay * v)
        for k in range(K0 + v, kE, v):          # thin updates inside the batch
            vb = min(v, n - k)
            upd(k, k, n - k, vb, K0, k - K0)
            upd(k, k + vb, vb, n - k - vb, K0, k - K0)
        m = n - kE
        if m <= 0:
            break
        vbn = min(v, m)
        for c0, cw in [(0, vbn)] + [(c0, min(chunk, m - c0)) for c0 in range(vbn, m, chunk)]:
            upd(kE, kE + c0, m, cw, K0, kE - K0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del A, P
    torch.cuda.empty_cache()
    return launches, flops, dt


def tslu_bench(cfx, torch, n, v, L, seed, reps=5):
    """The tournament alone (cfx_tslu: leaves and playoff rounds of one
    panel, no other work on the device) on N(0,1) panels of the heights the
    factorisation meets (rows = n - k), with the factorisation's leaf count,
    plus a single 2v-row node (one leaf of a merge's size): median time per
    call and per pivot step (HIP events).  Leaf counts follow the bench's
    minimum leaf height."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    def leaves_of(r):
        return min(L, max(1, -(-r // MIN_LEAF))) if MIN_LEAF else L
    cases = [(r, leaves_of(r)) for r in (n, (3 * n) // 4, n // 2, n // 4, n // 8, 4 * v)] + [(2 * v, 1), (v, 1)]
    for rows, leaves in cases:
        W = torch.randn(rows, v, dtype=torch.float64, device=dev, generator=g)
        work = cfx.workspace(rows, v, leaves, "fp64", 0, dev)
        times = []
        for it in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            cfx.tslu(W, v, leaves, work=work)
            e1.record()
            torch.cuda.synchronize()
            if it:
                times.append(e0.elapsed_time(e1))
        h = max(v, -(-rows // leaves))
        nl = -(-rows // h)
        levels = 1 + int(np.ceil(np.log2(nl))) if nl > 1 else 1
        ms = float(np.median(times))
        out.append({"rows": rows, "leaves": leaves, "leaf_rows": h, "levels": levels, "ms": round(ms, 4),
                    "us_per_pivot_step": round(1e3 * ms / (levels * v), 3)})
        log(f"tslu rows={rows} L={leaves}: {out[-1]}")
        del W, work
    return out


def cpu_baseline(A_host, n, v, L, panels):
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu baseline: oracle on the first {panels} panels, {threads} threads")
    t0 = time.perf_counter()
    O.getrf(A_host, v, L, npanels=panels)
    dt = time.perf_counter() - t0
    flops = lu_flops_of_columns(n, 0, min(n, panels * v))
    out = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "seconds": dt,
           "sample": f"first {panels} of {(n + v - 1) // v} panels of the same N={n} "
                     f"TP({v},{L}) factorisation (tournament, interchanges, both triangular "
                     f"solves, Schur update); flops = LU flops of those columns"}
    # the whole factorisation of this workload, timed when its stored
    # oracle result was written (tests/golden/make_c2_golden.py)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", f"c2_n{n}_seed0.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            if ("seconds" in z.files and int(z["v"]) == v and int(z["leaves"]) == L):
                sec = float(z["seconds"])
                out["full_factorisation"] = {"seconds": round(sec, 1), "threads": int(z["threads"]),
                                             "tflops": round(2.0 * n ** 3 / 3.0 / sec / 1e12, 5),
                                             "source": os.path.relpath(path, os.path.dirname(path) + "/../..")}
    return out


def masked_leg(cfx, torch, pristine, A_swapped, ipiv, n, v, L, lookahead, work, stream, reps=2):
    """cfx_getrf_masked (row masking, Sec. 7.3) on the same matrix and
    options as the timed steps: time per factorisation (HIP events, median
    of `reps` after one warm-up), the row-map phase against the interchange
    phase (the library's per-phase events), and whether the masked factors
    read through the row map equal the interchanged ones bit for bit."""
    dev = pristine.device
    M = torch.empty_like(pristine)
    rowmap = torch.empty(n, dtype=torch.int32, device=dev)
    ipm = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    times = []
    for it in range(reps + 1):
        M.copy_(pristine)
        torch.cuda.synchronize()
        if it == reps:
            cfx.profile_begin()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cfx.getrf_masked(M, v=v, leaves=L, lookahead=lookahead, work=work, ipiv=ipm, rowmap=rowmap, info=info,
                         min_leaf_rows=MIN_LEAF,
                         stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if it:
            times.append(e0.elapsed_time(e1))
    prof = cfx.profile_end()
    equal = bool(torch.equal(ipm, ipiv))
    rm = rowmap.long()
    for r0 in range(0, n, 4096):
        r1 = min(n, r0 + 4096)
        equal = equal and bool(torch.equal(M[rm[r0:r1]], A_swapped[r0:r1]))
    ms = float(np.median(times))
    out = {"getrf_ms": round(ms, 3), "getrf_tflops": round(2.0 * n ** 3 / 3.0 / (ms / 1e3) / 1e12, 3),
           "rowmap_phase_ms": round(prof["laswp_ms"], 3),
           "interchange_bytes_bound_gb": round(sum(2 * 2 * min(v, n - k) * n * 8 for k in range(0, n, v)) / 1e9, 2),
           "bitwise_equal_to_interchanged": equal}
    log(f"row masking: {out}")
    del M
    torch.cuda.empty_cache()
    return out


def delayed_leg(cfx, torch, pristine, A_ref, n, v, L, lookahead, work, stream, delays, reps=2):
    """The tile-stationary schedule (cfx_set_schur_delay) on the same matrix
    and options: time per factorisation (HIP events, median of `reps` after
    a warm-up), the Schur phase, the Frobenius residual of the factors, and
    the HBM bytes of its Schur launches from the committed counter runs of
    the matching replay (when present)."""
    out = {}
    M = torch.empty_like(pristine)
    ipiv = torch.empty(n, dtype=torch.int32, device=pristine.device)
    info = torch.empty(1, dtype=torch.int32, device=pristine.device)
    for d in delays:
        cfx.set_schur_delay(d)
        wk = cfx.workspace(n, v, L, "fp64", lookahead, pristine.device, min_leaf_rows=MIN_LEAF)
        times = []
        for it in range(reps + 1):
            M.copy_(pristine)
            torch.cuda.synchronize()
            if it == reps:
                cfx.profile_begin()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            cfx.getrf(M, v=v, leaves=L, lookahead=lookahead, work=wk, ipiv=ipiv, info=info, stream=stream,
                      min_leaf_rows=MIN_LEAF)
            e1.record(stream)
            torch.cuda.synchronize()
            if it:
                times.append(e0.elapsed_time(e1))
        prof = cfx.profile_end()
        cfx.set_schur_delay(1)
        ms = float(np.median(times))
        res = frob_residual(torch, pristine, M, _perm_of(ipiv.cpu().numpy()))
        r = {"getrf_ms": round(ms, 3), "getrf_tflops": round(2.0 * n ** 3 / 3.0 / (ms / 1e3) / 1e12, 3),
             "schur_ms": round(prof["schur_ms"], 3), "tslu_ms": round(prof["tslu_ms"], 3),
             "schur_launches": prof["schur_launches"], "frob_residual": res, "info": int(info.cpu()[0])}
        per = committed_traffic(n, v, L, launches=prof["schur_launches"], delay=d)
        if per is not None:
            tot = per * prof["schur_launches"]
            r["schur_hbm_gb"] = round(tot / 1e9, 2)
            r["ratio_to_xcd_bound"] = round(tot / lu_io_lower_bound_bytes(n, M_XCD), 3)
        out[f"delay_{d}"] = r
        log(f"tile-stationary d={d}: {r}")
        del wk
    del M
    torch.cuda.empty_cache()
    return out


def ir_leg(cfx, G, torch, n, v, L, conds, precs, seed, check_oracle):
    """Time-to-solution on A = H1 diag(s) H2 (8 seeded reflectors each side,
    s log-spaced to cond), 1 RHS: plain FP64 getrf + getrs, FP64 factors +
    GMRES-IR, and BF16 / FP16 / FP8 Schur updates + GMRES-IR, all to eta <= 5e-15
    (the refinement stops there; the plain solve's eta is reported)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {"n": n, "v": v, "leaves": L, "tol": 5e-15, "gmres_restart": 30, "gmres_tol": 1e-6,
           "max_outer": 20, "cases": []}
    work_lu = cfx.workspace(n, v, L, "fp64", 1, dev, min_leaf_rows=MIN_LEAF)
    for cond in conds:
        spec = G.householder_spec(n, cond, seed)
        A = G.householder_matrix(spec, device="cuda:0")
        b_host = G.rhs(n, 1, seed + 1)[:, 0]
        xs = G.householder_solution(spec, b_host)[:, 0]
        b = torch.from_numpy(b_host).to(dev)
        case = {"cond": cond}
        # plain FP64 solve
        F = A.clone()
        x = b.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ipiv, info = cfx.getrf(F, v=v, leaves=L, lookahead=1, work=work_lu, stream=stream, min_leaf_rows=MIN_LEAF)
        cfx.getrs(F, ipiv, x, stream=stream)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        r = b - A @ x
        eta_plain = float(r.abs().max() / (A.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()))
        case["fp64_solve"] = {"seconds": round(t_plain, 4), "eta_fp64_residual": eta_plain,
                              "forward_error": float(np.abs(x.cpu().numpy() - xs).max() / np.abs(xs).max())}
        del F
        torch.cuda.empty_cache()
        for prec in ["fp64"] + list(precs):
            nbytes = cfx.gesv_ir_buffer_size(n, 1, precision=prec, v=v, leaves=L, lookahead=1, min_leaf_rows=MIN_LEAF)
            work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            X = torch.empty_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, rep = cfx.gesv_ir(A, b, X=X, work=work, stream=stream, precision=prec, v=v, leaves=L, min_leaf_rows=MIN_LEAF,
                                 lookahead=1, tol=5e-15, max_outer=out["max_outer"],
                                 gmres_restart=out["gmres_restart"], gmres_tol=out["gmres_tol"])
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            xh = X.cpu().numpy()
            res = {"seconds": round(t, 4), "eta": rep["eta"], "eta_first": rep["eta_first"],
                   "outer": rep["outer"], "gmres_iterations": rep["inner"],
                   "converged": bool(rep["converged"]),
                   "forward_error": float(np.abs(xh - xs).max() / np.abs(xs).max()),
                   "speedup_vs_fp64_solve": round(t_plain / t, 3)}
            if check_oracle and prec != "fp64":
                from oracle import oracle as O
                res["eta_oracle"] = O.eta(A.cpu().numpy(), xh, b_host)
            case[f"{prec}_ir"] = res
            log(f"ir cond {cond:g} {prec}: {res}")
            del work
            torch.cuda.empty_cache()
        fp64_ir = case["fp64_ir"]["seconds"]
        for prec in precs:
            case[f"{prec}_ir"]["speedup_vs_fp64_ir"] = round(fp64_ir / case[f"{prec}_ir"]["seconds"], 3)
        out["cases"].append(case)
        del A
        torch.cuda.empty_cache()
    return out


def batched_leg(cfx, G, torch, count, seed, steps):
    """cfx_gesv_batched on `count` systems shaped like the batched workload:
    n ~ U{16..512}, nrhs ~ U{1..8}, A ~ N(0,1) + shift I with shift 0 or
    2 sqrt(n) (equal odds).  Entries come from a seeded device generator
    into two pooled buffers (one view per system, lda = n); a pristine copy
    restores them before every timed launch."""
    dev = torch.device("cuda:0")
    spec = G.batched_spec(count, seed)
    n = spec.sizes.astype(np.int64)
    r = spec.nrhs.astype(np.int64)
    offA = np.concatenate([[0], np.cumsum(n * n)])
    offB = np.concatenate([[0], np.cumsum(n * r)])
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    poolA0 = torch.randn(int(offA[-1]), dtype=torch.float64, device=dev, generator=gen)
    poolB0 = torch.randn(int(offB[-1]), dtype=torch.float64, device=dev, generator=gen)
    for i in range(count):   # diagonal shifts
        if spec.shift[i]:
            k = int(n[i])
            poolA0[int(offA[i]):int(offA[i + 1])].view(k, k).diagonal().add_(float(spec.shift[i]))
    poolA = poolA0.clone()
    poolB = poolB0.clone()
    As = [poolA[int(offA[i]):int(offA[i + 1])].view(int(n[i]), int(n[i])) for i in range(count)]
    Bs = [poolB[int(offB[i]):int(offB[i + 1])].view(int(n[i]), int(r[i])) for i in range(count)]
    batch = cfx.Batch(As, Bs)
    tuned = cfx.batched_tune()
    log(f"batched: tuned panel widths {tuned}")
    stream = torch.cuda.current_stream()
    times = []
    for it in range(steps + 1):
        poolA.copy_(poolA0)
        poolB.copy_(poolB0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = cfx.gesv_batched(batch, graph=True, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if it:   # the first call captures the graph: not timed
            times.append(e0.elapsed_time(e1))
    info_h = info.cpu().numpy()
    ms = float(np.median(times))
    lu_flops = float(np.sum(2.0 * n.astype(np.float64) ** 3 / 3.0))
    solve_flops = float(np.sum(2.0 * n.astype(np.float64) ** 2 * r))
    out = {"count": count, "seed": seed, "launch_ms": round(ms, 3), "launch_ms_all": [round(t, 3) for t in times],
           "lu_tflops": round(lu_flops / (ms / 1e3) / 1e12, 3),
           "lu_plus_solve_tflops": round((lu_flops + solve_flops) / (ms / 1e3) / 1e12, 3),
           "systems_per_s": round(count / (ms / 1e3), 1), "tuned_vb": tuned,
           "info_nonzero": int(np.count_nonzero(info_h)),
           "compulsory_bytes": float(np.sum(16.0 * n.astype(np.float64) ** 2 + 16.0 * n * r))}
    # spot check a few systems against the oracle (A restored from pristine)
    from oracle import oracle as O
    worst = 0.0
    for i in np.linspace(0, count - 1, 6).astype(int):
        k = int(n[i])
        A0 = poolA0[int(offA[i]):int(offA[i + 1])].view(k, k).cpu().numpy()
        B0 = poolB0[int(offB[i]):int(offB[i + 1])].view(k, int(r[i])).cpu().numpy()
        X = Bs[i].cpu().numpy()
        worst = max(worst, O.eta(A0, X, B0))
    out["spot_check_max_eta"] = worst
    log(f"batched: {out}")
    del poolA, poolB, poolA0, poolB0, As, Bs, batch
    torch.cuda.empty_cache()
    return out


def serve_leg(cfx, G, torch, rate, duration, seed, arena_gb, slots, nmax, pool=0, lowp_min_n=0,
              passes=("fp64", "bf16", "bf16_unrouted"), v=128, leaves=2, lookahead=0):
    """The serving loop on a seeded Poisson stream: arrivals at `rate` per
    second for `duration` seconds, n log-uniform in [64, nmax], cond
    log-uniform in [1e2, 1e8] (Householder construction), 1-16 right-hand
    sides, 30 % re-solves of an earlier request's factors (kept resident).
    The inputs are built on the device before the clock starts; requests are
    submitted at their arrival times from this thread.  One pass per entry
    of `passes`: "fp64" (FP64 factors), "bf16" (BF16 factors + GMRES-IR,
    target 5e-15, a request whose refinement does not reach it in 3 outer
    steps refactors in FP64; requests below `lowp_min_n` are routed to FP64
    factors) and "bf16_unrouted" (the same with every request in BF16).

    pool > 0 (long, fast streams whose distinct inputs would not fit in HBM):
    sizes are rounded to 24 log-spaced orders in [64, nmax] and each request
    takes one of `pool` matrices built for its order (each with its own
    condition number) and the first nrhs columns of one right-hand-side
    block per order; a re-solve uses its source's matrix."""
    dev = torch.device("cuda:0")
    reqs = G.serving_stream(rate, duration, seed, nmax=nmax)
    built = []
    if pool > 0:
        grid = np.unique(np.round(np.exp(np.linspace(np.log(64), np.log(nmax), 24))).astype(int))
        mats, rhs = {}, {}
        for gi, nn in enumerate(grid):
            nn = int(nn)
            mats[nn] = []
            for q in range(pool):
                gq = np.random.default_rng([seed, gi, q])
                cond = float(np.exp(gq.uniform(np.log(1e2), np.log(1e8))))
                mats[nn].append(G.householder_matrix(G.householder_spec(nn, cond, int(gq.integers(0, 2**31))),
                                                     device="cuda:0"))
            g = torch.Generator(device=dev)
            g.manual_seed(seed * 1000 + gi)
            rhs[nn] = torch.randn(nn, 16, dtype=torch.float64, device=dev, generator=g)
        choice = []
        for i, r in enumerate(reqs):
            if r.resolve_of >= 0:
                nn, q = choice[r.resolve_of]
            else:
                nn = int(grid[np.argmin(np.abs(np.log(grid) - np.log(r.n)))])
                q = r.seed % pool
            choice.append((nn, q))
            built.append((mats[nn][q], rhs[nn][:, :r.nrhs]))
        sizes = [c[0] for c in choice]
    else:
        for i, r in enumerate(reqs):
            if r.resolve_of < 0:
                A = G.householder_matrix(G.householder_spec(r.n, r.cond, r.seed % (2**31)), device="cuda:0")
            else:
                A = built[r.resolve_of][0]
            g = torch.Generator(device=dev)
            g.manual_seed(r.seed % (2**31))
            B = torch.randn(r.n, r.nrhs, dtype=torch.float64, device=dev, generator=g)
            built.append((A, B))
        sizes = [r.n for r in reqs]
    torch.cuda.synchronize()
    out = {"rate_per_s": rate, "duration_s": duration, "requests": len(reqs), "n_range": [64, nmax],
           "arena_gb": arena_gb, "slots": slots, "lowp_min_n": lowp_min_n,
           "factorisation": {"v": v, "leaves": leaves, "lookahead": lookahead},
           "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "default")}
    if pool > 0:
        out["inputs"] = f"pooled: orders rounded to {len(grid)} log-spaced sizes, {pool} matrices per size"
    nlog = max(50, len(reqs) // 20)
    for label in passes:
        prec = "fp64" if label == "fp64" else "bf16"
        kw = dict(precision=prec, v=v, leaves=leaves, lookahead=lookahead, tol=5e-15,
                  max_outer=4 if prec == "fp64" else 3, gmres_restart=20, gmres_tol=1e-6)
        srv = cfx.Server(int(arena_gb * (1 << 30)), max_slots=slots,
                         lowp_min_n=lowp_min_n if label == "bf16" else 0, **kw)
        tickets = [None] * len(reqs)
        xs = [None] * len(reqs)
        torch.cuda.synchronize()
        fid = {}
        results = [None] * len(reqs)
        t0 = time.perf_counter()
        pending = collections.deque()
        backlog_end = 0

        def collect(limit):
            # the oldest pending requests first (they finish roughly in order)
            k = 0
            while pending and k < limit:
                j = pending[0]
                res = srv.poll(tickets[j])
                if res is None:
                    break
                pending.popleft()
                results[j] = res
                xs[j] = None
                if reqs[j].resolve_of < 0:
                    fid[j] = res["factor_id"]
                k += 1

        for i, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.t_arrival:
                time.sleep(2e-4)
            A, B = built[i]
            xs[i] = torch.empty(sizes[i], r.nrhs, dtype=torch.float64, device=dev)
            if r.resolve_of >= 0 and r.resolve_of in fid:
                tickets[i] = srv.submit(A, B, xs[i], kind=cfx.RESOLVE, factor_id=fid[r.resolve_of])
            else:
                tickets[i] = srv.submit(A, B, xs[i], keep_resident=r.resolve_of < 0)
            pending.append(i)
            if (i + 1) % nlog == 0:
                log(f"serve {label}: submitted {i + 1}/{len(reqs)}, {len(pending)} pending")
            collect(64)
        backlog_end = len(pending)
        t_arrivals = time.perf_counter() - t0
        c = 0
        while pending:
            j = pending.popleft()
            results[j] = srv.wait(tickets[j], timeout=600)
            xs[j] = None
            if reqs[j].resolve_of < 0:
                fid[j] = results[j]["factor_id"]
            c += 1
            if c % nlog == 0:
                log(f"serve {label}: draining, {c}/{backlog_end} done")
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        del srv, xs                   # the arena goes before the next pass allocates its own
        torch.cuda.empty_cache()
        lat = np.array([r["t_done"] - r["t_submit"] for r in results])
        ok = [r for r in results if r["status"] == 0]
        new_flops = sum(2.0 * sizes[i] ** 3 / 3 for i, r in enumerate(results)
                        if r["status"] == 0 and not r["resident_hit"])
        solve_flops = sum(2.0 * sizes[i] ** 2 * reqs[i].nrhs for i, r in enumerate(results) if r["status"] == 0)
        etas = np.array([r["eta"] for r in ok])
        resolves = [i for i, q in enumerate(reqs) if q.resolve_of >= 0]
        hits = sum(1 for i in resolves if results[i]["resident_hit"])
        out[label] = {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                     "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                     "max_ms": round(1e3 * float(lat.max()), 3),
                     "wall_s": round(wall, 3),
                     "backlog_at_last_arrival": backlog_end,
                     "drain_s": round(wall - t_arrivals, 3),
                     "completed_per_s": round(len(ok) / wall, 1),
                     "lu_tflops": round(new_flops / wall / 1e12, 3),
                     "lu_plus_solve_tflops": round((new_flops + solve_flops) / wall / 1e12, 3),
                     "failed": len(results) - len(ok),
                     "eta_max": float(etas.max()) if len(etas) else None,
                     "eta_le_5e-15": int(np.sum(etas <= 5e-15)),
                     "resolves": len(resolves), "resident_hits": hits,
                     "fp64_fallbacks": sum(1 for r in ok if r.get("fallback", 0)),
                     "batched_requests": st["batched_requests"], "evictions": st["evictions"],
                     "bytes_peak_gb": round(st["bytes_peak"] / 2**30, 2)}
        log(f"serve {label}: {out[label]}")
    del built
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--v", type=int, default=256)
    ap.add_argument("--leaves", type=int, default=8)
    ap.add_argument("--min-leaf-rows", type=int, default=4096,
                    help="leaves of at least this many rows: a panel of r rows has min(L, ceil(r / R)) leaves "
                         "(0: L leaves for every panel)")
    ap.add_argument("--lookahead", type=int, default=1)
    ap.add_argument("--schur-wgs", type=int, default=None,
                    help="grid bound of the overlapped Schur launches (cfx_set_overlap_tuning; "
                         "-1 = by precision, the default; 0 = none)")
    ap.add_argument("--chunk", type=int, default=None, help="columns per overlapped Schur launch")
    ap.add_argument("--reserve-cus", type=int, default=None,
                    help="compute units kept free of the overlapped Schur launches (cfx_set_reserved_cus)")
    ap.add_argument("--one-stream", action="store_true",
                    help="issue the lookahead schedule on one stream (for PMC counter runs)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-masked", action="store_true", help="skip the row-masking leg")
    ap.add_argument("--delay", type=int, default=1,
                    help="panels per trailing update of the timed factorisation (tile-stationary schedule)")
    ap.add_argument("--delays", default="2,4",
                    help="delays of the tile-stationary leg (empty: skip it)")
    ap.add_argument("--cpu-panels", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ir", action="store_true", help="skip the mixed-precision IR leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--batched-count", type=int, default=20000)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-duration", type=float, default=6.0)
    ap.add_argument("--serve-nmax", type=int, default=8192)
    ap.add_argument("--serve-arena-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-pool", type=int, default=0,
                    help="pooled inputs: matrices per rounded order (0: one matrix per request)")
    ap.add_argument("--serve-lowp-min-n", type=int, default=32768,
                    help="the bf16 pass factors smaller requests in FP64 (measured crossover of BF16 + "
                         "GMRES-IR against the FP64 solve on this device)")
    ap.add_argument("--serve-passes", default="fp64,bf16,bf16_unrouted")
    ap.add_argument("--serve-only", action="store_true", help="run the serving leg alone")
    ap.add_argument("--serve-v", type=int, default=128, help="panel width of the served factorisations")
    ap.add_argument("--serve-leaves", type=int, default=2, help="tournament leaves of the served factorisations")
    ap.add_argument("--serve-lookahead", type=int, default=0)
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="hardware queues of the process (GPU_MAX_HW_QUEUES, set before the runtime starts; "
                         "the serving workers' streams share them)")
    ap.add_argument("--device-gen", action="store_true",
                    help="draw A and b on the device (seeded torch generator) instead of on the host; "
                         "used for the counter runs (no CPU baseline then)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--tslu-bench", action="store_true",
                    help="time the tournament alone (cfx_tslu) on panels of the factorisation's shapes and print "
                         "the results")
    ap.add_argument("--schur-replay", action="store_true",
                    help="run only the Schur-complement launches of one factorisation (one stream) "
                         "and print their statistics; for counter runs")
    ap.add_argument("--ir-conds", default="1e2,1e6,1e10")
    ap.add_argument("--ir-precs", default="bf16,fp16,fp8")
    ap.add_argument("--ir-oracle-check", action="store_true",
                    help="also evaluate eta of each IR result with the CPU oracle")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the factorisation runs on one GPU only (no sharding or collectives); "
              "a single N x N factorisation is one GPU's work. Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.hw_queues is not None:
        if not 1 <= args.hw_queues <= 32:
            raise SystemExit("--hw-queues takes 1..32")
        os.environ["GPU_MAX_HW_QUEUES"] = str(int(args.hw_queues))
    import torch
    import cfx_inputs as G
    from paper_2010_05975_amd import cfx

    n, v, L = args.n, args.v, args.leaves
    global MIN_LEAF
    MIN_LEAF = args.min_leaf_rows
    dev = torch.device("cuda:0")
    # every leg runs on a stream of its own (non-blocking, default priority):
    # launches on the legacy default stream synchronise with the library's
    # other streams and leave a gap of 30-60 us between dependent kernels
    torch.cuda.set_stream(torch.cuda.Stream(device=dev))
    if args.tslu_bench:
        print(json.dumps({"tslu_bench": tslu_bench(cfx, torch, n, v, L, args.seed)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serve": serve_leg(cfx, G, torch, args.serve_rate, args.serve_duration, args.seed + 13,
                                             args.serve_arena_gb, args.serve_slots, args.serve_nmax,
                                             args.serve_pool, args.serve_lowp_min_n,
                                             tuple(args.serve_passes.split(",")), args.serve_v,
                                             args.serve_leaves, args.serve_lookahead)}), flush=True)
        return
    if args.schur_replay:
        chunk = args.chunk or cfx.overlap_tuning()[1] or n     # 0: the whole rest in one launch
        launches, flops, dt = schur_replay(cfx, torch, n, v, chunk, args.seed, args.delay)
        out = {"schur_replay": {"n": n, "v": v, "chunk": chunk, "delay": args.delay, "launches": launches,
                                "flops": flops, "seconds": round(dt, 4), "tflops": round(flops / dt / 1e12, 3)}}
        if args.calibration_copy:
            src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps(out), flush=True)
        return
    if args.device_gen:
        log(f"generating A ({n}x{n}, N(0,1), device generator seed {args.seed})")
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        pristine = torch.randn(n, n, dtype=torch.float64, device=dev, generator=gen)
        pb = torch.randn(n, 1, dtype=torch.float64, device=dev, generator=gen)
        A_host = None
        args.no_cpu_baseline = True
    else:
        log(f"generating A ({n}x{n}, N(0,1), seed {args.seed})")
        A_host = G.normal_matrix(n, args.seed)
        b_host = G.rhs(n, 1, args.seed + 1)
        pristine = torch.from_numpy(A_host).to(dev)
        pb = torch.from_numpy(b_host).to(dev)
    A = torch.empty_like(pristine)
    B = torch.empty_like(pb)
    if args.delay != 1:
        cfx.set_schur_delay(args.delay)
    if args.reserve_cus is not None:
        cfx.set_reserved_cus(args.reserve_cus)
    work = cfx.workspace(n, v, L, "fp64", args.lookahead, dev, min_leaf_rows=MIN_LEAF)
    if args.schur_wgs is not None or args.chunk is not None or args.one_stream:
        w0, c0, _ = cfx.overlap_tuning()
        cfx.set_overlap_tuning(w0 if args.schur_wgs is None else args.schur_wgs,
                               c0 if args.chunk is None else args.chunk, 1 if args.one_stream else 0)
        log(f"overlap tuning {cfx.overlap_tuning()}")
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        A.copy_(pristine)
        B.copy_(pb)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        cfx.getrf(A, v=v, leaves=L, lookahead=args.lookahead, work=work, ipiv=ipiv, info=info, min_leaf_rows=MIN_LEAF,
                  stream=stream)
        e1.record(stream)
        cfx.getrs(A, ipiv, B, stream=stream)
        e2.record(stream)
        return e0, e1, e2

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    cfx.profile_begin()
    t0 = time.perf_counter()
    evs = []
    for i in range(args.steps):
        evs.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = cfx.profile_end()
    getrf_ms = sum(a.elapsed_time(b) for a, b, _ in evs) / args.steps
    getrs_ms = sum(b.elapsed_time(c) for _, b, c in evs) / args.steps
    ms = getrf_ms + getrs_ms
    log(f"timed {args.steps} steps: getrf {getrf_ms:.2f} ms, getrs {getrs_ms:.2f} ms")

    # correctness of the last step (outside the timed region): backward error
    # of the solve and ||P A - L U||_F / ||A||_F, the products formed by
    # torch's own FP64 matrix products (none of the library's kernels)
    with torch.no_grad():
        x = B[:, 0]
        r = pb[:, 0] - pristine @ x
        anorm = pristine.abs().sum(dim=1).max()
        eta = float(r.abs().max() / (anorm * x.abs().max() + pb.abs().max()))
        frob = frob_residual(torch, pristine, A, _perm_of(ipiv.cpu().numpy()))
        info_v = int(info.cpu()[0])
    log(f"eta {eta:.3e}, ||PA-LU||_F/||A||_F {frob:.3e}, info {info_v}")

    # the 64-right-hand-side solve with the same factors (outside the timed
    # steps): median of 3 launches, HIP events on the library's stream
    B64 = torch.randn(n, 64, dtype=torch.float64, device=dev, generator=torch.Generator(dev).manual_seed(2))
    t64 = []
    for _ in range(3):
        Bw = B64.clone()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        cfx.getrs(A, ipiv, Bw, stream=stream)
        f1.record(stream)
        torch.cuda.synchronize()
        t64.append(f0.elapsed_time(f1))
    getrs64_ms = sorted(t64)[1]
    del B64, Bw
    log(f"getrs with 64 right-hand sides: {getrs64_ms:.2f} ms")

    masked = None
    if not args.no_masked and args.delay == 1:
        masked = masked_leg(cfx, torch, pristine, A, ipiv, n, v, L, args.lookahead, work, stream)
    delayed = None
    if args.delays and args.delay == 1:
        delayed = delayed_leg(cfx, torch, pristine, A, n, v, L, args.lookahead, work, stream,
                              [int(x) for x in args.delays.split(",") if x])

    flops = 2.0 * n ** 3 / 3.0 + 2.0 * n * n
    value = flops / (ms / 1e3) / 1e12
    steps = max(args.steps, 1)
    launches_all = max(prof["schur_launches"], 1)      # over the timed steps
    launches = max(launches_all // steps, 1)            # per factorisation
    schur_avg_ms = prof["schur_ms"] / launches_all
    schur_avg_flops = prof["schur_flops"] / launches_all
    achieved = schur_avg_flops / (schur_avg_ms / 1e3) / 1e12 if schur_avg_ms > 0 else 0.0
    out = {
        "metric": "LU TFLOP/s & %MFMA peak at N=32768; IR speedup at 5e-15 bwd err; p50/p99",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 getrf+getrs, N={n}, v={v}, L={L} leaves"
                               + (f" of at least {MIN_LEAF} rows" if MIN_LEAF else "")
                               + f", A~N(0,1) seed {args.seed}, 1 RHS, lookahead={args.lookahead}"},
        "pct_fp64_peak": round(100 * value / FP64_PEAK_TFLOPS, 2),
        "getrf_ms": round(getrf_ms, 3),
        "getrs_ms": round(getrs_ms, 3),
        "getrs_64rhs_ms": round(getrs64_ms, 3),
        "getrf_tflops": round(2.0 * n ** 3 / 3.0 / (getrf_ms / 1e3) / 1e12, 3),
        "wall_s_timed_region": round(wall, 3),
        "phase_ms_per_step": {k: round(prof[k] / steps, 3)
                              for k in ("tslu_ms", "laswp_ms", "trsm_ms", "schur_ms")},
        "roofline": {"bound": "mfma", "kernel": "schur_f64_kernel",
                     "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": committed_traffic(n, v, L, launches=launches),
                     "hbm_read_bytes_per_launch": committed_traffic(n, v, L, "read_bytes_per_launch", launches),
                     "hbm_write_bytes_per_launch": committed_traffic(n, v, L, "write_bytes_per_launch",
                                                                     launches),
                     "avg_launch_ms": round(schur_avg_ms, 4),
                     "avg_launch_flops": schur_avg_flops},
        "hbm_vs_lower_bound": hbm_report(n, v, L, launches),
        "checks": {"eta": eta, "frob_residual": frob, "info": info_v},
    }
    if masked is not None:
        out["row_masking"] = masked
    if delayed is not None:
        out["tile_stationary"] = delayed
    del pristine, A, work
    torch.cuda.empty_cache()
    if not args.no_ir:
        conds = [float(c) for c in args.ir_conds.split(",") if c]
        precs = [p for p in args.ir_precs.split(",") if p]
        out["ir"] = ir_leg(cfx, G, torch, n, v, L, conds, precs, args.seed + 7, args.ir_oracle_check)
    if not args.no_batched:
        out["batched"] = batched_leg(cfx, G, torch, args.batched_count, args.seed + 11, max(args.steps, 1))
    if not args.no_serve:
        out["serve"] = serve_leg(cfx, G, torch, args.serve_rate, args.serve_duration, args.seed + 13,
                                 args.serve_arena_gb, args.serve_slots, args.serve_nmax, args.serve_pool,
                                 args.serve_lowp_min_n, tuple(args.serve_passes.split(",")), args.serve_v,
                                 args.serve_leaves, args.serve_lookahead)
    if args.calibration_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_host, n, v, L, args.cpu_panels)
    print(json.dumps(out), flush=True)


def frob_residual(torch, A0, LU, perm, block=2048):
    """||P A - L U||_F / ||A||_F on the device, block row by block row."""
    n = A0.shape[0]
    dperm = torch.from_numpy(np.ascontiguousarray(perm, dtype=np.int64)).to(A0.device)
    U = torch.triu(LU)
    num = torch.zeros((), dtype=torch.float64, device=A0.device)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        Lb = torch.tril(LU[r0:r1, :r1], diagonal=r0 - 1)
        idx = torch.arange(r1 - r0, device=A0.device)
        Lb[idx, idx + r0] = 1.0
        D = A0[dperm[r0:r1]] - Lb @ U[:r1]
        num += (D * D).sum()
        del Lb, D
    del U
    return float(torch.sqrt(num) / torch.linalg.norm(A0))


def _perm_of(ipiv):
    n = len(ipiv)
    perm = np.arange(n)
    for i in range(n):
        r = int(ipiv[i])
        if r != i:
            perm[i], perm[r] = perm[r], perm[i]
    return perm


if __name__ == "__main__":
    main()
