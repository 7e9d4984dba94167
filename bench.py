"""Benchmark: FP64 SpMV effective bandwidth on the largest FEM matrix, and
the Jacobi-PCG solves (FP64, mixed precision, multi-RHS, batched, served)
on the 3-D elasticity system.

One timed step is one FP64 SpMV y' = A' x' in the layout numbering (the
product the CG iteration performs) on the largest FEM matrix of the sparsity
sweep: Q1 hexahedral elasticity, 87^3 nodes, natural numbering, full
Neumann (1,975,509 rows, 156,365,811 non-zeros).  ``value`` is the
effective bandwidth on the algorithmic-bytes model 12 nnz + 8 n_cols +
8 n_rows (matrix values and int32 column indices once, x once, y once),
with the inputs resident in HBM, timed with HIP events over K back-to-back
launches on the launch stream.  The same JSON line reports the cold-cache
product (after a 1 GiB write, whose dirty lines are written back during the
timed launch, and after a 1 GiB read), the CPU oracle on the same matrix, and the 3-D elasticity system
(P1 Kuhn tetrahedra, 64^3 nodes, random node numbering, x = 0 face clamped:
774,144 rows, 33,967,818 non-zeros): its product, Jacobi-PCG to a true
relative residual of 1e-8 in FP64 and with FP32 / BF16 refinement, the
stream-ordered, multi-right-hand-side and batched solves, element assembly,
and the serving experiment.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Counter profile of the timed kernel (HBM bytes per launch) and the sources
# that determine that kernel's code and data layout: the profile is used only
# while they are unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles",
                               "spmv_f64_q1hex_elasticity87_traffic.md")
KERNEL_SOURCES = ["paper_1501_00324_amd/csrc/kernels.hip",
                  "paper_1501_00324_amd/csrc/device.h",
                  "paper_1501_00324_amd/csrc/layout.h",
                  "paper_1501_00324_amd/csrc/layout.cpp"]
CALIB_DOUBLES = 1 << 27          # plain copy of 1 GiB for counter scaling


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the timed product from the committed counter
    profile (FETCH_SIZE and WRITE_SIZE, each scaled by the counter's reading
    for a plain copy of known size), or None when the profile is missing or
    was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)\s*$", text, re.M))
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return int(round(float(vals["traffic_bytes_per_launch"])))
    except (KeyError, ValueError):
        return None


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def bench_small_batch(fs, W, oracle, d, torch, m=64):
    """m small systems (2-D Poisson, 48x48 nodes, each its own jittered
    mesh and right-hand side): one at a time vs. all m in shared launches."""
    mats, Ms, bs = [], [], []
    for i in range(m):
        A = W.poisson_2d_p1(48, seed=(4, i), bc="all")
        mats.append(A)
        Ms.append(fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows,
                                A.n_cols))
        bs.append(d(W.random_vector(A.n_rows, 4, W.BVEC, i)))
    fs.cg_solve(Ms[0], bs[0], precond=fs.PC_JACOBI)          # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs1 = [fs.cg_solve(M, b, precond=fs.PC_JACOBI)[0] for M, b in
           zip(Ms, bs)]
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    fs.cg_solve_batch(Ms[:2], bs[:2], precond=fs.PC_JACOBI)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xsb, infos = fs.cg_solve_batch(Ms, bs, precond=fs.PC_JACOBI)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    same = all(torch.equal(a.reshape(-1), bb.reshape(-1))
               for a, bb in zip(xs1, xsb))

    def worst_relres(xs):
        return max(float(np.linalg.norm(bs[i].cpu().numpy() - oracle.spmv(
            mats[i], xs[i].reshape(-1).cpu().numpy())) /
            np.linalg.norm(bs[i].cpu().numpy())) for i in range(m))

    worst = worst_relres(xsb)
    # one workgroup per system, whole solve in one launch: the first call
    # times the three workgroup sizes and keeps the fastest
    t0 = time.perf_counter()
    fs.cg_solve_batch_wg(Ms, bs, precond=fs.PC_JACOBI)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    t_wg, xsw, infw = None, None, None
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs_, inf_ = fs.cg_solve_batch_wg(Ms, bs, precond=fs.PC_JACOBI)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        if t_wg is None or t < t_wg:
            t_wg, xsw, infw = t, xs_, inf_
    by_threads = {}
    for th in (256, 512, 1024):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs_, _ = fs.cg_solve_batch_wg(Ms, bs, precond=fs.PC_JACOBI,
                                      wg_threads=th)
        torch.cuda.synchronize()
        by_threads[str(th)] = {
            "solves_per_s": m / (time.perf_counter() - t0),
            "bitwise_equal": all(torch.equal(a, c) for a, c in
                                 zip(xs_, xsw))}
    xa, _ = fs.cg_solve_batch_wg(Ms[:1], bs[:1], precond=fs.PC_JACOBI)
    wg = {"solves_per_s": m / t_wg, "speedup_vs_batched": t_b / t_wg,
          "speedup_vs_one_at_a_time": t_one / t_wg,
          "first_call_with_tuning_ms": t_tune * 1e3,
          "by_threads": by_threads,
          "device_ms_max": max(i["ms"] for i in infw),
          "iters_max": max(i["iters"] for i in infw),
          "all_converged": all(i["status"] == 0 for i in infw),
          "relres_oracle_worst": worst_relres(xsw),
          "bitwise_equal_to_alone": bool(torch.equal(xa[0], xsw[0]))}
    for M in Ms:
        M.close()
    return {"systems": m, "rows_each": mats[0].n_rows,
            "one_at_a_time_solves_per_s": m / t_one,
            "batched_solves_per_s": m / t_b,
            "speedup": t_one / t_b, "bitwise_equal_to_alone": bool(same),
            "relres_oracle_worst": worst,
            "iters_max": max(i["iters"] for i in infos),
            "one_workgroup_per_system": wg}


def serving_pool(W, n_mats=6):
    """P1-tet Laplacian (all boundary nodes removed) or elasticity (x = 0
    face clamped) meshes with random numbering, row counts log-uniform in
    [5e3, 5e5]."""
    g = W.rng(4, W.SIZES, 0)
    pool = []
    for i in range(n_mats):
        rows = float(np.exp(g.uniform(np.log(5e3), np.log(5e5))))
        if g.uniform() < 0.5:
            n = max(4, int(round(rows ** (1 / 3))) + 2)
            A = W.tet_p1(n, "laplace", seed=(4, 100 + i), bc="all",
                         permute=True)
        else:
            n = max(4, int(round((rows / 3) ** (1 / 3))))
            A = W.tet_p1(n, "elastic", seed=(4, 100 + i), bc="x0",
                         permute=True)
        pool.append(A)
    return pool


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_serving(fs, W, oracle, d, torch, n_req=32, lam_factors=(1, 2, 4)):
    """Poisson arrivals of CG requests (pool matrix, k ~ U{1..16} right-hand
    sides ~ U(-1,1)).  Baseline: the same requests served one at a time
    (FIFO, each request by cg_solve_multi, service times measured, queueing
    computed from the arrival times).  Server: live continuous batching."""
    pool = serving_pool(W)
    Ms = [fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows, A.n_cols)
          for A in pool]
    g = W.rng(4, W.ARRIVALS, 0)
    reqs = []
    for i in range(n_req):
        mi = int(g.integers(0, len(pool)))
        k = int(g.integers(1, 17))
        reqs.append((mi, k, d(W.random_vector(pool[mi].n_rows, 4, W.BVEC,
                                              1000 + i, k=k))))
    # warm every matrix once
    for M in Ms:
        fs.cg_solve(M, torch.ones(M.n_rows, dtype=torch.float64,
                                  device="cuda"), maxit=2, check=False)
    service, alone = [], []
    for mi, k, B in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, _ = fs.cg_solve_multi(Ms[mi], B, precond=fs.PC_JACOBI)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        alone.append(X)
    total_k = sum(k for _, k, _ in reqs)
    mu = n_req / sum(service)                   # requests per second
    log("serving: %d requests served one at a time in %.1f s"
        % (n_req, sum(service)))
    out = {"pool_rows": [A.n_rows for A in pool],
           "pool_nnz": [A.nnz for A in pool], "requests": n_req,
           "rhs_total": total_k,
           "one_at_a_time_requests_per_s": mu,
           "one_at_a_time_solves_per_s": total_k / sum(service),
           "by_lambda": []}
    same_all = True
    for f in lam_factors:
        lam = f * mu
        gaps = g.exponential(1.0 / lam, n_req)
        arrivals = np.cumsum(gaps) - gaps[0]
        # FIFO single-server baseline on the measured service times
        finish, lat_b = 0.0, []
        for a, s in zip(arrivals, service):
            finish = max(finish, a) + s
            lat_b.append(finish - a)
        srv = fs.Server(precond=fs.PC_JACOBI, check_every=16)
        t0 = time.perf_counter()
        xs = {}
        done = []
        for i, (mi, k, B) in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[i]:
                done += srv.poll()
                time.sleep(0.0002)
            rid, X = srv.submit(Ms[mi], B)
            xs[rid] = (i, X)
        done += srv.drain()
        makespan = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat_s = [dd["info"]["ms"] / 1e3 for dd in done]
        ok = all(dd["info"]["status"] == fs.FS_OK for dd in done)
        same = all(torch.equal(xs[dd["req_id"]][1], alone[xs[dd["req_id"]][0]])
                   for dd in done)
        same_all &= same
        log("serving: lambda = %.2f mu done in %.1f s" % (f, makespan))
        out["by_lambda"].append({
            "lambda_over_mu": f, "lambda_req_per_s": lam,
            "server": {"p50_ms": percentile(lat_s, 50) * 1e3,
                       "p99_ms": percentile(lat_s, 99) * 1e3,
                       "solves_per_s": total_k / makespan,
                       "requests_per_s": n_req / makespan,
                       "all_converged": ok, "peak_active": st["peak_active"],
                       "peak_bytes": st["peak_bytes"]},
            "one_at_a_time": {"p50_ms": percentile(lat_b, 50) * 1e3,
                              "p99_ms": percentile(lat_b, 99) * 1e3,
                              "solves_per_s": total_k / max(
                                  finish, arrivals[-1])}})
    out["bitwise_equal_to_alone"] = bool(same_all)
    # true residuals of one served run, recomputed by the oracle
    worst = 0.0
    for (mi, k, B), X in zip(reqs, alone):
        Bh, Xh = B.cpu().numpy(), X.cpu().numpy()
        for c in range(k):
            worst = max(worst, float(np.linalg.norm(
                Bh[:, c] - oracle.spmv(pool[mi], Xh[:, c].copy())) /
                np.linalg.norm(Bh[:, c])))
    out["relres_oracle_worst"] = worst
    for M in Ms:
        M.close()
    return out



def event_times_us(torch, fn, reps, stream, flush=None):
    """Per-call device times (HIP events on the launch stream) of reps calls
    of fn; flush() runs before each call (cold caches) outside the pair."""
    out = []
    for _ in range(reps):
        if flush is not None:
            flush()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1) * 1e3)
    return out


def dist(v):
    return {"median": percentile(v, 50), "p10": percentile(v, 10),
            "p90": percentile(v, 90), "n": len(v)}


def back_to_back_us(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / steps


def measure_matrix(fs, oracle, torch, A, d, steps, warmup, stream,
                   cold=True, extras=True):
    """Layout build, parity of the timed launch against the oracle on every
    row, warm (back to back, and per call) and cold product times, and the
    plain CSR product without a layout."""
    dev = torch.device("cuda:0")
    rp, ci, va = d(A.rowptr), d(A.col), d(A.val)
    M = fs.csr_create(rp, ci, va, A.n_rows, A.n_cols)
    info = fs.csr_info(M)
    import workloads as W
    x = W.random_vector(A.n_cols, 1, W.XVEC)
    perm = fs.csr_get_perm(M)
    xp = d(x[perm])
    yp = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    fs.spmv_perm(M, xp, yp)
    torch.cuda.synchronize()
    yo = oracle.spmv(A, x)[perm]
    err = np.abs(yp.cpu().numpy() - yo)
    ok = bool(np.all(err <= 1e-12 * oracle.spmv_abs(A, x)[perm]))
    bytes_alg = 12 * A.nnz + 8 * A.n_cols + 8 * A.n_rows
    fn = lambda: fs.spmv_perm(M, xp, yp)
    t_b2b = back_to_back_us(torch, fn, steps, warmup, stream)
    warm = event_times_us(torch, fn, 20, stream)
    out = {"n_rows": A.n_rows, "nnz": A.nnz, "parity_all_rows": ok,
           "max_abs_err": float(err.max()) if len(err) else 0.0,
           "us": t_b2b, "gbs": bytes_alg / (t_b2b * 1e-6) / 1e9,
           "warm_us": dist(warm),
           "slots": info["slots"], "padding": info["padding"],
           "groups_by_lanes": info["groups_by_lanes"],
           "reorder": info["reorder"], "t_build_ms": info["t_build_ms"]}
    out["frac"] = out["gbs"] / HBM_PEAK_GBS
    if cold:
        # two flushes of the caches (L2, MALL) and the TLB between launches:
        # writing 1 GiB (the reported cold figure; the caches are then full of
        # dirty lines, and writing them back to HBM falls inside the timed
        # launch), and reading 1 GiB (clean lines: only the product's own
        # misses are timed)
        junk = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        c = event_times_us(torch, fn, 20, stream,
                           flush=lambda: junk.fill_(1.0))
        out["cold_us"] = dist(c)
        out["cold_gbs"] = bytes_alg / (out["cold_us"]["median"] * 1e-6) / 1e9
        cr = event_times_us(torch, fn, 20, stream,
                            flush=lambda: junk.sum())
        out["cold_read_flush_us"] = dist(cr)
        out["cold_read_flush_gbs"] = bytes_alg / (
            out["cold_read_flush_us"]["median"] * 1e-6) / 1e9
        del junk
    if not extras:
        return M, out
    # plain CSR product (no layout) in caller numbering
    xd = d(x)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    fs.spmv_csr(rp, ci, va, A.n_rows, A.n_cols, xd, y)
    torch.cuda.synchronize()
    ok_csr = bool(np.all(np.abs(y.cpu().numpy() - oracle.spmv(A, x)) <=
                         1e-12 * oracle.spmv_abs(A, x)))
    t_csr = back_to_back_us(torch, lambda: fs.spmv_csr(
        rp, ci, va, A.n_rows, A.n_cols, xd, y), steps, warmup, stream)
    out["csr_plain"] = {"us": t_csr,
                        "gbs": bytes_alg / (t_csr * 1e-6) / 1e9,
                        "parity_all_rows": ok_csr}
    # the paper's alpha: products after which reordering the values into
    # the layout (per Newton step, through the stored map) has paid for
    # itself against the plain CSR product
    t_ref = back_to_back_us(torch, lambda: fs.csr_update_values(M, va), 10,
                            2, stream)
    gain = t_csr - t_b2b
    out["value_refresh_us"] = t_ref
    out["alpha_value_reorder"] = t_ref / gain if gain > 0 else None
    # the same for the one-time structural build of the layout (host)
    out["break_even_products"] = (info["t_build_ms"] * 1e3 / gain
                                  if gain > 0 else None)
    out["structural_build"] = build_times(fs, A, rp, ci, va, M, gain)
    return M, out


def build_times(fs, A, rp, ci, va, M, gain, reps=2):
    """The structural layout build on the host vs with its per-non-zero
    phases on the device (best of `reps` builds each, after the first build
    of the process), with the default row order and with the caller's
    numbering kept; the host layout is checked bit for bit against the
    default (device) build."""
    ref = fs.csr_get_layout(M)              # the default (device) build
    res = {"identical_layout": True,
           "device_ran": fs.csr_info(M)["build"] == fs.BUILD_DEVICE}
    for tag, extra in (("", {}), ("_no_reorder", {"reorder": fs.REORDER_NONE})):
        for name, b in (("host", fs.BUILD_HOST), ("device", fs.BUILD_DEVICE)):
            ts = []
            for _ in range(reps):
                N = fs.csr_create(rp, ci, va, A.n_rows, A.n_cols, build=b,
                                  **extra)
                ts.append(fs.csr_info(N)["t_build_ms"])
                if b == fs.BUILD_HOST and not extra:
                    lay = fs.csr_get_layout(N)
                    res["identical_layout"] &= all(
                        (ref[k] is None and lay[k] is None) or
                        (ref[k] is not None and lay[k] is not None and
                         np.array_equal(ref[k], lay[k])) for k in ref)
                N.close()
            res["%s%s_ms" % (name, tag)] = min(ts)
    res["break_even_products_device"] = (res["device_ms"] * 1e3 / gain
                                         if gain > 0 else None)
    return res


def bench_autotune(fs, oracle, torch, A, d, steps, warmup, stream,
                   default_us):
    """The layout autotuner on one matrix: the lanes-per-row and
    slots-per-load shapes it times, the one it keeps, and that layout's
    product against the default layout's (every output row checked against
    the oracle)."""
    import workloads as W
    t0 = time.perf_counter()
    M = fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows, A.n_cols,
                      autotune=1)
    t_tune = time.perf_counter() - t0
    info = fs.csr_info(M)
    x = W.random_vector(A.n_cols, 1, W.XVEC)
    perm = fs.csr_get_perm(M)
    xp = d(x[perm])
    yp = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
    fs.spmv_perm(M, xp, yp)
    torch.cuda.synchronize()
    ok = bool(np.all(np.abs(yp.cpu().numpy() - oracle.spmv(A, x)[perm]) <=
                     1e-12 * oracle.spmv_abs(A, x)[perm]))
    us = back_to_back_us(torch, lambda: fs.spmv_perm(M, xp, yp), steps,
                         warmup, stream)
    out = {"tune_s": t_tune, "candidates": info["tune_candidates"],
           "vec": info["vec"], "groups_by_lanes": info["groups_by_lanes"],
           "us": us, "default_layout_us": default_us,
           "speedup_vs_default": default_us / us, "parity_all_rows": ok}
    M.close()
    return out


def bench_async(fs, oracle, torch, A, M, d, b, reps):
    """One right-hand side: the host-driven solve (chunks of iterations as
    graphs, a state read per chunk) vs the stream-ordered solve (one
    cooperative launch)."""
    bd = d(b)
    fs.cg_solve(M, bd, precond=fs.PC_JACOBI)
    fs.cg_solve_async(M, bd, precond=fs.PC_JACOBI).info()
    t_h, t_a = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xh, ih = fs.cg_solve(M, bd, precond=fs.PC_JACOBI)
        t_h.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        res = fs.cg_solve_async(M, bd, precond=fs.PC_JACOBI)
        ia = res.info()
        t_a.append(time.perf_counter() - t0)
    xa = res.x.cpu().numpy()
    rel = float(np.linalg.norm(b - oracle.spmv(A, xa)) / np.linalg.norm(b))
    return {"n_rows": A.n_rows, "iters_host_driven": ih["iters"],
            "iters_async": ia["iters"],
            "host_driven_ms": dist([t * 1e3 for t in t_h]),
            "async_ms": dist([t * 1e3 for t in t_a]),
            "async_kernel_ms": ia["ms"],
            "speedup": float(np.median(t_h) / np.median(t_a)),
            "async_status": ia["status"], "async_relres_oracle": rel}


def bench_spmv_batch(fs, W, oracle, d, torch, stream, m=64):
    """m small products (2-D Poisson, 48x48 nodes, random numbering): one
    spmv call each vs one spmv_batch call."""
    mats, Ms, xs = [], [], []
    for i in range(m):
        A = W.poisson_2d_p1(48, seed=(5, i), bc="all", permute=True)
        mats.append(A)
        Ms.append(fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows,
                                A.n_cols))
        xs.append(d(W.random_vector(A.n_cols, 5, W.XVEC, i)))
    ys = [torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
          for A in mats]
    one = lambda: [fs.spmv(M, x, y) for M, x, y in zip(Ms, xs, ys)]
    bat = lambda: fs.spmv_batch(Ms, xs, ys)
    t_one = back_to_back_us(torch, one, 20, 3, stream)
    t_bat = back_to_back_us(torch, bat, 20, 3, stream)
    ok = all(np.all(np.abs(y.cpu().numpy() - oracle.spmv(A, x.cpu().numpy()))
                    <= 1e-12 * oracle.spmv_abs(A, x.cpu().numpy()))
             for A, x, y in zip(mats, xs, ys))
    for M in Ms:
        M.close()
    return {"products": m, "rows_each": mats[0].n_rows,
            "one_at_a_time_us_per_product": t_one / m,
            "batched_us_per_product": t_bat / m,
            "speedup": t_one / t_bat, "parity_all_rows": bool(ok)}


def bench_newton(fs, oracle, torch, A, d, stream, steps=4):
    """Repeated solves on one pattern (the paper's use: the assembler hands
    new values each Newton step, the pattern and the layout stay): per step
    the device-side value refresh through the stored CSR -> slot map, then a
    Jacobi-PCG solve warm-started from the previous step's solution."""
    import workloads as W
    diag = A.col == np.repeat(np.arange(A.n_rows), A.row_lengths())
    vals = []
    for st in range(1, steps + 1):
        v = A.val * (1.0 + 0.1 * st)
        v[diag] += 0.002 * st * np.abs(A.val[diag])
        vals.append(d(v))
    b = W.random_vector(A.n_rows, 1, W.BVEC)
    bd = d(b)
    M = fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows, A.n_cols)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    out = []
    for st, vd in enumerate(vals, 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fs.csr_update_values(M, vd)
        e1.record(stream)
        e1.synchronize()
        t0 = time.perf_counter()
        x, info = fs.cg_solve(M, bd, x=x, precond=fs.PC_JACOBI, x0_zero=0)
        ts = time.perf_counter() - t0
        _, cold = fs.cg_solve(M, bd, precond=fs.PC_JACOBI)
        out.append({"step": st, "refresh_us": e0.elapsed_time(e1) * 1e3,
                    "solve_ms": ts * 1e3, "iters_warm": info["iters"],
                    "iters_cold": cold["iters"], "status": info["status"]})
    Ah_vals = vals[-1].cpu().numpy()
    from workloads.meshes import CSR
    B = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, Ah_vals)
    rel = float(np.linalg.norm(b - oracle.spmv(B, x.cpu().numpy())) /
                np.linalg.norm(b))
    M.close()
    return {"steps": out, "relres_oracle_last": rel,
            "refresh_gbs": (20.0 * A.nnz) / (out[-1]["refresh_us"] * 1e-6)
            / 1e9}


def bench_assembly(fs, oracle, torch, A, d, stream, steps=20):
    """Finite-element assembly straight into the layout (asm_matrix: the
    element matrices summed per non-zero, element order) on the 3-D
    elasticity workload, with both plans (row groups summed in LDS, and
    per-slot gathers): plan build, kernel time against the algorithmic
    bytes (element values + their 4-byte positions read, FP64 result
    written), bitwise parity of every value and load entry against the
    oracle's element loop, and the value reorder it makes unnecessary."""
    from workloads.elements import config1_elements
    t = time.time()
    E = config1_elements()
    tg = time.time() - t
    M = fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows, A.n_cols)
    ked, red = d(E.ke), d(E.re)
    edd = d(E.edof)
    t = time.perf_counter()
    want = oracle.assemble_matrix(A, E.edof, E.ke)
    t_or = time.perf_counter() - t
    rwant = oracle.assemble_vector(A.n_rows, E.edof, E.re)
    out = {"n_elem": E.n_elem, "nde": E.nde, "t_generate_s": tg,
           "cpu_oracle_assembly_ms": t_or * 1e3}
    for name, plan in (("rowgroup", fs.ASM_ROWGROUP),
                       ("gather", fs.ASM_GATHER)):
        t = time.perf_counter()
        P = fs.asm_create(M, edd, plan=plan)
        t_plan = time.perf_counter() - t
        info = fs.asm_info(P)
        t_mat = back_to_back_us(torch, lambda: fs.asm_matrix(P, ked, stream),
                                steps, 3, stream)
        per = event_times_us(torch, lambda: fs.asm_matrix(P, ked, stream),
                             steps, stream)
        got = fs.csr_get_values(M).cpu().numpy()
        bytes_m = info["bytes_algorithmic_matrix"]
        out[name] = {
            "plan_ms": t_plan * 1e3, "contributions": info["contrib_matrix"],
            "index_entries_per_contribution":
                info["stored_matrix"] / info["contrib_matrix"],
            "matrix_us": t_mat, "matrix_us_per_launch": dist(per),
            "bytes_algorithmic": bytes_m,
            "gbs": bytes_m / (t_mat * 1e-6) / 1e9,
            "frac": bytes_m / (t_mat * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "device_bytes": info["device_bytes"],
            "parity_bitwise_all_values": bool(np.array_equal(
                got.view(np.int64), want.view(np.int64)))}
        if name == "rowgroup":
            # the element rows stored in the plan's order (the paper's
            # proposal: element routines write where assembly reads in order)
            pos, nrows = fs.asm_element_rows(P)
            ko = np.zeros((nrows, E.nde))
            keep = pos >= 0
            ko[pos[keep]] = E.ke.reshape(-1, E.nde)[keep]
            kod = d(ko)
            del ko
            t_ord = back_to_back_us(
                torch, lambda: fs.asm_matrix_ordered(P, kod, stream), steps,
                3, stream)
            got_o = fs.csr_get_values(M).cpu().numpy()
            out["ordered"] = {
                "matrix_us": t_ord,
                "gbs": bytes_m / (t_ord * 1e-6) / 1e9,
                "frac": bytes_m / (t_ord * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "buffer_rows": nrows,
                "parity_bitwise_all_values": bool(np.array_equal(
                    got_o.view(np.int64), want.view(np.int64)))}
            del kod
            r = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
            out["vector_us"] = back_to_back_us(
                torch, lambda: fs.asm_vector(P, red, r, stream), steps, 3,
                stream)
            out["system_us"] = back_to_back_us(
                torch, lambda: fs.asm_system(P, ked, red, r, stream), steps,
                3, stream)
            out["parity_bitwise_all_loads"] = bool(np.array_equal(
                r.cpu().numpy().view(np.int64), rwant.view(np.int64)))
        P.close()
    va = d(A.val)
    out["reorder_avoided_us"] = back_to_back_us(
        torch, lambda: fs.csr_update_values(M, va, stream), 10, 2, stream)
    # one Newton-style step on the assembled system: assemble K and R into
    # the layout, then Jacobi-PCG to 1e-8 (the paper's split of a step into
    # assembly and solver time)
    P = fs.asm_create(M, edd)
    r = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
    fs.cg_solve(M, r.fill_(1.0), maxit=2, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fs.asm_system(P, ked, red, r, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, ci = fs.cg_solve(M, r, precond=fs.PC_JACOBI, rtol=1e-8, check=False)
    t2 = time.perf_counter()
    from workloads.meshes import CSR
    K = CSR(A.n_rows, A.n_cols, A.rowptr, A.col, want)
    rel = float(np.linalg.norm(rwant - oracle.spmv(K, x.cpu().numpy())) /
                np.linalg.norm(rwant))
    out["newton_step"] = {"assemble_ms": (t1 - t0) * 1e3,
                          "solve_ms": (t2 - t1) * 1e3, "iters": ci["iters"],
                          "status": ci["status"], "relres_oracle": rel,
                          "assembly_share": (t1 - t0) / (t2 - t0)}
    P.close()
    M.close()
    return out


def run_sweep(fs, W, oracle, torch, d, steps, warmup, stream):
    """Every sweep matrix in natural and random numbering: layout, parity,
    product GB/s, the plain CSR product, build time."""
    rows = []
    for i, (name, *_rest) in enumerate(W.SWEEP):
        for permuted in (False, True):
            t = time.time()
            try:
                A = W.sweep_matrix(i, permuted)
            except NotImplementedError as e:
                log("sweep %s: skipped (%s)" % (name, e))
                rows.append({"matrix": name, "permuted": permuted,
                             "skipped": str(e)})
                break
            tg = time.time() - t
            M, r = measure_matrix(fs, oracle, torch, A, d, steps, warmup,
                                  stream, cold=False)
            del M
            r.update(matrix=name, permuted=permuted, t_generate_s=tg)
            # the oracle on the host: one thread, then all cores
            xh = W.random_vector(A.n_cols, 1, W.XVEC)
            bytes_alg = 12 * A.nnz + 8 * A.n_cols + 8 * A.n_rows
            t0 = time.perf_counter()
            oracle.spmv(A, xh)
            t1 = time.perf_counter()
            _, used = oracle.spmv_par(A, xh)
            t2 = time.perf_counter()
            r["cpu_oracle_gbs"] = bytes_alg / (t1 - t0) / 1e9
            r["cpu_oracle_all_cores_gbs"] = bytes_alg / (t2 - t1) / 1e9
            r["cpu_cores"] = used
            rows.append(r)
            log("sweep %s %s: %.1f GB/s (%.1f%% of peak), csr %.1f GB/s, "
                "parity %s" % (name, "perm" if permuted else "nat", r["gbs"],
                               100 * r["frac"], r["csr_plain"]["gbs"],
                               r["parity_all_rows"]))
    return rows


def headline_matrix(W):
    """The largest FEM matrix of the sweep: Q1 hexahedral elasticity, 87^3
    nodes, natural numbering, full Neumann (1,975,509 rows, 156,365,811
    non-zeros)."""
    i12 = [i for i, r in enumerate(W.SWEEP) if r[0].startswith("S12")][0]
    return W.SWEEP[i12][0], W.sweep_matrix(i12, False)


def bench_bf16_variants(fs, oracle, torch, A, M, bd, b, x64, cg):
    """Refinement with BF16 values on the elasticity matrix: the kept
    search direction and the restarted inner CG at three inner tolerances,
    and BF16 values stored after Jacobi scaling (D^-1/2 A D^-1/2 rounded).
    Each row: status, steps, inner iterations, oracle-recomputed residual,
    forward error against the FP64 solution, time."""
    rows = []
    for restart in (0, 1):
        for eta in (1e-1, 1e-2, 1e-3):
            for scaled in (0, 1):
                if scaled and eta != 1e-2:
                    continue
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xs, ci = fs.cg_solve(M, bd, precond=fs.PC_JACOBI, rtol=1e-8,
                                     precision=fs.PREC_IR_BF16,
                                     inner_rtol=eta, ir_restart=restart,
                                     ir_scaled=scaled, check=False)
                t = time.perf_counter() - t0
                xh = xs.cpu().numpy()
                rows.append({
                    "ir_restart": restart, "inner_rtol": eta,
                    "jacobi_scaled_storage": scaled,
                    "status": ci["status"], "outer": ci["outer"],
                    "inner": ci["iters"], "ms": t * 1e3,
                    "relres_oracle": float(np.linalg.norm(
                        b - oracle.spmv(A, xh)) / np.linalg.norm(b)),
                    "relres_gpu": ci["relres"],
                    "forward_err_vs_fp64": float(np.linalg.norm(xh - x64) /
                                                 np.linalg.norm(x64)),
                    "speedup_vs_fp64": cg["ms"] / (t * 1e3)})
                log("cg ir-bf16 %s" % json.dumps(rows[-1]))
    # Jacobi-scaled storage keeps contracting where plain BF16 stalls: the
    # restarted form with a large iteration budget, to see where it ends
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, ci = fs.cg_solve(M, bd, precond=fs.PC_JACOBI, rtol=1e-8,
                         precision=fs.PREC_IR_BF16, inner_rtol=1e-2,
                         ir_restart=1, ir_scaled=1, maxit=150000,
                         max_outer=1000, check=False)
    t = time.perf_counter() - t0
    xh = xs.cpu().numpy()
    rows.append({
        "ir_restart": 1, "inner_rtol": 1e-2, "jacobi_scaled_storage": 1,
        "budget": "maxit 150000, max_outer 1000",
        "status": ci["status"], "outer": ci["outer"], "inner": ci["iters"],
        "ms": t * 1e3,
        "relres_oracle": float(np.linalg.norm(b - oracle.spmv(A, xh)) /
                               np.linalg.norm(b)),
        "relres_gpu": ci["relres"],
        "forward_err_vs_fp64": float(np.linalg.norm(xh - x64) /
                                     np.linalg.norm(x64)),
        "speedup_vs_fp64": cg["ms"] / (t * 1e3)})
    log("cg ir-bf16 %s" % json.dumps(rows[-1]))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="only the timed product on the largest FEM matrix "
                         "(for counter profiles)")
    ap.add_argument("--only-multi", type=int, default=0, metavar="K",
                    help="only one K-column multi-RHS Jacobi-PCG solve on "
                         "the 3-D elasticity system (for counter profiles)")
    ap.add_argument("--only-small-batch", action="store_true",
                    help="only the 64 small systems: one at a time, "
                         "batched, one workgroup per system (for counter "
                         "profiles)")
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--no-asm", action="store_true",
                    help="skip the finite-element assembly measurement")
    ap.add_argument("--serving-full", action="store_true",
                    help="only the serving experiment: 500 requests per "
                         "arrival rate, lambda/mu in {0.25, 0.5, 0.75, "
                         "0.9, 1, 1.5, 2}, one JSON line")
    ap.add_argument("--sweep", action="store_true",
                    help="only the sparsity sweep: every sweep matrix, "
                         "natural and random numbering, one JSON line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB copy kernel first (reference "
                         "for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is a single-GPU "
              "SpMV/CG library and no multi-GPU run is part of this build "
              "(asked for --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1501_00324_amd as fs
    import workloads as W
    import oracle

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fs.load(build_if_missing=True)
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    stream = torch.cuda.current_stream()

    if args.serving_full:
        srv = bench_serving(fs, W, oracle, d, torch, n_req=500,
                            lam_factors=(0.25, 0.5, 0.75, 0.9, 1.0, 1.5, 2.0))
        print(json.dumps({"metric": "served CG solves: p50/p99 latency and "
                                    "solves/s vs one-at-a-time FP64 CG",
                          "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                          "serving": srv}), flush=True)
        release_host_cache(torch)
        return

    if args.sweep:
        rows = run_sweep(fs, W, oracle, torch, d, 50, 5, stream)
        print(json.dumps({"metric": "SpMV effective GB/s per sweep matrix",
                          "unit": "GB/s", "n_gpus": 1, "dtype": "f64",
                          "data": "synthetic", "peak_gbs": HBM_PEAK_GBS,
                          "sweep": rows}), flush=True)
        release_host_cache(torch)
        return

    if args.only_multi:
        A = W.config1_elasticity3d()
        M = fs.csr_create(d(A.rowptr), d(A.col), d(A.val), A.n_rows,
                          A.n_cols)
        k = args.only_multi
        Bk = d(W.random_vector(A.n_rows, 1, W.BVEC, 1, k=k))
        fs.cg_solve_multi(M, Bk, precond=fs.PC_JACOBI, maxit=3, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = fs.cg_solve_multi(M, Bk, precond=fs.PC_JACOBI,
                                     check=False)
        t = time.perf_counter() - t0
        print(json.dumps({"multi_rhs_k": k, "ms": t * 1e3,
                          "iters_max": max(i["iters"] for i in infos),
                          "all_converged": all(i["status"] == fs.FS_OK
                                               for i in infos)}), flush=True)
        M.close()
        release_host_cache(torch)
        return

    if args.only_small_batch:
        if args.calibrate_copy:
            ca = torch.ones(CALIB_DOUBLES, dtype=torch.float64, device=dev)
            cb = torch.empty_like(ca)
            for _ in range(3):
                torch.neg(ca, out=cb)
            torch.cuda.synchronize()
            del ca, cb
        print(json.dumps({"cg_batched_small": bench_small_batch(
            fs, W, oracle, d, torch)}), flush=True)
        release_host_cache(torch)
        return

    if args.calibrate_copy:
        ca = torch.ones(CALIB_DOUBLES, dtype=torch.float64, device=dev)
        cb = torch.empty_like(ca)
        for _ in range(3):
            torch.neg(ca, out=cb)
        torch.cuda.synchronize()
        log("calibration copy: 3 x neg of %d doubles (%d bytes read and "
            "%d written per launch)" % (CALIB_DOUBLES, 8 * CALIB_DOUBLES,
                                        8 * CALIB_DOUBLES))
        del ca, cb

    # ---- headline: the FP64 product on the largest FEM matrix
    t = time.time()
    hname, H = headline_matrix(W)
    tg = time.time() - t
    log("generated %s: %d rows, %d nnz in %.1f s" % (hname, H.n_rows, H.nnz,
                                                     tg))
    MH, prod = measure_matrix(fs, oracle, torch, H, d, args.steps,
                              args.warmup, stream,
                              extras=not args.only_headline)
    prod.update(matrix=hname, numbering="natural", t_generate_s=tg)
    us = prod["us"]
    gbs = prod["gbs"]
    bytes_alg = 12 * H.nnz + 8 * H.n_cols + 8 * H.n_rows
    h_rows, h_nnz = H.n_rows, H.nnz
    log("headline spmv_perm on %s: %.2f us/launch, %.1f GB/s (%.1f%% of "
        "peak); cold median %.2f us (%.1f%%); parity %s"
        % (hname, us, gbs, 100 * gbs / HBM_PEAK_GBS,
           prod["cold_us"]["median"], 100 * prod["cold_gbs"] / HBM_PEAK_GBS,
           prod["parity_all_rows"]))
    traffic = measured_traffic()

    def line(extra):
        out = {
            "metric": "SpMV effective GB/s (% HBM peak); CG solves/s + p99 "
                      "latency, FP64 vs mixed",
            "value": round(gbs, 2),
            "unit": "GB/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": us * 1e-3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "largest FEM matrix: Q1-hex elasticity, "
                                   "87^3 nodes, natural numbering, full "
                                   "Neumann (sweep S12)",
                       "n_rows": h_rows, "nnz": h_nnz,
                       "op": "spmv_perm (layout numbering, as inside CG)",
                       "bytes_per_spmv": bytes_alg},
            "pct_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
            "cold_pct_hbm_peak": round(100.0 * prod["cold_gbs"] /
                                       HBM_PEAK_GBS, 2),
            "cold_read_flush_pct_hbm_peak": round(
                100.0 * prod["cold_read_flush_gbs"] / HBM_PEAK_GBS, 2),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 2),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": traffic,
                         "dram_gbs": (round(traffic / (us * 1e-6) / 1e9, 1)
                                      if traffic else None),
                         "bytes_algorithmic": bytes_alg,
                         "kernel": "k_spmv_f64",
                         "cold_frac": round(prod["cold_gbs"] /
                                            HBM_PEAK_GBS, 4)},
            "paper_model_gbs": round(20 * h_nnz / (us * 1e-6) / 1e9, 2),
            "parity_all_rows": prod["parity_all_rows"],
            "spmv": prod,
        }
        out.update(extra)
        return out

    if args.only_headline:
        print(json.dumps(line({})), flush=True)
        MH.close()
        release_host_cache(torch)
        return

    # CPU oracle on a bounded sample of the headline workload: repeated
    # full products of the same matrix (single thread, then all cores)
    xh = W.random_vector(H.n_cols, 1, W.XVEC)
    cpu = cpu_all = None
    if args.cpu_seconds > 0:
        reps, tc = 0, 0.0
        t0 = time.perf_counter()
        while tc < args.cpu_seconds:
            oracle.spmv(H, xh)
            reps += 1
            tc = time.perf_counter() - t0
        cpu_gbs = bytes_alg * reps / tc / 1e9
        cpu = {"value": round(cpu_gbs, 3), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "cpu": host_cpu_model(),
               "sample": "%d full FP64 CSR products of the headline matrix "
                         "(%d nnz), single thread, %.1f s" % (reps, H.nnz,
                                                               tc)}
        log("cpu oracle: %s" % json.dumps(cpu))
        reps_p, tc_p, used = 0, 0.0, 1
        t0 = time.perf_counter()
        while tc_p < max(2.0, args.cpu_seconds / 2):
            _, used = oracle.spmv_par(H, xh)
            reps_p += 1
            tc_p = time.perf_counter() - t0
        cpu_all = {"value": round(bytes_alg * reps_p / tc_p / 1e9, 3),
                   "unit": "GB/s", "cores": used, "kind": "oracle",
                   "cpu": host_cpu_model(),
                   "sample": "%d full FP64 CSR products of the headline "
                             "matrix, rows split over %d OpenMP threads"
                             % (reps_p, used)}
        log("cpu oracle, all cores: %s" % json.dumps(cpu_all))
    MH.close()
    del MH, H
    torch.cuda.synchronize()

    # ---- config 1: the 3-D elasticity system the CG legs solve
    t = time.time()
    A = W.config1_elasticity3d()
    log("generated config-1 matrix: %d rows, %d nnz in %.1f s"
        % (A.n_rows, A.nnz, time.time() - t))
    M, c1 = measure_matrix(fs, oracle, torch, A, d, args.steps, args.warmup,
                           stream)
    c1_bytes = 12 * A.nnz + 8 * A.n_cols + 8 * A.n_rows
    log("config-1 spmv_perm: %.2f us/launch, %.1f GB/s; cold median %.2f us"
        % (c1["us"], c1["gbs"], c1["cold_us"]["median"]))
    c1["autotuned"] = bench_autotune(fs, oracle, torch, A, d, args.steps,
                                     args.warmup, stream, c1["us"])
    log("config-1 autotuned layout: %s" % json.dumps(c1["autotuned"]))

    # achievable streaming read rate (project kernel, 2 GiB, best of three
    # grid sizes): the practical ceiling the product is compared with
    buf = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    sink = torch.empty(16384, dtype=torch.float64, device=dev)
    stream_gbs = 0.0
    for blocks in (2048, 4096, 16384):
        t_rd = back_to_back_us(torch, lambda: fs.probe_read_bandwidth(
            buf, sink, blocks), 20, 3, stream)
        stream_gbs = max(stream_gbs, buf.numel() * 8 / (t_rd * 1e-6) / 1e9)
    del buf, sink
    log("streaming read probe: %.1f GB/s; headline product at %.1f%% of it"
        % (stream_gbs, 100 * gbs / stream_gbs))

    # caller numbering (gather of x + fused scatter of y) on config 1
    x = W.random_vector(A.n_cols, 1, W.XVEC)
    xd = d(x)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    us_caller = back_to_back_us(torch, lambda: fs.spmv(M, xd, y), args.steps,
                                args.warmup, stream)
    gbs_caller = c1_bytes / (us_caller * 1e-6) / 1e9
    log("config-1 spmv (caller numbering): %.2f us, %.1f GB/s"
        % (us_caller, gbs_caller))

    cg = ir = bf16 = multi = batch = asy = asy_small = sbatch = None
    newton = cpu_cg = None
    if not args.no_cg:
        b = W.random_vector(A.n_rows, 1, W.BVEC)
        bd = d(b)
        fs.cg_solve(M, bd, precond=fs.PC_JACOBI, maxit=3, check=False)

        def timed_solve(reps=3, **kw):
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xs, ci = fs.cg_solve(M, bd, precond=fs.PC_JACOBI, rtol=1e-8,
                                     check=False, **kw)
                times.append(time.perf_counter() - t0)
            xs_h = xs.cpu().numpy()
            rel = float(np.linalg.norm(b - oracle.spmv(A, xs_h)) /
                        np.linalg.norm(b))
            tmed = float(np.median(times))
            return xs_h, ci, {"status": ci["status"], "iters": ci["iters"],
                              "outer": ci["outer"], "ms": tmed * 1e3,
                              "solves_per_s": 1.0 / tmed,
                              "relres_oracle": rel, "relres_gpu": ci["relres"],
                              "replacements": ci["replacements"],
                              "gbs_per_solve": ci["bytes"] / tmed / 1e9}

        x64, ci64, cg = timed_solve(estimate_cond=1)
        cg.update(precond="jacobi", rtol=1e-8,
                  cond_est_jacobi=ci64.get("cond_est"))
        log("cg fp64: %s" % json.dumps(cg))
        ir = {}
        for name, prec, rs in (("f32", fs.PREC_IR_F32, 0),
                               ("f32_restart", fs.PREC_IR_F32, 1)):
            xl, _, r = timed_solve(reps=2, precision=prec, inner_rtol=1e-2,
                                   ir_restart=rs)
            r["forward_err_vs_fp64"] = float(np.linalg.norm(xl - x64) /
                                             np.linalg.norm(x64))
            r["speedup_vs_fp64"] = cg["ms"] / r["ms"]
            ir[name] = r
            log("cg ir-%s: %s" % (name, json.dumps(r)))
        bf16 = bench_bf16_variants(fs, oracle, torch, A, M, bd, b, x64, cg)
        ir["bf16"] = bf16
        ke = cg.get("cond_est_jacobi")
        ir["bf16_note"] = {
            "cond_est_jacobi": ke,
            "cond_est_times_2^-9": ke * 2.0 ** -9 if ke else None,
            "converged_variants": sum(r["status"] == fs.FS_OK
                                      for r in bf16),
            "best_relres": min(r["relres_oracle"] for r in bf16)}
        asy = bench_async(fs, oracle, torch, A, M, d, b, reps=3)
        log("cg stream-ordered (config 1): %s" % json.dumps(asy))
        A0 = W.config0_poisson2d()
        M0 = fs.csr_create(d(A0.rowptr), d(A0.col), d(A0.val), A0.n_rows,
                           A0.n_cols)
        asy_small = bench_async(fs, oracle, torch, A0, M0, d,
                                W.random_vector(A0.n_rows, 0, W.BVEC),
                                reps=20)
        M0.close()
        log("cg stream-ordered (config 0): %s" % json.dumps(asy_small))
        # k right-hand sides through one multi-column product per iteration
        multi = {}
        for k in (4, 8, 16):
            Bk = W.random_vector(A.n_rows, 1, W.BVEC, 1, k=k)
            Bkd = d(Bk)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Xk, infos = fs.cg_solve_multi(M, Bkd, precond=fs.PC_JACOBI,
                                          check=False)
            tk = time.perf_counter() - t0
            Xk_h = Xk.cpu().numpy()
            worst = max(float(np.linalg.norm(
                Bk[:, c] - oracle.spmv(A, Xk_h[:, c].copy())) /
                np.linalg.norm(Bk[:, c])) for c in range(k))
            multi[str(k)] = {
                "k": k, "ms": tk * 1e3, "solves_per_s": k / tk,
                "speedup_vs_one_at_a_time": (k / tk) / cg["solves_per_s"],
                "iters_max": max(i["iters"] for i in infos),
                "all_converged": all(i["status"] == fs.FS_OK
                                     for i in infos),
                "relres_oracle_worst": worst}
            log("cg multi-rhs k=%d: %s" % (k, json.dumps(multi[str(k)])))
        newton = bench_newton(fs, oracle, torch, A, d, stream)
        log("newton steps: %s" % json.dumps(newton))
        batch = bench_small_batch(fs, W, oracle, d, torch)
        log("batched small systems: %s" % json.dumps(batch))
        sbatch = bench_spmv_batch(fs, W, oracle, d, torch, stream)
        log("batched small products: %s" % json.dumps(sbatch))
        # the oracle's Jacobi-PCG on the host: config 0 to 1e-8, and a
        # bounded run of config-1 iterations scaled to the GPU's count
        A0 = W.config0_poisson2d()
        b0 = W.random_vector(A0.n_rows, 0, W.BVEC)
        t0 = time.perf_counter()
        _, st0, it0, _ = oracle.pcg(A0, b0, precond=1)
        t_c0 = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, _, it1, _ = oracle.pcg(A, b, precond=1, maxit=40)
        per_it = (time.perf_counter() - t0) / max(1, it1)
        cpu_cg = {"config0_ms": t_c0 * 1e3, "config0_iters": it0,
                  "config1_ms_per_iter": per_it * 1e3,
                  "config1_est_ms": per_it * 1e3 * cg["iters"],
                  "cores": 1, "kind": "oracle",
                  "sample": "config 0 solved to 1e-8; 40 config-1 "
                            "iterations, scaled to the GPU iteration count"}
        log("cpu oracle CG: %s" % json.dumps(cpu_cg))
    assembly = None
    if not args.no_asm:
        assembly = bench_assembly(fs, oracle, torch, A, d, stream)
        log("assembly: %s" % json.dumps(assembly))
    serving = None
    if args.serving_requests > 0:
        serving = bench_serving(fs, W, oracle, d, torch,
                                n_req=args.serving_requests,
                                lam_factors=(0.5, 1.0, 2.0))
        log("serving: %s" % json.dumps(serving))

    print(json.dumps(line({
        "cpu_baseline": cpu,
        "cpu_oracle_all_cores": cpu_all,
        "cpu_oracle_cg": cpu_cg,
        "stream_read_gbs": round(stream_gbs, 1),
        "pct_of_stream_read": round(100.0 * gbs / stream_gbs, 2),
        "config1_spmv": c1,
        "config1_spmv_caller_numbering_gbs": round(gbs_caller, 2),
        "cg": cg,
        "cg_mixed_precision": ir,
        "cg_stream_ordered": {"config1": asy, "config0": asy_small},
        "cg_multi_rhs": multi,
        "newton_repeated_solves": newton,
        "fe_assembly": assembly,
        "cg_batched_small": batch,
        "spmv_batched_small": sbatch,
        "serving": serving,
    })), flush=True)
    # explicit teardown while the runtime is fully up: every handle closed,
    # the device drained, torch's cached pinned host blocks returned
    M.close()
    torch.cuda.synchronize()
    release_host_cache(torch)


def release_host_cache(torch):
    import gc
    gc.collect()
    torch.cuda.synchronize()
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()


if __name__ == "__main__":
    main()
