"""Benchmark: eigenpairs/s of the mixed-precision MRRR solve on one MI355X.

Workload (one step = one full solve, inputs resident in HBM before timing):
    prescribed-spectrum tridiagonal, n = 20000, FP64 input/output with
    double-double internal arithmetic, all 20000 eigenpairs (eigenvalues
    geometric in magnitude from 1 down to 1e-8 with seeded random signs; T
    built from a seeded N(0,1) Lanczos start vector).

Prints ONE JSON line with the throughput, p50/p99 solve time, the roofline of
the dominant kernel (algorithmic FP64 flops per launch over its HIP-event
duration on the launch stream) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, FP64 vector (FMA = 2 flops)

# Algorithmic FP64 flops per row step (an FMA counts 2), see the design doc:
#   Sturm count, division-free stationary transform:  fma + mul + fma       = 5
#   twist pre-pass in binary64 (transform + quotient + gamma, averaged)     = 7
#   RQI sweep in double-double: 4 dd products (10) + 2 dd sums (11) + z^2   = 64
#   RQI sweep in binary64:      fma + mul + fma + z product + z^2           = 8
FLOPS_COUNT = 5.0
FLOPS_TWIST = 7.0
FLOPS_RQI = {"dd": 64.0, "f64": 8.0}


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source has changed since it was taken."""
    import hashlib

    prof = os.path.join(ROOT, "profiles", "counters_prescribed_n20000_fp64.md")
    src = os.path.join(ROOT, "paper_1304_1864_amd", "csrc", "mr3_kernels.hip")
    if not os.path.exists(prof):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(prof):
        f = line.split()
        if len(f) == 4 and f[0] == "traffic" and f[1] == kernel:
            kv = dict(x.split("=", 1) for x in f[2:])
            return float(kv["bytes_per_launch"]) if kv["source_sha256"] == sha else None
    return None


def build_workload(n: int, seed: int):
    import workloads as W

    d, e, lam = W.prescribed_spectrum(n, seed)
    return d, e


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def alg_flops(st, y: str) -> float:
    """Algorithmic FP64 flops of the last solve on a handle (its stats): Sturm
    counts, twist pre-pass and RQI sweeps at the per-row counts above."""
    return (st["bisect_row_steps"] * FLOPS_COUNT + st["twist_row_steps"] * FLOPS_TWIST
            + st["rqi_row_steps"] * FLOPS_RQI[y])


def cpu_baseline(d, e, n, budget_s=20.0, w_gpu=None, z_gpu=None):
    """Oracle (double-double bisection + inverse iteration) on a bounded
    sample: contiguous index chunks spread over the spectrum, on the cores
    this process may use (at most 16, the host share of one GPU).  After the
    timing, the GPU's eigenvalues (host array w_gpu) and eigenvectors (z_gpu(i)
    -> column i as a host array) of the sampled indices are compared with the
    oracle's: eigenvalue error over its gate 4 n eps ||T||_1, and the largest
    1 - |cos| between the two unit vectors."""
    import oracle

    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(16, avail)
    chunk = 512  # about 10-20 s of oracle work on 16 cores
    starts = [1, n // 4, n // 2, 3 * n // 4, n - chunk + 1]
    done = 0
    got = []
    t0 = time.perf_counter()
    for s in starts:
        hi, lo = oracle.eigvals(d, e, s, s + chunk - 1, threads=threads)
        Zr = oracle.eigvecs(d, e, hi, lo, threads=threads)
        got.append((s, hi + lo, Zr))
        done += chunk
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": done / dt, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} eigenpairs (index chunks of {chunk} at {starts[:done // chunk]}) "
                     f"of the same n={n} matrix, {dt:.1f} s",
           "host": {"nproc": os.cpu_count(), "usable": avail, "model": cpu_model()}}
    if w_gpu is not None:
        tn = float(np.max(np.abs(d) + np.concatenate([np.abs(e), [0.0]]) + np.concatenate([[0.0], np.abs(e)])))
        gate = 4 * n * 2.0 ** -53 * tn
        err, cos_gap = 0.0, 0.0
        for s, ref, Zr in got:
            err = max(err, float(np.max(np.abs(w_gpu[s - 1:s - 1 + ref.size] - ref))))
            if z_gpu is not None:
                for j in range(0, ref.size, 8):
                    z = z_gpu(s - 1 + j)
                    cos_gap = max(cos_gap, 1.0 - abs(float(z @ Zr[:, j])))
        out["gpu_vs_oracle_on_sample"] = {"eig_err_over_gate": round(err / gate, 5),
                                          "max_1_minus_abs_cos": float(f"{cos_gap:.3g}")}
    return out


def batched_c3(mr3, h, steps, warmup, plain_sample=512, seed=0):
    """4096 independent problems, n log-uniform in [32, 1024], d, e ~ N(0, 1),
    FP32 I/O, all eigenpairs: one mr3_solve_batched call per step (batched)
    against one mr3_solve_f32 per problem in sequence (plain, timed on the
    first ``plain_sample`` problems)."""
    import torch
    import workloads as W

    probs = W.batch_normal(4096, 32, 1024, seed=seed, dtype=np.float32)
    count = len(probs)
    n = [int(p[0].size) for p in probs]
    de_off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    total = int(sum(n))
    dcat = np.concatenate([p[0] for p in probs])
    ecat = np.zeros(total, np.float32)
    for p, o in zip(probs, de_off):
        ecat[o:o + p[1].size] = p[1]
    dev = torch.device("cuda:0")
    dg = torch.from_numpy(dcat).to(dev)
    eg = torch.from_numpy(ecat).to(dev)
    w_off = de_off.tolist()
    z_off = np.concatenate([[0], np.cumsum(np.array(n, np.int64) ** 2)[:-1]]).astype(np.int64).tolist()
    Wb = torch.empty(total, dtype=torch.float32, device=dev)
    Zb = torch.empty(int(sum(k * k for k in n)), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    # per-problem host arrays built once (int64 numpy arrays pass without a copy)
    n_a = np.array(n, dtype=np.int64)
    wo_a = np.array(w_off, dtype=np.int64)
    zo_a = np.array(z_off, dtype=np.int64)

    def step():
        return mr3.mr3_solve_batched(h, count, 32, n_a, de_off, dg, eg, None, Wb, wo_a, Zb, zo_a,
                                     n_a, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        ts = time.perf_counter()
        m = step()
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - ts) * 1e3)
    assert sum(m) == total
    batch_flops = alg_flops(h.stats(), "f64")
    # plain: one solve per problem, sequentially on one stream
    k = min(plain_sample, count)
    Wp = torch.empty(1024, dtype=torch.float32, device=dev)
    Zp = torch.empty((1024, 1024), dtype=torch.float32, device=dev)
    for i in range(min(8, k)):  # warm-up of the single-solve path
        mr3.mr3_solve_f32(h, n[i], dg[de_off[i]:], eg[de_off[i]:], mr3.RANGE_ALL, 0.0, 0.0, 1, n[i],
                          Wp, Zp, n[i], stream)
    torch.cuda.synchronize()
    pm = []
    plain_flops = 0.0
    t0 = time.perf_counter()
    for i in range(k):
        ts = time.perf_counter()
        mr3.mr3_solve_f32(h, n[i], dg[de_off[i]:], eg[de_off[i]:], mr3.RANGE_ALL, 0.0, 0.0, 1, n[i],
                          Wp, Zp, n[i], stream)
        torch.cuda.synchronize()
        pm.append((time.perf_counter() - ts) * 1e3)
        plain_flops += alg_flops(h.stats(), "f64")
    plain_s = time.perf_counter() - t0
    pairs_k = int(sum(n[:k]))
    med = float(np.median(ms))
    peak = FP64_VECTOR_PEAK_TFLOPS * 1e12
    return {
        "workload": "4096 tridiagonals, n log-uniform in [32, 1024] (sum n = %d), d, e ~ N(0,1), "
                    "fp32 I/O, fp64 internal, all eigenpairs, seed %d" % (total, seed),
        "batched": {"eigenpairs_per_s": round(total / (med / 1e3), 1), "p50_ms": round(med, 3),
                    "p99_ms": round(float(np.percentile(ms, 99)), 3), "steps": steps,
                    "roofline": {"bound": "alu", "achieved": round(batch_flops / (med / 1e3) / 1e12, 3),
                                 "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(batch_flops / (med / 1e3) / peak, 4),
                                 "what": "algorithmic FP64 flops of the whole solve / its time"}},
        "plain": {"eigenpairs_per_s": round(pairs_k / plain_s, 1),
                  "p50_ms_per_problem": round(float(np.median(pm)), 3),
                  "p99_ms_per_problem": round(float(np.percentile(pm, 99)), 3),
                  "roofline_frac": round(plain_flops / plain_s / peak, 5),
                  "sample": f"first {k} problems ({pairs_k} eigenpairs), one mr3_solve_f32 each"},
    }


def served_c5(mr3, n_req=2000, seed=0, window=64, calib=600, slots=2):
    """Served stream: requests with n log-uniform in [64, 8192], half FP32 /
    half FP64, 30% INDEX ranges of ceil(0.1 n), half U(-1,1) and half 1-2-1
    plus N(0, (1e-6)^2) noise, all vectors.  Saturation S from a closed loop
    (``window`` requests in flight), then Poisson arrivals at 0.5 S and
    0.8 S; latency = completion - arrival, including queueing."""
    import threading
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    reqs = W.served_requests(n_req, seed=seed)
    inputs = [(torch.from_numpy(r["d"]).to(dev), torch.from_numpy(r["e"]).to(dev)) for r in reqs]
    torch.cuda.synchronize()
    # plain: the same requests solved one call each, in sequence on one
    # stream; their algorithmic flops (from the solver's counters) price the
    # served throughput against the FP64 vector peak
    hp = mr3.Handle(0)
    nmax = max(r["n"] for r in reqs)
    Wp = {dt: torch.empty(nmax, dtype=dt, device=dev) for dt in (torch.float32, torch.float64)}
    Zp = {dt: torch.empty(nmax * nmax, dtype=dt, device=dev) for dt in (torch.float32, torch.float64)}

    def plain(i):
        kind, il, iu = reqs[i]["range"]
        d_, e_ = inputs[i]
        nn = d_.numel()
        fn = mr3.mr3_solve_f32 if d_.dtype == torch.float32 else mr3.mr3_solve_f64
        rk = mr3.RANGE_INDEX if kind == "index" else mr3.RANGE_ALL
        return fn(hp, nn, d_, e_, rk, 0.0, 0.0, il, iu, Wp[d_.dtype], Zp[d_.dtype], nn)

    for i in range(8):
        plain(i)
    torch.cuda.synchronize()
    n_plain = min(calib, n_req)
    flops_req, pl_ms, pairs_plain = [], [], 0
    t0 = time.perf_counter()
    for i in range(n_plain):
        ts = time.perf_counter()
        pairs_plain += plain(i)
        torch.cuda.synchronize()
        pl_ms.append((time.perf_counter() - ts) * 1e3)
        flops_req.append(alg_flops(hp.stats(), "f64" if inputs[i][0].dtype == torch.float32 else "dd"))
    t_plain = time.perf_counter() - t0
    hp.close()
    del Wp, Zp
    torch.cuda.empty_cache()
    peak = FP64_VECTOR_PEAK_TFLOPS * 1e12
    mean_flops = float(np.mean(flops_req))
    free, _ = torch.cuda.mem_get_info(0)
    srv = mr3.Server(mr3.Handle(0), hbm_budget_bytes=free // 2, max_batch=256, max_inflight=slots)

    def submit(i):
        kind, il, iu = reqs[i]["range"]
        return srv.submit(inputs[i][0], inputs[i][1], range=kind, il=il, iu=iu)

    # closed loop: keep `window` requests in flight
    done, t_first = [], None
    inflight = []
    k = 0
    t0 = time.perf_counter()
    while k < calib or inflight:
        while k < calib and len(inflight) < window:
            inflight.append(submit(k))
            k += 1
        res, _, _ = srv.wait(inflight.pop(0))
        done.append(res)
    t_closed = time.perf_counter() - t0
    sat = calib / t_closed

    def open_loop(rate, rs):
        gaps = rs.exponential(1.0 / rate, n_req)
        arrive = np.cumsum(gaps)
        tickets = [None] * n_req
        lag = np.zeros(n_req)
        ready = threading.Semaphore(0)
        base = time.monotonic()

        def producer():
            for i in range(n_req):
                dt = base + arrive[i] - time.monotonic()
                if dt > 0:
                    time.sleep(dt)
                lag[i] = max(0.0, time.monotonic() - (base + arrive[i]))
                tickets[i] = submit(i)
                ready.release()

        th = threading.Thread(target=producer)
        th.start()
        lat, bs = [], []
        for i in range(n_req):
            ready.acquire()
            res, _, _ = srv.wait(tickets[i])
            lat.append(res["done_ms"] - res["submit_ms"] + lag[i] * 1e3)
            bs.append(res["batch_size"])
        th.join()
        span = time.monotonic() - base
        return {"offered_req_per_s": round(rate, 1), "achieved_req_per_s": round(n_req / span, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_batch": round(float(np.mean(bs)), 2),
                "roofline_frac": round(mean_flops * n_req / span / peak, 5)}

    rs = np.random.default_rng(seed + 101)
    out = {"workload": f"{n_req} requests, n log-uniform in [64, 8192], 50/50 fp32/fp64 I/O, "
                       "30% index range of ceil(0.1 n), 50/50 U(-1,1) or 1-2-1 + N(0,(1e-6)^2), "
                       f"seed {seed}; HBM budget 50% of free",
           "slots": slots,
           "saturation_req_per_s": round(sat, 1),
           "saturation_eigenpairs_per_s": round(sum(r["m"] for r in done) / t_closed, 1),
           "saturation_roofline_frac": round(mean_flops * sat / peak, 5),
           "plain": {"req_per_s": round(n_plain / t_plain, 1),
                     "eigenpairs_per_s": round(pairs_plain / t_plain, 1),
                     "p50_ms": round(float(np.median(pl_ms)), 3),
                     "p99_ms": round(float(np.percentile(pl_ms, 99)), 3),
                     "roofline_frac": round(sum(flops_req) / t_plain / peak, 5),
                     "sample": f"first {n_plain} requests, one mr3_solve_f32/f64 each in sequence"},
           "mean_alg_flops_per_request": round(mean_flops, 1),
           "load_0.5": open_loop(0.5 * sat, rs),
           "load_0.8": open_loop(0.8 * sat, rs)}
    srv.close()
    return out


def single_legs(mr3, steps):
    """C1: n = 512 FP32 (U(-1,1) and 1-2-1), one mr3_solve_f32 per call, p50/p99
    latency; C2: glued Wilkinson n = 4096 FP64 (double-double), one
    mr3_solve_f64 per call.  Inputs resident on the device."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    h = mr3.Handle(0)
    for name, (d, e), reps in (("c1_uniform_n512_fp32", W.uniform(512, 0, np.float32), 200),
                               ("c1_121_n512_fp32", W.toeplitz_121(512, np.float32), 200),
                               ("c2_glued_wilkinson_n4096_fp64", W.glued_wilkinson(4096), max(steps, 10))):
        n = d.size
        dg, eg = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        Wt = torch.empty(n, dtype=dg.dtype, device=dev)
        Zt = torch.empty((n, n), dtype=dg.dtype, device=dev)
        fn = mr3.mr3_solve_f32 if d.dtype == np.float32 else mr3.mr3_solve_f64
        for _ in range(3):
            fn(h, n, dg, eg, mr3.RANGE_ALL, 0.0, 0.0, 1, n, Wt, Zt, n, stream)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            ts = time.perf_counter()
            fn(h, n, dg, eg, mr3.RANGE_ALL, 0.0, 0.0, 1, n, Wt, Zt, n, stream)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - ts) * 1e3)
        st = h.stats()
        med = float(np.median(ms))
        flops = alg_flops(st, "f64" if d.dtype == np.float32 else "dd")
        (o_off, o_diag), resid = mr3.check(dg.double(), eg.double(), Wt.double(), Zt.double().T, handle=h)
        gate = 10 * n * (2.0 ** -24 if d.dtype == np.float32 else 2.0 ** -53)
        out[name] = {"eigenpairs_per_s": round(n / (med / 1e3), 1), "p50_ms": round(med, 3),
                     "p99_ms": round(float(np.percentile(ms, 99)), 3), "calls": reps,
                     "roofline_frac": round(flops / (med / 1e3) / (FP64_VECTOR_PEAK_TFLOPS * 1e12), 5),
                     "tree": {"d_max": st["d_max"], "clusters": st["n_clusters"],
                              "largest_cluster": st["largest_cluster"]},
                     "orthogonality_over_gate": round(max(o_off, o_diag) / gate, 5),
                     "residual_over_gate": round(resid / gate, 5)}
    h.close()
    return out


def dense_leg(mr3, sizes=(2000, 4000), reps=3):
    """The dense pipeline (Sec. 4.2, Fig. 3): A = Q T Q^T for the
    prescribed-spectrum tridiagonal T and a seeded random orthogonal Q, all
    eigenpairs through mr3_dense_f64 (reduction, this solver,
    back-transformation) against torch.linalg.eigh on the same device (the
    plain dense path), with residual and orthogonality of both in units of
    n eps.  A is resident on the device; each call reduces a fresh copy."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    h = mr3.Handle(0)
    out = {}
    eps = 2.0 ** -53

    def quality(A, w, Z):
        n = A.shape[0]
        nA = A.abs().sum(dim=0).max()
        R = ((A @ Z - Z * w[None, :]).abs().sum(dim=0).max() / nA / (n * eps)).item()
        O = ((Z.T @ Z - torch.eye(Z.shape[1], dtype=Z.dtype, device=dev)).abs().max() / (n * eps)).item()
        return round(R, 4), round(O, 4)

    for n in sizes:
        d, e, _ = W.prescribed_spectrum(n, 0)
        A = torch.from_numpy(W.dense_from_tridiagonal(d, e, 1)).to(dev)
        Acm = A.t().contiguous()
        work = torch.empty_like(Acm)
        Wt = torch.empty(n, dtype=torch.float64, device=dev)
        Zt = torch.empty((n, n), dtype=torch.float64, device=dev)
        ms, ms_ref = [], []
        for k in range(reps + 1):
            work.copy_(Acm)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            mr3.mr3_dense_f64(h, n, work, n, mr3.RANGE_ALL, 0.0, 0.0, 1, n, Wt, Zt, n, stream)
            torch.cuda.synchronize()
            if k:
                ms.append((time.perf_counter() - ts) * 1e3)
        ours = quality(A, Wt, Zt.T)
        for k in range(reps + 1):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            wr, Zr = torch.linalg.eigh(A)
            torch.cuda.synchronize()
            if k:
                ms_ref.append((time.perf_counter() - ts) * 1e3)
        ref = quality(A, wr, Zr)
        out[f"dense_qtq_n{n}_fp64"] = {
            "mr3_dense_ms": round(float(np.median(ms)), 2),
            "torch_eigh_ms": round(float(np.median(ms_ref)), 2),
            "mr3_dense": {"residual_n_eps": ours[0], "orthogonality_n_eps": ours[1]},
            "torch_eigh": {"residual_n_eps": ref[0], "orthogonality_n_eps": ref[1]},
        }
    h.close()
    return out


def erep_study(mr3, reps=5):
    """The e-representation without cached derived data (derive_lld = 1)
    against the stored-lld variant on the n = 20000 prescribed matrix, FP64:
    solve time with per-stage device times, and the workspace sizes of the
    query (full speed and minimum)."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    n = 20000
    d, e, _ = W.prescribed_spectrum(n, 0)
    dg, eg = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
    Wt = torch.empty(n, dtype=torch.float64, device=dev)
    Zt = torch.empty((n, n), dtype=torch.float64, device=dev)
    for derive in (0, 1):
        h = mr3.Handle(0)
        h.set_params(precision=64, derive_lld=derive, profile=1)
        ms = []
        for k in range(reps + 1):
            ts = time.perf_counter()
            mr3.mr3_solve_f64(h, n, dg, eg, mr3.RANGE_ALL, 0.0, 0.0, 1, n, Wt, Zt, n)
            torch.cuda.synchronize()
            if k:
                ms.append((time.perf_counter() - ts) * 1e3)
        st = h.stats()
        print(json.dumps({"derive_lld": derive, "n": n, "p50_ms": round(float(np.median(ms)), 3),
                          "stage_ms": {k: round(v, 3) for k, v in zip(mr3.STAGES, st["stage_ms"])},
                          "workspace_full_bytes": mr3.mr3_workspace_bytes(h, n, mr3.RANGE_ALL, 0, 64),
                          "workspace_min_bytes": mr3.mr3_workspace_min_bytes(h, n, mr3.RANGE_ALL, 0, 64)}),
              flush=True)
        h.close()


def gaptol_study(mr3):
    """Clustering rho (largest cluster / n), tree depth and solve time against
    gaptol, with and without splitting by absolute gaps (gaptol_abs = gaptol)
    and with and without the refinement of cluster ends in y before the shift,
    on the synthetic stand-ins of the paper's matrix types.  FP64 gaptols
    below 20 n eps run with their brackets refined in y."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    cases = [
        ("uniform n=512 fp32", *W.uniform(512, 0, np.float32)),
        ("1-2-1 n=512 fp32", *W.toeplitz_121(512, np.float32)),
        ("N(0,1) n=1024 fp32", *W.normal(1024, 1, np.float32)),
        ("1-2-1 + noise n=8192 fp32", *W.toeplitz_121_noisy(8192, 0, 1e-6, np.float32)),
        ("1-2-1 + noise n=8192 fp64", *W.toeplitz_121_noisy(8192, 0, 1e-6, np.float64)),
        ("glued Wilkinson n=4096 fp64", *W.glued_wilkinson(4096)),
        ("prescribed n=20000 fp64", *W.prescribed_spectrum(20000, 0)[:2]),
    ]
    rows = []
    for name, d, e in cases:
        n = d.size
        prec = 32 if d.dtype == np.float32 else 64
        tols = (1e-3, 1e-4, 1e-5, 1e-6, 1e-7) if prec == 32 else (1e-3, 1e-5, 1e-8, 1e-10, 1e-12, 1e-13)
        dg, eg = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        for g in tols:
            for ab, ends in ((0.0, 0), (g, 0), (0.0, 1)):
                h = mr3.Handle(0)
                h.set_params(precision=prec, gaptol=g, gaptol_abs=ab, refine_ends=ends)
                try:
                    mr3.solve(dg, eg, handle=h)
                except mr3.MR3Error as err:
                    if err.code != mr3.MR3_ERR_GAPTOL:
                        raise
                    row = {"matrix": name, "gaptol": g, "abs_split": ab > 0, "refine_ends": ends,
                           "rejected": "gaptol below min(1e-3, eps_y sqrt(n) / eps_x)"}
                    rows.append(row)
                    print(json.dumps(row), flush=True)
                    h.close()
                    continue
                torch.cuda.synchronize()
                ts = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    Wg, Zg = mr3.solve(dg, eg, handle=h)
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t0) * 1e3)
                st = h.stats()
                row = {"matrix": name, "gaptol": g, "abs_split": ab > 0, "refine_ends": ends,
                       "rho": max(st["largest_cluster"], 1) / n, "d_max": st["d_max"],
                       "clusters": st["n_clusters"], "y_refined": st["n_y_refined"],
                       "best_candidate": st["n_best_candidate"], "ms": round(float(np.median(ts)), 3)}
                if prec == 64:
                    (off, diag), res = mr3.check(dg, eg, Wg, Zg, handle=h)
                    row["orth"] = max(off, diag)
                    row["resid"] = res
                rows.append(row)
                print(json.dumps(row), flush=True)
                h.close()
    return rows


def dqds_study(mr3, steps=3):
    """Initial eigenvalues by dqds (one lane per root) against bisection, by
    eigenpairs/s: the 4096-problem batch (n log-uniform in [32, 1024], FP32
    I/O) and single prescribed-spectrum problems (FP64 I/O).  initial_ms is
    the device time of the initial eigenvalues (dqds or slicing, then the
    bracket check and multisection)."""
    import torch
    import workloads as W

    dev = torch.device("cuda:0")
    rows = []

    def timed(run, h, eigenpairs, reps):
        run()
        torch.cuda.synchronize()
        ts, bis = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            bis.append(h.stats()["stage_ms"][1])
        ms = float(np.median(ts))
        return {"ms": round(ms, 3), "initial_ms": round(float(np.median(bis)), 3),
                "eigenpairs_per_s": round(eigenpairs / (ms / 1e3), 1),
                "dqds_roots": h.stats()["n_dqds_roots"],
                "dqds_transforms": h.stats()["dqds_transforms"]}

    probs = W.batch_normal(4096, 32, 1024, seed=0, dtype=np.float32)
    ds = [torch.from_numpy(p[0]).to(dev) for p in probs]
    es = [torch.from_numpy(p[1]).to(dev) for p in probs]
    total = sum(p[0].size for p in probs)
    cases = [("batch 4096 x n in [32, 1024] fp32", 32, lambda h: mr3.solve_batched(ds, es, handle=h), total)]
    for n in (256, 512, 1024):
        d, e, _ = W.prescribed_spectrum(n, 0)
        dg, eg = torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev)
        cases.append((f"prescribed n={n} fp64", 64,
                      (lambda dg, eg: (lambda h: mr3.solve(dg, eg, handle=h)))(dg, eg), n))
    for name, prec, fn, pairs in cases:
        for init in (mr3.MR3_INITIAL_BISECTION, mr3.MR3_INITIAL_DQDS):
            h = mr3.Handle(0)
            h.set_params(precision=prec, initial=init, profile=1)
            row = {"problem": name, "initial": "dqds" if init else "bisection"}
            # dqds runs one lane per root for seconds: one timed repetition
            row.update(timed(lambda: fn(h), h, pairs, steps if init == mr3.MR3_INITIAL_BISECTION else 1))
            rows.append(row)
            print(json.dumps(row), flush=True)
            h.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-subset", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the C1 and C2 single-problem legs")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense A = Q T Q^T leg")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (calibrates "
                         "hardware byte counters against a known traffic) and exit")
    ap.add_argument("--gaptol-study", action="store_true",
                    help="only run the clustering study against gaptol and exit")
    ap.add_argument("--erep-study", action="store_true",
                    help="only compare the e-representation without cached lld with the stored "
                         "variant (time, workspace) and exit")
    ap.add_argument("--dqds-study", action="store_true",
                    help="only run the dqds against bisection comparison of initial eigenvalues "
                         "and exit")
    args = ap.parse_args()
    if args.erep_study:
        import paper_1304_1864_amd as mr3

        erep_study(mr3)
        return
    if args.dqds_study:
        import paper_1304_1864_amd as mr3

        dqds_study(mr3)
        return
    if args.gaptol_study:
        import paper_1304_1864_amd as mr3

        gaptol_study(mr3)
        return
    if args.copy_probe:
        import torch

        x = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on a single device)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1304_1864_amd as mr3

    n = args.n
    d, e = build_workload(n, args.seed)
    dev = torch.device("cuda:0")
    dg = torch.from_numpy(d).to(dev)
    eg = torch.from_numpy(e).to(dev)
    W = torch.empty(n, dtype=torch.float64, device=dev)
    Zt = torch.empty((n, n), dtype=torch.float64, device=dev)
    h = mr3.Handle(0)
    h.set_params(precision=64, profile=1)
    stream = torch.cuda.current_stream()

    def step():
        return mr3.mr3_solve_f64(h, n, dg, eg, mr3.RANGE_ALL, 0.0, 0.0, 1, n, W, Zt, n, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times = []
    stage_ms = np.zeros(8)
    stage_launch = np.zeros(8)
    work = np.zeros(3)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        m = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        st = h.stats()
        stage_ms += np.array(st["stage_ms"])
        stage_launch += np.array(st["stage_launches"])
        work += np.array([st["bisect_row_steps"], st["rqi_row_steps"], st["twist_row_steps"]])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert m == n
    value = n * args.steps / elapsed
    times_ms = np.array(times) * 1e3

    # roofline of the dominant stage (FP64 VALU bound)
    flops = {
        "bisect": work[0] * FLOPS_COUNT,
        "rqi": work[2] * FLOPS_TWIST + work[1] * FLOPS_RQI["dd"],
    }
    idx = {"bisect": 1, "rqi": 3}
    dom = max(idx, key=lambda k: stage_ms[idx[k]])
    dom_ms = stage_ms[idx[dom]]
    achieved = flops[dom] / (dom_ms * 1e-3) / 1e12 if dom_ms > 0 else 0.0
    roofline = {
        "bound": "alu",
        "kernel": "k_rqi<dd>" if dom == "rqi" else "k_bisect",
        "achieved": round(achieved, 3),
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
        "traffic": profiled_traffic("k_rqi<dd>" if dom == "rqi" else "k_bisect_staged"),
        "launches": int(stage_launch[idx[dom]]),
        "avg_launch_ms": round(dom_ms / max(stage_launch[idx[dom]], 1), 3),
    }
    stages = {name: round(stage_ms[i] / args.steps, 3) for i, name in enumerate(mr3.STAGES)}
    st = h.stats()
    # residual and orthogonality of the last timed solve, on the device
    (o_off, o_diag), resid = mr3.check(dg, eg, W, Zt.T, handle=h)
    gate = 10 * n * 2.0 ** -53
    accuracy = {"orthogonality_over_gate": round(max(o_off, o_diag) / gate, 5),
                "residual_over_gate": round(resid / gate, 5),
                "gates": "max|Z^T Z - I| and max ||T z - lambda z||_1 / ||T||_1 against 10 n eps"}

    extra = {}
    if not args.no_subset:
        ms = []
        for k in range(1 + max(2, args.steps)):
            ts = time.perf_counter()
            mr3.mr3_solve_f64(h, n, dg, eg, mr3.RANGE_INDEX, 0.0, 0.0, 1, 2000, W, Zt, n, stream)
            torch.cuda.synchronize()
            if k:
                ms.append((time.perf_counter() - ts) * 1e3)
        extra["subset_il1_iu2000"] = {"eigenpairs_per_s": round(2000 / (np.median(ms) / 1e3), 1),
                                      "p50_ms": round(float(np.median(ms)), 3)}

    if not args.no_single:
        extra["single_problem_legs"] = single_legs(mr3, args.steps)
    if not args.no_batched:
        hb = mr3.Handle(0)
        extra["batched_vs_plain"] = batched_c3(mr3, hb, max(3, args.steps), 1)
        hb.close()
    if not args.no_served:
        extra["served"] = served_c5(mr3)
    if not args.no_dense:
        extra["dense_vs_plain"] = dense_leg(mr3)

    cpu = None
    if not args.no_cpu_baseline:
        step()  # the timed solve's results again, for the comparison on the sample
        torch.cuda.synchronize()
        cpu = cpu_baseline(d, e, n, w_gpu=W.cpu().numpy(), z_gpu=lambda i: Zt[i].cpu().numpy())
    out = {
        "metric": "eigenpairs/s (n=20000, fp64 I/O, dd internal) batched vs plain; p50/p99 solve ms",
        "value": round(value, 2),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "p50_ms": round(float(np.percentile(times_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(times_ms, 99)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+dd",
        "data": "synthetic",
        "config": {"workload": f"prescribed-spectrum tridiagonal n={n} (geometric |lambda| 1..1e-8, "
                               f"random signs, seed {args.seed}), fp64 I/O, dd internal, all eigenpairs",
                   "n": n, "range": "all", "path": "plain (one mr3_solve_f64 per step)"},
        "stage_ms_per_step": stages,
        "tree": {"d_max": st["d_max"], "clusters": st["n_clusters"],
                 "largest_cluster": st["largest_cluster"],
                 "rqi_iters_per_pair": round(st["n_rqi_iters"] / max(n, 1), 3),
                 "fallbacks": st["n_fallbacks"], "best_candidate": st["n_best_candidate"]},
        "roofline": roofline,
        "accuracy": accuracy,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
