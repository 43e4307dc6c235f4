#!/usr/bin/env python3
"""Benchmark: CQRRPT on one MI355X, FP64 and mixed precision side by side,
reported as GFLOP/s normalised by 2 m n^2 with orthogonality
||Q^T Q - I||_2, reconstruction ||A[:,J] - Q R||_F / ||A||_F and per-step
latency percentiles.

Headline workload (default): the largest configuration that fits one GPU,
m = 4,194,304, n = 2,048 (68.7 GB of FP64 input), A = U diag(s) V^T with Haar
U, V, s geometric from 1 to 1e-12 over the first 1,536 entries and 0 after,
plus iid Gaussian noise of std 1e-16; sketch d = 2,560 rows with 8 nonzeros
per column; first-stage tolerance 1e-14 (the planted rank sits at the noise
floor, so the numerical rank is 2,048 and every step does its full work).
The input is built on the device block by block (CholeskyQR2 of a Gaussian
for U), untimed.

One step = one full factorization (sketch, QRCP, both rank stages,
preconditioning solve, Gram, Cholesky, Q, R product) of the resident input,
plus the copy of its rank to the host. The timed region holds exactly
--steps back-to-back steps bracketed by device synchronisation, with the
library's per-stage events off; stage times come from a separate run.

Prints ONE JSON line.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = ("CQRRPT GFLOP/s (2mn² norm.) FP64 vs mixed @ ‖QᵀQ−I‖; "
          "p50/p99 ms")
PEAK_FP64_MFMA = 78.6e12
PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12
HEADLINE = "fp64_4194304x2048_rank1536"

# Matrix-core stages: (stage, kernel, algorithmic flops per launch from
# (m, k_o, k)).
MFMA_STAGES = (
    ("precondition", "trsm_inv_kernel + trsm_rpack_kernel + trsm_dv_kernel",
     lambda m, ko, k: m * ko * ko),
    ("gram", "gram_dv_kernel<32, 1> + gram128_reduce_kernel", lambda m, ko, k: m * ko * (ko + 1)),
    ("q_solve", "qform_pack_kernel + qform_dv_kernel", lambda m, ko, k: m * k * k),
)
MIXED_STAGES = (
    ("precondition", "trsm_rows_kernel<128, float, float>", lambda m, ko, k: m * ko * ko,
     PEAK_FP32_MFMA),
    ("gram", "syrk_kernel<float> + syrk_reduce_kernel", lambda m, ko, k: m * ko * (ko + 1),
     PEAK_FP64_MFMA),
    ("q_solve", "qform_kernel<256, float, double, double>", lambda m, ko, k: m * k * k,
     PEAK_FP64_MFMA),
)
FP32_LINES_STAGES = (
    ("precondition", "trsm_rows_kernel<128, float, float>", lambda m, ko, k: m * ko * ko,
     PEAK_FP32_MFMA),
    ("gram", "gram128_kernel<float, float> + gram128_reduce_kernel",
     lambda m, ko, k: m * ko * (ko + 1), PEAK_FP32_MFMA),
    ("q_solve", "qform_kernel<256, float, double, float>", lambda m, ko, k: m * k * k,
     PEAK_FP32_MFMA),
)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-runs", action="store_true",
                    help="only the headline workload (FP64 and mixed)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed headline run")
    ap.add_argument("--cpu-rows", type=int, default=65536)
    ap.add_argument("--cpu-cols", type=int, default=1024)
    ap.add_argument("--serving-requests", type=int, default=4096,
                    help="requests in the serving-stream runs (0 skips them)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run three plain 1 GiB device copies (reference kernel for "
                         "scaling HBM byte counters)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# Quality, evaluated on the GPU in FP64 outside the timed region, by row
# blocks (the largest inputs leave no room for m x n temporaries).
# ---------------------------------------------------------------------------

def quality(torch, A, Q, R, J, k, block=1 << 18):
    m, n = A.shape
    dev = A.device
    G = torch.zeros((k, k), dtype=torch.float64, device=dev)
    e2 = torch.zeros((), dtype=torch.float64, device=dev)
    a2 = torch.zeros((), dtype=torch.float64, device=dev)
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        Qb = Q[r0:r1]
        if k:
            G += Qb[:, :k].t() @ Qb[:, :k]
        Ab = A[r0:r1]
        e2 += torch.linalg.norm(Ab[:, J] - Qb @ R) ** 2
        a2 += torch.linalg.norm(Ab) ** 2
    orth = 0.0
    if k:
        G -= torch.eye(k, dtype=torch.float64, device=dev)
        orth = float(np.max(np.abs(np.linalg.eigvalsh(G.cpu().numpy()))))
    return orth, float(torch.sqrt(e2 / a2))


# ---------------------------------------------------------------------------
# Timed runs
# ---------------------------------------------------------------------------

def timed(P, torch, A, w, mode, tol, seed, steps, warmup, implicit=False, f=None):
    """--steps back-to-back factorizations, each with the copy of its rank to
    pinned host memory, between two synchronisations; per-step HIP events on
    the library's stream (torch's current stream) give the percentiles."""
    m, n, d, nnz = w["m"], w["n"], w["d"], w["nnz"]
    if f is None:
        f = P.Factorization(m, n, d, nnz, mode, implicit=implicit)
    rank_host = torch.empty((max(steps, 1), 1), dtype=torch.int64, pin_memory=True)
    for _ in range(warmup):
        f.run(A, seed, tol)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for i in range(steps):
        ev[i][0].record()
        f.run(A, seed, tol)
        rank_host[i].copy_(f.info_buf[:8].view(torch.int64), non_blocking=True)
        ev[i][1].record()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    per = np.array([a.elapsed_time(b) for a, b in ev])
    info = f.info()
    assert int(rank_host[steps - 1, 0]) == int(info.rank)
    ms = total_ms / steps
    return dict(f=f, ms=ms, wall_s=wall, p50=float(np.percentile(per, 50)),
                p99=float(np.percentile(per, 99)), min=float(per.min()),
                max=float(per.max()), rank=int(info.rank),
                rank_stage1=int(info.rank_stage1), passes=int(info.cholqr2_passes),
                orth_est=float(info.orth_est), gflops=2.0 * m * n * n / (ms * 1e-3) / 1e9)


def stage_run(P, torch, A, f, seed, tol, steps):
    """Per-stage HIP events (recorded by the library on its stream) over a
    separate run of ``steps`` factorizations; mean ms per stage."""
    torch.cuda.synchronize()
    P.stage_timing(steps)
    for _ in range(steps):
        f.run(A, seed, tol)
    rows = [P.stage_times(i) for i in range(steps)]
    P.stage_timing(0)
    return {k: float(np.mean([r[k] for r in rows])) for k in P.STAGES}


def rooflines(stages, w, ko, k, mixed=False, fp32_lines=False):
    """Per-kernel rooflines from the stage times: algorithmic work of one
    launch over its mean duration. Matrix-core stages in TFLOP/s against the
    peak of their instruction type; the sketch in GB/s against HBM (it reads
    A once: 8 m n bytes, plus 8 d n written per row chunk, not counted)."""
    m, n, d = w["m"], w["n"], w["d"]
    out = {}
    table = (FP32_LINES_STAGES if fp32_lines else MIXED_STAGES if mixed else
             tuple(s + (PEAK_FP64_MFMA,) for s in MFMA_STAGES))
    for stage, kernel, work, peak in table:
        t = stages[stage] * 1e-3
        flops = float(work(m, ko, k))
        out[stage] = {"kernel": kernel, "bound": "mfma", "unit": "TFLOP/s",
                      "achieved": flops / t / 1e12, "peak": peak / 1e12,
                      "frac": flops / t / peak, "avg_launch_ms": t * 1e3,
                      "algorithmic_flops_per_launch": flops}
    t = stages["sketch"] * 1e-3
    byts = 8.0 * m * n
    out["sketch"] = {"kernel": "saso_index_kernel + saso_partial_reg_kernel + saso_reduce_kernel",
                     "bound": "hbm", "unit": "GB/s", "achieved": byts / t / 1e9,
                     "peak": PEAK_HBM / 1e9, "frac": byts / t / PEAK_HBM,
                     "avg_launch_ms": t * 1e3, "algorithmic_bytes_per_launch": byts}
    qr_flops = 2.0 * d * n * n - 2.0 * n ** 3 / 3.0
    out["qrcp"] = {"kernel": "qrcp_reg_kernel", "bound": "latency",
                   "avg_launch_ms": stages["qrcp"], "flops": qr_flops,
                   "achieved_tflops": qr_flops / (stages["qrcp"] * 1e-3) / 1e12}
    return out


def kernel_source_hash():
    """Hash of the sources of the three matrix-core stages (tall.hip, gram.hip,
    qform_dv.hip)."""
    h = hashlib.sha256()
    for name in ("tall.hip", "gram.hip", "qform_dv.hip"):
        with open(os.path.join(HERE, "paper_2311_08316_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(stage):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    name = {"precondition": "trsm", "gram": "gram_dv", "q_solve": "qform"}.get(stage)
    if name is None:
        return None
    path = os.path.join(HERE, "profiles", f"{name}_fp64_4194304x2048_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                key, val = line.split("=", 1)
                vals[key.strip()] = val.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def headline_roofline(roofs):
    """The dominant kernel: the matrix-core stage with the longest launch."""
    stage = max(("precondition", "gram", "q_solve"), key=lambda s: roofs[s]["avg_launch_ms"])
    r = roofs[stage]
    return {"kernel": r["kernel"], "stage": stage, "bound": "mfma", "achieved": r["achieved"],
            "peak": r["peak"], "unit": "TFLOP/s", "frac": r["frac"],
            "traffic": measured_traffic(stage), "avg_launch_ms": r["avg_launch_ms"],
            "algorithmic_flops_per_launch": r["algorithmic_flops_per_launch"],
            "others": {s: v for s, v in roofs.items() if s != stage}}


# ---------------------------------------------------------------------------
# Measured ceilings
# ---------------------------------------------------------------------------

def measured_peaks(P, torch):
    n = 1 << 27  # 1 GiB of FP64
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 0.0
    for _ in range(5):
        torch.cuda.synchronize()
        e0.record()
        P.probe_copy(src, dst)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 16.0 * n / (e0.elapsed_time(e1) * 1e-3))
    del src, dst
    out = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    res = {"copy_GBps": best / 1e9, "copy_frac_of_datasheet": best / PEAK_HBM}
    for fp64, key, peak in ((True, "mfma_f64_TFLOPs", PEAK_FP64_MFMA),
                            (False, "mfma_f32_TFLOPs", PEAK_FP32_MFMA)):
        rate = 0.0
        for _ in range(3):
            torch.cuda.synchronize()
            e0.record()
            fl = P.probe_mfma(out, 4000, fp64=fp64)
            e1.record()
            torch.cuda.synchronize()
            rate = max(rate, fl / (e0.elapsed_time(e1) * 1e-3))
        res[key] = rate / 1e12
        res[key.replace("TFLOPs", "frac_of_datasheet")] = rate / peak
    return res


# ---------------------------------------------------------------------------
# CPU baseline and serving
# ---------------------------------------------------------------------------

def cpu_baseline(A_host_sample, w, seed, tol):
    """The oracle as it stands, on a bounded sample of the headline input."""
    from oracle import cqrrpt_oracle as O
    ms, ns = A_host_sample.shape
    ds = math.ceil(1.25 * ns)
    t0 = time.perf_counter()
    out = O.cqrrpt(A_host_sample, ds, w["nnz"], seed, tol)
    t = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        cores = min(cores, int(omp))
    return {"value": 2.0 * ms * ns * ns / t / 1e9, "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": f"one full oracle factorization of the leading {ms} x {ns} block of the "
                      f"headline input (d={ds}, nnz={w['nnz']}, tol={tol}); {t:.1f} s; "
                      f"GFLOP/s normalised by 2*{ms}*{ns}^2",
            "seconds": t, "rank": int(out["rank"])}


def serving_run(P, torch, W, count, mode, seed, slots=4, budget_gib=64.0, inflight_gib=96.0):
    """Serving stream: Poisson arrivals at the recipe's rate; each request's
    matrix is generated on the device at its arrival time and submitted. The
    client holds at most ``inflight_gib`` of inputs and outputs on the
    device; a request that arrives while the client is at that cap waits in
    the client's queue, and its latency still counts from its scheduled
    arrival. Latency = completion (the server's clock) - scheduled arrival;
    throughput = requests and 2mn^2 flops over the span from the first
    arrival to the last completion."""
    stream = W.serving_stream(count, seed=seed)
    srv = P.Server(int(budget_gib * 2 ** 30), slots=slots, mode=mode)
    live, done = [], []
    held = [0]

    def collect(block):
        keep = []
        for tk, r, nbytes, t_arr in live:
            fin = srv.poll(tk)
            if not fin and block:
                while not srv.poll(tk):
                    time.sleep(1e-4)
                fin = True
            if fin:
                ts, ta, td = srv.times(tk)
                _, _, _, info = srv.result(tk)
                done.append((t_arr, ts, ta, td, r, int(info.rank)))
                held[0] -= nbytes
            else:
                keep.append((tk, r, nbytes, t_arr))
        live[:] = keep

    t0 = time.perf_counter()
    clock0 = None
    for r in stream:
        wait = r["t"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        nbytes = 16 * r["m"] * r["n"]
        while held[0] + nbytes > inflight_gib * 2 ** 30 and live:
            collect(False)
            time.sleep(2e-4)
        A = W.serving_matrix_gpu(r["m"], r["n"], r["seed"])
        py_submit = time.perf_counter()
        tk = srv.submit(A, r["d"], r["nnz"], r["seed"], r["tol"])
        ts = srv.times(tk)[0]
        if clock0 is None:
            # Offset between the server's steady clock and perf_counter.
            clock0 = ts - py_submit * 1e3
        live.append((tk, r, nbytes, clock0 + (t0 + r["t"]) * 1e3))
        held[0] += nbytes
        del A
        collect(False)
    srv.drain()
    collect(True)
    srv.close()
    lat = np.array([td - t_arr for t_arr, ts, ta, td, r, k in done])
    queue = np.array([ta - t_arr for t_arr, ts, ta, td, r, k in done])
    span_s = (max(d[3] for d in done) - min(d[0] for d in done)) * 1e-3
    flops = sum(2.0 * r["m"] * r["n"] ** 2 for *_, r, k in done)
    full_rank = sum(1 for *_, r, k in done if k == r["n"])
    return {"requests": len(done), "slots": slots,
            "offered_rate_req_s": W.SERVING["rate_per_s"],
            "p50_latency_ms": float(np.percentile(lat, 50)),
            "p99_latency_ms": float(np.percentile(lat, 99)),
            "mean_queue_ms": float(queue.mean()),
            "throughput_req_s": len(done) / span_s,
            "gflops_2mn2": flops / span_s / 1e9, "span_s": span_s,
            "full_rank_results": full_rank}


def dense_sketch_run(P, torch, W, seed, reps=5):
    """CQRRPT on the 131,072 x 1,024 planted-rank input (tol 1e-14) with the
    Gaussian and SRHT operators (Sec. 2.3.1; S formed explicitly, the sketch
    one FP64 matrix-core product) beside the SASO: wall time per call
    (synchronous form) and rank."""
    A, w = W.make_workload_gpu("fp64_131072x1024_rank512", seed=seed)
    out = {}
    for name, kind in (("gaussian", P.SKETCH_GAUSSIAN), ("srht", P.SKETCH_SRHT)):
        P.factor_dense(A, w["d"], kind, seed, w["tol"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            Q, R, J, info = P.factor_dense(A, w["d"], kind, seed, w["tol"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        orth, recon = quality(torch, A, Q, R, J, int(info.rank))
        out[name] = {"ms_per_call": ms, "rank": int(info.rank), "orth": orth, "recon": recon}
        del Q, R, J
    log(f"dense sketches: {json.dumps(out)}")
    del A
    torch.cuda.empty_cache()
    return out


def gamma_sweep(P, torch, seed):
    """Sec. 5.2.1: runtime against the embedding dimension d = gamma n on
    Gaussian 131,072 x n inputs (nnz = 4, tol 1e-14), for the shapes whose
    sketch QRCP fits the register-resident kernel (d <= 2560)."""
    out = {}
    m = 131_072
    for n, gammas in ((1024, (1.0, 1.25, 1.5, 2.0, 2.5)), (2048, (1.0, 1.25))):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed + n)
        A = torch.randn((n, m), dtype=torch.float64, device="cuda", generator=gen).t()
        w = dict(m=m, n=n, nnz=4)
        for g in gammas:
            w["d"] = math.ceil(g * n)
            r = timed(P, torch, A, w, P.CQRRPT_FP64, 1e-14, seed, 5, 1)
            f = r.pop("f")
            st = stage_run(P, torch, A, f, seed, 1e-14, 1)
            out[f"{m}x{n}_gamma{g:g}"] = {"d": w["d"], "ms": r["ms"], "rank": r["rank"],
                                          "sketch_ms": st["sketch"], "qrcp_ms": st["qrcp"]}
            del f
        del A
        torch.cuda.empty_cache()
    log(f"gamma sweep: {json.dumps(out)}")
    return out


def hqrrp_study(P, torch, W, seed, reps=5):
    """Sec. 5.2.2: HQRRP (block 16, oversampling 8) against the GEQP3-order
    QRCP on sketch shapes (Gaussian d x n), and CQRRPT with HQRRP on the
    131,072 x 1,024 planted-rank input: time per call (device events around
    ``reps`` calls, each allocating through torch's cache), trailing-norm
    ratio max_l ||R_h[l:, l:]||_F / ||R_q[l:, l:]||_F (pivot quality against
    the QRCP's), rank and quality."""
    out = {}
    for d, n in ((1280, 1024), (2560, 2048)):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed + d)
        X = torch.randn((n, d), dtype=torch.float64, device="cuda", generator=gen).t()
        row = {}
        for name, fn in (("qrcp", lambda: P.qrcp(X)), ("hqrrp", lambda: P.hqrrp(X, 16, 8, seed))):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                r = fn()
            e1.record()
            torch.cuda.synchronize()
            row[name + "_ms"] = e0.elapsed_time(e1) / reps
            row[name + "_R"] = r[1]
        tq = torch.sqrt(torch.flip(torch.cumsum(torch.flip((torch.triu(row.pop("qrcp_R")) ** 2).sum(1), [0]), 0), [0]))
        th = torch.sqrt(torch.flip(torch.cumsum(torch.flip((torch.triu(row.pop("hqrrp_R")) ** 2).sum(1), [0]), 0), [0]))
        ratio = (th / torch.clamp(tq, min=1e-300)).cpu().numpy()
        row["trailing_hqrrp_over_qrcp_max"] = float(ratio.max())
        row["trailing_hqrrp_over_qrcp_median"] = float(np.median(ratio))
        out[f"sketch_{d}x{n}"] = row
        del X
    A, w = W.make_workload_gpu("fp64_131072x1024_rank512", seed=seed)
    for tol in (1e-14, 1e-9):
        P.factor_hqrrp(A, w["d"], w["nnz"], seed, tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            Q, R, J, info = P.factor_hqrrp(A, w["d"], w["nnz"], seed, tol)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        orth, recon = quality(torch, A, Q, R, J, int(info.rank))
        out[f"factor_131072x1024_tol{tol:g}"] = {"ms_per_call": ms, "rank": int(info.rank),
                                                 "orth": orth, "recon": recon}
        del Q, R, J
    del A
    torch.cuda.empty_cache()
    log(f"hqrrp: {json.dumps(out)}")
    return out


def high_coherence_study(P, torch, W, seed, m=32_768, n=500):
    """Sec. 4.2 on a smaller instance of the same construction (stacked
    identities, n rows scaled by 1e10, rotated by a random orthogonal
    matrix): pivot quality of CQRRPT with (gamma, nnz) = (1, 1) and
    (1.25, 4): |R[l,l]| / sigma_l (sigma from the singular values of R, which
    are A's) and ||C_l^GEQP3||_F / ||C_l^ours||_F (trailing blocks of the
    R factors; GEQP3 from LAPACK on the host), with rank, orthogonality and
    reconstruction."""
    import scipy.linalg
    A_h = W.high_coherence_matrix(m, n, seed + 4, boost=1e10)
    _, R3, _ = scipy.linalg.qr(A_h, mode="economic", pivoting=True)
    c3 = np.sqrt(np.cumsum((np.triu(R3) ** 2).sum(axis=1)[::-1])[::-1])
    A = torch.from_numpy(A_h).to("cuda").t().contiguous().t()
    out = {}
    for gamma, nnz in ((1.0, 1), (1.25, 4)):
        d = math.ceil(gamma * n)
        Q, R, J, info = P.factor(A, d, nnz, seed, 1e-14)
        k = int(info.rank)
        orth, recon = quality(torch, A, Q, R, J, k)
        Rh = R.cpu().numpy()
        sv = np.linalg.svd(Rh[:k, :], compute_uv=False)
        diag = np.abs(np.diag(Rh))[:k]
        ratio_r = diag / sv[:k]
        co = np.sqrt(np.cumsum((np.triu(Rh) ** 2).sum(axis=1)[::-1])[::-1])[:k]
        ratio_c = c3[:k] / np.maximum(co, 1e-300)
        out[f"gamma{gamma:g}_nnz{nnz}"] = {
            "d": d, "rank": k, "rank_stage1": int(info.rank_stage1),
            "chol_fail_col": int(info.chol_fail_col), "orth": orth, "recon": recon,
            "diag_over_sigma_min": float(ratio_r.min()), "diag_over_sigma_max": float(ratio_r.max()),
            "trailing_geqp3_over_ours_min": float(ratio_c.min()),
            "trailing_geqp3_over_ours_max": float(ratio_c.max())}
    log(f"high coherence: {json.dumps(out)}")
    del A
    torch.cuda.empty_cache()
    return out


def summary(r):
    keys = ("gflops", "ms", "p50", "p99", "min", "max", "rank", "rank_stage1", "passes",
            "orth", "recon", "orth_est")
    return {k: r[k] for k in keys if k in r}


def run_config(P, torch, W, name, seed, steps, modes, stage_steps=2, tols=None):
    A, w = W.make_workload_gpu(name, seed=seed)
    torch.cuda.synchronize()
    res = {}
    for mode_name, mode in modes:
        for tol in (tols or (w["tol"],)):
            r = timed(P, torch, A, w, mode, tol, seed, steps, 1)
            f = r.pop("f")
            r["orth"], r["recon"] = quality(torch, A, f.Q, f.R, f.J, r["rank"])
            st = stage_run(P, torch, A, f, seed, tol, stage_steps)
            r["stages_ms"] = st
            r["rooflines"] = rooflines(st, w, r["rank_stage1"], r["rank"],
                                       mixed=mode != P.CQRRPT_FP64,
                                       fp32_lines=mode == P.CQRRPT_MIXED_FP32_CHOLQR2)
            key = mode_name if tols is None else f"{mode_name}_tol{tol:g}"
            res[key] = r
            log(f"  {name} {key}: {json.dumps(summary(r))}")
            del f
    del A
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the factorization would shard by row blocks, with one all-reduce "
              "of the sketch and one of the Gram).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2311_08316_amd as P
    from paper_2311_08316_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    P.lib()
    t0 = time.perf_counter()
    A, w = W.make_workload_gpu(args.workload, seed=args.seed)
    torch.cuda.synchronize()
    log(f"generated {args.workload} in {time.perf_counter() - t0:.1f} s")
    m, n, d, nnz, tol = w["m"], w["n"], w["d"], w["nnz"], w["tol"]

    # Headline: FP64.
    main_res = timed(P, torch, A, w, P.CQRRPT_FP64, tol, args.seed, args.steps, args.warmup)
    f = main_res.pop("f")
    log(f"fp64: {main_res['ms']:.3f} ms/step, {main_res['gflops']:.0f} GFLOP/s, "
        f"rank {main_res['rank']}")
    main_res["orth"], main_res["recon"] = quality(torch, A, f.Q, f.R, f.J, main_res["rank"])
    stages = stage_run(P, torch, A, f, args.seed, tol, 2)
    roofs = rooflines(stages, w, main_res["rank_stage1"], main_res["rank"])
    roof = headline_roofline(roofs)
    log(f"fp64 quality orth {main_res['orth']:.2e} recon {main_res['recon']:.2e}; "
        f"stages {json.dumps({k: round(v, 3) for k, v in stages.items()})}")
    log(f"roofline: {json.dumps({k: v for k, v in roof.items() if k != 'others'})}")
    del f
    torch.cuda.empty_cache()

    # Mixed precision on the same input.
    mixed = None
    if not args.no_mixed:
        mr = timed(P, torch, A, w, P.CQRRPT_MIXED, tol, args.seed, args.steps, args.warmup)
        fm = mr.pop("f")
        mr["orth"], mr["recon"] = quality(torch, A, fm.Q, fm.R, fm.J, mr["rank"])
        mst = stage_run(P, torch, A, fm, args.seed, tol, 2)
        mixed = summary(mr)
        mixed.update({"mode": "mixed (FP32 preconditioning solve, FP64 CholeskyQR lines)",
                      "speedup_vs_fp64": main_res["ms"] / mr["ms"], "stages_ms": mst,
                      "rooflines": rooflines(mst, w, mr["rank_stage1"], mr["rank"], mixed=True)})
        log(f"mixed: {json.dumps(summary(mr))}")
        del fm
        torch.cuda.empty_cache()

    extra = {}
    if not args.no_extra_runs and not args.no_mixed:
        mc = timed(P, torch, A, w, P.CQRRPT_MIXED_CHECKED, tol, args.seed, 2, 1)
        fc = mc.pop("f")
        mc["orth"], mc["recon"] = quality(torch, A, fc.Q, fc.R, fc.J, mc["rank"])
        extra["headline_mixed_checked"] = summary(mc)
        extra["headline_mixed_checked"]["speedup_vs_fp64"] = main_res["ms"] / mc["ms"]
        log(f"mixed checked: {json.dumps(summary(mc))}")
        del fc
        torch.cuda.empty_cache()

    sample = None
    if not args.no_cpu_baseline:
        sample = np.asfortranarray(A[:min(args.cpu_rows, m), :min(args.cpu_cols, n)]
                                   .cpu().numpy())
    del A
    torch.cuda.empty_cache()

    peaks = measured_peaks(P, torch)
    log(f"measured peaks: {peaks}")

    if not args.no_extra_runs:
        fp64 = (("fp64", P.CQRRPT_FP64),)
        all3 = fp64 + (("mixed", P.CQRRPT_MIXED), ("mixed_checked", P.CQRRPT_MIXED_CHECKED),
                       ("mixed_fp32_lines_cholqr2", P.CQRRPT_MIXED_FP32_CHOLQR2))
        extra["fp64_10000x100_cond1e6"] = run_config(P, torch, W, "fp64_10000x100_cond1e6",
                                                     args.seed, 200, fp64)
        extra["fp64_131072x1024_rank512"] = run_config(
            P, torch, W, "fp64_131072x1024_rank512", args.seed, 20, fp64, tols=(1e-14, 1e-9))
        extra["mixed_1048576x512_cond1e10"] = run_config(
            P, torch, W, "mixed_1048576x512_cond1e10", args.seed, 10, all3)
        # Implicit Q on the 131072 x 1024 input.
        A2, w2 = W.make_workload_gpu("fp64_131072x1024_rank512", seed=args.seed)
        ir = timed(P, torch, A2, w2, P.CQRRPT_FP64, w2["tol"], args.seed, 10, 1, implicit=True)
        ir.pop("f")
        extra["implicit_q_131072x1024"] = summary(ir)
        log(f"implicit Q: {json.dumps(summary(ir))}")
        del A2
        torch.cuda.empty_cache()
        extra["dense_sketch_131072x1024"] = dense_sketch_run(P, torch, W, args.seed)
        extra["gamma_sweep"] = gamma_sweep(P, torch, args.seed)
        extra["high_coherence_32768x500"] = high_coherence_study(P, torch, W, args.seed)
        extra["hqrrp_vs_qrcp"] = hqrrp_study(P, torch, W, args.seed)
        if args.serving_requests > 0:
            srv = {}
            for name, mode in (("fp64", P.CQRRPT_FP64), ("mixed", P.CQRRPT_MIXED)):
                srv[name] = serving_run(P, torch, W, args.serving_requests, mode, args.seed)
                log(f"serving ({name}): {srv[name]}")
            extra["serving_stream"] = srv

    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x copy of 1 GiB (reads 1 GiB, writes 1 GiB each)")
        del src, dst

    cpu = None
    if sample is not None:
        cpu = cpu_baseline(sample, w, args.seed, tol)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": main_res["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "d": d, "nnz": nnz, "tol": tol,
                   "seed": args.seed, "mode": "fp64"},
        "p50_ms": main_res["p50"],
        "p99_ms": main_res["p99"],
        "min_ms": main_res["min"],
        "max_ms": main_res["max"],
        "rank": main_res["rank"],
        "orth": main_res["orth"],
        "recon": main_res["recon"],
        "stages_ms": stages,
        "roofline": roof,
        "mixed": mixed,
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
        "extra_runs": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
