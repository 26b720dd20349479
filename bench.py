#!/usr/bin/env python3
"""Throughput of the batched neural GCDF query on one MI355X.

One step = one pass of the whole query over one batch: 128 knots x 16,384
obstacle points (2,097,152 pairs), width-512 distance network on 16-bit matrix
cores (forward: BF16 products of hi/lo split activations; reverse sweep: FP16
products; FP32 accumulation; |dd| <= 1e-3, relative J error <= 1e-2), producing the
distance d, the 9-dim configuration Jacobian J and the per-knot minimum
(dmin, argmin) in one fused launch (gcdf_query).  Inputs are resident in HBM
before the timed region.

Prints one JSON line: pairs (queries) per second, plus
  roofline     : the fused kernel's algorithmic TFLOP/s vs the dense BF16 peak
                 (launch durations from HIP events on the launch stream);
  cpu_baseline : the FP64 CPU oracle on a bounded sample of the same pairs;
  modes        : the same workload in the other precisions (context, same metric);
  serving      : p50 / p99 latency of a Poisson request trace through gcdf_submit;
  constraints  : partitions around a 128-knot trajectory, the CSR query, the
                 Jacobian pattern and the single-step projection (HBM roofline);
  training     : steps/s of the width-256 training step (batch 65,536, Adam), with
                 the FP64 oracle's gradient timed on a 1,024-sample sub-batch and
                 the step's gradient on those samples against it;
  training_table1: the same with the paper's four-term Table I loss (FP32).
The serving and training legs carry their own roofline objects (algorithmic
TFLOP/s over wall time against the BF16, resp. FP32, dense peak); the FP32
configuration (64 x 4,096, width 256) carries its own oracle timing and errors.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16x2": 2500.0, "bf16x2_f16": 2500.0, "bf16": 2500.0, "fp32": 157.3}
DESCRIBE = {
    "bf16x2": "BF16 matrix cores, hi/lo split activations, FP32 accumulate",
    "bf16x2_f16": "BF16 matrix cores with hi/lo split activations forward, FP16 matrix cores for the reverse sweep, FP32 accumulate",
}
MEETS_BAR = {"fp32": True, "bf16x2": True, "bf16x2_f16": True, "bf16": False}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_query_bf16_traffic.json")
# the query kernel's code: the tile engine, the structures and constants it uses, and
# the source file that instantiates and launches it
KERNEL_SRCS = tuple(os.path.join(ROOT, "paper_2601_18548_amd", "csrc", f)
                    for f in ("gcdf_tile.h", "gcdf_internal.h", "gcdf_fused.hip"))


def flops_per_pair(width: int) -> int:
    """Algorithmic FLOPs of one query: 12 W^2 (three W x W layers forward and
    three transposed in the reverse sweep) + 38 W (input layer forward 18 W,
    its gradient 18 W, output layer 2 W).  Hi/lo duplicate MFMA work is not
    counted."""
    return 12 * width * width + 38 * width


def kernel_source_hash(text: str | None = None) -> str:
    """Hash of the query kernel's code (the given text, else the files of
    KERNEL_SRCS in order) with comments and blank space removed, so that a
    comment edit does not orphan counters taken on unchanged code."""
    import re

    if text is None:
        parts = []
        for path in KERNEL_SRCS:
            with open(path) as f:
                parts.append(f.read())
        text = "\n".join(parts)
    code = re.sub(r"//[^\n]*", "", text)
    code = "\n".join(" ".join(line.split()) for line in code.splitlines() if line.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(launch_pairs: int, precision: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if the
    kernel code changed since the counters were taken or they cover another
    launch size or precision."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_code_sha256_16") != kernel_source_hash() or t.get("pairs_per_launch") != launch_pairs
            or t.get("precision") != precision):
        return None
    return t.get("hbm_bytes_per_launch")


def _pmc_per_dispatch(directory: str, counter: str, kernel_prefix: str):
    """Per-dispatch values of one counter (summed over its instances) from a
    rocprofv3 --output-format csv run, for dispatches of kernels whose name
    starts with kernel_prefix."""
    import csv
    import glob

    per = {}
    for f in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter and row["Kernel_Name"].startswith(kernel_prefix):
                    per[row["Dispatch_Id"]] = per.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    return [per[k] for k in sorted(per, key=int)]


def write_traffic_record(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, width=512, precision="bf16x2_f16"):
    """HBM bytes per launch of the benchmark's fused kernel: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) scaled by what they read for 5 plain copies of
    1 GiB, keyed to the kernel code they were taken on."""
    kern = "void gcdf::fused_query<%d, %d, false, 1, false, false, false>" % (width, {"bf16x2_f16": 3, "bf16x2": 2}[precision])
    fetch = _pmc_per_dispatch(fetch_dir, "FETCH_SIZE", kern)
    write = _pmc_per_dispatch(write_dir, "WRITE_SIZE", kern)
    cf = _pmc_per_dispatch(cal_fetch_dir, "FETCH_SIZE", "__amd_rocclr_copyBuffer")
    cw = _pmc_per_dispatch(cal_write_dir, "WRITE_SIZE", "__amd_rocclr_copyBuffer")
    if not (fetch and write and cf and cw):
        raise SystemExit("missing counter rows")
    nbytes = 1 << 30
    ff = nbytes / (sum(cf) / len(cf) * 1024)
    fw = nbytes / (sum(cw) / len(cw) * 1024)
    rd = sum(fetch) / len(fetch) * 1024 * ff
    wr = sum(write) / len(write) * 1024 * fw
    rec = {"kernel": "fused_query<%d, %s> (dense, d + J + per-knot min)" % (width, precision.upper()),
           "precision": precision, "kernel_code_sha256_16": kernel_source_hash(),
           "pairs_per_launch": 128 * 16384,
           "fetch_size_kib_per_dispatch": fetch, "write_size_kib_per_dispatch": write,
           "copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                "fetch_size_kib": sum(cf) / len(cf), "write_size_kib": sum(cw) / len(cw),
                                "fetch_factor": ff, "write_factor": fw},
           "hbm_read_bytes_per_launch": rd, "hbm_write_bytes_per_launch": wr, "hbm_bytes_per_launch": rd + wr,
           "algorithmic_bytes_per_launch": {"inputs": 128 * 36 + 16384 * 12,
                                            "packed_weights_once": 6 * width * width * 2 + width * 4 * 16,
                                            "outputs": 128 * 16384 * 40},
           "commands": [
               "rocprofv3 --pmc %s -d $R/gpurun_out/<dir> -o p --output-format csv -- python3 $R/bench.py "
               "--steps 3 --warmup 1 --no-cpu-baseline --no-modes --serve-requests 0 --train-steps 0 "
               "--no-constraints --no-sphere   (once with FETCH_SIZE, once with WRITE_SIZE)" % "<counter>",
               "rocprofv3 --pmc <counter> -d $R/gpurun_out/<dir> -o p --output-format csv -- python3 $R/bench.py "
               "--copy-calibration 1024   (FETCH_SIZE, then WRITE_SIZE)",
               "python3 bench.py --traffic-from <FETCH_SIZE dir> <WRITE_SIZE dir> <copy FETCH_SIZE dir> "
               "<copy WRITE_SIZE dir>"],
           "run_from": "/tmp with TMPDIR=/tmp, R = repository root; the plain copy is torch's Tensor.copy_ of "
                       "1 GiB (the HIP runtime's copy kernel)"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"hbm_read_MB": rd / 1e6, "hbm_write_MB": wr / 1e6}))


def time_mode(g, torch, wk, precision, steps, warmup, keep_outputs=False):
    """Returns (seconds per step for gcdf_query, mean fused-kernel ms from events),
    plus the last launch's d and J (device tensors) with keep_outputs."""
    ctx = g.Context(wk.weights.to_blob(), wk.width, precision)
    kt = torch.from_numpy(wk.knots).cuda()
    pt = torch.from_numpy(wk.points).cuda()
    d = torch.empty((wk.K, wk.Np), dtype=torch.float32, device="cuda")
    J = torch.empty((wk.K, wk.Np, 9), dtype=torch.float32, device="cuda")
    dmin = torch.empty(wk.K, dtype=torch.float32, device="cuda")
    am = torch.empty(wk.K, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.query(kt, pt, d, J, dmin, am, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.query(kt, pt, d, J, dmin, am, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # fused kernel alone: eval_grad is exactly one launch of it
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        ctx.eval_grad(kt, pt, d, J, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    kms = sum(a.elapsed_time(b) for a, b in evs) / steps
    ctx.close()
    return (dt, kms, d, J) if keep_outputs else (dt, kms)


def serve_bench(g, torch, rate_hz: float, n_requests: int, seed: int = 7, precision: str = "bf16x2_f16",
                budget_gib: float = 16.0, slots: int = 64, ring: int = 128):
    """Poisson stream of trajectory-optimisation requests through gcdf_submit/gcdf_poll.

    Each request: K ~ U{16..256} knots, Np ~ U{512..32768} patch points, full
    outputs (d, J, per-knot min).  Inputs come from a pool of 32 device-resident
    clouds / knot sets (sliced to the request's K and Np); outputs from a ring of
    `ring` buffer sets, each reused only after its previous request completed.
    Latency = completion seen by gcdf_poll - scheduled arrival time.
    """
    import numpy as np

    from paper_2601_18548_amd import workloads as wl

    w = wl.weights(256, seed)
    ctx = g.Context(w.to_blob(), 256, precision, serve_mem_budget=int(budget_gib * (1 << 30)), serve_slots=slots)
    trace = wl.serving_trace(n_requests, rate_hz, seed)
    P = 32
    pool_p = [torch.from_numpy(wl.points_patches(32768, seed + 10 + i)).cuda() for i in range(P)]
    pool_k = [torch.from_numpy(wl.knots(256, seed + 100 + i)).cuda() for i in range(P)]
    kmax, npmax = 256, 32768
    outs = [(torch.empty(kmax * npmax, device="cuda"), torch.empty(kmax * npmax * 9, device="cuda"),
             torch.empty(kmax, device="cuda"), torch.empty(kmax, dtype=torch.int32, device="cuda"))
            for _ in range(min(ring, n_requests))]
    torch.cuda.synchronize()
    # warm the serving kernel once
    t = ctx.submit(pool_k[0][:16], pool_p[0][:512], outs[0][0][:16 * 512].view(16, 512),
                   outs[0][1][:16 * 512 * 9].view(16, 512, 9), outs[0][2][:16], outs[0][3][:16])
    while not ctx.poll(t):
        time.sleep(1e-4)
    tickets, owner = {}, [None] * len(outs)
    done_at = [None] * n_requests
    t0 = time.perf_counter()
    nxt = 0
    pairs = 0
    while nxt < n_requests or tickets:
        now = time.perf_counter() - t0
        if nxt < n_requests and now >= trace[nxt].arrival_s:
            r = trace[nxt]
            slot = nxt % len(outs)
            if owner[slot] is not None and done_at[owner[slot]] is None:
                pass  # buffer still in use: poll below, submit later (latency keeps counting)
            else:
                d, J, dm, am = outs[slot]
                pi = nxt % P
                tk = ctx.submit(pool_k[pi][:r.K], pool_p[pi][:r.Np], d[:r.K * r.Np].view(r.K, r.Np),
                                J[:r.K * r.Np * 9].view(r.K, r.Np, 9), dm[:r.K], am[:r.K])
                tickets[tk] = nxt
                owner[slot] = nxt
                pairs += r.K * r.Np
                nxt += 1
                continue
        for tk in list(tickets):
            if ctx.poll(tk):
                done_at[tickets.pop(tk)] = time.perf_counter() - t0
    elapsed = time.perf_counter() - t0
    lat = np.array([done_at[i] - trace[i].arrival_s for i in range(n_requests)]) * 1e3
    ctx.close()
    mean_pairs = float(np.mean([r.K * r.Np for r in trace]))
    # algorithmic work of the completed queries over the whole trace (wall clock,
    # arrival gaps and host admission included) against the dense BF16 peak
    tf = pairs * flops_per_pair(256) / elapsed / 1e12
    return {"offered_req_per_s": rate_hz, "requests": n_requests, "precision": precision, "width": 256,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "completed_req_per_s": n_requests / elapsed,
            "queries_per_s": pairs / elapsed, "offered_queries_per_s": rate_hz * mean_pairs,
            "overloaded": bool(n_requests / elapsed < 0.95 * rate_hz),
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                         "frac": tf / PEAK_TFLOPS[precision],
                         "work": "completed pairs x %d FLOP / trace wall time" % flops_per_pair(256)}}


def _event_ms(torch, stream, fn, reps: int) -> float:
    """Mean milliseconds of fn() on `stream`, from HIP events around each call."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / reps


def constraints_bench(g, torch, wk, reps: int = 5, n_knots: int = 128, radius: float = 1.5):
    """The solver-side calls on the benchmark cloud: partitions of the points around
    a 128-knot trajectory, the CSR query over them (same network and precision as
    the main workload), the Jacobian pattern, and the single-step projection over
    the dense outputs of the main workload (an HBM-bound epilogue: 80 B per row)."""
    from paper_2601_18548_amd import workloads as wl

    ctx = g.Context(wk.weights.to_blob(), wk.width, wk.precision)
    stream = torch.cuda.current_stream()
    tr = torch.from_numpy(wl.trajectory(n_knots, 901)).cuda()
    pt = torch.from_numpy(wk.points).cuda()
    kt = torch.from_numpy(wk.knots).cuda()
    out = {}
    ctx.partition(tr, pt, radius, ref_stride=9)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        off, idx = ctx.partition(tr, pt, radius, ref_stride=9)
    torch.cuda.synchronize()
    total = int(idx.shape[0])
    out["partition"] = {"knots": n_knots, "points": wk.Np, "radius_m": radius, "rows": total,
                        "ms_per_build_incl_size_sync": (time.perf_counter() - t0) / reps * 1e3}
    c = torch.empty(total, device="cuda")
    J = torch.empty((total, 9), device="cuda")
    ctx.eval_grad_csr(tr, pt, off, idx, c=c, J=J)
    kms = _event_ms(torch, stream, lambda: ctx.eval_grad_csr(tr, pt, off, idx, c=c, J=J, stream=stream), reps)
    fl = flops_per_pair(wk.width) * total
    out["csr_query"] = {"rows": total, "kernel_ms": kms, "rows_per_s": total / (kms * 1e-3),
                        "tflops": fl / (kms * 1e-3) / 1e12, "frac_of_peak": fl / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[wk.precision]}
    pms = _event_ms(torch, stream, lambda: ctx.jacobian_pattern(off, total, stream=stream), reps)
    out["jacobian_pattern"] = {"rows": total, "ms": pms, "bytes": 44 * total, "gbps": 44 * total / (pms * 1e-3) / 1e9}
    d = torch.empty((wk.K, wk.Np), device="cuda")
    Jd = torch.empty((wk.K, wk.Np, 9), device="cuda")
    ctx.eval_grad(kt, pt, d, Jd)
    m = [2.0, 2.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]
    ctx.project(kt, d, Jd, m)
    jms = _event_ms(torch, stream, lambda: ctx.project(kt, d, Jd, m, stream=stream), reps * 4)
    rows = wk.K * wk.Np
    gbps = 80.0 * rows / (jms * 1e-3) / 1e9
    out["projection"] = {"rows": rows, "kernel_ms": jms, "algorithmic_bytes_per_row": 80, "gbps": gbps,
                         "roofline": {"bound": "hbm", "achieved": gbps, "peak": 8000.0, "unit": "GB/s",
                                      "frac": gbps / 8000.0}}
    ctx.close()
    return out


def sphere_bench(g, torch, point_kernel_ms: float, reps: int = 10):
    """Sphere obstacles (x, y, z, r) with the 10-input network [p', r, a]: the
    benchmark shape (128 knots x 16,384 spheres, width 512, its precision), one fused
    eval_grad launch per rep, timed with HIP events on its stream."""
    from paper_2601_18548_amd import workloads as wl

    wk = wl.workload("sphere")
    ctx = g.Context(wk.weights.to_blob(), wk.width, wk.precision)
    stream = torch.cuda.current_stream()
    kt = torch.from_numpy(wk.knots).cuda()
    st = torch.from_numpy(wk.points).cuda()
    d = torch.empty((wk.K, wk.Np), device="cuda")
    J = torch.empty((wk.K, wk.Np, 9), device="cuda")
    ctx.eval_grad(kt, st, d, J)
    ms = _event_ms(torch, stream, lambda: ctx.eval_grad(kt, st, d, J, stream=stream), reps)
    pairs = wk.K * wk.Np
    # input layer 20 W (one more input than points), its gradient 18 W (the nine
    # configuration-facing inputs), output 2 W
    fl = (12 * wk.width * wk.width + 40 * wk.width) * pairs
    tf = fl / (ms * 1e-3) / 1e12
    ctx.close()
    return {"workload": "128 knots x 16384 spheres (x, y, z, r), width 512, %s, input [p', r, a]" % wk.precision,
            "kernel_ms": ms, "pairs_per_s": pairs / (ms * 1e-3), "tflops": tf, "frac_of_peak": tf / PEAK_TFLOPS[wk.precision],
            "vs_point_kernel": point_kernel_ms / ms}


def train_bench(torch, steps: int, warmup: int, batch: int = 65536, width: int = 256, cpu: bool = True):
    """Training step of the width-256 network: MSE against a seeded teacher's
    distances plus N(0, 1e-3) noise, hand-written forward/backward behind
    torch.autograd, Adam (lr 0.005) on FP32 master weights, BF16 matrix cores."""
    from paper_2601_18548_amd import train
    from paper_2601_18548_amd import workloads as wl

    teacher = wl.weights(width, seed=501, bf16_hidden=False)
    student = wl.weights(width, seed=502, bf16_hidden=False)
    k, p, noise = wl.training_batch(batch, 503)
    tr = train.Trainer(width, "bf16", max_batch=batch)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    with torch.no_grad():
        y = tr.forward(train.flat_params(teacher), kt, pt) + torch.from_numpy(noise).cuda()
    params = train.flat_params(student).requires_grad_(True)
    opt = train.adam(params, lr=5e-3, betas=(0.9, 0.999), trainer=tr)  # Adam packs the next step's weights
    loss0 = None
    for _ in range(warmup):
        loss0 = train.mse_step(params, opt, tr, kt, pt, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = train.mse_step(params, opt, tr, kt, pt, y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # algorithmic work per sample: forward 6 W^2, reverse 6 W^2, weight gradients 6 W^2
    fl = 18 * width * width * batch
    tf = fl * steps / el / 1e12
    out = {"steps_per_s": steps / el, "ms_per_step": el / steps * 1e3, "samples_per_s": batch * steps / el,
           "batch": batch, "width": width, "precision": "bf16 (FP32 master weights, FP32 accumulate)",
           "tflops_algorithmic": tf,
           "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                        "frac": tf / PEAK_TFLOPS["bf16"], "work": "18 W^2 FLOP per sample, whole step"},
           "loss_first": float(loss0.item()) if loss0 is not None else None, "loss_last": float(loss.item())}
    if cpu:
        # the FP64 oracle's loss gradient on a 1,024-sample sub-batch at the trained
        # parameters, timed, and the library's gradient on the same samples against it
        import numpy as np

        import oracle

        n = 1024
        blob = student.to_blob()[:wl.BLOB_HEADER_BYTES] + params.detach().cpu().numpy().astype("<f4").tobytes()
        ys = y[:n].contiguous()
        _, g_gpu = tr.mse(params.detach(), kt[:n].contiguous(), pt[:n].contiguous(), ys)
        g_gpu = g_gpu.cpu().numpy().astype(np.float64)
        t1 = time.perf_counter()
        _, gref = oracle.mse_grad(blob, k[:n], p[:n], ys.cpu().numpy())
        cpu_s = time.perf_counter() - t1
        errs, off = [], 0
        for a in gref:
            seg = g_gpu[off:off + a.size]
            off += a.size
            errs.append(float(np.linalg.norm(seg - a.ravel()) / max(np.linalg.norm(a), 1e-30)))
        out["cpu_baseline"] = {"value": n / cpu_s, "unit": "samples/s (loss + weight gradient)", "cores": 1,
                               "kind": "oracle", "sample": "the first %d samples of the batch, FP64, %.2f s" % (n, cpu_s)}
        out["gradient_vs_oracle"] = {"samples": n, "max_rel_err_per_array": max(errs),
                                     "arrays": "W1 b1 W2 b2 W3 b3 W4 b4 w_out b_out, norm-wise"}
    tr.close()
    return out


def table1_bench(g, torch, steps: int, warmup: int, batch: int = 65536, width: int = 256):
    """Training step on the paper's Table I loss (value, direction, weighted eikonal,
    tension; weights of Sec. V-A), FP32, targets = a seeded teacher's distances and
    configuration gradients, Adam: gcdf_train_table1 + gcdf_adam_step."""
    from paper_2601_18548_amd import train
    from paper_2601_18548_amd import workloads as wl

    teacher = wl.weights(width, seed=601, bf16_hidden=False)
    student = wl.weights(width, seed=602, bf16_hidden=False)
    k, p, noise = wl.training_batch(batch, 603)
    kt, pt = torch.from_numpy(k).cuda(), torch.from_numpy(p).cuda()
    tr = train.Trainer(width, "fp32", max_batch=batch)
    # targets: the teacher's distance and configuration gradient per sample, from a CSR
    # query with one row per knot (knot i, point i) (+ N(0, 1e-3) noise on the value)
    ctx = g.Context(teacher.to_blob(), width, "fp32")
    d = torch.empty(batch, device="cuda")
    J = torch.empty((batch, 9), device="cuda")
    idx = torch.arange(batch, dtype=torch.int64, device="cuda")
    off = torch.arange(batch + 1, dtype=torch.int64, device="cuda")
    ctx.eval_grad_csr(kt, pt, off, idx.to(torch.int32), c=d, J=J)
    ctx.close()
    fstar = (d + torch.from_numpy(noise).cuda()).contiguous()
    m_diag = [4.0, 4.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]
    params = train.flat_params(student).requires_grad_(True)
    opt = train.Adam(params, lr=1e-3)
    first = None
    for _ in range(warmup):
        losses, gr = tr.table1(params.detach(), kt, pt, fstar, J, m_diag)
        params.grad = gr
        opt.step()
        first = float(losses[4]) if first is None else first
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        losses, gr = tr.table1(params.detach(), kt, pt, fstar, J, m_diag)
        params.grad = gr
        opt.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tr.close()
    # algorithmic work per sample: 12 W x W products in the loss pass (forward, reverse,
    # tangent, adjoint) + 6 in the weight gradients + the query for J (6)
    fl = 24 * width * width * batch
    tf = fl * steps / el / 1e12
    return {"steps_per_s": steps / el, "ms_per_step": el / steps * 1e3, "batch": batch, "width": width,
            "precision": "fp32", "loss": "Table I, lambda = (5, 0.1, 0.01, 0.01), M = diag(4, 4, 1, ..., 1)",
            "tflops_algorithmic": tf,
            "roofline": {"bound": "mfma", "achieved": tf, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                         "frac": tf / PEAK_TFLOPS["fp32"], "work": "24 W^2 FLOP per sample, whole step"},
            "loss_first": first, "loss_last": float(losses[4])}


def cpu_baseline(wk, seconds: float, torch=None, d_gpu=None, J_gpu=None):
    """The FP64 oracle timed on a bounded random sample of the workload's pairs.
    With the timed launch's outputs (d_gpu, J_gpu), also their errors against the
    oracle on that sample: returns (baseline, accuracy or None)."""
    import numpy as np

    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    blob = wk.weights.to_blob()
    r = np.random.default_rng(123)
    n = 64
    while True:
        ki = r.integers(0, wk.K, n)
        pi = r.integers(0, wk.Np, n)
        t0 = time.perf_counter()
        dr, Jr = oracle.eval_pairs(blob, wk.knots, wk.points, ki, pi, nthreads=threads)
        el = time.perf_counter() - t0
        if el >= seconds * 0.5 or n >= 1 << 22:
            break
        n = int(n * min(16.0, max(2.0, seconds / max(el, 1e-3))))
    rate = n / el
    # the same oracle on one core, on the first pairs of the sample (~1/8 of the time)
    n1 = max(64, min(n, int(rate * seconds / 8 / max(1, oracle.threads(threads)))))
    t0 = time.perf_counter()
    oracle.eval_pairs(blob, wk.knots, wk.points, ki[:n1], pi[:n1], nthreads=1)
    rate1 = n1 / (time.perf_counter() - t0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    base = {"value": rate, "unit": "queries/s", "cores": oracle.threads(threads), "kind": "oracle",
            "sample": "%d random (knot, point) pairs of the same workload, value + Jacobian in FP64, %.1f s" % (n, el),
            "value_1_core": rate1, "sample_1_core": "the first %d pairs of that sample" % n1, "cpu_model": model}
    if d_gpu is None:
        return base, None
    kd, pd = torch.from_numpy(ki).to(d_gpu.device), torch.from_numpy(pi).to(d_gpu.device)
    d = d_gpu[kd, pd].cpu().numpy().astype(np.float64)
    J = J_gpu[kd, pd].cpu().numpy().astype(np.float64).reshape(-1, 9)
    Jr = np.asarray(Jr).reshape(-1, 9)
    dd = np.abs(d - np.asarray(dr))
    nr = np.linalg.norm(Jr, axis=1)
    rel = np.linalg.norm(J - Jr, axis=1) / np.maximum(nr, 1e-3 * np.median(nr))
    acc = {"vs": "FP64 oracle", "pairs": int(n), "max_abs_dd": float(dd.max()), "mean_abs_dd": float(dd.mean()),
           "max_rel_J": float(rel.max()), "p99_rel_J": float(np.percentile(rel, 99)), "mean_rel_J": float(rel.mean()),
           "rel_J": "|J - J_ref| / max(|J_ref|, 1e-3 median |J_ref|) per pair"}
    return base, acc


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bf16", choices=["bf16", "fp32", "small"])
    ap.add_argument("--precision", default=None, choices=sorted(PEAK_TFLOPS),
                    help="precision of the timed query and the serving trace (default: the workload's)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true", help="skip the runs of the workload in the other precisions")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests in the serving trace (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--no-constraints", action="store_true", help="skip the partition / CSR / projection leg")
    ap.add_argument("--no-sphere", action="store_true", help="skip the sphere-obstacle leg")
    ap.add_argument("--train-steps", type=int, default=100, help="timed training steps (0: skip)")
    ap.add_argument("--serve-sweep", default="", help="comma-separated arrival rates: print one serving line each")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="write the HBM traffic record from the CSV output of four rocprofv3 --pmc runs "
                         "(FETCH_SIZE and WRITE_SIZE of this benchmark's short run, then of "
                         "--copy-calibration 1024) and exit; needs no GPU")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic_record(*args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the query shards by knots or points "
              "with no exchange but a K-value min all-reduce); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4, "copies": 5}), flush=True)
        return

    import paper_2601_18548_amd as g
    from paper_2601_18548_amd import workloads as wl

    g.library()  # fails loudly if the HIP library is missing
    if args.serve_sweep:
        for rate in [float(x) for x in args.serve_sweep.split(",")]:
            print(json.dumps({"serving": serve_bench(g, torch, rate, args.serve_requests,
                                                     precision=args.precision or "bf16x2_f16")}), flush=True)
        return
    wk = wl.workload(args.workload)
    if args.precision:
        wk.precision = args.precision
    pairs = wk.K * wk.Np
    print("bench: workload %s (%d knots x %d points, width %d, %s), %d steps after %d warmup" %
          (args.workload, wk.K, wk.Np, wk.width, wk.precision, args.steps, args.warmup), file=sys.stderr, flush=True)
    step_s, kernel_ms, d_out, J_out = time_mode(g, torch, wk, wk.precision, args.steps, args.warmup, keep_outputs=True)
    value = pairs / step_s
    fl = flops_per_pair(wk.width) * pairs
    achieved = fl / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[wk.precision]
    print("bench: %.3f ms/step, fused kernel %.3f ms, %.1f TFLOP/s" % (step_s * 1e3, kernel_ms, achieved),
          file=sys.stderr, flush=True)
    out = {
        "metric": "GCDF value+Jacobian queries/s (BF16 vs FP32 at <=1e-3 err); p50/p99 latency",
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # forward products BF16 (hi/lo split), reverse-sweep products FP16, FP32 accumulation
        "dtype": {"bf16x2_f16": "bf16x2/f16"}.get(wk.precision, wk.precision),
        "data": "synthetic (seeded knots, patch point clouds, He-normal random weights)",
        "config": {
            "workload": "%d knots x %d points, distance MLP 9->%dx4->1 SiLU, %s" %
                        (wk.K, wk.Np, wk.width, DESCRIBE.get(wk.precision, wk.precision)),
            "knots": wk.K, "points": wk.Np, "width": wk.width, "precision": wk.precision,
            "pairs_per_step": pairs, "outputs": "d, J (9 per pair), per-knot min + argmin",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(pairs, wk.precision),
            "kernel": "fused_query (one launch = %d pairs x %d FLOP)" % (pairs, flops_per_pair(wk.width)),
            "kernel_ms": kernel_ms,
        },
    }
    if not args.no_modes and args.workload == "bf16":
        modes = {}
        others = [p for p in ("bf16x2", "bf16x2_f16") if p != wk.precision]
        for prec, st in [("fp32", 3), ("bf16", args.steps)] + [(p, args.steps) for p in others]:
            s, kms = time_mode(g, torch, wk, prec, st, 1)
            a = flops_per_pair(wk.width) * pairs / (kms * 1e-3) / 1e12
            modes[prec] = {"queries_per_s": pairs / s, "kernel_ms": kms, "tflops": a,
                           "frac_of_peak": a / PEAK_TFLOPS[prec], "peak": PEAK_TFLOPS[prec],
                           "meets_1e-3": MEETS_BAR[prec]}
            print("bench: mode %s %.3f ms/step" % (prec, s * 1e3), file=sys.stderr, flush=True)
        # the FP32 configuration at its own shape: 64 knots x 4,096 points, width 256
        wk2 = wl.workload("fp32")
        s2, kms2, d2, J2 = time_mode(g, torch, wk2, "fp32", 10, 2, keep_outputs=True)
        a2 = flops_per_pair(wk2.width) * wk2.K * wk2.Np / (kms2 * 1e-3) / 1e12
        modes["fp32_64x4096_w256"] = {"queries_per_s": wk2.K * wk2.Np / s2, "kernel_ms": kms2, "tflops": a2,
                                      "frac_of_peak": a2 / PEAK_TFLOPS["fp32"], "peak": PEAK_TFLOPS["fp32"],
                                      "meets_1e-3": True}
        if not args.no_cpu_baseline:
            # the oracle on this configuration's own pairs, and the launch's errors on them
            b2, acc2 = cpu_baseline(wk2, args.cpu_seconds / 2, torch, d2, J2)
            modes["fp32_64x4096_w256"]["cpu_baseline"] = b2
            modes["fp32_64x4096_w256"]["accuracy"] = acc2
            print("bench: fp32 64x4096 oracle %.0f queries/s (%d cores), accuracy %s" %
                  (b2["value"], b2["cores"], json.dumps(acc2)), file=sys.stderr, flush=True)
        del d2, J2
        out["modes"] = modes
    if args.serve_requests > 0:
        out["serving"] = serve_bench(g, torch, args.serve_rate, args.serve_requests, precision=wk.precision)
        print("bench: serving p50 %.1f ms p99 %.1f ms" % (out["serving"]["p50_ms"], out["serving"]["p99_ms"]),
              file=sys.stderr, flush=True)
    if not args.no_constraints and args.workload == "bf16":
        out["constraints"] = constraints_bench(g, torch, wk)
        print("bench: constraints %s" % json.dumps(out["constraints"]), file=sys.stderr, flush=True)
    if not args.no_sphere and args.workload == "bf16":
        out["sphere"] = sphere_bench(g, torch, kernel_ms)
        print("bench: sphere %s" % json.dumps(out["sphere"]), file=sys.stderr, flush=True)
    if args.train_steps > 0:
        # 100 untimed steps first: the step time settles only after ~20 ms of them
        out["training"] = train_bench(torch, args.train_steps, 100, cpu=not args.no_cpu_baseline)
        print("bench: training %.3f ms/step" % out["training"]["ms_per_step"], file=sys.stderr, flush=True)
    if args.train_steps > 0:
        out["training_table1"] = table1_bench(g, torch, max(5, args.train_steps // 20), 2)
        print("bench: Table I training %.3f ms/step" % out["training_table1"]["ms_per_step"], file=sys.stderr,
              flush=True)
    if not args.no_cpu_baseline:
        # the oracle's sample doubles as an accuracy check of the timed launch's outputs
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(wk, args.cpu_seconds, torch, d_out, J_out)
        print("bench: accuracy %s" % json.dumps(out["accuracy"]), file=sys.stderr, flush=True)
    del d_out, J_out
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
