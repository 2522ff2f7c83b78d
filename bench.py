"""Benchmark of the node-aware SpMV hot path on one MI355X.

One step = one apply of the plan: the exchange that fills every process's
ghost buffer from v (section 2.1 / section 4 messages as device gathers) and
the split product w = A_on v + A_off ghost, over the largest paper-shaped
workload (KKT-like random matrix, N = 2^22, n_p = 2048, ppn = 16, float64),
inputs resident in HBM.  Prints ONE JSON line on stdout; progress goes to
stderr.

Timing protocol: HIP events around every apply on the stream it runs on,
after the warm-up applies; the median, 10th and 90th percentile over the
timed applies.  Per-launch times come from a second pass of as many
applies with an event between the two launches as well.  "Cold" applies
follow a 1 GiB scratch write that evicts the L2 caches and the 256 MB
Infinity Cache, then a 1 GiB read of a second buffer, so that the caches
hold neither data of the apply nor dirty lines of the flush (whose
write-back would otherwise land inside the timed apply; that variant is
reported too, as cold_write_only); "warm" applies run back to back.
value = algorithmic bytes of one apply / the cold median.

Algorithmic bytes count every array element the method must touch once:
  product:  nnz*(s_a + 4) + 2*(N+1)*4 (two row pointers) + N*s_v (v)
            + G*s_v (ghosts) + N*s_v (w)
  gather:   G*(4 + 2*s_v)                                  (standard mode)
  NAP:      E*(4 + 2*s_v) + H*(8 + 2*s_v) + G_on*(8 + 2*s_v)  (+2*E*s_v if copied)
An apply is two launches (LOCAL: exchange gather with the on-process product;
REMOTE: [NAP scatter and] the off-process product); each launch's bytes for
the roofline count what that launch must touch, the REMOTE launch reading and
rewriting the partial w of the rows that have off-process entries.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
FLUSH_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(st, s_a, s_v):
    n, nnz, g = st["n"], st["nnz"], st["ghosts"]
    return nnz * (s_a + 4) + 2 * (n + 1) * 4 + n * s_v + g * s_v + n * s_v


def exchange_bytes(st, s_v, exchange_copy=False, direct=False):
    ph = st["phases"]
    if st["mode"] == "standard":
        return st["ghosts"] * (4 + 2 * s_v)
    e = ph["INTER"]["elems"]
    if direct:      # the pack only: the product reads ghosts where they lie
        return e * (4 + 2 * s_v) + (2 * e * s_v if exchange_copy else 0)
    g_on = ph["L2"]["elems"]
    h = st["ghosts"] - g_on
    b = e * (4 + 2 * s_v) + h * (8 + 2 * s_v) + g_on * (8 + 2 * s_v)
    return b + (2 * e * s_v if exchange_copy else 0)


def apply_bytes(st, s_a, s_v):
    return spmv_bytes(st, s_a, s_v) + exchange_bytes(st, s_v)


def launch_bytes(st, s_a, s_v, rows_off):
    """Algorithmic bytes of the LOCAL and REMOTE launches of a standard apply."""
    n, g = st["n"], st["ghosts"]
    local = (st["ghosts"] * (4 + 2 * s_v) + st["nnz_on"] * (s_a + 4) + (n + 1) * 4
             + n * s_v + n * s_v)
    remote = st["nnz_off"] * (s_a + 4) + (n + 1) * 4 + g * s_v + 2 * rows_off * s_v
    return local, remote


def rows_with_off_entries(a, n_p, row_starts):
    import numpy as np
    if row_starts is None:
        b = a.n // n_p
        starts = np.arange(n_p + 1, dtype=np.int64) * b
        starts[-1] = a.n
    else:
        starts = np.asarray(row_starts, np.int64)
    rows = np.repeat(np.arange(a.n), np.diff(a.rowptr))
    own_r = np.searchsorted(starts, rows, side="right")
    own_c = np.searchsorted(starts, a.col, side="right")
    return int(np.unique(rows[own_r != own_c]).size)


def source_hash() -> str:
    """Hash of the kernel and launch-schedule sources with comments and blank
    lines removed, so a recorded counter summary stays valid across
    comment-only edits."""
    import re
    h = hashlib.sha256()
    for f in ("kernels.hpp", "napspmv.hip", "schedule.hpp", "schedule.cpp"):
        with open(os.path.join(ROOT, "paper_1612_08060_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM traffic per launch of a kernel from the committed counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_hash():
        return None
    return t.get("bytes_per_launch")


def pct(xs, scale=1.0, nd=5):
    import numpy as np
    a = np.asarray(xs, dtype=np.float64) * scale
    return {"median": round(float(np.median(a)), nd), "p10": round(float(np.percentile(a, 10)), nd),
            "p90": round(float(np.percentile(a, 90)), nd), "mean": round(float(a.mean()), nd),
            "n": int(a.size)}


class Flush:
    """Cache eviction before a cold apply: a 1 GiB scratch write, then (unless
    write_only) a 1 GiB read of a second buffer that leaves only clean lines
    in the caches."""

    def __init__(self, torch, dev, write_only=False):
        self.torch = torch
        self.buf = torch.empty(FLUSH_BYTES, dtype=torch.uint8, device=dev)
        self.rd = None if write_only else torch.ones(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        self.k = 0

    def __call__(self):
        self.k = (self.k + 1) & 0x7f
        self.buf.fill_(self.k)
        if self.rd is not None:
            self.torch.sum(self.rd)


def time_applies(torch, plan, v, w, nap, steps, warmup, flush=None):
    """HIP event times (ms) on the apply's stream.  After `warmup` untimed
    applies: `steps` applies, each bracketed by two events (with `flush`,
    each after a cache flush outside its events), then `steps` more with a
    third event between the two launches, for the per-launch times (an
    event between the launches adds a small gap of its own, so the apply
    times come from the first pass).  Returns (apply, local, remote, wall ms
    per apply of the first pass)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.apply(v, w, stream=stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        if flush is not None:
            flush()
        ev[k][0].record(stream)
        plan.apply(v, w, stream=stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    apply_ = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        if flush is not None:
            flush()
        ev[k][0].record(stream)
        plan.apply_stage(nap.STAGE_LOCAL, v, w, stream=stream)
        ev[k][1].record(stream)
        plan.apply_stage(nap.STAGE_REMOTE, v, w, stream=stream)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    local = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    remote = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    return apply_, local, remote, wall


def time_calls(torch, fn, steps, warmup, flush=None):
    """HIP event times (ms) of `steps` calls of fn() on the current stream."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for k in range(steps):
        if flush is not None:
            flush()
        ev[k][0].record(stream)
        fn()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def _time_ms(torch, fn, reps):
    """Average ms of fn() over reps back-to-back calls (HIP events)."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_denominator(torch, dev):
    """Median time of a plain 1 GiB device-to-device copy (torch's copy
    kernel); bandwidth counts its read and its write."""
    x = torch.ones(FLUSH_BYTES // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    ms = time_calls(torch, lambda: y.copy_(x), 10, 3)
    import numpy as np
    med = float(np.median(ms))
    return {"kernel": "torch copy_ of 1 GiB float64", "median_ms": round(med, 4),
            "gbs": round(2 * FLUSH_BYTES / (med * 1e-3) / 1e9, 1)}


def config_row(torch, nap, plan, v, w, nbytes, steps, warmup, flush, nnz=None, graph=False,
               unit="ms"):
    """Cold and warm apply percentiles of one plan, GB/s at the medians and,
    optionally, per-apply time of a replayed HIP graph."""
    scale = 1000.0 if unit == "us" else 1.0
    cold, _, _, _ = time_applies(torch, plan, v, w, nap, steps, warmup, flush)
    warm, loc, rem, wall = time_applies(torch, plan, v, w, nap, steps, warmup)
    row = {f"cold_{unit}": pct(cold, scale), f"warm_{unit}": pct(warm, scale),
           "warm_local_ms": pct(loc)["median"], "warm_remote_ms": pct(rem)["median"],
           "bytes_per_apply": nbytes}
    import numpy as np
    cm, wm = float(np.median(cold)), float(np.median(warm))
    row["gbs_cold"] = round(nbytes / (cm * 1e-3) / 1e9, 1)
    row["gbs_warm"] = round(nbytes / (wm * 1e-3) / 1e9, 1)
    row["frac_of_hbm_peak_cold"] = round(row["gbs_cold"] / PEAK_HBM_GBS, 4)
    if nnz is not None:
        row["gflops_cold"] = round(2 * nnz / (cm * 1e-3) / 1e9, 1)
    if graph:
        # 50 back-to-back applies captured in one HIP graph: per-apply device
        # time without the host's launch overhead
        cg = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        with torch.cuda.stream(cs):
            plan.apply(v, w, stream=cs)
            cs.synchronize()
            with torch.cuda.graph(cg, stream=cs):
                for _ in range(50):
                    plan.apply(v, w, stream=cs)
        torch.cuda.synchronize()
        row[f"graph_{unit}_per_apply"] = round(_time_ms(torch, cg.replay, 5) / 50 * scale, 4)
        del cg
    return row


def bench_batched(torch, nap, dev, reps=20):
    """256 uneven row blocks of a 27-point stencil, float32 values: the whole
    product as one graph-captured launch pair (autotuned), against one launch
    pair per block (eager, and captured in one graph)."""
    import numpy as np
    from workloads import config, to_f32
    wl = config(4)
    a = wl.csr
    p = nap.Plan(a.rowptr, a.col, to_f32(a.val), a.n, wl.n_p, wl.ppn, mode="standard",
                 dtype="f32", row_starts=wl.row_starts)
    v = torch.from_numpy(to_f32(wl.v)).to(dev)
    w = torch.empty_like(v)
    default_graph = p.graph(v, w)
    default_ms = _time_ms(torch, default_graph.launch, reps)
    default_graph.close()
    tune_ms = p.autotune(v, w, reps=3)
    tuning = {k: p.get_param(k) for k in ("block_nnz", "window", "gather_item", "remote_nnz")}
    g = p.graph(v, w)
    batched_ms = _time_ms(torch, g.launch, reps)
    torch.cuda.synchronize()
    w_batched = w.clone()
    p.prepare_partitions()
    w2 = torch.empty_like(v)

    def parts():
        for t in range(wl.n_p):
            p.apply_partition(t, v, w2)
    parts_eager_ms = _time_ms(torch, parts, max(3, reps // 4))
    cg = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        parts()
        cs.synchronize()
        with torch.cuda.graph(cg, stream=cs):
            parts()
    torch.cuda.synchronize()
    parts_graph_ms = _time_ms(torch, cg.replay, reps)
    same = bool(torch.equal(w_batched, w2))
    st = p.stats
    nbytes = apply_bytes(st, 4, 4)
    g.close()
    p.close()
    sizes = np.diff(wl.row_starts)
    return {"workload": wl.name, "n": a.n, "nnz": a.nnz, "blocks": wl.n_p,
            "block_rows_min_median_max": [int(sizes.min()), int(np.median(sizes)), int(sizes.max())],
            "dtype": "f32", "bytes_per_apply": nbytes,
            "graph_default_tuning_ms": round(default_ms, 5),
            "graph_autotuned_ms": round(batched_ms, 5),
            "graph_autotuned_gbs": round(nbytes / (batched_ms * 1e-3) / 1e9, 1),
            "autotuned": tuning, "autotune_best_eager_ms": round(tune_ms, 5),
            "per_block_launches_eager_ms": round(parts_eager_ms, 4),
            "per_block_launches_graph_ms": round(parts_graph_ms, 4),
            "speedup_vs_per_block_eager": round(parts_eager_ms / batched_ms, 2),
            "speedup_vs_per_block_graph": round(parts_graph_ms / batched_ms, 2),
            "per_block_equals_batched_bitwise": same}


def _serving_plans(nap, torch, dev, mix, dtypes):
    """One plan per matrix of the mix with the given value type per matrix;
    returns (plans, device vectors, algorithmic bytes per apply)."""
    from workloads import bf16_bits, to_f32
    vals = {"f64": lambda x: x, "f32": to_f32, "bf16": bf16_bits}
    plans, vecs, nbytes = [], [], []
    for wl, dt in zip(mix, dtypes):
        a = wl.csr
        plans.append(nap.Plan(a.rowptr, a.col, vals[dt](a.val), a.n, wl.n_p, wl.ppn,
                              mode="standard", dtype=dt))
        vecs.append(torch.from_numpy(wl.v if dt == "f64" else to_f32(wl.v)).to(dev))
        sa = {"f64": 8, "f32": 4, "bf16": 2}[dt]
        nbytes.append(apply_bytes(plans[-1].stats, sa, 8 if dt == "f64" else 4))
    return plans, vecs, nbytes


def bench_multi_batch(torch, nap, dev, mix):
    """napspmv_batch_apply over separate plans (different matrices) in one
    launch sequence, against the same products applied one after another."""
    import numpy as np
    from workloads import to_f32
    pick = [k for k, wl in enumerate(mix) if wl.dtypes[0] == "f32"][:16]
    sub = [mix[k] for k in pick]
    plans, vecs, nbytes = _serving_plans(nap, torch, dev, sub, ["f32"] * len(sub))
    outs = [torch.empty_like(x) for x in vecs]
    b = nap.Batch(len(plans))
    batch_ms = _time_ms(torch, lambda: b.apply(plans, vecs, outs), 20)
    torch.cuda.synchronize()
    got = [o.clone() for o in outs]
    seq_ms = _time_ms(torch, lambda: [p.apply(x, o) for p, x, o in zip(plans, vecs, outs)], 20)
    torch.cuda.synchronize()
    same = all(bool(torch.equal(x, y)) for x, y in zip(got, outs))
    total = float(sum(nbytes))
    b.close()
    for p in plans:
        p.close()
    return {"products": len(plans), "dtype": "f32",
            "rows": [int(w.csr.n) for w in sub], "bytes": int(total),
            "batch_apply_ms": round(batch_ms, 4), "batch_gbs": round(total / (batch_ms * 1e-3) / 1e9, 1),
            "one_by_one_ms": round(seq_ms, 4), "one_by_one_gbs": round(total / (seq_ms * 1e-3) / 1e9, 1),
            "speedup": round(seq_ms / batch_ms, 2), "batched_equals_one_by_one_bitwise": same}


def bench_serving(torch, nap, dev, n_req=3000, warm=300, rhos=(0.5, 0.8, 0.95, 2.0)):
    """Poisson-arrival requests on 64 resident matrices of mixed size.

    The baseline is every request served alone, in arrival order, on the
    plain float64 path (a 1-slot server without batching); its capacity is
    its own sustained closed-loop throughput (every request queued at once),
    and arrival rates are rho times that capacity.  Served: 4 slots, batches
    up to 16, 16 GiB workspace budget, on the same float64 plans (equal
    accuracy) and on the mix's own value types (float64/float32/bfloat16 in
    turn).  Workspaces are reserved before any timed replay, so no replay
    allocates.  A sample of served results is checked against the oracle."""
    import numpy as np
    from oracle import spmv as oracle_spmv
    from workloads import poisson_arrivals, serving_mix
    mix = serving_mix()
    f64_plans, f64_vecs, f64_bytes = _serving_plans(nap, torch, dev, mix, ["f64"] * len(mix))
    own = [wl.dtypes[0] for wl in mix]
    mx_plans, mx_vecs, mx_bytes = _serving_plans(nap, torch, dev, mix, own)
    setups = {"serial_f64": (f64_plans, f64_vecs, f64_bytes, 1, 1, ["f64"] * len(mix)),
              "served_f64": (f64_plans, f64_vecs, f64_bytes, 4, 16, ["f64"] * len(mix)),
              "served_mixed": (mx_plans, mx_vecs, mx_bytes, 4, 16, own)}
    servers = {}
    for name, (plans, vecs, nb, slots, batch, _) in setups.items():
        srv = nap.Server(slots=slots, max_batch=batch, workspace_budget=16 << 30)
        pids = [srv.add(p) for p in plans]
        srv.reserve(slots * 2)
        servers[name] = (srv, pids)
    # closed-loop capacity of the serial baseline
    ids0, _ = poisson_arrivals(1000, 1.0, len(mix), seed=55)
    srv, pids = servers["serial_f64"]
    outs0 = [torch.empty_like(f64_vecs[i]) for i in ids0]
    t0 = time.perf_counter()
    lat0, _ = srv.replay([pids[i] for i in ids0], np.zeros(len(ids0), np.int64),
                         [f64_vecs[i] for i in ids0], outs0)
    torch.cuda.synchronize()
    capacity = len(ids0) / (time.perf_counter() - t0)
    del outs0
    out = {"matrices": len(mix), "rows_min_max": [min(w.csr.n for w in mix), max(w.csr.n for w in mix)],
           "nnz_total": int(sum(w.csr.nnz for w in mix)), "requests": n_req, "discarded": warm,
           "value_types_mixed": {d: own.count(d) for d in ("f64", "f32", "bf16")},
           "serial_f64_closed_loop_capacity_rps": round(capacity, 1), "runs": []}
    errs = {}
    for rho in rhos:
        ids, arr = poisson_arrivals(n_req, rho * capacity, len(mix), seed=5)
        row = {"rho": rho, "rate_rps": round(rho * capacity, 1)}
        for name, (plans, vecs, nb, slots, batch, dts) in setups.items():
            if name == "serial_f64" and rho > 1.0:
                continue                   # an unstable queue: no steady state to report
            srv, pids = servers[name]
            outs = [torch.empty_like(vecs[i]) for i in ids]
            lat, bs = srv.replay([pids[i] for i in ids], arr, [vecs[i] for i in ids], outs)
            torch.cuda.synchronize()
            keep = slice(warm, None)
            l_us = lat[keep] / 1e3
            span_s = (arr[-1] + lat[-1] - arr[warm]) / 1e9
            total_b = float(sum(nb[i] for i in ids[keep]))
            hist = np.bincount(bs[keep], minlength=batch + 1)[1:]
            row[name] = {"p50_us": round(float(np.percentile(l_us, 50)), 1),
                         "p99_us": round(float(np.percentile(l_us, 99)), 1),
                         "mean_batch": round(float(bs[keep].mean()), 2),
                         "batch_histogram": {str(k + 1): int(c) for k, c in enumerate(hist) if c},
                         "gbs": round(total_b / span_s / 1e9, 1)}
            # oracle check of a sample of results (the last 12 of each run)
            for k in range(n_req - 12, n_req):
                i = int(ids[k])
                dt, wl = dts[i], mix[i]
                got = outs[k].cpu().numpy().astype(np.float64)
                if dt == "f64":
                    ok = bool(np.array_equal(got, oracle_spmv.spmv_split(wl.csr, wl.v, wl.n_p)))
                    e = errs.setdefault(f"{name}:f64_bitwise_vs_split_order", [0, 0])
                    e[0] += int(ok)
                    e[1] += 1
                else:
                    ref = oracle_spmv.spmv(wl.csr, wl.v)
                    r = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
                    key = f"{name}:{dt}_max_rel_err"
                    errs[key] = max(errs.get(key, 0.0), r)
            del outs
        out["runs"].append(row)
        log(f"serving rho={rho}: " + ", ".join(
            f"{k} p50 {row[k]['p50_us']} p99 {row[k]['p99_us']} us batch {row[k]['mean_batch']}"
            for k in setups if k in row))
    out["oracle_check"] = {k: (f"{v[0]}/{v[1]}" if isinstance(v, list) else v) for k, v in errs.items()}
    for srv, _ in servers.values():
        srv.close()
    for p in f64_plans + mx_plans:
        p.close()
    return out


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def _time_oracle(fn, budget_s):
    fn()                                   # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    return (time.perf_counter() - t0) / reps, reps


def cpu_baseline(wl, budget_s, lib_build_s):
    """The oracle on the host cores: its float64 CSR SpMV (plain C, OpenMP)
    on all the cores this process may use and on one core, over the full
    workload matrix, and its standard-mode plan build (NumPy) once."""
    import numpy as np
    from oracle import plan_vec
    from oracle import spmv as oracle_spmv
    a = wl.csr
    threads = len(os.sched_getaffinity(0))
    used = oracle_spmv.threads_used(threads)
    w = np.empty(a.n)
    nbytes = a.nnz * 12 + (a.n + 1) * 8 + 2 * a.n * 8
    dt, reps = _time_oracle(lambda: oracle_spmv.spmv(a, wl.v, threads=threads, out=w), budget_s)
    dt1, reps1 = _time_oracle(lambda: oracle_spmv.spmv(a, wl.v, threads=1, out=w), budget_s)
    t0 = time.perf_counter()
    plan_vec.standard_plan(a, wl.n_p, wl.ppn, wl.row_starts)
    plan_s = time.perf_counter() - t0
    return {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": used,
            "kind": "oracle",
            "sample": f"{reps} float64 CSR SpMVs of the full workload matrix "
                      f"({a.nnz} nnz) on {used} threads, {dt * 1e3:.1f} ms each; "
                      f"bytes nnz*12+(N+1)*8+2*N*8",
            "cpu_model": cpu_model(),
            "gflops": round(2 * a.nnz / dt / 1e9, 2),
            "single_core": {"value": round(nbytes / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                            "ms_per_spmv": round(dt1 * 1e3, 1), "reps": reps1},
            "plan_build_s": {"oracle_standard": round(plan_s, 2),
                             "library_standard": round(lib_build_s, 3)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--block-nnz", type=int, default=-1)
    ap.add_argument("--window", type=int, default=-1)
    ap.add_argument("--gather-item", type=int, default=-1)
    ap.add_argument("--remote-nnz", type=int, default=-1)
    ap.add_argument("--extras", type=int, default=1,
                    help="also time the other configurations, NAP mode and reduced precision")
    ap.add_argument("--batched", type=int, default=1, help="also run the batched workloads")
    ap.add_argument("--serving", type=int, default=1, help="also run the serving workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib", type=int, default=0,
                    help="end with the counter calibration kernels: three plain 1 GiB device "
                         "copies and three line-permuted gathers of 512 MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the whole hot path lives on one device); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1612_08060_amd as nap
    from workloads import bf16_bits, config, digest, to_f32

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nap.load_library()
    dev = torch.device("cuda:0")
    flush = Flush(torch, dev)
    t = time.perf_counter()
    wl = config(args.config)
    a = wl.csr
    log(f"workload {wl.name}: n={a.n} nnz={a.nnz} ({time.perf_counter() - t:.1f}s) "
        f"sha256={digest(a.rowptr, a.col, a.val, wl.v)[:16]}")

    plan = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="standard", dtype="f64",
                    row_starts=wl.row_starts)
    tuning = {"block_nnz": args.block_nnz, "window": args.window, "gather_item": args.gather_item,
              "remote_nnz": args.remote_nnz}
    for k, x in tuning.items():
        plan.set_param(k, x)
    tuning = {k: plan.get_param(k) for k in tuning}
    st = plan.stats
    log(f"standard plan: build {st['build_seconds']:.2f}s upload {st['upload_seconds']:.2f}s "
        f"tuning {tuning}")
    v = torch.from_numpy(wl.v).to(dev)
    w = torch.empty_like(v)

    # the timed region: K cold applies, then K warm ones, then K after a
    # write-only flush
    cold, c_loc, c_rem, _ = time_applies(torch, plan, v, w, nap, args.steps, args.warmup, flush)
    warm, w_loc, w_rem, wall = time_applies(torch, plan, v, w, nap, args.steps, args.warmup)
    cold_wo, o_loc, o_rem, _ = time_applies(torch, plan, v, w, nap, args.steps, 0,
                                            Flush(torch, dev, write_only=True))
    total = apply_bytes(st, 8, 8)
    rows_off = rows_with_off_entries(a, wl.n_p, wl.row_starts)
    lb, rb = launch_bytes(st, 8, 8, rows_off)
    ms = float(np.median(cold))
    log(f"apply cold median {ms:.4f} ms, warm median {np.median(warm):.4f} ms "
        f"(cold local {np.mean(c_loc):.4f}, remote {np.mean(c_rem):.4f})")
    # roofline of the dominant launch: its mean duration over every timed
    # launch (cold, warm and write-only cold), the average a kernel trace of
    # the same command reports
    loc_ms = float(np.mean(c_loc + w_loc + o_loc))
    rem_ms = float(np.mean(c_rem + w_rem + o_rem))
    dom = "k_local" if loc_ms >= rem_ms else "k_remote"
    dom_ms, dom_bytes = (loc_ms, lb) if dom == "k_local" else (rem_ms, rb)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    copy = copy_denominator(torch, dev)
    gbs_cold = total / (ms * 1e-3) / 1e9
    gbs_warm = total / (float(np.median(warm)) * 1e-3) / 1e9
    result = {
        "metric": "SpMV GB/s vs HBM peak; NAP vs std ghost bytes; serve p50/p99 latency",
        # value: the split SpMV plus ghost gather, algorithmic GB/s; the ghost
        # bytes and the serving latencies are the ghost_bytes and serving fields
        "value": round(gbs_cold, 2),
        "value_is": "split SpMV + ghost gather, algorithmic GB/s per apply at the cold median",
        "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": a.n, "nnz": a.nnz, "n_p": wl.n_p, "ppn": wl.ppn,
                   "mode": "standard", "bytes_per_step": total, "tuning": tuning},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(f"{dom}_kkt_f64"), "kernel": dom,
                     "kernel_ms": round(dom_ms, 5), "kernel_bytes": dom_bytes,
                     "kernel_ms_is": "mean of every timed launch (cold, warm, write-only cold)"},
        "timing": {"cold_ms": pct(cold), "warm_ms": pct(warm), "cold_write_only_ms": pct(cold_wo),
                   "warm_wall_ms_per_apply": round(wall, 5),
                   "cold_launch_ms": {"k_local": pct(c_loc), "k_remote": pct(c_rem)},
                   "warm_launch_ms": {"k_local": pct(w_loc), "k_remote": pct(w_rem)},
                   "flush": "cold: 1 GiB device write then 1 GiB read of another buffer before "
                            "each apply; cold_write_only: the write alone"},
        "frac_of_hbm_peak": {"cold": round(gbs_cold / PEAK_HBM_GBS, 4),
                             "warm": round(gbs_warm / PEAK_HBM_GBS, 4)},
        "copy_denominator": dict(copy, frac_cold=round(gbs_cold / copy["gbs"], 4)),
        "gflops": round(2 * a.nnz / (ms * 1e-3) / 1e9, 1),
        "launches": {"k_local": {"bytes": lb, "mean_ms": round(loc_ms, 5),
                                 "gbs": round(lb / (loc_ms * 1e-3) / 1e9, 1)},
                     "k_remote": {"bytes": rb, "mean_ms": round(rem_ms, 5),
                                  "gbs": round(rb / (rem_ms * 1e-3) / 1e9, 1)}},
        "plan_build_s": {"standard": round(st["build_seconds"], 3)},
    }
    plan.close()
    steps2 = max(10, args.steps // 2)

    if args.extras:
        cfgs = {}
        # reduced-precision values, float32 accumulation: error against the
        # float64 oracle's product
        from oracle import spmv as oracle_spmv
        ref = oracle_spmv.spmv(a, wl.v)
        vf = torch.from_numpy(to_f32(wl.v)).to(dev)
        for dt, vals in (("f32", to_f32(a.val)), ("bf16", bf16_bits(a.val))):
            pr = nap.Plan(a.rowptr, a.col, vals, a.n, wl.n_p, wl.ppn, mode="standard",
                          dtype=dt, row_starts=wl.row_starts)
            wr = torch.empty_like(vf)
            sr = pr.stats
            row = config_row(torch, nap, pr, vf, wr, apply_bytes(sr, 4 if dt == "f32" else 2, 4),
                             steps2, 3, flush, nnz=a.nnz)
            got = wr.cpu().numpy().astype(np.float64)
            row["rel_err_vs_f64_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            row["speedup_vs_f64_cold"] = round(ms / row["cold_ms"]["median"], 3)
            cfgs[f"{wl.name}_{dt}"] = row
            pr.close()
            log(f"{dt}: cold {row['cold_ms']['median']} ms, {row['gbs_cold']} GB/s")
        del vf
        # NAP mode on the same workload: same ghosts, node-aware messages
        pn = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts)
        sn = pn.stats
        w2 = torch.empty_like(v)
        row = config_row(torch, nap, pn, v, w2, apply_bytes(sn, 8, 8), steps2, 3, flush)
        torch.cuda.synchronize()
        pl = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="standard", dtype="f64",
                      row_starts=wl.row_starts)
        pl.apply(v, w)
        torch.cuda.synchronize()
        pl.close()
        row["bitwise_equal_to_standard"] = bool(torch.equal(w, w2))
        cfgs[f"{wl.name}_nap_f64"] = row
        result["plan_build_s"]["nap"] = round(sn["build_seconds"], 3)
        sph, nph = st["phases"], sn["phases"]
        result["ghost_bytes"] = {
            "standard_inter": {"msgs": sph["INTER"]["msgs"], "bytes": sph["INTER"]["elems"] * 8,
                               "max_msgs_sent": sph["INTER"]["max_msgs_sent"],
                               "max_bytes_sent": sph["INTER"]["max_elems_sent"] * 8},
            "nap_inter": {"msgs": nph["INTER"]["msgs"], "bytes": nph["INTER"]["elems"] * 8,
                          "max_msgs_sent": nph["INTER"]["max_msgs_sent"],
                          "max_bytes_sent": nph["INTER"]["max_elems_sent"] * 8},
            "standard_intra_bytes": sph["L2"]["elems"] * 8,
            "nap_intra_bytes": (nph["L0"]["elems"] + nph["L1"]["elems"] + nph["L2"]["elems"]) * 8,
        }
        pn.close()
        del w2
        # the 2D 5-point Laplacian 64x64 (launch-bound) and the 3D 7-point
        # Laplacian 128^3, both modes
        for k, unit in ((1, "us"), (2, "ms")):
            wk = config(k)
            ak = wk.csr
            vk = torch.from_numpy(wk.v).to(dev)
            for mode in ("standard", "nap"):
                pk = nap.Plan(ak.rowptr, ak.col, ak.val, ak.n, wk.n_p, wk.ppn, mode=mode, dtype="f64")
                wkk = torch.empty_like(vk)
                row = config_row(torch, nap, pk, vk, wkk, apply_bytes(pk.stats, 8, 8),
                                 100, 10, flush, nnz=ak.nnz, graph=True, unit=unit)
                cfgs[f"{wk.name}_{mode}_f64"] = row
                pk.close()
                log(f"{wk.name} {mode}: cold {row[f'cold_{unit}']['median']} {unit}, "
                    f"graph {row[f'graph_{unit}_per_apply']} {unit}")
            del vk
        result["configs"] = cfgs

        ext = {}
        # algorithm NAPSpMV's three-part product, exchange beside the on_node product
        bn = apply_bytes(sn, 8, 8)
        p3 = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts, variant=("three_way",))
        w3 = torch.empty_like(v)
        t3, _, _, _ = time_applies(torch, p3, v, w3, nap, steps2, 2)
        ext["nap_three_way_f64"] = {"warm_ms": pct(t3),
                                    "gbs_warm": round(bn / (np.median(t3) * 1e-3) / 1e9, 1)}
        p3.close()
        del w3
        # direct reads (a device option outside the paper's algorithm: the
        # off_node -> on_node and fully local steps move no data)
        pd = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts, variant=("direct",))
        wd = torch.empty_like(v)
        td, _, _, _ = time_applies(torch, pd, v, wd, nap, steps2, 2)
        torch.cuda.synchronize()
        bd = spmv_bytes(sn, 8, 8) + exchange_bytes(sn, 8, direct=True)
        ext["nap_direct_reads_f64_not_the_papers_nap"] = {
            "warm_ms": pct(td), "gbs_warm_own_bytes": round(bd / (np.median(td) * 1e-3) / 1e9, 1),
            "bitwise_equal_to_standard": bool(torch.equal(w, wd))}
        pd.close()
        del wd
        # message statistics of the mapping variants (host-only plans)
        var = {}
        for name in ("owner_map", "split", "dedup"):
            with nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap",
                          row_starts=wl.row_starts, host_only=True, variant=(name,)) as ph:
                q = ph.stats["phases"]
            var[name] = {k: {"msgs": q[k]["msgs"], "elems": q[k]["elems"],
                             "max_msgs_sent": q[k]["max_msgs_sent"]} for k in ("INTER", "L0", "L1", "L2")}
        result["nap_variant_messages"] = var
        # third hierarchy level: intra-node messages on and off a socket of 8 ranks
        lev = {"procs_per_socket": 8}
        for mode in ("standard", "nap"):
            with nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode=mode,
                          row_starts=wl.row_starts, host_only=True) as ph:
                q = ph.level_stats(8)
            lev[mode] = {k: {side: {"msgs": q[k][side]["msgs"], "bytes": q[k][side]["elems"] * 8}
                             for side in ("on_socket", "off_socket")}
                         for k in ("L0", "L1", "L2") if mode == "nap" or k == "L2"}
        result["socket_level"] = lev
        # the socket level as a plan: each intra-node step routed per socket pair
        pk = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts, sockets=8)
        wk = torch.empty_like(v)
        tk, _, _, _ = time_applies(torch, pk, v, wk, nap, steps2, 2)
        torch.cuda.synchronize()
        sk = pk.socket_stats()
        lev["socket_plan"] = {
            "build_s": round(pk.stats["build_seconds"], 3), "warm_ms": pct(tk),
            "bitwise_equal_to_standard": bool(torch.equal(w, wk)),
            "workspace_bytes": pk.workspace_bytes,
            "phases": {k: {"msgs": x["msgs"], "elems": x["elems"], "max_msgs_sent": x["max_msgs_sent"]}
                       for k, x in sk.items()}}
        pk.close()
        del wk
        # strided partition (row r on process r mod n_p): process-major v and w
        strided = {}
        for mode in ("standard", "nap"):
            ps_ = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode=mode, dtype="f64",
                           strided=True)
            rows = torch.from_numpy(ps_.rows()).to(dev)
            vs_ = v[rows].contiguous()
            ws_ = torch.empty_like(vs_)
            ts, _, _, _ = time_applies(torch, ps_, vs_, ws_, nap, steps2, 2)
            ss = ps_.stats
            bs = apply_bytes(ss, 8, 8)
            q = ss["phases"]
            strided[mode] = {"warm_ms": pct(ts), "gbs_warm": round(bs / (np.median(ts) * 1e-3) / 1e9, 1),
                             "ghosts": ss["ghosts"], "inter_msgs": q["INTER"]["msgs"],
                             "inter_bytes": q["INTER"]["elems"] * 8,
                             "max_inter_msgs_sent": q["INTER"]["max_msgs_sent"]}
            ps_.close()
            del vs_, ws_, rows
        result["strided_partition"] = strided
        result["extras"] = ext

    if args.batched:
        log("batched 256-block workload ...")
        result["batched"] = bench_batched(torch, nap, dev)
        from workloads import serving_mix
        log("multi-matrix batch ...")
        result["multi_matrix_batch"] = bench_multi_batch(torch, nap, dev, serving_mix())
    if args.serving:
        log("serving workload ...")
        result["serving"] = bench_serving(torch, nap, dev)
    if args.cpu_seconds > 0:
        log("timing the CPU oracle ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, st["build_seconds"])
    if args.calib:
        # counter calibration: a plain copy (read and write 1 GiB each) and a
        # gather that reads every 128-byte line of a 512 MiB source exactly
        # once, in a random line order, 16 consecutive lanes per line (plus
        # the int64 index stream of the same size)
        x = torch.ones(FLUSH_BYTES // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        src = torch.ones((FLUSH_BYTES // 2) // 8, dtype=torch.float64, device=dev)
        lines = src.numel() // 16
        perm = torch.randperm(lines, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
        idx = (perm.view(-1, 1) * 16 + torch.arange(16, device=dev).view(1, -1)).reshape(-1)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.index_select(src, 0, idx, out=dst)
        torch.cuda.synchronize()
        result["calibration"] = {"copy_bytes_each_way": FLUSH_BYTES,
                                 "gather_source_bytes": src.numel() * 8,
                                 "gather_index_bytes": idx.numel() * 8,
                                 "gather_write_bytes": dst.numel() * 8}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
