"""Benchmark of the node-aware SpMV hot path on one MI355X.

One step = one apply of the plan: the exchange that fills every process's
ghost buffer from v (section 2.1 / section 4 messages as device gathers) and
the split product w = A_on v + A_off ghost, over the largest paper-shaped
workload (KKT-like random matrix, N = 2^22, n_p = 2048, ppn = 16, float64),
inputs resident in HBM.  Prints ONE JSON line on stdout; progress goes to
stderr.

value = algorithmic bytes of one apply / time per apply (GB/s).  The bytes
count every array element the method must touch once:
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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


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


def measured_traffic(name: str, launch_bytes: float):
    """HBM traffic of the dominant kernel from the committed counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_hash():
        return None
    return t.get("bytes_per_launch")


def time_apply(plan, v, w, steps, warmup, torch, nap):
    """Warm up, then time exactly `steps` applies; events bracket each of the
    two launches on the stream they run on."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.apply(v, w, stream=stream)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        plan.apply_stage(nap.STAGE_LOCAL, v, w, stream=stream)
        ev[k][1].record(stream)
        plan.apply_stage(nap.STAGE_REMOTE, v, w, stream=stream)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    local = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    remote = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    return (t1 - t0) * 1e3 / steps, sum(local) / steps, sum(remote) / steps


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_ms(torch, fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


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
    default_ms = _time_ms(torch, lambda: p.apply(v, w), reps)
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
    nbytes = spmv_bytes(st, 4, 4) + exchange_bytes(st, 4)
    g.close()
    p.close()
    sizes = np.diff(wl.row_starts)
    return {"workload": wl.name, "n": a.n, "nnz": a.nnz, "blocks": wl.n_p,
            "block_rows_min_median_max": [int(sizes.min()), int(np.median(sizes)), int(sizes.max())],
            "dtype": "f32", "bytes_per_apply": nbytes,
            "batched_graph_ms": round(batched_ms, 5),
            "batched_gbs": round(nbytes / (batched_ms * 1e-3) / 1e9, 1),
            "default_tuning_ms": round(default_ms, 5), "autotuned": tuning,
            "autotune_best_ms": round(tune_ms, 5),
            "per_block_launches_eager_ms": round(parts_eager_ms, 4),
            "per_block_launches_graph_ms": round(parts_graph_ms, 4),
            "speedup_vs_per_block_eager": round(parts_eager_ms / batched_ms, 2),
            "speedup_vs_per_block_graph": round(parts_graph_ms / batched_ms, 2),
            "per_block_equals_batched_bitwise": same}


def bench_serving(torch, nap, dev, n_req=3000, warm=300, rhos=(0.5, 0.8, 0.95)):
    """Poisson-arrival requests on 64 resident matrices of mixed size, type
    and value precision, served with continuous batching (4 slots, batches
    up to 16, 16 GiB workspace budget), against each request served alone in
    arrival order on the plain float64 path."""
    import numpy as np
    from workloads import bf16_bits, poisson_arrivals, serving_mix, to_f32
    mix = serving_mix()
    vals = {"f64": lambda x: x, "f32": to_f32, "bf16": bf16_bits}
    served, plain, vin, vin64, nbytes = [], [], [], [], []
    for wl in mix:
        a, dt = wl.csr, wl.dtypes[0]
        served.append(nap.Plan(a.rowptr, a.col, vals[dt](a.val), a.n, wl.n_p, wl.ppn,
                               mode="standard", dtype=dt))
        plain.append(nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="standard"))
        vin.append(torch.from_numpy(wl.v if dt == "f64" else to_f32(wl.v)).to(dev))
        vin64.append(torch.from_numpy(wl.v).to(dev))
        st = served[-1].stats
        sa = {"f64": 8, "f32": 4, "bf16": 2}[dt]
        sv = 8 if dt == "f64" else 4
        nbytes.append(spmv_bytes(st, sa, sv) + exchange_bytes(st, sv))
    # serial float64 capacity: mean service time over a uniform matrix choice
    w64 = [torch.empty_like(x) for x in vin64]
    service = [_time_ms(torch, lambda k=k: plain[k].apply(vin64[k], w64[k]), 5)
               for k in range(len(mix))]
    capacity = 1000.0 / float(np.mean(service))          # requests per second
    out = {"matrices": len(mix), "rows_min_max": [min(w.csr.n for w in mix), max(w.csr.n for w in mix)],
           "nnz_total": int(sum(w.csr.nnz for w in mix)), "requests": n_req, "discarded": warm,
           "serial_f64_mean_service_ms": round(float(np.mean(service)), 4),
           "serial_f64_capacity_rps": round(capacity, 1), "runs": []}
    for rho in rhos:
        ids, arr = poisson_arrivals(n_req, rho * capacity, len(mix), seed=5)
        row = {"rho": rho, "rate_rps": round(rho * capacity, 1)}
        for label, plans, vecs, slots, batch in (("serial_f64", plain, vin64, 1, 1),
                                                 ("served", served, vin, 4, 16)):
            srv = nap.Server(slots=slots, max_batch=batch, workspace_budget=16 << 30)
            pids = [srv.add(pl) for pl in plans]
            outs = [torch.empty_like(vecs[i]) for i in ids]
            lat, bs = srv.replay([pids[i] for i in ids], arr, [vecs[i] for i in ids], outs)
            torch.cuda.synchronize()
            keep = slice(warm, None)
            l_us = lat[keep] / 1e3
            span_s = (arr[-1] + lat[-1] - arr[warm]) / 1e9
            total_b = float(sum(nbytes[i] for i in ids[keep]))
            row[label] = {"p50_us": round(float(np.percentile(l_us, 50)), 1),
                          "p99_us": round(float(np.percentile(l_us, 99)), 1),
                          "mean_batch": round(float(bs[keep].mean()), 2),
                          "gbs": round(total_b / span_s / 1e9, 1)}
            if label == "served":
                errs = {}
                for k in range(warm, min(n_req, warm + 200)):
                    i = int(ids[k])
                    dt = mix[i].dtypes[0]
                    ref = torch.empty_like(vin64[i])
                    plain[i].apply(vin64[i], ref)
                    r = ref.cpu().numpy()
                    e = float(np.linalg.norm(outs[k].cpu().numpy().astype(np.float64) - r)
                              / max(np.linalg.norm(r), 1e-300))
                    errs[dt] = max(errs.get(dt, 0.0), e)
                row[label]["max_rel_err_vs_f64"] = errs
            srv.close()
        out["runs"].append(row)
    for pl in served + plain:
        pl.close()
    return out


def cpu_baseline(wl, budget_s):
    """The oracle's float64 CSR SpMV (plain C, OpenMP) on the host cores."""
    import numpy as np
    from oracle import spmv as oracle_spmv
    a = wl.csr
    threads = len(os.sched_getaffinity(0))
    used = oracle_spmv.threads_used(threads)
    w = np.empty(a.n)
    oracle_spmv.spmv(a, wl.v, threads=threads, out=w)          # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle_spmv.spmv(a, wl.v, threads=threads, out=w)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    nbytes = a.nnz * 12 + (a.n + 1) * 8 + 2 * a.n * 8
    return {"value": round(nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": used,
            "kind": "oracle",
            "sample": f"{reps} float64 CSR SpMVs of the full workload matrix "
                      f"({a.nnz} nnz), {dt * 1e3:.1f} ms each; bytes nnz*12+(N+1)*8+2*N*8"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--block-nnz", type=int, default=-1)
    ap.add_argument("--window", type=int, default=-1)
    ap.add_argument("--gather-item", type=int, default=-1)
    ap.add_argument("--remote-nnz", type=int, default=-1)
    ap.add_argument("--extras", type=int, default=1, help="also time NAP mode and reduced precision")
    ap.add_argument("--batched", type=int, default=1, help="also run the batched 256-block workload")
    ap.add_argument("--serving", type=int, default=1, help="also run the serving workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="end with three plain 1 GiB device copies (counter calibration)")
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
    t = time.perf_counter()
    wl = config(args.config)
    a = wl.csr
    log(f"workload {wl.name}: n={a.n} nnz={a.nnz} ({time.perf_counter() - t:.1f}s) "
        f"sha256={digest(a.rowptr, a.col, a.val, wl.v)[:16]}")

    t = time.perf_counter()
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

    ms, local_ms, remote_ms = time_apply(plan, v, w, args.steps, args.warmup, torch, nap)
    total = spmv_bytes(st, 8, 8) + exchange_bytes(st, 8)
    rows_off = rows_with_off_entries(a, wl.n_p, wl.row_starts)
    lb, rb = launch_bytes(st, 8, 8, rows_off)
    log(f"apply {ms:.4f} ms  (local {local_ms:.4f} ms, remote {remote_ms:.4f} ms)")
    dom = "k_local" if local_ms >= remote_ms else "k_remote"
    dom_ms, dom_bytes = (local_ms, lb) if dom == "k_local" else (remote_ms, rb)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(f"{dom}_kkt_f64", dom_bytes)
    result = {
        "metric": "SpMV GB/s vs HBM peak; NAP vs std ghost bytes; serve p50/p99 latency",
        # value: the split SpMV plus ghost gather, algorithmic GB/s; the ghost
        # bytes and the serving latencies are the ghost_bytes and serving fields
        "value": round(total / (ms * 1e-3) / 1e9, 2),
        "value_is": "split SpMV + ghost gather, algorithmic GB/s per apply",
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
                     "traffic": traffic, "kernel": dom,
                     "kernel_ms": round(dom_ms, 5), "kernel_bytes": dom_bytes},
        "frac_of_hbm_peak": round(total / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "gflops": round(2 * a.nnz / (ms * 1e-3) / 1e9, 1),
        "launches": {"k_local": {"ms": round(local_ms, 5), "bytes": lb,
                                 "gbs": round(lb / (local_ms * 1e-3) / 1e9, 1)},
                     "k_remote": {"ms": round(remote_ms, 5), "bytes": rb,
                                  "gbs": round(rb / (remote_ms * 1e-3) / 1e9, 1)}},
        "plan_build_s": {"standard": round(st["build_seconds"], 3)},
    }
    plan.close()

    if args.extras:
        ext = {}
        # NAP mode: same ghosts, node-aware messages
        pn = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts)
        sn = pn.stats
        w2 = torch.empty_like(v)
        ms_n, ex_n, sp_n = time_apply(pn, v, w2, max(10, args.steps // 2), 2, torch, nap)
        bn = spmv_bytes(sn, 8, 8) + exchange_bytes(sn, 8)
        torch.cuda.synchronize()
        ext["nap_f64"] = {"ms": round(ms_n, 5), "gbs": round(bn / (ms_n * 1e-3) / 1e9, 1),
                          "local_ms": round(ex_n, 5), "remote_ms": round(sp_n, 5),
                          "bitwise_equal_to_standard": bool(torch.equal(w, w2))}
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
        # algorithm NAPSpMV's three-part product, exchange beside the on_node product
        p3 = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts, variant=("three_way",))
        w3 = torch.empty_like(v)
        ms_3, ex_3, sp_3 = time_apply(p3, v, w3, max(10, args.steps // 2), 2, torch, nap)
        ext["nap_three_way_f64"] = {"ms": round(ms_3, 5), "gbs": round(bn / (ms_3 * 1e-3) / 1e9, 1),
                                    "local_ms": round(ex_3, 5), "remote_ms": round(sp_3, 5)}
        p3.close()
        del w3
        # direct reads: off-node ghosts read in place from the received buffer
        pd = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap", dtype="f64",
                      row_starts=wl.row_starts, variant=("direct",))
        wd = torch.empty_like(v)
        ms_d, ex_d, sp_d = time_apply(pd, v, wd, max(10, args.steps // 2), 2, torch, nap)
        torch.cuda.synchronize()
        bd = spmv_bytes(sn, 8, 8) + exchange_bytes(sn, 8, direct=True)
        ext["nap_direct_f64"] = {"ms": round(ms_d, 5), "gbs": round(bd / (ms_d * 1e-3) / 1e9, 1),
                                 "local_ms": round(ex_d, 5), "remote_ms": round(sp_d, 5),
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
        # strided partition (row r on process r mod n_p): process-major v and w
        strided = {}
        for mode in ("standard", "nap"):
            ps_ = nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode=mode, dtype="f64",
                           strided=True)
            rows = torch.from_numpy(ps_.rows()).to(dev)
            vs_ = v[rows].contiguous()
            ws_ = torch.empty_like(vs_)
            ms_s, ex_s, sp_s = time_apply(ps_, vs_, ws_, max(10, args.steps // 2), 2, torch, nap)
            ss = ps_.stats
            bs = spmv_bytes(ss, 8, 8) + exchange_bytes(ss, 8)
            q = ss["phases"]
            strided[mode] = {"ms": round(ms_s, 5), "gbs": round(bs / (ms_s * 1e-3) / 1e9, 1),
                             "ghosts": ss["ghosts"], "inter_msgs": q["INTER"]["msgs"],
                             "inter_bytes": q["INTER"]["elems"] * 8,
                             "max_inter_msgs_sent": q["INTER"]["max_msgs_sent"]}
            ps_.close()
            del vs_, ws_, rows
        result["strided_partition"] = strided
        # reduced-precision values, float32 accumulation; error against the
        # float64 apply above (itself checked against the oracle by the tests)
        ref = w.cpu().numpy()
        vf = torch.from_numpy(to_f32(wl.v)).to(dev)
        for dt, vals in (("f32", to_f32(a.val)), ("bf16", bf16_bits(a.val))):
            pr = nap.Plan(a.rowptr, a.col, vals, a.n, wl.n_p, wl.ppn, mode="standard",
                          dtype=dt, row_starts=wl.row_starts)
            wr = torch.empty_like(vf)
            ms_r, ex_r, sp_r = time_apply(pr, vf, wr, max(10, args.steps // 2), 2, torch, nap)
            sr = pr.stats
            br = spmv_bytes(sr, 4 if dt == "f32" else 2, 4) + exchange_bytes(sr, 4)
            got = wr.cpu().numpy().astype(np.float64)
            ext[dt] = {"ms": round(ms_r, 5), "gbs": round(br / (ms_r * 1e-3) / 1e9, 1),
                       "speedup_vs_f64": round(ms / ms_r, 3),
                       "rel_err_vs_f64_apply": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
            pr.close()
        # the 3D 7-point Laplacian, 128^3, n_p = 1024 at ppn = 16 (float64)
        wl2 = config(2)
        a2 = wl2.csr
        v2 = torch.from_numpy(wl2.v).to(dev)
        lap = {}
        for mode in ("standard", "nap"):
            p2 = nap.Plan(a2.rowptr, a2.col, a2.val, a2.n, wl2.n_p, wl2.ppn, mode=mode, dtype="f64")
            w2 = torch.empty_like(v2)
            ms2, ex2, sp2 = time_apply(p2, v2, w2, max(10, args.steps // 2), 2, torch, nap)
            s2 = p2.stats
            b2 = spmv_bytes(s2, 8, 8) + exchange_bytes(s2, 8)
            lap[mode] = {"ms": round(ms2, 5), "gbs": round(b2 / (ms2 * 1e-3) / 1e9, 1),
                         "local_ms": round(ex2, 5), "remote_ms": round(sp2, 5)}
            p2.close()
            del w2
        ext["laplace3d_128cube_np1024_ppn16_f64"] = lap
        del v2
        result["extras"] = ext

    if args.batched:
        log("batched 256-block workload ...")
        result["batched"] = bench_batched(torch, nap, dev)
    if args.serving:
        log("serving workload ...")
        result["serving"] = bench_serving(torch, nap, dev)
    if args.cpu_seconds > 0:
        log("timing the CPU oracle ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    if args.calib_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
