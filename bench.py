"""Benchmark of the temporal 3-path sampling path on one MI355X.

Default workload (the largest single-GPU configuration): the Bitcoin-like
graph (5*10^7 vertices, 3*10^8 edges, Zipf(1.9) endpoints with hubs over 10^6
edges, Geometric(0.5) repeats per pair, times uniform over seven years), the
4-cycle motif M4-0, delta in {3,600; 86,400} and k = 10^8 samples per delta.
A step is one pass of the whole hot path: adjacency build (tc_build_graph),
weights and scan for both deltas in one call (tc_path_weights_batch), and
sampling with closure
and reduction for both deltas in one batched launch sequence
(tc_batch_estimate).  The edge arrays are resident in HBM before the timed
region.  `value` is samples per second of the whole step (2 * 10^8 samples
per step); per-stage times, algorithmic and counter-measured HBM GB/s, the
roofline of the dominant kernel and the CPU oracle timed on a bounded sample
of the same workload are reported beside it.  Extra keys hold the medium
workload's step and the learned proposal's comparison on that graph.

Other workloads: --workload medium | tiny (one delta, six motifs),
--workload batched (six motifs x four deltas on the Bitcoin-like graph, the
whole path captured in one HIP graph and replayed).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bfloat16 MFMA
KERNELS = ["k_paths", "k_listcount_reg", "k_listcount_lds", "k_listcount_wide", "k_windows",
           "k_scan_apply", "k_radix_scatter"]
# Kernel -> source file whose hash must match the stored counter readings.
KERNEL_SRC = {"k_paths": "tc_sample.hip", "k_listcount_reg": "tc_sample.hip",
              "k_listcount_lds": "tc_sample.hip", "k_listcount_wide": "tc_sample.hip",
              "k_windows": "tc_weights.hip", "k_scan_apply": "tc_weights.hip",
              "k_radix_scatter": "tc_build.hip"}
# the kernels each timed span covers, for counter-based traffic per span
SPAN_KERNELS = {"k_windows": ["k_mp_split_coarse", "k_mp_split", "k_mp_rank", "k_combine"]}
PMC_FILES = {"bitcoin": os.path.join(ROOT, "profiles", "pmc_traffic_bitcoin.txt"),
             "medium": os.path.join(ROOT, "profiles", "pmc_traffic_medium.txt")}
# stages of a step -> kernels whose counter traffic makes up the stage
STAGE_KERNELS = {
    "build": ["k_init_build", "k_validate", "k_plan", "k_trange", "k_fold_hist", "k_hash_clear",
              "k_rec_init", "k_radix_hist", "k_col_sum", "k_col_scan", "k_col_apply", "k_radix_scatter",
              "k_rec_xform", "k_emit", "k_offsets", "k_hash_insert"],
    "weights": ["k_mp_split_coarse", "k_mp_split", "k_mp_rank", "k_combine", "k_scan_tiles",
                "k_scan_tiles_sets", "k_scan_apply"],
    "sample": ["k_zero_result", "k_store_ptrs", "k_zero_counters", "k_paths", "k_listcount_reg",
               "k_listcount_lds", "k_listcount_wide", "k_listcount_w128", "k_listcount_big", "k_finalize"],
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bitcoin",
                    choices=["bitcoin", "medium", "tiny", "batched"],
                    help="bitcoin: the headline step; medium/tiny: one delta, six motifs; "
                         "batched: six motifs x four deltas on the Bitcoin-like graph, the "
                         "whole path in one captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the medium-workload and learned-proposal extra keys")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal versus method comparison")
    ap.add_argument("--cpu-sample", type=int, default=10**6,
                    help="samples per delta the oracle draws for the CPU baseline")
    ap.add_argument("--learned-seeds", type=int, default=32)
    ap.add_argument("--k-ref", type=float, default=1e10,
                    help="samples of the reference estimate C_ref")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB device-to-device first (reference for HBM counters)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one step of the workload and nothing else (for counter runs)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_alg_bytes(kernel, m, units, nd=1):
    """Algorithmic bytes of one launch: a per-unit figure times the units the
    launch processes.  Data-dependent searches inside adjacency lists and
    pair runs are not counted, so these are lower bounds.
      k_paths          per sample: ceil(log2(m+1)) probes of S (8 B each), the
                       centre edge with its window metadata (32 B), the two end
                       edges (16 B each)
      k_windows        per edge of a call over nd deltas: read the (vertex,
                       time) keys of both CSRs once (24 B), and per delta write
                       lo_in, a, lo_out, b (16 B) and the 32-byte path record
      k_scan_apply     per edge: read a, b (8 B), write S (8 B)
      k_radix_scatter  per element and pass: read and write a 16-byte edge
                       record (32 B)"""
    if kernel == "k_paths":
        per = 8 * math.ceil(math.log2(m + 1)) + 32 + 2 * 16
    elif kernel == "k_windows":
        per = 24 + (16 + 32) * nd
    elif kernel == "k_scan_apply":
        per = 16
    elif kernel == "k_radix_scatter":
        per = 32
    else:
        return None, None
    return per * units, per


def stage_alg_bytes(stage, m, k_total, nd=1):
    """Algorithmic bytes of a stage per step (the floors of the hot-path
    scope): build 64 B per edge (input 16 B + three 16-byte orders), weights
    per edge the in and out keys once (16 B) and per delta S (8 B) and the
    window metadata (16 B), sampling per sample as k_paths above."""
    if stage == "build":
        return 64 * m
    if stage == "weights":
        return (16 + 24 * nd) * m
    if stage == "sample":
        return (8 * math.ceil(math.log2(m + 1)) + 64) * k_total
    return None


def source_hash(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2409_08975_amd", "csrc", name), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def _pmc(workload):
    """(meta dict, {kernel: fields}) of the committed counter summary of a
    workload (a one-step profile run), or ({}, {})."""
    f = PMC_FILES.get(workload)
    if not f or not os.path.exists(f):
        return {}, {}
    meta, rows = {}, {}
    for line in open(f):
        if line.startswith("meta "):
            meta = dict(kv.split("=", 1) for kv in line.split()[1:] if "=" in kv)
            continue
        d = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if "kernel" in d and "hbm_bytes_per_launch" in d:
            rows[d["kernel"]] = d
    return meta, rows


def _current(d):
    from paper_2409_08975_amd.rocprof_summary import source_sha
    return d is not None and d.get("src_sha") == source_sha(d["kernel"])


def stored_traffic(workload, kernel):
    """HBM bytes per launch of a kernel from the committed counter summary of
    this workload, if it was taken on the current source (else None).  A
    timed span of several kernels (k_windows) gets its kernels' total bytes
    divided by the number of spans in the profiled run."""
    meta, rows = _pmc(workload)
    if kernel in SPAN_KERNELS:
        spans = float(meta.get("weights_calls", 0))
        parts = [rows.get(x) for x in SPAN_KERNELS[kernel]]
        if not spans or not all(_current(d) for d in parts):
            return None
        return sum(float(d["total_bytes"]) for d in parts) / spans
    d = rows.get(kernel)
    return float(d["hbm_bytes_per_launch"]) if _current(d) else None


def stage_traffic(workload, stage):
    """HBM bytes per step of one stage from the committed counters (the
    profiled run times one step: the total over the stage's kernels)."""
    meta, rows = _pmc(workload)
    steps = float(meta.get("profile_steps", 0))
    if not steps:
        return None
    parts = [rows[x] for x in STAGE_KERNELS[stage] if x in rows]
    if not parts or not all(_current(d) for d in parts):
        return None
    return sum(float(d["total_bytes"]) for d in parts) / steps


def event_ms(fn, stream):
    """Run fn() on `stream` and return (result, milliseconds between HIP events)."""
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    r = fn()
    b.record(stream)
    b.synchronize()
    return r, a.elapsed_time(b)


def host_info():
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff}


def cpu_threads():
    """Threads for the oracle: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when that is set (the host's share for one GPU)."""
    n = host_info()["affinity_cpus"]
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


# ------------------------------------------------------------ step runs -----
def run_steps(tcb, g, deltas, motifs, k, seed, steps, warmup, stream, dev, label):
    """Time `steps` whole-path steps (build, the weights of every delta in one
    batched call, sampling of every delta in one batched sequence).  Returns
    a dict of figures."""
    import torch
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    torch.cuda.synchronize()
    nd = len(deltas)
    nm = len(motifs)
    ws_s = torch.empty(tcb.batch_workspace_bytes(k, nd, nm), dtype=torch.uint8, device=dev)
    outs = [tcb.new_result(nm, k, dev) for _ in deltas]

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        G = tcb.tc_build_graph(g.n, src, dst, tt)
        ev[1].record(stream)
        Ws = tcb.tc_path_weights_batch(G, deltas)
        ev[2].record(stream)
        tcb.tc_batch_estimate(G, Ws, motifs, k, seed, outs=outs, workspace=ws_s)
        ev[3].record(stream)
        return G, Ws, ev

    for i in range(warmup):
        G, Ws, ev = step()
        torch.cuda.synchronize()
        G.check()
        for o in outs:
            o.check()
        log(f"[bench] {label} warmup {i} done")
        del G, Ws
    torch.cuda.synchronize()
    tcb.timing_reset()
    tcb.timing_enable(True)
    t_start = time.perf_counter()
    evs = []
    keep = None
    for i in range(steps):
        # the previous step's workspaces are released before the next build
        # (the caching allocator hands the same blocks back)
        G = Ws = keep = None
        G, Ws, ev = step()
        keep = (G, Ws)
        evs.append(ev)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    tcb.timing_enable(False)
    ktime = {}
    for kname in KERNELS:
        ms, n = tcb.timing_read(kname)
        if n:
            ktime[kname] = (ms, n)
    tcb.timing_reset()
    G, Ws = keep
    G.check()
    for o in outs:
        o.check()
    build = np.mean([e[0].elapsed_time(e[1]) for e in evs])
    wts = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    samp = np.mean([e[2].elapsed_time(e[3]) for e in evs])
    ms_per_step = t_total * 1000.0 / steps
    log(f"[bench] {label}: {steps} steps, {ms_per_step:.3f} ms/step; build {build:.3f} ms, "
        f"weights ({nd} deltas) {wts:.3f} ms, sampling {samp:.3f} ms")
    res = {"ms_per_step": ms_per_step, "build_ms": float(build), "weights_ms": wts,
           "sample_ms": float(samp), "ktime": ktime, "G": G, "Ws": Ws, "outs": outs, "nd": nd,
           "tensors": (src, dst, tt)}
    return res


def kernel_table(ktime, m, k_total, steps, workload, nd=1):
    kernels = {}
    for kname, (ms, n) in ktime.items():
        per_launch_ms = ms / n
        entry = {"ms_per_step": ms / steps, "launches_per_step": n / steps,
                 "ms_per_launch": per_launch_ms}
        u = None
        if kname == "k_paths":
            u = k_total / (n / steps)  # samples per launch
        elif kname in ("k_windows", "k_scan_apply", "k_radix_scatter"):
            u = m
        if u is not None:
            alg, per = kernel_alg_bytes(kname, m, u, nd if kname == "k_windows" else 1)
            gbs = alg / (per_launch_ms * 1e-3) / 1e9
            entry.update({"alg_bytes_per_unit": per, "alg_bytes_per_launch": alg,
                          "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS})
            tr = stored_traffic(workload, kname)
            entry["hbm_bytes_per_launch"] = tr
            if tr:
                entry["hbm_GBs"] = tr / (per_launch_ms * 1e-3) / 1e9
        kernels[kname] = entry
    return kernels


def roofline_of(kernels):
    cand = {k: v for k, v in kernels.items() if "achieved_GBs" in v}
    dom = max(cand, key=lambda x: cand[x]["ms_per_step"])
    d = cand[dom]
    roof = {"bound": "hbm", "achieved": round(d["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(d["frac_of_hbm_peak"], 4),
            "traffic": d.get("hbm_bytes_per_launch"), "kernel": dom,
            "ms_per_launch": round(d["ms_per_launch"], 4),
            "alg_bytes_per_unit": d["alg_bytes_per_unit"]}
    if roof["traffic"]:
        tgbs = roof["traffic"] / (d["ms_per_launch"] * 1e-3) / 1e9
        roof["traffic_GBs"] = round(tgbs, 1)
        roof["traffic_frac"] = round(tgbs / HBM_PEAK_GBS, 4)
    return roof


def stage_table(res, m, k_total, workload):
    out = {}
    spans = [("build", res["build_ms"]), ("weights", res["weights_ms"]),
             ("sample", res["sample_ms"])]
    for name, ms in spans:
        base = name
        alg = stage_alg_bytes(base, m, k_total, res["nd"])
        e = {"ms": ms, "alg_bytes": alg, "alg_GBs": alg / (ms * 1e-3) / 1e9,
             "alg_frac_of_hbm_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        tr = stage_traffic(workload, base)
        if tr is not None:
            e["hbm_bytes"] = tr
            e["hbm_GBs"] = tr / (ms * 1e-3) / 1e9
        out[name] = e
    return out


def rel_stderr(tcb, G, Ws, motifs, names, k, seed):
    """Relative standard error of each (delta, motif) estimate at k, from the
    second moment of a run with the same seed."""
    from paper_2409_08975_amd import learned as _learned
    out = {}
    for W in Ws:
        Rm = tcb.tc_sample_estimate(G, W, motifs, k, seed, moments=True)
        Rm.check("moments")
        row = {}
        for j, nm in enumerate(names):
            mm = _learned.moments(Rm, W, k, j)
            row[nm] = mm.stderr / mm.estimate if mm.estimate else None
        out[str(W.c.delta)] = row
    return out


def cpu_baseline(g, deltas, motifs, k, seed, n_sample, threads):
    """The oracle on the host's cores, on a bounded sample of the workload:
    the full build, the weights of the first delta and n_sample of its
    samples; the weights are scaled to every delta and the sampling to k per
    delta (the oracle's weights take about the same time for each delta)."""
    import oracle
    import synthgraph as sg
    mb = [sg.motif_bytes(M) for M in motifs]
    t0 = time.perf_counter()
    og = oracle.OracleGraph.from_graph(g, threads=threads)
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    ow = og.weights(deltas[0], threads=threads)
    t_w = time.perf_counter() - t0
    t0 = time.perf_counter()
    og.sample(ow, mb, n_sample, seed, threads=threads)
    t_s = time.perf_counter() - t0
    del ow, og
    nd = len(deltas)
    t_full = t_b + nd * t_w + nd * t_s * (k / n_sample)
    return {"value": nd * k / t_full, "unit": "samples/s", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle build of the full graph ({t_b:.1f} s), weights of delta "
                      f"{deltas[0]} ({t_w:.1f} s) counted for each of the {nd} deltas, "
                      f"{n_sample} of its {k} samples ({t_s:.2f} s) scaled by "
                      f"{nd * k / n_sample:.0f} to every delta's k; {threads} threads",
            "stage_s": {"build": t_b, "weights_first_delta": t_w,
                        "sample_measured": t_s, "samples_measured": n_sample},
            **host_info()}


def cpu_one_thread(g, delta, motifs, k, seed, n_sample):
    """The oracle on one thread (tiny: the whole job; larger graphs: a bounded
    number of samples, scaled)."""
    import oracle
    import synthgraph as sg
    mb = [sg.motif_bytes(M) for M in motifs]
    t0 = time.perf_counter()
    og = oracle.OracleGraph.from_graph(g, threads=1)
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    ow = og.weights(delta, threads=1)
    t_w = time.perf_counter() - t0
    ns = min(n_sample, k)
    t0 = time.perf_counter()
    og.sample(ow, mb, ns, seed, threads=1)
    t_s = time.perf_counter() - t0
    t_full = t_b + t_w + t_s * (k / ns)
    return {"value": k / t_full, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"build {t_b:.2f} s, weights {t_w:.2f} s, {ns} of {k} samples "
                      f"{t_s:.2f} s (scaled by {k / ns:.0f})"}


def learned_vs_method(tcb, G, Wt, motif, seeds, k_ref, stream):
    """Relative error against C_ref (the method at k_ref samples on its own
    stream) at k = 10^5, 10^6, 10^7 over `seeds` seeds, for the method and
    for three proposals (labels and pilots on another stream): the
    configured centre proposal (eps = 0.1, labels y = [X > 0], scores as the
    network gives them), a tuned one (eps = 0.01, soft labels min(1, X / 64),
    scores normalised by their maximum) and the window proposal (degree
    factors on the side edges, exponent and cap chosen by pilot runs), plus
    the time of each part."""
    from paper_2409_08975_amd import learned
    out = {"motif": "M4-0", "delta": int(Wt.c.delta), "seeds": seeds}
    ref, t_ref = event_ms(lambda: tcb.tc_sample_estimate(G, Wt, [motif], int(k_ref), 1,
                                                         stream_id=0x52454600, moments=True),
                          stream)
    ref.check("reference")
    mref = learned.moments(ref, Wt, int(k_ref))
    C = mref.estimate
    out["C_ref"] = C
    out["C_ref_rel_stderr"] = mref.stderr / C if C else None
    out["k_ref"] = int(k_ref)
    out["ref_ms"] = t_ref
    # the method's errors and times, shared by both comparisons
    method_rows = {}
    for k in (10**5, 10**6, 10**7):
        ep, tp = [], 0.0
        for sd in range(1, seeds + 1):
            r, t = event_ms(lambda: tcb.tc_sample_estimate(G, Wt, [motif], k, sd, stream_id=1),
                            stream)
            ep.append(float(r.estimate[0].item()))
            tp += t
        ep = np.array(ep)
        method_rows[k] = (float(np.sqrt(np.mean((ep - C) ** 2)) / C), tp / seeds)
    def evaluate(v, proposal, fixed):
        """Errors and times at each k, and the equal-error comparison: the
        proposal needs k / ratio samples for the method's error at k; its
        wall time counts the fixed cost of building the proposal set
        (training reported apart) plus sampling at k / ratio."""
        rows = []
        for k in (10**5, 10**6, 10**7):
            el, tl = [], 0.0
            for sd in range(1, seeds + 1):
                r, t = event_ms(lambda: tcb.tc_sample_estimate(G, proposal, [motif], k, sd,
                                                               stream_id=2), stream)
                el.append(float(r.estimate[0].item()))
                tl += t
            el = np.array(el)
            rows.append({"k": k, "rms_rel_err_method": method_rows[k][0],
                         "rms_rel_err_learned": float(np.sqrt(np.mean((el - C) ** 2)) / C),
                         "ms_per_estimate_method": method_rows[k][1],
                         "ms_per_estimate_learned": tl / seeds})
        v["by_k"] = rows
        ratio = v["variance_ratio"]
        if ratio:
            eq = []
            for row in rows:
                k = row["k"]
                t_m = row["ms_per_estimate_method"]
                t_l = fixed + row["ms_per_estimate_learned"] / ratio
                eq.append({"k_method": k, "k_learned": k / ratio, "wall_ms_method": t_m,
                           "wall_ms_learned": t_l, "learned_faster": t_l < t_m})
            big = rows[-1]
            per_m = big["ms_per_estimate_method"] / big["k"]
            per_l = big["ms_per_estimate_learned"] / big["k"] / ratio
            v["equal_error"] = {
                "samples_factor": ratio, "fixed_ms": fixed, "by_k": eq,
                "break_even_k": fixed / (per_m - per_l) if per_m > per_l else None}

    variants = {
        "configured": dict(eps=0.1, normalize=False, label_cap=0.0),
        "tuned": dict(eps=0.01, normalize=True, label_cap=64.0),
    }
    for name, vp in variants.items():
        v = {}
        tcb.timing_reset()
        tcb.timing_enable(True)
        lp = learned.LearnedProposal(G, Wt, motif, eps=vp["eps"], seed=11,
                                     normalize=vp["normalize"])
        _, v["features_ms"] = event_ms(lambda: tcb.tc_edge_features(G, Wt), stream)
        losses, v["train_ms"] = event_ms(
            lambda: lp.fit(n_labels=10**6, epochs=8, batch=8192, lr=3e-3,
                           label_cap=vp["label_cap"]), stream)
        v["train"] = {"labels": 10**6, "epochs": 8, "batch": 8192,
                      "label": "y = [X > 0]" if vp["label_cap"] == 0 else
                               f"min(1, X / {vp['label_cap']:g})",
                      "eps": vp["eps"], "normalized": vp["normalize"],
                      "loss_per_epoch": [round(float(x), 6) for x in losses.cpu().tolist()],
                      "label_rate": lp.label_rate}
        _, v["proposal_ms"] = event_ms(lp.build_proposal, stream)  # inference, h, q-scan
        v["proposal_status"] = lp.proposal.status()
        tcb.timing_enable(False)
        # network kernels: 2 (8*64 + 64*64 + 64) flops per row, both hidden layers on MFMA
        flop_row = 2 * (8 * 64 + 64 * 64 + 64)
        kt = {}
        for kname, rows in (("k_mlp_forward", G.m), ("k_mlp_grad", None), ("k_features", G.m)):
            ms, n = tcb.timing_read(kname)
            if not n:
                continue
            e = {"ms_per_launch": ms / n, "launches": n}
            if kname == "k_mlp_forward":
                tf = flop_row * rows / (ms / n * 1e-3) / 1e12
                e.update({"flop_per_row": flop_row, "rows": rows, "achieved_TFLOPs": tf,
                          "frac_of_bf16_dense_peak": tf / BF16_PEAK_TFLOPS})
            if kname == "k_mlp_grad":
                # forward plus backward: about three times the forward flops per row
                e["rows_per_launch"] = 8192
                e["achieved_TFLOPs"] = 3 * flop_row * 8192 / (ms / n * 1e-3) / 1e12
            kt[kname] = e
        tcb.timing_reset()
        v["kernels"] = kt
        mp, mi = lp.pilot(10**7, 0x5EED)
        v["variance_ratio"] = mp.var / mi.var if mi.var > 0 else None
        evaluate(v, lp.proposal, v["features_ms"] + v["proposal_ms"])
        out[name] = v
        del lp
    # the window proposal: degree factors on the side edges as well (the
    # exponent and cap chosen by pilot runs on the label stream)
    v = {}
    wp = learned.WindowProposal(G, Wt, motif)
    _, v["fit_ms"] = event_ms(lambda: wp.fit(k_pilot=10**6), stream)
    v["trials"] = [{"quarter": q, "cap": c, "pilot_var": var} for q, c, var in wp.trials]
    if wp.choice is not None:
        v["choice"] = {"quarter": wp.choice[0], "cap": wp.choice[1]}
        _, v["proposal_ms"] = event_ms(lambda: wp.build(*wp.choice), stream)  # factors, q-scan
        v["proposal_status"] = wp.proposal.status()
        mp, mw = wp.pilot(10**7, 0x5EED)
        v["variance_ratio"] = mp.var / mw.var if mw.var > 0 else None
        evaluate(v, wp.proposal, v["proposal_ms"])
    out["window"] = v
    del wp
    # the best learned variance ratio
    cands = [out[n].get("variance_ratio") for n in ("tuned", "window")]
    out["variance_ratio"] = max([c for c in cands if c] or [None])
    return out


def hbm_probe(dev, nbytes=4 << 30):
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of
    4 GiB (streaming read and write) and a gather of 8-byte words at random
    positions of a 4 GiB array (one line fetched per word), both timed with
    HIP events; the rates against which the kernels' figures can be read."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.int64, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    stream = torch.cuda.current_stream()
    b.copy_(a)
    _, t_copy = event_ms(lambda: b.copy_(a), stream)
    n = 1 << 26
    idx = torch.randint(0, a.numel(), (n,), device=dev, generator=torch.Generator(dev).manual_seed(5))
    out = torch.empty(n, dtype=torch.int64, device=dev)
    torch.index_select(a, 0, idx, out=out)
    _, t_gather = event_ms(lambda: torch.index_select(a, 0, idx, out=out), stream)
    res = {"copy_GBs": 2 * nbytes / (t_copy * 1e-3) / 1e9,
           "copy_bytes": 2 * nbytes, "copy_ms": t_copy,
           "random_gather_words_per_s": n / (t_gather * 1e-3),
           "random_gather_useful_GBs": (8 + 8 + 8) * n / (t_gather * 1e-3) / 1e9,
           "random_gather_ms": t_gather, "random_gather_words": n}
    del a, b, idx, out
    torch.cuda.empty_cache()
    return res


def run_medium_like(args, tcb, sg, which, stream, dev, with_learned):
    """One delta, six motifs (medium or tiny workload): the step figures."""
    P = sg.MEDIUM if which == "medium" else sg.TINY
    t0 = time.time()
    g = sg.gen_medium() if which == "medium" else sg.gen_tiny()
    log(f"[bench] generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    names = sg.SIX_MOTIFS
    motifs = [sg.MOTIFS[x] for x in names]
    delta, k, seed = P["delta"], P["k"], P["seed"]
    res = run_steps(tcb, g, [delta], motifs, k, seed, args.steps, args.warmup, stream, dev, which)
    kernels = kernel_table(res["ktime"], g.m, k, args.steps, which)
    G, Ws, outs = res["G"], res["Ws"], res["outs"]
    out = {
        "workload": f"{g.name}: n={g.n} m={g.m} delta={delta} k={k} motifs={','.join(names)}",
        "ms_per_step": res["ms_per_step"], "samples_per_s": k / (res["ms_per_step"] * 1e-3),
        "stages_ms": {"build": res["build_ms"], "weights": res["weights_ms"],
                      "sample": res["sample_ms"]},
        "stages": stage_table(res, g.m, k, which),
        "W": Ws[0].total(), "cnt": [str(c) for c in outs[0].counts()],
        "estimate": outs[0].estimate.cpu().tolist(),
        "roofline": roofline_of(kernels), "kernels": kernels,
        "rel_stderr_at_k": rel_stderr(tcb, G, Ws, motifs, names, k, seed)[str(delta)],
    }
    if with_learned:
        t0 = time.time()
        out["learned_vs_method"] = learned_vs_method(tcb, G, Ws[0], sg.MOTIFS["M4-0"],
                                                     args.learned_seeds, args.k_ref, stream)
        lv = out["learned_vs_method"]
        log(f"[bench] learned vs method in {time.time() - t0:.1f}s: variance ratio "
            f"configured {lv['configured']['variance_ratio']}, tuned {lv['tuned']['variance_ratio']}"
            f", window {lv['window'].get('variance_ratio')} {lv['window'].get('choice')}")
    return out, g


def run_batched(args):
    """Six spine-sharing motifs x delta in {600, 3600, 86400, 604800} on the
    Bitcoin-like graph, 10^8 samples per delta shared by the six motifs.  The
    whole path -- build, the four weight sets, the batched sampling with the
    autotuned launch shape -- is captured once in a HIP graph and replayed;
    every replay is checked bit for bit against an eager run."""
    import torch

    import paper_2409_08975_amd as tcb
    import synthgraph as sg

    dev = torch.device("cuda:0")
    P = sg.BITCOIN
    t0 = time.time()
    g = sg.gen_bitcoin_like()
    log(f"[bench] generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    n, m = g.n, g.m
    del g
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    motifs = [sg.MOTIFS[x] for x in sg.SIX_MOTIFS]
    deltas, k, seed = P["deltas"], P["k"], P["seed"]
    nd, nm = len(deltas), len(motifs)
    G, t_build = event_ms(lambda: tcb.tc_build_graph(n, src, dst, tt), stream)
    G.check()
    Ws, t_w = event_ms(lambda: tcb.tc_path_weights_batch(G, deltas), stream)
    log(f"[bench] eager build {t_build:.1f} ms, weights of {nd} deltas {t_w:.1f} ms")
    if args.profile_run:
        # one eager pass with the default launch shape (for counter runs)
        ws = torch.empty(tcb.batch_workspace_bytes(k, nd, nm), dtype=torch.uint8, device=dev)
        res, t_s = event_ms(lambda: tcb.tc_batch_estimate(G, Ws, motifs, k, seed, workspace=ws),
                            stream)
        print(json.dumps({"profile_run": "batched", "build_ms": t_build, "weights_ms": t_w,
                          "sample_ms": t_s, "profile_steps": 1}), flush=True)
        return
    # probes of 2^23 samples per delta, so that the chunk sizes (up to 2^25
    # samples over the deltas) differ in the probes as in the run
    best, probe_ms = tcb.tc_autotune(G, Ws, motifs, 2**23, seed=7)
    log(f"[bench] autotuned {best.as_dict()} ({probe_ms:.2f} ms per 2^23-sample probe)")
    ws = torch.empty(tcb.batch_workspace_bytes(k, nd, nm), dtype=torch.uint8, device=dev)
    ref = tcb.tc_batch_estimate(G, Ws, motifs, k, seed, workspace=ws)
    torch.cuda.synchronize()
    ref_counts = [r.counts() for r in ref]
    ref_est = [r.estimate.cpu().tolist() for r in ref]
    # per-delta status: a motif whose count reached 2^64 is named by bit 8 + j
    ref_status = [int(r.status.item()) & 0xFFFFFFFF for r in ref]
    if any(st & ~(tcb.TC_F_OVERFLOW | 0xFFFF00) for st in ref_status):
        raise tcb.TCDeviceError(max(ref_status), "batched reference")
    # the whole path in one graph, on workspaces allocated beforehand
    ws_g = torch.empty(tcb.graph_workspace_bytes(n, m), dtype=torch.uint8, device=dev)
    ws_w = torch.empty(tcb.weights_batch_workspace_bytes(m, nd), dtype=torch.uint8, device=dev)
    outs = [tcb.new_result(nm, k, dev) for _ in deltas]
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=side):
        G2 = tcb.tc_build_graph(n, src, dst, tt, workspace=ws_g)
        W2 = tcb.tc_path_weights_batch(G2, deltas, workspace=ws_w)
        tcb.tc_batch_estimate(G2, W2, motifs, k, seed, tuning=best, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        cg.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        _, t = event_ms(cg.replay, stream)
        times.append(t)
        for o, rc, rs in zip(outs, ref_counts, ref_status):
            assert (int(o.status.item()) & 0xFFFFFFFF) == rs, "replay status differs"
            assert o.counts() == rc, "replay differs from the eager result"
    ms = float(np.mean(times))
    log(f"[bench] replay of the whole path {ms:.1f} ms ({nd * k / (ms * 1e-3):.3g} samples/s), "
        f"every replay bit-identical to the eager run; status per delta "
        f"{[hex(x) for x in ref_status]}")
    # per-kernel times of the sampling, eager, with the chosen launch shape
    tcb.timing_reset()
    tcb.timing_enable(True)
    tcb.tc_batch_estimate(G, Ws, motifs, k, seed, tuning=best, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    tcb.timing_enable(False)
    kernels = {}
    for kname in ("k_paths", "k_listcount_reg", "k_listcount_lds", "k_listcount_wide",
                  "k_listcount_w128", "k_listcount_big"):
        kms, nl = tcb.timing_read(kname)
        if nl:
            kernels[kname] = {"ms_total": kms, "launches": nl, "ms_per_launch": kms / nl}
    tcb.timing_reset()
    log("[bench] sampling kernels (one eager pass): " +
        ", ".join(f"{kn}={v['ms_total']:.1f}ms/{v['launches']}" for kn, v in kernels.items()))
    roofline = None
    kp = kernels.get("k_paths")
    if kp:
        samples_per_launch = nd * k / kp["launches"]
        alg, per = kernel_alg_bytes("k_paths", m, samples_per_launch)
        gbs = alg / (kp["ms_per_launch"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_paths", "alg_bytes_per_unit": per}
    out = {
        "metric": "batched sampled temporal 3-paths/sec (six motifs x four deltas, whole path "
                  "in one graph replay)",
        "value": nd * k / (ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"bitcoin-like batched: n={n} m={m} deltas={deltas} "
                               f"k={k} per delta, six motifs, whole path captured",
                   "n": n, "m": m, "deltas": deltas, "k_per_delta": k,
                   "motifs": sg.SIX_MOTIFS, "seed": seed},
        "tuning": best.as_dict(), "autotune_probe_ms": probe_ms,
        "eager_build_ms": t_build, "eager_weights_ms": t_w,
        "W": {str(d): W.total() for d, W in zip(deltas, Ws)},
        "estimate": {str(d): e for d, e in zip(deltas, ref_est)},
        "overflowed_motifs": {str(d): [sg.SIX_MOTIFS[j] for j in range(nm) if st & (1 << (8 + j))]
                              for d, st in zip(deltas, ref_status)},
        "kernels": kernels, "roofline": roofline,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batched":
        run_batched(args)
        return

    import paper_2409_08975_amd as tcb
    import synthgraph as sg

    stream = torch.cuda.current_stream()

    if args.workload in ("medium", "tiny"):
        extra, g = run_medium_like(args, tcb, sg, args.workload, stream, dev,
                                   with_learned=not args.no_learned and args.workload == "medium")
        P = sg.MEDIUM if args.workload == "medium" else sg.TINY
        k = P["k"]
        out = {"metric": "sampled temporal 3-paths/sec and rel. error vs exact at fixed k; "
                         "learned vs plain",
               "value": extra["samples_per_s"], "unit": "samples/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": extra["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
               "data": "synthetic",
               "config": {"workload": extra["workload"], "n": g.n, "m": g.m,
                          "delta": P["delta"], "k": k, "motifs": sg.SIX_MOTIFS,
                          "seed": P["seed"]},
               "roofline": extra["roofline"]}
        out.update({kk: v for kk, v in extra.items() if kk not in ("workload", "roofline")})
        if not args.no_cpu_baseline:
            th = cpu_threads()
            out["cpu_baseline"] = cpu_baseline(g, [P["delta"]], [sg.MOTIFS[x] for x in
                                                                 sg.SIX_MOTIFS],
                                               k, P["seed"], min(args.cpu_sample, k), th)
            out["cpu_baseline_1thread"] = cpu_one_thread(
                g, P["delta"], [sg.MOTIFS[x] for x in sg.SIX_MOTIFS], k, P["seed"],
                min(args.cpu_sample, k))
        print(json.dumps(out), flush=True)
        return

    # ---- the headline: Bitcoin-like graph, M4-0, two deltas, k = 10^8 each ----
    P = sg.BITCOIN
    t0 = time.time()
    g = sg.gen_bitcoin_like()
    log(f"[bench] generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    deltas, k, seed = [3600, 86400], P["k"], P["seed"]
    names = ["M4-0"]
    motifs = [sg.MOTIFS[x] for x in names]
    if args.profile_run:
        res = run_steps(tcb, g, deltas, motifs, k, seed, 1, 0, stream, dev, "bitcoin profile")
        print(json.dumps({"profile_run": "bitcoin", "ms_per_step": res["ms_per_step"],
                          "weights_calls": 1, "profile_steps": 1}), flush=True)
        return
    res = run_steps(tcb, g, deltas, motifs, k, seed, args.steps, args.warmup, stream, dev,
                    "bitcoin")
    k_total = k * len(deltas)
    kernels = kernel_table(res["ktime"], g.m, k_total, args.steps, "bitcoin", len(deltas))
    G, Ws, outs = res["G"], res["Ws"], res["outs"]
    out = {
        "metric": "sampled temporal 3-paths/sec and rel. error vs exact at fixed k; "
                  "learned vs plain",
        "value": k_total / (res["ms_per_step"] * 1e-3),
        "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"bitcoin-like: n={g.n} m={g.m} deltas={deltas} k={k} per delta "
                               f"motif=M4-0",
                   "n": g.n, "m": g.m, "deltas": deltas, "k_per_delta": k, "motifs": names,
                   "seed": seed},
        "roofline": roofline_of(kernels),
        "stages": stage_table(res, g.m, k_total, "bitcoin"),
        "edge_deltas_per_s_weights": len(deltas) * g.m / (res["weights_ms"] * 1e-3),
        "sample_stage_samples_per_s": k_total / (res["sample_ms"] * 1e-3),
        "W": {str(d): W.total() for d, W in zip(deltas, Ws)},
        "cnt": {str(d): [str(c) for c in o.counts()] for d, o in zip(deltas, outs)},
        "estimate": {str(d): o.estimate.cpu().tolist() for d, o in zip(deltas, outs)},
        "rel_stderr_at_k": rel_stderr(tcb, G, Ws, motifs, names, k, seed),
        "kernels": kernels,
    }
    del G, Ws, outs, res
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out["hbm_probe"] = hbm_probe(dev)
    log(f"[bench] HBM probe: copy {out['hbm_probe']['copy_GBs']:.0f} GB/s, random 8-byte "
        f"gather {out['hbm_probe']['random_gather_words_per_s']:.3g} words/s")
    if not args.no_extras:
        extra, gm = run_medium_like(args, tcb, sg, "medium", stream, dev,
                                    with_learned=not args.no_learned)
        out["medium"] = extra
        del gm
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        th = cpu_threads()
        t0 = time.time()
        out["cpu_baseline"] = cpu_baseline(g, deltas, motifs, k, seed, args.cpu_sample, th)
        log(f"[bench] cpu baseline ({th} threads) in {time.time() - t0:.1f}s: "
            f"{out['cpu_baseline']['value']:.4g} samples/s")
        t0 = time.time()
        out["cpu_baseline_1thread_tiny"] = cpu_one_thread(
            sg.gen_tiny(), sg.TINY["delta"], [sg.MOTIFS["M4-0"]], sg.TINY["k"], sg.TINY["seed"],
            sg.TINY["k"])
        log(f"[bench] one-thread oracle on the tiny workload in {time.time() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
