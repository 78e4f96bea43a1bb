"""Benchmark of the temporal 3-path sampling path on one MI355X.

A step is one pass of the whole hot path over the medium workload (10^6
vertices, 2*10^7 edges, Zipf(2.1) endpoints, bursty timestamps over 30 days,
delta = 86,400 s, six motifs sharing the anchor, k = 10^7 samples):
adjacency build (tc_build_graph), weights and scan (tc_path_weights), and
sampling with closure and reduction (tc_sample_estimate).  The edge arrays are
resident in HBM before the timed region.  `value` is samples per second of the
whole step; per-stage times, edges/s and the roofline of the dominant kernel
are reported beside it, plus the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bfloat16 MFMA
KERNELS = ["k_paths", "k_listcount_reg", "k_windows", "k_scan_apply", "k_radix_scatter"]
# Kernel -> source file whose hash must match the stored counter readings.
KERNEL_SRC = {"k_paths": "tc_sample.hip", "k_listcount_reg": "tc_sample.hip",
              "k_windows": "tc_weights.hip", "k_scan_apply": "tc_weights.hip",
              "k_radix_scatter": "tc_build.hip"}
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_medium.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=["medium", "tiny", "batched"],
                    help="medium: the headline step; batched: six motifs x four deltas on the "
                         "Bitcoin-like graph in one captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--motifs", default="six", choices=["six", "M4-0"],
                    help="motif set of the step (the medium workload uses all six)")
    ap.add_argument("--cpu-sample", type=int, default=10**6,
                    help="samples the oracle draws for the CPU baseline")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal versus method comparison")
    ap.add_argument("--learned-seeds", type=int, default=32)
    ap.add_argument("--k-ref", type=float, default=1e10,
                    help="samples of the reference estimate C_ref")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB device-to-device first (reference for HBM counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, m, units):
    """Algorithmic bytes of one launch: a per-unit figure times the units the
    launch processes.  Data-dependent searches inside adjacency lists and
    pair runs are not counted, so these are lower bounds.
      k_paths          per sample: ceil(log2(m+1)) probes of S (8 B each), the
                       chosen edge with its window metadata (32 B), the two end
                       edges (16 B each)
      k_windows        per edge: read src, dst, t (16 B), write lo_in, a,
                       lo_out, b (16 B)
      k_scan_apply     per edge: read a, b (8 B), write S (8 B)
      k_radix_scatter  per element and pass: read and write a 4-byte key and its
                       12-byte payload {eid, other vertex, t - t_min} (32 B; the
                       record-carrying sorts of a graph whose times span less
                       than 2^32)"""
    if kernel == "k_paths":
        per = 8 * math.ceil(math.log2(m + 1)) + 32 + 2 * 16
    elif kernel == "k_windows":
        per = 32
    elif kernel == "k_scan_apply":
        per = 16
    elif kernel == "k_radix_scatter":
        per = 32
    else:
        return None, None
    return per * units, per


def source_hash(name):
    import hashlib
    with open(os.path.join(ROOT, "paper_2409_08975_amd", "csrc", name), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def stored_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current source of the kernel (else None)."""
    if not os.path.exists(PMC_FILE):
        return None
    want = source_hash(KERNEL_SRC[kernel])
    for line in open(PMC_FILE):
        f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if f.get("kernel") == kernel and f.get("src_sha") == want and "hbm_bytes_per_launch" in f:
            return float(f["hbm_bytes_per_launch"])
    return None


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


def learned_vs_method(tcb, G, Wt, motif, seeds, k_ref, stream):
    """Relative error against C_ref (the method at k_ref samples on its own
    stream) at k = 10^5, 10^6, 10^7 over `seeds` seeds, for the method and
    for the learned proposal (labels on another stream), plus the time of
    each part."""
    from paper_2409_08975_amd import learned
    out = {"motif": "M4-0", "delta": int(Wt.c.delta), "seeds": seeds}
    tcb.timing_reset()
    tcb.timing_enable(True)
    lp = learned.LearnedProposal(G, Wt, motif, seed=11)
    _, out["features_ms"] = event_ms(lambda: tcb.tc_edge_features(G, Wt), stream)
    losses, out["train_ms"] = event_ms(lambda: lp.fit(n_labels=10**6, epochs=8, batch=8192,
                                                      lr=3e-3, label_cap=64.0), stream)
    out["train"] = {"labels": 10**6, "epochs": 8, "batch": 8192, "label_cap": 64.0,
                    "eps": lp.eps, "normalized": lp.normalize,
                    "loss_per_epoch": [round(float(x), 6) for x in losses.cpu().tolist()],
                    "label_rate": lp.label_rate}
    _, out["proposal_ms"] = event_ms(lp.build_proposal, stream)  # inference, h, q-scan
    out["proposal_status"] = lp.proposal.status()
    tcb.timing_enable(False)
    # network kernels: 2 (8*64 + 64*64 + 64) flops per row, both hidden layers on MFMA
    flop_row = 2 * (8 * 64 + 64 * 64 + 64)
    kt = {}
    for name, rows in (("k_mlp_forward", G.m), ("k_mlp_grad", None), ("k_features", G.m)):
        ms, n = tcb.timing_read(name)
        if not n:
            continue
        e = {"ms_per_launch": ms / n, "launches": n}
        if name == "k_mlp_forward":
            tf = flop_row * rows / (ms / n * 1e-3) / 1e12
            e.update({"flop_per_row": flop_row, "rows": rows, "achieved_TFLOPs": tf,
                      "frac_of_bf16_dense_peak": tf / BF16_PEAK_TFLOPS})
        if name == "k_mlp_grad":
            # forward plus backward: about three times the forward flops per row
            e["rows_per_launch"] = 8192
            e["achieved_TFLOPs"] = 3 * flop_row * 8192 / (ms / n * 1e-3) / 1e12
        kt[name] = e
    tcb.timing_reset()
    out["kernels"] = kt
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
    mp, mi = lp.pilot(10**7, 0x5EED)
    out["variance_ratio"] = mp.var / mi.var if mi.var > 0 else None
    rows = []
    for k in (10**5, 10**6, 10**7):
        ep, el, tp, tl = [], [], 0.0, 0.0
        for sd in range(1, seeds + 1):
            r, t = event_ms(lambda: tcb.tc_sample_estimate(G, Wt, [motif], k, sd, stream_id=1),
                            stream)
            ep.append(float(r.estimate[0].item()))
            tp += t
            r, t = event_ms(lambda: tcb.tc_sample_estimate(G, lp.proposal, [motif], k, sd,
                                                           stream_id=2), stream)
            el.append(float(r.estimate[0].item()))
            tl += t
        ep, el = np.array(ep), np.array(el)
        rows.append({"k": k,
                     "rms_rel_err_method": float(np.sqrt(np.mean((ep - C) ** 2)) / C),
                     "rms_rel_err_learned": float(np.sqrt(np.mean((el - C) ** 2)) / C),
                     "ms_per_estimate_method": tp / seeds,
                     "ms_per_estimate_learned": tl / seeds})
    out["by_k"] = rows
    # Equal error: the learned proposal needs k / ratio samples for the error
    # of the method at k.  Its wall time counts features, inference, h and
    # the q-scan (training is reported apart), plus sampling at k / ratio,
    # from the per-sample time measured at each k.
    ratio = out["variance_ratio"]
    if ratio:
        fixed = out["features_ms"] + out["proposal_ms"]
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
        out["equal_error"] = {
            "samples_factor": ratio, "fixed_ms": fixed, "by_k": eq,
            "break_even_k": fixed / (per_m - per_l) if per_m > per_l else None}
    return out


def run_batched(args):
    """Six spine-sharing motifs x delta in {600, 3600, 86400, 604800} on the
    Bitcoin-like graph (5*10^7 vertices, 3*10^8 edges), 10^8 samples per
    delta shared by the six motifs, the whole batched sequence captured once
    in a HIP graph and replayed; launch shape from the autotuner.  Every
    replay is checked bit for bit against an eager call with the default
    launch shape."""
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
    del g
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    motifs = [sg.MOTIFS[x] for x in sg.SIX_MOTIFS]
    deltas, k, seed = P["deltas"], P["k"], P["seed"]
    G, t_build = event_ms(lambda: tcb.tc_build_graph(P["n"], src, dst, tt), stream)
    Ws, t_w = [], []
    for d in deltas:
        W, t = event_ms(lambda: tcb.tc_path_weights(G, d), stream)
        Ws.append(W)
        t_w.append(t)
    log(f"[bench] build {t_build:.1f} ms, weights {', '.join(f'{x:.1f}' for x in t_w)} ms")
    best, probe_ms = tcb.tc_autotune(G, Ws, motifs, 2**22, seed=7)
    log(f"[bench] autotuned {best.as_dict()} ({probe_ms:.2f} ms per 2^22-sample probe)")
    nd, nm = len(deltas), len(motifs)
    ws = torch.empty(tcb.batch_workspace_bytes(k, nd, nm), dtype=torch.uint8, device=dev)
    ref = tcb.tc_batch_estimate(G, Ws, motifs, k, seed, workspace=ws)
    torch.cuda.synchronize()
    ref_counts = [r.counts() for r in ref]
    # per-delta status: a motif whose count reached 2^64 is named by bit 8 + j
    ref_status = [int(r.status.item()) & 0xFFFFFFFF for r in ref]
    if any(st & ~(tcb.TC_F_OVERFLOW | 0xFFFF00) for st in ref_status):
        raise tcb.TCDeviceError(max(ref_status), "batched reference")
    outs = [tcb.new_result(nm, k, dev) for _ in deltas]
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=side):
        tcb.tc_batch_estimate(G, Ws, motifs, k, seed, tuning=best, outs=outs, workspace=ws)
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
    log(f"[bench] replay {ms:.1f} ms ({nd * k / (ms * 1e-3):.3g} samples/s), every replay "
        f"bit-identical to the eager call; status per delta {[hex(x) for x in ref_status]}")
    # per-kernel times of the same work, eager, with the chosen launch shape
    tcb.timing_reset()
    tcb.timing_enable(True)
    tcb.tc_batch_estimate(G, Ws, motifs, k, seed, tuning=best, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    tcb.timing_enable(False)
    kernels = {}
    for kname in ("k_paths", "k_listcount_reg", "k_listcount_lds", "k_listcount_wide",
                  "k_listcount_big"):
        kms, n = tcb.timing_read(kname)
        if n:
            kernels[kname] = {"ms_total": kms, "launches": n, "ms_per_launch": kms / n}
    tcb.timing_reset()
    log("[bench] kernels (one eager pass): " +
        ", ".join(f"{kn}={v['ms_total']:.1f}ms/{v['launches']}" for kn, v in kernels.items()))
    kp = kernels.get("k_paths")
    roofline = None
    if kp:
        samples_per_launch = nd * k / kp["launches"]
        alg, per = algorithmic_bytes("k_paths", G.m, samples_per_launch)
        gbs = alg / (kp["ms_per_launch"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_paths", "alg_bytes_per_unit": per}
    out = {
        "metric": "batched sampled temporal 3-paths/sec (six motifs x four deltas, one graph "
                  "replay)",
        "value": nd * k / (ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"bitcoin-like batched: n={P['n']} m={P['m']} deltas={deltas} "
                               f"k={k} per delta, six motifs", "n": P["n"], "m": P["m"],
                   "deltas": deltas, "k_per_delta": k, "motifs": sg.SIX_MOTIFS, "seed": seed},
        "tuning": best.as_dict(), "autotune_probe_ms": probe_ms,
        "build_ms": t_build, "weights_ms": dict(zip(map(str, deltas), t_w)),
        "edges_per_s_weights": {str(d): G.m / (t * 1e-3) for d, t in zip(deltas, t_w)},
        "W": {str(d): W.total() for d, W in zip(deltas, Ws)},
        "estimate": {str(d): o.estimate.cpu().tolist() for d, o in zip(deltas, outs)},
        "overflowed_motifs": {str(d): [sg.SIX_MOTIFS[j] for j in range(nm) if st & (1 << (8 + j))]
                              for d, st in zip(deltas, ref_status)},
        "kernels": kernels, "roofline": roofline,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload == "batched":
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                              "n_gpus": args.gpus}), flush=True)
            sys.exit(2)
        run_batched(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import paper_2409_08975_amd as tcb
    import synthgraph as sg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "medium":
        P = sg.MEDIUM
        t0 = time.time()
        g = sg.gen_medium()
    else:
        P = sg.TINY
        t0 = time.time()
        g = sg.gen_tiny()
    log(f"[bench] generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    delta, k, seed = P["delta"], P["k"], P["seed"]
    names = sg.SIX_MOTIFS if (args.workload == "medium" and args.motifs == "six") else ["M4-0"]
    motifs = [sg.MOTIFS[x] for x in names]
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    tt = torch.from_numpy(g.t).to(dev)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        G = tcb.tc_build_graph(g.n, src, dst, tt)
        ev[1].record(stream)
        W = tcb.tc_path_weights(G, delta)
        ev[2].record(stream)
        R = tcb.tc_sample_estimate(G, W, motifs, k, seed)
        ev[3].record(stream)
        return G, W, R, ev

    for i in range(args.warmup):
        G, W, R, ev = step()
        torch.cuda.synchronize()
        R.check()
        log(f"[bench] warmup {i} done")
    torch.cuda.synchronize()
    tcb.timing_reset()
    tcb.timing_enable(True)
    stage = np.zeros(3)
    t_start = time.perf_counter()
    evs = []
    for i in range(args.steps):
        G, W, R, ev = step()
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
    for ev in evs:
        for s in range(3):
            stage[s] += ev[s].elapsed_time(ev[s + 1])
    stage /= args.steps
    R.check()
    ms_per_step = t_total * 1000.0 / args.steps
    Wtot = W.total()
    counts = R.counts()
    est = R.estimate.cpu().tolist()
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step; stages ms "
        f"build={stage[0]:.3f} weights={stage[1]:.3f} sample={stage[2]:.3f}")

    # per-kernel rooflines; the dominant kernel is the one with the most time per step
    units = {"k_paths": None, "k_windows": g.m, "k_scan_apply": g.m, "k_radix_scatter": g.m}
    kernels = {}
    for kname, (ms, n) in ktime.items():
        per_launch_ms = ms / n
        u = units.get(kname)
        if kname == "k_paths":
            u = k / (n / args.steps)  # samples per launch (chunks of the k samples)
        alg, per = algorithmic_bytes(kname, g.m, u) if u is not None else (None, None)
        entry = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                 "ms_per_launch": per_launch_ms}
        if alg is not None:
            gbs = alg / (per_launch_ms * 1e-3) / 1e9
            entry.update({"alg_bytes_per_unit": per, "alg_bytes_per_launch": alg,
                          "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS})
            tr = stored_traffic(kname)
            entry["hbm_bytes_per_launch"] = tr
        kernels[kname] = entry
    dom = max(kernels, key=lambda x: kernels[x]["ms_per_step"])
    d = kernels[dom]
    roofline = {"bound": "hbm", "achieved": round(d.get("achieved_GBs", 0.0), 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d.get("frac_of_hbm_peak", 0.0), 4),
                "traffic": d.get("hbm_bytes_per_launch"), "kernel": dom,
                "ms_per_launch": round(d["ms_per_launch"], 4),
                "alg_bytes_per_unit": d.get("alg_bytes_per_unit")}
    if roofline["traffic"]:
        # the HBM bytes the kernel actually moves (counters) over the live
        # launch time: how busy the memory system is, beside the algorithmic
        # fraction above
        tgbs = roofline["traffic"] / (d["ms_per_launch"] * 1e-3) / 1e9
        roofline["traffic_GBs"] = round(tgbs, 1)
        roofline["traffic_frac"] = round(tgbs / HBM_PEAK_GBS, 4)
    log(f"[bench] kernels: " + ", ".join(f"{k_}={v['ms_per_step']:.3f}ms" for k_, v in kernels.items()))

    out = {
        "metric": "sampled temporal 3-paths/sec and rel. error vs exact at fixed k; learned vs plain",
        "value": k / (ms_per_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{g.name}: n={g.n} m={g.m} delta={delta} k={k} "
                               f"motifs={','.join(names)}",
                   "n": g.n, "m": g.m, "delta": delta, "k": k, "motifs": names, "seed": seed},
        "stages_ms": {"build": stage[0], "weights": stage[1], "sample": stage[2]},
        "edges_per_s": g.m / (stage[1] * 1e-3),
        "sample_stage_samples_per_s": k / (stage[2] * 1e-3),
        "W": Wtot,
        "cnt": [str(c) for c in counts],
        "estimate": est,
        "roofline": roofline,
        "kernels": kernels,
    }

    # relative standard error of each motif's estimate at this k (second moment run)
    Rm = tcb.tc_sample_estimate(G, W, motifs, k, seed, moments=True)
    Rm.check("moments")
    from paper_2409_08975_amd import learned as _learned
    rse = []
    for j in range(len(motifs)):
        mm = _learned.moments(Rm, W, k, j)
        rse.append(mm.stderr / mm.estimate if mm.estimate else None)
    out["rel_stderr_at_k"] = dict(zip(names, rse))

    if not args.no_learned and args.workload == "medium":
        t0 = time.time()
        out["learned_vs_method"] = learned_vs_method(tcb, G, W, sg.MOTIFS["M4-0"],
                                                     args.learned_seeds, args.k_ref, stream)
        log(f"[bench] learned vs method in {time.time() - t0:.1f}s: variance ratio "
            f"{out['learned_vs_method']['variance_ratio']}")

    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.default_threads()
        kc = min(args.cpu_sample, k)
        t0 = time.perf_counter()
        og = oracle.OracleGraph.from_graph(g)
        t_b = time.perf_counter() - t0
        t0 = time.perf_counter()
        ow = og.weights(delta, threads=threads)
        t_w = time.perf_counter() - t0
        t0 = time.perf_counter()
        E = og.sample(ow, [sg.motif_bytes(M) for M in motifs], kc, seed, threads=threads)
        t_s = time.perf_counter() - t0
        t_full = t_b + t_w + t_s * (k / kc)
        out["cpu_baseline"] = {
            "value": k / t_full, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"full build ({t_b:.2f}s, 1 thread) and weights ({t_w:.2f}s) of the "
                      f"same graph, {kc} of the {k} samples ({t_s:.2f}s), sampling time "
                      f"scaled by {k / kc:.0f}",
        }
        if E.cnt[:1] and kc == k:
            out["cpu_baseline"]["cnt_match"] = E.cnt == counts
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
