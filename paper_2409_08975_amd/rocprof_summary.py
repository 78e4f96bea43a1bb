"""Short text summaries of rocprofv3 runs of ``bench.py`` (kernel durations and
HBM traffic per kernel), written for the ``profiles/`` folder.

  python -m paper_2409_08975_amd.rocprof_summary stats <run_results.db> <out.txt> <command>
  python -m paper_2409_08975_amd.rocprof_summary pmc <fetch.db> <write.db> <out.txt> <fetch cmd> <write cmd> [meta]

The traffic summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by
what the same counters read for a 1 GiB device-to-device copy recorded in
the same run (bench.py --calib-copy), and tags each kernel with a hash of its
source file so a reader can tell whether the figures still describe the code.
Launches that moved less than 64 KiB (time-sort passes that the device plan
leaves idle) are left out of the per-launch averages; the totals count every
launch.  `meta` (key=value words) describes the profiled run, e.g. how many
steps it timed.
"""
from __future__ import annotations

import collections
import hashlib
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_08975_amd", "csrc")
CALIB_BYTES = 1 << 30

# kernel base name -> source file holding it
KERNEL_SRC = {
    "k_paths": "tc_sample.hip", "k_listcount_reg": "tc_sample.hip",
    "k_listcount_lds": "tc_sample.hip", "k_listcount_wide": "tc_sample.hip",
    "k_listcount_big": "tc_sample.hip", "k_listcount_w128": "tc_sample.hip",
    "k_windows": "tc_weights.hip", "k_mp_rank": "tc_weights.hip", "k_combine": "tc_weights.hip",
    "k_scan_tiles": "tc_weights.hip", "k_scan_tiles_sets": "tc_weights.hip", "k_scan_apply": "tc_weights.hip",
    "k_radix_scatter": "tc_build.hip",
    "k_radix_hist": "tc_build.hip", "k_hash_insert": "tc_build.hip", "k_emit": "tc_build.hip",
    "k_offsets": "tc_build.hip",
    "k_rec_xform": "tc_build.hip", "k_mp_split": "tc_weights.hip",
    "k_mp_split_coarse": "tc_weights.hip", "k_rec_init": "tc_build.hip",
    "k_col_sum": "tc_build.hip", "k_col_scan": "tc_build.hip", "k_col_apply": "tc_build.hip",
    "k_hash_clear": "tc_build.hip", "k_validate": "tc_build.hip", "k_plan": "tc_build.hip",
    "k_fold_hist": "tc_build.hip",
    "k_init_build": "tc_build.hip", "k_trange": "tc_build.hip",
    "k_zero_result": "tc_sample.hip", "k_store_ptrs": "tc_sample.hip",
    "k_zero_counters": "tc_sample.hip", "k_finalize": "tc_sample.hip",
}
IDLE_BYTES = 64 * 1024


def short_name(n: str) -> str:
    n = n.split("(")[0].replace("void ", "").replace("tc::", "")
    return n.strip()


def base_name(n: str) -> str:
    return short_name(n).split("<")[0]


def source_sha(kernel: str):
    f = KERNEL_SRC.get(base_name(kernel))
    if f is None:
        return None
    with open(os.path.join(CSRC, f), "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()[:12]


def kernel_durations(db: str):
    """{kernel: [calls, total_us, min_us, max_us]} from a rocpd kernel trace."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    ni = cols.index("name") if "name" in cols else cols.index("kernel_name")
    si, ei = cols.index("start"), cols.index("end")
    agg = {}
    for r in cur.execute("select * from kernels"):
        d = (r[ei] - r[si]) / 1e3
        a = agg.setdefault(short_name(r[ni]), [0, 0.0, 1e30, 0.0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    con.close()
    return agg


def stats_text(db: str, command: str, top: int = 30) -> str:
    agg = kernel_durations(db)
    tot = sum(a[1] for a in agg.values()) or 1.0
    lines = [f"# rocprofv3 kernel trace summary", f"# command: {command}",
             f"# {'kernel':58s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} "
             f"{'min_us':>10s} {'max_us':>10s} {'%':>6s}"]
    for n, a in sorted(agg.items(), key=lambda x: -x[1][1])[:top]:
        lines.append(f"  {n[:58]:58s} {a[0]:6d} {a[1]:11.1f} {a[1] / a[0]:10.1f} {a[2]:10.1f} "
                     f"{a[3]:10.1f} {100 * a[1] / tot:6.2f}")
    return "\n".join(lines) + "\n"


def _counter_rows(db: str, counter: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name=?",
                       (counter,)).fetchall()
    con.close()
    return rows


def pmc_text(fetch_db: str, write_db: str, fetch_cmd: str, write_cmd: str, meta: str = "") -> str:
    fetch = _counter_rows(fetch_db, "FETCH_SIZE")
    write = _counter_rows(write_db, "WRITE_SIZE")
    fc = [v for n, v in fetch if "copyBuffer" in n and v * 1024 > CALIB_BYTES / 4]
    wc = [v for n, v in write if "copyBuffer" in n and v * 1024 > CALIB_BYTES / 4]
    if not fc or not wc:
        raise SystemExit("no 1 GiB calibration copy in the counter runs (bench.py --calib-copy)")
    ff = CALIB_BYTES / (fc[0] * 1024.0)
    wf = CALIB_BYTES / (wc[0] * 1024.0)
    # the two runs launch the same kernels in the same order: pair them up
    per = collections.OrderedDict()
    for rows, key, fac in ((fetch, "f", ff), (write, "w", wf)):
        cnt = collections.Counter()
        for n, v in rows:
            sn = short_name(n)
            lst = per.setdefault(sn, [])
            i = cnt[sn]
            cnt[sn] += 1
            while len(lst) <= i:
                lst.append({"f": 0.0, "w": 0.0})
            lst[i][key] = v * 1024.0 * fac
    lines = ["# HBM traffic per kernel launch from rocprofv3 counters",
             f"# fetch run: {fetch_cmd}", f"# write run: {write_cmd}",
             f"# calibration: 1 GiB device copy reads FETCH_SIZE={fc[0]:.0f} KiB "
             f"(factor {ff:.4f}) and WRITE_SIZE={wc[0]:.0f} KiB (factor {wf:.4f})",
             "# per launch: average over launches that moved at least 64 KiB; total: every "
             "launch of the run",
             f"# {'kernel':44s} {'launches':>8s} {'active':>6s} {'read MB':>10s} {'write MB':>10s}"
             f" {'total MB':>10s}"]
    keyed = []
    for n, lst in per.items():
        if "copyBuffer" in n:
            continue
        act = [x for x in lst if x["f"] + x["w"] >= IDLE_BYTES]
        rf = sum(x["f"] for x in act) / max(1, len(act))
        rw = sum(x["w"] for x in act) / max(1, len(act))
        tot = sum(x["f"] + x["w"] for x in lst)
        lines.append(f"  {n[:44]:44s} {len(lst):8d} {len(act):6d} {rf / 1e6:10.2f} "
                     f"{rw / 1e6:10.2f} {tot / 1e6:10.2f}")
        sha = source_sha(n)
        if sha is not None:
            keyed.append((base_name(n), sha, rf, rw, tot, len(lst), len(act)))
    # one keyed line per kernel base name (instantiations summed)
    merged = collections.OrderedDict()
    for b, sha, rf, rw, tot, nl, na in keyed:
        if b not in merged:
            merged[b] = [sha, rf * na, rw * na, tot, nl, na]
        else:
            e = merged[b]
            e[1] += rf * na
            e[2] += rw * na
            e[3] += tot
            e[4] += nl
            e[5] += na
    out = []
    if meta:
        out.append("meta " + meta)
    for b, (sha, rfa, rwa, tot, nl, na) in merged.items():
        na1 = max(1, na)
        out.append(f"kernel={b} src_sha={sha} hbm_bytes_per_launch={(rfa + rwa) / na1:.0f} "
                   f"read_bytes_per_launch={rfa / na1:.0f} write_bytes_per_launch={rwa / na1:.0f} "
                   f"launches={nl} active_launches={na} total_bytes={tot:.0f}")
    return "\n".join(lines) + "\n\n" + "\n".join(out) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        text = stats_text(argv[1], argv[3])
        with open(argv[2], "w") as f:
            f.write(text)
    elif len(argv) >= 6 and argv[0] == "pmc":
        text = pmc_text(argv[1], argv[2], argv[4], argv[5], argv[6] if len(argv) > 6 else "")
        with open(argv[3], "w") as f:
            f.write(text)
    else:
        raise SystemExit(__doc__)
    print(text)


if __name__ == "__main__":
    main(sys.argv[1:])
