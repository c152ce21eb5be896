"""Short text summaries of rocprofv3 output (CSV format, ``-f csv``).

  python -m paper_1310_6380_amd.profile_summary stats DIR --cmd "..."
      per-kernel table of a ``--kernel-trace --stats`` run (calls, total and
      average duration, share of the GPU time);
  python -m paper_1310_6380_amd.profile_summary traffic --fetch DIR --write DIR
         --copy-fetch DIR --copy-write DIR --copy-bytes B --cmd "..."
      HBM bytes per dispatch of every kernel from two ``--pmc`` runs
      (FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch), each scaled by
      what the same counter reads for the library's plain copy kernel (copy16)
      moving B bytes each way.
  python -m paper_1310_6380_amd.profile_summary mfma DIR --cmd "..."
      matrix-core figures per kernel from one ``--pmc
      SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_BF16
      SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE --kernel-trace`` run: matrix-core
      flops per dispatch (512 per MOP) and their rate over the traced
      duration against the dense peak of the type (the busy-cycle counter is
      collected but not reported: its normalisation per SIMD is not
      established on this part).

Both print Markdown on stdout.  Each traffic row carries the digest of the
source file of its kernel (and the shared headers) it was taken on; figures
for other sources are stale.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


SHARED_HEADERS = ("common.h", "kernels.h")
# kernel families timed as one launch -> a kernel of the family
FAMILY = {"backtransform": "backtransform_2s", "tridiag_eig": "tridiag_invit", "rayleigh_ritz": "rr_product",
          "potrf_trtri": "potrf_diag", "zgemm": "zgemm_kernel", "structure_factors": "sf_mfma_pass_a",
          "combine_coefficients": "combine_coefficients"}


def kernel_source(name: str):
    """The HIP source file that defines kernel `name` (or a kernel of that family)."""
    name = FAMILY.get(name, name)
    csrc = os.path.join(HERE, "csrc")
    pat = re.compile(r"__global__[^;{]*?\b" + re.escape(name) + r"\s*\(", re.S)
    for f in sorted(os.listdir(csrc)):
        if f.endswith(".hip"):
            with open(os.path.join(csrc, f)) as fh:
                if pat.search(fh.read()):
                    return f
    return None


def source_digest(name: str) -> str:
    """SHA-256 of the file defining the kernel and of the shared headers: counter
    figures taken on other sources of that kernel do not apply."""
    f = kernel_source(name)
    if f is None:
        return "unknown"
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for g in (f,) + SHARED_HEADERS:
        with open(os.path.join(csrc, g), "rb") as fh:
            h.update(g.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def base_name(kernel: str) -> str:
    """'void mvpb::hb2st<double>(mvpb::EigItem const*, int)' -> 'hb2st'."""
    k = kernel.split("(")[0]
    k = re.sub(r"<.*>", "", k)
    k = k.split()[-1] if k.split() else k
    return k.split("::")[-1]


def _find(dirpath: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {dirpath}")
    return hits[0]


def _col(header, *names):
    low = [h.lower() for h in header]
    for n in names:
        if n.lower() in low:
            return low.index(n.lower())
    raise SystemExit(f"none of the columns {names} in {header}")


def read_stats(dirpath: str):
    with open(_find(dirpath, "kernel_stats.csv")) as fh:
        rows = list(csv.reader(fh))
    h = rows[0]
    cn, cc = _col(h, "Name", "KernelName"), _col(h, "Calls")
    ct, ca = _col(h, "TotalDurationNs"), _col(h, "AverageNs")
    out = [(r[cn], int(r[cc]), float(r[ct]), float(r[ca])) for r in rows[1:] if r]
    return sorted(out, key=lambda t: -t[2])


def read_counters(dirpath: str, counter: str, reduce=None):
    """{kernel base name: [value per dispatch]} of one counter (rows of a
    dispatch summed, or combined by ``reduce``)."""
    with open(_find(dirpath, "counter_collection.csv")) as fh:
        rows = list(csv.reader(fh))
    h = rows[0]
    cd = _col(h, "Dispatch_Id", "Dispatch-Id", "dispatch_id")
    ck = _col(h, "Kernel_Name", "Kernel-Name", "kernel_name")
    cc = _col(h, "Counter_Name", "Counter-Name", "counter_name")
    cv = _col(h, "Counter_Value", "Counter-Value", "counter_value")
    per = {}
    names = {}
    for r in rows[1:]:
        if not r or r[cc] != counter:
            continue
        v = float(r[cv])
        d = r[cd]
        per[d] = v if d not in per else (reduce(per[d], v) if reduce else per[d] + v)
        names[d] = base_name(r[ck])
    out = collections.defaultdict(list)
    for d, v in per.items():
        out[names[d]].append(v)
    return out


def cmd_stats(a):
    st = read_stats(a.dir)
    tot = sum(t[2] for t in st) or 1.0
    print(f"# {a.title}\n")
    print(f"command: `{a.cmd}`\n")
    print("| kernel | calls | total ms | avg us | share |")
    print("|---|---:|---:|---:|---:|")
    for name, calls, total, avg in st[: a.top]:
        print(f"| {base_name(name)} | {calls} | {total / 1e6:.3f} | {avg / 1e3:.1f} | {100 * total / tot:.1f}% |")
    print(f"\nall kernels: {tot / 1e6:.3f} ms")


def cmd_traffic(a):
    fetch = read_counters(a.fetch, "FETCH_SIZE")
    write = read_counters(a.write, "WRITE_SIZE")
    cf = read_counters(a.copy_fetch, "FETCH_SIZE").get("copy16")
    cw = read_counters(a.copy_write, "WRITE_SIZE").get("copy16")
    if not cf or not cw:
        raise SystemExit("no copy16 dispatch in the calibration runs")
    kib = a.copy_bytes / 1024.0
    f_fetch = kib / (sum(cf) / len(cf))
    f_write = kib / (sum(cw) / len(cw))
    print(f"# {a.title}\n")
    print(f"command (FETCH_SIZE pass): `{a.cmd_fetch}`\n")
    print(f"command (WRITE_SIZE pass): `{a.cmd_write}`\n")
    print(f"calibration: `{a.cmd_copy}` (copy16 moving {a.copy_bytes} bytes each way; "
          f"FETCH_SIZE {sum(cf) / len(cf):.1f} KiB, WRITE_SIZE {sum(cw) / len(cw):.1f} KiB per dispatch)\n")
    print(f"scale factors: fetch {f_fetch:.4f}, write {f_write:.4f}\n")
    print("| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | calibrated bytes/dispatch "
          "| source digest |")
    print("|---|---:|---:|---:|---:|---|")
    rows = {}
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, []), write.get(k, [])
        fa = sum(fv) / len(fv) if fv else 0.0
        wa = sum(wv) / len(wv) if wv else 0.0
        rows[k] = (max(len(fv), len(wv)), fa, wa, 1024.0 * (fa * f_fetch + wa * f_write))
    # the two back-transform kernels are timed as one launch
    if "backtransform_2s" in rows and "backtransform_s1" in rows:
        a2, a1 = rows["backtransform_2s"], rows["backtransform_s1"]
        rows["backtransform"] = (a2[0], a2[1] + a1[1], a2[2] + a1[2], a2[3] + a1[3])
    for k, (nd, fa, wa, b) in sorted(rows.items(), key=lambda kv: -kv[1][3] * kv[1][0]):
        print(f"| {k} | {nd} | {fa:.1f} | {wa:.1f} | {b:.0f} | {source_digest(k)} |")


def read_durations(dirpath: str):
    """{dispatch id: (kernel base name, duration ns)} from a kernel trace."""
    with open(_find(dirpath, "kernel_trace.csv")) as fh:
        rows = list(csv.reader(fh))
    h = rows[0]
    cd = _col(h, "Dispatch_Id", "Dispatch-Id", "dispatch_id")
    ck = _col(h, "Kernel_Name", "Kernel-Name", "kernel_name")
    cs, ce = _col(h, "Start_Timestamp", "Start-Timestamp"), _col(h, "End_Timestamp", "End-Timestamp")
    return {r[cd]: (base_name(r[ck]), float(r[ce]) - float(r[cs])) for r in rows[1:] if r}


def cmd_mfma(a):
    dur = read_durations(a.dir)
    with open(_find(a.dir, "counter_collection.csv")) as fh:
        rows = list(csv.reader(fh))
    h = rows[0]
    cd, cc, cv = (_col(h, "Dispatch_Id", "Dispatch-Id", "dispatch_id"), _col(h, "Counter_Name", "Counter-Name"),
                  _col(h, "Counter_Value", "Counter-Value"))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for r in rows[1:]:
        if not r:
            continue
        v = float(r[cv])
        d = per[r[cd]]
        if r[cc] == "GRBM_GUI_ACTIVE":
            d[r[cc]] = max(d[r[cc]], v)
        else:
            d[r[cc]] += v
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    for d, cnt in per.items():
        if d not in dur:
            continue
        name, ns = dur[d]
        g = agg[name]
        g["n"] += 1
        g["ns"] += ns
        for k, v in cnt.items():
            g[k] += v
    print(f"# {a.title}\n")
    print(f"command: `{a.cmd}`\n")
    print("| kernel | dispatches | avg us | FP64 MFMA GFLOP/dispatch | FP64 TFLOP/s (of 78.6) | "
          "BF16 MFMA GFLOP/dispatch | BF16 TFLOP/s (of 2500) | source digest |")
    print("|---|---:|---:|---:|---:|---:|---:|---|")
    order = sorted(agg.items(), key=lambda kv: -kv[1]["ns"])
    for name, g in order[: a.top]:
        n = g["n"]
        f64 = 512.0 * g["SQ_INSTS_VALU_MFMA_MOPS_F64"] / n
        b16 = 512.0 * g["SQ_INSTS_VALU_MFMA_MOPS_BF16"] / n
        us = g["ns"] / n / 1e3
        print(f"| {name} | {int(n)} | {us:.1f} | {f64 / 1e9:.4f} | {f64 / (us * 1e6) if us else 0:.2f} | "
              f"{b16 / 1e9:.4f} | {b16 / (us * 1e6) if us else 0:.2f} | {source_digest(name)} |")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--top", type=int, default=30)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--cmd-copy", required=True)
    t.add_argument("--title", default="HBM traffic per dispatch")
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("--cmd", required=True)
    m.add_argument("--title", default="matrix-core counters per dispatch")
    m.add_argument("--top", type=int, default=30)
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "traffic": cmd_traffic, "mfma": cmd_mfma}[a.what](a)


if __name__ == "__main__":
    main(sys.argv[1:])
