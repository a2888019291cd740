"""Per-kernel summary of rocprofv3 runs of ``bench.py`` for one encrypted CutMax call
(one request, or the 16-request batch of ``--batch-only``).

Inputs are rocprofv3 output directories written with ``--output-format csv`` (the
``*_kernel_trace.csv`` / ``*_counter_collection.csv`` pair):

* ``--trace DIR``: a ``--kernel-trace --stats`` run (durations);
* ``--fetch DIR`` / ``--write DIR``: ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` runs;
* ``--valu DIR``: a run with SQ_INSTS_VALU, SQ_INSTS_VALU_{FMA,MUL,ADD}_F64, GRBM_GUI_ACTIVE;
* ``--lds DIR``: a run with SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT, SQ_LDS_IDX_ACTIVE;
* ``--tex DIR``: a run with TA_TA_BUSY and TD_TD_BUSY (the texture address and data
  units of the vector memory path, one of each per CU);
* ``--bench-json FILE``: bench.py's JSON line with the event profiler's algorithmic
  bytes per kernel and the digest of the library sources that ran;
* ``--per-launch NAME`` (with ``--trace``): instead of the table, every dispatch of the
  kernel class NAME in the timed call, in launch order, with its template instance and
  duration.

The dispatches of the timed CutMax are the second half of those between the last
encryption kernel (k_encfinish) and the first decryption kernel (k_decmul): the bench
runs one warm-up CutMax and one timed CutMax on the same ciphertext, so both halves
launch the same kernel sequence (checked).

Byte counters are calibrated with the bench's plain copy of 64 limb vectors (the
k_copy dispatches with grid 65536 x 64, 32 MiB read and 32 MiB written each): the
scale of each counter is known bytes / counter value.  VALU utilisation is
SQ_INSTS_VALU / (256 CUs x kernel cycles at 2.4 GHz): every CU retires at most one
wave64 VALU instruction per cycle (4 SIMDs, 4 cycles each), FP64 included.  The busy
fractions of the texture units are their busy-cycle counts summed over the 256 CUs,
divided by 256 x kernel cycles.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
from collections import OrderedDict, defaultdict

CLOCK_HZ = 2.4e9
CUS = 256
HBM_PEAK = 8.0e12


def _one(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_class(name: str) -> str:
    """Library-level name of a dispatch (the NTT template arguments spelled out)."""
    m = re.search(r"k_ntt<(\d+), (\d+), (true|false), (true|false), (\d+), (\d+)(?:, (\d+))?>", name)
    if m:
        p2, inv, pro, epi = m.group(3) == "true", m.group(4) == "true", int(m.group(5)), int(m.group(6))
        s = "ntt_" + ("inv" if inv else "fwd") + ("_pass2" if p2 else "_pass1")
        s += {1: "_lift", 2: "_tensor"}.get(pro, "") + {1: "_moddown", 2: "_rescale", 3: "_moddown_rescale",
                                          4: "_moddown_chain"}.get(epi, "")
        if m.group(7) and int(m.group(7)):
            s += "_factored"
        return s
    base = re.sub(r"\(.*", "", name)
    base = re.sub(r"^void ", "", base)
    base = re.sub(r"<.*", "", base.split("::")[-1])
    # the batched and LDS-staged rotation key products book under the same name
    return "k_inner_product_rot" if base in ("k_inner_product_rot_reg", "k_inner_product_rot_lds") else base


def _trace(d: str):
    rows = list(csv.DictReader(open(_one(d, "kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _counters(d: str):
    out = defaultdict(dict)
    for r in csv.DictReader(open(_one(d, "counter_collection.csv"))):
        out[int(r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def cutmax_window(rows):
    names = [kernel_class(r["Kernel_Name"]) for r in rows]
    enc = max(i for i, n in enumerate(names) if n == "k_encfinish")
    dec = min(i for i, n in enumerate(names) if n == "k_decmul" and i > enc)
    span = rows[enc + 1:dec]
    half = len(span) // 2
    a, b = span[:half], span[half:]
    if len(a) != len(b) or [kernel_class(r["Kernel_Name"]) for r in a] != \
            [kernel_class(r["Kernel_Name"]) for r in b]:
        raise RuntimeError("warm-up and timed CutMax launch different kernel sequences")
    return b


def copy_dispatches(rows):
    return [r for r in rows if kernel_class(r["Kernel_Name"]) == "k_copy" and r.get("Grid_Size_Y") == "64"
            and r.get("Grid_Size_X") == "65536"]


def summarize(trace=None, fetch=None, write=None, valu=None, lds=None, bench_json=None, tex=None):
    base = trace or fetch or write or valu or lds or tex
    rows = _trace(base)
    win = cutmax_window(rows)
    dur = {}
    for r in win:
        dur[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    order = OrderedDict()
    for r in win:
        order.setdefault(kernel_class(r["Kernel_Name"]), []).append(int(r["Dispatch_Id"]))

    def per_pass(d, counter, known_bytes):
        """(window dispatch id -> calibrated bytes, scale), matched by position within the window."""
        if not d:
            return None, None
        prow = _trace(d)
        pwin = cutmax_window(prow)
        cnt = _counters(d)
        cal = [cnt[int(r["Dispatch_Id"])][counter] for r in copy_dispatches(prow)]
        scale = known_bytes / (sum(cal) / len(cal))
        vals = {int(w["Dispatch_Id"]): cnt[int(p["Dispatch_Id"])][counter] * scale for w, p in zip(win, pwin)}
        return vals, scale

    copy_bytes = 64 * 65536 * 8
    fvals, fscale = per_pass(fetch, "FETCH_SIZE", copy_bytes)
    wvals, wscale = per_pass(write, "WRITE_SIZE", copy_bytes)

    def raw(d, counters):
        if not d:
            return None
        prow = _trace(d)
        pwin = cutmax_window(prow)
        cnt = _counters(d)
        return {int(w["Dispatch_Id"]): {c: cnt[int(p["Dispatch_Id"])].get(c, 0.0) for c in counters}
                for w, p in zip(win, pwin)}

    vv = raw(valu, ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
                    "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_TRANS_F64"])
    ll = raw(lds, ["SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE"])
    tx = raw(tex, ["TA_TA_BUSY", "TD_TD_BUSY"])
    alg = {}
    digest = None
    if bench_json:
        # the default line ({"metric": ...}) books the single CutMax's kernels; a --batch-only
        # line ({"batched": ...}) books the batch's
        lines = [ln for ln in open(bench_json).read().splitlines()
                 if ln.startswith('{"metric"') or ln.startswith('{"batched"')]
        bj = json.loads(lines[-1])
        digest = bj.get("src_digest")
        kern = bj.get("kernels") or (bj.get("batched") or {}).get("kernels") or {}
        for k, v in kern.items():
            alg[k] = v["bytes"] / v["launches"] if v["launches"] else 0.0

    total = sum(dur.values())
    res = []
    for name, ids in order.items():
        n = len(ids)
        t = sum(dur[i] for i in ids)
        e = {"kernel": name, "launches": n, "total_ms": t * 1e3, "avg_us": t / n * 1e6, "share": t / total}
        if fvals:
            e["fetch_MiB"] = sum(fvals[i] for i in ids) / n / 2**20
        if wvals:
            e["write_MiB"] = sum(wvals[i] for i in ids) / n / 2**20
        if fvals and wvals:
            e["hbm_GBps"] = sum(fvals[i] + wvals[i] for i in ids) / t / 1e9
        if name in alg:
            e["alg_MiB"] = alg[name] / 2**20
        if vv:
            ins = sum(vv[i]["SQ_INSTS_VALU"] for i in ids)
            e["valu_util"] = ins / (CUS * t * CLOCK_HZ)
            f64 = sum(vv[i]["SQ_INSTS_VALU_FMA_F64"] + vv[i]["SQ_INSTS_VALU_MUL_F64"] + vv[i]["SQ_INSTS_VALU_ADD_F64"]
                      for i in ids)
            e["f64_share"] = f64 / ins if ins else 0.0
            e["int32_share"] = sum(vv[i]["SQ_INSTS_VALU_INT32"] for i in ids) / ins if ins else 0.0
        if ll:
            act = sum(ll[i]["SQ_LDS_IDX_ACTIVE"] for i in ids)
            e["lds_conflict"] = sum(ll[i]["SQ_LDS_BANK_CONFLICT"] for i in ids) / act if act else 0.0
        if tx:
            e["ta_busy"] = sum(tx[i]["TA_TA_BUSY"] for i in ids) / (CUS * t * CLOCK_HZ)
            e["td_busy"] = sum(tx[i]["TD_TD_BUSY"] for i in ids) / (CUS * t * CLOCK_HZ)
        res.append(e)
    res.sort(key=lambda e: -e["total_ms"])
    return {"dispatches": len(win), "total_ms": total * 1e3, "fetch_scale": fscale, "write_scale": wscale,
            "src_digest": digest, "kernels": res}


def per_launch(trace: str, name: str):
    """[(template instance, grid x, microseconds)] of the class' dispatches in the timed call"""
    out = []
    for r in cutmax_window(_trace(trace)):
        if kernel_class(r["Kernel_Name"]) != name:
            continue
        inst = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("he::", "")
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        out.append((inst, r.get("Grid_Size_X", ""), us))
    return out


def to_markdown(s) -> str:
    cols = [("kernel", "{}"), ("launches", "{}"), ("total_ms", "{:.3f}"), ("avg_us", "{:.1f}"), ("share", "{:.1%}"),
            ("alg_MiB", "{:.1f}"), ("fetch_MiB", "{:.1f}"), ("write_MiB", "{:.1f}"), ("hbm_GBps", "{:.0f}"),
            ("valu_util", "{:.1%}"), ("f64_share", "{:.0%}"), ("int32_share", "{:.0%}"), ("lds_conflict", "{:.1%}"),
            ("ta_busy", "{:.0%}"), ("td_busy", "{:.0%}")]
    present = [c for c in cols if any(c[0] in e for e in s["kernels"])]
    out = ["| " + " | ".join(c[0] for c in present) + " |", "|" + "---|" * len(present)]
    for e in s["kernels"]:
        out.append("| " + " | ".join(fmt.format(e[c]) if c in e else "" for c, fmt in present) + " |")
    hdr = [f"dispatches in one timed call: {s['dispatches']}, kernel time {s['total_ms']:.3f} ms"]
    if s["fetch_scale"]:
        hdr.append(f"FETCH_SIZE calibration (plain copy of known size): x{s['fetch_scale'] / 1024:.4f} "
                   f"(bytes per counted KiB / 1024)")
    if s["write_scale"]:
        hdr.append(f"WRITE_SIZE calibration: x{s['write_scale'] / 1024:.4f}")
    return "\n".join(hdr) + "\n\n" + "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    for k in ("trace", "fetch", "write", "valu", "lds", "tex"):
        ap.add_argument("--" + k)
    ap.add_argument("--bench-json", help="a file holding bench.py's JSON line (algorithmic bytes, "
                    "source digest); the counter runs' own logs hold one")
    ap.add_argument("--json-out", help="also write the summary as JSON to this file")
    ap.add_argument("--per-launch", help="list every dispatch of this kernel class instead")
    a = ap.parse_args()
    if a.per_launch:
        rows = per_launch(a.trace, a.per_launch)
        print("| # | instance | grid | us |\n|---|---|---|---|")
        for i, (inst, gx, us) in enumerate(rows):
            print(f"| {i} | `{inst}` | {gx} | {us:.1f} |")
        return
    s = summarize(a.trace, a.fetch, a.write, a.valu, a.lds, a.bench_json, a.tex)
    if a.json_out:
        with open(a.json_out, "w") as fh:
            json.dump(s, fh, indent=1)
    print(to_markdown(s))


if __name__ == "__main__":
    main()
