"""Summaries of rocprofv3 CSV output for the library's kernels.

  python -m paper_2308_15020_amd.profsum trace <..._kernel_trace.csv>
      per (kernel, grid) dispatch count, average / total duration, share
  python -m paper_2308_15020_amd.profsum traffic <FETCH csv> <WRITE csv> --copy-mib M [--kernel k_eval_group]
      HBM bytes per dispatch of one kernel from the two counter passes,
      scaled by the plain elementwise kernel; with the kernel sources' hash
  python -m paper_2308_15020_amd.profsum pmc <..._counter_collection.csv> [--copy-mib M]
      per (kernel, grid) average of each counter per dispatch; with
      --copy-mib, the same counters for the largest plain copy dispatch and
      the factor (M MiB / counter) that turns FETCH_SIZE / WRITE_SIZE into
      bytes
  python -m paper_2308_15020_amd.profsum cards <trace csv> --sq <csv> --fetch <csv> --write <csv>
      --copy-mib M --kernels "k_pull<4| 4| true>,..."
      one JSON card per kernel template (see cards())
"""
from __future__ import annotations

import argparse
import csv
import re
from collections import defaultdict


def short(name: str) -> str:
    name = re.sub(r"\s+", " ", name)
    m = re.search(r"(k_\w+)(<[^()]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name[:200]


def trace(path: str, top: int = 25) -> str:
    acc = defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(path)):
        key = (short(r["Kernel_Name"]), r.get("Grid_Size_X", "?") + "x" + r.get("Grid_Size_Y", "?"))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        acc[key][0] += 1
        acc[key][1] += d
    tot = sum(v[1] for v in acc.values())
    lines = [f"{'kernel':<60} {'grid':>14} {'calls':>6} {'avg_us':>9} {'total_us':>10} {'share':>6}"]
    for (k, g), (n, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{k[:60]:<60} {g:>14} {n:>6} {t / n:>9.2f} {t:>10.1f} {t / tot:>6.3f}")
    fams = defaultdict(lambda: [0, 0.0])
    for (k, _g), (n, t) in acc.items():
        f = family_of(k)
        if f is not None:
            fams[f][0] += n
            fams[f][1] += t
    for f, (n, t) in fams.items():
        lines.append(f"family {f}: {n} dispatches, average {t / n:.2f} us, total {t:.1f} us, share {t / tot:.3f}")
    return "\n".join(lines)


def pmc(path: str, copy_mib: float = 0.0, top: int = 25) -> str:
    acc = defaultdict(lambda: defaultdict(float))
    calls = defaultdict(set)
    for r in csv.DictReader(open(path)):
        key = (short(r["Kernel_Name"]), r.get("Grid_Size", r.get("Grid_Size_X", "?")))
        acc[key][r["Counter_Name"]] += float(r["Counter_Value"])
        calls[key].add(r["Dispatch_Id"])
    names = sorted({c for v in acc.values() for c in v})
    lines = [f"{'kernel':<60} {'grid':>10} {'calls':>6} " + " ".join(f"{c:>16}" for c in names)]
    order = sorted(acc.items(), key=lambda kv: -max(kv[1].values()) / len(calls[kv[0]]))
    for key, cv in order[:top]:
        n = len(calls[key])
        lines.append(f"{key[0][:60]:<60} {key[1]:>10} {n:>6} " + " ".join(f"{cv[c] / n:>16.1f}" for c in names))
    if copy_mib > 0:
        # FETCH_SIZE / WRITE_SIZE are in KiB: the plain elementwise kernel that
        # reads and writes copy_mib MiB gives the scale of each counter
        cands = [k for k in acc if "elementwise" in k[0].lower()]
        lines.append("")
        lines.append(f"calibration: plain elementwise kernel reading and writing {copy_mib:g} MiB")
        for c in names:
            best = max(cands, key=lambda k: acc[k][c] / len(calls[k]), default=None)
            if best is None or acc[best][c] <= 0:
                continue
            per = acc[best][c] / len(calls[best])
            lines.append(f"  {c}: {per:.1f} KiB per dispatch -> scale {copy_mib * 1024 / per:.4f}")
    return "\n".join(lines)


def kernel_source_hash() -> str:
    """SHA-256 over every device and host source of the library (a change to
    any kernel, or to how it is launched, invalidates recorded counters)."""
    import hashlib
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(here)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(here, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def family_of(name: str) -> str | None:
    """The family a template belongs to (a name with `*` for its segment
    shape), or None: the per-bin FP64 root-of-unity kernels
    k_eval<float, double, SEG, L, true>."""
    m = re.fullmatch(r"k_eval<float, double, \d+, \d+, true>", name)
    return "k_eval<float, double, *, *, true>" if m else None


def _by_template(path, counter=None):
    """Per kernel template name, and per family (family_of): (sum of values
    or durations, dispatches)."""
    acc = defaultdict(float)
    calls = defaultdict(set)
    for r in csv.DictReader(open(path)):
        name = short(r["Kernel_Name"])
        fam = family_of(name)
        if fam is not None:
            if counter is None:
                acc[fam] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                calls[fam].add(r.get("Dispatch_Id", r.get("Correlation_Id", len(calls[fam]))))
            elif r["Counter_Name"] == counter:
                acc[fam] += float(r["Counter_Value"])
                calls[fam].add(r["Dispatch_Id"])
        if counter is None:
            acc[name] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            calls[name].add(r.get("Dispatch_Id", r.get("Correlation_Id", len(calls[name]))))
        elif r["Counter_Name"] == counter:
            acc[name] += float(r["Counter_Value"])
            calls[name].add(r["Dispatch_Id"])
    return {k: (acc[k], len(calls[k])) for k in acc}


def cards(trace_csv, sq_csv, fetch_csv, write_csv, copy_mib, kernels):
    """One `card:` line (JSON) per kernel template: rocprof average duration
    (kernel trace), VALU instructions and VALU-active cycles per dispatch (SQ
    pass), HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE scaled by the
    plain elementwise kernel of copy_mib MiB, and the sources' hash."""
    import json
    tr = _by_template(trace_csv)
    vi = _by_template(sq_csv, "SQ_INSTS_VALU")
    va = _by_template(sq_csv, "SQ_ACTIVE_INST_VALU")
    fe = _by_template(fetch_csv, "FETCH_SIZE")
    wr = _by_template(write_csv, "WRITE_SIZE")
    sf, sw = _calib(fetch_csv, "FETCH_SIZE", copy_mib), _calib(write_csv, "WRITE_SIZE", copy_mib)
    out = []
    for k in kernels:
        c = {"kernel_name": k, "source_sha256": kernel_source_hash()}
        if k in tr:
            c["rocprof_avg_us"] = round(tr[k][0] / tr[k][1], 2)
            c["rocprof_dispatches"] = tr[k][1]
        if k in vi:
            c["valu_insts_per_launch"] = round(vi[k][0] / vi[k][1], 1)
        if k in va:
            c["valu_active_per_launch"] = round(va[k][0] / va[k][1], 1)
        if k in fe and k in wr and sf and sw:
            rb = fe[k][0] / fe[k][1] * 1024 * sf
            wb = wr[k][0] / wr[k][1] * 1024 * sw
            c.update({"read_bytes_per_launch": round(rb), "write_bytes_per_launch": round(wb),
                      "traffic_bytes_per_launch": round(rb + wb)})
        out.append("card: " + json.dumps(c))
    return "\n".join(out)


def _per_dispatch(path, counter, match):
    tot, calls = 0.0, set()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
            tot += float(r["Counter_Value"])
            calls.add(r["Dispatch_Id"])
    return tot / max(1, len(calls)), len(calls)


def _calib(path, counter, copy_mib):
    best = 0.0
    acc = defaultdict(float)
    calls = defaultdict(set)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and "elementwise" in r["Kernel_Name"].lower():
            acc[r["Kernel_Name"]] += float(r["Counter_Value"])
            calls[r["Kernel_Name"]].add(r["Dispatch_Id"])
    for k in acc:
        best = max(best, acc[k] / len(calls[k]))
    return copy_mib * 1024 / best if best > 0 else None


def traffic(fetch_csv, write_csv, kernel, copy_mib):
    """HBM bytes per dispatch of `kernel`: FETCH_SIZE and WRITE_SIZE (KiB)
    scaled by what they read for a plain elementwise kernel of copy_mib MiB."""
    f, nf = _per_dispatch(fetch_csv, "FETCH_SIZE", kernel)
    w, nw = _per_dispatch(write_csv, "WRITE_SIZE", kernel)
    sf, sw = _calib(fetch_csv, "FETCH_SIZE", copy_mib), _calib(write_csv, "WRITE_SIZE", copy_mib)
    rb = f * 1024 * sf
    wb = w * 1024 * sw
    return "\n".join([
        f"traffic_kernel: {kernel}",
        f"source_sha256: {kernel_source_hash()}",
        f"fetch_kib_per_dispatch: {f:.1f} ({nf} dispatches), scale {sf:.4f}",
        f"write_kib_per_dispatch: {w:.1f} ({nw} dispatches), scale {sw:.4f}",
        f"read_bytes_per_launch: {rb:.0f}",
        f"write_bytes_per_launch: {wb:.0f}",
        f"traffic_bytes_per_launch: {rb + wb:.0f}",
    ])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=["trace", "pmc", "traffic", "cards"])
    ap.add_argument("csv")
    ap.add_argument("csv2", nargs="?", default=None, help="traffic: the WRITE_SIZE csv")
    ap.add_argument("--copy-mib", type=float, default=0.0)
    ap.add_argument("--kernel", default="k_eval_group")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--sq", default=None, help="cards: the SQ counter csv")
    ap.add_argument("--fetch", default=None, help="cards: the FETCH_SIZE csv")
    ap.add_argument("--write", default=None, help="cards: the WRITE_SIZE csv")
    ap.add_argument("--kernels", default="", help="cards: comma-separated kernel template names ('|' inside)")
    a = ap.parse_args()
    if a.kind == "cards":
        ks = [k.replace("|", ",") for k in a.kernels.split(",") if k]
        print(cards(a.csv, a.sq, a.fetch, a.write, a.copy_mib, ks))
        return
    if a.kind == "trace":
        print(trace(a.csv, a.top))
    elif a.kind == "pmc":
        print(pmc(a.csv, a.copy_mib, a.top))
    else:
        print(traffic(a.csv, a.csv2, a.kernel, a.copy_mib))


if __name__ == "__main__":
    main()
