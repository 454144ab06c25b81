"""Summarises rocprofv3 CSV output into the short text files kept in profiles/.

    python profile_summary.py stats <kernel_stats.csv> <out.txt> "<command>"
    python profile_summary.py pmc <fetch_counter_collection.csv> <write_counter_collection.csv> <out.txt> \
        "<fetch command>" "<write command>" <calibration bytes>
    python profile_summary.py counters <counter_collection.csv> <out.txt> "<command>"

`stats` keeps each kernel's call count, total and average duration.
`counters` keeps, per kernel, the average per dispatch of every counter of
one --pmc pass.
`pmc` keeps, per kernel, the average FETCH_SIZE and WRITE_SIZE per dispatch (KiB)
and the scale factors read off the calibration launches bench.py makes with
--copy-calibration: a 1 GiB fill (written bytes) and a 1 GiB device copy
(read bytes); factor = known bytes / counter bytes.
"""
import csv
import glob
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash():
    """sha256 over the HIP sources; bench.py trusts a counter summary only while it matches"""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "paper_2602_05081_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def stats(src, out, cmd):
    rows = list(csv.DictReader(open(src)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    with open(out, "w") as fh:
        fh.write("# rocprofv3 --kernel-trace --stats summary\n# command: %s\n" % cmd)
        fh.write("%-72s %6s %12s %12s %7s\n" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
        for r in rows[:30]:
            fh.write("%-72s %6s %12.3f %12.2f %7.2f\n" % (r["Name"][:72], r["Calls"],
                                                          float(r["TotalDurationNs"]) / 1e6,
                                                          float(r["AverageNs"]) / 1e3, float(r["Percentage"])))


def _per_kernel(src):
    acc = defaultdict(list)
    rows = list(csv.DictReader(open(src)))
    for r in rows:
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return acc, rows


def pmc(fsrc, wsrc, out, fcmd, wcmd, calib_bytes):
    fa, frows = _per_kernel(fsrc)
    wa, wrows = _per_kernel(wsrc)
    calib = float(calib_bytes)
    copy = max((float(r["Counter_Value"]) for r in frows if "copyBuffer" in r["Kernel_Name"]), default=0.0)
    fill = max((float(r["Counter_Value"]) for r in wrows if "FillFunctor" in r["Kernel_Name"]), default=0.0)
    ffac = calib / (copy * 1024.0) if copy else float("nan")
    wfac = calib / (fill * 1024.0) if fill else float("nan")
    with open(out, "w") as fh:
        fh.write("# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE summary (KiB per dispatch, raw counter values)\n")
        fh.write("# fetch command: %s\n# write command: %s\n" % (fcmd, wcmd))
        fh.write("# source hash: %s\n" % source_hash())
        fh.write("# calibration: 1 GiB device copy FETCH_SIZE = %.1f KiB -> fetch factor %.4f; "
                 "1 GiB fill WRITE_SIZE = %.1f KiB -> write factor %.4f\n" % (copy, ffac, fill, wfac))
        fh.write("%-72s %6s %16s %16s %14s\n" % ("kernel", "calls", "FETCH_KiB", "WRITE_KiB", "HBM_MB_scaled"))
        names = sorted(set(fa) | set(wa), key=lambda k: -(sum(fa.get(k, [0])) + sum(wa.get(k, [0]))))
        for k in names[:25]:
            f = sum(fa.get(k, [0])) / max(1, len(fa.get(k, [])))
            w = sum(wa.get(k, [0])) / max(1, len(wa.get(k, [])))
            fh.write("%-72s %6d %16.1f %16.1f %14.2f\n" % (k[:72], max(len(fa.get(k, [])), len(wa.get(k, []))), f, w,
                                                           (f * ffac + w * wfac) * 1024 / 1e6))


def counters(src, out, cmd):
    acc = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    names = []
    for r in csv.DictReader(open(src)):
        k, c = r["Kernel_Name"], r["Counter_Name"]
        acc[k][c] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
        if c not in names:
            names.append(c)
    kernels = sorted(acc, key=lambda k: -sum(acc[k].values()) / len(disp[k]))
    with open(out, "w") as fh:
        fh.write("# rocprofv3 --pmc summary (average per dispatch)\n# command: %s\n" % cmd)
        fh.write("# source hash: %s\n" % source_hash())
        fh.write("%-48s %6s" % ("kernel", "calls") + "".join(" %16s" % c for c in names) + "\n")
        for k in kernels[:12]:
            n = len(disp[k])
            fh.write("%-48s %6d" % (k[:48], n) + "".join(" %16.4g" % (acc[k][c] / n) for c in names) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6], sys.argv[7])
