"""HBM traffic of the CG update kernel from two rocprofv3 counter runs.

Usage (GPU):
  rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d A -- \\
      python3 bench.py --pmc-probe
  rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d B -- \\
      python3 bench.py --pmc-probe
  python -m paper_2001_06613_amd.pmc_traffic A B profiles/cg_update_traffic.json

Each run holds the dispatches of one whole solve and one plain copy of
COPY_BYTES bytes (read once, written once).  The counters report KiB per
dispatch; each is scaled by what it reads for the copy (bytes known), so
the result is HBM bytes per launch of the kernel, averaged over its
launches like the benchmark's achieved bandwidth.  The record carries the
SHA-256 of the kernel's source code (comments and spacing removed): the
benchmark reports it only while that code is unchanged.
"""

import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL = "cgv_update_kernel<2,"    # every form (launch bound, first step) matches
LABEL = "cgv_update_kernel<2, *>"
# every source the kernel is built from
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("cg_tiles.hip", "reduce.h", "stml_dev.h", "launch.h")]
COPY_BYTES = 512 << 20


def _rows(d):
    paths = glob.glob(os.path.join(d, "**", "*counter_collection.csv"),
                      recursive=True)
    if not paths:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value)} for one counter."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        k, old = out.get(key, (name, 0.0))
        out[key] = (name, old + v)
    return out


def _mean(vals):
    return sum(vals) / len(vals) if vals else float("nan")


def _code(text):
    """Source text without comments and blank space: the hash follows the
    code, not its commentary."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_sha():
    h = hashlib.sha256()
    for path in SOURCES:
        with open(path, encoding="utf-8") as fh:
            h.update(_code(fh.read()).encode())
    return h.hexdigest()


def summarise(fetch_dir, write_dir):
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = _per_dispatch(_rows(d), counter)
        kern = [v for n, v in disp.values() if KERNEL in n]
        # the largest dispatch that is not ours: the plain copy
        copy = max((v for n, v in disp.values() if "stml" not in n),
                   default=float("nan"))
        res[counter] = {"kernel_kib_mean": _mean(kern),
                        "launches": len(kern), "copy_kib": copy}
    f, w = res["FETCH_SIZE"], res["WRITE_SIZE"]
    scale_f = COPY_BYTES / (f["copy_kib"] * 1024.0)
    scale_w = COPY_BYTES / (w["copy_kib"] * 1024.0)
    per_launch = (f["kernel_kib_mean"] * 1024.0 * scale_f +
                  w["kernel_kib_mean"] * 1024.0 * scale_w)
    sha = source_sha()
    return {"kernel": LABEL, "hbm_bytes_per_launch": per_launch,
            "fetch_kib_per_launch": f["kernel_kib_mean"],
            "write_kib_per_launch": w["kernel_kib_mean"],
            "fetch_scale": scale_f, "write_scale": scale_w,
            "launches": f["launches"], "copy_bytes": COPY_BYTES,
            "source_sha256": sha}


if __name__ == "__main__":
    rec = summarise(sys.argv[1], sys.argv[2])
    with open(sys.argv[3], "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))
