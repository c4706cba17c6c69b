"""HBM traffic of the benchmark's kernels from two rocprofv3 counter runs.

Reads the per-dispatch counter CSVs of a FETCH_SIZE run and a WRITE_SIZE run
of the same benchmark command, scales each counter by what it reads for the
plain 1 GiB device copy that bench.py performs before its timed region (so the
figures are in bytes of HBM traffic), averages per kernel class, and writes a
small JSON record with a digest of the kernel sources it was measured on.
bench.py reports `traffic` only while that digest still matches.

    python -m paper_1710_07041_amd.traffic FETCH.csv WRITE.csv OUT.json "command"
"""
from __future__ import annotations

import csv
import hashlib
import json
import re
import sys
from collections import defaultdict
from pathlib import Path

PKG = Path(__file__).resolve().parent
KERNEL_SOURCES = ["csrc/sap.hip", "csrc/dslash.hip", "csrc/dd_device.h", "csrc/block_ops.h", "csrc/engine.hip"]
COPY_BYTES = 1 << 30

CLASS_PATTERNS = [
    (r"k_sap_sweep<float,", "sap_sweep_f32"),
    (r"k_sap_sweep<double,", "sap_sweep_f64"),
    (r"k_sap_sweep<__half,", "sap_sweep_f16"),
    (r"k_dslash<float, double,", "dslash_f32in_f64"),
    (r"k_dslash<double, double,", "dslash_f64"),
    (r"k_dslash<float, float,", "dslash_f32"),
    (r"k_dslash<__half,", "dslash_f16"),
    (r"k_dots_lag<", "cgs_dots"),
    (r"k_update_lag<", "cgs_update"),
    (r"k_update_dots<", "restart_norm"),
    (r"k_update_normalize<", "restart_norm"),
]


def _code_only(text: str) -> str:
    """The source without // comments, /* */ comments and blank lines, so a
    comment edit does not invalidate a measurement."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
    return "\n".join(ln for ln in lines if ln.strip())


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(_code_only((PKG / rel).read_text()).encode())
    return h.hexdigest()[:16]


def classify(name: str) -> str | None:
    for pat, cls in CLASS_PATTERNS:
        if re.search(pat, name):
            return cls
    return None


def read(path: str, counter: str):
    per = defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        kib = float(r["Counter_Value"])
        name = r["Kernel_Name"]
        if "copyBuffer" in name or "copy" in name.lower() and "dd::" not in name:
            copies.append(kib)
        cls = classify(name)
        if cls:
            per[cls].append(kib)
    return per, (max(copies) if copies else None)


def main(fetch_csv, write_csv, out_json, command):
    fetch, fcopy = read(fetch_csv, "FETCH_SIZE")
    write, wcopy = read(write_csv, "WRITE_SIZE")
    if not fcopy or not wcopy:
        raise SystemExit("no calibration copy found in the counter runs")
    sf = COPY_BYTES / (fcopy * 1024.0)
    sw = COPY_BYTES / (wcopy * 1024.0)
    kernels = {}
    for cls in sorted(set(fetch) | set(write)):
        f = sum(fetch.get(cls, [0])) / max(len(fetch.get(cls, [])), 1)
        w = sum(write.get(cls, [0])) / max(len(write.get(cls, [])), 1)
        kernels[cls] = {"dispatches": len(fetch.get(cls, [])), "fetch_kib": round(f, 1), "write_kib": round(w, 1),
                        "traffic_bytes": round(f * 1024 * sf + w * 1024 * sw)}
    rec = {"command": command, "source_digest": source_digest(),
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": fcopy, "write_kib": wcopy,
                                "fetch_scale": round(sf, 4), "write_scale": round(sw, 4)},
           "kernels": kernels}
    Path(out_json).write_text(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main(*sys.argv[1:5])
