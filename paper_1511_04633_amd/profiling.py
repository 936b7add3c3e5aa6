"""HBM traffic of the step kernel from rocprofv3 counter runs.

Two ``rocprofv3 --pmc`` runs of bench.py (FETCH_SIZE, then WRITE_SIZE; KiB
per dispatch) are scaled by what the same counters read for the runtime's
plain copy kernel (``__amd_rocclr_copyBuffer``, which bench.py's copy probe
launches on a buffer of known size): on MI355X FETCH_SIZE reads half the
copied bytes and WRITE_SIZE all of them.  The result is tied to a hash of
the kernel sources; bench.py reports it only while that hash matches.

Usage: python -m paper_1511_04633_amd.profiling FETCH_CSV WRITE_CSV STORAGE N
prints the JSON entry for profiles/traffic.json.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/collide.hpp", "csrc/kernels.hpp", "csrc/lbmx.hip"]
# element bytes of the (flow, energy) populations per storage format
BYTES = {"f64": (8, 8), "f32": (4, 4), "f16": (2, 2), "bf16": (2, 2), "f16_f32": (2, 4),
         "bf16_f32": (2, 4), "f16_i16": (2, 2)}


def lattice_bytes(storage, n):
    bf, bg = BYTES[storage]
    return n ** 3 * (19 * bf + 7 * bg)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_kernel(path):
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic_entry(fetch_csv, write_csv, storage, n):
    fetch, write = _per_kernel(fetch_csv), _per_kernel(write_csv)
    copy_kib = lattice_bytes(storage, n) / 1024.0  # bench.py's copy probe size
    cf = [v for v in fetch["__amd_rocclr_copyBuffer"] if v > 0.5 * copy_kib / 2]
    cw = [v for v in write["__amd_rocclr_copyBuffer"] if v > 0.5 * copy_kib]
    s_fetch = copy_kib / statistics.median(cf)
    s_write = copy_kib / statistics.median(cw)
    step = [k for k in fetch if "k_step" in k][0]
    f_kib = statistics.median(fetch[step]) * s_fetch
    w_kib = statistics.median(write[step]) * s_write
    algo = 2 * lattice_bytes(storage, n)
    return {"storage": storage, "n": n, "kernel": step,
            "fetch_kib_raw": statistics.median(fetch[step]),
            "write_kib_raw": statistics.median(write[step]),
            "scale_fetch": round(s_fetch, 5), "scale_write": round(s_write, 5),
            "traffic_bytes": round((f_kib + w_kib) * 1024.0),
            "algorithmic_bytes": algo,
            "traffic_over_algorithmic": round((f_kib + w_kib) * 1024.0 / algo, 5),
            "source_sha256": kernel_source_hash()}


if __name__ == "__main__":
    print(json.dumps(traffic_entry(sys.argv[1], sys.argv[2], sys.argv[3], int(sys.argv[4])),
                     indent=1))
