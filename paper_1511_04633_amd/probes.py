"""HBM streaming probes (measurement, not part of the solver).

``python -m paper_1511_04633_amd.probes --build`` compiles csrc/probes/*.hip
for gfx950 into executables next to their sources; ``--run`` runs them and
prints their tables (on a GPU).  They establish what MI355X streams at for
plain reads, writes and copies and for the step kernel's own access pattern
without arithmetic, the ceilings the step kernel is measured against.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PROBES = os.path.join(HERE, "csrc", "probes")
NAMES = ("stream", "pull")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build() -> None:
    for name in NAMES:
        subprocess.check_call([HIPCC, *FLAGS, "-o", os.path.join(PROBES, name),
                               os.path.join(PROBES, name + ".hip")], stderr=subprocess.DEVNULL)


def run() -> int:
    for name in NAMES:
        exe = os.path.join(PROBES, name)
        if not os.path.exists(exe):
            raise FileNotFoundError(f"{exe} not built (python -m paper_1511_04633_amd.probes --build)")
        print(f"== {name}", flush=True)
        rc = subprocess.call([exe])
        if rc != 0:
            return rc
    return 0


if __name__ == "__main__":
    if "--build" in sys.argv:
        build()
    if "--run" in sys.argv:
        sys.exit(run())
