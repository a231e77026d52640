"""HBM traffic of a kernel from rocprofv3 counter runs.

Two ``rocprofv3 --pmc`` runs of the same command give FETCH_SIZE and
WRITE_SIZE (KiB per dispatch); two more runs of ``bench.py
--copy-calibration BYTES`` give the same counters for a plain device copy of
known size, from which the counters' scale factors follow.  ``summarize``
turns the four CSV directories into one JSON record (per-dispatch bytes for
the kernels whose name starts with a prefix, the factors, and a hash of the
kernel sources the counters belong to); ``traffic_bytes`` gives the scaled
bytes per launch, or None when the sources have changed since.

The same module summarizes instruction counters of a kernel (SQ_WAVES,
SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS in one run, SQ_INSTS_MFMA in
another) into a record from which ``valu_issue`` gives the VALU lane
operations per launch and their rate as a fraction of the chip's VALU issue
peak (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; a wave64 VALU instruction
takes four cycles of one SIMD).

Usage:
    python -m paper_1010_1386_amd.traffic [--per-run K] FETCH_DIR WRITE_DIR COPYF_DIR COPYW_DIR \\
        KERNEL_PREFIX GRID COPY_BYTES OUT.json
    python -m paper_1010_1386_amd.traffic [--per-run K] --insts SQ_DIR MFMA_DIR KERNEL_PREFIX GRID OUT.json

GRID "any" takes every grid size; --per-run K sums the matching dispatches and
divides by K (a stage of several launches, K pipeline runs profiled).
"""

from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("stages.h", "ures.h", "ures_regs.h", "modarith.h", "device.h", "kernels.hip", "job.cpp")


def sources_sha256():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(PKG, "csrc", name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9  # lane operations per second


def _per_dispatch(directory, prefix, grid=None, counter=None, steps=None):
    """Mean counter value per dispatch of the matching kernels; with `steps`,
    the sum over all matching dispatches divided by `steps` (per pipeline run,
    when a stage is several launches)."""
    paths = glob.glob(os.path.join(directory, "*counter_collection.csv"))
    if not paths:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    vals = []
    with open(paths[0]) as fh:
        for row in csv.DictReader(fh):
            name = row["Kernel_Name"].replace("void ", "")
            if counter is not None and row["Counter_Name"] != counter:
                continue
            if name.startswith(prefix) and (grid is None or row["Grid_Size"] == str(grid)):
                vals.append(float(row["Counter_Value"]))
    if not vals:
        raise ValueError(f"no dispatch of {prefix!r} (grid {grid}) in {paths[0]}")
    return sum(vals) / (steps if steps else len(vals))


def summarize(fetch_dir, write_dir, copyf_dir, copyw_dir, prefix, grid, copy_bytes, steps=None):
    fetch_kib = _per_dispatch(fetch_dir, prefix, grid, steps=steps)
    write_kib = _per_dispatch(write_dir, prefix, grid, steps=steps)
    copy_fetch_kib = _per_dispatch(copyf_dir, "__amd_rocclr_copyBuffer")
    copy_write_kib = _per_dispatch(copyw_dir, "__amd_rocclr_copyBuffer")
    return {
        "kernel_prefix": prefix,
        "grid_size": grid,
        "per": "pipeline run (all matching launches)" if steps else "dispatch",
        "fetch_kib_per_dispatch": fetch_kib,
        "write_kib_per_dispatch": write_kib,
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": copy_fetch_kib,
        "copy_write_kib": copy_write_kib,
        # a plain copy of copy_bytes reads and writes copy_bytes each
        "fetch_factor": copy_bytes / 1024.0 / copy_fetch_kib,
        "write_factor": copy_bytes / 1024.0 / copy_write_kib,
        "sources_sha256": sources_sha256(),
    }


def traffic_bytes(record):
    """Scaled HBM bytes per launch, or None if the kernel sources changed."""
    if record.get("sources_sha256") != sources_sha256():
        return None
    return 1024.0 * (record["fetch_kib_per_dispatch"] * record["fetch_factor"] +
                     record["write_kib_per_dispatch"] * record["write_factor"])


def summarize_insts(sq_dir, mfma_dir, prefix, grid, steps=None):
    rec = {"kernel_prefix": prefix, "grid_size": grid,
           "per": "pipeline run (all matching launches)" if steps else "dispatch"}
    for key, counter in (("waves", "SQ_WAVES"), ("valu_insts", "SQ_INSTS_VALU"), ("salu_insts", "SQ_INSTS_SALU"),
                         ("lds_insts", "SQ_INSTS_LDS")):
        rec[key] = _per_dispatch(sq_dir, prefix, grid, counter, steps)
    rec["mfma_insts"] = _per_dispatch(mfma_dir, prefix, grid, "SQ_INSTS_MFMA", steps)
    rec["sources_sha256"] = sources_sha256()
    return rec


def valu_issue(record, launch_s):
    """(VALU lane operations per launch, their rate / the VALU issue peak), or
    None when the kernel sources have changed since the counters were taken."""
    if record.get("sources_sha256") != sources_sha256():
        return None
    ops = 64.0 * record["valu_insts"]
    return ops, ops / launch_s / VALU_LANE_OPS_PEAK


def main(argv):
    steps = None
    if len(argv) > 2 and argv[1] == "--per-run":  # --per-run K: sums over K pipeline runs, all grids
        steps = int(argv[2])
        argv = argv[:1] + argv[3:]
    if len(argv) == 7 and argv[1] == "--insts":
        rec = summarize_insts(argv[2], argv[3], argv[4], None if argv[5] == "any" else argv[5], steps)
        with open(argv[6], "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        print(json.dumps(rec))
        return 0
    if len(argv) != 9:
        print(__doc__, file=sys.stderr)
        return 2
    rec = summarize(argv[1], argv[2], argv[3], argv[4], argv[5], None if argv[6] == "any" else argv[6],
                    int(argv[7]), steps)
    with open(argv[8], "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
