"""Write the stored expected resultants under tests/golden/ (calls only oracle/ and workloads/).

Usage:  python tests/golden/make_golden.py [--configs 1 2 4 6] [--jobs N]

For each workload the oracle's exact resultant is stored as its degree, a
SHA-256 digest of the canonical decimal coefficient list (lowest power first,
comma separated) and, for small results, the coefficients themselves.  The
GPU parity tests recompute the digest from the library's output, so a match
is bit-exact equality of every coefficient.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def digest(coeffs):
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


def record(name, R, keep_all):
    rec = {"name": name, "degree": len(R) - 1, "sha256": digest(R),
           "max_bits": max((abs(c).bit_length() for c in R), default=0)}
    if keep_all:
        rec["coeffs"] = [str(c) for c in R]
    else:
        idx = sorted(set([0, 1, len(R) // 2, len(R) - 2, len(R) - 1]) & set(range(len(R))))
        rec["samples"] = {str(i): str(R[i]) for i in idx}
    return rec


def _job(args):
    name, f, g, var, keep_all = args
    t0 = time.time()
    R = oracle.res(f, g, var)
    rec = record(name, R, keep_all)
    rec["oracle_seconds"] = round(time.time() - t0, 2)
    return rec


def jobs_for(cfg):
    if cfg == 1:
        f, g = workloads.config1()
        return [("cfg1_y", f, g, "y", True), ("cfg1_x", f, g, "x", True)]
    if cfg == 2:
        f, g = workloads.config2()
        return [("cfg2_y", f, g, "y", False), ("cfg2_x", f, g, "x", False)]
    if cfg == 4:
        out = []
        for k, (f, g) in enumerate(workloads.config4()):
            Ft, Gt = oracle.bivar_trim(f), oracle.bivar_trim(g)
            if len(Ft) - 1 + len(Gt) - 1 <= 24:
                out.append((f"cfg4_{k}_y", f, g, "y", False))
        return out
    if cfg == 6:  # large-coefficient random curves (paper Table 3), first pair of each set
        out = []
        for deg, k, sparse in ((9, 128, False), (9, 512, False), (9, 512, True), (15, 128, False)):
            f, g = workloads.table3_curves(deg, k, sparse)[0]
            name = f"t3_{deg}_{k}_{'sparse' if sparse else 'dense'}"
            out.append((name + "_y", f, g, "y", False))
        return out
    raise ValueError(cfg)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, nargs="+", default=[1])
    ap.add_argument("--jobs", type=int, default=os.cpu_count())
    a = ap.parse_args()
    for cfg in a.configs:
        jobs = jobs_for(cfg)
        with ProcessPoolExecutor(max_workers=min(a.jobs, len(jobs))) as ex:
            recs = list(ex.map(_job, jobs))
        path = os.path.join(HERE, f"cfg{cfg}.json")
        with open(path, "w") as fh:
            json.dump({"config": cfg, "generator": "tests/golden/make_golden.py (oracle.res)",
                       "records": recs}, fh, indent=1)
        print(path, len(recs), "records", flush=True)


if __name__ == "__main__":
    main()
