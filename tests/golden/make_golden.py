"""Write the stored expected resultants under tests/golden/ (calls only oracle/ and workloads/).

Usage:  python tests/golden/make_golden.py [--configs 1 2 4 5 6 40 50] [--jobs N]

For each workload the oracle's exact resultant is stored as its degree, a
SHA-256 digest of the canonical decimal coefficient list (lowest power first,
comma separated) and, for small results, the coefficients themselves.  The
GPU parity tests recompute the digest from the library's output, so a match
is bit-exact equality of every coefficient.

Configs 4 and 5 (the batch of 512 and the serving stream) store the full
oracle on every problem whose Sylvester matrix has order r = m_y + n_y <= 32.
Configs 40 and 50 store modular checks of every problem of those workloads:
for two 61-bit check primes q and seeded points t, the oracle's determinant
of the Sylvester matrix specialised at t over Z_q, which must equal R(t) mod q
(evaluation commutes with the determinant, Sec. 4.1; a wrong R passes one
check with probability at most deg R / q).
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


R_FULL = 32  # order of the Sylvester matrix up to which the full oracle runs


def _order(f, g, var):
    if var == "x":
        f, g = oracle.bivar_transpose(f), oracle.bivar_transpose(g)
    return len(oracle.bivar_trim(f)) - 1 + len(oracle.bivar_trim(g)) - 1


def _modq_job(args):
    name, f, g, var, seed = args
    import random
    rnd = random.Random(seed)
    qs = oracle.next_check_primes(8)
    checks = []
    for j in range(2):
        q = qs[(seed + j) % len(qs)]
        t = rnd.randrange(q)
        checks.append({"q": str(q), "t": str(t), "value": str(oracle.res_at_point_mod(f, g, t, q, var))})
    return {"name": name, "var": var, "checks": checks}


def modq_jobs_for(cfg):
    if cfg == 40:
        return [(f"cfg4_{k}_y", f, g, "y", k) for k, (f, g) in enumerate(workloads.config4())]
    if cfg == 50:
        return [(f"cfg5_{k}_{v}", f, g, v, k) for k, (f, g, v) in enumerate(workloads.config5())]
    raise ValueError(cfg)


def jobs_for(cfg):
    if cfg == 1:
        f, g = workloads.config1()
        return [("cfg1_y", f, g, "y", True), ("cfg1_x", f, g, "x", True)]
    if cfg == 2:
        f, g = workloads.config2()
        return [("cfg2_y", f, g, "y", False), ("cfg2_x", f, g, "x", False)]
    if cfg == 4:
        out = [(f"cfg4_{k}_y", f, g, "y", False) for k, (f, g) in enumerate(workloads.config4())
               if _order(f, g, "y") <= R_FULL]
        # largest first, so that the pool's last jobs are short
        return sorted(out, key=lambda j: -_order(j[1], j[2], j[3]))
    if cfg == 5:
        out = [(f"cfg5_{k}_{v}", f, g, v, False) for k, (f, g, v) in enumerate(workloads.config5())
               if _order(f, g, v) <= R_FULL]
        return sorted(out, key=lambda j: -_order(j[1], j[2], j[3]))
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
        modq = cfg in (40, 50)
        jobs = modq_jobs_for(cfg) if modq else jobs_for(cfg)
        with ProcessPoolExecutor(max_workers=min(a.jobs, len(jobs))) as ex:
            recs = list(ex.map(_modq_job if modq else _job, jobs))
        recs.sort(key=lambda r: [int(x) if x.isdigit() else x for x in r["name"].split("_")])
        path = os.path.join(HERE, f"cfg{cfg}.json")
        with open(path, "w") as fh:
            json.dump({"config": cfg, "generator": "tests/golden/make_golden.py (oracle.res_at_point_mod)"
                       if modq else "tests/golden/make_golden.py (oracle.res)",
                       "records": recs}, fh, indent=1)
        print(path, len(recs), "records", flush=True)


if __name__ == "__main__":
    main()
