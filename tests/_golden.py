"""Stored expected values (tests/golden/*.json, written by make_golden.py from the oracle) and
the checks that compare a library result with them."""

from __future__ import annotations

import hashlib
import json
import os

from oracle import poly_eval_mod

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def digest(coeffs):
    """SHA-256 of the canonical decimal coefficient list (lowest power first)."""
    return hashlib.sha256(",".join(str(c) for c in coeffs).encode()).hexdigest()


def load(cfg):
    """Records of tests/golden/cfg<cfg>.json by name."""
    with open(os.path.join(HERE, f"cfg{cfg}.json")) as fh:
        return {r["name"]: r for r in json.load(fh)["records"]}


def check_full(R, rec):
    """Bit-exact equality with the oracle's resultant (degree, digest, stored coefficients)."""
    assert len(R) - 1 == rec["degree"], (rec["name"], len(R) - 1, rec["degree"])
    if "coeffs" in rec:
        assert [str(c) for c in R] == rec["coeffs"], rec["name"]
    for i, v in rec.get("samples", {}).items():
        assert str(R[int(i)]) == v, (rec["name"], i)
    assert digest(R) == rec["sha256"], rec["name"]


def check_modq(R, rec):
    """R(t) mod q equals the oracle's determinant of the Sylvester matrix specialised at t over Z_q."""
    for c in rec["checks"]:
        q, t, v = int(c["q"]), int(c["t"]), int(c["value"])
        assert poly_eval_mod(R, t, q) == v, (rec["name"], q, t)
