"""CPU check of the kernels' per-lane arithmetic (host build) against the oracle.

The device code for evaluation and the univariate resultant over Z_p is plain
__host__ __device__ C++ (csrc/ures.h, csrc/modarith.h).  tests/hostsim
compiles it for the host; here it is compared with the oracle's Gaussian
elimination of the formal-degree Sylvester matrix mod p on random and
degenerate inputs (vanishing leading coefficients, zero polynomials, common
factors, degree drops in the remainder sequence).
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import det_mod, poly_eval_mod
from workloads import rng_for

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "hostsim", "libhostsim.so")
SRC = os.path.join(HERE, "hostsim", "hostsim.cpp")
PRIMES = [1431655751, 1431655747, 1431655703, 1073741827]  # 2^30 < p < 2^32 / 3, as the library's table


@pytest.fixture(scope="module")
def hs():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC),
            os.path.getmtime(os.path.join(HERE, "..", "paper_1010_1386_amd", "csrc", "ures.h")),
            os.path.getmtime(os.path.join(HERE, "..", "paper_1010_1386_amd", "csrc", "ures_regs.h")),
            os.path.getmtime(os.path.join(HERE, "..", "paper_1010_1386_amd", "csrc", "modarith.h"))):
        subprocess.check_call(["hipcc", "-O2", "-fPIC", "-shared", "-o", LIB, SRC])
    lib = ctypes.CDLL(LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.hs_ures.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                            ctypes.POINTER(ctypes.c_int)]
    lib.hs_eval.argtypes = [ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p,
                            ctypes.POINTER(ctypes.c_int), ctypes.c_uint32, u32p]
    lib.hs_ures_regs.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                 ctypes.POINTER(ctypes.c_int)]
    lib.hs_ures_regs2.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.hs_ures_regs_gen.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.hs_ures_regs2_gen.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
    lib.hs_ures_regs_long.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                      ctypes.POINTER(ctypes.c_int)]
    lib.hs_ures_group.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_int, u32p, u32p, u32p,
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    return lib


def ures(hs, p, A, B, K=1):
    """The lane code: one lane (K = 1), a group of K lanes on K host threads, or
    (K = "regs8", "regs24", ...) the register form for degrees up to that bound."""
    m, n = len(A) - 1, len(B) - 1
    a = (ctypes.c_uint32 * len(A))(*A)
    b = (ctypes.c_uint32 * len(B))(*B)
    out = ctypes.c_uint32()
    bad = ctypes.c_int()
    if isinstance(K, str) and K.startswith("long"):
        nmax = int(K[4:])
        assert hs.hs_ures_regs_long(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad)) == 0
    elif isinstance(K, str) and K.startswith("lgen"):
        nmax = int(K[4:])
        gen = ctypes.c_int()
        assert hs.hs_ures_regs_gen(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad), ctypes.byref(gen)) == 0
    elif isinstance(K, str) and K.startswith("gen"):
        nmax = int(K[3:])
        agree, gen = ctypes.c_int(), ctypes.c_int()
        assert hs.hs_ures_regs2_gen(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad), ctypes.byref(agree),
                                    ctypes.byref(gen)) == 0
        assert agree.value == 1, "the two lanes of the pair disagree"
    elif isinstance(K, str) and K.startswith("pair"):
        nmax = int(K[4:])
        agree = ctypes.c_int()
        assert hs.hs_ures_regs2(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad), ctypes.byref(agree)) == 0
        assert agree.value == 1, "the two lanes of the pair disagree"
    elif isinstance(K, str):
        nmax = int(K[4:])
        assert hs.hs_ures_regs(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad)) == 0
    elif K == 1:
        hs.hs_ures(p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad))
    else:
        agree = ctypes.c_int()
        assert hs.hs_ures_group(K, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad), ctypes.byref(agree)) == 0
        assert agree.value == 1, "lanes of the group disagree"
    return out.value, bool(bad.value)


KS = [1, 2, 4, 8, "regs16", "pair16", "gen16", "lgen16"]


def sylvester_det_mod(A, B, p):
    """det of the formal Sylvester matrix (A rows first, highest power first) mod p."""
    m, n = len(A) - 1, len(B) - 1
    r = m + n
    if r == 0:
        return 1 % p
    S = [[0] * r for _ in range(r)]
    for i in range(n):
        for t in range(m + 1):
            S[i][i + t] = A[m - t]
    for l in range(m):
        for t in range(n + 1):
            S[n + l][l + t] = B[n - t]
    return det_mod(S, p)


def polymul_mod(a, b, p):
    out = [0] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] = (out[i + j] + u * v) % p
    return out


@pytest.mark.parametrize("K", KS)
@pytest.mark.parametrize("seed", range(30))
def test_random_generic(hs, seed, K):
    rng = rng_for(950, seed)
    p = PRIMES[seed % len(PRIMES)]
    m, n = int(rng.integers(0, 12)), int(rng.integers(0, 12))
    A = [int(v) for v in rng.integers(0, p, m + 1)]
    B = [int(v) for v in rng.integers(0, p, n + 1)]
    got, _ = ures(hs, p, A, B, K)
    assert got == sylvester_det_mod(A, B, p)


@pytest.mark.parametrize("K", [1, 2, 4, 8, "regs32", "pair32", "gen32", "lgen32"])
@pytest.mark.parametrize("seed", range(6))
def test_random_large_degree(hs, seed, K):
    """Degrees 13..40: every lane of a group runs several four-way fused updates."""
    rng = rng_for(953, seed)
    p = PRIMES[seed % len(PRIMES)]
    m, n = int(rng.integers(13, 41)), int(rng.integers(13, 41))
    if isinstance(K, str):
        m, n = min(m, 32), min(n, 32)
    A = [int(v) for v in rng.integers(0, p, m + 1)]
    B = [int(v) for v in rng.integers(0, p, n + 1)]
    got, _ = ures(hs, p, A, B, K)
    assert got == sylvester_det_mod(A, B, p)


@pytest.mark.parametrize("K", KS)
@pytest.mark.parametrize("seed", range(60))
def test_degenerate(hs, seed, K):
    """Small primes-like structure: tiny coefficient alphabet forces zero leading
    coefficients, degree drops by more than one and common factors."""
    rng = rng_for(951, seed)
    p = PRIMES[seed % len(PRIMES)]
    m, n = int(rng.integers(0, 8)), int(rng.integers(0, 8))
    alphabet = [0, 0, 1, p - 1, 2]
    A = [alphabet[int(v)] for v in rng.integers(0, len(alphabet), m + 1)]
    B = [alphabet[int(v)] for v in rng.integers(0, len(alphabet), n + 1)]
    if seed % 3 == 0 and m >= 1 and n >= 1:  # plant a common factor (y - 3)
        c = [p - 3, 1]
        A = polymul_mod(c, A[:m], p)
        B = polymul_mod(c, B[:n], p)
    got, bad = ures(hs, p, A, B, K)
    assert got == sylvester_det_mod(A, B, p), (p, A, B)
    assert bad == (A[-1] == 0 or B[-1] == 0)


@pytest.mark.parametrize("K", KS)
def test_remainder_degree_drops(hs, K):
    """Remainder sequences whose degree falls by more than one at a time."""
    p = PRIMES[0]
    cases = [
        ([1, 0, 0, 0, 1], [1, 0, 1]),          # y^4+1 vs y^2+1: remainder constant
        ([5, 0, 0, 0, 0, 1], [0, 0, 1]),       # y^5+5 vs y^2: remainder constant
        ([1, 2, 1], [1, 1]),                   # (y+1)^2 vs y+1: zero remainder
        ([3, 0, 0, 1], [7, 0, 0, 0, 0, 0, 2]), # deg A < deg B at the start
        ([0, 0, 0, 0], [1, 2, 3]),             # A = 0 with formal degree 3
        ([0, 0, 4, 0], [1, 2, 0]),             # both leading coefficients vanish
        ([2, 3, 0, 0], [1, 1, 1]),             # deg A = 1 < formal 3
        ([2, 3, 4], [6, 0, 0, 0]),             # deg B = 0 < formal 3
    ]
    for A, B in cases:
        got, _ = ures(hs, p, A, B, K)
        assert got == sylvester_det_mod(A, B, p), (A, B)


@pytest.mark.parametrize("seed", range(10))
def test_eval_rows(hs, seed):
    rng = rng_for(952, seed)
    p = PRIMES[seed % len(PRIMES)]
    nrows, stride = int(rng.integers(1, 6)), int(rng.integers(1, 9))
    coeff = [int(v) for v in rng.integers(0, p, nrows * stride)]
    rdeg = [int(rng.integers(-1, stride)) for _ in range(nrows)]
    x = int(rng.integers(0, 5000))
    out = (ctypes.c_uint32 * nrows)()
    hs.hs_eval(p, nrows, stride, (ctypes.c_uint32 * len(coeff))(*coeff), (ctypes.c_int * nrows)(*rdeg), x, out)
    for j in range(nrows):
        row = coeff[j * stride: j * stride + rdeg[j] + 1]
        assert out[j] == poly_eval_mod(row, x, p)


@pytest.mark.parametrize("form", ["regs", "pair", "gen", "lgen"])
@pytest.mark.parametrize("nmax", [8, 16, 24, 32])
@pytest.mark.parametrize("seed", range(40))
def test_register_form_shapes(hs, form, nmax, seed):
    """The register form on its own shapes (|m - n| <= 1, generic and with planted
    degree drops, vanishing leading coefficients and common factors) and on
    shapes it hands to the general code."""
    rng = rng_for(954, seed)
    p = PRIMES[seed % len(PRIMES)]
    n = int(rng.integers(1, nmax + 1))
    kind = seed % 5
    m = n + int(rng.integers(-1, 2)) if kind != 4 else int(rng.integers(0, nmax + 1))
    m = max(0, min(nmax, m))
    A = [int(v) for v in rng.integers(0, p, m + 1)]
    B = [int(v) for v in rng.integers(0, p, n + 1)]
    if kind == 1 and m >= 2 and n >= 2:  # common factor (y - 5): a zero remainder
        A = polymul_mod([p - 5, 1], A[:m], p)
        B = polymul_mod([p - 5, 1], B[:n], p)
    if kind == 2:  # small alphabet: remainders that drop by more than one degree
        alphabet = [0, 0, 1, p - 1]
        A = [alphabet[int(v)] for v in rng.integers(0, 4, m + 1)]
        B = [alphabet[int(v)] for v in rng.integers(0, 4, n + 1)]
        A[-1] = A[-1] or 1
        B[-1] = B[-1] or 1
    if kind == 3:  # a vanishing leading coefficient
        A[-1] = 0
    got, bad = ures(hs, p, A, B, "%s%d" % (form, nmax))
    assert got == sylvester_det_mod(A, B, p), (m, n, kind)
    assert bad == (A[-1] == 0 or B[-1] == 0)


@pytest.mark.parametrize("nmax", [8, 24, 32])
def test_branch_free_chain_takes_generic_inputs(hs, nmax):
    """Random coefficients of the register form's shapes stay on the branch-free
    chain (no restart), and its value is the Sylvester determinant; planted
    degree drops and vanishing leading coefficients restart."""
    rng = rng_for(955, nmax)
    p = PRIMES[0]
    for trial in range(12):
        n = int(rng.integers(1, nmax + 1))
        m = max(1, min(nmax, n + int(rng.integers(-1, 2))))
        A = [int(v) for v in rng.integers(1, p, m + 1)]
        B = [int(v) for v in rng.integers(1, p, n + 1)]
        kind = trial % 3
        if kind == 1:
            A[-1] = 0
        if kind == 2 and m >= 2 and n >= 2:  # common factor (y - 5): the remainders end in zero
            A = polymul_mod([p - 5, 1], A[:m], p)
            B = polymul_mod([p - 5, 1], B[:n], p)
        a = (ctypes.c_uint32 * len(A))(*A)
        b = (ctypes.c_uint32 * len(B))(*B)
        out, bad, agree, gen = ctypes.c_uint32(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert hs.hs_ures_regs2_gen(nmax, p, m, n, a, b, ctypes.byref(out), ctypes.byref(bad), ctypes.byref(agree),
                                    ctypes.byref(gen)) == 0
        assert agree.value == 1
        assert out.value == sylvester_det_mod(A, B, p), (m, n, kind)
        assert gen.value == (1 if kind == 0 else 0) or (kind == 2 and min(m, n) < 2), (m, n, kind)


@pytest.mark.parametrize("nmax", [8, 16, 24, 32])
@pytest.mark.parametrize("seed", range(60))
def test_general_shapes_register_form(hs, nmax, seed):
    """The one-lane register form for any shape (first division on rows, then the
    branch-free chain): long and short A, generic coefficients, planted common
    factors, remainders that drop by more than one degree, vanishing leading
    coefficients of either input, and constants."""
    rng = rng_for(956, 100 * nmax + seed)
    p = PRIMES[seed % len(PRIMES)]
    kind = seed % 6
    m = int(rng.integers(0, nmax + 1))
    n = int(rng.integers(0, nmax + 1))
    if kind in (0, 1, 2) and abs(m - n) < 2 and nmax >= 8:  # mostly the long shapes
        m = min(nmax, n + 2 + int(rng.integers(0, nmax // 2)))
        if seed % 2:
            m, n = n, m
    A = [int(v) for v in rng.integers(1, p, m + 1)]
    B = [int(v) for v in rng.integers(1, p, n + 1)]
    if kind == 1 and m >= 2 and n >= 2:  # common factor (y - 7): a zero remainder somewhere
        A = polymul_mod([p - 7, 1], A[:m], p)
        B = polymul_mod([p - 7, 1], B[:n], p)
    if kind == 2:  # small alphabet: remainders that drop by more than one degree
        alphabet = [0, 0, 1, p - 1]
        A = [alphabet[int(v)] for v in rng.integers(0, 4, m + 1)]
        B = [alphabet[int(v)] for v in rng.integers(0, 4, n + 1)]
        A[-1] = A[-1] or 1
        B[-1] = B[-1] or 1
    if kind == 3:
        A[-1] = 0
    if kind == 4:
        B[-1] = 0
    got, bad = ures(hs, p, A, B, "long%d" % nmax)
    assert got == sylvester_det_mod(A, B, p), (m, n, kind)
    assert bad == (A[-1] == 0 or B[-1] == 0)
