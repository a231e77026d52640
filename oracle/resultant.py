"""Resultant of two bivariate integer polynomials as a Sylvester determinant over Z[x].

Test infrastructure only (see the package docstring).  Parity status: pinned --
against the Leibniz expansion on tiny inputs, against sympy's ``resultant`` on
small random inputs, against closed forms (linear cases, constant cases,
res_y(y - a(x), g) = g(x, a(x))) and against resultant identities
(antisymmetry, multiplicativity, scaling, row-operation invariance,
common-root divisibility); see ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

from itertools import permutations

from .poly import ExactDivisor, bivar_transpose, bivar_trim, pmul, pmulsub, psub, ptrim


def _ycoeffs(F):
    """Rows of a trimmed bivariate array: F[j] = f_j^(y)(x) in Z[x] (paper Sec. 2)."""
    return bivar_trim(F)


def sylvester(fy, gy):
    """Sylvester matrix S^(y)(f, g) over Z[x] (paper Sec. 3.1, the displayed S^(y)).

    ``fy[j]`` / ``gy[j]`` are the coefficients of y^j (polynomials in x), with
    the top entries nonzero so that m_y = len(fy) - 1 and n_y = len(gy) - 1
    are the actual y-degrees.  Rows 0..n_y-1 hold f, shifted one column per
    row, highest y-power first; rows n_y..n_y+m_y-1 hold g the same way.
    """
    my, ny = len(fy) - 1, len(gy) - 1
    r = my + ny
    S = [[[] for _ in range(r)] for _ in range(r)]
    for i in range(ny):
        for t in range(my + 1):
            S[i][i + t] = list(fy[my - t])
    for l in range(my):
        for t in range(ny + 1):
            S[ny + l][l + t] = list(gy[ny - t])
    return S


def _l1(a):
    return sum(abs(c) for c in a)


def bareiss_det(M):
    """Determinant of a square matrix over Z[x] by fraction-free elimination (Bareiss).

    With row pivoting when a pivot vanishes (each swap flips the sign).  Every
    step divides by the previous pivot; the division is exact in Z[x] and is
    verified (``ExactDivisor`` re-multiplies), so an inexact step raises.
    Returns the determinant as a trimmed coefficient list.
    """
    r = len(M)
    if r == 0:
        return [1]
    M = [[ptrim(e) for e in row] for row in M]
    if r == 1:
        return M[0][0]
    # Per-row weight for the Hadamard-type bound on every intermediate minor:
    # on |x| = 1 an entry is at most its coefficient 1-norm in absolute value.
    rho = [sum(_l1(e) ** 2 for e in row) for row in M]
    sign = 1
    prev = [1]
    perm = list(range(r))
    for k in range(r - 1):
        if not M[k][k]:
            piv = next((i for i in range(k + 1, r) if M[i][k]), None)
            if piv is None:
                return []
            M[k], M[piv] = M[piv], M[k]
            perm[k], perm[piv] = perm[piv], perm[k]
            sign = -sign
        div = ExactDivisor(prev)
        lead_bits = sum(rho[perm[t]].bit_length() for t in range(k + 1))
        akk = M[k][k]
        rowk = M[k]
        for i in range(k + 1, r):
            aik = M[i][k]
            qbits = (lead_bits + rho[perm[i]].bit_length() + 1) // 2 + 1
            rowi = M[i]
            for j in range(k + 1, r):
                num = pmulsub(akk, rowi[j], aik, rowk[j])
                rowi[j] = div.div(num, qbits)
            rowi[k] = []
        prev = akk
    det = M[r - 1][r - 1]
    return det if sign > 0 else psub([], det)


def res(F, G, var="y"):
    """res(f, g, var) in Z[x] (var='y') or Z[y] (var='x') as a trimmed coefficient list.

    Conventions where the paper is silent: a zero input gives the zero
    polynomial ``[]``; two inputs constant in ``var`` give ``[1]`` (empty
    determinant); the actual degrees in ``var`` are used (zero padding is
    trimmed), as in the paper's definition of m_y and n_y (Sec. 2).
    """
    if var == "x":
        F, G = bivar_transpose(F), bivar_transpose(G)
    elif var != "y":
        raise ValueError("var must be 'x' or 'y'")
    fy, gy = _ycoeffs(F), _ycoeffs(G)
    if not fy or not gy:
        return []
    return ptrim(bareiss_det(sylvester(fy, gy)))


def res_y(F, G):
    return res(F, G, "y")


def res_x(F, G):
    return res(F, G, "x")


def leibniz_det(M):
    """Determinant over Z[x] by the permutation expansion (brute force, r <= 7)."""
    r = len(M)
    if r == 0:
        return [1]
    acc = []
    for perm in permutations(range(r)):
        inv = 0
        for a in range(r):
            for b in range(a + 1, r):
                if perm[a] > perm[b]:
                    inv += 1
        term = [1]
        for row, col in enumerate(perm):
            term = pmul(term, M[row][col])
            if not term:
                break
        if term:
            acc = psub(acc, term) if inv & 1 else psub(acc, psub([], term))
    return ptrim(acc)


def degree_bound(F, G, var="y"):
    """Upper bound on deg R: min(n_y m_x + m_y n_x, n_y m + m_y n - m_y n_y).

    The first term bounds each product of n_y entries of f-rows and m_y
    entries of g-rows by their x-degrees; the second is the same count with
    the x-degree of the coefficient of y^k bounded by (total degree - k), which
    gives m*n when m_y = m and n_y = n (paper Sec. 3.1: deg R <= m n).
    Returns -1 for a zero input.
    """
    if var == "x":
        F, G = bivar_transpose(F), bivar_transpose(G)
    F, G = bivar_trim(F), bivar_trim(G)
    if not F or not G:
        return -1
    my, ny = len(F) - 1, len(G) - 1
    mx = max(len(r) for r in F) - 1
    nx = max(len(r) for r in G) - 1
    m = max(j + len(r) - 1 for j, r in enumerate(F) if r)
    n = max(j + len(r) - 1 for j, r in enumerate(G) if r)
    return min(ny * mx + my * nx, ny * m + my * n - my * ny)


def hadamard_bound_sq(F, G, var="y"):
    """B^2 = (sum_j ||f_j||_1^2)^n_y (sum_j ||g_j||_1^2)^m_y, with |coeff of R| <= B.

    On |x| = 1 each Sylvester row has 2-norm at most sqrt(sum_j ||f_j||_1^2)
    (or the g analogue); Hadamard's inequality bounds |R(x)| there, and every
    coefficient of R is a Fourier coefficient on the unit circle.
    """
    if var == "x":
        F, G = bivar_transpose(F), bivar_transpose(G)
    F, G = bivar_trim(F), bivar_trim(G)
    if not F or not G:
        return 0
    my, ny = len(F) - 1, len(G) - 1
    sf = sum(_l1(r) ** 2 for r in F)
    sg = sum(_l1(r) ** 2 for r in G)
    return sf ** ny * sg ** my
