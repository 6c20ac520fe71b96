"""Oracle: minimal matrix generator and rank read-out.

Section 2.5 ("Block Wiedemann Rank Algorithm", steps 3 and 4) computes the
minimal matrix generator F(x) in F^{s x s}[x] of the sequence {S_k} and returns
rank = deg det F - codeg det F.  In Popov form deg det F is the sum of the row
degrees; the codegree is 0 when det F(0) != 0, and otherwise comes from the low
coefficients of det F (the paper suggests interpolating only those).
Section 2.4 computes the generator through a sigma-basis (the PM-Basis
algorithm of Giorgi, Jeannerod and Villard, ISSAC 2003); this oracle uses the
plain iterative sigma-basis (M-Basis, one order at a time) of the same paper,
which PM-Basis accelerates.

Conventions (the paper leaves them to the cited work):

* S(x) = sum_{k<L} S_k x^k and G(x) = [S(x); -I_s] (2s x s).  A row [p, r] of
  an order-L sigma-basis satisfies p S - r = 0 mod x^L.
* Shift t = (0^s, 1^s): a row's shifted degree is delta = max(deg p, deg r + 1).
* The generator is made of the s basis rows of smallest shifted degree (ties:
  smaller row index).  Row i of F is the reversal of p_i by delta_i:
  F_i(x) = x^delta_i p_i(1/x), so that sum_j F_{i,j} S_{l+j} = 0 for all
  l + delta_i <= L - 1.
* Popov form: rows have a pivot = the rightmost entry of maximal degree,
  pivots are monic, lie in distinct columns, row i holds the pivot of column
  i, and every other entry of a pivot column has smaller degree than the pivot.

Pins (CPU tests): s = 1 against textbook Berlekamp-Massey and against the
brute-force minimal polynomial of B by dense Krylov vectors; the Popov row
degrees against the kernel dimensions of block Hankel matrices (brute-force
linear algebra); annihilation on extra sequence terms; codegree by local Smith
form against det F by evaluation and interpolation; the read-out against
rank(B^n) by dense powering and against the rank by elimination.

Everything uses Python integers or int64 arrays with a reduction after every
product (products of residues are below 2^62).
"""
from __future__ import annotations

import numpy as np


def _inv(a, p):
    a %= p
    if a == 0:
        raise ZeroDivisionError("inverse of 0 mod p")
    return pow(int(a), p - 2, p)


# --------------------------------------------------------------------------- #
# Berlekamp-Massey (scalar case, s = 1)
# --------------------------------------------------------------------------- #

def berlekamp_massey(seq, p):
    """Textbook Berlekamp-Massey over GF(p).

    Returns (ell, f) where ell is the linear complexity and f (list of ell + 1
    coefficients, low degree first, monic) is the minimal generating polynomial
    f(x) = x^ell C(1/x), so that sum_j f_j a_{i+j} = 0 for all i with
    i + ell < len(seq).  C is the connection polynomial; when deg C < ell, f is
    divisible by x^(ell - deg C).
    """
    a = [int(x) % p for x in seq]
    C = [1]
    Bp = [1]
    ell = 0
    mgap = 1
    b = 1
    for i, ai in enumerate(a):
        disc = ai
        for j in range(1, ell + 1):
            if j < len(C):
                disc = (disc + C[j] * a[i - j]) % p
        if disc == 0:
            mgap += 1
            continue
        coef = disc * _inv(b, p) % p
        T = C[:]
        need = len(Bp) + mgap
        if len(C) < need:
            C = C + [0] * (need - len(C))
        for j, bj in enumerate(Bp):
            C[j + mgap] = (C[j + mgap] - coef * bj) % p
        if 2 * ell <= i:
            ell = i + 1 - ell
            Bp = T
            b = disc
            mgap = 1
        else:
            mgap += 1
    C = (C + [0] * (ell + 1))[: ell + 1]
    f = [C[ell - j] for j in range(ell + 1)]
    return ell, f


# --------------------------------------------------------------------------- #
# polynomial matrices: arrays of shape (deg + 1, rows, cols), low degree first
# --------------------------------------------------------------------------- #

def _trim(P):
    d = P.shape[0]
    while d > 1 and not P[d - 1].any():
        d -= 1
    return P[:d]


def poly_deg(coeffs):
    """Degree of a polynomial given as a 1-D coefficient array (-1 for zero)."""
    nz = np.flatnonzero(np.asarray(coeffs))
    return int(nz[-1]) if nz.size else -1


def _matmul_mod(A, B, p):
    """Constant matrix product mod p with per-product reduction (entries < 2^31)."""
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    if p < (1 << 16):
        return (A @ B) % p
    out = np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    for t in range(A.shape[1]):
        out = (out + (A[:, t:t + 1] * B[t:t + 1, :]) % p) % p
    return out


def mbasis(G, order, shift, p):
    """Iterative sigma-basis (M-Basis) of G (array (>= order, m, n)) of the given order.

    Returns (P, d): P of shape (deg + 1, m, m) with P G = 0 mod x^order, and the
    shifted row degrees d (list of m ints), starting from ``shift``.
    Each order: compute the residual coefficient, eliminate its rows in the
    order of increasing shifted degree (ties: row index) with the earlier
    non-zero rows as pivots, then multiply the pivot rows by x.
    """
    G = np.asarray(G, dtype=np.int64) % p
    m = G.shape[1]
    P = np.zeros((1, m, m), dtype=np.int64)
    P[0] = np.eye(m, dtype=np.int64)
    d = [int(x) for x in shift]
    for k in range(order):
        dp = P.shape[0]
        Delta = np.zeros((m, G.shape[2]), dtype=np.int64)
        for j in range(min(k, dp - 1) + 1):
            Delta = (Delta + _matmul_mod(P[j], G[k - j], p)) % p
        rows = sorted(range(m), key=lambda i: (d[i], i))
        pivots = []
        for i in rows:
            for q, c in pivots:
                if Delta[i, c]:
                    f = int(Delta[i, c]) * _inv(int(Delta[q, c]), p) % p
                    Delta[i] = (Delta[i] - f * Delta[q]) % p
                    P[:, i, :] = (P[:, i, :] - f * P[:, q, :]) % p
            nz = np.flatnonzero(Delta[i])
            if nz.size:
                pivots.append((i, int(nz[0])))
        if pivots:
            P = np.concatenate([P, np.zeros((1, m, m), dtype=np.int64)], axis=0)
            for q, _ in pivots:
                P[1:, q, :] = P[:-1, q, :].copy()
                P[0, q, :] = 0
                d[q] += 1
        P = _trim(P)
    return P, d


def min_generator(S, p):
    """Minimal left generator of the sequence S (array (L, s, s)) via M-Basis of [S; -I].

    Returns (F, delta, Prow) with F of shape (D + 1, s, s), F_i(x) = x^delta_i p_i(1/x),
    delta the shifted degrees of the chosen rows and Prow their p-parts (deg + 1, s, s).
    """
    S = np.asarray(S, dtype=np.int64) % p
    L, s, _ = S.shape
    G = np.zeros((L, 2 * s, s), dtype=np.int64)
    G[:, :s, :] = S
    G[0, s:, :] = (-np.eye(s, dtype=np.int64)) % p
    P, d = mbasis(G, L, [0] * s + [1] * s, p)
    chosen = sorted(range(2 * s), key=lambda i: (d[i], i))[:s]
    delta = [d[i] for i in chosen]
    Prow = P[:, chosen, :s]
    D = max(delta) if delta else 0
    F = np.zeros((D + 1, s, s), dtype=np.int64)
    for r, i in enumerate(chosen):
        if P.shape[0] > delta[r] + 1 and P[delta[r] + 1:, i, :s].any():
            raise AssertionError("p-part degree exceeds the shifted degree")
        for j in range(min(P.shape[0], delta[r] + 1)):
            F[delta[r] - j, r, :] = P[j, i, :s]
    return _trim(F), delta, Prow


def annihilates(F, S, p):
    """True when sum_j F_{i,j} S_{l+j} = 0 for every row i and every l with l + deg_i < len(S)."""
    S = np.asarray(S, dtype=np.int64) % p
    L = S.shape[0]
    s = F.shape[1]
    for i in range(s):
        di = max((j for j in range(F.shape[0]) if F[j, i].any()), default=-1)
        if di < 0:
            return False
        for l in range(0, L - di):
            acc = np.zeros(S.shape[2], dtype=np.int64)
            for j in range(di + 1):
                acc = (acc + _matmul_mod(F[j, i][None, :], S[l + j], p)[0]) % p
            if acc.any():
                return False
    return True


# --------------------------------------------------------------------------- #
# row reduction and Popov form
# --------------------------------------------------------------------------- #

def _row_pivot(F, i):
    """(degree, column) of the rightmost entry of maximal degree in row i; (-1, -1) for a zero row."""
    best = (-1, -1)
    for c in range(F.shape[2]):
        dg = poly_deg(F[:, i, c])
        if dg >= best[0] and dg >= 0:
            best = (dg, c)
    return best


def weak_popov(F, p):
    """Mulders-Storjohann simple transformations until row pivots lie in distinct columns.

    The result is row reduced, so deg det equals the sum of its row degrees.
    """
    F = np.array(F, dtype=np.int64) % p
    s = F.shape[1]
    while True:
        piv = [_row_pivot(F, i) for i in range(s)]
        clash = None
        for i in range(s):
            for j in range(s):
                if i != j and piv[i][1] >= 0 and piv[i][1] == piv[j][1] and piv[i][0] >= piv[j][0]:
                    clash = (i, j)
                    break
            if clash:
                break
        if clash is None:
            return _trim(F)
        i, j = clash
        c = piv[i][1]
        shift = piv[i][0] - piv[j][0]
        f = int(F[piv[i][0], i, c]) * _inv(int(F[piv[j][0], j, c]), p) % p
        need = F.shape[0]
        # row_i -= f x^shift row_j  (degree of row_j + shift <= degree of row_i)
        for t in range(need - shift):
            F[t + shift, i, :] = (F[t + shift, i, :] - f * F[t, j, :]) % p


def _rref(M, p):
    """Reduced row echelon form over GF(p) of a dense int matrix (list of lists); returns (rows, pivot cols)."""
    A = [[int(x) % p for x in r] for r in M]
    nrow = len(A)
    ncol = len(A[0]) if nrow else 0
    piv_cols = []
    r = 0
    for c in range(ncol):
        pr = next((i for i in range(r, nrow) if A[i][c]), None)
        if pr is None:
            continue
        A[r], A[pr] = A[pr], A[r]
        inv = _inv(A[r][c], p)
        A[r] = [(x * inv) % p for x in A[r]]
        for i in range(nrow):
            if i != r and A[i][c]:
                f = A[i][c]
                A[i] = [(x - f * y) % p for x, y in zip(A[i], A[r])]
        piv_cols.append(c)
        r += 1
        if r == nrow:
            break
    return A[:r], piv_cols


def popov_form(F, p):
    """Popov form of a nonsingular s x s polynomial matrix (tiny sizes: dense linear algebra).

    The Popov basis of the row module is its reduced Groebner basis for the
    term order "degree first, then column index" (x^d e_c > x^d' e_c' iff
    d > d', or d = d' and c > c').  After a weak Popov reduction the row module
    elements of degree <= D are the span of x^j F_i (deg F_i + j <= D); the
    reduced row echelon form of that span, with monomials ordered from the
    largest down, holds each Popov row as the echelon row whose leading
    monomial is the smallest one for its column.
    """
    W = weak_popov(F, p)
    s = W.shape[1]
    degs = [_row_pivot(W, i)[0] for i in range(s)]
    if min(degs) < 0:
        raise ValueError("singular polynomial matrix")
    D = max(degs)
    # monomial x^d e_c -> column index in "largest first" order
    def col_of(dg, c):
        return (D - dg) * s + (s - 1 - c)
    rows = []
    for i in range(s):
        for j in range(D - degs[i] + 1):
            v = [0] * ((D + 1) * s)
            for dg in range(W.shape[0]):
                for c in range(s):
                    x = int(W[dg, i, c])
                    if x and dg + j <= D:
                        v[col_of(dg + j, c)] = x
            rows.append(v)
    R, piv = _rref(rows, p)
    out_rows = {}
    for vec, pc in zip(R, piv):
        dg = D - pc // s
        c = s - 1 - pc % s
        if c not in out_rows or dg < out_rows[c][0]:
            out_rows[c] = (dg, vec)
    if len(out_rows) != s:
        raise ValueError("Popov extraction failed")
    Dp = max(dg for dg, _ in out_rows.values())
    P = np.zeros((Dp + 1, s, s), dtype=np.int64)
    for c, (dg, vec) in out_rows.items():
        for pcol, x in enumerate(vec):
            if x:
                ddg = D - pcol // s
                cc = s - 1 - pcol % s
                P[ddg, c, cc] = x
    return _trim(P)


def row_degrees(F):
    return [_row_pivot(F, i)[0] for i in range(F.shape[1])]


# --------------------------------------------------------------------------- #
# determinant valuation (codegree) and determinant by evaluation/interpolation
# --------------------------------------------------------------------------- #

def _series_inv(u, K, p):
    """Inverse of a power series with u[0] != 0, modulo x^K."""
    out = [0] * K
    inv0 = _inv(int(u[0]), p)
    for k in range(K):
        acc = 1 if k == 0 else 0
        for j in range(1, min(k, len(u) - 1) + 1):
            acc = (acc - int(u[j]) * out[k - j]) % p
        out[k] = acc * inv0 % p
    return out


def _valuation_truncated(M, K, p):
    """Sum of pivot valuations of M (array (>=1, s, s)) over GF(p)[[x]] mod x^K; None if precision ran out."""
    s = M.shape[1]
    A = [[[int(M[k, i, j]) % p if k < M.shape[0] else 0 for k in range(K)] for j in range(s)] for i in range(s)]

    def val(series):
        for k, x in enumerate(series):
            if x:
                return k
        return K

    total = 0
    for t in range(s):
        best = None
        for i in range(t, s):
            for j in range(t, s):
                v = val(A[i][j])
                if best is None or v < best[0]:
                    best = (v, i, j)
        v, bi, bj = best
        if v >= K:
            return None
        A[t], A[bi] = A[bi], A[t]
        for row in A:
            row[t], row[bj] = row[bj], row[t]
        u = A[t][t][v:]
        uinv = _series_inv(u, K - v, p)
        for i in range(t + 1, s):
            w = A[i][t][v:]
            # q = (A[i][t] / x^v) * u^{-1} mod x^(K-v)
            q = [0] * (K - v)
            for a in range(K - v):
                if w[a]:
                    for b in range(K - v - a):
                        q[a + b] = (q[a + b] + w[a] * uinv[b]) % p
            for j in range(t, s):
                src = A[t][j]
                dst = A[i][j]
                for a in range(K - v):
                    if q[a]:
                        for b in range(K - a):
                            if src[b]:
                                dst[a + b] = (dst[a + b] - q[a] * src[b]) % p
        total += v
    return total


def det_valuation(M, p, max_k=None):
    """x-adic valuation of det M for an s x s polynomial matrix, by local Smith form over GF(p)[[x]].

    Starts at precision x^4 and doubles until every pivot is found; returns
    None when det M = 0 (precision beyond ``max_k``, default s * (deg M + 1) + 1).
    """
    M = np.asarray(M, dtype=np.int64) % p
    s = M.shape[1]
    if max_k is None:
        max_k = s * M.shape[0] + 2
    K = 4
    while True:
        r = _valuation_truncated(M, K, p)
        if r is not None:
            return r
        if K > max_k:
            return None
        K *= 2


def _det_modp(A, p):
    A = [[int(x) % p for x in r] for r in A]
    n = len(A)
    det = 1
    for c in range(n):
        pr = next((i for i in range(c, n) if A[i][c]), None)
        if pr is None:
            return 0
        if pr != c:
            A[c], A[pr] = A[pr], A[c]
            det = -det
        det = det * A[c][c] % p
        inv = _inv(A[c][c], p)
        for i in range(c + 1, n):
            if A[i][c]:
                f = A[i][c] * inv % p
                A[i] = [(x - f * y) % p for x, y in zip(A[i], A[c])]
    return det % p


def det_by_interpolation(F, p):
    """det F as a coefficient list, by evaluation at deg-bound + 1 points and Lagrange interpolation."""
    F = np.asarray(F, dtype=np.int64) % p
    s = F.shape[1]
    bound = sum(max(0, r) for r in row_degrees(F)) if s else 0
    pts = list(range(1, bound + 2))
    if len(pts) >= p:
        raise ValueError("field too small for interpolation")
    vals = []
    for x0 in pts:
        E = [[sum(int(F[k, i, j]) * pow(x0, k, p) for k in range(F.shape[0])) % p for j in range(s)]
             for i in range(s)]
        vals.append(_det_modp(E, p))
    # Lagrange interpolation
    coeffs = [0] * len(pts)
    for i, (xi, yi) in enumerate(zip(pts, vals)):
        if yi == 0:
            continue
        num = [1]
        den = 1
        for j, xj in enumerate(pts):
            if j == i:
                continue
            num = [(a - xj * b) % p for a, b in zip([0] + num, num + [0])]
            den = den * (xi - xj) % p
        f = yi * _inv(den, p) % p
        for k in range(len(num)):
            coeffs[k] = (coeffs[k] + f * num[k]) % p
    return coeffs


# --------------------------------------------------------------------------- #
# the read-out
# --------------------------------------------------------------------------- #

def rank_from_generator(F, p):
    """rank = deg det F - codeg det F (Section 2.5, step 4).

    deg det F is the sum of the row degrees of a row-reduced form (weak Popov,
    which the Popov form refines); the codegree is 0 when det F(0) != 0 and
    otherwise the x-adic valuation of det F by local Smith form.
    """
    W = weak_popov(F, p)
    degs = row_degrees(W)
    if min(degs) < 0:
        raise ValueError("generator is singular")
    deg_det = sum(degs)
    if _det_modp(W[0].tolist(), p) != 0:
        return deg_det
    codeg = det_valuation(W, p)
    if codeg is None:
        raise ValueError("generator has zero determinant")
    return deg_det - codeg


def rank_from_sequence(S, p):
    """Read the rank out of a sequence: minimal generator via M-Basis, then deg det - codeg det."""
    F, _, _ = min_generator(S, p)
    return rank_from_generator(F, p)


# --------------------------------------------------------------------------- #
# brute-force pins
# --------------------------------------------------------------------------- #

def minpoly_dense(B, p):
    """Minimal polynomial of a dense n x n matrix over GF(p), by the first linear dependency
    among vec(I), vec(B), vec(B^2), ...  Returns monic coefficients, low degree first."""
    n = len(B)
    pw = [[int(i == j) for j in range(n)] for i in range(n)]
    vecs = []
    for d in range(n + 1):
        vecs.append([x for row in pw for x in row])
        # solve for a dependency of the last vector on the previous ones
        if d > 0:
            M = [list(col) for col in zip(*vecs)]  # n^2 x (d+1)
            R, piv = _rref(M, p)
            if len(piv) < d + 1:
                # kernel vector with last coordinate 1
                # columns 0..d-1 are pivots (independent), column d is free
                coef = [0] * (d + 1)
                coef[d] = 1
                for row, pc in zip(R, piv):
                    coef[pc] = (-row[d]) % p
                return coef
        pw = [[sum(pw[i][t] * int(B[t][j]) for t in range(n)) % p for j in range(n)] for i in range(n)]
    raise AssertionError("unreachable: Cayley-Hamilton")


def rank_of_power(B, p, e=None):
    """rank over GF(p) of B^e (default e = n), by dense powering."""
    n = len(B)
    e = n if e is None else e
    R = [[int(i == j) for j in range(n)] for i in range(n)]
    for _ in range(e):
        R = [[sum(R[i][t] * int(B[t][j]) for t in range(n)) % p for j in range(n)] for i in range(n)]
    _, piv = _rref(R, p) if n else ([], [])
    return len(piv)


def hankel_generator_degrees(S, p, dmax):
    """Brute-force row degrees of a minimal generator from block Hankel kernel dimensions.

    dim_d = dim{f of degree <= d : sum_j f_j S_{i+j} = 0, i = 0..L-1-d}
    = sum_i max(0, d - delta_i + 1) for a minimal generator with row degrees
    delta (predictable degree property).  Returns the sorted delta list found
    for d = 0..dmax (degrees above dmax are not reported).
    """
    S = np.asarray(S, dtype=np.int64) % p
    L, s, _ = S.shape
    dims = []
    for d in range(dmax + 1):
        rows = []
        for j in range(d + 1):
            for a in range(s):
                rows.append([int(S[i + j, a, b]) for i in range(L - d) for b in range(s)])
        _, piv = _rref(rows, p)
        dims.append(s * (d + 1) - len(piv))
    count_le = [dims[0]] + [dims[d] - dims[d - 1] for d in range(1, dmax + 1)]
    out = []
    prev = 0
    for d, c in enumerate(count_le):
        out += [d] * (c - prev)
        prev = c
    return out


def sequence_length(nb: int, s: int) -> int:
    """Number of sequence terms: 2 + ceil(2 nb / s) (step 2 of the rank algorithm in
    Section 2.5 asks for 2n/s + O(1) terms; Table "tab:r-time" counts 2 + 2r/p)."""
    return 2 + -(-2 * nb // s)
