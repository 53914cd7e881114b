"""Pins of the SYRK, TRMM and TRSM oracle (fip_oracle_l3.c) against what mathematics fixes,
each independent of the oracle's own loops:

- small-integer operands: the result is exact, compared with Python integer arithmetic on
  triangles built by NumPy's tril / triu (SYRK: op(A) @ op(A).T; TRMM: op(T) @ B, B @ op(T));
- fractions.Fraction brute force on every tiny shape: within gamma_k of the exact value;
- structure: SYRK's other triangle of C is left alone bit for bit, lower and upper results are
  transposes of each other bit for bit (the same products in the same order); TRMM never reads
  the other triangle of A (nor a unit diagonal): NaN there leaves the result finite;
- identity: a unit-diagonal T with NaN everywhere it is not read gives alpha B + beta C0;
- storage: a row-major call equals the column-major call on the same memory with the
  transposes swapped (index plumbing checked against a second route);
- TRSM: integer systems (integer X times an integer triangle with a +-1 diagonal) solved
  exactly, tiny diagonally dominant systems within a few roundings per step of the exact
  rational solution (Fraction Gauss-Jordan), alpha = 0 reads nothing.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

U64 = 2.0 ** -53


def stored(layout, rows, cols, values, ld=None, pad=np.nan):
    ld = ld or synth.min_ld(layout, rows, cols)
    return synth.fill_stored(layout, rows, cols, ld, values, np.float64, pad), ld


def view(buf, layout, rows, cols, ld):
    return synth.op_view(buf, layout, "N", rows, cols, ld)


def tri(values, uplo, diag):
    """T from a square array by NumPy's own triangle routines."""
    T = np.tril(values) if uplo == "L" else np.triu(values)
    if diag == "U":
        T = T.copy()
        np.fill_diagonal(T, 1)
    return T


# ---------------------------------------------------------------- SYRK

@pytest.mark.parametrize("layout,uplo,trans", list(itertools.product([COL, ROW], "LU", "NT")))
def test_syrk_integer_exact(layout, uplo, trans):
    g = synth.rng(3)
    n, k = 23, 31
    opA = g.integers(-8, 9, size=(n, k))
    C0 = g.integers(-8, 9, size=(n, n))
    A, lda = stored(layout, *((k, n) if trans == "T" else (n, k)),
                    opA.T if trans == "T" else opA, pad=np.nan)
    C, ldc = stored(layout, n, n, C0, ld=n + 3)
    Cref, D = oracle.syrk(layout, uplo, trans, n, k, 3.0, A, lda, -2.0, C, ldc)
    full = 3 * (opA @ opA.T) - 2 * C0
    got = view(Cref, layout, n, n, ldc)
    mask = np.tril(np.ones((n, n), bool)) if uplo == "L" else np.triu(np.ones((n, n), bool))
    assert np.array_equal(got[mask], full[mask].astype(np.float64))
    # the other triangle and the ld padding keep C0's bits
    other = np.ones(C.size, bool)
    view(other.reshape(-1), layout, n, n, ldc)[mask] = False
    assert np.array_equal(Cref[other].view(np.uint64), C[other].view(np.uint64))
    dfull = 3 * (np.abs(opA) @ np.abs(opA).T) + 2 * np.abs(C0)
    assert np.array_equal(view(D, layout, n, n, ldc)[mask], dfull[mask].astype(np.float64))


def test_syrk_lower_and_upper_are_transposes_bitwise():
    g = synth.rng(4)
    n, k = 37, 29
    A, lda = stored(COL, n, k, g.uniform(-1, 1, (n, k)))
    C0 = g.uniform(-1, 1, (n, n))
    C0 = C0 + C0.T
    C, ldc = stored(COL, n, n, C0)
    L, _ = oracle.syrk(COL, "L", "N", n, k, 1.5, A, lda, 0.5, C, ldc)
    Up, _ = oracle.syrk(COL, "U", "N", n, k, 1.5, A, lda, 0.5, C, ldc)
    Lv, Uv = view(L, COL, n, n, ldc), view(Up, COL, n, n, ldc)
    il = np.tril_indices(n)
    assert np.array_equal(Lv[il], Uv.T[il])


def test_syrk_row_major_is_column_major_of_the_transposes():
    """Row-major A (n x k, 'N') is the column-major A^T: the same memory with trans 'T' gives
    the same op(A); row-major C's lower triangle is the column-major view's upper one."""
    g = synth.rng(5)
    n, k = 19, 26
    A = g.uniform(-1, 1, n * k)
    C = g.uniform(-1, 1, n * n)
    r, _ = oracle.syrk(ROW, "L", "N", n, k, 1.25, A, k, 0.75, C, n)
    c, _ = oracle.syrk(COL, "U", "T", n, k, 1.25, A, k, 0.75, C, n)
    assert np.array_equal(r.view(np.uint64), c.view(np.uint64))


def test_syrk_fraction_bruteforce_tiny():
    g = synth.rng(6)
    for n, k in itertools.product(range(1, 5), range(0, 5)):
        opA = g.uniform(-1, 1, (n, k))
        C0 = g.uniform(-1, 1, (n, n))
        A, lda = stored(COL, n, max(k, 1), opA if k else np.zeros((n, 1)))
        C, ldc = stored(COL, n, n, C0)
        Cref, D = oracle.syrk(COL, "L", "N", n, k, 0.7, A, lda, -1.3, C, ldc)
        got = view(Cref, COL, n, n, ldc)
        dd = view(D, COL, n, n, ldc)
        gam = k * U64 / (1 - k * U64) + 3 * U64
        for i in range(n):
            for j in range(i + 1):
                s = sum((Fraction(opA[i, p]) * Fraction(opA[j, p]) for p in range(k)), Fraction(0))
                exact = Fraction(0.7) * s + Fraction(-1.3) * Fraction(C0[i, j])
                assert abs(Fraction(got[i, j]) - exact) <= Fraction(gam) * Fraction(dd[i, j]) * 2


def test_syrk_beta_zero_and_alpha_zero_read_nothing():
    n, k = 6, 4
    A, lda = stored(COL, n, k, np.full((n, k), np.nan))
    C, ldc = stored(COL, n, n, np.full((n, n), 2.0))
    Cref, _ = oracle.syrk(COL, "U", "N", n, k, 0.0, A, lda, 0.5, C, ldc)
    assert np.all(np.triu(view(Cref, COL, n, n, ldc)) == np.triu(np.full((n, n), 1.0)))
    A2, _ = stored(COL, n, k, np.ones((n, k)))
    C2, _ = stored(COL, n, n, np.full((n, n), np.nan))
    Cref, _ = oracle.syrk(COL, "L", "N", n, k, 1.0, A2, lda, 0.0, C2, ldc)
    assert np.all(view(Cref, COL, n, n, ldc)[np.tril_indices(n)] == 4.0)


# ---------------------------------------------------------------- TRMM

CASES = list(itertools.product([COL, ROW], "LR", "LU", "NT", "NU"))


@pytest.mark.parametrize("layout,side,uplo,trans,diag", CASES)
def test_trmm_integer_exact_and_unreferenced_entries(layout, side, uplo, trans, diag):
    g = synth.rng(11)
    m, n = 17, 13
    ka = m if side == "L" else n
    Avals = g.integers(-8, 9, size=(ka, ka)).astype(np.float64)
    T = tri(Avals, uplo, diag)
    # what TRMM must not read is NaN: the other triangle, and the diagonal when it is unit
    Apoison = Avals.copy()
    notref = ~(np.tril(np.ones((ka, ka), bool)) if uplo == "L" else np.triu(np.ones((ka, ka), bool)))
    if diag == "U":
        notref |= np.eye(ka, dtype=bool)
    Apoison[notref] = np.nan
    A, lda = stored(layout, ka, ka, Apoison, ld=ka + 2)
    Bv = g.integers(-8, 9, size=(m, n))
    B, ldb = stored(layout, m, n, Bv.astype(np.float64), ld=(m if layout == COL else n) + 1)
    C0 = g.integers(-8, 9, size=(m, n))
    C, ldc = stored(layout, m, n, C0.astype(np.float64))
    Cref, D = oracle.trmm(layout, side, uplo, trans, diag, m, n, 2.0, A, lda, B, ldb, -3.0, C,
                          ldc)
    opT = (T.T if trans == "T" else T).astype(np.int64)
    prod = opT @ Bv if side == "L" else Bv @ opT
    expect = (2 * prod - 3 * C0).astype(np.float64)
    got = view(Cref, layout, m, n, ldc)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, expect)
    absprod = np.abs(opT) @ np.abs(Bv) if side == "L" else np.abs(Bv) @ np.abs(opT)
    assert np.array_equal(view(D, layout, m, n, ldc), (2 * absprod + 3 * np.abs(C0)).astype(float))


def test_trmm_unit_identity():
    g = synth.rng(12)
    m, n = 9, 7
    for side, uplo in itertools.product("LR", "LU"):
        ka = m if side == "L" else n
        # the diagonal (unit) and the other triangle are not read: NaN; the referenced strict
        # triangle is zero, so T = I
        Avals = np.full((ka, ka), np.nan)
        Avals[np.tril_indices(ka, -1) if uplo == "L" else np.triu_indices(ka, 1)] = 0.0
        A, lda = stored(COL, ka, ka, Avals)
        Bv = g.uniform(-1, 1, (m, n))
        B, ldb = stored(COL, m, n, Bv)
        C0 = g.uniform(-1, 1, (m, n))
        C, ldc = stored(COL, m, n, C0)
        Cref, _ = oracle.trmm(COL, side, uplo, "N", "U", m, n, 1.5, A, lda, B, ldb, 0.25, C, ldc)
        assert np.array_equal(view(Cref, COL, m, n, ldc), 1.5 * Bv + 0.25 * C0)


def test_trmm_fraction_bruteforce_tiny():
    g = synth.rng(13)
    for m, n, side, uplo, trans in itertools.product(range(1, 4), range(1, 4), "LR", "LU", "NT"):
        ka = m if side == "L" else n
        Av = g.uniform(-1, 1, (ka, ka))
        T = tri(Av, uplo, "N")
        opT = T.T if trans == "T" else T
        Bv = g.uniform(-1, 1, (m, n))
        C0 = g.uniform(-1, 1, (m, n))
        A, lda = stored(COL, ka, ka, Av)
        B, ldb = stored(COL, m, n, Bv)
        C, ldc = stored(COL, m, n, C0)
        Cref, D = oracle.trmm(COL, side, uplo, trans, "N", m, n, 0.9, A, lda, B, ldb, 1.1, C,
                              ldc)
        got, dd = view(Cref, COL, m, n, ldc), view(D, COL, m, n, ldc)
        gam = ka * U64 / (1 - ka * U64) + 3 * U64
        for i, j in itertools.product(range(m), range(n)):
            terms = (Fraction(opT[i, p]) * Fraction(Bv[p, j]) for p in range(ka)) \
                if side == "L" else \
                (Fraction(Bv[i, p]) * Fraction(opT[p, j]) for p in range(ka))
            exact = Fraction(0.9) * sum(terms, Fraction(0)) + Fraction(1.1) * Fraction(C0[i, j])
            assert abs(Fraction(got[i, j]) - exact) <= 2 * Fraction(gam) * Fraction(dd[i, j])


def test_trmm_row_major_is_column_major_with_sides_swapped():
    """Row-major storage is the transposed column-major view of the same memory: a row-major
    TRMM (side s, uplo u) equals the column-major one on the same buffers with the side and
    the triangle swapped and m, n exchanged."""
    g = synth.rng(14)
    m, n = 11, 8
    for side, uplo, trans, diag in itertools.product("LR", "LU", "NT", "NU"):
        ka = m if side == "L" else n
        A = g.uniform(-1, 1, ka * ka)
        B = g.uniform(-1, 1, m * n)
        C = g.uniform(-1, 1, m * n)
        r, _ = oracle.trmm(ROW, side, uplo, trans, diag, m, n, 1.5, A, ka, B, n, 0.5, C, n)
        c, _ = oracle.trmm(COL, "R" if side == "L" else "L", "U" if uplo == "L" else "L", trans,
                           diag, n, m, 1.5, A, ka, B, n, 0.5, C, n)
        assert np.array_equal(r.view(np.uint64), c.view(np.uint64)), (side, uplo, trans, diag)


# ---------------------------------------------------------------- TRSM
#
# The oracle solves op(T) X = alpha B (side L) or X op(T) = alpha B (side R) by substitution.
# Pins: exact solutions of integer systems built by multiplying an integer X with an integer
# triangle of +-1 diagonal (every step of the substitution is an exact integer operation);
# exact rational solutions (Fraction) on tiny systems; what the solve never reads; alpha = 0;
# and the row-major / column-major identity.

def _tri_system(g, ka, uplo, diag, ints=True):
    if ints:
        Av = g.integers(-3, 4, size=(ka, ka)).astype(np.float64)
        np.fill_diagonal(Av, g.choice([-1.0, 1.0], size=ka))
    else:
        # strongly diagonally dominant: |off-diagonal row sum| < |diagonal| / 2
        Av = g.uniform(-1, 1, (ka, ka)) / (2 * ka)
        np.fill_diagonal(Av, g.choice([-1.0, 1.0], size=ka) * g.uniform(1, 2, size=ka))
    return Av, tri(Av, uplo, diag)


@pytest.mark.parametrize("layout,side,uplo,trans,diag", CASES)
def test_trsm_integer_systems_exact(layout, side, uplo, trans, diag):
    """alpha B = op(T) X (or X op(T)) for integer X: the oracle returns X exactly; the other
    triangle, and a unit diagonal, are NaN (never read)."""
    g = synth.rng(31)
    m, n = 15, 11
    ka = m if side == "L" else n
    Av, T = _tri_system(g, ka, uplo, diag)
    notref = ~(np.tril(np.ones((ka, ka), bool)) if uplo == "L" else np.triu(np.ones((ka, ka), bool)))
    if diag == "U":
        notref |= np.eye(ka, dtype=bool)
    Apoison = Av.copy()
    Apoison[notref] = np.nan
    A, lda = stored(layout, ka, ka, Apoison, ld=ka + 3)
    X = g.integers(-5, 6, size=(m, n)).astype(np.int64)
    opT = (T.T if trans == "T" else T).astype(np.int64)
    rhs = opT @ X if side == "L" else X @ opT          # = alpha B with alpha = 0.5
    B, ldb = stored(layout, m, n, (2 * rhs).astype(np.float64), ld=(m if layout == COL else n) + 2)
    got = oracle.trsm(layout, side, uplo, trans, diag, m, n, 0.5, A, lda, B, ldb)
    assert np.array_equal(view(got, layout, m, n, ldb), X.astype(np.float64))
    # the ld padding of X is B's, untouched
    mask = np.ones(got.size, bool)
    if layout == COL:
        mask.reshape(n, ldb)[:, :m] = False
    else:
        mask.reshape(m, ldb)[:, :n] = False
    assert np.array_equal(got[mask], B[mask], equal_nan=True)


def test_trsm_fraction_bruteforce_tiny():
    """Exact rational solution of every tiny diagonally dominant system: the oracle is within
    a few roundings per step of it."""
    g = synth.rng(32)
    for m, n, side, uplo, trans, diag in itertools.product(range(1, 4), range(1, 4), "LR", "LU",
                                                          "NT", "NU"):
        ka = m if side == "L" else n
        Av, T = _tri_system(g, ka, uplo, diag, ints=False)
        opT = [[Fraction(v) for v in row] for row in (T.T if trans == "T" else T)]
        Bv = g.uniform(-1, 1, (m, n))
        A, lda = stored(COL, ka, ka, Av)
        B, ldb = stored(COL, m, n, Bv)
        got = view(oracle.trsm(COL, side, uplo, trans, diag, m, n, 1.25, A, lda, B, ldb),
                   COL, m, n, ldb)
        # exact solve, one right-hand side at a time, by Fraction elimination (Gauss-Jordan
        # on the small dense system S x = alpha b, S = op(T) or op(T)^T)
        S = opT if side == "L" else [list(r) for r in zip(*opT)]
        for v in range(n if side == "L" else m):
            b = [Fraction(1.25) * Fraction(Bv[r, v] if side == "L" else Bv[v, r]) for r in range(ka)]
            M = [S[r][:] + [b[r]] for r in range(ka)]
            for c in range(ka):
                piv = M[c][c]
                M[c] = [x / piv for x in M[c]]
                for r in range(ka):
                    if r != c and M[r][c] != 0:
                        f = M[r][c]
                        M[r] = [x - f * y for x, y in zip(M[r], M[c])]
            exact = [M[r][ka] for r in range(ka)]
            xmax = max(abs(x) for x in exact)
            for r in range(ka):
                gv = got[r, v] if side == "L" else got[v, r]
                assert abs(Fraction(gv) - exact[r]) <= 16 * (ka + 2) * Fraction(U64) * xmax, \
                    (m, n, side, uplo, trans, diag)


def test_trsm_alpha_zero_reads_nothing():
    A = np.full(25, np.nan)
    B = np.full(5 * 4, np.nan)
    X = oracle.trsm(COL, "L", "L", "N", "N", 5, 4, 0.0, A, 5, B, 5)
    assert np.array_equal(X, np.zeros(20))


def test_trsm_row_major_is_column_major_with_sides_swapped():
    g = synth.rng(33)
    m, n = 9, 7
    for side, uplo, trans, diag in itertools.product("LR", "LU", "NT", "NU"):
        ka = m if side == "L" else n
        Av, _ = _tri_system(g, ka, uplo, diag, ints=False)
        A = Av.reshape(-1)
        B = g.uniform(-1, 1, m * n)
        r = oracle.trsm(ROW, side, uplo, trans, diag, m, n, 1.5, A, ka, B, n)
        c = oracle.trsm(COL, "R" if side == "L" else "L", "U" if uplo == "L" else "L", trans,
                        diag, n, m, 1.5, A, ka, B, n)
        assert np.array_equal(r.view(np.uint64), c.view(np.uint64)), (side, uplo, trans, diag)
