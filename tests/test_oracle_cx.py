"""Pins of the complex-GEMM oracle (oracle/fip_oracle_cx.c) against what mathematics fixes.

The oracle writes out the BLAS complex gemm definition and the 1m expansion (the formats of
the 1m method, which the paper cites as a transformation carried out by the packing stage,
Sec. 5).  Each check reaches the expected value by another route: NumPy's complex matmul
(an independent implementation, within the rounding bound), exact Gaussian-integer products
through NumPy's integer matmul on the real and imaginary parts, exact rational brute force
with fractions.Fraction, the real oracle run on the 1m-expanded operands, and invariants
(conjugation, identity, BLAS quick-return rules).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2302_08417_amd import synth
from paper_2302_08417_amd.synth import COL, ROW

U64 = 2.0 ** -53
TRANS = ["N", "T", "C"]


def run(c):
    return oracle.zgemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                        c.transB, c.beta, c.C, c.ldc)


def cview(buf, c):
    return synth.op_view(buf, c.layout, "N", c.m, c.n, c.ldc)


def bits(z):
    return np.ascontiguousarray(z).view(np.float64)


def op(c, which):
    if which == "A":
        return synth.cx_op_view(c.A, c.layout, c.transA, c.m, c.k, c.lda)
    return synth.cx_op_view(c.B, c.layout, c.transB, c.k, c.n, c.ldb)


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", list(itertools.product(TRANS, TRANS)))
def test_matches_numpy_complex_matmul(layout, tA, tB):
    """NumPy's complex128 matmul (another summation order) agrees within the bound."""
    c = synth.make_cx_case(layout, 29, 23, 31, tA, tB, ld_pad=7, seed=100 * layout + 10 * TRANS.index(tA) + TRANS.index(tB))
    Cref, D = run(c)
    ref = c.alpha * (op(c, "A") @ op(c, "B")) + c.beta * cview(c.C, c)
    got, d = cview(Cref, c), cview(D, c)
    gam = 2 * (2 * c.k + 4) * U64
    assert np.all(np.abs(got.real - ref.real) <= gam * d)
    assert np.all(np.abs(got.imag - ref.imag) <= gam * d)


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("C", "T"), ("T", "C"), ("C", "C")])
def test_gaussian_integers_exact(layout, tA, tB):
    """Gaussian-integer operands and scalars: every product and partial sum is an integer far
    below 2^53, so the result is exact; compare with four integer matmuls of the parts."""
    c = synth.make_cx_case(layout, 37, 41, 53, tA, tB, ld_pad=3, alpha=2 - 3j, beta=-1 + 2j,
                           seed=5, dist="int")
    Cref, _ = run(c)
    a, b = op(c, "A"), op(c, "B")
    ar, ai = a.real.astype(np.int64), a.imag.astype(np.int64)
    br, bi = b.real.astype(np.int64), b.imag.astype(np.int64)
    pr, pi = ar @ br - ai @ bi, ar @ bi + ai @ br
    c0 = cview(c.C, c)
    c0r, c0i = c0.real.astype(np.int64), c0.imag.astype(np.int64)
    exp_r = 2 * pr + 3 * pi + (-1 * c0r - 2 * c0i)
    exp_i = 2 * pi - 3 * pr + (-1 * c0i + 2 * c0r)
    got = cview(Cref, c)
    assert np.array_equal(got.real, exp_r.astype(np.float64))
    assert np.array_equal(got.imag, exp_i.astype(np.float64))


def _fc(z):
    return Fraction(float(z.real)), Fraction(float(z.imag))


def test_fraction_bruteforce_tiny_shapes():
    """Exact rational complex arithmetic on every tiny shape: each component of the oracle
    lies within gamma_{2k+4} * D of the exact value (D is the oracle's own bound, checked
    here against its exact rational value too)."""
    g = synth.rng(91)
    dims = [0, 1, 2, 3]
    count = 0
    for m, n, k in itertools.product(dims, dims, dims):
        layout = int(g.integers(0, 2))
        tA, tB = TRANS[int(g.integers(0, 3))], TRANS[int(g.integers(0, 3))]
        alpha = complex(g.uniform(-2, 2), g.uniform(-2, 2))
        beta = complex(*(g.choice([0.0, 1.0]), g.uniform(-1, 1))) if count % 3 else 0j
        c = synth.make_cx_case(layout, m, n, k, tA, tB, ld_pad=int(g.integers(0, 2)) * 2,
                               alpha=alpha, beta=beta, seed=4000 + count)
        count += 1
        Cref, D = run(c)
        if m == 0 or n == 0:
            assert np.array_equal(Cref.view(np.float64), c.C.view(np.float64), equal_nan=True)
            continue
        a, b, c0 = op(c, "A"), op(c, "B"), cview(c.C, c)
        alr, ali = Fraction(alpha.real), Fraction(alpha.imag)
        ber, bei = Fraction(beta.real), Fraction(beta.imag)
        gam = Fraction(2 * k + 4) * Fraction(U64) / (1 - Fraction(2 * k + 4) * Fraction(U64))
        cv, dv = cview(Cref, c), cview(D, c)
        for i in range(m):
            for j in range(n):
                sr = si = sd = Fraction(0)
                for p in range(k):
                    xr, xi = _fc(a[i, p])
                    yr, yi = _fc(b[p, j])
                    sr += xr * yr - xi * yi
                    si += xr * yi + xi * yr
                    sd += (abs(xr) + abs(xi)) * (abs(yr) + abs(yi))
                er, ei = alr * sr - ali * si, alr * si + ali * sr
                de = (abs(alr) + abs(ali)) * sd
                if beta != 0:
                    cr, ci = _fc(c0[i, j])
                    er += ber * cr - bei * ci
                    ei += ber * ci + bei * cr
                    de += (abs(ber) + abs(bei)) * (abs(cr) + abs(ci))
                gr, gi = _fc(cv[i, j])
                assert abs(gr - er) <= gam * de, (m, n, k, i, j)
                assert abs(gi - ei) <= gam * de, (m, n, k, i, j)
                assert abs(Fraction(float(dv[i, j])) - de) <= gam * de


def test_conjugate_transpose_is_conjugated_transpose():
    """op 'C' on a stored A gives bit for bit the result of op 'N' on a stored conj(A)^T."""
    c = synth.make_cx_case(COL, 19, 17, 13, "C", "N", seed=12)
    Cref, _ = run(c)
    a_h = op(c, "A")   # conj(A)^T as a plain m x k matrix
    d = synth.make_cx_case(COL, 19, 17, 13, "N", "N", seed=12)
    d.A = synth.fill_stored(COL, c.m, c.k, c.m, a_h, np.complex128)
    d.lda = c.m
    d.B, d.ldb, d.C, d.ldc = c.B, c.ldb, c.C, c.ldc
    Dref, _ = run(d)
    assert np.array_equal(bits(cview(Cref, c)), bits(cview(Dref, d)))


def test_identity():
    """op(A) = I: C = alpha op(B) + beta C0 up to the epilogue's roundings; alpha = 1,
    beta = 0 gives op(B) exactly."""
    n = 21
    c = synth.make_cx_case(COL, n, 9, n, "N", "C", alpha=1, beta=0, seed=3)
    c.A = synth.fill_stored(COL, n, n, n, np.eye(n, dtype=np.complex128), np.complex128)
    c.lda = n
    c.C = np.full_like(c.C, complex(np.nan, np.nan))
    Cref, _ = run(c)
    assert np.array_equal(cview(Cref, c), op(c, "B"))


def test_quick_return_rules():
    """alpha = 0 reads neither A nor B (NaN there does not propagate); beta = 0 does not read
    C0 (NaN there does not propagate); k = 0 gives beta * C0."""
    c = synth.make_cx_case(COL, 7, 5, 4, "N", "N", alpha=0, beta=2 - 1j, seed=1)
    c.A[:] = complex(np.nan, np.nan)
    c.B[:] = complex(np.nan, np.nan)
    Cref, _ = run(c)
    assert np.allclose(cview(Cref, c), (2 - 1j) * cview(c.C, c), rtol=0, atol=0)
    c = synth.make_cx_case(COL, 7, 5, 4, "N", "N", alpha=1 + 1j, beta=0, seed=1)
    c.C[:] = complex(np.nan, np.nan)
    Cref, _ = run(c)
    assert np.isfinite(bits(cview(Cref, c))).all()
    c = synth.make_cx_case(COL, 7, 5, 0, "N", "N", alpha=1 + 1j, beta=0.5j, seed=1)
    Cref, _ = run(c)
    assert np.array_equal(cview(Cref, c), 0.5j * cview(c.C, c))


def test_nan_propagates_along_row_and_column():
    c = synth.make_cx_case(COL, 6, 5, 4, "N", "N", seed=2)
    c.A[2 + 1 * c.lda] = complex(0.5, np.nan)     # opA[2, 1]: imaginary part NaN
    c.B[3 + 4 * c.ldb] = complex(np.nan, 0.25)    # opB[3, 4]: real part NaN
    Cref, _ = run(c)
    bad = ~np.isfinite(bits(cview(Cref, c)).reshape(6, 5, 2)).all(axis=2)
    want = np.zeros((6, 5), bool)
    want[2, :] = True
    want[:, 4] = True
    assert np.array_equal(bad, want)


def test_entries_match_full_reference_bitwise():
    c = synth.make_cx_case(ROW, 33, 27, 19, "T", "C", ld_pad=5, seed=21)
    Cref, D = run(c)
    rows, cols = synth.sample_entries(c.m, c.n, 200, 4)
    v, d = oracle.zgemm_entries(c.layout, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                                c.transB, c.beta, c.C, c.ldc, rows, cols)
    cv, dv = cview(Cref, c), cview(D, c)
    assert np.array_equal(bits(v), bits(cv[rows, cols]))
    assert np.array_equal(d, dv[rows, cols])


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", list(itertools.product(TRANS, TRANS)))
def test_1m_real_product_is_complex_product(layout, tA, tB):
    """The real oracle on the 1m-expanded operands (A1e, 2m x 2k; B1r, 2k x n) gives the real
    view of the complex product (rows 2i, 2i+1: re, im of entry i), exactly on Gaussian
    integers."""
    c = synth.make_cx_case(layout, 11, 9, 14, tA, tB, ld_pad=2, alpha=1, beta=0, seed=31,
                           dist="int")
    Cref, _ = run(c)
    A1e = oracle.expand_1m(c.A, 0, c.layout, c.transA, c.m, c.k, c.lda)
    B1r = oracle.expand_1m(c.B, 1, c.layout, c.transB, c.n, c.k, c.ldb)
    assert A1e.shape == (2 * c.m, 2 * c.k) and B1r.shape == (2 * c.k, c.n)
    R, _ = oracle.gemm(COL, 2 * c.m, c.n, 2 * c.k, 1.0, A1e.reshape(-1, order="F"), 2 * c.m, "N",
                       B1r.reshape(-1, order="F"), 2 * c.k, "N", 0.0,
                       np.zeros(2 * c.m * c.n), 2 * c.m)
    R = R.reshape(c.n, 2 * c.m).T
    got = cview(Cref, c)
    assert np.array_equal(R[0::2, :], got.real) and np.array_equal(R[1::2, :], got.imag)


def test_1m_expansion_structure():
    """Each 2 x 2 block of A1e is [[re, -im], [im, re]] of op(A)[i, p]; column j of B1r holds
    (re, im) pairs of op(B)[:, j]."""
    c = synth.make_cx_case(ROW, 5, 4, 3, "C", "T", ld_pad=1, seed=8)
    A1e = oracle.expand_1m(c.A, 0, c.layout, c.transA, c.m, c.k, c.lda)
    a = op(c, "A")
    for i, p in itertools.product(range(c.m), range(c.k)):
        blk = A1e[2 * i:2 * i + 2, 2 * p:2 * p + 2]
        assert blk[0, 0] == a[i, p].real and blk[1, 1] == a[i, p].real
        assert blk[1, 0] == a[i, p].imag and blk[0, 1] == -a[i, p].imag
    B1r = oracle.expand_1m(c.B, 1, c.layout, c.transB, c.n, c.k, c.ldb)
    b = op(c, "B")
    assert np.array_equal(B1r[0::2, :], b.real) and np.array_equal(B1r[1::2, :], b.imag)


@pytest.mark.parametrize("is_b", [0, 1])
@pytest.mark.parametrize("layout,t", [(COL, "N"), (COL, "C"), (ROW, "N"), (ROW, "T")])
def test_pack_1m_unpacks_to_expansion(is_b, layout, t):
    """The 1m pack is the real pack of the expansion: reshaping its blocks exposes the
    expanded operand tile by tile, zero padded, in the complex operand's storage orientation."""
    mn, k, MNT, KT = 13, 11, 8, 4
    if is_b:
        c = synth.make_cx_case(layout, 1, mn, k, "N", t, ld_pad=3, seed=17)
        X, ld = c.B, c.ldb
    else:
        c = synth.make_cx_case(layout, mn, 1, k, t, "N", ld_pad=3, seed=17)
        X, ld = c.A, c.lda
    E = oracle.expand_1m(X, is_b, layout, t, mn, k, ld)
    out = oracle.pack_1m(X, is_b, layout, t, mn, k, ld, MNT, KT)
    emn, ek = (2 * mn, 2 * k) if not is_b else (mn, 2 * k)
    opx = E.T if is_b else E                      # oriented (mn, k)
    nt, nk = -(-emn // MNT), -(-ek // KT)
    padded = np.zeros((nt * MNT, nk * KT))
    padded[:emn, :ek] = opx
    tiles = padded.reshape(nt, MNT, nk, KT).transpose(0, 2, 1, 3)
    if oracle.mn_contiguous(is_b, layout, t):
        got = out.reshape(nt, nk, KT, MNT).transpose(0, 1, 3, 2)
    else:
        got = out.reshape(nt, nk, MNT, KT)
    assert np.array_equal(got, tiles)
