"""Pins of the oracle against what mathematics fixes (no GPU needed).

The oracle (oracle/fip_oracle.c) is the plain definition
    Cref = alpha * op(A) op(B) + beta * C0        (paper Sec. 2.1, with BLAS alpha/beta/op)
plus a per-entry bound D and a reference pack (Sec. 2.1-2.2).  Nothing here
re-types its loops: each check reaches the expected value by another route
(identity / permutation matrices, exact integer products through NumPy's
integer matmul on NumPy views of the stored buffers, exact rational brute
force with fractions.Fraction, invariants).
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


def run_oracle(c: synth.GemmCase):
    return oracle.gemm(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B, c.ldb,
                       c.transB, c.beta, c.C, c.ldc)


def opv(c, which):
    if which == "A":
        return synth.op_view(c.A, c.layout, c.transA, c.m, c.k, c.lda)
    if which == "B":
        return synth.op_view(c.B, c.layout, c.transB, c.k, c.n, c.ldb)
    return synth.op_view(c.C, c.layout, "N", c.m, c.n, c.ldc)


def cview(buf, c):
    return synth.op_view(buf, c.layout, "N", c.m, c.n, c.ldc)


def set_op(c, which, values):
    """Overwrite the stored operand so that op(X) == values (ld padding stays NaN)."""
    if which == "A":
        t, (r, cc), ld = c.transA, (c.m, c.k), c.lda
    else:
        t, (r, cc), ld = c.transB, (c.k, c.n), c.ldb
    sr, sc = synth.stored_shape(t, r, cc)
    stored = values.T if synth.is_trans(t) else values
    buf = synth.fill_stored(c.layout, sr, sc, ld, stored, np.float64)
    if which == "A":
        c.A = buf
    else:
        c.B = buf


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("T", "N"), ("N", "T"), ("C", "C")])
@pytest.mark.parametrize("pad", [0, 7])
def test_identity_left_and_right(layout, tA, tB, pad):
    c = synth.make_case(layout, 13, 9, 13, tA, tB, ld_pad=pad, alpha=1.0, beta=0.0,
                        seed=11 + pad)
    c.C[:] = np.nan  # beta = 0: C0 must not be read
    set_op(c, "A", np.eye(13))
    Cref, D = run_oracle(c)
    assert np.array_equal(cview(Cref, c), opv(c, "B"))
    c2 = synth.make_case(layout, 9, 11, 11, tA, tB, ld_pad=pad, alpha=1.0, beta=0.0, seed=12)
    c2.C[:] = np.nan
    set_op(c2, "B", np.eye(11))
    Cref2, _ = run_oracle(c2)
    assert np.array_equal(cview(Cref2, c2), opv(c2, "A"))


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("T", "T"), ("N", "C"), ("T", "N")])
def test_permutation_exact(layout, tA, tB):
    m = 17
    g = synth.rng(5)
    perm = g.permutation(m)
    P = np.zeros((m, m))
    P[np.arange(m), perm] = 1.0  # (P X)[i] = X[perm[i]]; P is not symmetric
    c = synth.make_case(layout, m, 6, m, tA, tB, ld_pad=3, alpha=1.0, beta=0.0, seed=6)
    set_op(c, "A", P)
    Cref, _ = run_oracle(c)
    assert np.array_equal(cview(Cref, c), opv(c, "B")[perm, :])
    # right-multiplication permutes columns: (Y P)[:, j] = sum_i Y[:, i] P[i, j]
    c2 = synth.make_case(layout, 5, m, m, tA, tB, ld_pad=0, alpha=1.0, beta=0.0, seed=8)
    set_op(c2, "B", P)
    Cref2, _ = run_oracle(c2)
    inv = np.argsort(perm)
    assert np.array_equal(cview(Cref2, c2), opv(c2, "A")[:, inv])


@pytest.mark.parametrize("layout", [COL, ROW])
@pytest.mark.parametrize("tA", TRANS)
@pytest.mark.parametrize("tB", TRANS)
def test_small_integer_products_exact(layout, tA, tB):
    g = synth.rng(101)
    for trial in range(3):
        m, n, k = (int(v) for v in g.integers(1, 40, size=3))
        pad = int(g.integers(0, 2)) * 7
        c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, alpha=3.0, beta=-2.0,
                            dist="int", seed=200 + trial)
        Cref, D = run_oracle(c)
        iA = opv(c, "A").astype(np.int64)
        iB = opv(c, "B").astype(np.int64)
        iC = opv(c, "C").astype(np.int64)
        exact = 3 * (iA @ iB) - 2 * iC
        assert np.array_equal(cview(Cref, c), exact.astype(np.float64))
        dexact = 3 * (np.abs(iA) @ np.abs(iB)) + 2 * np.abs(iC)
        assert np.array_equal(cview(D, c), dexact.astype(np.float64))


def test_large_k_integer_exact():
    # entries in [-8, 8]: |sum| <= 64 k, exact in binary64 for any tested k
    c = synth.make_case(COL, 7, 5, 3000, "T", "N", alpha=1.0, beta=1.0, dist="int", seed=3)
    Cref, _ = run_oracle(c)
    exact = opv(c, "A").astype(np.int64) @ opv(c, "B").astype(np.int64) + opv(c, "C").astype(np.int64)
    assert np.array_equal(cview(Cref, c), exact.astype(np.float64))


def _frac_gemm(c):
    A, B, C = opv(c, "A"), opv(c, "B"), opv(c, "C")
    al, be = Fraction(c.alpha), Fraction(c.beta)
    out = [[None] * c.n for _ in range(c.m)]
    dd = [[None] * c.n for _ in range(c.m)]
    for i in range(c.m):
        for j in range(c.n):
            s = sum((Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(c.k)),
                    Fraction(0))
            sa = sum((abs(Fraction(float(A[i, p]))) * abs(Fraction(float(B[p, j])))
                      for p in range(c.k)), Fraction(0))
            cc = Fraction(float(C[i, j])) if c.beta != 0.0 else Fraction(0)  # beta = 0: C unread
            out[i][j] = al * s + be * cc
            dd[i][j] = abs(al) * sa + abs(be) * abs(cc)
    return out, dd


def test_fraction_bruteforce_tiny_shapes():
    """Exact rational result on every tiny shape: |Cref - exact| <= gamma_{k+2} * D_exact."""
    g = synth.rng(77)
    dims = [0, 1, 2, 3, 5]
    count = 0
    for m, n, k in itertools.product(dims, dims, dims):
        layout = int(g.integers(0, 2))
        tA, tB = TRANS[int(g.integers(0, 3))], TRANS[int(g.integers(0, 3))]
        pad = int(g.integers(0, 2)) * 7
        alpha = float(g.uniform(-2, 2))
        beta = float(g.choice([0.0, 1.0, float(g.uniform(-2, 2))]))
        c = synth.make_case(layout, m, n, k, tA, tB, ld_pad=pad, alpha=alpha, beta=beta,
                            seed=1000 + count)
        if beta == 0.0:
            c.C = np.where(np.isnan(c.C), c.C, np.nan)
        count += 1
        Cref, D = run_oracle(c)
        if m == 0 or n == 0:
            # nothing may be written: the buffer is C0 untouched
            assert np.array_equal(Cref, c.C, equal_nan=True)
            continue
        exact, dexact = _frac_gemm(c)
        gam = Fraction(k + 2) * Fraction(U64) / (1 - Fraction(k + 2) * Fraction(U64))
        cv, dv = cview(Cref, c), cview(D, c)
        for i in range(m):
            for j in range(n):
                err = abs(Fraction(float(cv[i, j])) - exact[i][j])
                assert err <= gam * dexact[i][j], (m, n, k, i, j)
                # D is itself a rounded non-negative sum: relative error <= gamma
                assert abs(Fraction(float(dv[i, j])) - dexact[i][j]) <= gam * dexact[i][j]


def test_bound_equals_result_for_nonnegative_data():
    c = synth.make_case(ROW, 23, 19, 31, "T", "N", ld_pad=7, alpha=1.25, beta=0.75, seed=9)
    c.A, c.B, c.C = np.abs(c.A), np.abs(c.B), np.abs(c.C)
    Cref, D = run_oracle(c)
    assert np.array_equal(cview(Cref, c), cview(D, c))


@pytest.mark.parametrize("layout", [COL, ROW])
def test_alpha_zero_does_not_read_ab(layout):
    c = synth.make_case(layout, 8, 7, 6, "T", "N", ld_pad=7, alpha=0.0, beta=0.5, seed=4)
    c.A[:] = np.nan
    c.B[:] = np.nan
    Cref, D = run_oracle(c)
    assert np.array_equal(cview(Cref, c), 0.5 * opv(c, "C"))
    assert np.array_equal(cview(D, c), 0.5 * np.abs(opv(c, "C")))


@pytest.mark.parametrize("layout", [COL, ROW])
def test_beta_zero_does_not_read_c(layout):
    c = synth.make_case(layout, 8, 7, 6, "N", "T", ld_pad=0, alpha=1.0, beta=0.0, seed=4)
    c.C[:] = np.nan
    Cref, _ = run_oracle(c)
    assert np.all(np.isfinite(cview(Cref, c)))


def test_k_zero_is_scaled_c():
    c = synth.make_case(COL, 9, 4, 0, "N", "N", ld_pad=7, alpha=2.0, beta=-0.25, seed=2)
    Cref, _ = run_oracle(c)
    assert np.array_equal(cview(Cref, c), -0.25 * opv(c, "C"))


def test_padding_of_c_untouched():
    c = synth.make_case(COL, 9, 4, 5, "N", "N", ld_pad=7, seed=2, pad_value=-123.0)
    Cref, _ = run_oracle(c)
    mask = np.ones(c.C.size, dtype=bool)
    for j in range(c.n):
        mask[j * c.ldc: j * c.ldc + c.m] = False
    assert np.array_equal(Cref[mask], c.C[mask])


def test_nan_propagates_along_its_row_and_column():
    c = synth.make_case(COL, 10, 8, 12, "N", "N", alpha=1.0, beta=1.0, seed=7)
    c.A[3 + 5 * c.lda] = np.nan  # op(A)[3, 5]
    c.B[2 + 6 * c.ldb] = np.inf  # op(B)[2, 6]
    Cref, _ = run_oracle(c)
    cv = cview(Cref, c)
    assert np.all(np.isnan(cv[3, :]))
    assert np.all(~np.isfinite(cv[:, 6]))
    mask = np.ones_like(cv, dtype=bool)
    mask[3, :] = False
    mask[:, 6] = False
    assert np.all(np.isfinite(cv[mask]))


@pytest.mark.parametrize("layout", [COL, ROW])
def test_entries_match_full_reference_bitwise(layout):
    c = synth.make_case(layout, 37, 29, 41, "T", "C", ld_pad=7, seed=21)
    Cref, D = run_oracle(c)
    rows, cols = synth.sample_entries(c.m, c.n, 200, seed=3)
    v, d = oracle.gemm_entries(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B,
                               c.ldb, c.transB, c.beta, c.C, c.ldc, rows, cols)
    assert np.array_equal(v, cview(Cref, c)[rows, cols])
    assert np.array_equal(d, cview(D, c)[rows, cols])


@pytest.mark.parametrize("layout", [COL, ROW])
def test_freivalds_exact_on_integers(layout):
    c = synth.make_case(layout, 33, 27, 45, "N", "T", ld_pad=7, alpha=2.0, beta=-3.0,
                        dist="int", seed=31)
    x = synth.rng(4).choice([-1.0, 1.0], size=c.n)
    y, bound = oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B,
                                c.ldb, c.transB, c.beta, c.C, c.ldc, x)
    iA, iB, iC = (opv(c, w).astype(np.int64) for w in "ABC")
    ix = x.astype(np.int64)
    assert np.array_equal(y, (2 * (iA @ (iB @ ix)) - 3 * (iC @ ix)).astype(np.float64))
    assert np.array_equal(bound, (2 * (np.abs(iA) @ (np.abs(iB) @ np.abs(ix)))
                                  + 3 * (np.abs(iC) @ np.abs(ix))).astype(np.float64))


@pytest.mark.parametrize("layout", [COL, ROW])
def test_freivalds_finds_a_planted_error(layout):
    """A result that is right except for one entry: the probe flags exactly that entry's row,
    for an error as small as a few times the tolerance, and flags nothing on the right
    result."""
    c = synth.make_case(layout, 40, 35, 50, "T", "N", ld_pad=7, seed=37)
    Cref, _ = run_oracle(c)
    x = synth.rng(9).choice([-1.0, 1.0], size=c.n)
    y, bound = oracle.freivalds(c.layout, c.m, c.n, c.k, c.alpha, c.A, c.lda, c.transA, c.B,
                                c.ldb, c.transB, c.beta, c.C, c.ldc, x)
    tol = 4 * c.k * 2.0 ** -53 * bound + 2.0 * (c.n + c.k + 4) * 2.0 ** -53 * bound
    good = cview(Cref, c) @ x
    assert np.all(np.abs(good - y) <= tol)
    for (i, j), rel in [((0, 0), 1e-6), ((17, 34), 1e-9), ((39, 20), 50.0)]:
        bad = cview(Cref, c).copy()
        bad[i, j] += rel * bound[i]
        flagged = np.abs(bad @ x - y) > tol
        assert flagged[i] and flagged.sum() == 1, (i, j, rel)


def test_materialize_matches_numpy_views():
    for layout, t, pad in itertools.product([COL, ROW], TRANS, [0, 7]):
        c = synth.make_case(layout, 6, 5, 4, t, t, ld_pad=pad, seed=1)
        assert np.array_equal(oracle.materialize_op(layout, t, 6, 4, c.A, c.lda), opv(c, "A"))
        assert np.array_equal(oracle.materialize_op(layout, t, 4, 5, c.B, c.ldb), opv(c, "B"))


# ---------------------------------------------------------------- reference pack

def _encoded_case(layout, t, rows, cols, pad, dtype):
    """Stored buffer whose op() entry (r, c) holds 1000*r + c + 1 (so 0 marks padding)."""
    vals = (1000 * np.arange(rows)[:, None] + np.arange(cols)[None, :] + 1).astype(np.float64)
    sr, sc = synth.stored_shape(t, rows, cols)
    ld = synth.min_ld(layout, sr, sc) + pad
    stored = vals.T if synth.is_trans(t) else vals
    return synth.fill_stored(layout, sr, sc, ld, stored, dtype), ld, vals


def _storage_runs_along_mn(buf, layout, t, rows, cols, ld, is_b):
    """Independent route to the orientation: NumPy's own strides of the op() view."""
    v = synth.op_view(buf, layout, t, rows, cols, ld)
    mn_axis = 1 if is_b else 0
    return v.strides[mn_axis] == v.itemsize and v.strides[1 - mn_axis] != v.itemsize


def test_orientation_rule_matches_numpy_strides():
    for is_b, layout, t in itertools.product([0, 1], [COL, ROW], TRANS):
        rows, cols = (7, 5) if is_b else (5, 7)
        buf, ld, _ = _encoded_case(layout, t, rows, cols, 3, np.float64)
        assert oracle.mn_contiguous(is_b, layout, t) == \
            _storage_runs_along_mn(buf, layout, t, rows, cols, ld, is_b)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_pack_block_structure_bruteforce(dtype):
    """Every (mn, k) <= 9, (MNT, KT) in {1..4}^2 (so every (MT, NT, KT) in {1..4}^3 over the
    two operands), both operands, all layouts/trans:
    reshaping the packed buffer to (tiles, ksteps, KT, MNT) for operands stored along MN,
    or (tiles, ksteps, MNT, KT) for operands stored along k, must expose op(X) tile by
    tile with zero fill outside op(X)."""
    for mn, k, MNT, KT in itertools.product(range(0, 10), range(0, 10), range(1, 5), range(1, 5)):
        for layout, t, is_b in itertools.product([COL, ROW], ["N", "T"], [0, 1]):
            rows, cols = (k, mn) if is_b else (mn, k)
            buf, ld, vals = _encoded_case(layout, t, rows, cols, 3, dtype)
            out = oracle.pack(buf, is_b, layout, t, mn, k, ld, MNT, KT)
            nt, nk = -(-mn // MNT), -(-k // KT)
            assert out.size == nt * nk * MNT * KT
            if out.size == 0:
                continue
            # op(X) oriented as (mn, k), zero padded to the tile grid
            opx = vals.T if is_b else vals
            padded = np.zeros((nt * MNT, nk * KT))
            padded[:mn, :k] = opx
            tiles = padded.reshape(nt, MNT, nk, KT).transpose(0, 2, 1, 3)  # (nt, nk, MNT, KT)
            mn_major = (layout == COL) != (t == "T") if not is_b else (layout == COL) == (t == "T")
            if mn_major:
                got = out.reshape(nt, nk, KT, MNT).transpose(0, 1, 3, 2)
            else:
                got = out.reshape(nt, nk, MNT, KT)
            assert np.array_equal(got.astype(np.float64), tiles), (mn, k, MNT, KT, layout, t, is_b)


def test_pack_is_a_bit_copy():
    vals = np.array([-0.0, np.nan, 5e-324, -np.inf, 1.0, -2.5], dtype=np.float64)
    bits = vals.view(np.uint64).copy()
    bits[1] = 0x7FF8DEADBEEF0001  # NaN with a payload
    X = bits.view(np.float64).reshape(2, 3)  # op(A) = X (2 x 3), col-major stored
    buf = synth.fill_stored(COL, 2, 3, 2, X, np.float64)
    out = oracle.pack(buf, 0, COL, "N", 2, 3, 2, 4, 4)
    o = out.view(np.uint64).reshape(1, 1, 4, 4)
    for i in range(2):
        for p in range(3):
            assert o[0, 0, p, i] == X.view(np.uint64)[i, p]
    assert o[0, 0, 3, :].sum() == 0 and o[0, 0, :, 2:].sum() == 0  # +0.0 padding bits


def test_unpack_of_pack_is_op():
    g = synth.rng(8)
    for layout, t in itertools.product([COL, ROW], TRANS):
        m, k, MT, KT = 45, 37, 16, 8
        c = synth.make_case(layout, m, 1, k, t, "N", ld_pad=7, seed=int(g.integers(1 << 30)))
        out = oracle.pack(c.A, 0, layout, t, m, k, c.lda, MT, KT)
        nt, nk = -(-m // MT), -(-k // KT)
        if _storage_runs_along_mn(c.A, layout, t, m, k, c.lda, 0):
            blocks = out.reshape(nt, nk, KT, MT).transpose(0, 3, 1, 2)  # (nt, MT, nk, KT)
        else:
            blocks = out.reshape(nt, nk, MT, KT).transpose(0, 2, 1, 3)
        back = blocks.reshape(nt * MT, nk * KT)
        assert np.array_equal(back[:m, :k], opv(c, "A"))
        assert not back[m:, :].any() and not back[:, k:].any()
