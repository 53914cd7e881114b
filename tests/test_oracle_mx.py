"""Pins of the oracle's number formats for the mixed-precision forms (CPU only).

Each format routine of oracle/fip_oracle_mx.c is checked against something other than
itself: torch's CPU conversions (a library routine implementing the same standard
format), closed forms on bit patterns, exhaustive round trips over every code, and exact
identities of the three-term split.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def _f32_from_bits(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


def _edge_f32():
    bits = [0x00000000, 0x80000000, 0x3F800000, 0x3F808000, 0x3F818000, 0x3F80FFFF, 0x3F817FFF,
            0x7F7FFFFF, 0xFF7FFFFF, 0x7F7F8000, 0x00000001, 0x00800000, 0x007FFFFF, 0x7F800000,
            0xFF800000, 0x3EAAAAAB, 0xBF7FFFFF, 0x33800000, 0x477FE000]
    return _f32_from_bits(bits)


def test_bf16_ties_to_even_closed_form():
    # 1 + 2^-8 is halfway between bf16 1.0 (0x3F80, even) and 0x3F81: ties go to even.
    # 0x3F818000 is halfway between 0x3F81 (odd) and 0x3F82: goes up.
    out = oracle.bf16_round(_f32_from_bits([0x3F808000, 0x3F818000, 0x3F808001, 0x3F817FFF]))
    assert out.tolist() == [0x3F80, 0x3F82, 0x3F81, 0x3F81]


def test_bf16_round_matches_torch():
    g = np.random.default_rng(1)
    x = np.concatenate([_edge_f32(), g.standard_normal(200_000).astype(np.float32) *
                        np.float32(2.0) ** g.integers(-60, 60, 200_000).astype(np.float32),
                        _f32_from_bits(g.integers(0, 2 ** 32, 200_000, dtype=np.uint64)
                                       .astype(np.uint32))])
    x = x[~np.isnan(x)]
    ours = oracle.bf16_round(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_nan_stays_nan_and_decode_is_exact():
    n = oracle.bf16_round(_f32_from_bits([0x7FC00000, 0xFFC00001, 0x7F800001]))
    assert np.all(np.isnan(oracle.bf16_decode(n)))
    g = np.random.default_rng(2)
    h = g.integers(0, 2 ** 16, 100_000).astype(np.uint16)
    h = h[(h & 0x7F80) != 0x7F80]  # finite patterns
    v = oracle.bf16_decode(h)
    ref = torch.from_numpy(h.view(np.int16).copy()).view(torch.bfloat16).double().numpy()
    assert np.array_equal(v, ref)
    # a bf16 value converts to itself
    assert np.array_equal(oracle.bf16_round(v.astype(np.float32)), h)


def test_e4m3_decode_all_codes_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.e4m3_decode(codes)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).double().numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2 and nan[0x7F] and nan[0xFF]
    assert np.array_equal(ours[~nan], ref[~nan])
    # closed forms: largest finite, smallest subnormal, one
    assert ours[0x7E] == 448.0 and ours[0x01] == 2.0 ** -9 and ours[0x38] == 1.0
    assert ours[0x08] == 2.0 ** -6 and ours[0xFE] == -448.0


def test_e4m3_round_trip_every_code():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    back = oracle.e4m3_encode(oracle.e4m3_decode(codes))
    assert np.array_equal(back, codes)


def test_e4m3_encode_matches_torch_in_range():
    g = np.random.default_rng(3)
    x = np.concatenate([g.uniform(-448, 448, 100_000),
                        g.standard_normal(100_000) * 2.0 ** g.integers(-12, 8, 100_000)])
    x = x[np.abs(x) <= 448].astype(np.float32).astype(np.float64)
    ours = oracle.e4m3_encode(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_midpoints_tie_to_even_and_saturate():
    vals = oracle.e4m3_decode(np.arange(0x7F, dtype=np.uint8))  # 0 .. 448 ascending
    assert np.all(np.diff(vals) > 0)
    mids = (vals[:-1] + vals[1:]) / 2
    enc = oracle.e4m3_encode(mids)
    lo = np.arange(0x7E, dtype=np.uint8)
    expect = np.where(lo % 2 == 0, lo, lo + 1).astype(np.uint8)
    assert np.array_equal(enc, expect)
    sat = oracle.e4m3_encode([449.0, 464.0, 1e30, np.inf, -500.0, -np.inf])
    assert sat.tolist() == [0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0xFE]
    assert oracle.e4m3_encode([np.nan])[0] & 0x7F == 0x7F


def test_fp8_scale_exponent_definition():
    g = np.random.default_rng(4)
    for amax in np.concatenate([g.uniform(0, 1, 200) * 2.0 ** g.integers(-40, 40, 200),
                                [448.0, 449.0, 1.0, 447.99, 896.0, 224.0]]):
        e = oracle.fp8_scale_exponent(amax)
        assert amax * 2.0 ** e <= 448.0 < amax * 2.0 ** (e + 1), (amax, e)
    assert oracle.fp8_scale_exponent(0.0) == 0
    assert oracle.fp8_scale_exponent(1e-300) == 126  # clamped
    assert oracle.fp8_scale_exponent(1e300) == -126


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("axis", [0, 1])
def test_quantize_fp8_lines(layout, axis):
    g = np.random.default_rng(5 + 2 * layout + axis)
    rows, cols, pad = 37, 23, 3
    X = (g.uniform(-1, 1, (rows, cols)) * 2.0 ** g.uniform(-8, 8, (rows, 1)) *
         2.0 ** g.uniform(-8, 8, (1, cols))).astype(np.float32)
    X[5, :] = 0.0  # an all-zero row
    ld = (rows if layout == 0 else cols) + pad
    buf = np.full(ld * (cols if layout == 0 else rows), np.nan, dtype=np.float32)
    for r in range(rows):
        for c in range(cols):
            buf[r + c * ld if layout == 0 else r * ld + c] = X[r, c]
    Q, s = oracle.quantize_fp8(layout, rows, cols, buf, ld, axis)
    q = np.array([[Q[r + c * ld if layout == 0 else r * ld + c] for c in range(cols)]
                  for r in range(rows)], dtype=np.uint8)
    dec = oracle.e4m3_decode(q.reshape(-1)).reshape(rows, cols)
    amax = np.abs(X).max(axis=1 - axis)
    for line in range(rows if axis == 0 else cols):
        e = np.log2(s[line])
        assert e == int(e)
        if amax[line] == 0:
            assert s[line] == 1.0
        else:
            assert amax[line] * s[line] <= 448 < amax[line] * s[line] * 2
    scaled = X.astype(np.float64) * (s[:, None] if axis == 0 else s[None, :])
    # every decoded value is the E4M3 value nearest the scaled input
    vals = oracle.e4m3_decode(np.arange(0x7F, dtype=np.uint8))
    nearest = np.abs(np.abs(scaled)[..., None] - vals).min(axis=-1)
    assert np.all(np.abs(np.abs(dec) - np.abs(scaled)) <= nearest + 0.0)
    assert np.all((dec == 0) | (np.sign(dec) == np.sign(scaled)))


def test_split3_is_exact():
    g = np.random.default_rng(6)
    x = np.concatenate([_edge_f32()[:10], g.uniform(-1, 1, 100_000).astype(np.float32) *
                        np.float32(2.0) ** g.integers(-100, 100, 100_000).astype(np.float32)])
    x = x[np.isfinite(x)]
    # the split is exact wherever x's bfloat16 rounding is finite (not for |x| within half a
    # bfloat16 ulp of the binary32 maximum, which rounds to infinity)
    x = x[np.isfinite(oracle.bf16_decode(oracle.bf16_round(x)))]
    planes = oracle.split3(x)
    v = [oracle.bf16_decode(planes[t]) for t in range(3)]
    assert np.array_equal(v[0] + v[1] + v[2], x.astype(np.float64))
    # each term is the bf16 rounding of what is left
    assert np.array_equal(planes[0], oracle.bf16_round(x))
    r1 = (x.astype(np.float64) - v[0]).astype(np.float32)
    assert np.array_equal(planes[1], oracle.bf16_round(r1))
    # the terms shrink: |x1| <= ulp(x0)/2, |x2| <= ulp(x1)/2 (bf16 has 8 significant bits)
    nz = v[0] != 0
    assert np.all(np.abs(v[1][nz]) <= np.abs(v[0][nz]) * 2.0 ** -8)
    nz1 = v[1] != 0
    assert np.all(np.abs(v[2][nz1]) <= np.abs(v[1][nz1]) * 2.0 ** -8)


def _stored(layout, rows, cols, ld, values, dtype):
    from paper_2302_08417_amd import synth
    return synth.fill_stored(layout, rows, cols, ld, values, dtype, 0)


def test_pack_oriented_kmajor_bruteforce():
    """Forced K-major blocks expose op(X) tile by tile, (tiles, ksteps, MNT, KT), for every
    storage orientation; zero fill outside op(X)."""
    import itertools
    for mn, k, MNT, KT in itertools.product(range(0, 6), range(0, 6), range(1, 4), range(1, 4)):
        for layout, t, is_b in itertools.product([0, 1], ["N", "T"], [0, 1]):
            rows, cols = (k, mn) if is_b else (mn, k)
            vals = (np.arange(rows * cols, dtype=np.float64).reshape(rows, cols) + 1)
            srows, scols = (cols, rows) if t == "T" else (rows, cols)
            stored = vals.T if t == "T" else vals
            ld = (srows if layout == 0 else scols) + 2
            buf = _stored(layout, srows, scols, max(ld, 1), stored, np.uint16)
            out = oracle.pack_oriented(buf, is_b, layout, t, mn, k, max(ld, 1), MNT, KT, 1)
            nt, nk = -(-mn // MNT), -(-k // KT)
            if out.size == 0:
                continue
            opx = vals.T if is_b else vals
            padded = np.zeros((nt * MNT, nk * KT))
            padded[:mn, :k] = opx
            tiles = padded.reshape(nt, MNT, nk, KT).transpose(0, 2, 1, 3)
            assert np.array_equal(out.reshape(nt, nk, MNT, KT).astype(np.float64), tiles)


def test_pack_mx_split_planes():
    """Split-form pack: block b holds the K-major planes of x0, x1, x2 in that order, and
    summing the planes' values gives back op(X) exactly."""
    from paper_2302_08417_amd import synth
    c = synth.make_mx_case(synth.FORM_BF16X3, 0, 150, 9, 70, "T", "N", ld_pad=3, seed=11)
    MNT, KT = 128, 32
    raw = oracle.pack_mx(4, c.A, 0, 0, "T", c.m, c.k, c.lda)
    nt, nk = -(-c.m // MNT), -(-c.k // KT)
    planes = raw.view(np.uint16).reshape(nt, nk, 3, MNT, KT)
    vals = sum(oracle.bf16_decode(planes[:, :, t].reshape(-1)).reshape(nt, nk, MNT, KT)
               for t in range(3))
    opA = synth.op_view(c.A32, 0, "T", c.m, c.k, c.lda).astype(np.float64)
    padded = np.zeros((nt * MNT, nk * KT))
    padded[: c.m, : c.k] = opA
    assert np.array_equal(vals, padded.reshape(nt, MNT, nk, KT).transpose(0, 2, 1, 3))
    fast = oracle.pack_mx(5, c.A, 0, 0, "T", c.m, c.k, c.lda).view(np.uint16)
    assert np.array_equal(fast.reshape(nt, nk, 2, MNT, KT), planes[:, :, :2])
