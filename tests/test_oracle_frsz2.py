"""Pins for the oracle's FRSZ2 codec and baseline casts (CPU only).

Each pin checks the oracle against something other than itself: the
hand-derived worked vectors (tests/golden/frsz2_worked.txt), the value
definition of FRSZ2 as truncation onto the block's grid (Eq. 2 with "cut to
length l" read as truncation), an independent LSB-first bit packer, the
paper's four-step random-access decode route (Section IV-B), brute force over
every 16-bit code, and numpy's IEEE casts.
"""
import os
import struct

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "frsz2_worked.txt")
# l is a free parameter of the format (Section IV-A): the fixed widths and a
# spread of others, odd and even, below and above 16
ALL_L = [3, 4, 7, 8, 12, 13, 16, 17, 21, 24, 27, 31, 32]
BLOCK_A = [1.0, -0.75, 0.1, 0.0, -0.0, 3e-300, 2.0 ** -30, -(1 - 2.0 ** -53)] + [0.0] * 24
BLOCK_B = [0.5, 1e-5, -0.3]


# ---------------------------------------------------------------- helpers written from Eq. 2
def _bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def grid_codes(block, l):
    """Codes of one block by the value definition: with E the largest biased
    exponent field and u = 2^(max(E,1)-1023-(l-2)), the magnitude code is
    floor(|x|/u), computed in exact integer arithmetic."""
    bl = [_bits(float(v)) for v in block] + [0] * (32 - len(block))
    E = max((b >> 52) & 0x7FF for b in bl)
    Eeff = max(E, 1)
    codes = []
    for b in bl:
        s, e, f = b >> 63, (b >> 52) & 0x7FF, b & ((1 << 52) - 1)
        sig = ((1 << 52) | f) if e else f
        # |x| = sig * 2^(max(e,1)-1075); |x|/u = sig * 2^(max(e,1)-1075-Eeff+1023+l-2)
        sh = max(e, 1) - 1075 - Eeff + 1023 + l - 2
        mag = sig << sh if sh >= 0 else sig >> (-sh)
        assert mag < (1 << (l - 1))
        codes.append((s << (l - 1)) | mag)
    return E, codes


def pack_lsb_first(codes, l):
    """Independent packer: concatenate the codes as a little-endian bit
    string (code q at bits [q*l, (q+1)*l)) and cut it into 32-bit words."""
    bitstr = np.zeros(32 * l, np.uint8)
    for q, c in enumerate(codes):
        for t in range(l):
            bitstr[q * l + t] = (c >> t) & 1
    return np.packbits(bitstr, bitorder="little").view("<u4")


def unpack_codes(words, l, count=32):
    bits = np.unpackbits(np.asarray(words, "<u4").view(np.uint8), bitorder="little")
    return [int(sum(int(bits[q * l + t]) << t for t in range(l))) for q in range(count)]


def grid_decode(E, code, l):
    Eeff = max(E, 1)
    mag = code & ((1 << (l - 1)) - 1)
    v = float(mag) * 2.0 ** (Eeff - 1023 - (l - 2)) if Eeff - 1023 - (l - 2) > -1000 else \
        np.ldexp(float(mag), Eeff - 1023 - (l - 2))
    return -v if code >> (l - 1) else v


def _random_blocks(rng, nblk, spread):
    """Blocks of normal values with exponent spreads up to `spread` decades,
    mixed signs, some exact zeros, -0.0 and subnormals."""
    base = rng.standard_normal((nblk, 32))
    scale = 10.0 ** rng.uniform(-spread, 0, (nblk, 32))
    x = base * scale * 10.0 ** rng.uniform(-300, 300, (nblk, 1))
    x[rng.random(x.shape) < 0.03] = 0.0
    x[rng.random(x.shape) < 0.02] = -0.0
    sub = rng.random(x.shape) < 0.02
    x[sub] = rng.standard_normal(sub.sum()) * 1e-310
    return x.ravel()


# ---------------------------------------------------------------- golden worked vectors
def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.mark.parametrize("row", [r for r in _golden() if r[0] == "block"], ids=lambda r: f"{r[1]}{r[2]}")
def test_worked_vector_codes(row):
    _, name, l, exph, *codes = row
    l = int(l)
    block = BLOCK_A if name == "A" else BLOCK_B
    exps, words, bad = oracle.frsz2_encode(np.array(block), l)
    assert not bad
    assert int(exps[0]) == int(exph, 16)
    got = unpack_codes(words[:l], l)
    assert got[:len(codes)] == [int(c, 16) for c in codes]
    # tail padding and the zeros of block A are all-zero codes
    assert all(c == 0 for c in got[len(block):])


def test_worked_vector_words_and_decode():
    rows = _golden()
    for r in rows:
        if r[0] == "words":
            l = int(r[2])
            _, words, _ = oracle.frsz2_encode(np.array(BLOCK_A), l)
            assert [int(w) for w in words[:len(r) - 3]] == [int(x, 16) for x in r[3:]]
        if r[0] == "decode":
            l, idx, val = int(r[2]), int(r[3]), float(r[4])
            e, w, _ = oracle.frsz2_encode(np.array(BLOCK_A), l)
            assert oracle.frsz2_decode(e, w, 32, l)[idx] == val


# ---------------------------------------------------------------- value definition and packing
@pytest.mark.parametrize("l", ALL_L)
@pytest.mark.parametrize("spread", [0, 3, 12, 40])
def test_encode_matches_grid_definition_and_packer(l, spread):
    rng = np.random.default_rng(100 + l + spread)
    x = _random_blocks(rng, 40, spread)
    exps, words, bad = oracle.frsz2_encode(x, l)
    assert not bad
    for b in range(40):
        E, codes = grid_codes(x[32 * b:32 * b + 32], l)
        assert int(exps[b]) == E
        np.testing.assert_array_equal(words[b * l:(b + 1) * l], pack_lsb_first(codes, l))
        dec = oracle.frsz2_decode(exps[b:b + 1], words[b * l:(b + 1) * l], 32, l)
        ref = [grid_decode(E, c, l) for c in codes]
        assert [_bits(v) for v in dec] == [_bits(v) for v in ref]


@pytest.mark.parametrize("l", ALL_L)
def test_error_bound_sign_and_monotone(l):
    rng = np.random.default_rng(7 + l)
    x = _random_blocks(rng, 200, 6)
    exps, words, _ = oracle.frsz2_encode(x, l)
    d = oracle.frsz2_decode(exps, words, x.size, l)
    Eeff = np.maximum(np.repeat(exps.astype(np.int64), 32), 1)
    u = np.ldexp(1.0, (Eeff - 1023 - (l - 2)).astype(np.int32))
    err = np.abs(x) - np.abs(d)
    assert np.all(err >= 0)          # truncation toward zero
    assert np.all(err < u)           # less than one unit of the block grid
    assert np.all(np.signbit(d) == np.signbit(x))
    # relative bound for the block maximum (k = 0): 2^-(l-2)
    for b in range(200):
        blk = x[32 * b:32 * b + 32]
        i = int(np.argmax(np.abs(blk)))
        if blk[i] != 0 and np.abs(blk[i]) > 1e-300:
            assert abs(blk[i] - d[32 * b + i]) <= abs(blk[i]) * 2.0 ** -(l - 2)
    # monotone within a block
    for b in range(50):
        o = np.argsort(x[32 * b:32 * b + 32], kind="stable")
        assert np.all(np.diff(d[32 * b:32 * b + 32][o]) >= 0)


@pytest.mark.parametrize("l", ALL_L)
def test_idempotence_and_exact_roundtrip(l):
    rng = np.random.default_rng(11 * l)
    x = _random_blocks(rng, 100, 5)
    e1, w1, _ = oracle.frsz2_encode(x, l)
    d1 = oracle.frsz2_decode(e1, w1, x.size, l)
    e2, w2, _ = oracle.frsz2_encode(d1, l)
    # Q(D(Q(x))) == Q(x), except a block that is entirely zero/subnormal may
    # store E = 0 once and E = 1 after (same decoded values)
    d2 = oracle.frsz2_decode(e2, w2, x.size, l)
    assert np.array_equal(d1.view(np.uint64), d2.view(np.uint64))
    np.testing.assert_array_equal(w1, w2)
    # representable values (the block maximum holds its integer bit) round-trip
    nb = 64
    Es = rng.integers(1, 2047, nb)
    codes = rng.integers(0, 1 << l, (nb, 32), dtype=np.int64)
    codes[:, 0] |= 1 << (l - 2)
    vals = np.array([[grid_decode(int(Es[b]), int(c), l) for c in codes[b]] for b in range(nb)]).ravel()
    e3, w3, _ = oracle.frsz2_encode(vals, l)
    np.testing.assert_array_equal(e3, Es.astype(np.uint32))
    for b in range(nb):
        assert unpack_codes(w3[b * l:(b + 1) * l], l) == [int(c) for c in codes[b]]


@pytest.mark.parametrize("l", ALL_L)
def test_power_of_two_scaling_changes_only_exponent(l):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(32 * 20) * 10.0 ** rng.uniform(-5, 0, 32 * 20)
    e0, w0, _ = oracle.frsz2_encode(x, l)
    for t in (-40, -3, 1, 17, 200):
        e1, w1, _ = oracle.frsz2_encode(np.ldexp(x, t), l)
        np.testing.assert_array_equal(w0, w1)
        np.testing.assert_array_equal(e1.astype(np.int64), e0.astype(np.int64) + t)


@pytest.mark.parametrize("l", ALL_L)
def test_random_access_route_equals_closed_form(l):
    rng = np.random.default_rng(3 * l)
    x = _random_blocks(rng, 30, 20)
    # include blocks whose decoded values land in the subnormal range
    x[:32] = rng.standard_normal(32) * 1e-308
    x[32:64] = rng.standard_normal(32) * 3e-310
    exps, words, _ = oracle.frsz2_encode(x, l)
    full = oracle.frsz2_decode(exps, words, x.size, l)
    one = np.array([oracle.frsz2_decode_value(exps, words, i, l) for i in range(x.size)])
    assert np.array_equal(full.view(np.uint64), one.view(np.uint64))


@pytest.mark.parametrize("E", [1, 2, 60, 1023, 2000, 2046])
def test_bruteforce_all_16bit_codes(E):
    l = 16
    codes = np.arange(1 << 16, dtype=np.uint32)
    anchor = np.uint32(1 << (l - 2))  # integer bit set: pins the block exponent at E
    nblk = (codes.size + 30) // 31
    blocks = np.zeros((nblk, 32), np.uint32)
    blocks[:, 0] = anchor
    flat = blocks[:, 1:].reshape(-1)
    flat[:codes.size] = codes
    blocks[:, 1:] = flat.reshape(nblk, 31)
    words = np.zeros((nblk, 16), np.uint32)
    words[:] = (blocks[:, 0::2] | (blocks[:, 1::2] << 16))
    exps = np.full(nblk, E, np.uint32)
    dec = oracle.frsz2_decode(exps, words.ravel(), nblk * 32, l)
    e2, w2, bad = oracle.frsz2_encode(dec, l)
    assert not bad
    np.testing.assert_array_equal(e2, exps)
    np.testing.assert_array_equal(w2, words.ravel())


@pytest.mark.parametrize("l", [3, 5, 8, 11])
def test_bruteforce_every_code_of_small_widths(l):
    """Every l-bit code in every slot of a block, at a small, a middle and the
    top exponent: decoding then encoding gives the codes and exponent back."""
    for E in (1, 1023, 2046):
        codes = np.arange(1 << l, dtype=np.int64)
        anchor = 1 << (l - 2)
        per = 31
        nblk = (codes.size + per - 1) // per
        for shift in range(32):  # every code in every slot
            blocks = np.zeros((nblk, 32), np.int64)
            flat = np.zeros(nblk * per, np.int64)
            flat[:codes.size] = np.roll(codes, shift)
            slots = [q for q in range(32) if q != shift % 32]
            blocks[:, slots] = flat.reshape(nblk, per)
            blocks[:, shift % 32] = anchor
            vals = np.array([[grid_decode(E, int(c), l) for c in blocks[b]] for b in range(nblk)]).ravel()
            e2, w2, bad = oracle.frsz2_encode(vals, l)
            assert not bad
            np.testing.assert_array_equal(e2, np.full(nblk, E, np.uint32))
            for b in range(nblk):
                assert unpack_codes(w2[b * l:(b + 1) * l], l) == [int(c) for c in blocks[b]]
            if l > 5:
                break  # one arrangement suffices for the wider codes


def test_zero_and_subnormal_blocks():
    l = 32
    x = np.zeros(64)
    # subnormal multiples of the E_eff = 1 grid unit 2^(1-1023-30) are exact
    x[32:] = np.array([np.ldexp(float(k * 12345), -1052) for k in range(32)])
    e, w, bad = oracle.frsz2_encode(x, l)
    assert not bad and e[0] == 0 and e[1] == 0
    d = oracle.frsz2_decode(e, w, 64, l)
    assert np.array_equal(d, x)
    # below the grid unit they truncate to zero
    tiny = oracle.frsz2_encode(np.array([5e-324] * 32), l)
    assert np.all(oracle.frsz2_decode(tiny[0], tiny[1], 32, l) == 0)
    z = oracle.frsz2_decode(*oracle.frsz2_encode(np.array([-0.0] * 32), l)[:2], 32, l)
    assert np.all(np.signbit(z)) and np.all(z == 0)


def test_nonfinite_flag_and_tail_padding():
    for bad_val in (np.inf, -np.inf, np.nan):
        x = np.ones(70)
        x[40] = bad_val
        _, _, bad = oracle.frsz2_encode(x, 32)
        assert bad
    for l in (16, 21, 32):
        x = np.random.default_rng(1).standard_normal(37)
        e, w, bad = oracle.frsz2_encode(x, l)
        assert not bad and e.size == 2 and w.size == 2 * l
        assert unpack_codes(w[l:], l)[5:] == [0] * 27


# ---------------------------------------------------------------- float32 / float16 baselines
def _cast_inputs():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-9, 6, 20000)
    ties = []
    for e in range(-24, 16):  # exact half-way points of the float16 grid
        ulp = 2.0 ** max(e - 10, -24)
        for k in (1, 2, 3, 1023, 1024):
            ties.append((2.0 ** e if e >= -14 else 0.0) + (k + 0.5) * ulp)
    edge = [0.0, -0.0, 65504.0, 65519.999, 65520.0, 65536.0, 1e10, -1e10, 2.0 ** -24,
            2.0 ** -25, 3 * 2.0 ** -25, 2.0 ** -26, 6.1e-5, 5.96e-8, 1e-320, np.inf, -np.inf]
    return np.concatenate([x, np.array(ties), -np.array(ties), np.array(edge)])


def test_float16_matches_numpy():
    x = _cast_inputs()
    ref = x.astype(np.float16).view(np.uint16)
    got = np.array([oracle.f16_bits(v) for v in x], np.uint16)
    np.testing.assert_array_equal(got, ref)
    assert oracle.f16_bits(np.nan) & 0x7C00 == 0x7C00
    allh = np.arange(1 << 16, dtype=np.uint16)
    vals = allh.view(np.float16).astype(np.float64)
    got = np.array([oracle.f16_value(int(h)) for h in allh])
    fin = np.isfinite(vals)
    assert np.array_equal(got[fin].view(np.uint64), vals[fin].view(np.uint64))
    assert np.all(np.isnan(got[np.isnan(vals)]))


def test_basis_formats_match_numpy_casts():
    x = _cast_inputs()
    x = x[np.isfinite(x)][:5000]
    v32, _, _ = oracle.basis_encode("float32", x)
    np.testing.assert_array_equal(v32.view(np.float32)[:x.size], x.astype(np.float32))
    v16, _, _ = oracle.basis_encode("float16", x)
    np.testing.assert_array_equal(v16.view(np.uint16)[:x.size], x.astype(np.float16).view(np.uint16))
    small = x[np.abs(x) < 65504.0]
    for fmt in ("float64", "float32", "float16", "frsz2_16", "frsz2_21", "frsz2_32"):
        vals, exps, bad = oracle.basis_encode(fmt, small)
        d = oracle.basis_decode(fmt, vals, exps, small.size)
        assert not bad and d.shape == small.shape and np.all(np.isfinite(d))
        # rows beyond n (up to the next multiple of 32) are stored as zeros
        full = oracle.basis_decode(fmt, vals, exps, 32 * ((small.size + 31) // 32))
        assert np.all(full[small.size:] == 0)
    # float16 overflow is reported as non-finite
    assert oracle.basis_encode("float16", np.array([1.0, 7e4]))[2]


# ---------------------------------------------------------------- blocks of 64 values
def grid_codes_bs(block, l, bs):
    """grid_codes for a block of bs values (tail padded with +0.0)."""
    bl = [_bits(float(v)) for v in block] + [0] * (bs - len(block))
    E = max((b >> 52) & 0x7FF for b in bl)
    Eeff = max(E, 1)
    codes = []
    for b in bl:
        s, e, f = b >> 63, (b >> 52) & 0x7FF, b & ((1 << 52) - 1)
        sig = ((1 << 52) | f) if e else f
        sh = max(e, 1) - 1075 - Eeff + 1023 + l - 2
        mag = sig << sh if sh >= 0 else sig >> (-sh)
        codes.append((s << (l - 1)) | mag)
    return E, codes


def pack_lsb_first_n(codes, l):
    bitstr = np.zeros(len(codes) * l, np.uint8)
    for q, c in enumerate(codes):
        for t in range(l):
            bitstr[q * l + t] = (c >> t) & 1
    return np.packbits(bitstr, bitorder="little").view("<u4")


@pytest.mark.parametrize("l", [5, 16, 21, 32])
def test_block64_matches_grid_definition_and_packer(l):
    """Blocks of 64 values share one exponent: codes by the value definition
    on the 64-value block, packed LSB first into 2 l words; ragged tail."""
    rng = np.random.default_rng(200 + l)
    n = 64 * 9 + 23
    x = _random_blocks(rng, (n + 31) // 32, 8)[:n]
    exps, words, bad = oracle.frsz2_encode(x, l, bs=64)
    assert not bad and exps.size == 10 and words.size == 10 * 2 * l
    for b in range(10):
        E, codes = grid_codes_bs(x[64 * b:64 * b + 64], l, 64)
        assert int(exps[b]) == E
        np.testing.assert_array_equal(words[b * 2 * l:(b + 1) * 2 * l], pack_lsb_first_n(codes, l))
    d = oracle.frsz2_decode(exps, words, n, l, bs=64)
    Eeff = np.maximum(np.repeat(exps.astype(np.int64), 64)[:n], 1)
    u = np.ldexp(1.0, (Eeff - 1023 - (l - 2)).astype(np.int32))
    err = np.abs(x) - np.abs(d)
    assert np.all(err >= 0) and np.all(err < u) and np.all(np.signbit(d) == np.signbit(x))
    one = np.array([oracle.frsz2_decode_value(exps, words, i, l, bs=64) for i in range(n)])
    assert np.array_equal(one.view(np.uint64), d.view(np.uint64))


@pytest.mark.parametrize("l", [7, 16, 32])
def test_block64_is_two_blocks32_when_exponents_agree(l):
    """When both halves of a 64-value block have the same largest exponent,
    the 64-block's words are the two 32-blocks' words in sequence."""
    rng = np.random.default_rng(l)
    x = rng.uniform(-1, 1, 64 * 12)
    x[::32] = 1.5  # every 32-value half holds a value of exponent field 1023
    e64, w64, _ = oracle.frsz2_encode(x, l, bs=64)
    e32, w32, _ = oracle.frsz2_encode(x, l)
    np.testing.assert_array_equal(w64, w32)
    np.testing.assert_array_equal(e64, e32[::2])
    # halves with different maxima: the half with the smaller maximum is coarser
    y = x.copy()
    y[32:64] *= 2.0 ** -6
    e, w, _ = oracle.frsz2_encode(y, l, bs=64)
    d64 = oracle.frsz2_decode(e, w, y.size, l, bs=64)
    ee, ww, _ = oracle.frsz2_encode(y, l)
    d32 = oracle.frsz2_decode(ee, ww, y.size, l)
    assert np.all(np.abs(y[32:64] - d64[32:64]) >= np.abs(y[32:64] - d32[32:64]))
