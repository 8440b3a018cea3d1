"""GPU parity of the FRSZ2 codec (frsz2_compress / frsz2_decompress through
the C ABI) against the CPU oracle: compressed words and exponents bit-exact,
decompressed values bit-exact, for every l in [3, 32] (16, 21 and 32 on their
specialised kernels, the rest on the generic codec), ragged sizes, adversarial
blocks, non-finite input, and sampled blocks of a full 2^24-value column; the
generic codec at l = 16, 21, 32 stores the specialised kernels' bits."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
from tests._inputs import adversarial_blocks, mixed_vector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def u32(t):
    return t.cpu().numpy().view(np.uint32)

BITS = [16, 21, 32]
ALL_BITS = list(range(3, 33))  # 16, 21, 32 on their own kernels, the rest on the generic codec
SIZES = [1, 31, 32, 33, 1000, 2048 * 3 + 17, 100003]


def gpu_roundtrip(x, bits):
    xd = torch.from_numpy(x).cuda()
    exps, words = cb.frsz2_compress(xd, bits)
    dec = cb.frsz2_decompress(exps, words, x.size, bits)
    torch.cuda.synchronize()
    return u32(exps), u32(words), dec.cpu().numpy()


@pytest.mark.parametrize("bits", ALL_BITS)
@pytest.mark.parametrize("n", SIZES)
def test_compress_bit_exact_random(bits, n):
    x = mixed_vector(n, seed=n + bits)
    e, w, d = gpu_roundtrip(x, bits)
    oe, ow, bad = oracle.frsz2_encode(x, bits)
    assert not bad
    np.testing.assert_array_equal(e, oe)
    np.testing.assert_array_equal(w, ow)
    od = oracle.frsz2_decode(oe, ow, n, bits)
    assert np.array_equal(d.view(np.uint64), od.view(np.uint64))


@pytest.mark.parametrize("bits", ALL_BITS)
def test_compress_bit_exact_adversarial(bits):
    x = adversarial_blocks()
    e, w, d = gpu_roundtrip(x, bits)
    oe, ow, _ = oracle.frsz2_encode(x, bits)
    np.testing.assert_array_equal(e, oe)
    np.testing.assert_array_equal(w, ow)
    assert np.array_equal(d.view(np.uint64), oracle.frsz2_decode(oe, ow, x.size, bits).view(np.uint64))


@pytest.mark.parametrize("bits", BITS + [3, 9, 27])
def test_nonfinite_flag(bits):
    x = mixed_vector(200, seed=3)
    x[70] = np.inf
    x[150] = np.nan
    xd = torch.from_numpy(x).cuda()
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    exps, words = cb.frsz2_compress(xd, bits, nonfinite_flag=flag)
    assert int(flag.item()) == 1
    oe, ow, bad = oracle.frsz2_encode(x, bits)
    assert bad
    e = u32(exps)
    w = u32(words).reshape(-1, bits)
    ow = ow.reshape(-1, bits)
    np.testing.assert_array_equal(e, oe)
    for b in range(e.size):  # finite blocks stay bit-exact
        if oe[b] != 0x7FF:
            np.testing.assert_array_equal(w[b], ow[b])
    flag.zero_()
    cb.frsz2_compress(torch.from_numpy(mixed_vector(200, 4)).cuda(), bits, nonfinite_flag=flag)
    assert int(flag.item()) == 0


@pytest.mark.parametrize("bits", BITS + [5, 12, 27])
def test_full_size_column_sampled(bits):
    """A 2^24-value column of the tall-skinny benchmark basis (block scales
    10^u, u ~ U(-8,0)): sampled blocks bit-exact against the oracle, and the
    truncation bound checked on every value."""
    import synth
    n = 1 << 24
    col = next(synth.basis_columns(n, 1, seed=2))
    xd = torch.from_numpy(col).cuda()
    exps, words = cb.frsz2_compress(xd, bits)
    dec = cb.frsz2_decompress(exps, words, n, bits)
    # property on every value: 0 <= |x| - |x~| < 2^(max(E,1)-1023-(l-2)), signs kept
    E = torch.clamp(exps.to(torch.int64), min=1).repeat_interleave(32)
    u = torch.ldexp(torch.ones(n, dtype=torch.float64, device="cuda"), (E - 1023 - (bits - 2)).to(torch.float64))
    err = xd.abs() - dec.abs()
    assert bool((err >= 0).all()) and bool((err < u).all())
    assert bool((torch.signbit(dec) == torch.signbit(xd)).all())
    rng = np.random.default_rng(bits)
    blocks = np.unique(np.concatenate([[0, n // 32 - 1], rng.integers(0, n // 32, 3000)]))
    e = u32(exps)
    w = u32(words).reshape(-1, bits)
    for b in blocks:
        oe, ow, _ = oracle.frsz2_encode(col[32 * b:32 * b + 32], bits)
        assert e[b] == oe[0]
        np.testing.assert_array_equal(w[b], ow)


@pytest.mark.parametrize("l", BITS)
def test_generic_codec_stores_the_specialised_bits(l):
    """The generic-l formats at l = 16, 21, 32 store exactly the words and
    exponents of the specialised formats, and decode to the same values."""
    n = 2048 * 2 + 45
    x = mixed_vector(n, seed=40 + l)
    spec = cb.Basis.empty(f"frsz2_{l}", n, 1)
    gen = cb.Basis.empty(cb.frsz2_bits_format(l), n, 1)
    xd = torch.from_numpy(x).cuda()
    cb.cb_basis_store(spec, 0, xd)
    cb.cb_basis_store(gen, 0, xd)
    torch.cuda.synchronize()
    assert np.array_equal(spec.column(0).cpu().numpy(), gen.column(0).cpu().numpy())
    assert np.array_equal(u32(spec.column_exps(0)), u32(gen.column_exps(0)))
    a = cb.cb_basis_load(spec, 0).cpu().numpy()
    b = cb.cb_basis_load(gen, 0).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


B64 = ["frsz2b64_16", "frsz2b64_32", "frsz2b64_3", "frsz2b64_7", "frsz2b64_21", "frsz2b64_27"]


@pytest.mark.parametrize("fmt", B64)
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 2048 * 3 + 17, 100003])
def test_block64_store_bit_exact(fmt, n):
    """Blocks of 64 values (one exponent per 64 rows): the stored column and
    its exponents are bit-exact against the oracle's block-64 encoder, and the
    column decodes bit-exactly; ragged tails included."""
    x = mixed_vector(n, seed=7 * n + len(fmt))
    V = cb.Basis.empty(fmt, n, 2)
    cb.cb_basis_store(V, 1, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    vals, exps, _ = oracle.basis_encode(fmt, x)
    assert oracle.block_size(fmt) == 64 and exps.size == (n + 63) // 64
    np.testing.assert_array_equal(V.column(1).cpu().numpy(), vals)
    np.testing.assert_array_equal(u32(V.column_exps(1)), exps)
    back = cb.cb_basis_load(V, 1).cpu().numpy()
    assert np.array_equal(back.view(np.uint64), oracle.basis_decode(fmt, vals, exps, n).view(np.uint64))


@pytest.mark.parametrize("l", [16, 32])
def test_block64_generic_codec_stores_the_specialised_bits(l):
    n = 2048 * 2 + 77
    x = mixed_vector(n, seed=90 + l)
    spec = cb.Basis.empty(f"frsz2b64_{l}", n, 1)
    gen = cb.Basis.empty(f"frsz2b64g_{l}", n, 1)
    xd = torch.from_numpy(x).cuda()
    cb.cb_basis_store(spec, 0, xd)
    cb.cb_basis_store(gen, 0, xd)
    torch.cuda.synchronize()
    assert np.array_equal(spec.column(0).cpu().numpy(), gen.column(0).cpu().numpy())
    assert np.array_equal(u32(spec.column_exps(0)), u32(gen.column_exps(0)))
