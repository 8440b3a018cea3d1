"""The largest row count the library accepts, n = 2^31 - 4096 (every 32-bit
row index a kernel forms stays below 2^31): the frsz2_21 codec (codes that
straddle words) on a full column, checked bit-exactly against the oracle on
sampled blocks (the first, the last and 2000 seeded ones) and by the
truncation property on every value; the fused projection and update with two
frsz2_32 columns, checked against the oracle: h against the oracle's decode of
the stored words and its compensated dot product (in 2^27-row chunks whose
compensated sums are added by the oracle's compensated sum), the update on
sampled rows against the oracle's random-access decode."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
NMAX = (1 << 31) - 4096


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_codec_at_the_row_limit():
    n, bits = NMAX, 21
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    x *= torch.pow(10.0, -6.0 * torch.rand(n // 32, dtype=torch.float64, device="cuda",
                                             generator=g)).repeat_interleave(32)
    exps, words = cb.frsz2_compress(x, bits)
    dec = cb.frsz2_decompress(exps, words, n, bits)
    torch.cuda.synchronize()
    nb = n // 32
    blocks = np.unique(np.concatenate([[0, nb - 1], np.random.default_rng(3).integers(0, nb, 2000)]))
    bt = torch.from_numpy(blocks).cuda()
    rows = (bt[:, None] * 32 + torch.arange(32, device="cuda")[None, :]).reshape(-1)
    xs = x[rows].cpu().numpy().reshape(-1, 32)
    ws = words.view(-1, bits)[bt].cpu().numpy().view(np.uint32)
    es = u32(exps[bt])
    for k in range(blocks.size):
        oe, ow, _ = oracle.frsz2_encode(xs[k], bits)
        assert es[k] == oe[0], blocks[k]
        np.testing.assert_array_equal(ws[k], ow)
    ds = dec[rows].cpu().numpy().reshape(-1, 32)
    for k in range(0, blocks.size, 50):
        oe, ow, _ = oracle.frsz2_encode(xs[k], bits)
        assert np.array_equal(ds[k].view(np.uint64), oracle.frsz2_decode(oe, ow, 32, bits).view(np.uint64))
    # every value: 0 <= |x| - |x~| < 2^(max(E,1)-1023-(l-2)), signs kept (in chunks)
    step = 1 << 27
    for s in range(0, n, step):
        e = min(n, s + step)
        E = torch.clamp(exps[s // 32:e // 32].to(torch.int64), min=1).repeat_interleave(32)
        u = torch.ldexp(torch.ones(e - s, dtype=torch.float64, device="cuda"), (E - 1023 - (bits - 2)).double())
        err = x[s:e].abs() - dec[s:e].abs()
        assert bool((err >= 0).all()) and bool((err < u).all())
        assert bool((torch.signbit(dec[s:e]) == torch.signbit(x[s:e])).all())
        del E, u, err
    del x, dec, exps, words
    torch.cuda.empty_cache()


def test_projection_and_update_at_the_row_limit():
    n = NMAX
    g = torch.Generator(device="cuda")
    g.manual_seed(12)
    V = cb.Basis.empty("frsz2_32", n, 2)
    for c in range(2):
        v = torch.randn(n, dtype=torch.float64, device="cuda", generator=g) / np.sqrt(n)
        cb.cb_basis_store(V, c, v)
        del v
    w = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    h = cb.cb_cgs_project(V, 2, w).cpu().numpy()
    torch.cuda.synchronize()
    # the oracle's h from the stored words, chunk by chunk (chunks are whole
    # blocks), and the scale sum |v~ w| of the parity bound
    chunk = 1 << 27
    part = [[], []]
    absp = [[], []]
    for s0 in range(0, n, chunk):
        e0 = min(n, s0 + chunk)
        wc = w[s0:e0].cpu().numpy()
        for c in range(2):
            words = V.column(c).view(torch.int32)[s0:e0].cpu().numpy().view(np.uint32)
            ex = u32(V.column_exps(c)[s0 // 32:(e0 + 31) // 32])
            dec = oracle.frsz2_decode(ex, words, e0 - s0, 32)
            part[c].append(oracle.dot(dec, wc))
            absp[c].append(oracle.dot(np.abs(dec), np.abs(wc)))
            del words, ex, dec
        del wc
    for c in range(2):
        ones = np.ones(len(part[c]))
        ref = oracle.dot(np.array(part[c]), ones)
        scale = oracle.dot(np.array(absp[c]), ones)
        print(f"column {c}: h {h[c]!r} oracle {ref!r} scale {scale:.3e}")
        assert abs(h[c] - ref) <= 1e-12 * scale, (c, h[c], ref)
    # w -= V h on sampled rows against the oracle's random-access decode of
    # the blocks that hold them, and the fused norm
    rows_np = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(4).integers(0, n, 4096)]))
    rows = torch.from_numpy(rows_np).cuda()
    w0 = w[rows].cpu().numpy()
    d0 = [np.empty(rows_np.size), np.empty(rows_np.size)]
    for c in range(2):
        blk = torch.from_numpy(rows_np // 32).cuda()
        words = V.column(c).view(torch.int32).view(-1, 32)[blk].cpu().numpy().view(np.uint32)
        ex = u32(V.column_exps(c)[blk])
        for k, r in enumerate(rows_np):
            d0[c][k] = oracle.frsz2_decode_value(ex[k:k + 1], words[k], int(r % 32), 32)
    hd = torch.from_numpy(h).cuda()
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    cb.cb_cgs_subtract(V, 2, hd, w, norm2=nrm)
    got = w[rows].cpu().numpy()
    want = w0 - (h[0] * d0[0] + h[1] * d0[1])
    assert np.all(np.abs(got - want) <= 1e-14 * (np.abs(w0) + np.abs(h[0] * d0[0]) + np.abs(h[1] * d0[1])))
    # the norm: the oracle's compensated sum of squares over the updated w
    sq = []
    for s0 in range(0, n, chunk):
        wc = w[s0:min(n, s0 + chunk)].cpu().numpy()
        sq.append(oracle.dot(wc, wc))
        del wc
    ww = oracle.dot(np.array(sq), np.ones(len(sq)))
    assert abs(float(nrm.item()) - ww) <= 1e-12 * ww
