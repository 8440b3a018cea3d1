"""The arithmetic-intensity sweep kernel (the synthetic benchmark of Section
IV-C): its per-workgroup sums equal, to rounding, the same arithmetic applied
to the oracle's decode of the stored column, for every format, with a ragged
tail and with several row groups per workgroup."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
# frsz2_9, frsz2_27: the generic codec; frsz2b64_*: blocks of 64 values
FORMATS = list(oracle.FORMATS) + ["frsz2_9", "frsz2_27", "frsz2b64_16", "frsz2b64_32", "frsz2b64_21"]


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("n", [1000, 70001, 3_000_001])
def test_intensity_sums_match_decoded_arithmetic(fmt, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * np.repeat(10.0 ** rng.uniform(-3, 0, (n + 31) // 32), 32)[:n]
    V = cb.Basis.empty(fmt, n, 1)
    cb.cb_basis_store(V, 0, torch.from_numpy(x).cuda())
    vals, exps = V.column(0).cpu().numpy(), V.column_exps(0)
    dec = oracle.basis_decode(fmt, vals, exps.cpu().numpy().view(np.uint32) if exps is not None else
                              np.zeros(1, np.uint32), n)
    a, b = 0.999, 1e-3
    for ops in (0, 1, 5):
        part = cb.cb_intensity_run(V, 0, ops, a, b)
        torch.cuda.synchronize()
        y = dec.copy()
        for _ in range(ops):
            y = y * a + b
        got = float(part.sum().item())
        assert abs(got - y.sum()) <= 1e-12 * np.abs(y).sum() + 1e-300, (fmt, n, ops, got, y.sum())
    assert cb.cb_intensity_groups(n) == part.numel()


def test_intensity_argument_errors():
    V = cb.Basis.empty("frsz2_32", 100, 1)
    with pytest.raises(cb.CbError):
        cb.cb_intensity_run(V, 1, 0, 1.0, 0.0)
    with pytest.raises(cb.CbError):
        cb.cb_intensity_run(V, 0, -1, 1.0, 0.0)
