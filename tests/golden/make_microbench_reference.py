"""Write the oracle's reference for the kernel microbenchmark basis
(2^24 rows x 101 columns, column = N(0,1)/sqrt(n) scaled per 32-value block by
10^u, u ~ U(-8, 0), one stream default_rng(2); w ~ N(0,1)/sqrt(n) from
default_rng(1002)):

* for l = 16, 21, 32 and every column c, the SHA-256 of the oracle's FRSZ2
  encoding (the value words, then the exponent words, little-endian uint32),
  so that a GPU test can compare every block of every column;
* h_c = <D(Q(v_c)), w>, the fused decompress + projection, by the oracle's
  decoder and its compensated dot product, with s_c = sum_k |D(Q(v_c))_k w_k|
  (the scale of the parity bound |h_gpu - h| <= 1e-12 s_c);
* the SHA-256 of each generated column and of w (the inputs).

Calls only the oracle and the seeded input generators; takes ~10 minutes.

    python tests/golden/make_microbench_reference.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "microbench_oracle.json")
N, NCOLS, SEED = 1 << 24, 101, 2
WIDTHS = (16, 21, 32)


def main():
    t0 = time.time()
    w = synth.basis_probe_vector(N, SEED)
    out = {
        "workload": "tall-skinny basis 2^24 x 101, block scales 10^U(-8,0), seed 2; w from seed 1002",
        "n": N, "ncols": NCOLS, "seed": SEED,
        "w_sha256": hashlib.sha256(w.tobytes()).hexdigest(),
        "column_sha256": [],
        "encoded_sha256": {str(l): [] for l in WIDTHS},
        "h": {str(l): [] for l in WIDTHS},
        "abs_scale": {str(l): [] for l in WIDTHS},
    }
    absw = np.abs(w)
    for c, col in enumerate(synth.basis_columns(N, NCOLS, SEED)):
        out["column_sha256"].append(hashlib.sha256(col.tobytes()).hexdigest())
        for l in WIDTHS:
            exps, words, bad = oracle.frsz2_encode(col, l)
            assert not bad
            out["encoded_sha256"][str(l)].append(hashlib.sha256(words.tobytes() + exps.tobytes()).hexdigest())
            dec = oracle.frsz2_decode(exps, words, N, l)
            out["h"][str(l)].append(oracle.dot(dec, w))
            out["abs_scale"][str(l)].append(oracle.dot(np.abs(dec), absw))
        print(f"column {c}: {time.time() - t0:.0f}s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
