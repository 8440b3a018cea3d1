"""Stored oracle results for the GPU parity tests (read-only helpers).

perturbed_counts.json (written by golden/make_perturbed_counts.py, which calls
only the oracle) holds, for the parity cases whose basis keeps at most 16 bits
per value, the oracle's iteration count and its counts under last-bit
perturbations of b.  A GPU count must lie within 2% of the unperturbed
oracle's; for these cases it may instead lie within 2% of the range the
oracle spans under the perturbations, because such a basis turns last-bit
differences of the FP64 sums (whose order differs between any two correct
implementations) into differences of a few percent in the step count.
"""
import hashlib
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_cache = {}


def perturbed_cases() -> dict:
    if "pc" not in _cache:
        with open(os.path.join(GOLDEN, "perturbed_counts.json")) as f:
            _cache["pc"] = json.load(f)["cases"]
    return _cache["pc"]


def inputs_digest(A, b, x0=None) -> str:
    h = hashlib.sha256(A.sha256().encode() + np.ascontiguousarray(b).tobytes())
    if x0 is not None:
        h.update(np.ascontiguousarray(x0).tobytes())
    return h.hexdigest()


def within_2pct(a, b) -> bool:
    return abs(a - b) <= max(1, int(np.ceil(0.02 * b)))


def count_agrees(got: int, ref_iters: int, case: str = None, fmt: str = None, digest: str = None) -> bool:
    """True if `got` is within 2% of the oracle's `ref_iters`, or, for a case
    stored in perturbed_counts.json, within 2% of the range the oracle spans
    under last-bit perturbations of b.  The stored case must be for the same
    inputs (digest) and the same unperturbed count."""
    if within_2pct(got, ref_iters):
        return True
    if case is None:
        return False
    entry = perturbed_cases().get(f"{case}/{fmt}")
    if entry is None:
        return False
    assert entry["inputs_sha256"] == digest, f"{case}/{fmt}: inputs differ from the stored case"
    assert entry["oracle"] == ref_iters, f"{case}/{fmt}: stored oracle count {entry['oracle']} != {ref_iters}"
    counts = entry["perturbed"] + [entry["oracle"]]
    print(f"{case}/{fmt}: {got} outside 2% of {ref_iters}; stored oracle spread {sorted(counts)}")
    return 0.98 * min(counts) <= got <= 1.02 * max(counts)
