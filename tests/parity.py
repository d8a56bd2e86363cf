"""Comparison helpers for GPU-versus-oracle parity (test infrastructure)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

TOL_IMAGE = 2e-4  # per channel, absolute


def compare_image(gpu: np.ndarray, ref: dict, tol: float = TOL_IMAGE):
    """gpu [h, w, 4] against an oracle render with alternatives (oracle.render(...,
    with_alt=True)).  A pixel passes when it matches the oracle's result, or, where the
    oracle saw a near-threshold decision, the result with that decision flipped.
    Pixels whose camera validity is itself ambiguous are skipped.
    Returns (n_fail, max_err_over_passing_choice, details)."""
    prim = ref["rgba"]
    err = np.max(np.abs(gpu - prim), axis=-1)
    best = err.copy()
    if "alt" in ref:
        for f in range(O.N_ALT):
            use = ref["n_dec"] > f
            if not use.any():
                continue
            e = np.max(np.abs(gpu - ref["alt"][:, :, f]), axis=-1)
            best = np.where(use, np.minimum(best, e), best)
    skip = ref.get("skip", np.zeros(err.shape, bool))
    best = np.where(skip, 0.0, best)
    fail = best > tol
    return int(fail.sum()), float(best.max()), {
        "n_ambiguous": int((ref["n_dec"] > 0).sum()) if "n_dec" in ref else 0,
        "n_skipped": int(skip.sum()),
        "max_err_primary": float(np.where(skip, 0, err).max()),
        "worst_pixel": tuple(int(v) for v in np.unravel_index(np.argmax(best), best.shape)),
    }
