"""Per-tier comparison of full hierarchy states (test helper).

The ADOs of tier t = |n| shrink fast with t (after a few RK4 steps from a
state with only sigma_0 nonzero, tier t is built from t couplings), so a
deviation scaled by the largest entry of the whole state (|sigma_0| ~ 1) says
nothing about the deep tiers.  Here each tier is compared relative to its own
largest entry; a tier that is exactly zero in the reference must be exactly
zero in the result.
"""
from __future__ import annotations

import numpy as np


def match_oracle_order(lib_multi: np.ndarray, oracle_multi: np.ndarray) -> np.ndarray:
    """perm such that oracle ADO perm[i] has the multi-index of library ADO i."""
    index = {tuple(int(v) for v in r): i for i, r in enumerate(oracle_multi)}
    perm = np.array([index[tuple(int(v) for v in r)] for r in lib_multi])
    assert len(set(perm.tolist())) == len(oracle_multi) == len(lib_multi)
    return perm


def tier_errors(multi: np.ndarray, got: np.ndarray, want: np.ndarray):
    """[(tier, max |got - want|, max |want|)] for every tier of the hierarchy;
    got and want are [n_ados, N, N] in the order of `multi`."""
    tiers = np.sum(multi, axis=1)
    rows = []
    for t in range(int(tiers.max()) + 1):
        sel = tiers == t
        rows.append((t, float(np.max(np.abs(got[sel] - want[sel]))),
                     float(np.max(np.abs(want[sel])))))
    return rows


def assert_tiers(multi, got, want, tol: float, min_nonzero_tier: int | None = None):
    """Every tier within tol of its own largest entry; returns the deepest
    tier with a nonzero reference (checked against min_nonzero_tier)."""
    deepest = -1
    for t, err, scale in tier_errors(multi, got, want):
        if scale == 0.0:
            assert err == 0.0, f"tier {t}: reference is zero, result deviates by {err:.3e}"
            continue
        deepest = t
        assert err <= tol * scale, f"tier {t}: error {err:.3e} vs tier max {scale:.3e}"
    if min_nonzero_tier is not None:
        assert deepest >= min_nonzero_tier, (deepest, min_nonzero_tier)
    return deepest
