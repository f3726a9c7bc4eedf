"""Parameter-level variants of the lazy PCA.

posterior_matched: as the inertia q grows, the stationary law of the lazy PCA tends to the
square of the Gibbs posterior (doubled pair coupling and doubled data precision; see the
closed-form stationary law, Sec. 3 eq. (symm_ham_pca_stationary_measure), in the limit
where only w = x contributes).  Halving J and multiplying sigma by sqrt(2) therefore makes
the large-q limit the posterior of the original model.
"""
from __future__ import annotations

import math


def posterior_matched(params: dict) -> dict:
    """Copy of ``params`` with J halved and sigma multiplied by sqrt(2)."""
    out = dict(params)
    out["J"] = params["J"] / 2.0
    out["sigma"] = params["sigma"] * math.sqrt(2.0)
    return out
