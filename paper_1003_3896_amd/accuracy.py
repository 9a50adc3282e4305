"""Accuracy of an acceleration evaluation against a reference, in every metric this library
reports.  The paper defines no accuracy metric for the pair sum, so each is stated here:

  max_over_arms   max_i |a_i - r_i| / a_rms(c(i)),  a_rms(c) = sqrt(mean_{i in c} |r_i|^2) over the
                  rows of cluster c (robust where |r_i| -> 0 at a cluster centre)
  l2              sqrt(sum_i |a_i - r_i|^2 / sum_i |r_i|^2) over all rows
  rel_median/p99/max   quantiles of the per-particle |a_i - r_i| / |r_i| (rows with r_i = 0 skipped)
  s_median/p99/max     quantiles of |a_i - r_i| / S_i, where S_i is the sum of the magnitudes of
                  particle i's terms, G sum_j m_j |d_ij| / (|d_ij|^2 + eps^2)^{3/2} + |a_ext,i| (only
                  when the caller passes S_i: the library does not compute it)

S_i bounds the rounding error of any evaluation of the sum (each term's error is a multiple of the
unit roundoff times that term's magnitude), so the S_i metric gates the precision modes in the
tests: FP64 <= 1e-12, the double-single modes <= 1e-6.  The a_rms metric is the one that ignores
the conditioning of particle i's own sum: a particle with a close neighbour has |a_i| >> a_rms, and
FP32 rounding of that one large term shows in it.

Plain NumPy on arrays the caller already has; none of the method's arithmetic.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

# gates on the S_i metric (max over rows) and, for the modes whose close-pair rounding is unbounded
# in it, on the median (see gate())
S_MAX = {"fp64": 1e-12, "fp32ds": 1e-6, "fp32dl": 1e-6, "fp32c": 1e-3, "fp32": 1e-3}
S_MEDIAN = {"fp64": 1e-14, "fp32ds": 1e-7, "fp32dl": 1e-7, "fp32c": 1e-6, "fp32": 1e-6}


def accel_error(a, ref, offsets: Optional[Sequence[int]] = None, scale=None, rows=None,
                arms=None) -> Dict[str, float]:
    """Error metrics of accelerations ``a`` against ``ref`` (both (m, 3)).

    offsets: CSR cluster boundaries of the full batch; ``rows`` (indices into that batch, sorted)
    says which particles ``a``/``ref`` hold (default: all of them, in order).  a_rms is taken per
    cluster over the rows given, unless ``arms`` supplies it per cluster (e.g. from a full
    reference).  scale: S_i of the same rows, or None.
    """
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = ref.shape[0]
    rows = np.arange(m) if rows is None else np.asarray(rows)
    offsets = np.array([0, int(rows.max()) + 1 if m else 0]) if offsets is None else np.asarray(offsets)
    cl = np.searchsorted(offsets, rows, side="right") - 1
    d = np.linalg.norm(a - ref, axis=1)
    rn = np.linalg.norm(ref, axis=1)
    if arms is None:
        B = len(offsets) - 1
        sq = np.bincount(cl, weights=rn * rn, minlength=B)
        cnt = np.bincount(cl, minlength=B)
        arms = np.sqrt(sq / np.maximum(cnt, 1))
    arms_row = np.asarray(arms, dtype=np.float64)[cl]
    out: Dict[str, float] = {"rows": int(m)}
    with np.errstate(divide="ignore", invalid="ignore"):
        moa = np.where(arms_row > 0, d / arms_row, np.where(d == 0, 0.0, np.inf))
    out["max_over_arms"] = float(moa.max()) if m else 0.0
    den = float((rn * rn).sum())
    out["l2"] = float(np.sqrt((d * d).sum() / den)) if den > 0 else (0.0 if not d.any() else float("inf"))
    nz = rn > 0
    rel = d[nz] / rn[nz]
    if rel.size:
        out["rel_median"] = float(np.median(rel))
        out["rel_p99"] = float(np.quantile(rel, 0.99))
        out["rel_max"] = float(rel.max())
    if scale is not None:
        s = np.asarray(scale, dtype=np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            e = np.where(s > 0, d / s, np.where(d == 0, 0.0, np.inf))
            out["s_median"] = float(np.median(e))
            out["s_p99"] = float(np.quantile(e, 0.99))
        out["s_max"] = float(e.max())
    return out


def s_errors(a, ref, scale) -> np.ndarray:
    """Per-row |a_i - r_i| / S_i (0 where both the error and S_i vanish, inf where only S_i does)."""
    d = np.linalg.norm(np.asarray(a, dtype=np.float64) - ref, axis=1)
    s = np.asarray(scale, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(s > 0, d / s, np.where(d == 0, 0.0, np.inf))


def gate(stats: Dict[str, float], prec: str) -> bool:
    """True when the S_i metrics of ``stats`` meet the mode's gates (S_MAX, S_MEDIAN)."""
    return stats["s_max"] <= S_MAX[prec] and stats["s_median"] <= S_MEDIAN[prec]


def short(stats: Dict[str, float], digits: int = 3) -> Dict[str, float]:
    """The metrics rounded for a JSON line."""
    return {k: (v if isinstance(v, int) else float("%.*e" % (digits - 1, v))) for k, v in stats.items()}
