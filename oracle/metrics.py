"""Error measures of the paper's experiments, in FP64.  Test infrastructure only.

Sec. 3.1 prints E1, E2 and L2 in a garbled form: E1 puts a square root over a
signed ratio, E2's numerator subtracts the T=1 sum from itself, and L2 squares
the volume-weighted products but loses the sum and the square in its
denominator.  Reading used here (it reproduces Table 2's regular column):

    E1 = (sum v A |_T - sum v A |_0) / sum v A |_0
    E2 = (sum v A^2 |_T - sum v A^2 |_0) / sum v A^2 |_0
    L2 = sqrt( sum v (A_T - A_0)^2 / sum v A_0^2 )

with the particle volumes taken at the time written.  ``volume_weighted_l2``
is eq. (29) of Sec. 3.3.
"""
from __future__ import annotations

import numpy as np


def e1(v0, a0, vT, aT):
    """Relative change of the volume integral of A (Sec. 3.1, E1 as read above)."""
    s0 = np.sum(v0 * a0)
    return (np.sum(vT * aT) - s0) / s0


def e2(v0, a0, vT, aT):
    """Relative change of the integral of A^2 (Sec. 3.1, E2 as read above)."""
    s0 = np.sum(v0 * a0 * a0)
    return (np.sum(vT * aT * aT) - s0) / s0


def l2(v0, a0, aT):
    """Relative volume-weighted L2 distance between final and initial profiles (Sec. 3.1)."""
    return np.sqrt(np.sum(v0 * (aT - a0) ** 2) / np.sum(v0 * a0 * a0))


def volume_weighted_l2(vol, exact, approx):
    """Sec. 3.3 eq. (29): sqrt(sum V |u_exact - u|^2 / sum V |u_exact|^2)."""
    exact = np.atleast_2d(exact)
    approx = np.atleast_2d(approx)
    num = np.sum(vol * np.sum((exact - approx) ** 2, axis=0))
    den = np.sum(vol * np.sum(exact ** 2, axis=0))
    return np.sqrt(num / den)


def rel_l2(approx, exact):
    """Plain relative l2 error ||approx - exact||_2 / ||exact||_2 (parity gate norm)."""
    exact = np.asarray(exact, dtype=np.float64)
    approx = np.asarray(approx, dtype=np.float64)
    den = np.linalg.norm(exact)
    num = np.linalg.norm(approx - exact)
    return num / den if den > 0 else num


def rel_linf(approx, exact):
    """max |approx - exact| / max |exact| (reported beside the gate)."""
    exact = np.asarray(exact, dtype=np.float64)
    approx = np.asarray(approx, dtype=np.float64)
    den = np.max(np.abs(exact))
    num = np.max(np.abs(approx - exact))
    return num / den if den > 0 else num
