"""Pins of the error measures (Sec. 3.1 E1, E2, L2 as read; Sec. 3.3 eq. (29))
against values computed by hand on two-particle cases."""
import math

import numpy as np

from oracle import metrics


def test_volume_weighted_l2_two_particles_two_components():
    """eq. (29): the squared error of a particle is summed over the velocity
    components before it is weighted by that particle's volume, and the
    denominator is the same sum over the exact field.  Hand computation:
    vol = (1, 3); exact u = ((1, 0), (2, 1)) per (component, particle);
    approx = ((0, 0), (2, 3)):
      numerator   = 1*((1-0)^2 + (2-2)^2) + 3*((0-0)^2 + (1-3)^2) = 1 + 12 = 13
      denominator = 1*(1 + 4) + 3*(0 + 1) = 8."""
    vol = np.array([1.0, 3.0])
    exact = np.array([[1.0, 0.0], [2.0, 1.0]])
    approx = np.array([[0.0, 0.0], [2.0, 3.0]])
    got = metrics.volume_weighted_l2(vol, exact, approx)
    assert abs(got - math.sqrt(13.0 / 8.0)) < 1e-15
    # the weights belong to the particles, not the components: swapping the
    # volumes changes the value (a transposed weighting would not see it)
    swapped = metrics.volume_weighted_l2(vol[::-1], exact, approx)
    assert abs(swapped - math.sqrt((3.0 * 1.0 + 1.0 * 4.0) / (3.0 * 5.0 + 1.0 * 1.0))) < 1e-15
    # one component: the weighted relative L2 of a scalar field
    got1 = metrics.volume_weighted_l2(vol, exact[0], approx[0])
    assert abs(got1 - math.sqrt((1.0 * 1.0 + 3.0 * 0.0) / (1.0 * 1.0 + 3.0 * 0.0))) < 1e-15
    # exact answer -> 0; scaling both fields leaves it unchanged
    assert metrics.volume_weighted_l2(vol, exact, exact) == 0.0
    assert abs(metrics.volume_weighted_l2(vol, 7 * exact, 7 * approx) - got) < 1e-15


def test_sec31_measures_by_hand():
    """E1, E2, L2 (read as relative changes and the relative weighted distance) on
    v0 = (1, 1), A0 = (1, 0), vT = (2, 1), AT = (0.5, 1):
      E1 = (2*0.5 + 1*1 - 1) / 1 = 1;  E2 = (2*0.25 + 1 - 1) / 1 = 0.5;
      L2 = sqrt((1*0.25 + 1*1) / 1)."""
    v0, a0 = np.array([1.0, 1.0]), np.array([1.0, 0.0])
    vT, aT = np.array([2.0, 1.0]), np.array([0.5, 1.0])
    assert metrics.e1(v0, a0, vT, aT) == 1.0
    assert metrics.e2(v0, a0, vT, aT) == 0.5
    assert abs(metrics.l2(v0, a0, aT) - math.sqrt(1.25)) < 1e-15


def test_parity_norms_by_hand():
    assert abs(metrics.rel_l2([3.0, 4.0], [0.0, 5.0]) - math.sqrt(10.0) / 5.0) < 1e-15
    assert abs(metrics.rel_l2([1.0, 2.0], [1.0, 1.0]) - 1.0 / math.sqrt(2.0)) < 1e-15
    assert abs(metrics.rel_linf([1.0, -3.0], [2.0, -4.0]) - 1.0 / 4.0) < 1e-15
    assert metrics.rel_l2([1.0], [0.0]) == 1.0     # zero reference: absolute error
