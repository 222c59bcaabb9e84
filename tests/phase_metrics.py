"""Comparison helpers for eigenphase sets (test-side only)."""
import numpy as np

TWO_PI = 2.0 * np.pi


def circ_dist(a, b):
    """Circular distance between angles, elementwise, in [0, pi]."""
    d = np.mod(np.asarray(a) - np.asarray(b) + np.pi, TWO_PI) - np.pi
    return np.abs(d)


def phase_set_error(theta_a, theta_b):
    """Max circular distance between two sets of eigenphases per loop.

    Both are sorted per loop; the best cyclic shift of one against the other
    is taken (a phase at -pi+ and one at pi- are neighbours on the circle).
    Inputs (..., m). Returns the maximum over loops and bands.
    """
    a = np.sort(np.asarray(theta_a, dtype=np.float64), axis=-1)
    b = np.sort(np.asarray(theta_b, dtype=np.float64), axis=-1)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.shape[-1] == 0:
        return 0.0
    a2 = a.reshape(-1, a.shape[-1])
    b2 = b.reshape(-1, b.shape[-1])
    worst = 0.0
    for x, y in zip(a2, b2):
        best = np.inf
        for s in range(x.size):
            best = min(best, float(np.max(circ_dist(np.roll(x, s), y))))
        worst = max(worst, best)
    return worst


def projector_error(U_a, U_b):
    """Max-abs difference of the projectors U U^H of two bases (..., N, m)."""
    Pa = U_a @ np.conj(np.swapaxes(U_a, -1, -2))
    Pb = U_b @ np.conj(np.swapaxes(U_b, -1, -2))
    return float(np.max(np.abs(Pa - Pb))) if Pa.size else 0.0
