"""Noise measure of optimised pulses (Sec. 3.4, eq. noise), FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

nu_i = int_0^T |Omega_i(t) - Omega_i^smooth(t)| dt, where the smoothed pulse
comes from a Savitzky-Golay filter with a five-point cubic convolute
(Sec. 3.4).  The filter's value at a sample is the value, at that sample, of
the cubic that fits the samples of a five-point window best in the least-
squares sense.

Readings taken here:

* Pulses are piecewise constant on the nt intervals of length dt = T / nt, so
  the integral is dt * sum_j |u_ij - s_ij| over the samples u_ij.
* Window placement: a sample with two neighbours on each side uses the window
  centred on it; the first two (last two) samples use the window of the first
  (last) five samples, evaluated at their own position.  The paper does not say
  how the ends are treated; this is the usual polynomial fit at the edges.
* At least five samples are needed (nt >= 5).
"""

from __future__ import annotations

import numpy as np


def smooth_cubic5(x: np.ndarray) -> np.ndarray:
    """Savitzky-Golay five-point cubic smoothing of a 1-d sequence."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 5:
        raise ValueError("the five-point filter needs at least five samples")
    out = np.empty(n)
    for j in range(n):
        s = min(max(j - 2, 0), n - 5)  # first sample of the window
        pos = np.arange(s, s + 5, dtype=np.float64) - j
        V = np.vander(pos, 4, increasing=True)  # 1, p, p^2, p^3
        coef, *_ = np.linalg.lstsq(V, x[s:s + 5], rcond=None)
        out[j] = coef[0]  # the cubic at position 0 (sample j)
    return out


def pulse_noise(u: np.ndarray, T: float) -> np.ndarray:
    """nu_i for pulses u [n_ctrl, nt] on [0, T] (eq. noise)."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    dt = T / u.shape[1]
    return np.array([dt * np.sum(np.abs(row - smooth_cubic5(row))) for row in u])
