"""Fits used by the physics tests: damped sinusoid (optionally plus a decaying offset)."""
import numpy as np
from scipy.optimize import curve_fit


def fit_damped_cosine(t, a, k, c_guess, g_guess, offset=False):
    """Fit a(t) = A exp(-g t) cos(w t + ph) [+ C exp(-h t)]; returns (w, g)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    A0 = np.abs(a).max()
    if offset:
        f = lambda t, A, g, w, ph, C, h: A * np.exp(-g * t) * np.cos(w * t + ph) + C * np.exp(-h * t)
        p0 = [A0, g_guess, k * c_guess, 0.0, 0.0, g_guess]
    else:
        f = lambda t, A, g, w, ph: A * np.exp(-g * t) * np.cos(w * t + ph)
        p0 = [A0, g_guess, k * c_guess, 0.0]
    p, _ = curve_fit(f, t, a, p0=p0, maxfev=20000)
    return abs(p[2]), p[1]


def mode_amplitude(q, k, x):
    """Cosine Fourier coefficient of a periodic 1-D profile."""
    return 2.0 / q.size * np.sum(q * np.cos(k * x))


def sine_amplitude(q, k, x):
    return 2.0 / q.size * np.sum(q * np.sin(k * x))
