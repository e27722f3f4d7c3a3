"""Host post-processing of the observables (arXiv:1812.05401, Section 3).

* relative L2 error over the fluid nodes (Eq. 20);
* drag and lift coefficients C_D = F_D / (rho U^2 D / 2), C_L = F_L / (rho U^2 D / 2) (Eq. 22);
* Strouhal number St = f D / U (Eq. 23), the shedding frequency f taken from the mean period
  between linearly interpolated upward zero crossings of C_L - mean(C_L), after a moving average
  over 1/20 of the dominant period (found from the periodogram) and with hysteresis, so that
  rounding noise on C_L cannot add crossings; and, as a cross-check that noise cannot bias, f
  from the peak of the Hann-windowed, zero-padded periodogram (parabolic interpolation of the log
  magnitude around the peak bin);
* C_Dave = mean C_D and C_Lrms = rms of C_L - mean(C_L), over a window of the series.
"""
import math

import numpy as np


def l2_error(u, ua, where):
    """Eq. 20 for scalars or stacked vector components: sqrt(sum |u - ua|^2) / sqrt(sum |ua|^2)
    over the nodes selected by the boolean `where` ([ny, nx])."""
    u, ua = np.asarray(u, dtype=np.float64), np.asarray(ua, dtype=np.float64)
    if u.ndim == where.ndim + 1:
        num = sum(np.sum(((a - b) ** 2)[where]) for a, b in zip(u, ua))
        den = sum(np.sum((b ** 2)[where]) for b in ua)
    else:
        num = np.sum(((u - ua) ** 2)[where])
        den = np.sum((ua ** 2)[where])
    return math.sqrt(num / den)


def force_coefficients(fx, fy, u, d, rho=1.0):
    """Eq. 22: (C_D, C_L) from the force components on a body of reference length d."""
    q = 0.5 * rho * u * u * d
    return np.asarray(fx) / q, np.asarray(fy) / q


def upward_crossings(x, hysteresis=0.0):
    """Fractional indices where x crosses zero going up (linear interpolation).  With
    hysteresis h > 0 a crossing counts only if x has been below -h since the previous one."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    armed = hysteresis <= 0.0
    for i in range(len(x) - 1):
        if x[i] < -hysteresis:
            armed = True
        if armed and x[i] < 0 <= x[i + 1]:
            out.append(i + (-x[i]) / (x[i + 1] - x[i]))
            armed = hysteresis <= 0.0
    return np.asarray(out)


def dominant_period(x):
    """Period (in samples) of the strongest non-zero frequency of the periodogram."""
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    spec = np.abs(np.fft.rfft(x * np.hanning(len(x))))
    k = int(np.argmax(spec[1:])) + 1
    return len(x) / k


def strouhal(cl, d, u, min_periods=6):
    """Eq. 23 from a C_L series sampled once per step; None if fewer than `min_periods` full
    periods are present."""
    c = np.asarray(cl, dtype=np.float64)
    c = c - c.mean()
    if len(c) < 16 or not np.any(c):
        return None
    w = max(1, int(dominant_period(c) / 20))
    if w > 1:
        c = np.convolve(c, np.ones(w) / w, mode="valid")
    z = upward_crossings(c, hysteresis=0.5 * float(np.sqrt(np.mean(c * c))))
    if len(z) < min_periods + 1:
        return None
    period = (z[-1] - z[0]) / (len(z) - 1)
    return d / (period * u)


def strouhal_spectral(cl, d, u, pad=16):
    """Eq. 23 with f at the periodogram peak: Hann window, zero padding by `pad`, and a parabola
    through the log magnitudes of the peak bin and its neighbours.  None for a flat series."""
    c = np.asarray(cl, dtype=np.float64)
    c = c - c.mean()
    n = len(c)
    if n < 16 or not np.any(c):
        return None
    spec = np.abs(np.fft.rfft(c * np.hanning(n), n * pad))
    k = int(np.argmax(spec[1:-1])) + 1
    a, b, g = np.log(spec[k - 1:k + 2] + 1e-300)
    den = a - 2 * b + g
    dk = 0.5 * (a - g) / den if den != 0 else 0.0
    return d * (k + dk) / (n * pad) / u


def wake_statistics(fx, fy, u, d, first=0, rho=1.0):
    """C_Dave, C_Lrms and St over steps [first, end) of the per-step force series."""
    cd, cl = force_coefficients(np.asarray(fx)[first:], np.asarray(fy)[first:], u, d, rho)
    cl0 = cl - cl.mean()
    return {"C_Dave": float(cd.mean()), "C_Lrms": float(np.sqrt(np.mean(cl0 ** 2))),
            "St": strouhal(cl, d, u), "St_spectral": strouhal_spectral(cl, d, u),
            "C_Lmean": float(cl.mean()), "samples": int(len(cd))}
