"""Taylor's absolute dispersion (the check of the channel's centreline source,
Sec. III.A) in the closed forms that the dispersion tests compare with.

In homogeneous turbulence with frozen fields, the cross-stream particle
velocity of Eq.(4) is an Ornstein-Uhlenbeck process,
  v^{n+1} = a v^n + s xi,  a = 1 + G_22 dt,  s^2 = C0 eps dt,
and Eq.(2) moves the particle by y^{n+1} = y^n + v^n dt + (2 nu dt)^{1/2} xi'
(xi' independent of xi). Started from the stationary variance sig2 =
s^2 / (1 - a^2), the displacement after n steps has the variance
  dt^2 sig2 [n + 2 sum_{k=1}^{n-1} (n - k) a^k] + 2 nu n dt,
the discrete form of Taylor's result, which tends as dt -> 0 to
  2 sig2 T^2 (t/T - 1 + e^{-t/T}) + 2 nu t,  T = -1/G_22, t = n dt.
The mean concentration of a puff is then the initial distribution spread by
a Gaussian of that variance.
"""
import math

import numpy as np


def discrete_variance(n: int, dt: float, G: float, sig2: float, nu: float) -> float:
    a = 1.0 + G * dt
    k = np.arange(1, n, dtype=np.float64)
    return dt * dt * sig2 * (n + 2.0 * float(np.sum((n - k) * a ** k))) + 2.0 * nu * dt * n


def taylor_variance(t: float, T: float, sig2: float, nu: float) -> float:
    return 2.0 * sig2 * T * T * (t / T - 1.0 + math.exp(-t / T)) + 2.0 * nu * t


def stationary_c0eps(G: float, dt: float, sig2: float) -> float:
    """C0 eps that makes sig2 the stationary variance of the discrete process."""
    a = 1.0 + G * dt
    return sig2 * (1.0 - a * a) / dt


def band_profile(y, y0: float, h0: float, var: float):
    """Mean concentration across a band |y - y0| < h0 of unit concentration
    after spreading by a Gaussian of variance var."""
    s = math.sqrt(2.0 * var)
    y = np.asarray(y, np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * (erf((y - y0 + h0) / s) - erf((y - y0 - h0) / s))
