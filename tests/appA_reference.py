"""Closed-form solution of the planar heated two-layer channel (App. A,
"Analytic solution of planar heated channel").

Coordinates follow the appendix: x along the channel, y normal to the flat
interface with y = 0 on the interface, the lower layer (``b``) in -b < y <= 0
and the upper layer (``a``) in 0 < y < a.  The lower wall is held at
T_h + T_0 cos(omega x), the upper wall at T_c.  k_r is the conductivity ratio
and mu_r the viscosity ratio of the two layers; mu_h is the viscosity that
scales U_max.
"""
from __future__ import annotations

import numpy as np


def planar_channel(x, y, a, b, omega, T_h, T_c, T_0, sigma_t, mu_h, k_r=1.0, mu_r=1.0):
    """Return (u, v, T) of App. A at the points (x, y) (numpy broadcasting)."""
    ar, br = a * omega, b * omega
    f = 1.0 / (k_r * np.sinh(br) * np.cosh(ar) + np.sinh(ar) * np.cosh(br))
    Da = np.sinh(ar) ** 2 - ar ** 2
    Db = np.sinh(br) ** 2 - br ** 2
    C1a, C1b = np.sinh(ar) ** 2 / Da, np.sinh(br) ** 2 / Db
    C2a, C2b = -a * ar / Da, -b * br / Db
    C3a = (2 * ar - np.sinh(2 * ar)) / (2 * Da)
    C3b = (-2 * br + np.sinh(2 * br)) / (2 * Db)
    g = np.sinh(ar) * f
    h = (Da * Db) / (mu_r * Db * (np.sinh(2 * ar) - 2 * ar) + Da * (np.sinh(2 * br) - 2 * br))
    umax = -(T_0 * sigma_t / mu_h) * g * h
    upper = y > 0
    C1 = np.where(upper, C1a, C1b)
    C2 = np.where(upper, C2a, C2b)
    C3 = np.where(upper, C3a, C3b)
    wy = omega * y
    u = umax * ((C1 + omega * (C2 + C3 * y)) * np.cosh(wy) + (C3 + omega * C1 * y) * np.sinh(wy)) * np.sin(omega * x)
    v = -omega * umax * (C1 * y * np.cosh(wy) + (C2 + C3 * y) * np.sinh(wy)) * np.cos(omega * x)
    # Conduction part (Ma -> 0), k_r = k_a / k_b.  Solving the Laplace equation in
    # each layer with the wall values and continuity of T and k dT/dy at y = 0
    # gives the appendix's two cosine terms with the layers exchanged (the k_r
    # term belongs to the lower layer) and a lower-layer linear slope k_r times
    # the upper one; for k_r = 1 both coincide with the printed form.
    lin_a = ((T_c - T_h) * y + k_r * T_c * b + T_h * a) / (a + k_r * b)
    lin_b = (k_r * (T_c - T_h) * y + k_r * T_c * b + T_h * a) / (a + k_r * b)
    Ta = lin_a + T_0 * f * np.sinh(ar - wy) * np.cos(omega * x)
    Tb = lin_b + T_0 * f * (np.sinh(ar) * np.cosh(wy) - k_r * np.sinh(wy) * np.cosh(ar)) * np.cos(omega * x)
    T = np.where(upper, Ta, Tb)
    return u, v, T


def l2(num, ref):
    """Relative l2 norm of the magnitudes (Sec. 3.1 error norm)."""
    return float(np.sqrt(np.sum((np.abs(num) - np.abs(ref)) ** 2) / np.sum(np.abs(ref) ** 2)))
