"""Load-time functions of Sec. 5 (eqs. Ricker, Triangle, Lamb)."""

import math

import numpy as np


def ricker(t, t1, P0=1.0):
    """Ricker wavelet, eq. Ricker: (1 - tau^2) exp(-tau^2/2) P0, tau = (t - t1)/(t1/5)."""
    tau = (np.asarray(t, dtype=np.float64) - t1) / (t1 / 5.0)
    return (1.0 - tau * tau) * np.exp(-0.5 * tau * tau) * P0


def ricker_fm(t1):
    """Centre frequency of the Ricker wavelet, eq. Ricker_fm."""
    return 5.0 / (math.sqrt(2.0) * math.pi * t1)


def triangle(t, t1, P0=1.0):
    """Triangular pulse, eq. Triangle."""
    t = np.asarray(t, dtype=np.float64)
    return np.where((t >= 0) & (t <= 2 * t1), (1.0 - np.abs(t / t1 - 1.0)) * P0, 0.0)


def sine_burst(t, t1, n=5, P0=1.0):
    """Hann-windowed sine burst, eq. Lamb."""
    t = np.asarray(t, dtype=np.float64)
    val = np.sin(2 * np.pi * n * t / t1) * np.sin(np.pi * t / t1) ** 2 * P0
    return np.where((t >= 0) & (t <= t1), val, 0.0)


def table(t, P, dt):
    """P(t_n) given per step (R_ext at t_n = n dt, Alg. 1): P[n] for 0 <= n < len(P), 0 after."""
    P = np.asarray(P, dtype=np.float64)
    n = np.floor(np.asarray(t, dtype=np.float64) / dt + 0.5).astype(np.int64)
    inside = (n >= 0) & (n < len(P))
    return np.where(inside, P[np.clip(n, 0, len(P) - 1)], 0.0)


def evaluate(load, t):
    kind = load.get("kind", "ricker")
    if kind == "table":
        return table(t, load["P"], load["dt"])
    if kind == "ricker":
        return ricker(t, load["t1"], load.get("P0", 1.0))
    if kind == "triangle":
        return triangle(t, load["t1"], load.get("P0", 1.0))
    if kind == "sine_burst":
        return sine_burst(t, load["t1"], load.get("cycles", 5), load.get("P0", 1.0))
    raise ValueError(f"unknown load kind {kind}")
