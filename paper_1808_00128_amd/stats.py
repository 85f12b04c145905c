"""Chain statistics for the Metropolis sampler: integrated autocorrelation
time and effective sample size by the Gamma method with automatic windowing
(U. Wolff, "Monte Carlo errors with less errors", Comput. Phys. Commun. 156
(2004) 143), the error analysis the paper uses for its QAOA estimates; plus
total variation distance.  Measurement code: it reads chain outputs only.
"""
from __future__ import annotations

import numpy as np


def autocorrelation(series: np.ndarray, max_lag: int) -> np.ndarray:
    """Normalised autocorrelation rho(t), t = 0..max_lag, averaged over replicas.

    series: [R, N] (R independent chains of length N)."""
    a = np.asarray(series, dtype=np.float64)
    if a.ndim == 1:
        a = a[None, :]
    R, N = a.shape
    mean = a.mean()
    d = a - mean
    gamma = np.zeros(max_lag + 1)
    for t in range(max_lag + 1):
        gamma[t] = np.sum(d[:, : N - t] * d[:, t:]) / (R * (N - t))
    if gamma[0] <= 0:
        return np.zeros(max_lag + 1)
    return gamma / gamma[0]


def tau_int(series: np.ndarray, S: float = 1.5):
    """(tau_int, window W, its statistical error) by Wolff's automatic window:
    W is the first lag with g(W) = exp(-W / tau_W) - tau_W / sqrt(W N) < 0,
    tau_W = S / ln((2 tau(W) + 1) / (2 tau(W) - 1)); tau(W) is bias-corrected
    by (1 + (2W + 1) / N)."""
    a = np.asarray(series, dtype=np.float64)
    if a.ndim == 1:
        a = a[None, :]
    R, N = a.shape
    total = R * N
    max_lag = max(1, min(N // 2, 2000))
    rho = autocorrelation(a, max_lag)
    if not np.any(rho):
        return 0.5, 0, 0.0
    tau = 0.5
    W = max_lag
    for w in range(1, max_lag + 1):
        tau += rho[w]
        if tau <= 0.5:
            tau_w = 1e-12
        else:
            tau_w = S / np.log((2 * tau + 1) / (2 * tau - 1))
        g = np.exp(-w / tau_w) - tau_w / np.sqrt(w * total)
        if g < 0:
            W = w
            break
    tau = 0.5 + np.sum(rho[1: W + 1])
    tau *= 1.0 + (2 * W + 1) / total
    err = tau * np.sqrt(4.0 * (W + 0.5 - tau) / total) if W + 0.5 > tau else 0.0
    return float(max(tau, 0.5)), int(W), float(err)


def ess(series: np.ndarray) -> float:
    """Effective sample size: total samples / (2 tau_int)."""
    a = np.asarray(series, dtype=np.float64)
    n = a.size
    t, _, _ = tau_int(a)
    return n / (2.0 * t)


def total_variation(samples: np.ndarray, p: np.ndarray) -> float:
    """TV distance between the empirical law of integer samples and p."""
    hist = np.bincount(np.asarray(samples, dtype=np.int64).ravel(), minlength=p.size)[: p.size]
    hist = hist / max(1, hist.sum())
    return 0.5 * float(np.abs(hist - p).sum())


def qaoa_cost(x: np.ndarray, triples: np.ndarray, d: np.ndarray) -> np.ndarray:
    """C(z) = 1/2 sum_t d_t z_a z_b z_c with z_j = (-1)^{x_j} (Max-E3LIN2 objective)."""
    x = np.asarray(x, dtype=np.uint64)
    out = np.zeros(x.shape, np.float64)
    for (a, b, c), dd in zip(np.asarray(triples).tolist(), np.asarray(d).tolist()):
        par = ((x >> np.uint64(a)) ^ (x >> np.uint64(b)) ^ (x >> np.uint64(c))) & np.uint64(1)
        out += 0.5 * dd * (1.0 - 2.0 * par.astype(np.float64))
    return out
