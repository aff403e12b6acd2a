"""Gaussian random fields by circulant embedding (spectral synthesis).

Covariance: squared exponential  C(r) = sigma^2 * exp(-r^2 / (2 ell^2)).
The field is sampled on a regular grid of spacing h; the covariance is
embedded in a periodic grid of twice the size per axis, whose circulant
covariance matrix is diagonalised by the FFT.  For a real white-noise vector
w the filtered field F^-1(sqrt(lambda) * F w) has exactly the circulant
covariance, so its marginal variance is sigma^2 (negative embedding
eigenvalues, if any, are clipped to zero).
"""
from __future__ import annotations

import numpy as np


def grf(shape: tuple[int, ...], h: float, sigma: float = 1.0, ell: float = 0.1,
        seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    big = tuple(2 * s for s in shape)
    grids = np.meshgrid(*[np.minimum(np.arange(N), N - np.arange(N)) * h for N in big],
                        indexing="ij")
    r2 = sum(g * g for g in grids)
    c = sigma * sigma * np.exp(-r2 / (2.0 * ell * ell))
    lam = np.real(np.fft.fftn(c))
    lam = np.maximum(lam, 0.0)
    w = rng.standard_normal(big)
    y = np.real(np.fft.ifftn(np.sqrt(lam) * np.fft.fftn(w)))
    sl = tuple(slice(0, s) for s in shape)
    return np.ascontiguousarray(y[sl])
