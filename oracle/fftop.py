"""The coefficient matrix applied by FFT convolution (oracle side; test infrastructure).

Paper Sec. 5 (and the end of Sec. 2.2): G + T is a convolution on the regular
grid, so A x = x + kappa^2 b (K * x) is applied with a zero-padded circulant
embedding of size 2n x 2n.
"""
from __future__ import annotations

import numpy as np

from . import dense


class FFTOperator:
    def __init__(self, n: int, kappa: float, order: int):
        self.n, self.kappa = n, kappa
        Koff = dense.kernel_offsets(n, kappa, order)  # offsets -(n-1) .. n-1
        m = 2 * n
        C = np.zeros((m, m), dtype=complex)
        # circulant embedding: C[dy mod m, dx mod m] = K(dx, dy)
        d = np.arange(-(n - 1), n)
        C[np.ix_(d % m, d % m)] = Koff
        self.khat = np.fft.fft2(C)

    def conv(self, x):
        """(K x) for x of shape (..., n, n) in [i2, i1] order."""
        n, m = self.n, 2 * self.n
        x = np.asarray(x, dtype=complex).reshape(-1, n, n)
        P = np.zeros((x.shape[0], m, m), dtype=complex)
        P[:, :n, :n] = x
        y = np.fft.ifft2(self.khat[None] * np.fft.fft2(P))
        return y[:, :n, :n]

    def apply(self, b, x):
        """A x = x + kappa^2 b (K x)."""
        n = self.n
        x = np.asarray(x, dtype=complex).reshape(-1, n, n)
        return x + self.kappa ** 2 * np.asarray(b, dtype=float).reshape(1, n, n) * self.conv(x)
