"""Plain discrete Fourier transform on the periodic grid (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Convention (the paper works on the doubly periodic box [0, 2pi)^2, Sec. III):
grid points x_i = 2 pi i / N, y_j = 2 pi j / N, arrays indexed f[j][i]
(y first, x fastest).  Forward transform

    fhat[q][p] = sum_{j,i} f[j][i] exp(-2 pi i (p i + q j) / N)

and inverse  f = N^-2 sum fhat exp(+...).  Index p <-> wavenumber kx = p for
p < N/2 and p - N otherwise (integer wavenumbers because L = 2 pi).

The 1D matrix uses the exact reduction (k j) mod N of the exponent and a
table of exp(-2 pi i m / N) built from the first octant by exact quarter-turn
and reflection symmetries, so every twiddle is within about one ulp.
"""

import numpy as np


def twiddles(N):
    """Return (cos, sin) of 2 pi m / N for m = 0..N-1, octant-reduced."""
    m = np.arange(N, dtype=np.int64)
    q, r = np.divmod(4 * m, N)          # angle = (pi/2) (q + r/N)
    flip = 2 * r > N                    # residual angle above pi/4
    rr = np.where(flip, N - r, r)       # reflect: pi/2 - phi
    ang = (np.pi / 2.0) * rr.astype(np.float64) / N
    c, s = np.cos(ang), np.sin(ang)
    cphi = np.where(flip, s, c)
    sphi = np.where(flip, c, s)
    q = q % 4
    cos_t = np.select([q == 0, q == 1, q == 2, q == 3], [cphi, -sphi, -cphi, sphi])
    sin_t = np.select([q == 0, q == 1, q == 2, q == 3], [sphi, cphi, -sphi, -cphi])
    return cos_t, sin_t


_CACHE = {}


def dft_matrix(N):
    """Symmetric N x N matrix F[k][j] = exp(-2 pi i (k j mod N) / N)."""
    if N not in _CACHE:
        c, s = twiddles(N)
        idx = np.outer(np.arange(N), np.arange(N)) % N
        _CACHE[N] = c[idx] - 1j * s[idx]
    return _CACHE[N]


def fft2(f):
    """Unnormalised forward 2D DFT over the last two axes (batched)."""
    F = dft_matrix(f.shape[-1])
    return F @ np.asarray(f, dtype=np.complex128) @ F


def ifft2(fhat):
    """Inverse 2D DFT (1/N^2 normalisation) over the last two axes."""
    N = fhat.shape[-1]
    Fc = np.conj(dft_matrix(N))
    return (Fc @ fhat @ Fc) / (N * N)
