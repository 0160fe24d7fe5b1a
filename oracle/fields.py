"""Seeded initial fields and the first guess (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Random numbers.  The initial fields draw random phases / Gaussian amplitudes.
Both this oracle and the GPU library implement the same counter-based
generator from its published definition, SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): the n-th
output of the stream seeded with `seed` is mix(seed + n * 0x9E3779B97F4A7C15)
with the mix64 finaliser

    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31                                            (all mod 2^64).

A draw is keyed by the wavevector, so a seed gives the same low modes at every
grid size: n = 1 + stream + 4 * ((kx + 2048) + 4096 * (ky + 2048)) for the
representative (kx, ky) of the half plane {ky > 0} or {ky = 0, kx > 0}.  A
uniform number on [0, 1) is (z >> 11) * 2^-53.

Initial field (Sec. III: prescribed isotropic spectrum, random phases,
divergence-free, normalised energy).  The vorticity spectrum has modulus
sqrt(|k| E(|k|)) with E(k) = k^4 exp(-2 (k/k0)^2) on the half plane inside the
de-aliased band S, Hermitian mirror on the other half:
  kind 0: random phase        omega_hat = A(k) exp(2 pi i U)
  kind 1: Gaussian            omega_hat = A(k) (xi1 + i xi2) / sqrt(2)  (Box-Muller)
  kind 2: white noise in S    omega_hat = (xi1 + i xi2) / sqrt(2)
Kinds 0 and 1 are scaled to kinetic energy 1/2 <|u|^2> = target; kind 2 to
RMS(omega) = target.  A vorticity field is divergence-free by construction.
"""

import numpy as np

from .dft import fft2, ifft2
from .model import grid

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
KEY_OFFSET = 2048
KEY_SPAN = 4096


def splitmix64(seed, index):
    """index-th output (index >= 1) of SplitMix64 seeded with seed (uint64 arrays)."""
    seed = np.asarray(seed, dtype=np.uint64)
    index = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = seed + index * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(z):
    """53-bit uniform in [0, 1)."""
    return (np.asarray(z, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def mode_index(kx, ky, stream):
    kx = np.asarray(kx, dtype=np.int64)
    ky = np.asarray(ky, dtype=np.int64)
    return (1 + stream + 4 * ((kx + KEY_OFFSET) + KEY_SPAN * (ky + KEY_OFFSET))).astype(np.uint64)


def _half_plane_representative(kx, ky):
    """(kx, ky) if in {ky > 0} or {ky = 0, kx > 0}, else (-kx, -ky); and whether it flipped."""
    inside = (ky > 0) | ((ky == 0) & (kx > 0))
    return np.where(inside, kx, -kx), np.where(inside, ky, -ky), ~inside


def draw(seed, kx, ky, stream):
    return uniform01(splitmix64(np.uint64(seed), mode_index(kx, ky, stream)))


def energy_spectrum(kappa, k0):
    """E(k) = k^4 exp(-2 (k / k0)^2)."""
    return kappa ** 4 * np.exp(-2.0 * (kappa / k0) ** 2)


def init_field(N, seeds, kind=0, k0=4.0, target=0.5):
    """Physical vorticity fields [B][N][N] for the given seeds."""
    g = grid(N)
    out = []
    kx = g.ikx
    ky = g.iky
    rx, ry, flipped = _half_plane_representative(kx, ky)
    kappa = np.sqrt(g.k2)
    for seed in seeds:
        if kind == 0:
            U = draw(seed, rx, ry, 0)
            z = np.cos(2.0 * np.pi * U) + 1j * np.sin(2.0 * np.pi * U)
            amp = np.sqrt(kappa * energy_spectrum(kappa, k0))
        else:
            U1 = draw(seed, rx, ry, 1)
            U2 = draw(seed, rx, ry, 2)
            rad = np.sqrt(-2.0 * np.log(1.0 - U1))
            z = rad * (np.cos(2.0 * np.pi * U2) + 1j * np.sin(2.0 * np.pi * U2)) / np.sqrt(2.0)
            amp = np.sqrt(kappa * energy_spectrum(kappa, k0)) if kind == 1 else np.ones_like(kappa)
        z = np.where(flipped, np.conj(z), z)
        w_hat = g.mask * amp * z
        if kind in (0, 1):
            energy = 0.5 * float(np.sum(np.abs(w_hat) ** 2 * g.inv_k2)) / N ** 4
            w_hat = w_hat * np.sqrt(target / energy)
        else:
            rms = np.sqrt(float(np.sum(np.abs(w_hat) ** 2))) / N ** 2
            w_hat = w_hat * (target / rms)
        out.append(np.real(ifft2(w_hat)))
    return np.array(out)


def first_guess(N, stride, probes_uv):
    """Spectral interpolation of the probe velocities at t = 0 to a vorticity field.

    The paper starts from "the initial interpolated state" (Sec. III.A).  The
    coarse M x M probe grid (M = N / stride) is transformed, its Nyquist row and
    column are dropped, the coefficients are placed at the same wavenumbers of
    the N grid (scaled by (N/M)^2 for the unnormalised transforms), and the
    vorticity i kx v - i ky u is projected onto S.
    """
    g = grid(N)
    M = N // stride
    uh_c = fft2(probes_uv[0])
    vh_c = fft2(probes_uv[1])
    kc = np.arange(M)
    kc[kc >= M // 2] -= M
    keep = np.abs(kc) < (M + 1) // 2 if M % 2 else np.abs(kc) < M // 2
    uh = np.zeros((N, N), dtype=np.complex128)
    vh = np.zeros((N, N), dtype=np.complex128)
    scale = (N / M) ** 2
    for qc in range(M):
        if not keep[qc]:
            continue
        for pc in range(M):
            if not keep[pc]:
                continue
            q = kc[qc] % N
            p = kc[pc] % N
            uh[q, p] = scale * uh_c[qc, pc]
            vh[q, p] = scale * vh_c[qc, pc]
    w_hat = g.mask * (1j * g.kx * vh - 1j * g.ky * uh)
    return np.real(ifft2(w_hat))
