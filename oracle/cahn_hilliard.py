"""FP64 oracle of the Cahn-Hilliard spinodal mask generator (numpy, FFT-based).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU baseline use it; the
product library never imports it and it never imports the product.

What it follows (paper: "Three-dimensional photon transport in spinodal
photocatalytic aerogels", Sec. 2.2 and App. A):
  - Eq. CH with the double well f(phi) = phi^2 (1 - phi)^2, mobility M = 1;
  - Eq. CH_spectral, the semi-implicit Fourier spectral step
        phihat^{n+1}_k = (phihat^n_k - dt k^2 [f'(phi^n)]^_k) / (1 + dt kappa k^4),
    with k the angular wavenumber per voxel on each axis (2 pi m / N, m the
    signed frequency index), k^2 = kx^2 + ky^2 + kz^2;
  - Eq. kappa_cal, kappa = (1/2) (d_target / (8 pi))^2 in voxel units;
  - App. A: dt = min(0.5 / (kappa k_max^4), 1) with k_max = pi; the dominant size
    is the peak of the radial power spectral density, checked every 200 steps;
    integration stops when it enters [d_target - sigma/2, d_target + sigma/2] or
    after a hard cap; the binary mask is the rank threshold of the final field.
Readings where the paper is silent (listed with their reasons in the design
notes): the radial PSD is |phihat|^2 summed over shells of width 2 pi / N_max in
|k| (shell s holds s - 1/2 <= |k| N_max / (2 pi) < s + 1/2), the mean (k = 0)
excluded; the dominant size is half the wavelength of the peak shell,
pi / k_peak (one pore and one strut per period); the initial field is an input
(0.5 + N(0, 0.05^2) noise clipped to [0, 1] in the paper), so both sides start
from the same numbers.

The transform is numpy's real FFT (pocketfft) in double precision: a library
primitive used as one step, with nothing fused or reordered.
"""
from __future__ import annotations

import math

import numpy as np


def f_prime(phi: np.ndarray) -> np.ndarray:
    """f'(phi) for f = phi^2 (1 - phi)^2: 2 phi (1 - phi) (1 - 2 phi)."""
    return 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)


def f_second(phi):
    """f''(phi) = 2 - 12 phi + 12 phi^2 (negative inside the spinodal interval)."""
    return 2.0 - 12.0 * phi + 12.0 * phi * phi


def kappa_from_target(d_target_voxels: float) -> float:
    """Eq. kappa_cal in voxel units."""
    return 0.5 * (d_target_voxels / (8.0 * math.pi)) ** 2


def dt_from_kappa(kappa: float, k_max: float = math.pi) -> float:
    """App. A: the step limited by the explicit nonlinear term."""
    return min(0.5 / (kappa * k_max ** 4), 1.0)


def wavenumbers(shape):
    """k^2 on the rfftn grid of a field of shape (nz, ny, nx): shape (nz, ny, nx//2+1)."""
    nz, ny, nx = shape
    kz = 2.0 * math.pi * np.fft.fftfreq(nz)
    ky = 2.0 * math.pi * np.fft.fftfreq(ny)
    kx = 2.0 * math.pi * np.fft.rfftfreq(nx)
    return kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2


def spectrum(phi: np.ndarray) -> np.ndarray:
    """phihat = rfftn(phi) (unnormalised forward transform)."""
    return np.fft.rfftn(np.asarray(phi, dtype=np.float64))


def field(phihat: np.ndarray, shape) -> np.ndarray:
    """phi = irfftn(phihat) on the real grid of `shape`."""
    return np.fft.irfftn(phihat, s=shape, axes=(0, 1, 2))


def steps(phihat: np.ndarray, shape, n: int, dt: float, kappa: float) -> np.ndarray:
    """n steps of Eq. CH_spectral from phihat; returns the new spectrum."""
    k2 = wavenumbers(shape)
    denom = 1.0 + dt * kappa * k2 * k2
    ph = phihat.copy()
    for _ in range(n):
        phi = field(ph, shape)
        ph = (ph - dt * k2 * spectrum(f_prime(phi))) / denom
    return ph


def radial_psd(phihat: np.ndarray, shape) -> np.ndarray:
    """Sum of |phihat|^2 over shells of |k| (see the reading above), counting both
    halves of the real spectrum: psd[s] for s = 0 .. N_max/2 (s = 0 is empty: the
    mean is excluded).  The rfft axis holds each conjugate pair once, so modes with
    0 < kx_index < nx/2 are counted twice."""
    nz, ny, nx = shape
    nmax = max(shape)
    k2 = wavenumbers(shape)
    shell = np.floor(np.sqrt(k2) * nmax / (2.0 * math.pi) + 0.5).astype(np.int64)
    weight = np.full(k2.shape, 2.0)
    weight[:, :, 0] = 1.0
    if nx % 2 == 0:
        weight[:, :, -1] = 1.0
    p = (np.abs(phihat) ** 2) * weight
    p[0, 0, 0] = 0.0
    nb = nmax // 2 + 1
    keep = shell < nb
    return np.bincount(shell[keep].ravel(), weights=p[keep].ravel(), minlength=nb)[:nb]


def dominant_size(psd: np.ndarray, shape) -> float:
    """pi / k_peak of the peak shell (shell s has |k| = 2 pi s / N_max)."""
    s = int(np.argmax(psd[1:])) + 1
    return max(shape) / (2.0 * s)


def rank_threshold(phi: np.ndarray, porosity: float) -> np.ndarray:
    """The round(porosity N) voxels of highest phi are pore (1); equal values go to
    the lower linear index first (a stable sort of -phi)."""
    flat = np.asarray(phi, dtype=np.float64).ravel()
    n_pore = int(round(porosity * flat.size))
    order = np.argsort(-flat, kind="stable")
    mask = np.zeros(flat.size, dtype=np.uint8)
    mask[order[:n_pore]] = 1
    return mask.reshape(np.shape(phi))


def generate(phi0: np.ndarray, d_target: float, sigma: float, porosity: float, check_every: int = 200,
             max_steps: int = 50_000, dt: float | None = None, kappa: float | None = None):
    """App. A's loop: evolve from phi0, check the dominant size every `check_every`
    steps, stop when it lies in [d_target - sigma/2, d_target + sigma/2] or at the
    cap; binarise.  Returns (mask, field, steps_taken, sizes_seen)."""
    shape = phi0.shape
    kappa = kappa_from_target(d_target) if kappa is None else kappa
    dt = dt_from_kappa(kappa) if dt is None else dt
    ph = spectrum(phi0)
    n = 0
    sizes = []
    while n < max_steps:
        m = min(check_every, max_steps - n)
        ph = steps(ph, shape, m, dt, kappa)
        n += m
        size = dominant_size(radial_psd(ph, shape), shape)
        sizes.append(size)
        if d_target - 0.5 * sigma <= size <= d_target + 0.5 * sigma:
            break
    phi = field(ph, shape)
    return rank_threshold(phi, porosity), phi, n, sizes
