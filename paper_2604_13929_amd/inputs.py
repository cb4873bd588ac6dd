"""Seeded synthetic inputs: bicontinuous pore masks and batch job tables.

This module only *generates inputs*.  It holds none of the transport
arithmetic, so both the HIP path and the FP64 oracle can take their masks from
it without sharing any of the method.

Mask construction (a stand-in for the paper's Cahn-Hilliard masks, which are
not public): Cahn's random-wave construction of a Gaussian random field,

    f(x) = sum_{i < n_waves} cos(k_i . (x + 1/2) + theta_i),   |k_i| = 2 pi / lambda,

with directions uniform on the sphere and phases uniform in [0, 2 pi), both
drawn from ``numpy.random.default_rng(seed)``, evaluated in FP64 at voxel
centres.  The binary mask is then obtained by rank-based thresholding as the
paper does for its own field (App. A, Binarisation): the round(phi * N_vox)
voxels with the highest field value are labelled pore (1), the rest solid (0),
ties going to the lower linear index, so the achieved porosity is exact.
Layout: ``uint8[nz][ny][nx]``, x fastest.

The field is separable per wave, e^{i k.x} = e^{i kx x} e^{i ky y} e^{i kz z},
so it is evaluated as a complex matrix product over the wave index, in z-chunks.
"""
from __future__ import annotations

import math

import numpy as np

#: transport seed of the paper's production runs (App. B, Statistics)
PAPER_TRANSPORT_SEED = 20260809
#: geometry seed of the paper's production masks (App. A, Initial condition)
PAPER_MASK_SEED = 0


def wave_vectors(wavelength: float, seed: int, n_waves: int = 256):
    """Directions uniform on the unit sphere, |k| = 2 pi / wavelength, and phases."""
    rng = np.random.default_rng(seed)
    cos_t = 1.0 - 2.0 * rng.random(n_waves)
    azim = 2.0 * math.pi * rng.random(n_waves)
    phase = 2.0 * math.pi * rng.random(n_waves)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    kmag = 2.0 * math.pi / float(wavelength)
    k = np.stack([kmag * sin_t * np.cos(azim), kmag * sin_t * np.sin(azim), kmag * cos_t], axis=1)
    return k, phase


def cahn_field(nx: int, ny: int, nz: int, wavelength: float, seed: int, n_waves: int = 256) -> np.ndarray:
    """FP64 random-wave field sampled at voxel centres, shape (nz, ny, nx)."""
    k, phase = wave_vectors(wavelength, seed, n_waves)
    xs = np.arange(nx, dtype=np.float64) + 0.5
    ys = np.arange(ny, dtype=np.float64) + 0.5
    zs = np.arange(nz, dtype=np.float64) + 0.5
    ex = np.exp(1j * np.outer(k[:, 0], xs))                 # (W, nx)
    ey = np.exp(1j * np.outer(k[:, 1], ys))                 # (W, ny)
    ez = np.exp(1j * (np.outer(zs, k[:, 2]) + phase))       # (nz, W)
    field = np.empty((nz, ny, nx), dtype=np.float64)
    # plane[w, y, x] = ey[w, y] * ex[w, x]; field[z] = Re(ez[z, :] @ plane)
    ychunk = max(1, min(ny, (1 << 24) // max(1, n_waves * nx)))
    for y0 in range(0, ny, ychunk):
        y1 = min(ny, y0 + ychunk)
        plane = (ey[:, y0:y1, None] * ex[:, None, :]).reshape(n_waves, -1)
        field[:, y0:y1, :] = (ez @ plane).real.reshape(nz, y1 - y0, nx)
    return field


def rank_threshold(field: np.ndarray, porosity: float) -> np.ndarray:
    """Label the round(phi * N) highest values pore (1); ties to the lower linear index."""
    flat = np.ascontiguousarray(field).reshape(-1)
    n = flat.size
    n_pore = int(round(porosity * n))
    mask = np.zeros(n, dtype=np.uint8)
    if n_pore <= 0:
        return mask.reshape(field.shape)
    if n_pore >= n:
        mask[:] = 1
        return mask.reshape(field.shape)
    # value of the n_pore-th largest element
    thr = np.partition(flat, n - n_pore)[n - n_pore]
    above = flat > thr
    mask[above] = 1
    need = n_pore - int(above.sum())
    if need > 0:
        ties = np.flatnonzero(flat == thr)[:need]
        mask[ties] = 1
    return mask.reshape(field.shape)


def spinodal_mask(nx: int, ny: int, nz: int, wavelength: float, porosity: float,
                  seed: int = PAPER_MASK_SEED, n_waves: int = 256) -> np.ndarray:
    """Binary bicontinuous mask uint8[nz][ny][nx] (1 = pore) with exact porosity."""
    return rank_threshold(cahn_field(nx, ny, nz, wavelength, seed, n_waves), porosity)


def spinodal_mask_torch(nx: int, ny: int, nz: int, wavelength: float, porosity: float, seed: int = PAPER_MASK_SEED,
                        n_waves: int = 256, device="cuda"):
    """The same construction evaluated with torch (FP64, complex matmul) on ``device``.

    Returns a contiguous uint8 tensor [nz, ny, nx] on that device.  It differs from
    ``spinodal_mask`` only where two field values lie within rounding of the
    threshold; use one generator per experiment.
    """
    import torch

    k, phase = wave_vectors(wavelength, seed, n_waves)
    kt = torch.as_tensor(k, dtype=torch.float64, device=device)
    ph = torch.as_tensor(phase, dtype=torch.float64, device=device)
    xs = torch.arange(nx, dtype=torch.float64, device=device) + 0.5
    ys = torch.arange(ny, dtype=torch.float64, device=device) + 0.5
    zs = torch.arange(nz, dtype=torch.float64, device=device) + 0.5
    ex = torch.polar(torch.ones(n_waves, nx, dtype=torch.float64, device=device), torch.outer(kt[:, 0], xs))
    ey = torch.polar(torch.ones(n_waves, ny, dtype=torch.float64, device=device), torch.outer(kt[:, 1], ys))
    ez = torch.polar(torch.ones(nz, n_waves, dtype=torch.float64, device=device), torch.outer(zs, kt[:, 2]) + ph)
    plane = (ey[:, :, None] * ex[:, None, :]).reshape(n_waves, ny * nx)
    field = torch.matmul(ez, plane).real.reshape(-1)
    n = field.numel()
    n_pore = int(round(porosity * n))
    mask = torch.zeros(n, dtype=torch.uint8, device=device)
    if n_pore > 0:
        order = torch.sort(-field, stable=True).indices   # highest first, ties by lower index
        mask[order[:n_pore]] = 1
    return mask.reshape(nz, ny, nx).contiguous()


def ch_initial_field(nx: int, ny: int, nz: int, seed: int = PAPER_MASK_SEED, amplitude: float = 0.05) -> np.ndarray:
    """Initial condition of the Cahn-Hilliard generator (App. A): 0.5 plus independent
    Gaussian noise of standard deviation `amplitude` per voxel, clipped to [0, 1];
    numpy.random.default_rng(seed), float64 [nz, ny, nx]."""
    rng = np.random.default_rng(seed)
    return np.clip(0.5 + amplitude * rng.standard_normal((nz, ny, nx)), 0.0, 1.0)


def homogeneous_mask(nx: int, ny: int, nz: int, pore: bool = False) -> np.ndarray:
    """All-solid (or all-pore) slab."""
    return np.full((nz, ny, nx), 1 if pore else 0, dtype=np.uint8)


def batch_jobs(seed: int = 0, n_jobs: int = 64, wavelength: float = 16.0,
               side_min: int = 64, side_max: int = 256):
    """Job parameters of the uneven multi-mask batch, all drawn from ``seed``.

    side ~ U{side_min..side_max}, phi from {0.5,...,0.9}, solid mu_s in [0.2, 1.0],
    mu_a in [0.005, 0.05], g in [0.5, 0.9] (float32-representable), N log-uniform
    in [1e6, 1e7]; the mask of job j uses seed 1000 + j and the job's stream id is j.
    """
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        u = rng.random(6)
        side = side_min + int(math.floor((side_max - side_min + 1) * u[0]))
        phi = [0.5, 0.6, 0.7, 0.8, 0.9][int(math.floor(5 * u[1]))]
        jobs.append(dict(
            job=j, nx=side, ny=side, nz=side, porosity=phi, wavelength=wavelength,
            mask_seed=1000 + j,
            mu_s=float(np.float32(0.2 + 0.8 * u[2])),
            mu_a=float(np.float32(0.005 + 0.045 * u[3])),
            g=float(np.float32(0.5 + 0.4 * u[4])),
            n_photons=int(round(10.0 ** (6.0 + u[5]))),
            stream_id=j,
        ))
    return jobs


#: The workloads (voxel units, 1 voxel = 1 um).  mu values are float32-representable
#: numbers as the transport sees them.
WORKLOADS = {
    "M1": dict(nx=32, ny=32, nz=32, wavelength=8.0, porosity=0.70, n_photons=100_000),
    "M2a": dict(nx=256, ny=256, nz=256, wavelength=24.0, porosity=0.70, n_photons=100_000_000),
    "M2b": dict(nx=256, ny=256, nz=256, wavelength=24.0, porosity=0.90, n_photons=100_000_000),
    "M3": dict(nx=512, ny=512, nz=256, wavelength=32.0, porosity=0.90, n_photons=100_000_000),
}
SOLID_OPTICS = dict(mu_s=0.5, mu_a=float(np.float32(0.01)), g=float(np.float32(0.7)))
