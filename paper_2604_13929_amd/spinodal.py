"""Python binding of the Cahn-Hilliard spinodal mask generator (include/spinodal.h).

Argument marshalling only: torch allocates device memory, libphotonmc.so computes.
The spectrum is a complex128 tensor [nz, ny, nx//2 + 1] (numpy.fft.rfftn layout).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import photonmc as pm


def kappa_from_target(d_target_voxels: float) -> float:
    """Eq. kappa_cal: kappa_CH = (1/2) (d_target / (8 pi))^2, voxel units."""
    return 0.5 * (d_target_voxels / (8.0 * math.pi)) ** 2


def dt_from_kappa(kappa: float) -> float:
    """App. A: dt = min(0.5 / (kappa k_max^4), 1) with k_max = pi per voxel."""
    return min(0.5 / (kappa * math.pi ** 4), 1.0)


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    kappa: float
    dt: float

    def c(self) -> pm.McChGrid:
        return pm.McChGrid(self.nx, self.ny, self.nz, 0, self.kappa, self.dt)

    @property
    def spectrum_shape(self):
        return (self.nz, self.ny, self.nx // 2 + 1)

    @property
    def n_bins(self) -> int:
        return max(self.nx, self.ny, self.nz) // 2 + 1


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def workspace(grid: Grid, device) -> torch.Tensor:
    L = pm.load()
    g = grid.c()
    n = L.mc_ch_workspace_bytes(ctypes.byref(g))
    if n == 0:
        pm._check(-1, "mc_ch_workspace_bytes")
    return _ws(n, device)


def init(phi0: torch.Tensor, grid: Grid, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Spectrum of the real initial field phi0 (float64 [nz, ny, nx] on the GPU)."""
    L = pm.load()
    assert phi0.dtype == torch.float64 and phi0.is_contiguous() and tuple(phi0.shape) == (grid.nz, grid.ny, grid.nx)
    ws = workspace(grid, phi0.device) if ws is None else ws
    state = torch.empty(grid.spectrum_shape, dtype=torch.complex128, device=phi0.device)
    g = grid.c()
    pm._check(L.mc_ch_init(ctypes.byref(g), _ptr(phi0), _ptr(state), _ptr(ws), ws.numel(),
                           pm._stream(phi0.device)), "mc_ch_init")
    return state


def steps(state: torch.Tensor, grid: Grid, n: int, ws: torch.Tensor | None = None, timed: bool = False):
    """n steps of Eq. CH_spectral in place; with timed, returns the kernels' milliseconds."""
    L = pm.load()
    ws = workspace(grid, state.device) if ws is None else ws
    g = grid.c()
    pm._check(L.mc_ch_steps(ctypes.byref(g), int(n), _ptr(state), _ptr(ws), ws.numel(),
                            pm.MC_TIMED if timed else 0, pm._stream(state.device)), "mc_ch_steps")
    return L.mc_ch_elapsed_ms() if timed else None


def field(state: torch.Tensor, grid: Grid, ws: torch.Tensor | None = None) -> torch.Tensor:
    L = pm.load()
    ws = workspace(grid, state.device) if ws is None else ws
    phi = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float64, device=state.device)
    g = grid.c()
    pm._check(L.mc_ch_field(ctypes.byref(g), _ptr(state), _ptr(phi), _ptr(ws), ws.numel(),
                            pm._stream(state.device)), "mc_ch_field")
    return phi


def psd(state: torch.Tensor, grid: Grid, ws: torch.Tensor | None = None) -> torch.Tensor:
    L = pm.load()
    ws = workspace(grid, state.device) if ws is None else ws
    out = torch.empty(grid.n_bins, dtype=torch.float64, device=state.device)
    g = grid.c()
    pm._check(L.mc_ch_psd(ctypes.byref(g), _ptr(state), _ptr(out), _ptr(ws), ws.numel(),
                          pm._stream(state.device)), "mc_ch_psd")
    return out


def dominant_size(p: torch.Tensor, grid: Grid) -> float:
    """max(nx, ny, nz) / (2 s_peak): the size the stopping rule tests."""
    s = int(torch.argmax(p[1:]).item()) + 1
    return max(grid.nx, grid.ny, grid.nz) / (2.0 * s)


def rank_threshold(f: torch.Tensor, porosity: float | None = None, n_pore: int | None = None) -> torch.Tensor:
    """uint8 mask with the n_pore (= round(porosity N)) largest values of f set, ties to the lower index."""
    L = pm.load()
    assert f.dtype == torch.float64 and f.is_contiguous()
    n = f.numel()
    if n_pore is None:
        n_pore = int(round(porosity * n))
    ws = _ws(L.mc_rank_threshold_workspace_bytes(n), f.device)
    mask = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
    pm._check(L.mc_rank_threshold(_ptr(f), n, int(n_pore), _ptr(mask), _ptr(ws), ws.numel(),
                                  pm._stream(f.device)), "mc_rank_threshold")
    return mask


@dataclass
class Generated:
    mask: torch.Tensor | None
    field: torch.Tensor | None
    state: torch.Tensor
    steps: int
    size: float


def generate(phi0: torch.Tensor, grid: Grid, d_target: float, sigma: float, porosity: float,
             check_every: int = 200, max_steps: int = 50_000, want_field: bool = True,
             want_mask: bool = True) -> Generated:
    """App. A's loop (synchronous): evolve, check the dominant size every check_every steps,
    stop in the window or at max_steps, then field and rank binarisation."""
    L = pm.load()
    g = grid.c()
    ws = _ws(L.mc_ch_generate_workspace_bytes(ctypes.byref(g)), phi0.device)
    state = torch.empty(grid.spectrum_shape, dtype=torch.complex128, device=phi0.device)
    phi = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float64, device=phi0.device) if want_field else None
    mask = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.uint8, device=phi0.device) if want_mask else None
    n = ctypes.c_int32(0)
    size = ctypes.c_double(0.0)
    pm._check(L.mc_ch_generate(ctypes.byref(g), _ptr(phi0), float(d_target), float(sigma), int(check_every),
                               int(max_steps), float(porosity), _ptr(state),
                               _ptr(phi) if phi is not None else None, _ptr(mask) if mask is not None else None,
                               ctypes.byref(n), ctypes.byref(size), _ptr(ws), ws.numel(),
                               pm._stream(phi0.device)), "mc_ch_generate")
    return Generated(mask, phi, state, n.value, size.value)
