"""Python binding of the Cahn-Hilliard spinodal mask generator (include/spinodal.h).

Argument marshalling only: torch allocates device memory, libphotonmc.so computes.
The spectrum is a complex128 tensor [nz, ny, nx//2 + 1] (numpy.fft.rfftn layout).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import photonmc as pm


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


def grid_from_target(nx: int, ny: int, nz: int, d_target_voxels: float) -> Grid:
    """A grid whose kappa_CH (Eq. kappa_cal) and dt (App. A) come from
    mc_ch_grid_from_target for a target dominant size in voxels."""
    g = pm.McChGrid(nx, ny, nz, 0, 0.0, 0.0)
    pm._check(pm.load().mc_ch_grid_from_target(float(d_target_voxels), ctypes.byref(g)), "mc_ch_grid_from_target")
    return Grid(nx, ny, nz, g.kappa, g.dt)


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


def psd_peak(p: torch.Tensor, n_max: int):
    """mc_psd_peak: (peak shell, dominant size in voxels) of a radial PSD on the GPU."""
    L = pm.load()
    if not p.is_cuda:
        raise ValueError("psd must be a device tensor")
    q = p.to(torch.float64).contiguous()
    shell = torch.empty(1, dtype=torch.int32, device=q.device)
    size = torch.empty(1, dtype=torch.float64, device=q.device)
    pm._check(L.mc_psd_peak(_ptr(q), int(q.numel()), int(n_max), _ptr(shell), _ptr(size), pm._stream(q.device)),
              "mc_psd_peak")
    return int(shell.item()), float(size.item())


def dominant_size(p: torch.Tensor, grid: Grid) -> float:
    """The size App. A's stopping rule tests (mc_psd_peak)."""
    return psd_peak(p, max(grid.nx, grid.ny, grid.nz))[1]


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
