"""Python binding of the morphology and fluence analytics (include/analytics.h).

Argument marshalling only: torch allocates device memory, libphotonmc.so computes.
Axis numbering follows the C ABI: 0 = x, 1 = y, 2 = z (the beam axis).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import photonmc as pm


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def chord_histogram(mask: torch.Tensor, axis: int = 2) -> torch.Tensor:
    """int64 [2, n_axis + 1]: chords per phase (0 solid, 1 pore) and length."""
    L = pm.load()
    vol = pm.volume(mask)
    n = mask.shape[2 - axis]
    hist = torch.empty((2, n + 1), dtype=torch.int64, device=mask.device)
    pm._check(L.mc_chord_histogram(ctypes.byref(vol), int(axis), _ptr(hist), pm._stream(mask.device)),
              "mc_chord_histogram")
    return hist


def phase_contrast(depth: torch.Tensor, z0: int = 0) -> dict:
    """Depth-normalised solid and pore contrasts from mc_reduce's depth [3, nz]."""
    L = pm.load()
    d = depth.contiguous()
    out = torch.empty(5, dtype=torch.float64, device=d.device)
    pm._check(L.mc_phase_contrast(_ptr(d), int(d.shape[1]), int(z0), _ptr(out), pm._stream(d.device)),
              "mc_phase_contrast")
    v = out.cpu().tolist()
    return {"solid_mean": v[0], "solid_sd": v[1], "pore_mean": v[2], "pore_sd": v[3], "depths": int(v[4])}


def escape_paths(mask: torch.Tensor, optics: pm.Optics, n_photons: int, seed: int, bin_width: float, nbins: int,
                 thresholds=(), photon_begin: int = 0, stream_id: int = 0, fp64: bool = False) -> dict:
    """Sec. 3.5 (c): per-photon outcomes of photons [begin, begin + n) (mc_trace with no
    step records, on the device) binned by the in-pore path of the escaping ones."""
    L = pm.load()
    vol = pm.volume(mask)
    dev = mask.device
    ids = torch.arange(photon_begin, photon_begin + n_photons, dtype=torch.int64, device=dev)
    outc = torch.empty((n_photons, pm.PHOTON_DTYPE.itemsize), dtype=torch.uint8, device=dev)
    ws = pm.workspace(L.mc_run_workspace_bytes(ctypes.byref(vol)), dev)
    opt = optics.c()
    stream = pm._stream(dev)
    pm._check(L.mc_trace(ctypes.byref(vol), ctypes.byref(opt), ids.data_ptr(), n_photons, 0, seed, stream_id,
                         pm.MC_FP64 if fp64 else 0, None, outc.data_ptr(), ws.data_ptr(), ws.numel(), stream),
              "mc_trace")
    th = np.ascontiguousarray(np.asarray(thresholds, dtype=np.float64))
    nthr = int(th.size)
    hw = torch.empty(nbins, dtype=torch.int64, device=dev)
    hn = torch.empty(nbins, dtype=torch.int64, device=dev)
    aw = torch.empty(max(nthr, 1), dtype=torch.int64, device=dev)
    an = torch.empty(max(nthr, 1), dtype=torch.int64, device=dev)
    pm._check(L.mc_escape_path_histogram(outc.data_ptr(), n_photons, float(bin_width), int(nbins),
                                         th.ctypes.data if nthr else None, nthr, _ptr(hw), _ptr(hn),
                                         _ptr(aw) if nthr else None, _ptr(an) if nthr else None, stream),
              "mc_escape_path_histogram")
    return {"hist_w": hw, "hist_n": hn, "above_w": aw[:nthr], "above_n": an[:nthr], "outcomes": outc}


def bright_colocalization(mask: torch.Tensor, fluence: torch.Tensor, z0: int, frac: float = 0.1):
    """Per slice z >= z0: (k, solid voxels among the k brightest), int64 tensors."""
    L = pm.load()
    vol = pm.volume(mask)
    dev = mask.device
    nz = mask.shape[0]
    k = torch.empty(nz - z0, dtype=torch.int64, device=dev)
    s = torch.empty(nz - z0, dtype=torch.int64, device=dev)
    pm._check(L.mc_bright_colocalization(ctypes.byref(vol), _ptr(fluence.contiguous()), int(z0), float(frac),
                                         _ptr(k), _ptr(s), pm._stream(dev)),
              "mc_bright_colocalization")
    return k, s


def pore_distance(mask: torch.Tensor) -> torch.Tensor:
    """float64 [nz, ny, nx]: distance from each pore voxel to the nearest solid voxel."""
    L = pm.load()
    vol = pm.volume(mask)
    dev = mask.device
    out = torch.empty(tuple(mask.shape), dtype=torch.float64, device=dev)
    ws = pm.workspace(L.mc_pore_distance_workspace_bytes(ctypes.byref(vol)), dev)
    pm._check(L.mc_pore_distance(ctypes.byref(vol), _ptr(out), _ptr(ws), ws.numel(), pm._stream(dev)),
              "mc_pore_distance")
    return out


def pore_spearman(mask: torch.Tensor, fluence: torch.Tensor, z0: int):
    """Per slice z >= z0: (Spearman rho of fluence vs pore size over the pore voxels
    as float64, pore voxel count as int64)."""
    L = pm.load()
    vol = pm.volume(mask)
    dev = mask.device
    nz = mask.shape[0]
    rho = torch.empty(nz - z0, dtype=torch.float64, device=dev)
    n = torch.empty(nz - z0, dtype=torch.int64, device=dev)
    need = L.mc_pore_spearman_workspace_bytes(ctypes.byref(vol), int(z0))
    if need == 0:
        raise ValueError(f"mc_pore_spearman: no workspace size for z0={z0} and mask {tuple(mask.shape)}")
    ws = pm.workspace(need, dev)
    pm._check(L.mc_pore_spearman(ctypes.byref(vol), _ptr(fluence.contiguous()), int(z0), _ptr(rho), _ptr(n),
                                 _ptr(ws), ws.numel(), pm._stream(dev)), "mc_pore_spearman")
    return rho, n


def mask_psd(mask: torch.Tensor) -> torch.Tensor:
    """float64 [max(nx,ny,nz)/2 + 1]: radial power spectral density of the binary mask
    (shell sums of |m_hat|^2, the mean excluded); dominant size = N_max / (2 s_peak)."""
    L = pm.load()
    vol = pm.volume(mask)
    dev = mask.device
    nb = max(mask.shape) // 2 + 1
    out = torch.empty(nb, dtype=torch.float64, device=dev)
    need = L.mc_mask_psd_workspace_bytes(ctypes.byref(vol))
    if need == 0:
        raise ValueError(f"mc_mask_psd: unsupported grid {tuple(mask.shape)}: {L.mc_last_error().decode()}")
    ws = pm.workspace(need, dev)
    pm._check(L.mc_mask_psd(ctypes.byref(vol), _ptr(out), _ptr(ws), ws.numel(), pm._stream(dev)), "mc_mask_psd")
    return out
