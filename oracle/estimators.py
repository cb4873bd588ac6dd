"""FP64 reduction of an oracle fluence map to the paper's estimators.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain numpy, written
from the definitions:

* normalisation, Sec. 2.5 (Fluence normalisation, Eq. Phi_norm): a launched
  photon carries weight 2^31, N photons are spread over the Nx*Ny source face,
  so Phi/S0 of a voxel of unit volume is  F * Nx*Ny / (N * 2^31);
* solid-weighted average, Sec. 2.6, Eq. Phi_MC3D: sum(Phi s) / sum(s), s = 1 - m;
* volume average, Eq. Phi_MC1D, with the depth integral read as the voxel sum
  over z and L = Nz;
* pore average and the phase-contrast ratio r, Eq. r_def;
* the identity of Eq. dilution, evaluated with the achieved porosity;
* phase-resolved depth profiles as in App. B (Post-processing) and Fig. 4b;
* front/back ratio Phi(0)/Phi(L) as in Table S2, and L_opt = <Phi>_1D L / S0 as
  in the caption of Table 4;
* the fluence-weighted relative RMS deviation of Sec. 2.7, Eq. RMSw, and the
  unweighted and log-ratio variants reported beside it in Table S1 (App. B).
"""
from __future__ import annotations

import numpy as np

W1 = float(2 ** 31)


def normalise(F: np.ndarray, n_photons: int) -> np.ndarray:
    """Phi/S0 per voxel from a track-length tally F[nz][ny][nx] (weight units 2^-31)."""
    nz, ny, nx = F.shape
    return np.asarray(F, dtype=np.float64) * (nx * ny) / (float(n_photons) * W1)


def estimators(F: np.ndarray, mask: np.ndarray, n_photons: int) -> dict:
    """All reduced quantities of one run; F and mask are [nz][ny][nx]."""
    phi = normalise(F, n_photons)
    m = np.asarray(mask, dtype=np.float64)
    s = 1.0 - m
    nz, ny, nx = F.shape
    n_vox = nz * ny * nx
    out = {}
    out["porosity"] = m.sum() / n_vox
    out["phi3d"] = (phi * s).sum() / s.sum() if s.sum() > 0 else float("nan")
    out["phi1d"] = phi.sum() / (nx * ny * nz)
    out["phi_pore"] = (phi * m).sum() / m.sum() if m.sum() > 0 else float("nan")
    out["r"] = out["phi_pore"] / out["phi3d"]
    por = out["porosity"]
    # with no pore voxel the pore term of the identity is absent
    out["identity_rhs"] = 1.0 / (por * out["r"] + (1.0 - por)) if m.sum() > 0 else 1.0
    out["ratio"] = out["phi3d"] / out["phi1d"]
    depth = phi.sum(axis=(1, 2)) / (nx * ny)
    n_s = s.sum(axis=(1, 2))
    n_m = m.sum(axis=(1, 2))
    with np.errstate(invalid="ignore", divide="ignore"):
        out["depth_solid"] = np.where(n_s > 0, (phi * s).sum(axis=(1, 2)) / n_s, np.nan)
        out["depth_pore"] = np.where(n_m > 0, (phi * m).sum(axis=(1, 2)) / n_m, np.nan)
    out["depth"] = depth
    out["front_back"] = depth[0] / depth[-1] if depth[-1] != 0 else float("inf")
    out["L_opt"] = out["phi1d"] * nz
    return out


def _rms_depths(profile, reference):
    """The depths a relative deviation is defined at: reference finite and positive,
    profile finite (reading of the sums over z in Eq. RMSw)."""
    p = np.asarray(profile, dtype=np.float64)
    q = np.asarray(reference, dtype=np.float64)
    ok = np.isfinite(q) & (q > 0) & np.isfinite(p)
    return p[ok], q[ok]


def rms_w(profile: np.ndarray, reference: np.ndarray) -> float:
    """Eq. RMSw with the reference profile as weights and denominator."""
    p, q = _rms_depths(profile, reference)
    return float(np.sqrt((q * (p - q) ** 2 / q ** 2).sum() / q.sum()))


def rms_unweighted(profile: np.ndarray, reference: np.ndarray) -> float:
    """Table S1's unweighted variant: the weights of Eq. RMSw set to one."""
    p, q = _rms_depths(profile, reference)
    return float(np.sqrt((((p - q) / q) ** 2).mean()))


def rms_log(profile: np.ndarray, reference: np.ndarray) -> float:
    """Table S1's log variant: the RMS of ln(Phi_MC / Phi_DA), over the depths where
    the profile is positive too."""
    p, q = _rms_depths(profile, reference)
    ok = p > 0
    return float(np.sqrt((np.log(p[ok] / q[ok]) ** 2).mean()))
