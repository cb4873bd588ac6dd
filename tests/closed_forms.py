"""Closed forms used to pin the oracle (test tooling, FP64).

* Collimated-source diffusion approximation, Sec. 2.4: ballistic plus diffuse
  term (Eq. DA_total), particular solution A e^{-mu_t z} of Eq. DA_diff_eq,
  extrapolated boundaries Phi_diff(-z_b) = Phi_diff(L + z_b) = 0 with the
  constants of Eq. Cpm, the complete diffuse solution Eq. Phi_diff, and
  L_opt, <Phi>_DA of Eq. Lopt_DA.  Parameters as in Table 1 / Table 2:
  D = 1/[3(mu_a + mu_s')], kappa = sqrt(mu_a / D), z_b = (2/3) / mu_s',
  mu_t = mu_a + mu_s'.
* Beer-Lambert in a purely absorbing voxel column (no scattering): a photon
  launched into a column survives each solid voxel with probability e^{-mu_a}.
* Henyey-Greenstein moments and CDF.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def da_params(mu_a: float, mu_s_red: float) -> dict:
    D = 1.0 / (3.0 * (mu_a + mu_s_red))
    kappa = math.sqrt(mu_a / D)
    return dict(D=D, kappa=kappa, z_b=(2.0 / 3.0) / mu_s_red, mu_t=mu_a + mu_s_red,
                ell_star=1.0 / mu_s_red)


def da_profile(z, mu_a: float, mu_s_red: float, L: float, S0: float = 1.0):
    """Phi_DA(z) for a collimated planar source on a slab of thickness L."""
    p = da_params(mu_a, mu_s_red)
    D, kappa, z_b, mu_t = p["D"], p["kappa"], p["z_b"], p["mu_t"]
    A = mu_s_red * S0 / (D * (kappa ** 2 - mu_t ** 2))
    L_e = L + 2.0 * z_b
    sh = math.sinh(kappa * L_e)
    c_plus = -A * math.exp(-mu_t * (L + z_b)) / sh
    c_minus = -A * math.exp(mu_t * z_b) / sh
    z = np.asarray(z, dtype=np.float64)
    diff = A * np.exp(-mu_t * z) + c_plus * np.sinh(kappa * (z + z_b)) + c_minus * np.sinh(kappa * (L + z_b - z))
    return S0 * np.exp(-mu_t * z) + diff


def da_lopt(mu_a: float, mu_s_red: float, L: float) -> float:
    """L_opt = (1/S0) int_0^L Phi_DA dz (numerical quadrature of the closed form)."""
    val, _ = integrate.quad(lambda z: float(da_profile(z, mu_a, mu_s_red, L, 1.0)), 0.0, L,
                            epsabs=0.0, epsrel=1e-12, limit=200)
    return val


def da_mean(mu_a: float, mu_s_red: float, L: float, S0: float) -> float:
    return S0 * da_lopt(mu_a, mu_s_red, L) / L


def da_voxel_profile(nz: int, mu_a: float, mu_s_red: float) -> np.ndarray:
    """Voxel averages of Phi_DA/S0 over [z, z+1) for a slab of nz voxels."""
    out = np.empty(nz)
    for z in range(nz):
        out[z], _ = integrate.quad(lambda t: float(da_profile(t, mu_a, mu_s_red, float(nz), 1.0)), z, z + 1.0)
    return out


def beer_lambert_voxel(mask: np.ndarray, mu_a: float) -> np.ndarray:
    """Expected Phi/S0 per voxel for a purely absorbing solid, collimated along +z.

    A photon reaching voxel v has crossed s solid voxels above it with survival
    e^{-mu_a s}; inside a solid voxel the expected track is (1 - e^{-mu_a})/mu_a,
    inside a pore it is 1.
    """
    solid = (np.asarray(mask) == 0).astype(np.float64)
    above = np.cumsum(solid, axis=0) - solid          # solid voxels strictly above, per column
    inside = (1.0 - math.exp(-mu_a)) / mu_a
    return np.exp(-mu_a * above) * np.where(solid > 0, inside, 1.0)


def beer_lambert_voxel_dmua(mask: np.ndarray, mu_a: float) -> np.ndarray:
    """d/d mu_a of beer_lambert_voxel."""
    solid = (np.asarray(mask) == 0).astype(np.float64)
    above = np.cumsum(solid, axis=0) - solid
    e = np.exp(-mu_a * above)
    inside = (1.0 - math.exp(-mu_a)) / mu_a
    d_inside = (mu_a * math.exp(-mu_a) - (1.0 - math.exp(-mu_a))) / mu_a ** 2
    return np.where(solid > 0, -above * e * inside + e * d_inside, -above * e)


def beer_lambert_T(mask: np.ndarray, mu_a: float) -> float:
    """Expected transmittance: mean over columns of e^{-mu_a s_col}."""
    s_col = (np.asarray(mask) == 0).sum(axis=0).astype(np.float64)
    return float(np.exp(-mu_a * s_col).mean())


def hg_cdf(mu, g: float):
    """CDF of the Henyey-Greenstein phase function in mu = cos(theta)."""
    mu = np.asarray(mu, dtype=np.float64)
    if g == 0.0:
        return 0.5 * (mu + 1.0)
    return (1.0 - g * g) / (2.0 * g) * (1.0 / np.sqrt(1.0 + g * g - 2.0 * g * mu) - 1.0 / (1.0 + g))


def hg_moments(g: float):
    """E[mu] = g and E[mu^2] = (1 + 2 g^2)/3 for Henyey-Greenstein."""
    return g, (1.0 + 2.0 * g * g) / 3.0
