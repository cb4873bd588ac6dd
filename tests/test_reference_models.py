"""The library's host-side reference model and constants (no GPU needed), each
against something other than itself:

* mc_da_profile (Sec. 2.4) against the numerical quadrature of the printed
  closed form (tests/closed_forms.py), and against the paper's worked values
  (L_opt = 521 / 852 um, <Phi>_DA = 7.73e19 / 1.266e20 photon m^-2 s^-1) from
  tests/golden/diffusion_approximation.txt;
* mc_ch_grid_from_target (Eq. kappa_cal, App. A) against the printed
  kappa_CH = 0.1140 and dt = 0.0450, and against the Cahn-Hilliard oracle;
* argument checking of these calls and of mc_time_gate (its values are pinned in
  tests/test_time_gate.py).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import pytest

import closed_forms as cf
from oracle import cahn_hilliard as och
from paper_2604_13929_amd import photonmc as pm
from paper_2604_13929_amd import spinodal as sp
from conftest import golden

A_VOX = 1.45e-6


@pytest.mark.parametrize("mu_s,mu_a,g,phi,nz", [
    (0.5, 0.01, 0.7, 0.9, 256),       # the spinodal phi = 0.90 slab's effective medium
    (0.05, 0.001, 0.7, 0.0, 256),     # the matched homogeneous slab (same effective medium)
    (0.5, 0.01, 0.7, 0.7, 64),
    (2.0, 0.2, 0.0, 0.0, 40),         # thick: kappa L ~ 24
    (0.3, 0.02, 0.5, 0.5, 1),         # a single layer
])
def test_da_profile_is_the_voxel_mean_of_the_closed_form(mu_s, mu_a, g, phi, nz):
    prof, l_opt = pm.da_profile(mu_s, mu_a, g, phi, nz)
    mua, musr = (1 - phi) * mu_a, (1 - phi) * mu_s * (1 - g)
    want = cf.da_voxel_profile(nz, mua, musr)
    assert np.allclose(prof, want, rtol=1e-9, atol=0.0)
    assert l_opt == pytest.approx(cf.da_lopt(mua, musr, float(nz)), rel=1e-9)
    assert l_opt == pytest.approx(prof.sum(), rel=1e-14)


def test_da_profile_reproduces_the_papers_worked_values():
    """The paper's slab: 384 voxels of 1.45 um (Table 1), the effective coefficients it
    prints (Table 1 / Table S2) per voxel; L_opt in voxels times the voxel size, and
    <Phi>_DA = S0 L_opt / L."""
    for _, mua, musr, L, S0, lopt, phi_da, _, _, _ in golden("diffusion_approximation.txt"):
        nz = int(round(L / A_VOX))
        assert nz == 384
        _, l_vox = pm.da_profile(musr * A_VOX, mua * A_VOX, 0.0, 0.0, nz)
        assert l_vox * A_VOX == pytest.approx(lopt, rel=1e-3)
        assert S0 * l_vox / nz == pytest.approx(phi_da, rel=1e-3)


def test_da_profile_uses_the_effective_medium_scaling():
    """Eq. EMA_scaling: (mu_s, mu_a) at porosity phi equal (1 - phi)(mu_s, mu_a) at 0, and
    g enters only through mu_s (1 - g)."""
    a, la = pm.da_profile(0.5, 0.01, 0.7, 0.9, 128)
    b, lb = pm.da_profile(0.05, 0.001, 0.7, 0.0, 128)
    c, lc = pm.da_profile(0.015, 0.001, 0.0, 0.0, 128)
    assert np.allclose(a, b, rtol=1e-12) and np.allclose(b, c, rtol=1e-12) and la == pytest.approx(lc, rel=1e-12)


@pytest.mark.parametrize("args,needle", [
    ((0.5, 0.01, 0.7, 0.7, 0), b"nz"), ((0.5, 0.01, 1.0, 0.7, 8), b"|g|"), ((0.5, 0.01, 0.7, 1.0, 8), b"porosity"),
    ((0.5, 0.0, 0.7, 0.7, 8), b"effective"), ((0.0, 0.01, 0.7, 0.7, 8), b"effective"),
    ((0.02, 0.01, 0.0, 0.0, 8), b"degenerate"), ((5.0, 1.0, 0.0, 0.0, 200), b"overflows"),
])
def test_da_profile_rejects_bad_arguments(args, needle):
    L = pm.load()
    out = np.zeros(max(args[4], 1))
    l_opt = ctypes.c_double(0.0)
    rc = L.mc_da_profile(*args[:4], args[4], out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(l_opt))
    assert rc == -1 and needle in L.mc_last_error()


def test_grid_from_target_reproduces_app_a():
    for d_um, a_um, kappa, dt in golden("cahn_hilliard_calibration.txt"):
        g = sp.grid_from_target(384, 1024, 1024, d_um / a_um)
        assert round(g.kappa, 4) == kappa and round(g.dt, 4) == dt
        assert (g.nx, g.ny, g.nz) == (384, 1024, 1024)
    for d in (2.0, 3.0, 12.0, 17.4 / 1.45, 40.0, 200.0):
        g = sp.grid_from_target(8, 8, 8, d)
        assert g.kappa == pytest.approx(och.kappa_from_target(d), rel=1e-15)
        assert g.dt == pytest.approx(och.dt_from_kappa(och.kappa_from_target(d)), rel=1e-15)
    # small targets: the explicit bound exceeds 1 and dt is capped
    assert sp.grid_from_target(8, 8, 8, 2.0).dt == 1.0 and sp.grid_from_target(8, 8, 8, 2.6).dt < 1.0


def test_grid_from_target_and_gate_reject_bad_arguments():
    L = pm.load()
    g = pm.McChGrid(8, 8, 8, 0, 0.0, 0.0)
    for d in (0.0, -1.0, float("nan"), float("inf")):
        assert L.mc_ch_grid_from_target(d, ctypes.byref(g)) == -1
    assert L.mc_ch_grid_from_target(12.0, None) == -1
    t = ctypes.c_double(0.0)
    good = (0.5, 0.01, 0.7, 0.7, 64.0, 1.5, 1.0)
    assert L.mc_time_gate(*good, ctypes.byref(t)) == 0 and math.isfinite(t.value)
    for i, bad in ((0, -1.0), (1, float("nan")), (2, 1.0), (3, 1.5), (4, 0.0), (5, 0.9), (6, 0.0)):
        args = list(good)
        args[i] = bad
        assert L.mc_time_gate(*args, ctypes.byref(t)) == -1, (i, bad)
    assert L.mc_time_gate(*good, None) == -1
