"""The time gate of Eq. tend (mc_time_gate in the library) against the paper's
printed values: t_end = 2.46e-10 s at phi = 0.70 and 8.21e-11 s at phi = 0.90
(Sec. 2.5, "Photon budget, time gate and statistics"), from the shell values of
Table 2 (mu_a = 5159 1/m, mu_s' = 20118 1/m, n_eff = 1.746) and the slab of
Table 1 (384 voxels of 1.45 um).  The printed values carry three digits."""
from __future__ import annotations

import math

from paper_2604_13929_amd import photonmc as pm
from conftest import golden

A_VOX = 1.45e-6
L = 384 * A_VOX


def test_gate_reproduces_the_papers_values():
    for phi, mua, musr, n_eff, nvox, a_vox, printed in golden("time_gate.txt"):
        t = pm.time_gate_seconds(mua, musr, phi, nvox * a_vox, n_eff)
        assert math.isclose(t, printed, rel_tol=2e-3), (phi, t, printed)


def test_gate_in_voxels_is_c_t_end():
    for phi in (0.7, 0.9):
        mu_a, mu_s = 5159.0 * A_VOX, 20118.0 * A_VOX        # per voxel; g = 0 so mu_s' = mu_s
        g_vox = pm.time_gate_voxels(mu_s, mu_a, 0.0, phi, 384, 1.746)
        t = pm.time_gate_seconds(5159.0, 20118.0, phi, L, 1.746)
        assert math.isclose(g_vox * A_VOX / pm.SPEED_OF_LIGHT, t, rel_tol=1e-12)
    # the absorption floor wins for a thin, weakly scattering slab
    g_vox = pm.time_gate_voxels(0.0, 0.01, 0.0, 0.5, 4, 1.5)
    assert math.isclose(g_vox, 5 * 1.5 / 0.01, rel_tol=1e-12)
    # without absorption Eq. tend has no finite gate
    assert math.isinf(pm.time_gate_voxels(0.5, 0.0, 0.7, 0.5, 4, 1.5))
    # a thick scattering slab: the diffusive term wins
    g_vox = pm.time_gate_voxels(0.5, 0.01, 0.7, 0.5, 64, 1.5)
    assert math.isclose(g_vox, 18 * 1.5 * 64 ** 2 * 0.5 * (0.01 + 0.5 * 0.3), rel_tol=1e-12)
