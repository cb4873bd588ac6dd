"""Pins of the Cahn-Hilliard oracle (oracle/cahn_hilliard.py) against facts other
than itself:

* the paper's worked values: kappa_CH = 0.1140 for d_target = 17.4 um at 1.45 um
  voxels (Eq. kappa_cal), dt = 0.0450 (App. A), the spinodal interval
  (0.211, 0.789) and |f''(0.5)| = 1 (Sec. 2.2);
* exact conservation of the mean (the k = 0 mode of Eq. CH_spectral is untouched);
* the discrete linear growth factor of a single small Fourier mode around the
  spinodal centre, (1 + dt k^2) / (1 + dt kappa k^4) per step, on each axis and a
  diagonal (a swapped axis, a dropped k^2, 2 kappa for kappa or a sign fails it);
* the phi -> 1 - phi symmetry of the double well;
* the equilibrium interface phi = (1 + tanh(x / sqrt(2 kappa))) / 2 is stationary;
* the first decomposition selects the fastest-growing wavenumber of Eq. CH,
  k* = 1 / sqrt(2 kappa) (Eq. lambda_star), not the 2-kappa form of Eq. sigma_k;
* the radial PSD: Parseval and the peak shell of single-mode fields (shells by the
  nearest integer of |k| N_max / 2 pi);
* the rank threshold: exact count, order and index tie-break;
* the stopping rule of App. A.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import cahn_hilliard as ch
from conftest import golden


def test_paper_worked_values():
    for d_target, a_vox, kappa_printed, dt_printed in golden("cahn_hilliard_calibration.txt"):
        kappa = ch.kappa_from_target(d_target / a_vox)
        assert round(kappa, 4) == kappa_printed
        assert round(ch.dt_from_kappa(kappa), 4) == dt_printed
    roots = np.sort(np.roots([12.0, -12.0, 2.0]))
    assert np.allclose(np.round(roots, 3), [0.211, 0.789])
    assert ch.f_second(0.5) == -1.0
    assert ch.f_second(0.2) > 0 > ch.f_second(0.3)
    # f' is the derivative of f = phi^2 (1 - phi)^2
    x = np.linspace(-0.5, 1.5, 41)
    h = 1e-6
    f = lambda p: p * p * (1 - p) ** 2  # noqa: E731
    assert np.allclose(ch.f_prime(x), (f(x + h) - f(x - h)) / (2 * h), atol=1e-8)
    assert np.allclose(ch.f_second(x), (ch.f_prime(x + h) - ch.f_prime(x - h)) / (2 * h), atol=1e-7)


def test_mean_is_conserved_exactly():
    rng = np.random.default_rng(1)
    phi0 = np.clip(0.5 + 0.05 * rng.standard_normal((10, 12, 16)), 0, 1)
    ph0 = ch.spectrum(phi0)
    ph = ch.steps(ph0, phi0.shape, 50, 0.045, 0.114)
    assert ph[0, 0, 0] == ph0[0, 0, 0]
    assert abs(ch.field(ph, phi0.shape).mean() - phi0.mean()) < 1e-15


@pytest.mark.parametrize("mode", [(0, 0, 3), (0, 5, 0), (4, 0, 0), (2, 3, 1)])
def test_linear_growth_factor_of_one_mode(mode):
    shape = (16, 24, 32)
    nz, ny, nx = shape
    mz, my, mx = mode
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    eps, dt, kappa, n = 1e-6, 0.07, 0.6, 25
    theta = 2 * math.pi * (mx * x / nx + my * y / ny + mz * z / nz)
    phi0 = 0.5 + eps * np.cos(theta)
    ph = ch.steps(ch.spectrum(phi0), shape, n, dt, kappa)
    k2 = (2 * math.pi) ** 2 * ((mx / nx) ** 2 + (my / ny) ** 2 + (mz / nz) ** 2)
    g = (1 + dt * k2) / (1 + dt * kappa * k2 * k2)
    amp = ch.field(ph, shape) - 0.5
    want = eps * g ** n * np.cos(theta)
    assert np.abs(amp - want).max() < 1e-6 * eps * g ** n


def test_phi_to_one_minus_phi_symmetry():
    rng = np.random.default_rng(2)
    phi0 = np.clip(0.5 + 0.05 * rng.standard_normal((12, 12, 12)), 0, 1)
    shape = phi0.shape
    a = ch.field(ch.steps(ch.spectrum(phi0), shape, 300, 0.045, 0.114), shape)
    b = ch.field(ch.steps(ch.spectrum(1.0 - phi0), shape, 300, 0.045, 0.114), shape)
    assert np.abs(a + b - 1.0).max() < 1e-10
    assert np.abs(a - 0.5).max() > 0.3       # the field did decompose


def test_equilibrium_interface_is_stationary():
    kappa, nx = 2.0, 128
    x = np.arange(nx, dtype=np.float64)
    w = math.sqrt(2 * kappa)
    prof = 0.5 * (1 + np.tanh((x - 32) / w)) - 0.5 * (1 + np.tanh((x - 96) / w))
    phi0 = prof.reshape(1, 1, nx)
    ph = ch.steps(ch.spectrum(phi0), phi0.shape, 2000, 0.1, kappa)
    assert np.abs(ch.field(ph, phi0.shape) - phi0).max() < 2e-3
    # the same profile with the width of a 2 kappa gradient term relaxes visibly
    w2 = math.sqrt(4 * kappa)
    prof2 = 0.5 * (1 + np.tanh((x - 32) / w2)) - 0.5 * (1 + np.tanh((x - 96) / w2))
    ph2 = ch.steps(ch.spectrum(prof2.reshape(1, 1, nx)), phi0.shape, 2000, 0.1, kappa)
    assert np.abs(ch.field(ph2, phi0.shape) - prof2.reshape(1, 1, nx)).max() > 2e-2


def test_first_decomposition_picks_the_fastest_growing_mode():
    """sigma(k) = k^2 (1 - kappa k^2) for Eq. CH at phi = 0.5: peak at k* = 1/sqrt(2 kappa),
    a dominant size pi / k* = pi sqrt(2 kappa) (half of Eq. lambda_star's wavelength)."""
    kappa, n = 1.0, 64
    rng = np.random.default_rng(3)
    phi0 = 0.5 + 1e-4 * rng.standard_normal((n, n, n))
    ph = ch.steps(ch.spectrum(phi0), phi0.shape, 80, 0.05, kappa)      # t = 4, still linear
    psd = ch.radial_psd(ph, phi0.shape)
    s = int(np.argmax(psd[1:])) + 1
    k_star = 1 / math.sqrt(2 * kappa)
    assert abs(2 * math.pi * s / n - k_star) <= 2 * math.pi / n
    assert abs(2 * math.pi * s / n - 1 / math.sqrt(4 * kappa)) > 2 * math.pi / n


def test_radial_psd_parseval_and_peak():
    shape = (20, 24, 32)
    nz, ny, nx = shape
    rng = np.random.default_rng(4)
    # a band-limited field (all shells below N_max / 2)
    phi = np.zeros(shape)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for _ in range(6):
        m = rng.integers(-4, 5, 3)
        phi += rng.standard_normal() * np.cos(2 * math.pi * (m[0] * z / nz + m[1] * y / ny + m[2] * x / nx) + rng.random())
    ph = ch.spectrum(phi)
    psd = ch.radial_psd(ph, shape)
    total = phi.size * np.sum((phi - phi.mean()) ** 2)
    assert math.isclose(psd.sum(), total, rel_tol=1e-12)
    # a single mode lands in its shell
    # (0, 3, 4): |k| N_max / 2 pi = sqrt(4^2 + 4^2) = 5.66, in shell 6 (nearest, not floor)
    for m, s in (((0, 0, 5), 5), ((0, 6, 0), 8), ((2, 0, 0), 3), ((0, 3, 4), 6)):
        f = np.cos(2 * math.pi * (m[0] * z / nz + m[1] * y / ny + m[2] * x / nx))
        p = ch.radial_psd(ch.spectrum(f), shape)
        assert int(np.argmax(p)) == s, (m, np.argmax(p), s)
        assert ch.dominant_size(p, shape) == 32 / (2 * s)


def test_rank_threshold_definition():
    rng = np.random.default_rng(5)
    phi = np.round(rng.random((7, 9, 11)), 1)      # many ties
    for por in (0.0, 0.3, 0.5, 0.713, 1.0):
        m = ch.rank_threshold(phi, por).ravel()
        flat = phi.ravel()
        assert m.sum() == round(por * flat.size)
        if 0 < m.sum() < flat.size:
            lo, hi = flat[m == 1].min(), flat[m == 0].max()
            assert lo >= hi
            if lo == hi:   # the tied value: pores take the lower indices
                tied = np.flatnonzero(flat == lo)
                assert np.all(np.diff(m[tied].astype(int)) <= 0)


def test_stopping_rule():
    rng = np.random.default_rng(6)
    phi0 = np.clip(0.5 + 0.05 * rng.standard_normal((32, 32, 32)), 0, 1)
    kappa = 0.3
    mask, phi, n, sizes = ch.generate(phi0, d_target=4.0, sigma=1.0, porosity=0.7, check_every=40,
                                      max_steps=4000, dt=0.05, kappa=kappa)
    assert 3.5 <= sizes[-1] <= 4.5 and all(not (3.5 <= s <= 4.5) for s in sizes[:-1])
    assert n == 40 * len(sizes) and mask.sum() == round(0.7 * mask.size)
    # the hard cap
    _, _, n2, sizes2 = ch.generate(phi0, d_target=40.0, sigma=1.0, porosity=0.7, check_every=40,
                                   max_steps=120, dt=0.05, kappa=kappa)
    assert n2 == 120 and len(sizes2) == 3
