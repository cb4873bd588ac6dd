"""Pins of the analytics oracle (oracle/analytics.py) against facts other than
itself: hand-counted chords and an independent run-length count, conservation of
phase volume, the mean-chord ratio phi/(1 - phi) on lines with as many pore as
solid chords, the exact per-depth decomposition phi(z) c_pore + (1 - phi(z)) c_solid
= 1, the escape histograms against the walk's own escape channels, brute-force
brightest deciles, the distance transform against brute force, and the per-slice
Spearman correlation against rank counting, the no-ties closed form
1 - 6 sum d^2 / (n (n^2 - 1)) and its +-1 limits."""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import analytics as an
from oracle import estimators as est
from paper_2604_13929_amd import inputs

W1 = 2 ** 31
f32 = lambda x: float(np.float32(x))  # noqa: E731


def runs_by_diff(line):
    """Independent run-length count: change points of the sequence."""
    line = np.asarray(line)
    edges = np.flatnonzero(np.diff(line)) + 1
    starts = np.r_[0, edges]
    ends = np.r_[edges, line.size]
    return [(int(line[s]), int(e - s)) for s, e in zip(starts, ends)]


def test_chords_hand_counted():
    line = np.array([1, 1, 0, 1, 1, 1, 0, 0, 1, 1], dtype=np.uint8)
    m = line.reshape(10, 1, 1)
    h = an.chord_histogram(m, axis=0)
    assert h[1, 2] == 2 and h[1, 3] == 1 and h[0, 1] == 1 and h[0, 2] == 1 and h.sum() == 5
    st = an.chord_stats(h, thresholds=(2,))
    assert st["mean_pore"] == 7 / 3 and st["mean_solid"] == 1.5
    assert st["plen_pore_gt_2"] == 3 / 7


def test_chords_against_run_lengths_and_volume():
    m = inputs.spinodal_mask(12, 10, 14, 5.0, 0.6, seed=2)
    for axis in (0, 1, 2):
        h = an.chord_histogram(m, axis=axis)
        ref = np.zeros_like(h)
        lines = np.moveaxis(m, axis, -1).reshape(-1, m.shape[axis])
        for line in lines:
            for ph, ln in runs_by_diff(line):
                ref[ph, ln] += 1
        assert np.array_equal(h, ref)
        lengths = np.arange(h.shape[1])
        assert (lengths * h[1]).sum() == m.sum() and (lengths * h[0]).sum() == (m == 0).sum()


def test_mean_chord_ratio_on_balanced_lines():
    """Lines that start with one phase and end with the other hold as many chords of
    each phase, so mean pore / mean solid chord = pore / solid voxels."""
    rng = np.random.default_rng(3)
    lines = []
    while len(lines) < 200:
        line = (rng.random(40) < 0.7).astype(np.uint8)
        if line[0] != line[-1]:
            lines.append(line)
    m = np.array(lines).T.reshape(40, 200, 1)
    st = an.chord_stats(an.chord_histogram(m, axis=0))
    phi = m.mean()
    assert math.isclose(st["mean_pore"] / st["mean_solid"], phi / (1 - phi), rel_tol=1e-12)


def test_phase_contrast_decomposition(mask_m1):
    n = 20_000
    ref = oracle.run(mask_m1, 0.5, f32(0.01), f32(0.7), n, 31)
    e = est.estimators(ref["fluence"][0], mask_m1, n)
    pc = an.phase_contrast(e["depth"], e["depth_solid"], e["depth_pore"])
    phi_z = mask_m1.mean(axis=(1, 2))
    cs = e["depth_solid"] / e["depth"]
    cp = e["depth_pore"] / e["depth"]
    assert np.allclose(phi_z * cp + (1 - phi_z) * cs, 1.0, rtol=1e-12)
    assert math.isclose(pc["solid_mean"], cs.mean(), rel_tol=1e-12) and pc["depths"] == mask_m1.shape[0]
    h = inputs.homogeneous_mask(4, 4, 8)
    r = oracle.run(h, 0.5, f32(0.01), f32(0.7), 2000, 31)
    e2 = est.estimators(r["fluence"][0], h, 2000)
    pc2 = an.phase_contrast(e2["depth"], e2["depth_solid"], e2["depth_pore"])
    assert math.isclose(pc2["solid_mean"], 1.0, rel_tol=1e-12) and pc2["solid_sd"] < 1e-12


def test_escape_histogram_matches_walk_channels(mask_m1):
    ids = np.arange(3000, dtype=np.uint64)
    _, summ = oracle.trace(mask_m1, 0.5, f32(0.01), f32(0.7), ids, 41, max_rec=0)
    run = oracle.run(mask_m1, 0.5, f32(0.01), f32(0.7), 3000, 41, fluence=False)
    tot = oracle.totals(run)
    nz = mask_m1.shape[0]
    hw, hn, aw, an_ = an.escape_path_histogram(summ["fate"], summ["w_final"], summ["path_void"], 2.0, 40,
                                               thresholds=(float(nz), 10.0))
    assert hw.sum() == tot["esc_w"] and hn.sum() == tot["esc_n"]
    assert aw[0] == tot["esc_w_gtL"] and an_[0] == tot["esc_n_gtL"]
    assert aw[1] >= aw[0]


def test_bright_colocalization_brute_force():
    rng = np.random.default_rng(4)
    F = rng.integers(0, 5, size=(6, 5, 7))           # many ties
    m = (rng.random((6, 5, 7)) < 0.6).astype(np.uint8)
    k, s = an.bright_colocalization(F, m, z0=2, frac=0.1)
    for i, z in enumerate(range(2, 6)):
        f = F[z].ravel()
        kk = math.ceil(0.1 * f.size)
        # brute force: order by (-F, index)
        order = sorted(range(f.size), key=lambda j: (-f[j], j))[:kk]
        assert k[i] == kk and s[i] == sum(int(m[z].ravel()[j] == 0) for j in order)


def test_bright_colocalization_integer_ranking():
    """Tallies that differ by one near 2^62 (equal as float64) keep their order."""
    m = np.zeros((1, 1, 4), dtype=np.uint8)
    m[0, 0, 2] = 1
    base = 2 ** 62
    F = np.array([[[base, base, base + 1, base]]], dtype=np.int64)
    k, s = an.bright_colocalization(F, m, 0, 0.25)
    assert k[0] == 1 and s[0] == 0                  # the single brightest voxel is the pore voxel
    F2 = np.array([[[-(2 ** 63), 2 ** 63 - 1, 0, -1]]], dtype=np.int64)
    m2 = np.array([[[0, 1, 0, 0]]], dtype=np.uint8)
    k2, s2 = an.bright_colocalization(F2, m2, 0, 0.75)
    assert k2[0] == 3 and s2[0] == 2                # 2^63 - 1, 0, -1: the extreme minimum left out


def test_pore_distance_brute_force():
    for seed in (5, 6):
        m = inputs.spinodal_mask(9, 7, 8, 4.0, 0.7, seed=seed)
        assert np.array_equal(an.pore_distance(m), an.pore_distance_brute(m))


def _pearson(a, b):
    a = a - a.mean()
    b = b - b.mean()
    return float((a * b).sum() / math.sqrt((a * a).sum() * (b * b).sum()))


def test_pore_spearman_pins():
    # no ties: the closed form on rank differences
    rng = np.random.default_rng(8)
    x, y = rng.permutation(30).astype(float), rng.permutation(30).astype(float)
    n = 30
    closed = 1 - 6 * ((x - y) ** 2).sum() / (n * (n * n - 1))
    m = np.ones((1, 5, 6), dtype=np.uint8)
    m[0, 0, 0] = 0                                   # one solid voxel: distances vary
    dist = an.pore_distance(m)[0].ravel()
    # fluence equal to a strictly increasing function of the distance -> rho = +1, decreasing -> -1
    F = np.argsort(np.argsort(dist, kind="stable"), kind="stable").reshape(1, 5, 6) * 3 + 7
    sel = m[0].ravel() == 1
    # ties in the distance: Pearson of counted average ranks, whatever the fluence
    rho_up, npore = an.pore_spearman(F, m, 0)
    assert npore[0] == 29
    want = _pearson(an.average_ranks_brute(F[0].ravel()[sel]), an.average_ranks_brute(dist[sel]))
    assert math.isclose(rho_up[0], want, rel_tol=1e-12) and rho_up[0] > 0.9
    rho_dn, _ = an.pore_spearman(-F, m, 0)
    assert math.isclose(rho_dn[0], -want, rel_tol=1e-12)
    assert math.isclose(_pearson(an.average_ranks_brute(x), an.average_ranks_brute(y)), closed, rel_tol=1e-12)
    # distances without ties: a single row, solid at one end -> distance strictly increasing
    m2 = np.ones((1, 1, 31), dtype=np.uint8)
    m2[0, 0, 0] = 0
    F2 = np.zeros((1, 1, 31), dtype=np.int64)
    F2[0, 0, 1:] = x                                 # ranks of x against ranks 1..30 of the distance
    r2, n2 = an.pore_spearman(F2, m2, 0)
    closed2 = 1 - 6 * ((np.argsort(np.argsort(x)) - np.arange(30)) ** 2).sum() / (n * (n * n - 1))
    assert n2[0] == 30 and math.isclose(r2[0], closed2, rel_tol=1e-12)
    # degenerate slices: constant fluence, one pore voxel, no pore voxel
    m3 = np.zeros((3, 2, 2), dtype=np.uint8)
    m3[0] = 1
    m3[0, 0, 0] = 0
    m3[1, 1, 1] = 1
    r3, n3 = an.pore_spearman(np.ones((3, 2, 2), dtype=np.int64), m3, 0)
    assert list(n3) == [3, 1, 0] and np.all(np.isnan(r3))


def test_average_ranks_against_hand_count():
    r = an.average_ranks_brute(np.array([10, 20, 20, 5, 20]))
    assert list(r) == [2.0, 4.0, 4.0, 1.0, 4.0]


def test_mask_psd_stripes_closed_form():
    """Stripes of width 6 along x (period 12 in nx = 24): the transform is nonzero only at
    kx = 2h with odd h, where |m_hat|^2 = (ny nz)^2 * 4 / sin^2(pi h / 12); each such mode
    lies in shell kx and is counted with its conjugate."""
    nz, ny, nx = 6, 4, 24
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, :, (np.arange(nx) % 12) < 6] = 1
    p = an.mask_psd(m)
    want = np.zeros(nx // 2 + 1)
    for h in (1, 3, 5):
        want[2 * h] = 2 * (ny * nz) ** 2 * 4 / math.sin(math.pi * h / 12) ** 2
    assert np.allclose(p, want, rtol=1e-12, atol=1e-9 * want.max())
    s_peak = int(np.argmax(p[1:])) + 1
    assert max(m.shape) / (2 * s_peak) == 6.0           # the dominant size is the stripe width


def test_mask_psd_complement_invariance():
    """m and 1 - m differ only in the mean, which the PSD excludes."""
    m = inputs.spinodal_mask(12, 18, 24, 6.0, 0.7, seed=3)
    assert np.allclose(an.mask_psd(m), an.mask_psd(1 - m), rtol=1e-12, atol=1e-9)


def test_phase_contrast_hand_example():
    """Contrasts 1, 2, 3 (solid) and 2, 1, 0.5 (pore) of three depths, and a fourth depth
    with no light, which is skipped: means and sample standard deviations by hand."""
    t = np.array([1.0, 1.0, 2.0, 0.0])
    s = np.array([1.0, 2.0, 6.0, 0.0])
    p = np.array([2.0, 1.0, 1.0, 0.0])
    pc = an.phase_contrast(t, s, p)
    assert pc["depths"] == 3
    assert pc["solid_mean"] == 2.0 and math.isclose(pc["solid_sd"], 1.0, rel_tol=1e-15)
    assert math.isclose(pc["pore_mean"], 3.5 / 3, rel_tol=1e-15)
    dev = np.array([2.0, 1.0, 0.5]) - 3.5 / 3
    assert math.isclose(pc["pore_sd"], math.sqrt((dev ** 2).sum() / 2), rel_tol=1e-14)


def test_escape_histogram_hand_example():
    """Bins are [b w, (b + 1) w), the last one open; only escaping fates (4, 5) count;
    thresholds are strict."""
    fate = np.array([4, 5, 4, 4, 6, 5], dtype=np.uint32)
    w = np.array([10, 20, 30, 40, 50, 60], dtype=np.int64)
    pv = np.array([0.4, 1.6, 2.0, 9.9, 1.0, 1.0])
    hw, hn, aw, an_ = an.escape_path_histogram(fate, w, pv, 1.0, 4, thresholds=(1.0, 1.6))
    assert list(hn) == [1, 2, 1, 1] and list(hw) == [10, 80, 30, 40]
    assert list(aw) == [20 + 30 + 40, 30 + 40] and list(an_) == [3, 2]
