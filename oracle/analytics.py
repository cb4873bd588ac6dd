"""FP64 / integer oracle of the morphology and fluence analytics of Sec. 3.5.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU baseline use it; the
product library never imports it and it never imports the product.

What it follows (paper: "Three-dimensional photon transport in spinodal
photocatalytic aerogels", Sec. 3.5):
  (a) chord-length distributions of the binary mask along a chosen axis (the beam
      axis z in the paper): every maximal run of consecutive voxels of one phase on
      a line is a chord; mean chords and length-weighted tail fractions
      P_len(l > t) = sum_{l > t} l n(l) / sum_l l n(l);
  (b) phase-resolved fluence normalised at each depth by the lateral mean:
      c_solid(z) = <F>_solid(z) / <F>(z) and c_pore(z) likewise, and their mean and
      standard deviation over depth;
  (c) per-photon path statistics of escaping photons: the weighted and unweighted
      distribution of the in-pore path, and the fractions above thresholds;
  co-localisation: on each deep slice z >= z0, the brightest decile of voxels by
      fluence and the fraction of it that is solid; the local pore size by a
      Euclidean distance transform of the pore phase, and, inside the pore phase of
      each deep slice, the Spearman rank correlation of fluence with that size;
  and (Sec. 3.1, Fig. 2b) the radial power spectral density of the binary mask.
Readings where the paper is silent (listed with their reasons in the design
notes): chords cut by the slab faces count with their in-slab length; the
brightest decile of a slice is its ceil(0.1 N) voxels of highest fluence with
ties to the lower linear index (ranking inside one slice is what removing the
depth trend amounts to); the distance transform is the distance from a pore voxel
to the nearest solid voxel centre inside the volume (no periodic images), as
scipy.ndimage.distance_transform_edt computes it; the Spearman correlation takes
tied values at their average rank (scipy.stats.spearmanr), is computed per slice
z >= z0 over that slice's pore voxels, and is NaN where a slice has fewer than two
pore voxels or a constant rank vector.
"""
from __future__ import annotations

import math

import numpy as np


def chord_histogram(mask: np.ndarray, axis: int = 0) -> np.ndarray:
    """hist[phase][l] = number of chords of length l (phase 0 solid, 1 pore) along
    `axis` of a [nz, ny, nx] mask (axis 0 = z).  Shape (2, n_axis + 1)."""
    m = np.moveaxis(np.asarray(mask, dtype=np.uint8), axis, -1)
    n = m.shape[-1]
    lines = m.reshape(-1, n)
    hist = np.zeros((2, n + 1), dtype=np.int64)
    for line in lines:
        start = 0
        for i in range(1, n + 1):
            if i == n or line[i] != line[start]:
                hist[int(line[start]), i - start] += 1
                start = i
    return hist


def chord_stats(hist: np.ndarray, thresholds=()) -> dict:
    """Mean chord per phase and length-weighted tail fractions of the pore chords."""
    lengths = np.arange(hist.shape[1], dtype=np.float64)
    out = {}
    for ph, name in ((0, "solid"), (1, "pore")):
        n = hist[ph].astype(np.float64)
        total = (lengths * n).sum()
        out[f"mean_{name}"] = total / n.sum() if n.sum() else float("nan")
        for t in thresholds:
            out[f"plen_{name}_gt_{t}"] = (lengths * n)[lengths > t].sum() / total if total else float("nan")
    return out


def phase_contrast(depth_total: np.ndarray, depth_solid: np.ndarray, depth_pore: np.ndarray, z0: int = 0) -> dict:
    """Per-depth contrasts of the phase means to the lateral mean, over z >= z0 where
    the lateral mean is positive; mean and sample standard deviation over depth."""
    t = np.asarray(depth_total, dtype=np.float64)[z0:]
    s = np.asarray(depth_solid, dtype=np.float64)[z0:]
    p = np.asarray(depth_pore, dtype=np.float64)[z0:]
    oks = (t > 0) & np.isfinite(s)          # slices holding solid voxels
    okp = (t > 0) & np.isfinite(p)          # slices holding pore voxels
    cs, cp = s[oks] / t[oks], p[okp] / t[okp]
    return {"solid_mean": cs.mean() if cs.size else float("nan"), "solid_sd": cs.std(ddof=1) if cs.size > 1 else 0.0,
            "pore_mean": cp.mean() if cp.size else float("nan"), "pore_sd": cp.std(ddof=1) if cp.size > 1 else 0.0,
            "depths": int(((t > 0)).sum())}


def escape_path_histogram(fate: np.ndarray, w_final: np.ndarray, path_void: np.ndarray, bin_width: float,
                          nbins: int, thresholds=()):
    """Weighted (Q31 integer weights) and unweighted histograms of the in-pore path
    of escaping photons (fate 4 or 5): bin b holds b*width <= path < (b+1)*width, the
    last bin everything beyond; and the weight / count with path > each threshold."""
    esc = (fate == 4) | (fate == 5)
    pv = np.asarray(path_void, dtype=np.float64)[esc]
    w = np.asarray(w_final, dtype=np.int64)[esc]
    b = np.minimum(np.floor(pv / bin_width), nbins - 1).astype(np.int64)
    hw = np.bincount(b, weights=None, minlength=nbins)   # unweighted counts
    hist_w = np.zeros(nbins, dtype=np.int64)
    np.add.at(hist_w, b, w)
    above_w = np.array([int(w[pv > t].sum()) for t in thresholds], dtype=np.int64)
    above_n = np.array([int((pv > t).sum()) for t in thresholds], dtype=np.int64)
    return hist_w, hw.astype(np.int64), above_w, above_n


def bright_colocalization(fluence: np.ndarray, mask: np.ndarray, z0: int, frac: float = 0.1):
    """For each slice z >= z0: (k, solid_in_top) with k = ceil(frac * N_slice) voxels of
    highest fluence, ties to the lower index (stable ascending sort of a decreasing map
    of F).  An integer tally is ranked as integers: ~F = -F - 1 reverses the order of
    every int64 without overflow, so no two distinct tallies compare equal."""
    nz = fluence.shape[0]
    k_all, solid_all = [], []
    for z in range(z0, nz):
        f = np.asarray(fluence[z]).ravel()
        k = int(math.ceil(frac * f.size))
        rev = ~f if np.issubdtype(f.dtype, np.integer) else -f.astype(np.float64)
        top = np.argsort(rev, kind="stable")[:k]
        k_all.append(k)
        solid_all.append(int((np.asarray(mask[z]).ravel()[top] == 0).sum()))
    return np.array(k_all, dtype=np.int64), np.array(solid_all, dtype=np.int64)


def pore_distance(mask: np.ndarray) -> np.ndarray:
    """Euclidean distance from each pore voxel to the nearest solid voxel (0 in the
    solid), scipy's exact transform: a library routine used as one step."""
    from scipy import ndimage

    return ndimage.distance_transform_edt(np.asarray(mask, dtype=np.uint8) == 1)


def pore_distance_brute(mask: np.ndarray) -> np.ndarray:
    """The same by brute force over all solid voxels (small masks only)."""
    m = np.asarray(mask, dtype=np.uint8)
    solid = np.argwhere(m == 0).astype(np.float64)
    out = np.zeros(m.shape, dtype=np.float64)
    for idx in np.argwhere(m == 1):
        if solid.size:
            out[tuple(idx)] = math.sqrt(((solid - idx) ** 2).sum(axis=1).min())
        else:
            out[tuple(idx)] = math.inf
    return out


def pore_spearman(fluence: np.ndarray, mask: np.ndarray, z0: int):
    """For each slice z >= z0: (rho, n_pore), the Spearman correlation between the
    fluence and the pore distance transform over the pore voxels of the slice
    (scipy.stats.spearmanr as one library step), NaN where undefined."""
    from scipy import stats

    m = np.asarray(mask, dtype=np.uint8)
    dist = pore_distance(m)
    nz = m.shape[0]
    rho, npore = [], []
    for z in range(z0, nz):
        sel = m[z].ravel() == 1
        f = np.asarray(fluence[z]).ravel()[sel]        # integer tallies ranked as integers
        d = dist[z].ravel()[sel]
        npore.append(int(sel.sum()))
        if f.size < 2 or np.all(f == f[0]) or np.all(d == d[0]):
            rho.append(math.nan)
        else:
            rho.append(float(stats.spearmanr(f, d).statistic))
    return np.array(rho, dtype=np.float64), np.array(npore, dtype=np.int64)


def average_ranks_brute(x: np.ndarray) -> np.ndarray:
    """1-based ranks with ties averaged, by counting: rank_i = #{x_j < x_i} + (#{x_j == x_i} + 1) / 2."""
    x = np.asarray(x)
    return np.array([(x < v).sum() + ((x == v).sum() + 1) / 2 for v in x], dtype=np.float64)


def mask_psd(mask: np.ndarray) -> np.ndarray:
    """Radial PSD of the binary mask (values 0/1): the Cahn-Hilliard oracle's shell
    sums applied to the mask's forward transform (numpy's rfftn as one step)."""
    from oracle import cahn_hilliard as och

    m = np.asarray(mask, dtype=np.float64)
    return och.radial_psd(och.spectrum(m), m.shape)
