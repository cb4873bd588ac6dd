"""Pins of the oracle's paper boundary model (air pads, Fresnel reflection and
refraction at index steps, specular lateral mirrors, time gate) against facts
other than the oracle itself:

* the Fresnel reflectance against the angle form of the Fresnel equations, the
  normal-incidence and Brewster-angle values, reciprocity and Snell's law;
* the padded, index-matched, periodic, ungated model reproduces the plain model
  bit for bit (the pads are transparent and untallied);
* a non-scattering solid slab against the closed form of incoherent multiple
  reflection between two Fresnel interfaces (with and without absorption);
* the mean-path theorem with refractive index: under Lambertian illumination of a
  non-absorbing medium, the mean path inside a region is 4 * integral(n^2 dV) / S
  (the equilibrium radiance inside index n is n^2 times the outside one), so the
  solid and pore paths are 2 Nz (1 - phi) n^2 and 2 Nz phi separately;
* the gate: straight collimated photons through an empty slab are cut exactly at
  the gate; under Lambertian incidence the gated fraction is ((Nz + 2) / G)^2;
* mirrors by unfolding: mirror faces on a mask are the periodic walk on the
  mask unfolded to twice its lateral size, tallies folded back.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2604_13929_amd import inputs

W1 = 2 ** 31
PAPER = oracle.BOUNDARY_PAPER
N_SOLID = float(np.float32(1.746))          # paper: n_eff of the solid shell (Table 2)
f32 = lambda x: float(np.float32(x))  # noqa: E731


def batch_mean_sd(per_batch: np.ndarray):
    B = per_batch.shape[0]
    return per_batch.mean(axis=0), per_batch.std(axis=0, ddof=1) / math.sqrt(B)


def closure(tot, n):
    return tot["R"] + tot["T"] + tot["A"] + tot["RR"] + tot["lost"] + tot["gated"] - n * W1


# --------------------------------------------------------------------------
# Fresnel reflectance
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n1,n2", [(1.0, 1.746), (1.746, 1.0), (1.0, 1.5), (1.33, 1.0), (2.4, 1.746)])
def test_fresnel_against_angle_form(n1, n2):
    """R from cosines against r_s = -sin(i-t)/sin(i+t), r_p = tan(i-t)/tan(i+t)."""
    rng = np.random.default_rng(1)
    crit = math.asin(n2 / n1) if n1 > n2 else math.pi / 2
    for th in rng.uniform(1e-3, crit - 1e-3, 200):
        R, ct = oracle.fresnel(n1, n2, math.cos(th))
        tt = math.asin(n1 / n2 * math.sin(th))
        assert math.isclose(n1 * math.sin(th), n2 * math.sin(tt), rel_tol=1e-12)
        assert math.isclose(ct, math.cos(tt), rel_tol=1e-12, abs_tol=1e-15)
        rs = -math.sin(th - tt) / math.sin(th + tt)
        rp = math.tan(th - tt) / math.tan(th + tt)
        assert math.isclose(R, 0.5 * (rs * rs + rp * rp), rel_tol=1e-10, abs_tol=1e-15)
        # reciprocity: the same interface crossed the other way at the refracted angle
        R2, ct2 = oracle.fresnel(n2, n1, math.cos(tt))
        assert math.isclose(R, R2, rel_tol=1e-10, abs_tol=1e-15)
        assert math.isclose(ct2, math.cos(th), rel_tol=1e-9)


def test_fresnel_special_angles():
    for n1, n2 in [(1.0, N_SOLID), (N_SOLID, 1.0), (1.0, 1.5)]:
        R, ct = oracle.fresnel(n1, n2, 1.0)
        assert math.isclose(R, ((n1 - n2) / (n1 + n2)) ** 2, rel_tol=1e-14) and ct == 1.0
        # Brewster: r_p = 0 and r_s = (n1^2 - n2^2)/(n1^2 + n2^2)
        tb = math.atan(n2 / n1)
        R, _ = oracle.fresnel(n1, n2, math.cos(tb))
        assert math.isclose(R, 0.5 * ((n1 ** 2 - n2 ** 2) / (n1 ** 2 + n2 ** 2)) ** 2, rel_tol=1e-9)
    # total internal reflection beyond the critical angle, R -> 1 approaching it
    cc = math.sqrt(1.0 - (1.0 / N_SOLID) ** 2)      # cosine of the critical angle
    assert oracle.fresnel(N_SOLID, 1.0, cc * 0.999)[0] == 1.0
    assert oracle.fresnel(N_SOLID, 1.0, cc * 0.999)[1] == 0.0
    R_near = oracle.fresnel(N_SOLID, 1.0, cc * (1 + 1e-9))[0]
    assert 0.99 < R_near < 1.0
    # matched indices reflect nothing
    assert oracle.fresnel(1.3, 1.3, 0.37)[0] < 1e-30
    assert 0.0738 < ((1 - 1.746) / (1 + 1.746)) ** 2 < 0.0739     # value quoted for the paper's n_eff


# --------------------------------------------------------------------------
# padded model, index 1, periodic, no gate == plain model
# --------------------------------------------------------------------------
def test_padded_index_matched_model_equals_plain(mask_m1):
    n = 20_000
    a = oracle.run(mask_m1, 0.5, f32(0.01), f32(0.7), n, seed=11, nbatch=2, depth=True)
    b = oracle.run(mask_m1, 0.5, f32(0.01), f32(0.7), n, seed=11, nbatch=2, depth=True, boundary=PAPER)
    assert np.array_equal(a["fluence"], b["fluence"]) and np.array_equal(a["depth"], b["depth"])
    ta, tb = oracle.totals(a), oracle.totals(b)
    for k in ("R", "T", "A", "RR", "lost", "esc_w", "esc_w_gtL", "esc_n", "esc_n_gtL", "interactions", "gated",
              "esc_w_void_path", "path_total", "path_solid", "path_void"):
        assert ta[k] == tb[k], k
    # every photon crosses the top pad once on entry and one pad on escape (at least)
    assert tb["steps"] >= ta["steps"] + 2 * n
    # the same photons' traces, shifted by the entry step through the pad
    ids = np.arange(40, dtype=np.uint64) * 7
    ra, _ = oracle.trace(mask_m1, 0.5, f32(0.01), f32(0.7), ids, 11, max_rec=32)
    rb, _ = oracle.trace(mask_m1, 0.5, f32(0.01), f32(0.7), ids, 11, max_rec=33, boundary=PAPER)
    assert np.all(rb["iz"][:, 0] == -1) and np.all(rb["event"][:, 0] == 2)
    for c in ("ix", "iy", "fx", "fy", "ux", "uy", "uz", "w", "k"):
        live = ra["event"][:, :20] >= 0
        stays = live & (ra["iz"][:, :20] >= 0)
        assert np.array_equal(ra[c][:, :20][stays], rb[c][:, 1:21][stays]), c


# --------------------------------------------------------------------------
# non-scattering slab between two Fresnel interfaces
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mu_a", [0.0, 0.05])
@pytest.mark.parametrize("lateral", [0, 1])
def test_slab_multiple_reflection_closed_form(mu_a, lateral):
    """Collimated normal incidence on a solid slab with mu_s = 0: every crossing of
    a face reflects with r = ((n-1)/(n+1))^2, the slab transmits e^{-mu_a L} per pass:
        T = (1-r)^2 t / (1 - r^2 t^2),  R = r + r (1-r)^2 t^2 / (1 - r^2 t^2)."""
    nz, n = 12, 200_000
    mask = inputs.homogeneous_mask(4, 4, nz)
    B = 32
    res = oracle.run(mask, 0.0, mu_a, 0.0, n, seed=5, nbatch=B, fluence=False, boundary=PAPER,
                     lateral=lateral, n_solid=N_SOLID)
    tot = oracle.totals(res)
    assert closure(tot, n) == 0
    r = ((N_SOLID - 1) / (N_SOLID + 1)) ** 2
    t = math.exp(-f32(mu_a) * nz)
    T = (1 - r) ** 2 * t / (1 - r * r * t * t)
    R = r + r * (1 - r) ** 2 * t * t / (1 - r * r * t * t)
    for key, want in (("R", R), ("T", T), ("A", 1 - R - T)):
        per = res["ich"][:, oracle.ICH.index(key)] / (n / B * W1)
        m, sd = batch_mean_sd(per)
        assert abs(m - want) < 4 * sd + 1e-12, (key, m, want, sd)
    if mu_a == 0.0:
        assert tot["A"] == 0 and tot["R"] + tot["T"] == n * W1


# --------------------------------------------------------------------------
# mean path with refractive index: 4 integral(n^2 dV) / S
# --------------------------------------------------------------------------
def test_mean_path_invariance_with_index_homogeneous():
    B, n, nz = 16, 100_000, 12
    mask = inputs.homogeneous_mask(6, 6, nz)
    for lateral in (0, 1):
        r = oracle.run(mask, 0.5, 0.0, 0.7, n, seed=21, nbatch=B, source=1, fluence=False,
                       boundary=PAPER, lateral=lateral, n_solid=N_SOLID)
        ps = r["dch"][:, oracle.DCH.index("path_solid")] / (n / B)
        m, sd = batch_mean_sd(ps)
        assert abs(m - 2 * nz * N_SOLID ** 2) < 4 * sd, (lateral, m, 2 * nz * N_SOLID ** 2, sd)
        assert oracle.totals(r)["A"] == 0


def test_mean_path_invariance_with_index_on_mask():
    """Both phases of a bicontinuous mask, both illumination sides averaged: solid path
    2 Nz (1-phi) n^2, pore path 2 Nz phi, total 2 Nz [(1-phi) n^2 + phi]."""
    B, n = 16, 100_000
    mask = inputs.spinodal_mask(16, 16, 16, 6.0, 0.6, seed=3)
    phi = mask.mean()
    nz = mask.shape[0]
    for lateral in (0, 1):
        ps, pv = [], []
        for m in (mask, np.ascontiguousarray(mask[::-1])):
            r = oracle.run(m, 0.5, 0.0, 0.7, n, seed=22, nbatch=B, source=1, fluence=False,
                           boundary=PAPER, lateral=lateral, n_solid=N_SOLID)
            ps.append(r["dch"][:, oracle.DCH.index("path_solid")] / (n / B))
            pv.append(r["dch"][:, oracle.DCH.index("path_void")] / (n / B))
        ms, ss = batch_mean_sd(0.5 * (ps[0] + ps[1]))
        mv, sv = batch_mean_sd(0.5 * (pv[0] + pv[1]))
        assert abs(ms - 2 * nz * (1 - phi) * N_SOLID ** 2) < 4 * ss, (lateral, ms, ss)
        assert abs(mv - 2 * nz * phi) < 4 * sv, (lateral, mv, sv)


# --------------------------------------------------------------------------
# time gate
# --------------------------------------------------------------------------
def test_gate_cuts_straight_photons_exactly():
    """Empty slab, collimated: optical path 1 in the top pad, then layer z spans
    [1 + z, 2 + z]; each layer receives min(max(G - 1 - z, 0), 1) per photon."""
    nx, ny, nz, n = 3, 2, 8, 6000
    mask = inputs.homogeneous_mask(nx, ny, nz, pore=True)
    for G in (5.25, 3.0, 1.5, 9.75):
        res = oracle.run(mask, 0.5, f32(0.01), 0.0, n, seed=9, boundary=PAPER, gate=G, n_solid=N_SOLID)
        tot = oracle.totals(res)
        assert tot["gated"] == n * W1 and tot["R"] == tot["T"] == tot["A"] == 0
        layer = res["fluence"][0].sum(axis=(1, 2)) / (n * W1)
        want = np.clip(G - 1 - np.arange(nz), 0, 1)
        assert np.array_equal(layer, want), (G, layer, want)
    res = oracle.run(mask, 0.5, f32(0.01), 0.0, n, seed=9, boundary=PAPER, gate=float(nz + 2))
    tot = oracle.totals(res)
    assert tot["T"] == n * W1 and tot["gated"] == 0


def test_gate_lambertian_fraction():
    """Empty slab, Lambertian incidence: the optical path to the far pad's outer face
    is (Nz + 2)/cos(theta); P(cos < c) = c^2, so the gated fraction is ((Nz + 2)/G)^2."""
    nz, n, B = 6, 200_000, 32
    mask = inputs.homogeneous_mask(4, 4, nz, pore=True)
    G = 4.0 * (nz + 2)
    res = oracle.run(mask, 0.5, 0.0, 0.0, n, seed=13, nbatch=B, source=1, fluence=False, boundary=PAPER,
                     lateral=1, gate=G)
    assert closure(oracle.totals(res), n) == 0
    per = res["ich"][:, oracle.ICH.index("gated")] / (n / B * W1)
    m, sd = batch_mean_sd(per)
    assert abs(m - ((nz + 2) / G) ** 2) < 4 * sd


def test_gate_closure_and_fates(mask_m1):
    n = 20_000
    res = oracle.run(mask_m1, 0.5, f32(0.01), f32(0.7), n, seed=17, boundary=PAPER, lateral=1,
                     n_solid=N_SOLID, gate=150.0)
    tot = oracle.totals(res)
    assert closure(tot, n) == 0 and tot["gated"] > 0 and tot["lost"] == 0
    ids = np.arange(200, dtype=np.uint64)
    recs, summ = oracle.trace(mask_m1, 0.5, f32(0.01), f32(0.7), ids, 17, max_rec=4096, boundary=PAPER,
                              lateral=1, n_solid=N_SOLID, gate=150.0)
    gated = summ["fate"] == 9
    assert gated.any()
    # the optical path never passes the gate: sum of n * d over each trace
    for i in np.flatnonzero(gated)[:20]:
        v = recs[i][recs[i]["event"] >= 0]
        solid = np.array([(0 <= z < mask_m1.shape[0]) and mask_m1[z, y, x] == 0
                          for x, y, z in zip(v["ix"], v["iy"], v["iz"])])
        lopt = np.sum(np.where(solid, N_SOLID, 1.0) * v["d"])
        assert math.isclose(lopt, 150.0, rel_tol=1e-12)


def test_reflections_keep_the_voxel_and_flip_the_normal(mask_m1):
    ids = np.arange(100, dtype=np.uint64)
    recs, _ = oracle.trace(mask_m1, 0.5, f32(0.01), f32(0.7), ids, 23, max_rec=256, boundary=PAPER,
                           lateral=1, n_solid=N_SOLID)
    seen = 0
    for row in recs:
        for j in range(row.size - 1):
            ev = row["event"][j]
            if ev in (10, 11, 12) and row["event"][j + 1] >= 0:
                a = ev - 10
                c = "xyz"[a]
                nxt = row[j + 1]
                assert (nxt["ix"], nxt["iy"], nxt["iz"]) == (row["ix"][j], row["iy"][j], row["iz"][j])
                assert nxt["u" + c] == -row["u" + c][j] and nxt["f" + c] in (0.0, 1.0)
                seen += 1
            if ev in (0, 1, 2) and row["event"][j + 1] >= 0:
                # a crossing conserves n * (tangential direction): Snell's law on every face
                u0 = np.array([row["ux"][j], row["uy"][j], row["uz"][j]])
                u1 = np.array([row["ux"][j + 1], row["uy"][j + 1], row["uz"][j + 1]])
                assert math.isclose(np.linalg.norm(u1), 1.0, rel_tol=1e-12)
                i0 = (row["ix"][j], row["iy"][j], row["iz"][j])
                i1 = (row["ix"][j + 1], row["iy"][j + 1], row["iz"][j + 1])

                def idx(v):
                    x, y, z = v
                    return N_SOLID if (0 <= z < mask_m1.shape[0] and mask_m1[z, y, x] == 0) else 1.0
                t = [b for b in range(3) if b != ev]
                assert np.allclose(idx(i0) * u0[t], idx(i1) * u1[t], rtol=1e-12, atol=1e-15)
    assert seen > 50


# --------------------------------------------------------------------------
# mirrors by unfolding
# --------------------------------------------------------------------------
def test_mirror_faces_equal_the_unfolded_periodic_walk():
    """Mirror lateral faces on mask M equal periodic faces on M unfolded to 2nx x 2ny
    (each copy mirrored), with the source over the whole unfolded face; fold the
    tallies back and compare per-voxel means within 4 sigma (chi^2 per voxel ~ 1)."""
    nx, ny, nz = 6, 5, 10
    M = inputs.spinodal_mask(nx, ny, nz, 4.0, 0.6, seed=7)
    top = np.concatenate([M, M[:, :, ::-1]], axis=2)
    U = np.ascontiguousarray(np.concatenate([top, top[:, ::-1, :]], axis=1))
    n, B = 200_000, 16
    kw = dict(nbatch=B, boundary=PAPER, n_solid=N_SOLID)
    a = oracle.run(M, 0.5, f32(0.02), f32(0.7), n, seed=31, lateral=1, **kw)
    b = oracle.run(U, 0.5, f32(0.02), f32(0.7), n, seed=32, lateral=0, **kw)
    Fa = a["fluence"] * (nx * ny) / (n / B * W1)                  # Phi / S0 per batch
    Fu = b["fluence"] * (4 * nx * ny) / (n / B * W1)
    Fb = 0.25 * (Fu[..., :ny, :nx] + Fu[..., :ny, nx:][..., ::-1]
                 + Fu[..., ny:, :nx][..., ::-1, :] + Fu[..., ny:, nx:][..., ::-1, ::-1])
    ma, sa = batch_mean_sd(Fa)
    mb, sb = batch_mean_sd(Fb)
    z = (ma - mb) / np.sqrt(sa ** 2 + sb ** 2)
    assert np.mean(z ** 2) < 1.3 and np.abs(z).max() < 5.0
    for key in ("R", "T", "A"):
        pa = a["ich"][:, oracle.ICH.index(key)] / (n / B * W1)
        pb = b["ich"][:, oracle.ICH.index(key)] / (n / B * W1)
        (m1, s1), (m2, s2) = batch_mean_sd(pa), batch_mean_sd(pb)
        assert abs(m1 - m2) < 4 * math.hypot(s1, s2), key


def test_boundary_validation(mask_m1):
    with pytest.raises(ValueError):
        oracle.run(mask_m1, 0.5, 0.01, 0.7, 10, seed=1, lateral=1)             # mirrors need the paper model
    with pytest.raises(ValueError):
        oracle.run(mask_m1, 0.5, 0.01, 0.7, 10, seed=1, n_solid=1.5)           # so does an index
    with pytest.raises(ValueError):
        oracle.run(mask_m1, 0.5, 0.01, 0.7, 10, seed=1, boundary=PAPER, n_solid=0.9)
    with pytest.raises(ValueError):
        oracle.run(mask_m1, 0.5, 0.01, 0.7, 10, seed=1, boundary=PAPER, gate=0.0)
    with pytest.raises(ValueError):
        oracle.run(mask_m1, 0.5, 0.01, 0.7, 10, seed=1, boundary=2)
