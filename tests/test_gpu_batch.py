"""Batched multi-mask launch: every job of a batch against the FP64 oracle on the
same photons (jobs spanning the 64-job workload's sizes, porosities and optics, with
stream ids and photon ranges other than 0); job k of a batch equals a plain run of
job k, bit for bit, for any launch shape; the captured graph replays the same bits;
the reduction of every job equals mc_reduce on that job; the autotuner returns a
usable shape; the per-job escape-path histograms (Sec. 3.5 (c)) equal single runs'
and the oracle's."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from oracle import analytics as oan
from oracle import estimators as est
from paper_2604_13929_amd import inputs
from paper_2604_13929_amd import photonmc as pm

pytestmark = pytest.mark.gpu
f32 = lambda x: float(np.float32(x))  # noqa: E731


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pm.load()


@pytest.fixture(scope="module")
def small_jobs():
    """Six jobs of uneven (ragged) size, porosity and optics."""
    spec = [(37, 29, 23, 0.6, 0.5, 0.01, 0.7, 20000), (16, 16, 40, 0.9, 1.0, 0.05, 0.5, 5000),
            (48, 48, 48, 0.5, 0.2, 0.005, 0.9, 30000), (8, 8, 8, 0.7, 0.7, 0.02, 0.6, 1),
            (24, 40, 12, 0.8, 0.3, 0.03, 0.8, 12345), (32, 32, 32, 0.7, 0.5, 0.01, 0.7, 40000)]
    jobs = []
    for i, (nx, ny, nz, phi, mus, mua, g, n) in enumerate(spec):
        m = torch.from_numpy(inputs.spinodal_mask(nx, ny, nz, 8.0, phi, seed=100 + i)).cuda()
        jobs.append(pm.BatchJob(m, pm.Optics(f32(mus), f32(mua), f32(g)), n, seed=20260809, stream_id=i,
                                photon_begin=7 * i))
    return jobs


W1 = 2 ** 31
# the largest rounding 4096 segments' deposits can add up to (each rounded to a whole deposit quantum)
ROUNDING_4096 = 0.5 * pm.DEPOSIT_QUANTUM * 4096


@pytest.fixture(scope="module")
def oracle_jobs():
    """Six jobs at the corners of the 64-job workload's ranges (phi 0.5 / 0.9, solid mu_s
    0.2 / 1.0, mu_a 0.005 / 0.05, g 0.5 / 0.9) and one in the middle, on ragged cubes of
    16 to 48 voxels, each with its own stream id and a photon range that does not start
    at 0."""
    spec = [(16, 16, 16, 0.5, 0.2, 0.005, 0.5, 3, 1000),
            (48, 48, 48, 0.9, 1.0, 0.05, 0.9, 7, 123_456),
            (37, 29, 23, 0.5, 1.0, 0.005, 0.9, 11, 5),
            (24, 40, 47, 0.9, 0.2, 0.05, 0.5, 13, 999_999),
            (45, 20, 31, 0.6, 0.45, 0.01, 0.8, 42, 77),
            (33, 33, 33, 0.7, 0.6, 0.0275, 0.7, 63, 2 ** 31)]
    jobs = []
    for i, (nx, ny, nz, phi, mus, mua, g, sid, begin) in enumerate(spec):
        m = inputs.spinodal_mask(nx, ny, nz, 8.0, phi, seed=200 + i)
        jobs.append((m, pm.BatchJob(torch.from_numpy(m).cuda(), pm.Optics(f32(mus), f32(mua), f32(g)), 60_000,
                                    seed=20260809, stream_id=sid, photon_begin=begin)))
    return jobs


def _oracle_of(m, j: pm.BatchJob, nbatch):
    o = j.optics
    return oracle.run(m, o.mu_s, o.mu_a, o.g, j.n_photons, j.seed, photon_begin=j.photon_begin,
                      stream_id=j.stream_id, nbatch=nbatch)


def test_batch_jobs_match_oracle(oracle_jobs):
    """FP32 batch: per job, the globals within 0.5 %, R/T/A within 0.5 % of the launched
    weight, steps within 0.1 %, and every voxel within 4 sigma of the oracle's spread
    over 32 photon batches (voxels the oracle never reached must be exactly 0)."""
    banner("batch of 6 (FP32) vs the FP64 oracle, job by job")
    b = pm.run_batch([j for _, j in oracle_jobs], tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    for k, (m, j) in enumerate(oracle_jobs):
        n = j.n_photons
        ref = _oracle_of(m, j, 32)
        tot = oracle.totals(ref)
        Fb = ref["fluence"]
        F_o = Fb.sum(axis=0)
        e = est.estimators(F_o, m, n)
        s = b.summary(k)
        sc = b.results[k].scalar_dict()
        assert sc["launched"] == n and s["closure_exact"] == 1.0 and sc["lost"] == 0, k
        for key in ("phi3d", "phi1d", "phi_pore", "r", "L_opt"):
            assert abs(s[key] - e[key]) <= 5e-3 * abs(e[key]), (k, key, s[key], e[key])
        for key in ("R", "T", "A"):
            assert abs(sc[key] - tot[key]) <= 5e-3 * n * W1, (k, key)
        assert abs(sc["steps"] - tot["steps"]) <= 1e-3 * tot["steps"], k
        F_g = b.results[k].fluence.cpu().numpy().astype(np.float64)
        sd = Fb.std(axis=0, ddof=1) * math.sqrt(Fb.shape[0])
        on = sd > 0
        assert np.all(np.abs(F_g - F_o)[on] <= 4 * sd[on]), k
        assert np.all(F_g[~on] == F_o[~on]), k
        print(f"job {k}: phi3d {s['phi3d']:.6f} (oracle {e['phi3d']:.6f}), steps {sc['steps']} "
              f"(oracle {tot['steps']})")


def test_batch_paper_model_jobs_match_oracle():
    """Jobs under the paper's boundary model in one FP32 batch (air pads, solid index
    1.746 with Fresnel faces; lateral mirrors with a time gate of 300 voxels, periodic
    faces with none), next to a plain job: per job, the globals (gated fraction
    included) within 0.5 %, R/T/A within 0.5 % of the launched weight, steps within
    0.1 %, and every voxel within 4 sigma of the oracle's spread over 32 photon batches."""
    banner("batch mixing paper-model and plain jobs (FP32) vs the FP64 oracle, job by job")
    spec = [(24, 20, 28, 0.7, 0.5, 0.01, 0.7, pm.LATERAL_MIRROR, 300.0, 5, 11),
            (32, 16, 20, 0.6, 0.3, 0.02, 0.8, pm.LATERAL_PERIODIC, 0.0, 9, 4_321),
            (20, 20, 20, 0.8, 0.8, 0.03, 0.6, None, 0.0, 17, 0)]
    jobs = []
    for i, (nx, ny, nz, phi, mus, mua, g, lateral, gate, sid, begin) in enumerate(spec):
        m = inputs.spinodal_mask(nx, ny, nz, 8.0, phi, seed=300 + i)
        if lateral is None:
            opt = pm.Optics(f32(mus), f32(mua), f32(g))
        else:
            opt = pm.paper_optics(f32(mus), f32(mua), f32(g), n_solid=f32(1.746), lateral=lateral, gate=gate)
        jobs.append((m, pm.BatchJob(torch.from_numpy(m).cuda(), opt, 40_000, seed=20260809, stream_id=sid,
                                    photon_begin=begin)))
    b = pm.run_batch([j for _, j in jobs], tune=pm.Tune(256, 16, 64, 8, 8))
    torch.cuda.synchronize()
    for k, (m, j) in enumerate(jobs):
        o, n = j.optics, j.n_photons
        kw = dict(boundary=o.boundary, lateral=o.lateral, n_solid=o.n_solid if o.n_solid else 1.0,
                  gate=o.gate if o.gate > 0 else float("inf"))
        ref = oracle.run(m, o.mu_s, o.mu_a, o.g, n, j.seed, photon_begin=j.photon_begin, stream_id=j.stream_id,
                         nbatch=32, **kw)
        tot = oracle.totals(ref)
        Fb = ref["fluence"]
        F_o = Fb.sum(axis=0)
        e = est.estimators(F_o, m, n)
        s = b.summary(k)
        sc = b.results[k].scalar_dict()
        assert sc["launched"] == n and s["closure_exact"] == 1.0 and sc["lost"] == 0, k
        for key in ("phi3d", "phi1d", "phi_pore", "r"):
            assert abs(s[key] - e[key]) <= 5e-3 * abs(e[key]), (k, key, s[key], e[key])
        for key in ("R", "T", "A", "gated"):
            assert abs(sc[key] - tot[key]) <= 5e-3 * n * W1, (k, key, sc[key], tot[key])
        assert abs(sc["steps"] - tot["steps"]) <= 1e-3 * tot["steps"], k
        if o.gate > 0:
            assert tot["gated"] > 0, k                     # the gate cuts some photons
        F_g = b.results[k].fluence.cpu().numpy().astype(np.float64)
        sd = Fb.std(axis=0, ddof=1) * math.sqrt(Fb.shape[0])
        on = sd > 0
        assert np.all(np.abs(F_g - F_o)[on] <= 4 * sd[on]), k
        assert np.all(F_g[~on] == F_o[~on]), k
        print(f"job {k}: phi3d {s['phi3d']:.6f} (oracle {e['phi3d']:.6f}), gated {sc['gated'] / (n * W1):.4f} "
              f"(oracle {tot['gated'] / (n * W1):.4f})", flush=True)


def test_batch_fp64_jobs_equal_oracle(oracle_jobs):
    """FP64 transport in the batch: every integer channel of every job equals the
    oracle's, and the fluence equals it up to the per-segment rounding of deposits in
    at least 99.9 % of the voxels.  The rest may differ by FP64 trajectory drift: over
    a walk of hundreds of steps the rounding of two FP64 evaluations of the same steps
    grows through shallow face crossings (one photon of job 2, mu_s 1.0, g 0.9, reached
    3e-6 voxel after 700 steps without changing a decision), which moves that much
    track length between neighbouring voxels: bounded here by 1e-6 of the voxel's
    tally."""
    banner("batch of 6 (FP64 transport) vs the FP64 oracle: integer channels exact")
    b = pm.run_batch([j for _, j in oracle_jobs], tune=pm.Tune(128, 8, 64, 8), fp64=True)
    torch.cuda.synchronize()
    for k, (m, j) in enumerate(oracle_jobs):
        ref = _oracle_of(m, j, 1)
        tot = oracle.totals(ref)
        sc = b.results[k].scalar_dict()
        for key in ("R", "T", "A", "RR", "lost", "esc_w", "esc_w_gtL", "esc_n", "esc_n_gtL", "steps",
                    "interactions"):
            assert sc[key] == tot[key], (k, key, sc[key], tot[key])
        F_g = b.results[k].fluence.cpu().numpy().astype(np.float64)
        F_o = ref["fluence"][0]
        diff = np.abs(F_g - F_o)
        bad = diff > 1e-9 * F_o + ROUNDING_4096
        if bad.any():
            _report_fluence_mismatch(m, j, F_g, F_o, bad)
        assert bad.mean() <= 1e-3, k
        assert np.all(diff <= 1e-6 * F_o + ROUNDING_4096), k


def _report_fluence_mismatch(m, j, F_g, F_o, bad):
    """Print what names the failing voxels and the photons whose outcomes differ."""
    idx = np.argwhere(bad)
    print(f"{len(idx)} voxels outside the rounding bound; worst:", flush=True)
    diff = np.abs(F_g - F_o)
    for z, y, x in idx[np.argsort(-diff[bad])][:8]:
        print(f"  (z {z}, y {y}, x {x}) pore {m[z, y, x]}: gpu {F_g[z, y, x]:.6e} oracle {F_o[z, y, x]:.6e} "
              f"diff {F_g[z, y, x] - F_o[z, y, x]:.6e}", flush=True)
    ids = np.arange(j.photon_begin, j.photon_begin + j.n_photons, dtype=np.uint64)
    _, go = pm.trace(j.mask, j.optics, ids, 0, j.seed, stream_id=j.stream_id, fp64=True)
    o = j.optics
    _, oo = oracle.trace(m, o.mu_s, o.mu_a, o.g, ids, j.seed, max_rec=0, stream_id=j.stream_id)
    diff_ph = np.zeros(len(ids), dtype=bool)
    for f in ("fate", "steps", "interactions", "A", "w_final"):
        diff_ph |= go[f].astype(np.int64) != oo[f].astype(np.int64)
    diff_ph |= np.abs(go["path_void"] - oo["path_void"]) > 1e-6
    print(f"{diff_ph.sum()} photons end differently; first: {ids[diff_ph][:5]}, "
          f"oracle min_gap there {oo['min_gap'][diff_ph][:5]}", flush=True)


def _plain(j: pm.BatchJob, fp64=False):
    r = pm.run(j.mask, j.optics, j.n_photons, j.seed, photon_begin=j.photon_begin, stream_id=j.stream_id, fp64=fp64)
    return r, pm.reduce(j.mask, r)


def test_batch_equals_plain_runs(small_jobs):
    banner("batch of 6 == 6 plain runs, bitwise, several launch shapes")
    plains = [_plain(j) for j in small_jobs]
    for tune in (pm.Tune(256, 16, 256, 16), pm.Tune(64, 4, 7, 1), pm.Tune(512, 32, 4096, 64),
                 pm.Tune(256, 16, 256, 16, 1), pm.Tune(128, 8, 64, 8, 64)):
        b = pm.run_batch(small_jobs, tune=tune)
        torch.cuda.synchronize()
        for k, (r, s) in enumerate(plains):
            assert torch.equal(b.results[k].fluence, r.fluence), (tune, k)
            assert torch.equal(b.results[k].scalars, r.scalars), (tune, k)
            bs = b.summary(k)
            for key in ("phi3d", "phi1d", "r", "R", "T", "A", "closure_exact"):
                a, c = bs[key], s[key]
                assert (a == c) or (np.isnan(a) and np.isnan(c)), (k, key)
            assert np.array_equal(bs.depth, s.depth, equal_nan=True)
    # every job staged in the line layout instead of the plane layout: the same bits
    for fp64 in (False, True):
        b = pm.run_batch(small_jobs, tune=pm.Tune(256, 16, 256, 16), fp64=fp64, line_staging=True)
        torch.cuda.synchronize()
        for k, j in enumerate(small_jobs):
            r = plains[k][0] if not fp64 else _plain(j, fp64=True)[0]
            assert torch.equal(b.results[k].fluence, r.fluence), ("lines", fp64, k)
            assert torch.equal(b.results[k].scalars, r.scalars), ("lines", fp64, k)


def test_batch_with_extreme_extents_equals_plain_runs():
    banner("batch of masks at the extent limit (65535 along one axis) == plain runs, bitwise")
    rng = np.random.default_rng(3)
    shapes = [(65535, 1, 1), (1, 1, 65535), (1, 65535, 2), (9, 10, 11)]
    jobs = []
    for i, sh in enumerate(shapes):
        m = torch.from_numpy((rng.random(sh) < 0.7).astype(np.uint8)).cuda()
        jobs.append(pm.BatchJob(m, pm.Optics(0.5, f32(0.01), f32(0.7)), 3000 + 100 * i, seed=20260809,
                                stream_id=i))
    b = pm.run_batch(jobs, tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        r, s = _plain(j)
        assert torch.equal(b.results[k].fluence, r.fluence), k
        assert torch.equal(b.results[k].scalars, r.scalars), k


def test_batch_fp64_equals_plain_fp64(small_jobs):
    banner("batch FP64 transport == plain FP64")
    b = pm.run_batch(small_jobs[:3], tune=pm.Tune(128, 8, 64, 8), fp64=True)
    for k in range(3):
        r, _ = _plain(small_jobs[k], fp64=True)
        assert torch.equal(b.results[k].fluence, r.fluence) and torch.equal(b.results[k].scalars, r.scalars)


def test_batch_accumulate_equals_whole(small_jobs):
    banner("batch resume: two halves accumulate to the whole")
    whole = pm.run_batch(small_jobs, tune=pm.Tune(256, 8, 128, 16))
    first = [pm.BatchJob(j.mask, j.optics, max(1, j.n_photons // 2), j.seed, j.stream_id, j.photon_begin, False)
             for j in small_jobs]
    second = [pm.BatchJob(j.mask, j.optics, j.n_photons - f.n_photons, j.seed, j.stream_id,
                          j.photon_begin + f.n_photons, False) for j, f in zip(small_jobs, first)]
    keep = [i for i, s in enumerate(second) if s.n_photons > 0]
    part = pm.run_batch(first, tune=pm.Tune(256, 8, 128, 16))
    sub = pm.Batch.__new__(pm.Batch)
    sub.results = [part.results[i] for i in keep]
    pm.run_batch([second[i] for i in keep], tune=pm.Tune(64, 16, 32, 4), accumulate_into=sub)
    torch.cuda.synchronize()
    for k in range(len(small_jobs)):
        assert torch.equal(part.results[k].fluence, whole.results[k].fluence), k
        assert torch.equal(part.results[k].scalars, whole.results[k].scalars), k


def test_graph_replays_match_eager(small_jobs):
    banner("captured graph: 3 replays with eager work between, each == eager")
    eager = pm.run_batch(small_jobs, tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    ref_f = [r.fluence.clone() for r in eager.results]
    ref_s = [r.scalars.clone() for r in eager.results]
    ref_q = [q.clone() for q in eager.summaries]
    g = pm.BatchGraph(small_jobs, tune=pm.Tune(256, 16, 256, 16))
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for k in range(len(small_jobs)):
            assert torch.equal(g.batch.results[k].fluence, ref_f[k]), (rep, k)
            assert torch.equal(g.batch.results[k].scalars, ref_s[k]), (rep, k)
            assert torch.equal(g.batch.summaries[k].nan_to_num(-1), ref_q[k].nan_to_num(-1)), (rep, k)
        # unrelated eager work in between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        pm.run(small_jobs[0].mask, small_jobs[0].optics, 1000, 1)
        torch.cuda.synchronize()
    g.close()


def test_autotune_returns_usable_shape(small_jobs, tmp_path, monkeypatch):
    banner("autotune + cache")
    monkeypatch.setenv("PHOTONMC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    t = pm.autotune_batch(small_jobs)
    assert t.block in (64, 128, 256, 512) and 1 <= t.waves_per_cu <= 32 and t.chunk >= 1 and 1 <= t.refill <= 64
    assert (tmp_path / "tune.txt").read_text().strip()
    b = pm.run_batch(small_jobs)          # tune=None: taken from the cache
    r, _ = _plain(small_jobs[2])
    torch.cuda.synchronize()
    assert torch.equal(b.results[2].fluence, r.fluence)


def test_oversize_job_takes_the_direct_path():
    """A job whose staging tally exceeds the log's 26-bit indices (here 512 x 512 x 258
    voxels) sends the whole batch through one atomic per voxel visit; every job must
    still equal its plain run (which logs) bit for bit."""
    banner("batch with a 512x512x258 job (direct deposits) == plain runs")
    g = torch.Generator(device="cuda").manual_seed(5)
    big = (torch.rand((258, 512, 512), generator=g, device="cuda") < 0.7).to(torch.uint8)
    small = torch.from_numpy(inputs.spinodal_mask(16, 16, 16, 8.0, 0.7, seed=3)).cuda()
    assert ((258 + 3) // 4) * 256 * 256 * 16 > 2 ** 26         # more staging words than a log index holds
    jobs = [pm.BatchJob(big, pm.Optics(f32(0.5), f32(0.01), f32(0.7)), 20000, seed=20260809, stream_id=0),
            pm.BatchJob(small, pm.Optics(f32(0.8), f32(0.02), f32(0.6)), 5000, seed=20260809, stream_id=1)]
    b = pm.run_batch(jobs, tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        r, _ = _plain(j)
        assert torch.equal(b.results[k].fluence, r.fluence), k
        assert torch.equal(b.results[k].scalars, r.scalars), k
    del b, big
    torch.cuda.empty_cache()


def test_batch_mixes_plane_and_line_layouts():
    """A job whose three plane tables exceed 192 MiB (384 x 384 x 360 voxels: 3 x 53 M words) but
    whose line-layout tally fits the log's 26-bit indices stages in lines, beside jobs staged in
    planes, in one logged launch; every job equals its plain run bit for bit."""
    banner("batch mixing a line-layout job (384x384x360) with plane-layout jobs == plain runs")
    g = torch.Generator(device="cuda").manual_seed(6)
    big = (torch.rand((360, 384, 384), generator=g, device="cuda") < 0.7).to(torch.uint8)
    assert 3 * 384 * 384 * 360 * 4 > 192 * 2 ** 20          # planes do not fit
    assert 192 * 192 * 90 * 16 <= 2 ** 26                    # lines fit a log index
    small = [torch.from_numpy(inputs.spinodal_mask(n, n + 3, n - 2, 8.0, 0.7, seed=7 + n)).cuda() for n in (17, 30)]
    jobs = [pm.BatchJob(small[0], pm.Optics(f32(0.8), f32(0.02), f32(0.6)), 6000, seed=20260809, stream_id=1),
            pm.BatchJob(big, pm.Optics(f32(0.5), f32(0.01), f32(0.7)), 20000, seed=20260809, stream_id=0),
            pm.BatchJob(small[1], pm.Optics(f32(0.4), f32(0.005), f32(0.9)), 9000, seed=20260809, stream_id=2)]
    b = pm.run_batch(jobs, tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        r, _ = _plain(j)
        assert torch.equal(b.results[k].fluence, r.fluence), k
        assert torch.equal(b.results[k].scalars, r.scalars), k
    del b, big
    torch.cuda.empty_cache()


# job 1 (5000 photons) bins paths of 4 voxels and more into its last bin; job 3 has one photon
ESC_BINS = [(1.5, 96), (0.25, 16), None, (0.5, 512), (3.0, 1), (1.5, 96)]


def _esc_jobs(small_jobs):
    """Five plain jobs of the small batch and one under the paper boundary model."""
    paper = pm.BatchJob(small_jobs[5].mask, pm.paper_optics(0.5, f32(0.01), f32(0.7), n_solid=f32(1.746),
                                                            lateral=pm.LATERAL_MIRROR, gate=400.0),
                        20000, seed=20260809, stream_id=9, photon_begin=11)
    return small_jobs[:5] + [paper]


@pytest.mark.parametrize("fp64", [False, True])
def test_batch_escape_histograms_equal_single_runs(small_jobs, fp64):
    """Each job's escape-path histogram kept by the batched walk equals that of
    mc_run_escape_histogram of the job alone, bin for bin, for several launch shapes;
    the tallies are those of mc_run_batch; a job without bins keeps none."""
    banner(f"batched escape-path histograms == single-run histograms (fp64={fp64})")
    jobs = _esc_jobs(small_jobs)
    base = pm.run_batch(jobs, tune=pm.Tune(256, 16, 256, 16), fp64=fp64)
    singles = {}
    for k, j in enumerate(jobs):
        if ESC_BINS[k] is not None:
            singles[k] = pm.run(j.mask, j.optics, j.n_photons, j.seed, photon_begin=j.photon_begin,
                                stream_id=j.stream_id, fp64=fp64, escape_bins=ESC_BINS[k])
    for tune in (pm.Tune(256, 16, 256, 16), pm.Tune(64, 4, 7, 1, 1), pm.Tune(512, 32, 4096, 64, 32)):
        b = pm.run_batch(jobs, tune=tune, fp64=fp64, escape_bins=ESC_BINS)
        torch.cuda.synchronize()
        for k in range(len(jobs)):
            r = b.results[k]
            assert torch.equal(r.fluence, base.results[k].fluence), (tune, k)
            assert torch.equal(r.scalars, base.results[k].scalars), (tune, k)
            if ESC_BINS[k] is None:
                assert r.escape_hist_w is None
                continue
            assert torch.equal(r.escape_hist_w, singles[k].escape_hist_w), (tune, k)
            assert torch.equal(r.escape_hist_n, singles[k].escape_hist_n), (tune, k)
            sc = r.scalar_dict()
            assert int(r.escape_hist_w.sum()) == sc["esc_w"] and int(r.escape_hist_n.sum()) == sc["esc_n"], k
    # the single-bin job holds every escape in its one bin; job 1 uses its overflow bin
    assert int(b.results[4].escape_hist_n[0]) == b.results[4].scalar_dict()["esc_n"] > 0
    assert int(b.results[1].escape_hist_n[-1]) > 0


def test_batch_escape_histogram_fp64_equals_oracle(small_jobs):
    """FP64 batch: a job's histogram equals the one the oracle's per-photon outcomes
    (fate, final Q31 weight, in-pore path) give, bin for bin."""
    banner("batched FP64 escape-path histogram == oracle per-photon outcomes, binned")
    jobs = _esc_jobs(small_jobs)
    b = pm.run_batch(jobs, tune=pm.Tune(256, 16, 256, 16), fp64=True, escape_bins=ESC_BINS)
    torch.cuda.synchronize()
    for k in (0, 1, 5):
        j = jobs[k]
        o = j.optics
        m = j.mask.cpu().numpy()
        ids = np.arange(j.photon_begin, j.photon_begin + j.n_photons, dtype=np.uint64)
        kw = dict(w_roulette=o.w_roulette, roulette_m=o.roulette_m, source=o.source, boundary=o.boundary,
                  lateral=o.lateral, n_solid=o.n_solid if o.n_solid else 1.0,
                  gate=o.gate if o.gate > 0 else float("inf"))
        _, summ = oracle.trace(m, o.mu_s, o.mu_a, o.g, ids, j.seed, max_rec=1, stream_id=j.stream_id, **kw)
        width, nbins = ESC_BINS[k]
        hw, hn, _, _ = oan.escape_path_histogram(summ["fate"], summ["w_final"], summ["path_void"], width, nbins)
        gw, gn = b.results[k].escape_hist_w.cpu().numpy(), b.results[k].escape_hist_n.cpu().numpy()
        # FP64 paths agree to ~1e-6 voxel after long walks; a path that close to a bin edge may bin either way
        q = summ["path_void"] / width
        esc = (summ["fate"] == 4) | (summ["fate"] == 5)
        near = int((esc & (np.abs(q - np.round(q)) < 1e-5) & (q > 0.5) & (q < nbins - 0.5)).sum())
        assert gn.sum() == hn.sum() and gw.sum() == hw.sum(), k
        assert np.abs(gn - hn).sum() <= 2 * near, (k, near)
        if near == 0:
            assert np.array_equal(gn, hn) and np.array_equal(gw, hw), k


def test_batch_escape_histograms_accumulate(small_jobs):
    """Two photon halves of a batch, the second accumulating, give the whole
    batch's histograms and tallies."""
    banner("batched escape-path histograms: two halves accumulate to the whole")
    jobs = _esc_jobs(small_jobs)
    whole = pm.run_batch(jobs, tune=pm.Tune(256, 8, 128, 16), escape_bins=ESC_BINS)
    first = [pm.BatchJob(j.mask, j.optics, max(1, j.n_photons // 2), j.seed, j.stream_id, j.photon_begin, False)
             for j in jobs]
    second = [pm.BatchJob(j.mask, j.optics, j.n_photons - f.n_photons, j.seed, j.stream_id,
                          j.photon_begin + f.n_photons, False) for j, f in zip(jobs, first)]
    keep = [i for i, s in enumerate(second) if s.n_photons > 0]
    part = pm.run_batch(first, tune=pm.Tune(256, 8, 128, 16), escape_bins=ESC_BINS)
    sub = pm.Batch.__new__(pm.Batch)
    sub.results = [part.results[i] for i in keep]
    pm.run_batch([second[i] for i in keep], tune=pm.Tune(64, 16, 32, 4), accumulate_into=sub,
                 escape_bins=[ESC_BINS[i] for i in keep])
    torch.cuda.synchronize()
    for k in range(len(jobs)):
        assert torch.equal(part.results[k].fluence, whole.results[k].fluence), k
        assert torch.equal(part.results[k].scalars, whole.results[k].scalars), k
        if ESC_BINS[k] is not None:
            assert torch.equal(part.results[k].escape_hist_w, whole.results[k].escape_hist_w), k
            assert torch.equal(part.results[k].escape_hist_n, whole.results[k].escape_hist_n), k
