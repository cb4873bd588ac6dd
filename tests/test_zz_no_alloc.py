"""mc_run_noalloc, the entry point for callers that cannot allocate device memory,
through the C ABI against mc_run on the same arguments: two calls in a row, the
second with a smaller input (the fixed scratch keeps the first call's contents),
FP64 transport, a split run accumulated, the largest volume the scratch holds, and
the host-side refusal of larger volumes and of MC_TIMED before any device work."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from paper_2604_13929_amd import inputs
from paper_2604_13929_amd import photonmc as pm

pytestmark = pytest.mark.gpu
SEED = 20260809
f32 = lambda x: float(np.float32(x))  # noqa: E731
OPT = pm.Optics(0.5, f32(0.01), f32(0.7))


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pm.load()


def _same(a: pm.RunResult, b: pm.RunResult):
    torch.cuda.synchronize()
    return torch.equal(a.fluence, b.fluence) and torch.equal(a.scalars, b.scalars)


def test_noalloc_equals_mc_run_on_consecutive_calls():
    banner("mc_run_noalloc == mc_run: a 48x40x36 run, then a smaller 16x12x10 run")
    big = torch.from_numpy(inputs.spinodal_mask(48, 40, 36, 8.0, 0.7, seed=21)).cuda()
    small = torch.from_numpy(inputs.spinodal_mask(16, 12, 10, 6.0, 0.6, seed=22)).cuda()
    a = pm.run_noalloc(big, OPT, 60_000, SEED, photon_begin=11, stream_id=5)
    assert _same(a, pm.run(big, OPT, 60_000, SEED, photon_begin=11, stream_id=5))
    b = pm.run_noalloc(small, pm.Optics(f32(0.9), f32(0.03), f32(0.6)), 7_000, SEED, stream_id=2)
    assert _same(b, pm.run(small, pm.Optics(f32(0.9), f32(0.03), f32(0.6)), 7_000, SEED, stream_id=2))
    assert int(b.scalars[pm.SCALARS.index("launched")].item()) == 7_000


def test_noalloc_fp64_and_accumulate():
    banner("mc_run_noalloc: FP64 transport, and a split run accumulated == the whole")
    m = torch.from_numpy(inputs.spinodal_mask(24, 24, 24, 8.0, 0.7, seed=23)).cuda()
    assert _same(pm.run_noalloc(m, OPT, 20_000, SEED, fp64=True), pm.run(m, OPT, 20_000, SEED, fp64=True))
    part = pm.run_noalloc(m, OPT, 8_000, SEED)
    pm.run_noalloc(m, OPT, 12_000, SEED, photon_begin=8_000, accumulate=part)
    assert _same(part, pm.run(m, OPT, 20_000, SEED))


def test_noalloc_at_the_scratch_limit():
    L = pm.load()
    assert L.mc_run_noalloc_max_bricks() == 2 ** 21
    banner("mc_run_noalloc at 2^21 bricks (512^3 voxels) == mc_run")
    g = torch.Generator(device="cuda").manual_seed(7)
    m = (torch.rand((512, 512, 512), generator=g, device="cuda") < 0.7).to(torch.uint8)
    a = pm.run_noalloc(m, OPT, 3_000, SEED)
    r = pm.run(m, OPT, 3_000, SEED)
    assert _same(a, r)
    del a, r, m
    torch.cuda.empty_cache()


def test_noalloc_refuses_before_any_device_work():
    banner("mc_run_noalloc refuses an oversize volume and MC_TIMED on the host")
    L = pm.load()
    opt = OPT.c()
    dummy = ctypes.c_void_p(16)           # never dereferenced: the call returns before any launch
    for nx, ny, nz, flags, rc_want, needle in ((516, 512, 512, 0, -4, b"scratch"),
                                               (8, 8, 8, pm.MC_TIMED, -1, b"MC_TIMED")):
        vol = pm.McVolume(nx, ny, nz, 0, dummy.value)
        rc = L.mc_run_noalloc(ctypes.byref(vol), ctypes.byref(opt), 0, 10, SEED, 0, flags, dummy, dummy, None, None)
        assert rc == rc_want and needle in L.mc_last_error(), (rc, L.mc_last_error())
