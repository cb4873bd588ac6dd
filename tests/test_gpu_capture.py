"""The plain path under HIP stream capture: mc_run + mc_reduce (and mc_run_noalloc)
recorded into one graph by torch's capture, replayed three times with unrelated eager
work and synchronisations in between; every replay equals the eager run bit for bit
(tallies, summary, depth profiles).  The path clears its tallies and counters with
fill kernels, so the graph holds no memset node."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2604_13929_amd import photonmc as pm

pytestmark = pytest.mark.gpu
SEED = 20260809
OPT = pm.Optics(0.5, float(np.float32(0.01)), float(np.float32(0.7)))
N = 200_000


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pm.load()


def banner(msg):
    print(f"[gpu] {msg}", flush=True)


def _unrelated_eager_work(d):
    x = torch.randn(1 << 20, device="cuda")
    (x * 2).sum().item()
    pm.run(d, OPT, 1000, 1)
    torch.cuda.synchronize()


@pytest.mark.parametrize("noalloc", [False, True])
def test_run_and_reduce_replay_from_a_graph(mask_m1, noalloc):
    banner(f"mc_run{'_noalloc' if noalloc else ''} + mc_reduce captured into a graph, 3 replays == eager")
    d = torch.from_numpy(mask_m1).cuda()
    run = pm.run_noalloc if noalloc else pm.run
    eager = run(d, OPT, N, SEED)
    q_e, dep_e, _ = pm.reduce_async(d, eager)
    torch.cuda.synchronize()
    ref = (eager.fluence.clone(), eager.scalars.clone(), q_e.clone(), dep_e.clone())

    # warm the binding's allocations on a side stream, as torch's capture asks
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        warm = run(d, OPT, N, SEED)
        pm.reduce_async(d, warm)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = run(d, OPT, N, SEED)
        q, dep, ws = pm.reduce_async(d, res)
    torch.cuda.synchronize()
    for rep in range(3):
        res.fluence.fill_(-1)          # the replay must clear the tallies itself
        res.scalars.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res.fluence, ref[0]), rep
        assert torch.equal(res.scalars, ref[1]), rep
        assert torch.equal(q.nan_to_num(-7.0), ref[2].nan_to_num(-7.0)), rep
        assert torch.equal(dep.nan_to_num(-7.0), ref[3].nan_to_num(-7.0)), rep
        _unrelated_eager_work(d)
    del g, ws
