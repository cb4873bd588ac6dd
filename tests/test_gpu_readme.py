"""The README's quick start runs as written (with fewer photons), and the other
entry points it lists are callable with the arguments it shows."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_quick_start_runs_as_written():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu] README quick start", flush=True)
    text = open(os.path.join(ROOT, "README.md")).read()
    code = re.search(r"## Quick start \(Python\)\s+```python\n(.*?)```", text, flags=re.S).group(1)
    code = code.replace("n_photons=10**8", "n_photons=10**6")
    assert "n_photons=10**6" in code
    ns: dict = {}
    exec(compile(code, "README quick start", "exec"), ns)
    s, res = ns["s"], ns["res"]
    assert s["closure_exact"] == 1.0 and res.scalar_dict()["launched"] == 10 ** 6
    assert 0.0 < s["phi3d"] and np.isfinite(s["r"])


def test_listed_entry_points_exist():
    """(CPU) every Python entry point the README's table names exists."""
    from paper_2604_13929_amd import analytics, photonmc, spinodal
    text = open(os.path.join(ROOT, "README.md")).read()
    table = text[text.index("| Module | Entry points |"):text.index("## C ABI")]
    mods = {"photonmc": photonmc, "spinodal": spinodal, "analytics": analytics}
    for line in table.splitlines()[2:]:
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) != 2 or cells[0].strip("`") not in mods:
            continue
        mod = mods[cells[0].strip("`")]
        for name in re.findall(r"`([A-Za-z_][A-Za-z0-9_]*)(?:\(|`)", cells[1]):
            assert hasattr(mod, name), (cells[0], name)
