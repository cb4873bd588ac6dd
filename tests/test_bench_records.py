"""bench.py's host-side helpers, without a GPU: the roofs it derives from the committed
counter records, the guard that drops a record whose kernel sources changed, the check of
every oracle comparison against the stated tolerances, and the paper's context ratios."""
from __future__ import annotations

import json
import math

import pytest

import bench


def _record(path):
    with open(path) as fh:
        return json.load(fh)


def test_plain_roofs_reproduce_the_record():
    """At the record's own launch (its photons, steps and kernel time) the derived roofs are
    the record's: requests per step, the request rate against the ceiling, the VALU
    instructions per step and a VALU busy fraction within (0, 1]."""
    rec = _record(bench.TRAFFIC_RECORD)
    traffic, atomic, valu = bench.plain_roofs(rec, rec["photons"], rec["photon_steps"], rec["kernel_trace_avg_ms"])
    assert traffic == pytest.approx(rec["traffic_bytes_per_launch"])
    assert atomic["requests_per_step"] == pytest.approx(rec["atomic_requests_per_launch"] / rec["photon_steps"])
    rate = rec["atomic_requests_per_launch"] / (rec["kernel_trace_avg_ms"] * 1e-3)
    assert atomic["frac"] == pytest.approx(rate / rec["request_ceiling_per_s"])
    assert 0.5 < atomic["frac"] <= 1.05
    assert valu["instructions_per_step"] == pytest.approx(rec["valu"]["SQ_INSTS_VALU"] / rec["photon_steps"])
    assert 0.0 < valu["frac"] <= 1.5
    # the clock the GRBM cycles imply is the chip's (about 2.4 GHz)
    assert 1.5e9 < valu["clock_hz"] < 3.0e9
    assert valu["roof_photon_steps_per_s"] * valu["frac"] == pytest.approx(valu["achieved_photon_steps_per_s"])


def test_plain_roofs_scale_with_the_launch():
    """Half the photons in half the time: the same rates, half the requests and bytes."""
    rec = _record(bench.TRAFFIC_RECORD)
    full = bench.plain_roofs(rec, rec["photons"], rec["photon_steps"], 1000.0)
    half = bench.plain_roofs(rec, rec["photons"] // 2, rec["photon_steps"] / 2, 500.0)
    assert half[0] == pytest.approx(full[0] / 2)
    assert half[1]["requests_per_launch"] == pytest.approx(full[1]["requests_per_launch"] / 2)
    assert half[1]["frac"] == pytest.approx(full[1]["frac"])
    assert half[2]["frac"] == pytest.approx(full[2]["frac"])


def test_records_are_dropped_when_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "source_sha256", lambda: "0" * 64)
    assert bench.recorded_traffic(10 ** 8) is None
    roof = bench.walk_roofline("batched", 10 ** 11, 2000.0)
    assert roof["atomic_request_roof"] is None
    assert roof["achieved"] == pytest.approx(10 ** 11 * bench.BYTES_PER_STEP / 2.0 / 1e9)


def test_walk_roofline_from_the_matching_record(monkeypatch):
    rec = _record(bench.FORMS_RECORD)
    monkeypatch.setattr(bench, "source_sha256", lambda: rec["source_sha256"])
    r = rec["batched"]
    roof = bench.walk_roofline("batched", r["photon_steps"], r["pmc_launch_ms"]["atomic"])
    a = roof["atomic_request_roof"]
    assert a["requests_per_step"] == pytest.approx(r["atomic_requests_per_launch"] / r["photon_steps"])
    assert a["frac"] == pytest.approx(r["atomic_requests_per_launch"] / (r["pmc_launch_ms"]["atomic"] * 1e-3)
                                      / rec["request_ceiling_per_s"])
    assert roof["traffic"] == pytest.approx(r["traffic_bytes_per_launch"])


def test_oracle_tolerance_failures():
    good = {"oracle_error": {"phi3d": 1e-5, "R": 2e-5, "steps": 5e-4},
            "rows": {"M1": {"oracle": {"relative_error": {"phi3d": 1e-4, "steps": 1.5e-3}}}},
            "batched": {"oracle": {"job1": {"relative_error": {"A": 4e-3}}}},
            "morphology_control": {"oracle": {"M3": {"relative_error": {"r": 1e-5, "steps": 1e-3}}}}}
    assert bench.oracle_tolerance_failures(good) == []
    bad = json.loads(json.dumps(good))
    bad["oracle_error"]["steps"] = 2e-3                     # the plain workload's steps bound is 0.1 %
    bad["rows"]["M1"]["oracle"]["relative_error"]["phi3d"] = 6e-3
    bad["morphology_control"]["oracle"]["M3"]["relative_error"]["r"] = math.nan
    fails = bench.oracle_tolerance_failures(bad)
    assert len(fails) == 3
    assert any(f.startswith("plain.steps") for f in fails)
    assert any(f.startswith("M1.phi3d") for f in fails)
    assert any(f.startswith("morphology_M3.r") for f in fails)


def test_paper_context_reports_both_sides():
    line = {"results": {"ratio": 0.96}, "rows": {"M2b_256cube_phi090": {"phi3d": 1.3, "phi1d": 1.4}},
            "paper_boundary": {"paper_optics": {"ratio": 1.48}}}
    c = bench.paper_context(line)["ratio_phi3d_over_phi1d"]
    assert (c["paper_phi070"], c["paper_phi090"]) == (1.515, 1.774)
    assert c["this_run"] == {"plain_model_phi070": 0.96, "plain_model_phi090": pytest.approx(1.3 / 1.4),
                             "paper_model_paper_optics_phi070": 1.48}
    assert bench.paper_context({"results": {"ratio": 1.0}})["ratio_phi3d_over_phi1d"]["this_run"] == \
        {"plain_model_phi070": 1.0}
