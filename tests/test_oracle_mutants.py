"""Mutation tests of the oracle's pins: copies of the oracle with one planted,
plausible mistake each (a sign, a dropped term, a wrong index, constant or tie rule)
must fail the CPU pin suites.  The C walk is rebuilt with gcc and loaded through
ORACLE_LIB; the Python parts (Cahn-Hilliard, analytics) run from a mutated copy of
the oracle package placed ahead of the repository on the import path.  The real
oracle is never modified; the copies live in a temporary directory.

A mutant that no pin catches would show that a mistake of that kind could hide in
the oracle; every mutant listed here is caught."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
SUITES = ["tests/test_oracle_dda.py", "tests/test_oracle_pins.py", "tests/test_oracle_boundary.py",
          "tests/test_estimators_inputs.py"]

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("hg_backward", "ct = (1.0 + g * g - t * t) / (2.0 * g);", "ct = -(1.0 + g * g - t * t) / (2.0 * g);"),
    ("survival_uses_mu_a", "S_q = (uint64_t)llround(P->mu_s / mu_t_solid * 4294967296.0);",
     "S_q = (uint64_t)llround(P->mu_a / mu_t_solid * 4294967296.0);"),
    ("no_pore_deposit", "if (S->fluence) S->fluence[v] += (double)w * d;",
     "if (S->fluence && solid) S->fluence[v] += (double)w * d;"),
    ("roulette_biased", "const uint32_t T_m = (uint32_t)llround(16777216.0 / (double)P->roulette_m);",
     "const uint32_t T_m = (uint32_t)llround(16777216.0 / (double)(P->roulette_m + 1));"),
    ("rotation_sign", "nuy = stt * (uy * uz * cp + ux * sp) / tn + uy * ct;",
     "nuy = stt * (uy * uz * cp - ux * sp) / tn + uy * ct;"),
    ("wrap_off_by_one", "if (st->ix == nx) st->ix = 0;", "if (st->ix == nx) st->ix = 1;"),
    ("face_tie_to_later_axis", "if (dist[1] < dist[axis]) axis = 1;", "if (dist[1] <= dist[axis]) axis = 1;"),
    ("interaction_tie_to_face", "int interact = (s_int <= d_face);", "int interact = (s_int < d_face);"),
    ("free_path_halved", "            st->tau = -log(u_open_closed(r[2]));\n        }",
     "            st->tau = -0.5 * log(u_open_closed(r[2]));\n        }"),
    ("absorb_rounds_down", "const int64_t w_new = (int64_t)(((uint64_t)st->w * S_q + 2147483648ull) >> 32);",
     "const int64_t w_new = (int64_t)(((uint64_t)st->w * S_q) >> 32) + 1;"),
    ("depth_phase_swapped", "if (S->depth) S->depth[(solid ? 0 : 1) * nz + st->iz] += (double)w * d;",
     "if (S->depth) S->depth[(solid ? 1 : 0) * nz + st->iz] += (double)w * d;"),
    ("solid_path_not_counted", "            st->l_solid += d;\n", "            st->l_solid += 0.0 * d;\n"),
    # the paper's boundary model
    ("fresnel_p_uses_cos_i", "const double rp = (n1 * ct - n2 * cos_i) / (n1 * ct + n2 * cos_i);",
     "const double rp = (n1 * cos_i - n2 * ct) / (n1 * cos_i + n2 * ct);"),
    ("fresnel_s_only", "return 0.5 * (rs * rs + rp * rp);", "return rs * rs;"),
    ("snell_eta_inverted", "const double eta = n_here / n_next;", "const double eta = n_next / n_here;"),
    ("tir_never", "if (sin_t2 >= 1.0) {", "if (sin_t2 > 1.0e300) {"),
    ("mirror_keeps_sign", "            uu[axis] = -uu[axis];\n", "            uu[axis] = uu[axis];\n"),
    ("gate_ignores_index", "if (st->l_opt + n_here * d > P->gate) {", "if (st->l_opt + d > P->gate) {"),
    ("pads_thick", "} else if (j[2] < -1 || j[2] > nz) {", "} else if (j[2] < -2 || j[2] > nz + 1) {"),
    ("fresnel_choice_reversed", "                    if (U < R) {", "                    if (U >= R) {"),
]


# (name, file under oracle/, text, replacement, pin suites)
CH = ["tests/test_oracle_ch.py"]
AN = ["tests/test_oracle_analytics.py"]
ES = ["tests/test_estimators_inputs.py"]
PY_MUTANTS = [
    ("f_prime_sign", "cahn_hilliard.py", "return 2.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi)",
     "return 2.0 * phi * (1.0 - phi) * (2.0 * phi - 1.0)", CH),
    ("semi_implicit_k2", "cahn_hilliard.py", "denom = 1.0 + dt * kappa * k2 * k2", "denom = 1.0 + dt * kappa * k2", CH),
    ("kappa_cal_factor", "cahn_hilliard.py", "(d_target_voxels / (8.0 * math.pi)) ** 2",
     "(d_target_voxels / (4.0 * math.pi)) ** 2", CH),
    ("psd_weight_x0", "cahn_hilliard.py", "weight[:, :, 0] = 1.0", "weight[:, :, 0] = 2.0", CH),
    ("psd_shell_floor", "cahn_hilliard.py", "nmax / (2.0 * math.pi) + 0.5).astype", "nmax / (2.0 * math.pi)).astype", CH),
    ("dominant_size_wavelength", "cahn_hilliard.py", "return max(shape) / (2.0 * s)", "return max(shape) / s", CH),
    ("rank_ties_upper", "cahn_hilliard.py", 'order = np.argsort(-flat, kind="stable")',
     'order = (flat.size - 1) - np.argsort(-flat[::-1], kind="stable")', CH),
    ("chord_face_dropped", "analytics.py", "if i == n or line[i] != line[start]:",
     "if i < n and line[i] != line[start]:", AN),
    ("plen_threshold_ge", "analytics.py", "(lengths * n)[lengths > t]", "(lengths * n)[lengths >= t]", AN),
    ("contrast_sd_population", "analytics.py", "cs.std(ddof=1) if cs.size > 1", "cs.std(ddof=0) if cs.size > 1", AN),
    ("escape_bin_round", "analytics.py", "np.floor(pv / bin_width)", "np.round(pv / bin_width)", AN),
    ("decile_k_floor", "analytics.py", "k = int(math.ceil(frac * f.size))", "k = int(frac * f.size)", AN),
    ("decile_ties_upper", "analytics.py", 'top = np.argsort(rev, kind="stable")[:k]',
     'top = ((f.size - 1) - np.argsort(rev[::-1], kind="stable"))[:k]', AN),
    ("spearman_is_pearson", "analytics.py", "stats.spearmanr(f, d).statistic", "stats.pearsonr(f, d).statistic", AN),
    ("mask_psd_of_complement_mean", "analytics.py", "m = np.asarray(mask, dtype=np.float64)",
     "m = np.asarray(mask, dtype=np.float64) * 2.0", AN),
    ("front_back_second_layer", "estimators.py", 'out["front_back"] = depth[0] / depth[-1]',
     'out["front_back"] = depth[1] / depth[-1]', ES),
    ("front_back_penultimate_layer", "estimators.py", 'out["front_back"] = depth[0] / depth[-1]',
     'out["front_back"] = depth[0] / depth[-2]', ES),
    ("l_opt_lateral_axis", "estimators.py", 'out["L_opt"] = out["phi1d"] * nz', 'out["L_opt"] = out["phi1d"] * nx', ES),
    ("rms_log_unsquared", "estimators.py", "np.log(p[ok] / q[ok]) ** 2", "np.abs(np.log(p[ok] / q[ok]))", ES),
    ("rms_depths_keep_zero_reference", "estimators.py", "ok = np.isfinite(q) & (q > 0) & np.isfinite(p)",
     "ok = np.isfinite(q) & (q >= 0) & np.isfinite(p)", ES),
    ("rms_w_unweighted", "estimators.py", "np.sqrt((q * (p - q) ** 2 / q ** 2).sum() / q.sum())",
     "np.sqrt(((p - q) ** 2 / q ** 2).mean())", ES),
]


def _run_c_mutant(name, old, new, source, workdir):
    assert source.count(old) == 1, f"mutation site of {name} not found once in oracle.c"
    src = os.path.join(workdir, "oracle_mutant.c")
    with open(src, "w") as f:
        f.write(source.replace(old, new))
    lib = os.path.join(workdir, "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                           src, "-o", lib, "-lm"])
    env = dict(os.environ, ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", *SUITES, "-x", "-q", "-m", "not gpu",
                           "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def _run_py_mutant(name, fname, old, new, suites, workdir):
    pkg = os.path.join(workdir, "oracle")
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("__pycache__"))
    path = os.path.join(pkg, fname)
    with open(path) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site of {name} not found once in oracle/{fname}"
    with open(path, "w") as f:
        f.write(text.replace(old, new))
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([workdir, ROOT]))
    env.pop("ORACLE_LIB", None)
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"], cwd=workdir, env=env,
                           capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().startswith(pkg), probe.stdout + probe.stderr
    return subprocess.run([sys.executable, "-m", "pytest", *[os.path.join(ROOT, t) for t in suites], "-x", "-q",
                           "-m", "not gpu", "-p", "no:cacheprovider", "--rootdir", ROOT], cwd=workdir, env=env,
                          capture_output=True, text=True, timeout=900)


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every mutant built and run against its pin suites, four at a time."""
    with open(SRC) as f:
        source = f.read()
    jobs = {}
    with ThreadPoolExecutor(max_workers=4) as pool:
        for name, old, new in MUTANTS:
            d = str(tmp_path_factory.mktemp(name))
            jobs[name] = pool.submit(_run_c_mutant, name, old, new, source, d)
        for name, fname, old, new, suites in PY_MUTANTS:
            d = str(tmp_path_factory.mktemp(name))
            jobs[name] = pool.submit(_run_py_mutant, name, fname, old, new, suites, d)
        return {name: fut.result() for name, fut in jobs.items()}


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS] + [m[0] for m in PY_MUTANTS])
def test_mutant_is_caught(name, outcomes):
    r = outcomes[name]
    assert r.returncode == 1, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
