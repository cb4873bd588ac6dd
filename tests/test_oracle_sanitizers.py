"""The oracle under the host sanitizers: its C source, compiled with gcc together with a
small driver into stand-alone executables built with AddressSanitizer + UndefinedBehavior-
Sanitizer (no recovery) and with ThreadSanitizer, runs both boundary models, the test
source, the caps and the degenerate optics through orc_run (several threads and batches,
with fluence, gradient and depth outputs), orc_trace and a photon stepped by orc_step to its end without a report, and
every run closes its energy balance exactly.  Host code only: nothing here touches a GPU."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

DRIVER = r"""
#include "oracle.c"
#include <stdio.h>

enum { NX = 12, NY = 10, NZ = 14, NB = 2 };
static uint8_t mask[NZ][NY][NX];

static int run_and_close(const orc_problem *P, uint64_t begin, uint64_t n, int nthreads, const char *what)
{
    double *F = calloc((size_t)NB * NX * NY * NZ, sizeof(double));
    double *G = calloc((size_t)NB * 6 * NZ, sizeof(double));
    double *D = calloc((size_t)NB * 2 * NZ, sizeof(double));
    int64_t ich[NB][ORC_NI];
    double dch[NB][ORC_ND];
    memset(ich, 0, sizeof ich);
    memset(dch, 0, sizeof dch);
    if (!F || !G || !D) return 1;
    if (orc_run(P, begin, n, nthreads, NB, F, G, D, &ich[0][0], &dch[0][0]) != 0) {
        fprintf(stderr, "%s: orc_run refused the problem\n", what);
        return 1;
    }
    int64_t sum = 0;
    for (int b = 0; b < NB; ++b)
        sum += ich[b][ORC_R] + ich[b][ORC_T] + ich[b][ORC_A] + ich[b][ORC_RR] + ich[b][ORC_LOST] + ich[b][ORC_GATED];
    free(F);
    free(G);
    free(D);
    if (sum != (int64_t)n * (int64_t)2147483648LL) {
        fprintf(stderr, "%s: closure %lld != %llu * 2^31\n", what, (long long)sum, (unsigned long long)n);
        return 1;
    }
    return 0;
}

int main(void)
{
    for (int z = 0; z < NZ; ++z)
        for (int y = 0; y < NY; ++y)
            for (int x = 0; x < NX; ++x) mask[z][y][x] = (uint8_t)(((x * 7 + y * 5 + z * 3) % 10) < 6);
    orc_problem P;
    memset(&P, 0, sizeof P);
    P.nx = NX; P.ny = NY; P.nz = NZ; P.mask = &mask[0][0][0];
    P.mu_s = 0.5; P.mu_a = 0.01; P.g = 0.7; P.w_roulette = 1e-4; P.roulette_m = 10;
    P.path_cap = 0.0; P.source = 0; P.seed = 20260809ull; P.stream_id = 3; P.max_steps = 1u << 24;
    P.boundary = 0; P.lateral = 0; P.n_solid = 1.0; P.gate = INFINITY;
    int bad = 0;
    bad |= run_and_close(&P, 5, 3000, 4, "plain");
    orc_problem L = P; L.source = 1;
    bad |= run_and_close(&L, 0, 1000, 3, "lambertian");
    orc_problem C = P; C.path_cap = 7.5; C.max_steps = 40;
    bad |= run_and_close(&C, 0, 1000, 2, "caps");
    orc_problem A = P; A.mu_s = 0.0;
    bad |= run_and_close(&A, 0, 1000, 2, "pure absorber");
    orc_problem S = P; S.mu_a = 0.0; S.g = 0.0;
    bad |= run_and_close(&S, 0, 1000, 2, "no absorption");
    orc_problem Q = P; Q.boundary = 1; Q.lateral = 1; Q.n_solid = 1.746; Q.gate = 300.0;
    bad |= run_and_close(&Q, 11, 2000, 4, "paper model, mirrors");
    Q.lateral = 0; Q.gate = INFINITY;
    bad |= run_and_close(&Q, 0, 1000, 2, "paper model, periodic");

    uint64_t ids[6] = {0, 1, 7, 123, 4567, 99999};
    orc_rec *recs = calloc(6 * 64, sizeof(orc_rec));
    orc_photon summ[6];
    if (!recs || orc_trace(&P, ids, 6, 64, recs, summ) != 0 || orc_trace(&Q, ids, 6, 64, recs, summ) != 0) bad = 1;
    free(recs);
    orc_state st;
    double gap = 0.0;
    launch(&Q, 5, &st);
    for (int i = 0; i < 200; ++i) {
        const int ev = orc_step(&Q, 5, &st, &gap);
        if (ev < 0) { bad = 1; break; }
        if (terminal(ev)) break;
    }
    double ct = 0.0;
    (void)orc_fresnel(1.746, 1.0, 0.3, &ct);
    (void)orc_fresnel(1.0, 1.746, 0.99, &ct);
    if (!bad) printf("oracle under sanitizers: ok\n");
    return bad;
}
"""


def _build_and_run(tmp_path, name, flags):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc is not available")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / name
    cmd = [cc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", *flags, f"-I{ORACLE_DIR}", str(src), "-lm",
           "-lpthread", "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle under sanitizers: ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    _build_and_run(tmp_path, "oracle_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])


def test_oracle_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, "oracle_tsan", ["-fsanitize=thread"])
