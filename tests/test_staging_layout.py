"""The staging tally's two layouts, on the host: the device header's index functions,
compiled by hipcc into a host program (no GPU), map every voxel of several ragged
volumes to a word of its own, inside its table, and back to the same voxel; the 16
words of a line are one 4 x 4 plane one voxel thin (plane layout) or one 2 x 2 x 4
block (line layout); the tables are whole lines.  A deposit may go to any table, so
these properties are what makes the staged totals exact."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_13929_amd", "csrc")

PROGRAM = r"""
#include "walk.hpp"
#include <cstdio>
#include <cstdlib>
#include <vector>
using namespace pmc;

static int check(int nx, int ny, int nz)
{
    Job J = {};
    J.nx = nx; J.ny = ny; J.nz = nz;
    J.lnx = (nx + 1) / 2; J.lny = (ny + 1) / 2;
    const int lnz = (nz + 3) / 4;
    const PlaneDims P = plane_dims(nx, ny, nz);
    J.stage_off1 = P.off1; J.stage_off2 = P.off2;   // as the host fills a job
    if (P.words % 16 || P.off1 % 16 || P.off2 % 16) { printf("tables not whole lines\n"); return 1; }
    const uint64_t first[4] = {0, P.off1, P.off2, P.words};
    // plane layout
    J.stage_planes = 1;
    std::vector<int64_t> owner(P.words, -1);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint64_t v = ((uint64_t)z * ny + y) * nx + x;
                for (uint32_t t = 0; t < 3; ++t) {
                    const uint32_t i = plane_index(P, nx, ny, t, x, y, z);
                    if (i < first[t] || i >= first[t + 1]) { printf("plane %u: word %u outside its table\n", t, i); return 1; }
                    if (owner[i] != -1) { printf("plane %u: word %u shared\n", t, i); return 1; }
                    owner[i] = (int64_t)v;
                    if (stage_voxel(J, i) != v) { printf("plane %u: word %u maps back to another voxel\n", t, i); return 1; }
                    // the line's 16 words: one voxel thin across axis t, a 4 x 4 group in the others
                    const uint32_t base = i & ~15u;
                    for (uint32_t k = 0; k < 16; ++k) {
                        const uint32_t j = base + k;
                        const int64_t w = owner[j];
                        if (w < 0) continue;
                        const int wx = (int)(w % nx), wy = (int)((w / nx) % ny), wz = (int)(w / ((int64_t)nx * ny));
                        const int c[3] = {x, y, z}, d[3] = {wx, wy, wz};
                        for (int a = 0; a < 3; ++a) {
                            const bool ok = a == (int)t ? c[a] == d[a] : c[a] / 4 == d[a] / 4;
                            if (!ok) { printf("plane %u: line %u mixes voxels\n", t, base >> 4); return 1; }
                        }
                    }
                }
            }
    // line layout
    J.stage_planes = 0;
    const uint64_t words = (uint64_t)J.lnx * J.lny * lnz * 16;
    std::vector<int64_t> own2(words, -1);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint64_t v = ((uint64_t)z * ny + y) * nx + x;
                const uint32_t i = stage_index(J.lnx, J.lny, x, y, z);
                if (i >= words || own2[i] != -1) { printf("line layout: word %u outside or shared\n", i); return 1; }
                own2[i] = (int64_t)v;
                if (stage_voxel(J, i) != v) { printf("line layout: word %u maps back to another voxel\n", i); return 1; }
                const uint32_t line = i >> 4;
                const uint32_t want = ((uint32_t)(z / 4) * J.lny + y / 2) * J.lnx + x / 2;
                if (line != want) { printf("line layout: voxel in line %u, expected %u\n", line, want); return 1; }
            }
    return 0;
}

int main()
{
    const int shapes[][3] = {{1, 1, 1}, {1, 1, 9}, {5, 7, 9}, {13, 4, 6}, {16, 16, 16}, {33, 17, 9}, {3, 40, 2}, {64, 3, 21}};
    for (const auto &s : shapes)
        if (check(s[0], s[1], s[2])) { printf("in volume %d x %d x %d\n", s[0], s[1], s[2]); return 1; }
    // the table sizes of the 256^3 workload: three tables of 2^24 words (192 MiB), the line layout 2^24
    const PlaneDims P = plane_dims(256, 256, 256);
    if (P.words != 3ull << 24 || P.off1 != 1u << 24 || P.off2 != 2u << 24) { printf("256^3 tables\n"); return 1; }
    printf("staging layouts: ok\n");
    return 0;
}
"""


def test_staging_layouts_are_exact_maps(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not available")
    src = tmp_path / "layout.hip"
    src.write_text(PROGRAM)
    exe = tmp_path / "layout"
    build = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", f"-I{CSRC}",
                            f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)],
                           capture_output=True, text=True, timeout=600)
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "staging layouts: ok" in run.stdout
