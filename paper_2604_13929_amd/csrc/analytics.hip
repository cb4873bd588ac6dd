// analytics.hip -- morphology and fluence analytics of Sec. 3.4: chord-length
// histograms, depth-normalised phase contrast, escape-path histograms, the
// brightest-decile co-localisation per slice, and the exact Euclidean distance
// transform of the pore phase.
//
// These are scans over the mask, the fluence tally or per-photon records, so they
// are bound by memory traffic or launch count, not arithmetic: one thread per line
// for the line scans (lines laid out so that neighbouring threads read
// neighbouring bytes), global 64-bit atomics for the histograms, the shared radix
// select for the per-slice deciles, and the separable distance transform of
// Felzenszwalb & Huttenlocher (2012): a two-sided scan along x, then the lower
// envelope of parabolas along y and along z.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "analytics.h"
#include "internal.hpp"
#include "select.hpp"

using namespace pmc::host;

namespace {

constexpr int kThreads = 256;
constexpr int kInf = 0x3fffffff;          // "no solid voxel on this line yet" for squared distances
constexpr long long kEdtChunk = 65536;    // lines per launch of an envelope pass

__global__ void k_zero_i64(long long *p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// line l of axis a: element j at base + j * stride
struct LineGeo {
    int n;            // length
    long long lines;  // number of lines
};

__device__ __forceinline__ size_t line_elem(int axis, long long l, int j, int nx, int ny)
{
    if (axis == 2) return (size_t)j * nx * ny + (size_t)l;                         // l = y * nx + x
    if (axis == 1) {                                                               // l = z * nx + x
        const long long z = l / nx, x = l - z * nx;
        return ((size_t)z * ny + j) * nx + (size_t)x;
    }
    return (size_t)l * nx + j;                                                     // l = z * ny + y
}

__global__ void k_chords(const uint8_t *__restrict__ mask, int axis, int n, long long lines, int nx, int ny,
                         unsigned long long *hist)
{
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= lines) return;
    int start = 0;
    uint8_t cur = mask[line_elem(axis, l, 0, nx, ny)];
    for (int j = 1; j <= n; ++j) {
        const uint8_t v = j < n ? mask[line_elem(axis, l, j, nx, ny)] : (uint8_t)(cur ^ 1u);
        if (v != cur) {
            atomicAdd(&hist[(size_t)(cur ? 1 : 0) * (n + 1) + (j - start)], 1ull);
            start = j;
            cur = v;
        }
    }
}

// one thread: fixed order, exact sample variance by two passes
__global__ void k_contrast(const double *__restrict__ depth, int nz, int z0, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double ss = 0.0, sp = 0.0;
    int ns = 0, np = 0, nd = 0;
    for (int z = z0; z < nz; ++z) {
        const double t = depth[z], s = depth[nz + z], p = depth[2 * nz + z];
        if (!(t > 0.0)) continue;
        ++nd;
        if (isfinite(s)) { ss += s / t; ++ns; }
        if (isfinite(p)) { sp += p / t; ++np; }
    }
    const double ms = ns ? ss / ns : NAN, mp = np ? sp / np : NAN;
    double vs = 0.0, vp = 0.0;
    for (int z = z0; z < nz; ++z) {
        const double t = depth[z], s = depth[nz + z], p = depth[2 * nz + z];
        if (!(t > 0.0)) continue;
        if (isfinite(s)) vs += (s / t - ms) * (s / t - ms);
        if (isfinite(p)) vp += (p / t - mp) * (p / t - mp);
    }
    out[0] = ms;
    out[1] = ns > 1 ? sqrt(vs / (ns - 1)) : 0.0;
    out[2] = mp;
    out[3] = np > 1 ? sqrt(vp / (np - 1)) : 0.0;
    out[4] = (double)nd;
}

struct Thresholds {
    double t[8];
};

__global__ void k_escape_hist(const mc_photon_rec *__restrict__ rec, long long n, double width, int nbins,
                              Thresholds th, int nthr, unsigned long long *hw, unsigned long long *hn,
                              unsigned long long *aw, unsigned long long *an)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const mc_photon_rec r = rec[i];
        if (r.fate != 4u && r.fate != 5u) continue;
        const double pv = r.path_void;
        const long long b = std::min((long long)floor(pv / width), (long long)nbins - 1);
        atomicAdd(&hw[b], (unsigned long long)r.w_final);
        atomicAdd(&hn[b], 1ull);
        for (int k = 0; k < nthr; ++k) {
            if (pv > th.t[k]) {
                atomicAdd(&aw[k], (unsigned long long)r.w_final);
                atomicAdd(&an[k], 1ull);
            }
        }
    }
}

__global__ void k_fill_value(long long *p, long long n, long long v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// solid voxels among the marked ones of one slice, added to *out
__global__ void k_count_solid(const uint8_t *__restrict__ top, const uint8_t *__restrict__ mask, long long n,
                              unsigned long long *out)
{
    unsigned long long c = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        c += (top[i] && mask[i] == 0) ? 1ull : 0ull;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// Distance transform, pass 1: squared distance along x to the nearest solid
// voxel of the same line (two scans), kInf where the line has none.
__global__ void k_edt_x(const uint8_t *__restrict__ mask, int nx, long long lines, int *__restrict__ g)
{
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= lines) return;
    const uint8_t *m = mask + (size_t)l * nx;
    int *o = g + (size_t)l * nx;
    int d = kInf;
    for (int x = 0; x < nx; ++x) {
        d = m[x] == 0 ? 0 : (d == kInf ? kInf : d + 1);
        o[x] = d;
    }
    d = kInf;
    for (int x = nx - 1; x >= 0; --x) {
        d = m[x] == 0 ? 0 : (d == kInf ? kInf : d + 1);
        const int e = std::min(o[x], d);
        o[x] = e == kInf ? kInf : e * e;
    }
}

// Passes 2 and 3: along y (axis 1) or z (axis 2), f(q) -> min_p f(p) + (q - p)^2
// over the line, by the lower envelope of the parabolas rooted at the finite f(p)
// (Felzenszwalb & Huttenlocher).  One thread per line of this chunk; scratch
// arrays laid out [k][line] so that neighbouring threads touch neighbouring words.
// The envelope is built before any output is written, so the pass runs in place.
__global__ void k_edt_env(int *g, int axis, int n, long long line0, long long nlines, int nx, int ny, int *sv,
                          int *sf, double *sz)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlines) return;
    const long long l = line0 + t;
    const long long C = nlines;
    auto V = [&](int k) -> int & { return sv[(size_t)k * C + t]; };
    auto F = [&](int k) -> int & { return sf[(size_t)k * C + t]; };
    auto Z = [&](int k) -> double & { return sz[(size_t)k * C + t]; };
    int k = -1;
    for (int q = 0; q < n; ++q) {
        const int fq = g[line_elem(axis, l, q, nx, ny)];
        if (fq >= kInf) continue;
        if (k < 0) {
            k = 0;
            V(0) = q;
            F(0) = fq;
            Z(0) = -INFINITY;
            Z(1) = INFINITY;
            continue;
        }
        double s;
        for (;;) {
            const int vk = V(k);
            s = ((double)fq + (double)q * q - ((double)F(k) + (double)vk * vk)) / (2.0 * (q - vk));
            if (s <= Z(k)) --k;     // Z(0) = -inf stops this at k = 0
            else break;
        }
        ++k;
        V(k) = q;
        F(k) = fq;
        Z(k) = s;
        Z(k + 1) = INFINITY;
    }
    if (k < 0) return;              // no solid voxel reaches this line: stays kInf
    int j = 0;
    for (int q = 0; q < n; ++q) {
        while (Z(j + 1) < (double)q) ++j;
        const int d = q - V(j);
        g[line_elem(axis, l, q, nx, ny)] = d * d + F(j);
    }
}

__global__ void k_edt_out(const int *__restrict__ g, long long n, double *dist)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int d = g[i];
        dist[i] = d >= kInf ? INFINITY : sqrt((double)d);
    }
}

unsigned blocks_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65535)); }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

int mc_chord_histogram(const mc_volume *vol, int32_t axis, int64_t *hist, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (axis < 0 || axis > 2) return fail(MC_EINVAL, "axis must be 0 (x), 1 (y) or 2 (z)");
    if (!hist) return fail(MC_EINVAL, "hist is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const int n = axis == 0 ? vol->nx : (axis == 1 ? vol->ny : vol->nz);
    const long long lines = (long long)vol->nx * vol->ny * vol->nz / n;
    const long long nh = 2ll * (n + 1);
    hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(nh)), dim3(kThreads), 0, s, (long long *)hist, nh);
    hipLaunchKernelGGL(k_chords, dim3((unsigned)((lines + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, vol->mask,
                       axis, n, lines, vol->nx, vol->ny, (unsigned long long *)hist);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_phase_contrast(const double *depth, int32_t nz, int32_t z0, double *out, void *hip_stream)
{
    clear_error();
    if (!depth || !out) return fail(MC_EINVAL, "NULL argument");
    if (nz < 1 || z0 < 0 || z0 >= nz) return fail(MC_EINVAL, "need nz >= 1 and 0 <= z0 < nz");
    hipLaunchKernelGGL(k_contrast, dim3(1), dim3(64), 0, (hipStream_t)hip_stream, depth, nz, z0, out);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_escape_path_histogram(const mc_photon_rec *rec, int64_t n, double bin_width, int32_t nbins,
                             const double *thresholds, int32_t nthr, int64_t *hist_w, int64_t *hist_n,
                             int64_t *above_w, int64_t *above_n, void *hip_stream)
{
    clear_error();
    if (!rec || !hist_w || !hist_n) return fail(MC_EINVAL, "NULL argument");
    if (n < 0 || nbins < 1 || !(bin_width > 0.0) || !isfinite(bin_width))
        return fail(MC_EINVAL, "need n >= 0, nbins >= 1 and a finite bin_width > 0");
    if (nthr < 0 || nthr > 8) return fail(MC_EINVAL, "nthr must be 0..8");
    if (nthr > 0 && (!thresholds || !above_w || !above_n)) return fail(MC_EINVAL, "thresholds and above_* needed");
    Thresholds th;
    memset(&th, 0, sizeof th);
    for (int k = 0; k < nthr; ++k) th.t[k] = thresholds[k];
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(nbins)), dim3(kThreads), 0, s, (long long *)hist_w, (long long)nbins);
    hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(nbins)), dim3(kThreads), 0, s, (long long *)hist_n, (long long)nbins);
    if (nthr > 0) {
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(kThreads), 0, s, (long long *)above_w, (long long)nthr);
        hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(kThreads), 0, s, (long long *)above_n, (long long)nthr);
    }
    if (n > 0)
        hipLaunchKernelGGL(k_escape_hist, dim3(blocks_for(n)), dim3(kThreads), 0, s, rec, (long long)n, bin_width, nbins,
                           th, nthr, (unsigned long long *)hist_w, (unsigned long long *)hist_n,
                           (unsigned long long *)above_w, (unsigned long long *)above_n);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_bright_colocalization_workspace_bytes(const mc_volume *vol)
{
    clear_error();
    if (check_volume(vol)) return 0;
    const long long n = (long long)vol->nx * vol->ny;
    return align256((size_t)n) + pmc::sel::workspace_bytes(n);
}

int mc_bright_colocalization(const mc_volume *vol, const int64_t *fluence, int32_t z0, double frac,
                             int64_t *top_count, int64_t *top_solid, void *workspace, size_t workspace_bytes,
                             void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!fluence || !top_count || !top_solid || !workspace) return fail(MC_EINVAL, "NULL argument");
    if (z0 < 0 || z0 >= vol->nz) return fail(MC_EINVAL, "need 0 <= z0 < nz");
    if (!(frac > 0.0 && frac <= 1.0)) return fail(MC_EINVAL, "frac must be in (0, 1]");
    const size_t need = mc_bright_colocalization_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t s = (hipStream_t)hip_stream;
    const long long n = (long long)vol->nx * vol->ny;
    const long long k = (long long)ceil(frac * (double)n);
    const int slices = vol->nz - z0;
    uint8_t *top = (uint8_t *)workspace;
    void *sel_ws = (char *)workspace + align256((size_t)n);
    hipLaunchKernelGGL(k_fill_value, dim3(blocks_for(slices)), dim3(kThreads), 0, s, (long long *)top_count,
                       (long long)slices, k);
    hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(slices)), dim3(kThreads), 0, s, (long long *)top_solid,
                       (long long)slices);
    for (int z = z0; z < vol->nz; ++z) {
        const long long *f = (const long long *)fluence + (size_t)z * n;
        if ((rc = pmc::sel::enqueue_top<long long>(f, n, k, top, sel_ws, s))) return rc;
        hipLaunchKernelGGL(k_count_solid, dim3(blocks_for(n)), dim3(kThreads), 0, s, top, vol->mask + (size_t)z * n, n,
                           (unsigned long long *)(top_solid + (z - z0)));
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_pore_distance_workspace_bytes(const mc_volume *vol)
{
    clear_error();
    if (check_volume(vol)) return 0;
    const size_t nvox = (size_t)vol->nx * vol->ny * vol->nz;
    const int nmax = std::max(vol->ny, vol->nz);
    const long long lines = std::max((long long)vol->nx * vol->nz, (long long)vol->nx * vol->ny);
    const size_t C = (size_t)std::min<long long>(kEdtChunk, lines);
    return align256(nvox * sizeof(int)) + align256(C * (nmax + 1) * sizeof(int)) * 2 +
           align256(C * (nmax + 2) * sizeof(double));
}

int mc_pore_distance(const mc_volume *vol, double *dist, void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!dist || !workspace) return fail(MC_EINVAL, "NULL argument");
    const size_t need = mc_pore_distance_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    if ((long long)vol->nx * vol->nx + (long long)vol->ny * vol->ny + (long long)vol->nz * vol->nz >= kInf)
        return fail(MC_EINVAL, "volume too large for 32-bit squared distances");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nx = vol->nx, ny = vol->ny, nz = vol->nz;
    const size_t nvox = (size_t)nx * ny * nz;
    const int nmax = std::max(ny, nz);
    const long long max_lines = std::max((long long)nx * nz, (long long)nx * ny);
    const long long C = std::min<long long>(kEdtChunk, max_lines);
    char *b = (char *)workspace;
    int *g = (int *)b;
    int *sv = (int *)(b + align256(nvox * sizeof(int)));
    int *sf = (int *)((char *)sv + align256((size_t)C * (nmax + 1) * sizeof(int)));
    double *sz = (double *)((char *)sf + align256((size_t)C * (nmax + 1) * sizeof(int)));
    const long long xl = (long long)ny * nz;
    hipLaunchKernelGGL(k_edt_x, dim3((unsigned)((xl + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, vol->mask, nx, xl,
                       g);
    for (int axis = 1; axis <= 2; ++axis) {
        const int n = axis == 1 ? ny : nz;
        if (n == 1) continue;
        const long long lines = (long long)nx * (axis == 1 ? nz : ny);
        for (long long l0 = 0; l0 < lines; l0 += C) {
            const long long cl = std::min(C, lines - l0);
            hipLaunchKernelGGL(k_edt_env, dim3((unsigned)((cl + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, g, axis,
                               n, l0, cl, nx, ny, sv, sf, sz);
        }
    }
    hipLaunchKernelGGL(k_edt_out, dim3(blocks_for((long long)nvox)), dim3(kThreads), 0, s, g, (long long)nvox, dist);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // extern "C"
