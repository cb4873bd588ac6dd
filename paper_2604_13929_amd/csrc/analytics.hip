// analytics.hip -- morphology and fluence analytics of Sec. 3.5: chord-length
// histograms, depth-normalised phase contrast, escape-path histograms, the
// brightest-decile co-localisation per slice, the exact Euclidean distance
// transform of the pore phase, and the per-slice Spearman correlation of fluence
// with pore size.
//
// These are scans over the mask, the fluence tally or per-photon records, so they
// are bound by memory traffic or launch count, not arithmetic: line scans with
// neighbouring lanes on neighbouring bytes, histograms in LDS, a radix select per
// slice in one workgroup for the deciles.  The distance transform is separable: a
// two-sided scan along x, then along y and along z an outward scan from each voxel
// over LDS-staged lines that stops, exact, once the squared radius passes the best
// value; lines it leaves open (far from any solid) are redone by the lower
// envelope of parabolas of Felzenszwalb & Huttenlocher (2012).  The Spearman
// correlation compacts each slice's pore voxels, ranks the fluence by one
// device-wide rocPRIM radix sort of (slice, fluence) keys over just the bits the
// data occupy, ranks the small integer squared distances by counting in LDS, and
// averages tied ranks.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "analytics.h"
#include "internal.hpp"

using namespace pmc::host;

namespace {

constexpr int kThreads = 256;
constexpr int kInf = 0x3fffffff;          // "no solid voxel on this line yet" for squared distances
constexpr long long kEdtChunk = 16384;    // envelope scratch slots: lines redone at once

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

// One thread per line; the workgroup counts its chords in an LDS histogram of
// 2 (n + 1) words and adds the non-zero bins to the global one at the end (global
// atomics on a few hundred hot bins would serialise).  Lines whose histogram does
// not fit in LDS go to the global-atomic variant.
__global__ __launch_bounds__(kThreads) void k_chords(const uint8_t *__restrict__ mask, int axis, int n, long long lines,
                                                     int nx, int ny, unsigned long long *hist)
{
    extern __shared__ unsigned int hs[];
    const int nh = 2 * (n + 1);
    for (int i = (int)threadIdx.x; i < nh; i += kThreads) hs[i] = 0u;
    __syncthreads();
    for (long long l = (long long)blockIdx.x * kThreads + threadIdx.x; l < lines; l += (long long)gridDim.x * kThreads) {
        int start = 0;
        uint8_t cur = mask[line_elem(axis, l, 0, nx, ny)];
        for (int j = 1; j <= n; ++j) {
            const uint8_t v = j < n ? mask[line_elem(axis, l, j, nx, ny)] : (uint8_t)(cur ^ 1u);
            if (v != cur) {
                atomicAdd(&hs[(cur ? 1 : 0) * (n + 1) + (j - start)], 1u);
                start = j;
                cur = v;
            }
        }
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < nh; i += kThreads)
        if (hs[i]) atomicAdd(&hist[i], (unsigned long long)hs[i]);
}

// The same count with the lines staged in LDS: a workgroup of kChordTile threads
// loads kChordTile lines whole with coalesced reads (axis 0: consecutive x-lines;
// axis 1: consecutive x at one z; axis 2: consecutive positions of the xy plane) into
// rows of an odd number of words, one row per line, so that both the transposing
// byte stores and the threads' row reads fall in distinct banks; each thread then
// scans its row four voxels per LDS read.  (Splitting a row among four threads that
// read bytes measured slower: 72-103 against 48-54 us per axis at 256^3.)
constexpr int kChordTile = 128;

__host__ __device__ inline int chord_words(int n) { return ((n + 3) / 4) | 1; }

template <int AXIS>
__global__ __launch_bounds__(kChordTile) void k_chords_tile(const uint8_t *__restrict__ mask, int n, int nx, int ny,
                                                            int nz, unsigned long long *hist)
{
    extern __shared__ unsigned int hs[];             // 2 (n + 1) counters, then the tile rows
    unsigned int *rows = hs + 2 * (n + 1);
    uint8_t *tile = reinterpret_cast<uint8_t *>(rows);
    const int t = (int)threadIdx.x, nh = 2 * (n + 1), words = chord_words(n), pitch = 4 * words;
    for (int i = t; i < nh; i += kChordTile) hs[i] = 0u;
    size_t base;
    long long stride;
    int w;
    if (AXIS == 0) {
        const long long l0 = (long long)blockIdx.x * kChordTile;
        w = (int)std::min<long long>(kChordTile, (long long)ny * nz - l0);
        base = (size_t)l0 * nx;
        stride = 1;
    } else if (AXIS == 1) {
        const int per_z = (nx + kChordTile - 1) / kChordTile;
        const int z = (int)blockIdx.x / per_z, x0 = ((int)blockIdx.x - z * per_z) * kChordTile;
        w = std::min(kChordTile, nx - x0);
        base = (size_t)z * ny * nx + x0;
        stride = nx;
    } else {
        const long long l0 = (long long)blockIdx.x * kChordTile;
        w = (int)std::min<long long>(kChordTile, (long long)nx * ny - l0);
        base = (size_t)l0;
        stride = (long long)nx * ny;
    }
    if (AXIS == 0) {
        for (int e = t; e < w * n; e += kChordTile) {
            const int c = e / n, j = e - c * n;
            tile[c * pitch + j] = mask[base + e];
        }
    } else {
        for (int e = t; e < n * w; e += kChordTile) {
            const int j = e / w, c = e - j * w;
            tile[c * pitch + j] = mask[base + j * stride + c];
        }
    }
    __syncthreads();
    if (t < w) {
        const unsigned int *row = rows + t * words;
        unsigned int cur = row[0] & 0xffu;
        int start = 0;
        for (int q = 0; 4 * q < n; ++q) {
            const unsigned int wv = row[q];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = 4 * q + b;
                const unsigned int v = (wv >> (8 * b)) & 0xffu;
                if (j > 0 && j < n && v != cur) {
                    atomicAdd(&hs[(cur ? 1 : 0) * (n + 1) + (j - start)], 1u);
                    start = j;
                    cur = v;
                }
            }
        }
        atomicAdd(&hs[(cur ? 1 : 0) * (n + 1) + (n - start)], 1u);   // the run that ends the line
    }
    __syncthreads();
    for (int i = t; i < nh; i += kChordTile)
        if (hs[i]) atomicAdd(&hist[i], (unsigned long long)hs[i]);
}

// LDS bytes of k_chords_tile for lines of n voxels
size_t chord_tile_lds(int n)
{
    return sizeof(unsigned int) * (2 * ((size_t)n + 1) + (size_t)kChordTile * chord_words(n));
}

__global__ void k_chords_global(const uint8_t *__restrict__ mask, int axis, int n, long long lines, int nx, int ny,
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

// one wavefront, sample variance by two passes: lane l takes the depths z0 + l,
// z0 + l + 64, ...; the sums are reduced to lane 0 in a fixed order and the means
// broadcast for the second pass
__device__ __forceinline__ double wave_sum_to_all(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    return __shfl(v, 0);
}

__global__ __launch_bounds__(64) void k_contrast(const double *__restrict__ depth, int nz, int z0, double *out)
{
    const int lane = (int)threadIdx.x;
    double ss = 0.0, sp = 0.0, ns = 0.0, np = 0.0, nd = 0.0;   // counts are exact in double
    for (int z = z0 + lane; z < nz; z += 64) {
        const double t = depth[z], s = depth[nz + z], p = depth[2 * nz + z];
        if (!(t > 0.0)) continue;
        nd += 1.0;
        if (isfinite(s)) { ss += s / t; ns += 1.0; }
        if (isfinite(p)) { sp += p / t; np += 1.0; }
    }
    ss = wave_sum_to_all(ss);
    sp = wave_sum_to_all(sp);
    ns = wave_sum_to_all(ns);
    np = wave_sum_to_all(np);
    nd = wave_sum_to_all(nd);
    const double ms = ns > 0.0 ? ss / ns : NAN, mp = np > 0.0 ? sp / np : NAN;
    double vs = 0.0, vp = 0.0;
    for (int z = z0 + lane; z < nz; z += 64) {
        const double t = depth[z], s = depth[nz + z], p = depth[2 * nz + z];
        if (!(t > 0.0)) continue;
        if (isfinite(s)) vs += (s / t - ms) * (s / t - ms);
        if (isfinite(p)) vp += (p / t - mp) * (p / t - mp);
    }
    vs = wave_sum_to_all(vs);
    vp = wave_sum_to_all(vp);
    if (lane == 0) {
        out[0] = ms;
        out[1] = ns > 1.0 ? sqrt(vs / (ns - 1.0)) : 0.0;
        out[2] = mp;
        out[3] = np > 1.0 ? sqrt(vp / (np - 1.0)) : 0.0;
        out[4] = nd;
    }
}

struct Thresholds {
    double t[8];
};

// Escape-path histograms with the bins in LDS (weights 64-bit, counts 32-bit per
// workgroup) and the threshold sums kept per thread, then reduced per wave: one
// global atomic per wave and threshold instead of one per photon.
constexpr int kEscLdsBins = 2048;

template <bool LDS>
__global__ __launch_bounds__(kThreads) void k_escape_hist(const mc_photon_rec *__restrict__ rec, long long n,
                                                          double width, int nbins, Thresholds th, int nthr,
                                                          unsigned long long *hw, unsigned long long *hn,
                                                          unsigned long long *aw, unsigned long long *an)
{
    __shared__ unsigned long long sw[LDS ? kEscLdsBins : 1];
    __shared__ unsigned int sn[LDS ? kEscLdsBins : 1];
    if (LDS) {
        for (int i = (int)threadIdx.x; i < nbins; i += kThreads) {
            sw[i] = 0ull;
            sn[i] = 0u;
        }
        __syncthreads();
    }
    unsigned long long tw[8], tn[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) tw[k] = tn[k] = 0ull;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const mc_photon_rec r = rec[i];
        if (r.fate != 4u && r.fate != 5u) continue;
        const double pv = r.path_void;
        const int b = pmc::escape_path_bin(pv, width, nbins);
        if (LDS) {
            atomicAdd(&sw[b], (unsigned long long)r.w_final);
            atomicAdd(&sn[b], 1u);
        } else {
            atomicAdd(&hw[b], (unsigned long long)r.w_final);
            atomicAdd(&hn[b], 1ull);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < nthr && pv > th.t[k]) {
                tw[k] += (unsigned long long)r.w_final;
                tn[k] += 1ull;
            }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= nthr) break;
        unsigned long long a = tw[k], c = tn[k];
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            c += __shfl_xor(c, o);
        }
        if ((threadIdx.x & 63) == 0 && c) {
            atomicAdd(&aw[k], a);
            atomicAdd(&an[k], c);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int i = (int)threadIdx.x; i < nbins; i += kThreads)
            if (sn[i]) {
                atomicAdd(&hw[i], sw[i]);
                atomicAdd(&hn[i], (unsigned long long)sn[i]);
            }
    }
}

// Brightest fraction of one slice per workgroup: an MSB-first radix select over
// the order-preserving key of the int64 tally finds the k-th largest key T and how
// many keys equal to T are taken; a pass in index order then takes every key above
// T and the first `need` keys equal to T (ties to the lower index) and counts the
// solid voxels among them.  A first pass over the slice finds the bits all its keys
// share (their minimum and maximum), so the 11-bit digits start at the highest bit
// that differs.  A digit pass reads the slice while more than kTopCand keys are
// still in the running; once they fit, one pass copies them to LDS and the
// remaining digits are resolved there.
constexpr int kTopThreads = 1024;
constexpr int kTopBits = 11;
constexpr int kTopBins = 1 << kTopBits;
constexpr int kTopCand = 6144;   // 48 KB of LDS

__device__ __forceinline__ unsigned long long tally_key(long long v) { return (unsigned long long)v ^ 0x8000000000000000ull; }

// inclusive prefix sum over the workgroup's threads in thread order
__device__ __forceinline__ unsigned int block_inclusive_scan(unsigned int v, unsigned int *wsum)
{
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned int u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    unsigned int before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    __syncthreads();
    return v + before;
}

__global__ __launch_bounds__(kTopThreads) void k_slice_top(const long long *__restrict__ F, const uint8_t *__restrict__ mask,
                                                          long long n, int z0, long long k, long long *top_count,
                                                          long long *top_solid)
{
    __shared__ unsigned int h[kTopBins];
    __shared__ unsigned int wsum[kTopThreads / 64];
    __shared__ unsigned long long cand[kTopCand];
    __shared__ unsigned long long s_prefix, s_min, s_max;
    __shared__ long long s_k;
    __shared__ unsigned int s_count, s_ncand;
    const size_t base = (size_t)(z0 + blockIdx.x) * (size_t)n;
    const long long *f = F + base;
    const uint8_t *m = mask + base;
    const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) {
        s_min = ~0ull;
        s_max = 0ull;
        s_ncand = 0u;
    }
    __syncthreads();
    {
        unsigned long long lo = ~0ull, hi = 0ull;
        for (long long i = t; i < n; i += kTopThreads) {
            const unsigned long long key = tally_key(f[i]);
            lo = min(lo, key);
            hi = max(hi, key);
        }
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, (unsigned long long)__shfl_xor(lo, o));
            hi = max(hi, (unsigned long long)__shfl_xor(hi, o));
        }
        if (lane == 0) {
            atomicMin(&s_min, lo);
            atomicMax(&s_max, hi);
        }
    }
    __syncthreads();
    const unsigned long long diff = s_min ^ s_max;
    // bits at and above `top` are resolved: they equal those of `prefix`
    int top = diff ? 64 - __clzll((long long)diff) : 0;
    unsigned long long prefix = top >= 64 ? 0ull : (s_min & (~0ull << top));
    long long kk = k;
    bool in_lds = false;
    while (top > 0) {
        const int bits = min(kTopBits, top), sh = top - bits, nb = 1 << bits;
        const unsigned long long hi_mask = top >= 64 ? 0ull : (~0ull << top);
        for (int i = t; i < nb; i += kTopThreads) h[i] = 0u;
        __syncthreads();
        if (in_lds) {
            const int nc = (int)s_ncand;
            for (int j = t; j < nc; j += kTopThreads) {
                const unsigned long long key = cand[j];
                if ((key & hi_mask) == prefix) atomicAdd(&h[(key >> sh) & (unsigned long long)(nb - 1)], 1u);
            }
        } else {
            for (long long i0 = 0; i0 < n; i0 += kTopThreads) {
                const long long i = i0 + t;
                int d = -1;
                if (i < n) {
                    const unsigned long long key = tally_key(f[i]);
                    if ((key & hi_mask) == prefix) d = (int)((key >> sh) & (unsigned long long)(nb - 1));
                }
                // a wave whose candidates share one digit adds them with one atomic
                const int d0 = __shfl(d, 0);
                if (__ballot(d == d0) == ~0ull) {
                    if (lane == 0 && d0 >= 0) atomicAdd(&h[d0], 64u);
                } else if (d >= 0) {
                    atomicAdd(&h[d], 1u);
                }
            }
        }
        __syncthreads();
        // thread t holds digits nb-1-2t and nb-2-2t: the prefix over threads runs from the top digit down
        const int dhi = nb - 1 - 2 * t, dlo = dhi - 1;
        const unsigned int chi = dhi >= 0 ? h[dhi] : 0u, clo = dlo >= 0 ? h[dlo] : 0u;
        const unsigned int incl = block_inclusive_scan(chi + clo, wsum);
        const unsigned int excl = incl - chi - clo;
        if ((long long)excl < kk && kk <= (long long)incl) {
            const bool in_hi = (long long)(excl + chi) >= kk;
            const int d = in_hi ? dhi : dlo;
            s_prefix = prefix | ((unsigned long long)d << sh);
            s_k = kk - (long long)(in_hi ? excl : excl + chi);
            s_count = in_hi ? chi : clo;
        }
        __syncthreads();
        prefix = s_prefix;
        kk = s_k;
        top = sh;
        if (!in_lds && top > 0 && s_count <= (unsigned int)kTopCand) {
            // the keys still in the running fit in LDS: copy them there (any order)
            const unsigned long long keep = ~0ull << top;
            for (long long i0 = 0; i0 < n; i0 += kTopThreads) {
                const long long i = i0 + t;
                unsigned long long key = 0ull;
                bool match = false;
                if (i < n) {
                    key = tally_key(f[i]);
                    match = (key & keep) == prefix;
                }
                const unsigned long long bal = __ballot(match);
                if (bal) {
                    unsigned int at = 0u;
                    if (lane == 0) at = atomicAdd(&s_ncand, (unsigned int)__popcll(bal));
                    at = __shfl(at, 0);
                    if (match) cand[at + __popcll(bal & ((1ull << lane) - 1ull))] = key;
                }
            }
            in_lds = true;
            __syncthreads();
        }
    }
    const unsigned long long T = prefix;
    const long long need = kk;
    long long run = 0;
    unsigned int solid = 0;
    for (long long i0 = 0; i0 < n; i0 += kTopThreads) {
        const long long i = i0 + t;
        unsigned long long key = 0ull;
        if (i < n) key = tally_key(f[i]);
        const bool eq = i < n && key == T;
        const unsigned long long bal = __ballot(eq);
        if (lane == 0) wsum[wave] = (unsigned int)__popcll(bal);
        __syncthreads();
        long long off = run + __popcll(bal & ((1ull << lane) - 1ull));
        long long tot = 0;
        for (int w = 0; w < kTopThreads / 64; ++w) {
            if (w < wave) off += wsum[w];
            tot += wsum[w];
        }
        const bool take = i < n && (key > T || (eq && off < need));
        solid += (take && m[i] == 0) ? 1u : 0u;
        run += tot;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) solid += __shfl_xor(solid, o);
    if (lane == 0) wsum[wave] = solid;
    __syncthreads();
    if (t == 0) {
        long long sum = 0;
        for (int w = 0; w < kTopThreads / 64; ++w) sum += wsum[w];
        top_solid[blockIdx.x] = sum;
        top_count[blockIdx.x] = k;
    }
}

// Distance transform, pass 1: squared distance along x to the nearest solid
// voxel of the same line, kInf where the line has none.  One wavefront per line,
// lane = x within a 64-voxel chunk: an inclusive max-scan across the lanes of
// "x if solid" (carried from chunk to chunk) gives the nearest solid voxel on the
// left, a min-scan from the right end the nearest on the right; every load and
// store is a contiguous run of the line.
__global__ __launch_bounds__(kThreads) void k_edt_x(const uint8_t *__restrict__ mask, int nx, long long lines,
                                                    int *__restrict__ g)
{
    const long long l = (long long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (l >= lines) return;                        // the whole wavefront leaves together
    const int lane = (int)(threadIdx.x & 63);
    const uint8_t *m = mask + (size_t)l * nx;
    int *o = g + (size_t)l * nx;
    int carry = -1;                                // nearest solid voxel at or left of the chunk start
    for (int x0 = 0; x0 < nx; x0 += 64) {
        const int x = x0 + lane;
        int v = (x < nx && m[x] == 0) ? x : -1;
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(v, off);
            if (lane >= off) v = std::max(v, u);
        }
        v = std::max(v, carry);
        carry = __shfl(v, 63);
        if (x < nx) o[x] = v;
    }
    constexpr int kNone = 0x7fffffff;
    carry = kNone;                                 // nearest solid voxel at or right of the chunk end
    for (int x0 = ((nx - 1) / 64) * 64; x0 >= 0; x0 -= 64) {
        const int x = x0 + lane;
        int v = (x < nx && m[x] == 0) ? x : kNone;
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_down(v, off);
            if (lane + off < 64) v = std::min(v, u);
        }
        v = std::min(v, carry);
        carry = __shfl(v, 0);
        if (x < nx) {
            const int left = o[x];
            int d = kInf;
            if (left >= 0) d = x - left;
            if (v != kNone) d = std::min(d, v - x);
            o[x] = d == kInf ? kInf : d * d;
        }
    }
}

// Passes 2 and 3: along y (axis 1) or z (axis 2), f(q) -> min_p f(p) + (q - p)^2
// over the line through q.  First one thread per voxel (neighbouring threads on
// neighbouring x, so every load is coalesced) scans outward from q: a candidate at
// distance r costs at least r^2, so the scan stops, exact, once r^2 reaches the best
// value found, or at the ends of the line.  In a porous mask that is after a few
// voxels; a voxel still open after kEdtReach steps marks its line, and the marked
// lines are redone whole by the lower envelope of parabolas (Felzenszwalb &
// Huttenlocher), O(n) per line, which bounds the worst case (lines far from any
// solid voxel).  in and out are distinct buffers.
constexpr int kEdtReach = 64;

// grid: x over the voxels of one z-slice (nx * ny < 2^30 where the transform is
// allowed), y over the slices
template <int AXIS>
__global__ __launch_bounds__(kThreads) void k_edt_scan(const int *__restrict__ in, int *__restrict__ out,
                                                       uint8_t *__restrict__ open_line, int nx, int ny, int nz)
{
    const int n = AXIS == 1 ? ny : nz;
    const int plane = nx * ny;
    const long long stride = AXIS == 1 ? (long long)nx : (long long)plane;
    const int z = (int)blockIdx.y;
    for (int p = (int)(blockIdx.x * kThreads + threadIdx.x); p < plane; p += (int)(gridDim.x * kThreads)) {
        const int y = p / nx, x = p - y * nx;
        const long long i = (long long)z * plane + p;
        const int q = AXIS == 1 ? y : z;
        int best = in[i];
        bool done = false;
        for (int r = 1; r <= kEdtReach + 1; ++r) {
            const int r2 = r * r;
            const bool lo = q - r >= 0, hi = q + r < n;
            if (r2 >= best || (!lo && !hi)) {
                done = true;
                break;
            }
            if (r > kEdtReach) break;
            if (lo) {
                const int v = in[i - r * stride];
                if (v < kInf) best = std::min(best, v + r2);
            }
            if (hi) {
                const int v = in[i + r * stride];
                if (v < kInf) best = std::min(best, v + r2);
            }
        }
        out[i] = best;
        if (!done) open_line[AXIS == 1 ? (long long)z * nx + x : (long long)y * nx + x] = 1;
    }
}

// The same scan with the lines staged in LDS: a workgroup takes tx consecutive
// x-columns of the n voxels along AXIS at one position of the remaining axis (z for
// y-lines, y for z-lines), loads them once with coalesced runs of tx words, and
// scans there; candidates, early stop and open-line marks are those of k_edt_scan,
// so the results are the same.  The tile is [n][tx] words, tx a power of two.  On
// the 256^3 workload narrow tiles (more workgroups per CU) measured fastest for
// the whole transform: 0.42 ms at 8 columns, 0.45 at 16, 0.57 at 32, 0.86 at 64,
// against 0.67 ms for the scan from global memory.
#ifndef MC_EDT_TILE_X
#define MC_EDT_TILE_X 8
#endif
constexpr int kEdtTileX = MC_EDT_TILE_X;
constexpr int kEdtTileWords = 16384;       // 64 KB of LDS

template <int AXIS>
__global__ __launch_bounds__(kThreads) void k_edt_tile(const int *__restrict__ in, int *__restrict__ out,
                                                       uint8_t *__restrict__ open_line, int nx, int ny, int nz,
                                                       int tx_log)
{
    extern __shared__ int tile[];
    const int n = AXIS == 1 ? ny : nz;
    const int tx = 1 << tx_log;
    const long long stride = AXIS == 1 ? (long long)nx : (long long)nx * ny;
    const int x0 = (int)blockIdx.x << tx_log, other = (int)blockIdx.y;
    const long long base = (AXIS == 1 ? (long long)other * nx * ny : (long long)other * nx) + x0;
    const int w = min(tx, nx - x0);
    const int cells = n << tx_log;
    for (int e = (int)threadIdx.x; e < cells; e += kThreads) {
        const int q = e >> tx_log, c = e & (tx - 1);
        if (c < w) tile[e] = in[base + q * stride + c];
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < cells; e += kThreads) {
        const int q = e >> tx_log, c = e & (tx - 1);
        if (c >= w) continue;
        int best = tile[e];
        bool done = false;
        for (int r = 1; r <= kEdtReach + 1; ++r) {
            const int r2 = r * r;
            const bool lo = q - r >= 0, hi = q + r < n;
            if (r2 >= best || (!lo && !hi)) {
                done = true;
                break;
            }
            if (r > kEdtReach) break;
            if (lo) {
                const int v = tile[e - (r << tx_log)];
                if (v < kInf) best = std::min(best, v + r2);
            }
            if (hi) {
                const int v = tile[e + (r << tx_log)];
                if (v < kInf) best = std::min(best, v + r2);
            }
        }
        out[base + q * stride + c] = best;
        if (!done) open_line[(long long)other * nx + x0 + c] = 1;
    }
}

// the tile width for lines of n voxels: the widest power of two up to kEdtTileX (and
// no wider than nx needs) whose tile fits kEdtTileWords, but not below 8 columns
// where nx has them; -1 where no such tile fits, and the scan then runs from
// global memory
int edt_tile_log(int n, int nx)
{
    int lg = 0;
    while ((1 << lg) < kEdtTileX && (1 << lg) < nx) ++lg;
    while (lg > 3 && ((long long)n << lg) > kEdtTileWords) --lg;
    return ((long long)n << lg) <= kEdtTileWords ? lg : -1;
}

// list of the marked lines (order irrelevant: each is redone independently)
__global__ void k_edt_collect(const uint8_t *__restrict__ open_line, long long lines, int *list, int *count)
{
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < lines; l += (long long)gridDim.x * blockDim.x)
        if (open_line[l]) list[atomicAdd(count, 1)] = (int)l;
}

__global__ void k_edt_clear(uint8_t *open_line, long long lines, int *count)
{
    for (long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x; l < lines; l += (long long)gridDim.x * blockDim.x)
        open_line[l] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

// Lower envelope of the parabolas rooted at the finite in(p) of the listed lines,
// one thread per line; scratch arrays laid out [k][slot] so that neighbouring
// threads touch neighbouring words; C slots, a thread takes lines t, t + C, ...
__global__ void k_edt_env(const int *__restrict__ in, int *__restrict__ out, int axis, int n, const int *list,
                          const int *count, long long C, int nx, int ny, int *sv, int *sf, double *sz)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C) return;
    auto V = [&](int k) -> int & { return sv[(size_t)k * C + t]; };
    auto F = [&](int k) -> int & { return sf[(size_t)k * C + t]; };
    auto Z = [&](int k) -> double & { return sz[(size_t)k * C + t]; };
    const long long cnt = *count;
    for (long long idx = t; idx < cnt; idx += C) {
        const long long l = list[idx];
        int k = -1;
        for (int q = 0; q < n; ++q) {
            const int fq = in[line_elem(axis, l, q, nx, ny)];
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
        if (k < 0) {                    // no solid voxel reaches this line
            for (int q = 0; q < n; ++q) out[line_elem(axis, l, q, nx, ny)] = kInf;
            continue;
        }
        int j = 0;
        for (int q = 0; q < n; ++q) {
            while (Z(j + 1) < (double)q) ++j;
            const int d = q - V(j);
            out[line_elem(axis, l, q, nx, ny)] = d * d + F(j);
        }
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

// Pore-phase Spearman correlation.  Compaction of the pore voxels of slice z0 + s in
// index order (keys of fluence and squared distance), in chunks of kSpChunk voxels
// of one slice, one workgroup each; the chunks' offsets come from a scan of their
// pore counts.  Each chunk also records the largest fluence (as unsigned: a negative
// tally reads as 2^63 or more) and squared distance among its pore voxels, in
// cmax[2c] and cmax[2c + 1], and k_chunk_max reduces them into stats[1] and stats[2].
constexpr int kSpThreads = 1024;
constexpr int kSpChunk = 8192;
constexpr int kRankBins = 16128;   // counting ranks: prefix array of up to this many ints (63 KB of LDS)

// pore voxels of chunk c = s * cps + j: voxels [j kSpChunk, (j + 1) kSpChunk) of slice z0 + s
__global__ __launch_bounds__(kSpThreads) void k_chunk_pore_count(const uint8_t *__restrict__ mask, long long n_slice,
                                                                 int z0, int cps, int *counts)
{
    const int c = (int)blockIdx.x, sl = c / cps, j = c - sl * cps;
    const long long lo = (long long)j * kSpChunk, hi = std::min(n_slice, lo + kSpChunk);
    const uint8_t *m = mask + (size_t)(z0 + sl) * n_slice;
    int cnt = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += kSpThreads) cnt += m[i] ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    __shared__ int w[kSpThreads / 64];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int i = 0; i < kSpThreads / 64; ++i) sum += w[i];
        counts[c] = sum;
    }
}

// One workgroup: exclusive scan of the chunk counts into coff (where each chunk's
// pore voxels start), begin / end of every slice, and stats[0] = the number of pore
// voxels over all slices (below 2^31).
__global__ __launch_bounds__(kSpThreads) void k_offsets(const int *__restrict__ counts, int nchunks, int cps, int *coff,
                                                        int *begin, int *end, unsigned long long *stats)
{
    __shared__ unsigned int wsum[kSpThreads / 64];
    __shared__ unsigned int s_carry;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    for (int c0 = 0; c0 < nchunks; c0 += kSpThreads) {
        const int c = c0 + (int)threadIdx.x;
        const unsigned int v = c < nchunks ? (unsigned int)counts[c] : 0u;
        const unsigned int carry = s_carry;
        const unsigned int incl = carry + block_inclusive_scan(v, wsum);
        if (c < nchunks) {
            coff[c] = (int)(incl - v);
            if (c % cps == 0) begin[c / cps] = (int)(incl - v);
            if (c % cps == cps - 1) end[c / cps] = (int)incl;
        }
        __syncthreads();
        if (threadIdx.x == kSpThreads - 1) s_carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) stats[0] = (unsigned long long)s_carry;
}

__global__ __launch_bounds__(kSpThreads) void k_compact(const uint8_t *__restrict__ mask, const long long *__restrict__ F,
                                                        const int *__restrict__ g, long long n_slice, int z0, int cps,
                                                        const int *__restrict__ coff, long long *kf, int *kd, int *pos,
                                                        unsigned long long *cmax)
{
    __shared__ int wcount[kSpThreads / 64];
    __shared__ unsigned long long wmax[2][kSpThreads / 64];
    const int c = (int)blockIdx.x, sl = c / cps, j = c - sl * cps;
    const long long lo = (long long)j * kSpChunk, hi = std::min(n_slice, lo + kSpChunk);
    const size_t base = (size_t)(z0 + sl) * n_slice;
    int run = coff[c];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    unsigned long long fmax = 0ull, dmax = 0ull;
    for (long long i0 = lo; i0 < hi; i0 += kSpThreads) {
        const long long i = i0 + threadIdx.x;
        const bool p = i < hi && mask[base + i] != 0;
        const unsigned long long bal = __ballot(p);
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kSpThreads / 64; ++w) {
            if (w < wave) off += wcount[w];
            tot += wcount[w];
        }
        if (p) {
            const int at = run + off + __popcll(bal & ((1ull << lane) - 1ull));
            const long long f = F[base + i];
            const int d = g[base + i];
            kf[at] = f;
            kd[at] = d;
            pos[at] = at;
            fmax = max(fmax, (unsigned long long)f);
            dmax = max(dmax, (unsigned long long)(unsigned)d);
        }
        run += tot;
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) {
        fmax = max(fmax, (unsigned long long)__shfl_xor(fmax, o));
        dmax = max(dmax, (unsigned long long)__shfl_xor(dmax, o));
    }
    if (lane == 0) {
        wmax[0][wave] = fmax;
        wmax[1][wave] = dmax;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long v = 0ull;
        for (int w = 0; w < kSpThreads / 64; ++w) v = max(v, wmax[threadIdx.x][w]);
        cmax[2 * c + threadIdx.x] = v;
    }
}

// stats[1], stats[2] = the largest of the chunks' maxima (one workgroup)
__global__ __launch_bounds__(kSpThreads) void k_chunk_max(const unsigned long long *__restrict__ cmax, int nchunks,
                                                          unsigned long long *stats)
{
    __shared__ unsigned long long wmax[2][kSpThreads / 64];
    unsigned long long f = 0ull, d = 0ull;
    for (int c = (int)threadIdx.x; c < nchunks; c += kSpThreads) {
        f = max(f, cmax[2 * c]);
        d = max(d, cmax[2 * c + 1]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        f = max(f, (unsigned long long)__shfl_xor(f, o));
        d = max(d, (unsigned long long)__shfl_xor(d, o));
    }
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    if (lane == 0) {
        wmax[0][wave] = f;
        wmax[1][wave] = d;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long v = 0ull;
        for (int w = 0; w < kSpThreads / 64; ++w) v = max(v, wmax[threadIdx.x][w]);
        stats[1 + threadIdx.x] = v;
    }
}

// composite sort keys of slice s: (s << bits) | key, for keys in [0, 2^bits)
template <typename K>
__global__ __launch_bounds__(kSpThreads) void k_compose(const K *__restrict__ key, const int *__restrict__ begin,
                                                        const int *__restrict__ end, unsigned bits,
                                                        unsigned long long *out)
{
    const unsigned long long hi = (unsigned long long)blockIdx.x << bits;
    for (int i = begin[blockIdx.x] + (int)threadIdx.x; i < end[blockIdx.x]; i += kSpThreads)
        out[i] = hi | (unsigned long long)key[i];
}

// average rank (1-based; ties share the mean of their positions) of every element of
// a sorted segment, written at its compact position.  With composite keys the sorted
// array is slice-major, so its slices sit at the same offsets as the compacted ones
// and equal composite keys are equal keys of one slice.
template <typename K>
__global__ void k_avg_rank(const K *__restrict__ sorted, const int *__restrict__ perm, const int *__restrict__ begin,
                           const int *__restrict__ end, int nseg, int total, double *rank)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        // the segment holding i
        int lo_s = 0, hi_s = nseg - 1;
        while (lo_s < hi_s) {
            const int mid = (lo_s + hi_s + 1) >> 1;
            if (begin[mid] <= i) lo_s = mid;
            else hi_s = mid - 1;
        }
        const int b = begin[lo_s], e = end[lo_s];
        const K v = sorted[i];
        if ((i == b || sorted[i - 1] != v) && (i == e - 1 || sorted[i + 1] != v)) {   // no tie
            rank[perm[i]] = (double)(i - b) + 1.0;
            continue;
        }
        int lo = b, hi = (int)i;                 // first position with key == v
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sorted[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        int lo2 = (int)i, hi2 = e - 1;           // last position with key == v
        while (lo2 < hi2) {
            const int mid = (lo2 + hi2 + 1) >> 1;
            if (sorted[mid] > v) hi2 = mid - 1;
            else lo2 = mid;
        }
        rank[perm[i]] = 0.5 * (double)((lo - b) + (lo2 - b)) + 1.0;
    }
}

// Ranks of small non-negative integer keys within each slice by counting.  With
// below(v) keys of the slice smaller than v and count(v) equal to v, the average
// 1-based rank of v is below(v) + (count(v) + 1) / 2, the value the sorted ranks
// give.  P[1 + v] first counts v; its inclusive scan leaves P[v] = below(v) for
// v = 0 .. nbins.  Keys lie in [0, nbins).
__global__ __launch_bounds__(kSpThreads) void k_count_rank(const int *__restrict__ key, const int *__restrict__ begin,
                                                           const int *__restrict__ end, int nbins, double *rank)
{
    extern __shared__ unsigned int P[];   // nbins + 1 entries
    __shared__ unsigned int wsum[kSpThreads / 64];
    const int b = begin[blockIdx.x], e = end[blockIdx.x], t = (int)threadIdx.x;
    for (int v = t; v <= nbins; v += kSpThreads) P[v] = 0u;
    __syncthreads();
    for (int i = b + t; i < e; i += kSpThreads) atomicAdd(&P[key[i] + 1], 1u);
    __syncthreads();
    // thread t scans the run [lo, hi) of P
    const int per = (nbins + kSpThreads) / kSpThreads;
    const int lo = min(t * per, nbins + 1), hi = min(lo + per, nbins + 1);
    unsigned int sum = 0u;
    for (int v = lo; v < hi; ++v) sum += P[v];
    unsigned int run = block_inclusive_scan(sum, wsum) - sum;
    for (int v = lo; v < hi; ++v) {
        run += P[v];
        P[v] = run;
    }
    __syncthreads();
    for (int i = b + t; i < e; i += kSpThreads) {
        const int v = key[i];
        const unsigned int below = P[v], count = P[v + 1] - below;
        rank[i] = (double)below + 0.5 * (double)(count + 1u);
    }
}

// Pearson correlation of the two rank vectors of each segment, centred on the exact
// mean rank (n + 1)/2; fixed summation order per workgroup
__global__ __launch_bounds__(kSpThreads) void k_rank_corr(const double *__restrict__ rf, const double *__restrict__ rd,
                                                          const int *__restrict__ begin, const int *__restrict__ end,
                                                          double *rho, long long *npore)
{
    __shared__ double sh[3][kSpThreads];
    const int b = begin[blockIdx.x], e = end[blockIdx.x];
    const double m = 0.5 * (double)(e - b + 1);
    double sxy = 0.0, sxx = 0.0, syy = 0.0;
    for (int i = b + (int)threadIdx.x; i < e; i += kSpThreads) {
        const double x = rf[i] - m, y = rd[i] - m;
        sxy += x * y;
        sxx += x * x;
        syy += y * y;
    }
    sh[0][threadIdx.x] = sxy;
    sh[1][threadIdx.x] = sxx;
    sh[2][threadIdx.x] = syy;
    __syncthreads();
    for (int o = kSpThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        npore[blockIdx.x] = e - b;
        rho[blockIdx.x] = (sh[1][0] > 0.0 && sh[2][0] > 0.0) ? sh[0][0] / sqrt(sh[1][0] * sh[2][0]) : NAN;
    }
}

// distance transform scratch: two squared-distance buffers, the open-line marks
// and list of the larger line family, the envelope's C-slot scratch
struct EdtScratch {
    int *g, *h, *list, *count, *sv, *sf;
    uint8_t *open;
    double *sz;
    long long C;
};

struct EdtSizes {
    size_t g, open, list, env_i, env_d, total;
    long long C;
};

EdtSizes edt_sizes(const mc_volume *vol)
{
    EdtSizes z;
    const size_t nvox = (size_t)vol->nx * vol->ny * vol->nz;
    const int nmax = std::max(vol->ny, vol->nz);
    const long long lines = std::max((long long)vol->nx * vol->nz, (long long)vol->nx * vol->ny);
    z.C = std::min<long long>(kEdtChunk, lines);
    z.g = align256(nvox * sizeof(int));
    z.open = align256((size_t)lines);
    z.list = align256((size_t)lines * sizeof(int) + sizeof(int));
    z.env_i = align256((size_t)z.C * (nmax + 1) * sizeof(int));
    z.env_d = align256((size_t)z.C * (nmax + 2) * sizeof(double));
    z.total = 2 * z.g + z.open + z.list + 2 * z.env_i + z.env_d;
    return z;
}

size_t edt_bytes(const mc_volume *vol) { return edt_sizes(vol).total; }

EdtScratch edt_layout(const mc_volume *vol, void *ws)
{
    const EdtSizes z = edt_sizes(vol);
    EdtScratch e;
    char *b = (char *)ws;
    e.C = z.C;
    e.g = (int *)b;
    b += z.g;
    e.h = (int *)b;
    b += z.g;
    e.open = (uint8_t *)b;
    b += z.open;
    e.count = (int *)b;
    e.list = e.count + 1;
    b += z.list;
    e.sv = (int *)b;
    b += z.env_i;
    e.sf = (int *)b;
    b += z.env_i;
    e.sz = (double *)b;
    return e;
}

// squared distances (int, kInf where no solid voxel exists) into e.g
int enqueue_sqdist(const mc_volume *vol, const EdtScratch &e, hipStream_t s)
{
    const int nx = vol->nx, ny = vol->ny, nz = vol->nz;
    const long long xl = (long long)ny * nz;
    const dim3 grid((unsigned)std::min<long long>(1024, ((long long)nx * ny + kThreads - 1) / kThreads), (unsigned)nz);
    hipLaunchKernelGGL(k_edt_x, dim3((unsigned)((xl + kThreads / 64 - 1) / (kThreads / 64))), dim3(kThreads), 0, s,
                       vol->mask, nx, xl, e.g);
    const unsigned env_grid = (unsigned)((e.C + kThreads - 1) / kThreads);
    // y: g -> h, z: h -> g
    for (int axis = 1; axis <= 2; ++axis) {
        const int *in = axis == 1 ? e.g : e.h;
        int *out = axis == 1 ? e.h : e.g;
        const int n = axis == 1 ? ny : nz;
        const long long lines = (long long)nx * (axis == 1 ? nz : ny);
        hipLaunchKernelGGL(k_edt_clear, dim3(blocks_for(lines)), dim3(kThreads), 0, s, e.open, lines, e.count);
        const int lg = edt_tile_log(n, nx);
        if (lg >= 0) {
            const dim3 tgrid((unsigned)((nx + (1 << lg) - 1) >> lg), (unsigned)(axis == 1 ? nz : ny));
            const size_t lds = sizeof(int) * ((size_t)n << lg);
            if (axis == 1)
                hipLaunchKernelGGL(k_edt_tile<1>, tgrid, dim3(kThreads), lds, s, in, out, e.open, nx, ny, nz, lg);
            else
                hipLaunchKernelGGL(k_edt_tile<2>, tgrid, dim3(kThreads), lds, s, in, out, e.open, nx, ny, nz, lg);
        } else if (axis == 1) {
            hipLaunchKernelGGL(k_edt_scan<1>, grid, dim3(kThreads), 0, s, in, out, e.open, nx, ny, nz);
        } else {
            hipLaunchKernelGGL(k_edt_scan<2>, grid, dim3(kThreads), 0, s, in, out, e.open, nx, ny, nz);
        }
        hipLaunchKernelGGL(k_edt_collect, dim3(blocks_for(lines)), dim3(kThreads), 0, s, e.open, lines, e.list, e.count);
        hipLaunchKernelGGL(k_edt_env, dim3(env_grid), dim3(kThreads), 0, s, in, out, axis, n, e.list, e.count, e.C, nx, ny,
                           e.sv, e.sf, e.sz);
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

bool too_large(const mc_volume *vol)
{
    return (long long)vol->nx * vol->nx + (long long)vol->ny * vol->ny + (long long)vol->nz * vol->nz >= kInf;
}

int sp_chunks_per_slice(const mc_volume *vol)
{
    return (int)(((long long)vol->nx * vol->ny + kSpChunk - 1) / kSpChunk);
}

// Spearman workspace layout after the distance transform's
struct SpLayout {
    size_t edt, counts, coff, cmax, begin, end, stats, kf, kd, pos, kc, kc_s, perm, rf, rd, tmp, total;
    size_t tmp_bytes;
    hipError_t status;   // of rocPRIM's storage queries (they ask the runtime for the device)
};

SpLayout sp_layout(const mc_volume *vol, int z0, long long npore_max, hipStream_t stream)
{
    SpLayout L;
    const int nseg = vol->nz - z0;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off += align256(bytes); return at; };
    L.edt = take(edt_bytes(vol));
    const long long nchunks = (long long)nseg * sp_chunks_per_slice(vol);
    L.counts = take(sizeof(int) * nchunks);
    L.coff = take(sizeof(int) * nchunks);
    L.cmax = take(sizeof(unsigned long long) * 2 * nchunks);
    L.begin = take(sizeof(int) * nseg);
    L.end = take(sizeof(int) * nseg);
    L.stats = take(sizeof(unsigned long long) * 3);
    L.kf = take(sizeof(long long) * npore_max);
    L.kd = take(sizeof(int) * npore_max);
    L.pos = take(sizeof(int) * npore_max);
    L.kc = take(sizeof(unsigned long long) * npore_max);
    L.kc_s = take(sizeof(unsigned long long) * npore_max);
    L.perm = take(sizeof(int) * npore_max);
    L.rf = take(sizeof(double) * npore_max);
    L.rd = take(sizeof(double) * npore_max);
    // rocPRIM's temporary storage for the larger of the device-wide sort of composite
    // keys and the per-slice sort of raw fluence keys (taken when the composite keys
    // would need more than 64 bits)
    size_t t1 = 0, t2 = 0;
    L.status = rocprim::radix_sort_pairs(nullptr, t1, (const unsigned long long *)nullptr, (unsigned long long *)nullptr,
                                         (const int *)nullptr, (int *)nullptr, (unsigned)npore_max, 0u, 64u, stream);
    if (L.status == hipSuccess)
        L.status = rocprim::segmented_radix_sort_pairs(nullptr, t2, (const long long *)nullptr, (long long *)nullptr,
                                                       (const int *)nullptr, (int *)nullptr, (unsigned)npore_max,
                                                       (unsigned)nseg, (const int *)nullptr, (const int *)nullptr, 0, 64,
                                                       stream);
    L.tmp_bytes = std::max(t1, t2);
    L.tmp = take(L.tmp_bytes);
    L.total = off;
    return L;
}

// number of significant bits of v (0 for v == 0)
unsigned bit_width(unsigned long long v) { return v ? 64u - (unsigned)__builtin_clzll(v) : 0u; }

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
    const size_t lds = sizeof(unsigned int) * (size_t)nh;
    if (chord_tile_lds(n) <= 65536) {
        const size_t tl = chord_tile_lds(n);
        const long long tiles = axis == 0 ? ((long long)vol->ny * vol->nz + kChordTile - 1) / kChordTile
                              : axis == 1 ? (long long)vol->nz * ((vol->nx + kChordTile - 1) / kChordTile)
                                          : ((long long)vol->nx * vol->ny + kChordTile - 1) / kChordTile;
        if (axis == 0)
            hipLaunchKernelGGL(k_chords_tile<0>, dim3((unsigned)tiles), dim3(kChordTile), tl, s, vol->mask, n, vol->nx,
                               vol->ny, vol->nz, (unsigned long long *)hist);
        else if (axis == 1)
            hipLaunchKernelGGL(k_chords_tile<1>, dim3((unsigned)tiles), dim3(kChordTile), tl, s, vol->mask, n, vol->nx,
                               vol->ny, vol->nz, (unsigned long long *)hist);
        else
            hipLaunchKernelGGL(k_chords_tile<2>, dim3((unsigned)tiles), dim3(kChordTile), tl, s, vol->mask, n, vol->nx,
                               vol->ny, vol->nz, (unsigned long long *)hist);
    } else if (lds <= 65536) {
        const unsigned grid = (unsigned)std::min<long long>(1024, (lines + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_chords, dim3(grid), dim3(kThreads), lds, s, vol->mask, axis, n, lines, vol->nx, vol->ny,
                           (unsigned long long *)hist);
    } else {
        hipLaunchKernelGGL(k_chords_global, dim3((unsigned)((lines + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                           vol->mask, axis, n, lines, vol->nx, vol->ny, (unsigned long long *)hist);
    }
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
    if (n > 0) {
        const unsigned grid = (unsigned)std::min<long long>(1024, (n + kThreads - 1) / kThreads);
        if (nbins <= kEscLdsBins)
            hipLaunchKernelGGL(k_escape_hist<true>, dim3(grid), dim3(kThreads), 0, s, rec, (long long)n, bin_width, nbins,
                               th, nthr, (unsigned long long *)hist_w, (unsigned long long *)hist_n,
                               (unsigned long long *)above_w, (unsigned long long *)above_n);
        else
            hipLaunchKernelGGL(k_escape_hist<false>, dim3(grid), dim3(kThreads), 0, s, rec, (long long)n, bin_width,
                               nbins, th, nthr, (unsigned long long *)hist_w, (unsigned long long *)hist_n,
                               (unsigned long long *)above_w, (unsigned long long *)above_n);
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_bright_colocalization(const mc_volume *vol, const int64_t *fluence, int32_t z0, double frac,
                             int64_t *top_count, int64_t *top_solid, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!fluence || !top_count || !top_solid) return fail(MC_EINVAL, "NULL argument");
    if (z0 < 0 || z0 >= vol->nz) return fail(MC_EINVAL, "need 0 <= z0 < nz");
    if (!(frac > 0.0 && frac <= 1.0)) return fail(MC_EINVAL, "frac must be in (0, 1]");
    const long long n = (long long)vol->nx * vol->ny;
    if (n >= 0x7fffffffLL) return fail(MC_EINVAL, "nx * ny must stay below 2^31");
    const long long k = std::min(n, std::max(1LL, (long long)ceil(frac * (double)n)));
    hipLaunchKernelGGL(k_slice_top, dim3((unsigned)(vol->nz - z0)), dim3(kTopThreads), 0, (hipStream_t)hip_stream,
                       (const long long *)fluence, vol->mask, n, (int)z0, k, (long long *)top_count,
                       (long long *)top_solid);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_pore_distance_workspace_bytes(const mc_volume *vol)
{
    clear_error();
    if (check_volume(vol)) return 0;
    return edt_bytes(vol);
}

int mc_pore_distance(const mc_volume *vol, double *dist, void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!dist || !workspace) return fail(MC_EINVAL, "NULL argument");
    const size_t need = mc_pore_distance_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    if (too_large(vol)) return fail(MC_EINVAL, "volume too large for 32-bit squared distances");
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nvox = (size_t)vol->nx * vol->ny * vol->nz;
    const EdtScratch e = edt_layout(vol, workspace);
    if ((rc = enqueue_sqdist(vol, e, s))) return rc;
    int *g = e.g;
    hipLaunchKernelGGL(k_edt_out, dim3(blocks_for((long long)nvox)), dim3(kThreads), 0, s, g, (long long)nvox, dist);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_pore_spearman_workspace_bytes(const mc_volume *vol, int32_t z0)
{
    clear_error();
    if (check_volume(vol) || z0 < 0 || z0 >= vol->nz) return 0;
    const long long npore_max = (long long)vol->nx * vol->ny * (vol->nz - z0);
    if (npore_max >= 0x7fffffffLL) return 0;
    const SpLayout L = sp_layout(vol, z0, npore_max, (hipStream_t)0);
    if (L.status != hipSuccess) {
        fail(MC_EHIP, "sizing the sorts: %s", hipGetErrorString(L.status));
        return 0;
    }
    return L.total;
}

int mc_pore_spearman(const mc_volume *vol, const int64_t *fluence, int32_t z0, double *rho, int64_t *n_pore,
                     void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!fluence || !rho || !n_pore || !workspace) return fail(MC_EINVAL, "NULL argument");
    if (z0 < 0 || z0 >= vol->nz) return fail(MC_EINVAL, "need 0 <= z0 < nz");
    if (too_large(vol)) return fail(MC_EINVAL, "volume too large for 32-bit squared distances");
    const long long n_slice = (long long)vol->nx * vol->ny;
    const long long npore_max = n_slice * (vol->nz - z0);
    if (npore_max >= 0x7fffffffLL) return fail(MC_EINVAL, "nx * ny * (nz - z0) must stay below 2^31");
    hipStream_t s = (hipStream_t)hip_stream;
    const SpLayout L = sp_layout(vol, z0, npore_max, s);
    if (L.status != hipSuccess) return fail(MC_EHIP, "sizing the sorts: %s", hipGetErrorString(L.status));
    if (workspace_bytes < L.total) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    char *b = (char *)workspace;
    const EdtScratch e = edt_layout(vol, b + L.edt);
    if ((rc = enqueue_sqdist(vol, e, s))) return rc;
    const int nseg = vol->nz - z0;
    int *counts = (int *)(b + L.counts), *coff = (int *)(b + L.coff);
    unsigned long long *cmax = (unsigned long long *)(b + L.cmax);
    int *begin = (int *)(b + L.begin), *end = (int *)(b + L.end);
    unsigned long long *stats = (unsigned long long *)(b + L.stats);
    long long *kf = (long long *)(b + L.kf);
    int *kd = (int *)(b + L.kd), *pos = (int *)(b + L.pos), *perm = (int *)(b + L.perm);
    unsigned long long *kc = (unsigned long long *)(b + L.kc), *kc_s = (unsigned long long *)(b + L.kc_s);
    double *rf = (double *)(b + L.rf), *rd = (double *)(b + L.rd);
    const int cps = sp_chunks_per_slice(vol);
    const int nchunks = nseg * cps;
    hipLaunchKernelGGL(k_chunk_pore_count, dim3(nchunks), dim3(kSpThreads), 0, s, vol->mask, n_slice, z0, cps, counts);
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(kSpThreads), 0, s, (const int *)counts, nchunks, cps, coff, begin, end,
                       stats);
    hipLaunchKernelGGL(k_compact, dim3(nchunks), dim3(kSpThreads), 0, s, vol->mask, (const long long *)fluence, e.g,
                       n_slice, z0, cps, (const int *)coff, kf, kd, pos, cmax);
    hipLaunchKernelGGL(k_chunk_max, dim3(1), dim3(kSpThreads), 0, s, (const unsigned long long *)cmax, nchunks, stats);
    HIP_TRY(hipGetLastError());
    // the pore count sizes the sorts and the key maxima fix their bit ranges: bring
    // those three numbers to the host
    unsigned long long st[3] = {0ull, 0ull, 0ull};
    {
        const hipError_t err = hipMemcpyAsync(st, stats, sizeof(st), hipMemcpyDeviceToHost, s);
        const hipError_t err2 = err == hipSuccess ? hipStreamSynchronize(s) : err;
        if (err2 != hipSuccess) return fail(MC_EHIP, "reading the pore count: %s", hipGetErrorString(err2));
    }
    const long long total = (long long)st[0];
    if (total > 0) {
        const unsigned sbits = bit_width((unsigned long long)(nseg - 1));
        const unsigned fbits = bit_width(st[1]), dbits = bit_width(st[2]);
        size_t tmp = L.tmp_bytes;
        if (fbits < 64 && sbits + fbits <= 64) {   // no negative tally, and room for the slice number
            hipLaunchKernelGGL(k_compose<long long>, dim3(nseg), dim3(kSpThreads), 0, s, (const long long *)kf,
                               (const int *)begin, (const int *)end, fbits, kc);
            HIP_TRY(rocprim::radix_sort_pairs(b + L.tmp, tmp, (const unsigned long long *)kc, kc_s, (const int *)pos,
                                              perm, (unsigned)total, 0u, std::max(1u, sbits + fbits), s));
            hipLaunchKernelGGL(k_avg_rank<unsigned long long>, dim3(blocks_for(total)), dim3(256), 0, s,
                               (const unsigned long long *)kc_s, (const int *)perm, (const int *)begin,
                               (const int *)end, nseg, (int)total, rf);
        } else {
            // negative tallies, or tallies too wide to share 64 bits with the slice number
            long long *kf_s = (long long *)kc_s;
            HIP_TRY(rocprim::segmented_radix_sort_pairs(b + L.tmp, tmp, (const long long *)kf, kf_s, (const int *)pos,
                                                        perm, (unsigned)total, (unsigned)nseg, (const int *)begin,
                                                        (const int *)end, 0, 64, s));
            hipLaunchKernelGGL(k_avg_rank<long long>, dim3(blocks_for(total)), dim3(256), 0, s, (const long long *)kf_s,
                               (const int *)perm, (const int *)begin, (const int *)end, nseg, (int)total, rf);
        }
        if (st[2] + 2 <= (unsigned long long)kRankBins) {
            // squared distances are small: rank them by counting in LDS
            const int nbins = (int)st[2] + 1;
            hipLaunchKernelGGL(k_count_rank, dim3(nseg), dim3(kSpThreads), sizeof(unsigned int) * (nbins + 1), s,
                               (const int *)kd, (const int *)begin, (const int *)end, nbins, rd);
        } else {
            // squared distances are below 2^30 and the slice number below 2^31:
            // composite keys always fit
            hipLaunchKernelGGL(k_compose<int>, dim3(nseg), dim3(kSpThreads), 0, s, (const int *)kd, (const int *)begin,
                               (const int *)end, dbits, kc);
            tmp = L.tmp_bytes;
            HIP_TRY(rocprim::radix_sort_pairs(b + L.tmp, tmp, (const unsigned long long *)kc, kc_s, (const int *)pos,
                                              perm, (unsigned)total, 0u, std::max(1u, sbits + dbits), s));
            hipLaunchKernelGGL(k_avg_rank<unsigned long long>, dim3(blocks_for(total)), dim3(256), 0, s,
                               (const unsigned long long *)kc_s, (const int *)perm, (const int *)begin,
                               (const int *)end, nseg, (int)total, rd);
        }
    }
    hipLaunchKernelGGL(k_rank_corr, dim3(nseg), dim3(kSpThreads), 0, s, (const double *)rf, (const double *)rd,
                       (const int *)begin, (const int *)end, rho, (long long *)n_pore);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // extern "C"
