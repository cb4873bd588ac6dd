// Exact top-k marking on the GPU: mask[i] = 1 for the k largest values of an
// array, equal values going to the lower index.  An MSB-first radix select over
// an order-preserving 64-bit key (11-bit digits, six passes) finds the k-th
// largest key T and how many of the keys equal to T are taken; a chunked scan in
// index order then marks them.  Used by the rank binarisation of the spinodal
// generator (double fields) and by the brightest-decile statistics (int64
// fluence tallies).  Every kernel has internal linkage.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.hpp"

namespace pmc {
namespace sel {
namespace {

constexpr int kThreads = 256;
constexpr int kDigitBits = 11;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kChunk = kThreads * 16;      // elements per marking workgroup

struct SelectState {
    unsigned long long prefix;   // key bits chosen so far
    long long k;                 // rank still to find inside the current candidates (1-based, from the top)
    long long pad[6];
};

// order-preserving maps to uint64 (-0.0 and +0.0 map alike)
__device__ __forceinline__ unsigned long long key_of(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v + 0.0);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ unsigned long long key_of(long long v)
{
    return (unsigned long long)v ^ 0x8000000000000000ull;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_hist(const T *__restrict__ f, long long n, const SelectState *st,
                                                   unsigned long long *hist, int shift, int bits)
{
    __shared__ unsigned int h[kDigits];
    for (int i = (int)threadIdx.x; i < kDigits; i += kThreads) h[i] = 0u;
    __syncthreads();
    const int top = shift + bits;
    const unsigned long long hi_mask = top >= 64 ? 0ull : (~0ull << top);
    const unsigned long long prefix = st->prefix;
    const unsigned long long dmask = (1ull << bits) - 1ull;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const unsigned long long key = key_of(f[i]);
        if ((key & hi_mask) == prefix) atomicAdd(&h[(key >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < (1 << bits); i += kThreads)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

__global__ void k_select(SelectState *st, unsigned long long *hist, int shift, int bits)
{
    if (threadIdx.x == 0) {
        long long k = st->k, above = 0;
        int d = (1 << bits) - 1;
        for (; d > 0; --d) {
            if (above + (long long)hist[d] >= k) break;
            above += (long long)hist[d];
        }
        st->k = k - above;
        st->prefix |= (unsigned long long)d << shift;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < kDigits; i += (int)blockDim.x) hist[i] = 0ull;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_count_eq(const T *__restrict__ f, long long n, const SelectState *st,
                                                       long long *counts)
{
    __shared__ int wsum[kThreads / 64];
    const unsigned long long key_t = st->prefix;
    const long long base = (long long)blockIdx.x * kChunk;
    int c = 0;
    for (int it = 0; it < kChunk / kThreads; ++it) {
        const long long i = base + it * kThreads + threadIdx.x;
        if (i < n && key_of(f[i]) == key_t) ++c;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += wsum[w];
        counts[blockIdx.x] = t;
    }
}

// exclusive scan of the per-chunk counts, one workgroup: each thread scans a
// contiguous segment
__global__ __launch_bounds__(kThreads) void k_scan(long long *counts, int nchunks)
{
    __shared__ long long seg[kThreads];
    const int per = (nchunks + kThreads - 1) / kThreads;
    const int b0 = (int)threadIdx.x * per, b1 = std::min(nchunks, b0 + per);
    long long s = 0;
    for (int b = b0; b < b1; ++b) s += counts[b];
    seg[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int t = 0; t < kThreads; ++t) {
            const long long v = seg[t];
            seg[t] = run;
            run += v;
        }
    }
    __syncthreads();
    long long run = seg[threadIdx.x];
    for (int b = b0; b < b1; ++b) {
        const long long v = counts[b];
        counts[b] = run;
        run += v;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_mark(const T *__restrict__ f, long long n, const SelectState *st,
                                                   const long long *__restrict__ offsets, uint8_t *mask)
{
    __shared__ int wcount[kThreads / 64];
    const unsigned long long key_t = st->prefix;
    const long long need = st->k;
    const long long base = (long long)blockIdx.x * kChunk;
    long long run = offsets[blockIdx.x];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    for (int it = 0; it < kChunk / kThreads; ++it) {
        const long long i = base + it * kThreads + threadIdx.x;
        unsigned long long key = 0ull;
        if (i < n) key = key_of(f[i]);
        const bool eq = i < n && key == key_t;
        const unsigned long long bal = __ballot(eq);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wave; ++w) woff += wcount[w];
        int tot = 0;
        for (int w = 0; w < kThreads / 64; ++w) tot += wcount[w];
        if (i < n) mask[i] = (uint8_t)(key > key_t || (eq && run + woff + before < need));
        run += tot;
        __syncthreads();
    }
}

__global__ void k_fill_u8(uint8_t *p, long long n, uint8_t v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_init_state(SelectState *st, unsigned long long *hist, long long k)
{
    if (threadIdx.x == 0) {
        st->prefix = 0ull;
        st->k = k;
    }
    for (int i = (int)threadIdx.x; i < kDigits; i += (int)blockDim.x) hist[i] = 0ull;
}

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// device workspace of enqueue_top for n elements
inline size_t workspace_bytes(long long n)
{
    const size_t nchunks = (size_t)((n + kChunk - 1) / kChunk);
    return align256(sizeof(SelectState)) + align256(sizeof(unsigned long long) * kDigits) +
           align256(sizeof(long long) * nchunks);
}

// mask = the k largest of f[0..n) (ties to the lower index), 1 <= n, 0 <= k <= n;
// asynchronous on s.  The caller has validated the arguments and the workspace.
template <typename T>
int enqueue_top(const T *f, long long n, long long k, uint8_t *mask, void *ws, hipStream_t s)
{
    const unsigned grid = (unsigned)std::min<long long>(4096, (n + kThreads - 1) / kThreads);
    if (k == 0 || k == n) {
        hipLaunchKernelGGL(k_fill_u8, dim3(grid), dim3(kThreads), 0, s, mask, n, (uint8_t)(k == n ? 1 : 0));
        HIP_TRY(hipGetLastError());
        return MC_OK;
    }
    char *b = (char *)ws;
    SelectState *st = (SelectState *)b;
    unsigned long long *hist = (unsigned long long *)(b + align256(sizeof(SelectState)));
    long long *counts = (long long *)(b + align256(sizeof(SelectState)) + align256(sizeof(unsigned long long) * kDigits));
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(kThreads), 0, s, st, hist, k);
    // digits from the top: bits 63..53, 52..42, 41..31, 30..20, 19..9, 8..0
    for (int shift = 64 - kDigitBits; shift > -kDigitBits; shift -= kDigitBits) {
        const int sh = std::max(shift, 0);
        const int bits = shift >= 0 ? kDigitBits : kDigitBits + shift;
        hipLaunchKernelGGL(k_hist<T>, dim3(grid), dim3(kThreads), 0, s, f, n, st, hist, sh, bits);
        hipLaunchKernelGGL(k_select, dim3(1), dim3(kThreads), 0, s, st, hist, sh, bits);
    }
    const long long nchunks = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_count_eq<T>, dim3((unsigned)nchunks), dim3(kThreads), 0, s, f, n, st, counts);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kThreads), 0, s, counts, (int)nchunks);
    hipLaunchKernelGGL(k_mark<T>, dim3((unsigned)nchunks), dim3(kThreads), 0, s, f, n, st, counts, mask);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // namespace
}  // namespace sel
}  // namespace pmc
