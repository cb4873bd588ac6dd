// spinodal.hip -- Cahn-Hilliard spinodal mask generator (Sec. 2.2, Eq. CH,
// Eq. CH_spectral; App. A): the semi-implicit Fourier spectral step in FP64,
// the radial power spectral density of the stopping rule, and the exact rank
// binarisation.
//
// Design (gfx950): the spectrum lives in HBM as complex double [nz][ny][nx/2+1].
// Every transform is a Stockham FFT (radices 2, 3, 4) over whole lines held in
// LDS, 4096 complex values per 256-thread workgroup, so one line is read and
// written once per pass.  One time step is four in-place passes over the
// spectrum-sized work array W, with the state S touched only in the z pass:
//   y pass   W <- inverse FFT_y(W)
//   x pass   W <- FFT_x(f'(inverse FFT_x(W)))       (real field only in LDS)
//   y pass   W <- FFT_y(W)
//   z pass   S <- (S - dt k^2 FFT_z(W)) / (1 + dt kappa k^4);  W <- inverse FFT_z(S)
// i.e. ten spectrum-sized transfers per step instead of the fifteen of two
// separate 3-D transforms and an update.  Columns along y and z are read as
// tiles of consecutive kx (contiguous in memory) and transformed as lines in LDS.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "select.hpp"
#include "analytics.h"
#include "spinodal.h"

using namespace pmc::host;

// The transforms and the update may contract multiply-adds into FMAs: unlike the
// photon walk, nothing here has to be bitwise independent of launch shape, and a
// given binary still gives the same bits on every run.
#pragma clang fp contract(fast)

namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 4096;           // complex doubles transformed per workgroup (64 KiB)
constexpr int kColRadixLog = 2;           // k_colpass keeps radix-4 stages (measured faster there)
constexpr int kColElems = kLdsElems + 64; // LDS of the column passes: lines padded to n + 1
constexpr int kMaxStages = 12;
constexpr int kMaxN = 1024;
constexpr int kTwElems = 768;             // LDS twiddles: n/2 for even n (w(m + n/2) = -w(m)), n for odd n <= 729
constexpr int kPadElems = 4400;           // LDS of the compile-time lengths: lines padded by one per 16
constexpr int kPadTw = 528;               // their twiddles: n/2 padded by one per 32
// The x pass of the compile-time lengths takes 2048 complex values per workgroup
// (two or more line pairs): 35 KB of LDS with the padding, 43 KB with the
// twiddles, so three workgroups share a CU (at 1024: 2003 us against 2200 with
// 4096 values, two workgroups per CU, and 2185 with 1024 values, one pair).
constexpr int kXElems = 2048;
constexpr int kXPadElems = 2200;

// LDS index of element i of a line: the compile-time lengths insert one pad
// element per 16 (and one per 32 in the twiddle table), which spreads the
// strided accesses of the early and middle stages over the banks.
template <int N> __device__ __forceinline__ int pidx(int i) { return N > 0 ? i + (i >> 4) : i; }
template <int N> __device__ __forceinline__ int tidx(int i) { return N > 0 ? i + (i >> 5) : i; }

// Host-side geometry of the LDS layouts (must match the kernels).
constexpr bool static_length(int n) { return n == 1024 || n == 512 || n == 384 || n == 256; }
inline int line_stride(int n, bool column)
{
    return static_length(n) ? n + n / 16 + (column ? 1 : 0) : n + (column ? 1 : 0);
}

// Per-stage constants, with FP32 reciprocals for the index divisions.
struct Plan {
    int32_t n;
    int32_t nstages;
    int32_t radix[kMaxStages];
    int32_t ns[kMaxStages];        // product of the radices before the stage
    float inv_nb[kMaxStages];      // 1 / (n / radix)
    float inv_ns[kMaxStages];      // 1 / ns
};

// x / d for 0 <= x < 2^22 and 1 <= d < 2^22, with inv = 1/d in FP32: the
// product is off by at most one, which the remainder corrects.
__device__ __forceinline__ int fdiv(int x, int d, float inv)
{
    int q = (int)((float)x * inv);
    const int r = x - q * d;
    if (r < 0) q -= 1;
    else if (r >= d) q += 1;
    return q;
}

// radix-3 stages first, then radix 4, then one radix 2 if the power of two is odd
bool make_plan(int n, Plan *p)
{
    memset(p, 0, sizeof *p);
    p->n = n;
    int m = n, threes = 0, twos = 0;
    while (m % 3 == 0) { m /= 3; ++threes; }
    while (m % 2 == 0) { m /= 2; ++twos; }
    if (m != 1) return false;
    int s = 0;
    for (int i = 0; i < threes; ++i) p->radix[s++] = 3;
    for (int i = 0; i < twos / 2; ++i) p->radix[s++] = 4;
    if (twos % 2) p->radix[s++] = 2;
    p->nstages = s;
    int ns = 1;
    for (int i = 0; i < s; ++i) {
        p->ns[i] = ns;
        p->inv_nb[i] = 1.0f / (float)(n / p->radix[i]);
        p->inv_ns[i] = 1.0f / (float)ns;
        ns *= p->radix[i];
    }
    return s <= kMaxStages;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Small DFTs, forward (sign -1) or inverse (sign +1).
template <int R> __device__ __forceinline__ void dft(double2 *v, bool inv);

template <> __device__ __forceinline__ void dft<2>(double2 *v, bool)
{
    const double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
}

template <> __device__ __forceinline__ void dft<4>(double2 *v, bool inv)
{
    const double2 s02 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
    const double2 d02 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
    const double2 s13 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
    const double2 d13 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
    // forward: -i d13; inverse: +i d13
    const double2 r = inv ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
    v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
    v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
    v[1] = make_double2(d02.x + r.x, d02.y + r.y);
    v[3] = make_double2(d02.x - r.x, d02.y - r.y);
}

// radix 8: two radix-4 DFTs of the even and odd inputs, joined with w8^k
template <> __device__ __forceinline__ void dft<8>(double2 *v, bool inv)
{
    constexpr double h = 0.70710678118654752440;   // sqrt(2)/2
    const double sg = inv ? 1.0 : -1.0;
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e, inv);
    dft<4>(o, inv);
    const double2 t[4] = {o[0], make_double2(h * (o[1].x - sg * o[1].y), h * (o[1].y + sg * o[1].x)),
                          make_double2(-sg * o[2].y, sg * o[2].x),
                          make_double2(-h * (o[3].x + sg * o[3].y), h * (sg * o[3].x - o[3].y))};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = make_double2(e[k].x + t[k].x, e[k].y + t[k].y);
        v[k + 4] = make_double2(e[k].x - t[k].x, e[k].y - t[k].y);
    }
}

// radix 16 as 4 x 4: radix-4 DFTs over n1 of v[4 n1 + n2], twiddles w16^(n2 k1),
// radix-4 DFTs over n2 giving X[k1 + 4 k2]
template <> __device__ __forceinline__ void dft<16>(double2 *v, bool inv)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    // cos and sin of 2 pi m / 16, m = 0..9
    constexpr double kc[10] = {1.0, c1, h, s1, 0.0, -s1, -h, -c1, -1.0, -c1};
    constexpr double ks[10] = {0.0, s1, h, c1, 1.0, c1, h, s1, 0.0, -s1};
    const double sg = inv ? 1.0 : -1.0;
    double2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        double2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
        dft<4>(t, inv);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            const int m = n2 * k1;
            a[n2][k1] = m == 0 ? t[k1] : cmul(t[k1], make_double2(kc[m], sg * ks[m]));
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        double2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft<4>(t, inv);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
}

template <> __device__ __forceinline__ void dft<3>(double2 *v, bool inv)
{
    constexpr double kS = 0.86602540378443864676;  // sqrt(3)/2
    const double2 t = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
    const double2 u = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
    const double2 m = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    // forward: y1 = m - i s u, y2 = m + i s u; inverse swaps them
    const double2 isu = make_double2(-kS * u.y, kS * u.x);
    v[0] = make_double2(v[0].x + t.x, v[0].y + t.y);
    if (!inv) {
        v[1] = make_double2(m.x - isu.x, m.y - isu.y);
        v[2] = make_double2(m.x + isu.x, m.y + isu.y);
    } else {
        v[1] = make_double2(m.x + isu.x, m.y + isu.y);
        v[2] = make_double2(m.x - isu.x, m.y - isu.y);
    }
}

// One Stockham stage of radix R over `nlines` lines of length n in LDS (line l
// at buf + l * ls): butterfly j of a line reads elements j + r n/R, twiddles
// them by w^(r (j mod ns)) with w = exp(-+ 2 pi i / (ns R)), transforms, and
// writes them to (j / ns) ns R + (j mod ns) + r ns.  Values wait in registers
// between the read and the write barrier, so one LDS buffer suffices.
template <int R>
__device__ __forceinline__ void stage(double2 *buf, int n, int ns, int nlines, int ls, bool inv, const double2 *tw,
                                      float inv_nb, float inv_ns)
{
    constexpr int kPer = (kLdsElems / R + kThreads - 1) / kThreads;
    const int nb = n / R;
    const int total = nlines * nb;
    const int tstep = n / (ns * R);
    double2 v[kPer][R];
    int dst[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int b = (int)threadIdx.x + q * kThreads;
        dst[q] = -1;
        if (b < total) {
            const int line = fdiv(b, nb, inv_nb), j = b - line * nb;
            const int jm = j - fdiv(j, ns, inv_ns) * ns;
            const double2 *src = buf + line * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = src[j + r * nb];
                if (r) {
                    int m = jm * r * tstep;
                    double sg = 1.0;
                    if (!(n & 1) && m >= (n >> 1)) {
                        m -= n >> 1;
                        sg = -1.0;
                    }
                    double2 w = tw[m];
                    w.x *= sg;
                    w.y *= inv ? -sg : sg;
                    x = cmul(x, w);
                }
                v[q][r] = x;
            }
            dft<R>(v[q], inv);
            dst[q] = line * ls + (j - jm) * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (dst[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[q] + r * ns] = v[q][r];
        }
    }
    __syncthreads();
}

// Copy the twiddles a transform of length n reads into LDS: the first n/2 when n
// is even, all n when n is odd.
template <int N>
__device__ __forceinline__ void load_twiddles(double2 *tw_s, const double2 *__restrict__ tw, int n)
{
    const int m = (n & 1) ? n : n >> 1;
    for (int i = (int)threadIdx.x; i < m; i += kThreads) tw_s[tidx<N>(i)] = tw[i];
}

// Unnormalised FFT of every line (forward: exp(-2 pi i j k / n)); tw is the
// table staged by load_twiddles.
__device__ void fft_lines(double2 *buf, int ls, int nlines, const Plan &P, const double2 *tw, bool inv)
{
    for (int s = 0; s < P.nstages; ++s) {
        const int R = P.radix[s], ns = P.ns[s];
        if (R == 4) stage<4>(buf, P.n, ns, nlines, ls, inv, tw, P.inv_nb[s], P.inv_ns[s]);
        else if (R == 2) stage<2>(buf, P.n, ns, nlines, ls, inv, tw, P.inv_nb[s], P.inv_ns[s]);
        else stage<3>(buf, P.n, ns, nlines, ls, inv, tw, P.inv_nb[s], P.inv_ns[s]);
    }
}

// Compile-time plans for the common extents, every divisor and stride a
// constant: the radix-3 stages, then the power of two 2^t in ceil(t / 4) stages
// of radix 16, 8, 4 or 2 as even as possible (1024 = 16 8 8, 512 = 8 8 8,
// 384 = 3 16 8, 256 = 16 16): fewer passes through LDS than radix 4.
constexpr int c_threes(int n) { int t = 0; while (n % 3 == 0) { n /= 3; ++t; } return t; }
constexpr int c_twos(int n) { while (n % 3 == 0) n /= 3; int t = 0; while (n % 2 == 0) { n /= 2; ++t; } return t; }
// ML: largest radix 2^ML (4: up to 16; 2: radix 4 only)
constexpr int c_two_stages(int n, int ML) { return (c_twos(n) + ML - 1) / ML; }
constexpr int c_stages(int n, int ML) { return c_threes(n) + c_two_stages(n, ML); }
constexpr int c_radix(int n, int s, int ML)
{
    const int t3 = c_threes(n);
    if (s < t3) return 3;
    const int S = c_two_stages(n, ML), t2 = c_twos(n), i = s - t3;
    return 1 << (t2 / S + (i < t2 % S ? 1 : 0));
}
constexpr int c_ns(int n, int s, int ML)
{
    int p = 1;
    for (int i = 0; i < s; ++i) p *= c_radix(n, i, ML);
    return p;
}

template <int R, int N, int NS, bool INV>
__device__ __forceinline__ void stage_c(double2 *buf, int ls, int nlines, const double2 *tw)
{
    constexpr int NB = N / R;
    constexpr int TSTEP = N / (NS * R);
    constexpr int kPer = (kLdsElems / R + kThreads - 1) / kThreads;
    const int total = nlines * NB;
    double2 v[kPer][R];
    int dst[kPer], dst2[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int b = (int)threadIdx.x + q * kThreads;
        dst[q] = -1;
        dst2[q] = 0;
        if (b < total) {
            const int line = b / NB, j = b - line * NB;
            const int jm = j % NS;
            const double2 *src = buf + line * ls;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = src[pidx<N>(j + r * NB)];
                if (r) {
                    int m = jm * r * TSTEP;
                    double2 w;
                    if constexpr ((N & 1) == 0) {
                        const bool hi = m >= N / 2;
                        w = tw[tidx<N>(hi ? m - N / 2 : m)];
                        if (hi) w = make_double2(-w.x, -w.y);
                    } else {
                        w = tw[tidx<N>(m)];
                    }
                    if (INV) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[q][r] = x;
            }
            dft<R>(v[q], INV);
            dst[q] = line * ls;
            dst2[q] = (j - jm) * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (dst[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[q] + pidx<N>(dst2[q] + r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int N, int S, bool INV, int ML>
__device__ __forceinline__ void fft_c(double2 *buf, int ls, int nlines, const double2 *tw)
{
    if constexpr (S < c_stages(N, ML)) {
        stage_c<c_radix(N, S, ML), N, c_ns(N, S, ML), INV>(buf, ls, nlines, tw);
        fft_c<N, S + 1, INV, ML>(buf, ls, nlines, tw);
    }
}

// Transform dispatch: N > 0 selects the compile-time plan for that length, with
// radices up to 2^ML.
template <int N, int ML = 4>
__device__ __forceinline__ void fft_any(double2 *buf, int ls, int nlines, const Plan &P, const double2 *tw, bool inv)
{
    if constexpr (N > 0) {
        if (inv) fft_c<N, 0, true, ML>(buf, ls, nlines, tw);
        else fft_c<N, 0, false, ML>(buf, ls, nlines, tw);
    } else {
        fft_lines(buf, ls, nlines, P, tw, inv);
    }
}

// Tables: forward twiddles exp(-2 pi i m / n) and k^2 = (2 pi m' / n)^2 with m'
// the signed frequency of index m (the rfft axis x keeps m' = m).
__global__ void k_tables(double2 *tw, double *k2, int n, int half)
{
    const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m < n) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = make_double2(c, -s);
    }
    const int nk = half ? n / 2 + 1 : n;
    if (m < nk) {
        const int ms = (!half && m >= (n + 1) / 2) ? m - n : m;
        const double k = (2.0 * M_PI) * ((double)ms * (1.0 / (double)n));
        k2[m] = k * k;
    }
}

// Cooperative copy of `total` elements: each thread issues U global loads before
// it writes any of them, so U loads per thread are in flight at once.
template <int U, class T, class Load, class Store>
__device__ __forceinline__ void gather(int total, Load load, Store store)
{
    for (int e0 = (int)threadIdx.x; e0 < total; e0 += U * kThreads) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * kThreads;
            if (e < total) v[u] = load(e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * kThreads;
            if (e < total) store(e, v[u]);
        }
    }
}

enum { X_INIT = 0, X_NONLIN = 1, X_FIELD = 2, X_MASK = 3 };

// Lines along x.  X_INIT: real line -> forward transform, half spectrum out;
// X_MASK: the same from a uint8 mask line (0 or 1 as doubles).
// X_NONLIN: half spectrum -> inverse -> f'(phi) -> forward -> half spectrum.
// X_FIELD: half spectrum -> inverse -> real line out.  `scale` = 1/(nx ny nz).
//
// Two real lines share one complex transform: lines a = 2m and b = 2m + 1 of
// the workgroup travel as z = a + i b.  Forward, A_k = (Z_k + conj Z_(n-k)) / 2
// and B_k = (Z_k - conj Z_(n-k)) / 2i; inverse, Z_k = A_k + i B_k over the
// Hermitian extensions of A and B, and a, b are the real and imaginary parts of
// the result.  The imaginary parts of bins 0 and n/2 are dropped, as a real
// inverse transform drops them.  While loading, A_j sits at j and B_j at n - j
// (0 < j < n/2), their real bins 0 and n/2 in the two halves of slots 0 and n/2,
// so a pair needs exactly n slots.  `L` is the number of lines per workgroup
// (even except in the last workgroup).
template <int MODE, int N>
__global__ __launch_bounds__(kThreads) void k_xpass(const double *__restrict__ rin, double2 *spec,
                                                     double *__restrict__ rout, int nx, int nlines_total, int L,
                                                     Plan P, const double2 *__restrict__ tw, double scale,
                                                     const uint8_t *__restrict__ mask_in)
{
    __shared__ double2 buf[N > 0 ? kXPadElems : kLdsElems];
    __shared__ double2 tw_s[N > 0 ? kPadTw : kTwElems];
    load_twiddles<N>(tw_s, tw, nx);
    double *bd = reinterpret_cast<double *>(buf);   // bd[2 p] = buf[p].x, bd[2 p + 1] = buf[p].y
    const int hx = nx / 2 + 1, half = nx / 2, ls = N > 0 ? nx + nx / 16 : nx;
    const int line0 = (int)blockIdx.x * L;
    const int nl = min(L, nlines_total - line0);
    const int np = (nl + 1) >> 1;
    const int tid = (int)threadIdx.x;
    const float inv_nx = 1.0f / (float)nx, inv_hx = 1.0f / (float)hx;
    if (MODE == X_INIT || MODE == X_MASK) {
        // the block's lines are contiguous in memory
        const double *src = rin + (size_t)line0 * nx;
        const uint8_t *msrc = mask_in + (size_t)line0 * nx;
        gather<8, double>(
            nl * nx, [&](int e) { return MODE == X_MASK ? (double)msrc[e] : src[e]; },
            [&](int e, double v) {
                const int l = fdiv(e, nx, inv_nx), x = e - l * nx;
                bd[2 * ((l >> 1) * ls + pidx<N>(x)) + (l & 1)] = v;
            });
        if (nl & 1)
            for (int x = tid; x < nx; x += kThreads) bd[2 * ((nl >> 1) * ls + pidx<N>(x)) + 1] = 0.0;
        __syncthreads();
    } else {
        const double2 *src = spec + (size_t)line0 * hx;
        gather<8, double2>(
            nl * hx, [&](int e) { return src[e]; },
            [&](int e, double2 v) {
                const int l = fdiv(e, hx, inv_hx), j = e - l * hx;
                const int base = (l >> 1) * ls;
                if (j == 0 || j == half) bd[2 * (base + pidx<N>(j)) + (l & 1)] = v.x;
                else buf[base + pidx<N>((l & 1) ? nx - j : j)] = v;
            });
        if (nl & 1) {                                  // the last pair has no b line
            const int base = (nl >> 1) * ls;
            for (int j = tid; j <= half; j += kThreads) {
                if (j == 0 || j == half) bd[2 * (base + pidx<N>(j)) + 1] = 0.0;
                else buf[base + pidx<N>(nx - j)] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        const int nk = half - 1;                        // bins 0 < k < n/2 of every pair
        if (nk > 0) {
            const float inv_nk = 1.0f / (float)nk;
            for (int e = tid; e < np * nk; e += kThreads) {
                const int m = fdiv(e, nk, inv_nk), k = 1 + (e - m * nk);
                const int pa = m * ls + pidx<N>(k), pb = m * ls + pidx<N>(nx - k);
                const double2 a = buf[pa], b = buf[pb];
                buf[pa] = make_double2(a.x - b.y, a.y + b.x);
                buf[pb] = make_double2(a.x + b.y, b.x - a.y);
            }
        }
        __syncthreads();
        fft_any<N>(buf, ls, np, P, tw_s, true);
        if (MODE == X_FIELD) {
            for (int e = tid; e < nl * nx; e += kThreads) {
                const int l = fdiv(e, nx, inv_nx), x = e - l * nx;
                rout[(size_t)(line0 + l) * nx + x] = bd[2 * ((l >> 1) * ls + pidx<N>(x)) + (l & 1)] * scale;
            }
            return;
        }
        for (int e = tid; e < np * nx; e += kThreads) {
            const int m = fdiv(e, nx, inv_nx), x = e - m * nx;
            const int p = m * ls + pidx<N>(x);
            const double2 z = buf[p];
            const double a = z.x * scale, b = z.y * scale;
            buf[p] = make_double2(2.0 * a * (1.0 - a) * (1.0 - 2.0 * a), 2.0 * b * (1.0 - b) * (1.0 - 2.0 * b));
        }
        __syncthreads();
    }
    fft_any<N>(buf, ls, np, P, tw_s, false);
    for (int e = tid; e < nl * hx; e += kThreads) {
        const int l = fdiv(e, hx, inv_hx), k = e - l * hx;
        const int base = (l >> 1) * ls;
        const double2 zk = buf[base + pidx<N>(k)], zr = buf[base + pidx<N>(k == 0 ? 0 : nx - k)];
        spec[(size_t)(line0 + l) * hx + k] = (l & 1) ? make_double2(0.5 * (zk.y + zr.y), -0.5 * (zk.x - zr.x))
                                                     : make_double2(0.5 * (zk.x + zr.x), 0.5 * (zk.y - zr.y));
    }
}

// Workgroup ids are dealt to the 8 XCDs in turn; give each XCD a contiguous
// range of tiles instead, so that neighbouring tiles, which share 128-byte
// lines, meet in the same L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_order(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

// Column addressing: element j of column (plane p, kx = x0 + c).  Along y the
// plane is z; along z the plane is y.
template <int AXIS>
__device__ __forceinline__ size_t col_addr(int j, int p, int x, int ny, int hx)
{
    return AXIS == 1 ? ((size_t)p * ny + j) * hx + x : ((size_t)j * ny + p) * hx + x;
}

// In-place FFT along y (AXIS 1) or z (AXIS 2) of T-column tiles.
template <int AXIS, int N>
__global__ __launch_bounds__(kThreads) void k_colpass(double2 *A, int ny, int hx, int n, int T, int tiles, Plan P,
                                                       const double2 *__restrict__ tw, int inv)
{
    __shared__ double2 buf[N > 0 ? kPadElems : kColElems];
    __shared__ double2 tw_s[N > 0 ? kPadTw : kTwElems];
    load_twiddles<N>(tw_s, tw, n);
    const int bid = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int p = bid / tiles, tile = bid - p * tiles;
    // lines padded to an odd stride: the transposing loads hit distinct banks
    const int x0 = tile * T, nc = min(T, hx - x0), ls = (N > 0 ? n + n / 16 : n) + 1;
    const int tid = (int)threadIdx.x;
    const float inv_nc = 1.0f / (float)nc;
    gather<8, double2>(
        n * nc,
        [&](int e) {
            const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
            return A[col_addr<AXIS>(j, p, x0 + c, ny, hx)];
        },
        [&](int e, double2 v) {
            const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
            buf[c * ls + pidx<N>(j)] = v;
        });
    __syncthreads();
    fft_any<N, kColRadixLog>(buf, ls, nc, P, tw_s, inv != 0);
    for (int e = tid; e < n * nc; e += kThreads) {
        const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
        A[col_addr<AXIS>(j, p, x0 + c, ny, hx)] = buf[c * ls + pidx<N>(j)];
    }
}

enum { Z_INV = 0, Z_INIT = 1, Z_UPDATE = 2 };

// The z pass.  Z_INV: W = inverse FFT_z(S).  Z_INIT: S = FFT_z(W).  Z_UPDATE:
// S = (S - dt k^2 FFT_z(W)) / (1 + dt kappa k^4) (Eq. CH_spectral, evaluated in
// that order).  With write_w (Z_INIT, Z_UPDATE) W = inverse FFT_z(S) as well, the
// start of the next step.
template <int MODE, int N>
__global__ __launch_bounds__(kThreads) void k_zpass(double2 *S, double2 *W, int ny, int hx, int nz, int T, int tiles,
                                                     Plan P, const double2 *__restrict__ tw,
                                                     const double *__restrict__ kx2, const double *__restrict__ ky2,
                                                     const double *__restrict__ kz2, double dt, double kappa,
                                                     int write_w)
{
    __shared__ double2 buf[N > 0 ? kPadElems : kColElems];
    __shared__ double2 tw_s[N > 0 ? kPadTw : kTwElems];
    load_twiddles<N>(tw_s, tw, nz);
    const int bid = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int y = bid / tiles, tile = bid - y * tiles;
    const int x0 = tile * T, nc = min(T, hx - x0), ls = (N > 0 ? nz + nz / 16 : nz) + 1;
    const int tid = (int)threadIdx.x;
    const float inv_nc = 1.0f / (float)nc;
    const double2 *src = MODE == Z_INV ? S : W;
    gather<8, double2>(
        nz * nc,
        [&](int e) {
            const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
            return src[col_addr<2>(j, y, x0 + c, ny, hx)];
        },
        [&](int e, double2 v) {
            const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
            buf[c * ls + pidx<N>(j)] = v;
        });
    __syncthreads();
    if (MODE != Z_INV) {
        fft_any<N>(buf, ls, nc, P, tw_s, false);
        const double dtk = dt * kappa;
        // the old state comes in with U loads in flight per thread (Z_UPDATE);
        // Z_INIT stores the transform as the state
        gather<8, double2>(
            nz * nc,
            [&](int e) {
                if (MODE != Z_UPDATE) return make_double2(0.0, 0.0);
                const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
                return S[col_addr<2>(j, y, x0 + c, ny, hx)];
            },
            [&](int e, double2 s) {
                const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
                double2 v = buf[c * ls + pidx<N>(j)];
                if (MODE == Z_UPDATE) {
                    const double k2 = kz2[j] + ky2[y] + kx2[x0 + c];
                    const double den = 1.0 + dtk * k2 * k2;
                    const double g = dt * k2;
                    v = make_double2((s.x - g * v.x) / den, (s.y - g * v.y) / den);
                }
                S[col_addr<2>(j, y, x0 + c, ny, hx)] = v;
                buf[c * ls + pidx<N>(j)] = v;
            });
        __syncthreads();
        if (!write_w) return;
    }
    fft_any<N>(buf, ls, nc, P, tw_s, true);
    for (int e = tid; e < nz * nc; e += kThreads) {
        const int j = fdiv(e, nc, inv_nc), c = e - j * nc;
        W[col_addr<2>(j, y, x0 + c, ny, hx)] = buf[c * ls + pidx<N>(j)];
    }
}

// Radial PSD: per-block partial shell sums in LDS, then a fixed-order sum over
// the blocks.
constexpr int kPsdBlocks = 512;

__global__ __launch_bounds__(kThreads) void k_psd_partial(const double2 *__restrict__ S, int nx, int ny, int nz,
                                                          const double *__restrict__ kx2,
                                                          const double *__restrict__ ky2,
                                                          const double *__restrict__ kz2, double *partial, int nb)
{
    __shared__ double bins[kMaxN / 2 + 1];
    for (int i = (int)threadIdx.x; i < nb; i += kThreads) bins[i] = 0.0;
    __syncthreads();
    const int hx = nx / 2 + 1;
    const int nmax = max(nx, max(ny, nz));
    const size_t total = (size_t)nz * ny * hx;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (size_t)gridDim.x * kThreads) {
        const int x = (int)(i % hx);
        const size_t r = i / hx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        if (i == 0) continue;
        const double k2 = kz2[z] + ky2[y] + kx2[x];
        const int s = (int)floor(sqrt(k2) * (double)nmax / (2.0 * M_PI) + 0.5);
        if (s >= nb) continue;
        const double2 v = S[i];
        const double w = (x == 0 || 2 * x == nx) ? 1.0 : 2.0;
        atomicAdd(&bins[s], (v.x * v.x + v.y * v.y) * w);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < nb; i += kThreads) partial[(size_t)blockIdx.x * nb + i] = bins[i];
}

// one workgroup per shell: the partial sums of the shell, tree-reduced in LDS in a
// fixed order
__global__ __launch_bounds__(kThreads) void k_psd_sum(const double *__restrict__ partial, int nblocks, int nb,
                                                      double *psd)
{
    __shared__ double red[kThreads];
    const int s = (int)blockIdx.x;
    double acc = 0.0;
    for (int b = (int)threadIdx.x; b < nblocks; b += kThreads) acc += partial[(size_t)b * nb + s];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) psd[s] = red[0];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Geo {
    int nx, ny, nz, hx;
    size_t spec_elems;      // nz * ny * hx
    Plan px, py, pz;
    int Lx;                 // x lines per workgroup
    int Ty, Tz, tiles_y, tiles_z;
    // workspace offsets (bytes)
    size_t w_off, twx, twy, twz, kx2, ky2, kz2, psd_off, total;
};

int geometry(const mc_ch_grid *g, Geo *G)
{
    if (!g) return fail(MC_EINVAL, "grid is NULL");
    if (g->reserved != 0) return fail(MC_EINVAL, "mc_ch_grid.reserved must be 0");
    if (g->nx < 2 || g->nx > kMaxN || (g->nx & 1)) return fail(MC_EINVAL, "nx must be even, 2..%d", kMaxN);
    if (g->ny < 1 || g->ny > kMaxN || g->nz < 1 || g->nz > kMaxN) return fail(MC_EINVAL, "ny, nz must be 1..%d", kMaxN);
    if ((long long)g->nx * g->ny * g->nz >= (1ll << 31)) return fail(MC_EINVAL, "nx*ny*nz must be < 2^31");
    if (!(g->kappa > 0.0) || !isfinite(g->kappa) || !(g->dt > 0.0) || !isfinite(g->dt))
        return fail(MC_EINVAL, "kappa and dt must be finite and > 0");
    memset(G, 0, sizeof *G);
    G->nx = g->nx;
    G->ny = g->ny;
    G->nz = g->nz;
    G->hx = g->nx / 2 + 1;
    if (!make_plan(g->nx, &G->px) || !make_plan(g->ny, &G->py) || !make_plan(g->nz, &G->pz))
        return fail(MC_EINVAL, "every extent must be a product of powers of 2 and 3");
    G->spec_elems = (size_t)G->nz * G->ny * G->hx;
    // two real lines per complex transform
    G->Lx = 2 * std::max(1, (static_length(G->nx) ? kXElems : kLdsElems) / G->nx);
    // column tiles: padded lines must fit the LDS buffer and the stage registers
    auto tile = [](int n, int lds_static, int elems_static) {
        const int lds = static_length(n) ? lds_static : kColElems;
        const int elems = static_length(n) ? elems_static : kLdsElems;
        return std::max(1, std::min(lds / line_stride(n, true), elems / n));
    };
    G->Ty = tile(G->ny, kPadElems, kLdsElems);
    // the full tile for z too: half-size z tiles (three workgroups per CU, 80-byte
    // column runs) measured slower, 3602 against 3468 us at 384 x 1024 x 1024
    G->Tz = tile(G->nz, kPadElems, kLdsElems);
    G->tiles_y = (G->hx + G->Ty - 1) / G->Ty;
    G->tiles_z = (G->hx + G->Tz - 1) / G->Tz;
    size_t off = 0;
    G->w_off = off;
    off += align_up(G->spec_elems * sizeof(double2));
    G->twx = off;
    off += align_up(sizeof(double2) * G->nx);
    G->twy = off;
    off += align_up(sizeof(double2) * G->ny);
    G->twz = off;
    off += align_up(sizeof(double2) * G->nz);
    G->kx2 = off;
    off += align_up(sizeof(double) * G->hx);
    G->ky2 = off;
    off += align_up(sizeof(double) * G->ny);
    G->kz2 = off;
    off += align_up(sizeof(double) * G->nz);
    G->psd_off = off;
    off += align_up(sizeof(double) * kPsdBlocks * (kMaxN / 2 + 1));
    G->total = off;
    return MC_OK;
}

struct Ptrs {
    double2 *W;
    double2 *twx, *twy, *twz;
    double *kx2, *ky2, *kz2;
    double *psd_partial;
};

Ptrs pointers(const Geo &G, void *ws)
{
    char *b = (char *)ws;
    Ptrs p;
    p.W = (double2 *)(b + G.w_off);
    p.twx = (double2 *)(b + G.twx);
    p.twy = (double2 *)(b + G.twy);
    p.twz = (double2 *)(b + G.twz);
    p.kx2 = (double *)(b + G.kx2);
    p.ky2 = (double *)(b + G.ky2);
    p.kz2 = (double *)(b + G.kz2);
    p.psd_partial = (double *)(b + G.psd_off);
    return p;
}

int prepare(const mc_ch_grid *g, void *ws, size_t ws_bytes, hipStream_t s, Geo *G, Ptrs *P)
{
    int rc = geometry(g, G);
    if (rc) return rc;
    if (!ws) return fail(MC_EINVAL, "workspace is NULL");
    if (ws_bytes < G->total) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, G->total);
    *P = pointers(*G, ws);
    hipLaunchKernelGGL(k_tables, dim3((G->nx + 255) / 256), dim3(256), 0, s, P->twx, P->kx2, G->nx, 1);
    hipLaunchKernelGGL(k_tables, dim3((G->ny + 255) / 256), dim3(256), 0, s, P->twy, P->ky2, G->ny, 0);
    hipLaunchKernelGGL(k_tables, dim3((G->nz + 255) / 256), dim3(256), 0, s, P->twz, P->kz2, G->nz, 0);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

// Lengths with a compile-time plan; any other length takes the runtime plan.
template <class F>
void with_length(int n, F &&f)
{
    switch (n) {
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 384: f(std::integral_constant<int, 384>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
    }
}

void enqueue_col(const Geo &G, int axis, double2 *A, const Ptrs &P, bool inv, hipStream_t s)
{
    if (axis == 1) {
        if (G.ny == 1) return;
        with_length(G.ny, [&](auto nc) {
            hipLaunchKernelGGL((k_colpass<1, decltype(nc)::value>), dim3((unsigned)(G.nz * G.tiles_y)), dim3(kThreads),
                               0, s, A, G.ny, G.hx, G.ny, G.Ty, G.tiles_y, G.py, P.twy, inv ? 1 : 0);
        });
    } else {
        if (G.nz == 1) return;
        with_length(G.nz, [&](auto nc) {
            hipLaunchKernelGGL((k_colpass<2, decltype(nc)::value>), dim3((unsigned)(G.ny * G.tiles_z)), dim3(kThreads),
                               0, s, A, G.ny, G.hx, G.nz, G.Tz, G.tiles_z, G.pz, P.twz, inv ? 1 : 0);
        });
    }
}

template <int MODE>
void enqueue_x(const Geo &G, const double *rin, double2 *spec, double *rout, const Ptrs &P, hipStream_t s,
               const uint8_t *mask_in = nullptr)
{
    const int lines = G.nz * G.ny;
    const double scale = 1.0 / ((double)G.nx * (double)G.ny * (double)G.nz);
    with_length(G.nx, [&](auto nc) {
        hipLaunchKernelGGL((k_xpass<MODE, decltype(nc)::value>), dim3((unsigned)((lines + G.Lx - 1) / G.Lx)),
                           dim3(kThreads), 0, s, rin, spec, rout, G.nx, lines, G.Lx, G.px, P.twx, scale, mask_in);
    });
}

template <int MODE>
void enqueue_z(const Geo &G, double2 *S, const Ptrs &P, double dt, double kappa, bool write_w, hipStream_t s)
{
    with_length(G.nz, [&](auto nc) {
        hipLaunchKernelGGL((k_zpass<MODE, decltype(nc)::value>), dim3((unsigned)(G.ny * G.tiles_z)), dim3(kThreads), 0,
                           s, S, P.W, G.ny, G.hx, G.nz, G.Tz, G.tiles_z, G.pz, P.twz, P.kx2, P.ky2, P.kz2, dt, kappa,
                           write_w ? 1 : 0);
    });
}

pmc::host::Timing g_ch_timing;

int ch_time(hipStream_t s, bool begin)
{
    Timing &t = g_ch_timing;
    if (!t.start) {
        HIP_TRY(hipEventCreate(&t.start));
        HIP_TRY(hipEventCreate(&t.stop));
    }
    if (begin) {
        HIP_TRY(hipEventRecord(t.start, s));
        t.armed = false;
    } else {
        HIP_TRY(hipEventRecord(t.stop, s));
        t.armed = true;
    }
    return MC_OK;
}

size_t rank_ws_bytes(int64_t n) { return pmc::sel::workspace_bytes((long long)n); }

}  // namespace

// App. A's dominant structural size from a radial PSD (reading: half the peak
// wavelength, one pore and one strut per period): the first shell s >= 1 holding
// the largest value, and n_max / (2 s).
__host__ __device__ inline int psd_peak_shell(const double *psd, int n_bins)
{
    int peak = 1;
    for (int i = 2; i < n_bins; ++i)
        if (psd[i] > psd[peak]) peak = i;
    return peak;
}

__host__ __device__ inline double dominant_size(int n_max, int peak) { return (double)n_max / (2.0 * peak); }

__global__ void k_psd_peak(const double *__restrict__ psd, int32_t n_bins, int32_t n_max, int32_t *__restrict__ peak,
                           double *__restrict__ size)
{
    if (threadIdx.x != 0) return;
    const int s = psd_peak_shell(psd, n_bins);
    if (peak) *peak = s;
    if (size) *size = dominant_size(n_max, s);
}

extern "C" {

int mc_ch_grid_from_target(double d_target, mc_ch_grid *g)
{
    clear_error();
    if (!g) return fail(MC_EINVAL, "grid is NULL");
    if (!(d_target > 0.0) || !isfinite(d_target)) return fail(MC_EINVAL, "d_target must be finite and > 0");
    // Eq. kappa_cal
    const double pi = 3.141592653589793;
    const double r = d_target / (8.0 * pi);
    g->kappa = 0.5 * r * r;
    // App. A: the explicit nonlinear term bounds the step, dt = min(0.5 / (kappa k_max^4), 1), k_max = pi
    const double k2 = pi * pi;
    const double dt = 0.5 / (g->kappa * k2 * k2);
    g->dt = dt < 1.0 ? dt : 1.0;
    return MC_OK;
}

int mc_psd_peak(const double *psd, int32_t n_bins, int32_t n_max, int32_t *peak_shell, double *size, void *hip_stream)
{
    clear_error();
    if (!psd || (!peak_shell && !size)) return fail(MC_EINVAL, "NULL argument");
    if (n_bins < 2) return fail(MC_EINVAL, "n_bins must be >= 2 (shell 0 is the mean)");
    if (n_max < 1) return fail(MC_EINVAL, "n_max must be >= 1");
    hipLaunchKernelGGL(k_psd_peak, dim3(1), dim3(64), 0, (hipStream_t)hip_stream, psd, n_bins, n_max, peak_shell, size);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_ch_workspace_bytes(const mc_ch_grid *g)
{
    clear_error();
    Geo G;
    if (geometry(g, &G)) return 0;
    return G.total;
}

int mc_ch_init(const mc_ch_grid *g, const double *phi0, double *state, void *workspace, size_t workspace_bytes,
               void *hip_stream)
{
    clear_error();
    if (!phi0 || !state) return fail(MC_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    Geo G;
    Ptrs P;
    int rc = prepare(g, workspace, workspace_bytes, s, &G, &P);
    if (rc) return rc;
    enqueue_x<X_INIT>(G, phi0, P.W, nullptr, P, s);
    enqueue_col(G, 1, P.W, P, false, s);
    if (G.nz == 1) {
        HIP_TRY(hipMemcpyAsync(state, P.W, G.spec_elems * sizeof(double2), hipMemcpyDeviceToDevice, s));
    } else {
        enqueue_z<Z_INIT>(G, (double2 *)state, P, g->dt, g->kappa, false, s);
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_ch_steps(const mc_ch_grid *g, int32_t n_steps, double *state, void *workspace, size_t workspace_bytes,
                int flags, void *hip_stream)
{
    clear_error();
    if (!state) return fail(MC_EINVAL, "state is NULL");
    if (n_steps < 0) return fail(MC_EINVAL, "n_steps must be >= 0");
    hipStream_t s = (hipStream_t)hip_stream;
    Geo G;
    Ptrs P;
    int rc = geometry(g, &G);
    if (rc) return rc;
    if (G.nz == 1) return fail(MC_EINVAL, "mc_ch_steps needs nz >= 2 (the step is fused with the z transform)");
    if ((rc = prepare(g, workspace, workspace_bytes, s, &G, &P))) return rc;
    double2 *S = (double2 *)state;
    const bool timed = (flags & MC_TIMED) != 0;
    if (timed && (rc = ch_time(s, true))) return rc;
    if (n_steps > 0) enqueue_z<Z_INV>(G, S, P, g->dt, g->kappa, true, s);
    for (int32_t i = 0; i < n_steps; ++i) {
        enqueue_col(G, 1, P.W, P, true, s);
        enqueue_x<X_NONLIN>(G, nullptr, P.W, nullptr, P, s);
        enqueue_col(G, 1, P.W, P, false, s);
        enqueue_z<Z_UPDATE>(G, S, P, g->dt, g->kappa, i + 1 < n_steps, s);
    }
    HIP_TRY(hipGetLastError());
    if (timed && (rc = ch_time(s, false))) return rc;
    return MC_OK;
}

int mc_ch_field(const mc_ch_grid *g, const double *state, double *phi, void *workspace, size_t workspace_bytes,
                void *hip_stream)
{
    clear_error();
    if (!state || !phi) return fail(MC_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    Geo G;
    Ptrs P;
    int rc = prepare(g, workspace, workspace_bytes, s, &G, &P);
    if (rc) return rc;
    if (G.nz == 1) {
        HIP_TRY(hipMemcpyAsync(P.W, state, G.spec_elems * sizeof(double2), hipMemcpyDeviceToDevice, s));
    } else {
        enqueue_z<Z_INV>(G, (double2 *)state, P, g->dt, g->kappa, true, s);
    }
    enqueue_col(G, 1, P.W, P, true, s);
    enqueue_x<X_FIELD>(G, nullptr, P.W, phi, P, s);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_ch_psd(const mc_ch_grid *g, const double *state, double *psd, void *workspace, size_t workspace_bytes,
              void *hip_stream)
{
    clear_error();
    if (!state || !psd) return fail(MC_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    Geo G;
    Ptrs P;
    int rc = prepare(g, workspace, workspace_bytes, s, &G, &P);
    if (rc) return rc;
    const int nb = std::max(G.nx, std::max(G.ny, G.nz)) / 2 + 1;
    hipLaunchKernelGGL(k_psd_partial, dim3(kPsdBlocks), dim3(kThreads), 0, s, (const double2 *)state, G.nx, G.ny, G.nz,
                       P.kx2, P.ky2, P.kz2, P.psd_partial, nb);
    hipLaunchKernelGGL(k_psd_sum, dim3(nb), dim3(kThreads), 0, s, P.psd_partial, kPsdBlocks, nb, psd);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

static void mask_grid(const mc_volume *vol, mc_ch_grid *g)
{
    memset(g, 0, sizeof *g);
    g->nx = vol->nx;
    g->ny = vol->ny;
    g->nz = vol->nz;
    g->kappa = 1.0;   // unused by the transforms
    g->dt = 1.0;
}

size_t mc_mask_psd_workspace_bytes(const mc_volume *vol)
{
    clear_error();
    if (check_volume(vol)) return 0;
    mc_ch_grid g;
    mask_grid(vol, &g);
    Geo G;
    if (geometry(&g, &G)) return 0;
    return G.total;
}

int mc_mask_psd(const mc_volume *vol, double *psd, void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!psd) return fail(MC_EINVAL, "psd is NULL");
    mc_ch_grid g;
    mask_grid(vol, &g);
    hipStream_t s = (hipStream_t)hip_stream;
    Geo G;
    Ptrs P;
    if ((rc = prepare(&g, workspace, workspace_bytes, s, &G, &P))) return rc;
    // forward transform of the mask into W: x (from the bytes), y, then z in place
    enqueue_x<X_MASK>(G, nullptr, P.W, nullptr, P, s, vol->mask);
    enqueue_col(G, 1, P.W, P, false, s);
    if (G.nz > 1) enqueue_z<Z_INIT>(G, P.W, P, g.dt, g.kappa, false, s);
    const int nb = std::max(G.nx, std::max(G.ny, G.nz)) / 2 + 1;
    hipLaunchKernelGGL(k_psd_partial, dim3(kPsdBlocks), dim3(kThreads), 0, s, (const double2 *)P.W, G.nx, G.ny, G.nz,
                       P.kx2, P.ky2, P.kz2, P.psd_partial, nb);
    hipLaunchKernelGGL(k_psd_sum, dim3(nb), dim3(kThreads), 0, s, P.psd_partial, kPsdBlocks, nb, psd);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

double mc_ch_elapsed_ms(void)
{
    Timing &t = g_ch_timing;
    if (!t.armed) return -1.0;
    if (hipEventSynchronize(t.stop) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) return -1.0;
    return (double)ms;
}

size_t mc_rank_threshold_workspace_bytes(int64_t n)
{
    clear_error();
    if (n < 1 || n >= (1ll << 40)) return 0;
    return rank_ws_bytes(n);
}

int mc_rank_threshold(const double *field, int64_t n, int64_t n_pore, uint8_t *mask, void *workspace,
                      size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    if (!field || !mask || !workspace) return fail(MC_EINVAL, "NULL argument");
    if (n < 1 || n >= (1ll << 40)) return fail(MC_EINVAL, "n must be in [1, 2^40)");
    if (n_pore < 0 || n_pore > n) return fail(MC_EINVAL, "n_pore must be in [0, n]");
    const size_t need = rank_ws_bytes(n);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return pmc::sel::enqueue_top(field, (long long)n, (long long)n_pore, mask, workspace, (hipStream_t)hip_stream);
}

size_t mc_ch_generate_workspace_bytes(const mc_ch_grid *g)
{
    clear_error();
    Geo G;
    if (geometry(g, &G)) return 0;
    const size_t n = (size_t)G.nx * G.ny * G.nz;
    return G.total + align_up(n * sizeof(double)) + align_up(sizeof(double) * (kMaxN / 2 + 1)) +
           rank_ws_bytes((int64_t)n);
}

int mc_ch_generate(const mc_ch_grid *g, const double *phi0, double d_target, double sigma, int32_t check_every,
                   int32_t max_steps, double porosity, double *state, double *phi_out, uint8_t *mask,
                   int32_t *steps_taken, double *last_size, void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    if (!phi0 || !state || !workspace) return fail(MC_EINVAL, "NULL argument");
    if (check_every < 1 || max_steps < 0) return fail(MC_EINVAL, "check_every must be >= 1 and max_steps >= 0");
    if (!(porosity >= 0.0 && porosity <= 1.0)) return fail(MC_EINVAL, "porosity must be in [0, 1]");
    if (!(d_target > 0.0) || !(sigma >= 0.0)) return fail(MC_EINVAL, "d_target must be > 0 and sigma >= 0");
    Geo G;
    int rc = geometry(g, &G);
    if (rc) return rc;
    const size_t need = mc_ch_generate_workspace_bytes(g);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t n = (size_t)G.nx * G.ny * G.nz;
    char *b = (char *)workspace;
    double *field = (double *)(b + G.total);
    double *psd = (double *)(b + G.total + align_up(n * sizeof(double)));
    void *rank_ws = b + G.total + align_up(n * sizeof(double)) + align_up(sizeof(double) * (kMaxN / 2 + 1));
    const int nmax = std::max(G.nx, std::max(G.ny, G.nz));
    const int nb = nmax / 2 + 1;
    if ((rc = mc_ch_init(g, phi0, state, workspace, G.total, hip_stream))) return rc;
    int32_t done = 0;
    double size = 0.0;
    double host_psd[kMaxN / 2 + 1];
    while (done < max_steps) {
        const int32_t m = std::min(check_every, max_steps - done);
        if ((rc = mc_ch_steps(g, m, state, workspace, G.total, 0, hip_stream))) return rc;
        done += m;
        if ((rc = mc_ch_psd(g, state, psd, workspace, G.total, hip_stream))) return rc;
        HIP_TRY(hipMemcpyAsync(host_psd, psd, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        size = dominant_size(nmax, psd_peak_shell(host_psd, nb));
        if (size >= d_target - 0.5 * sigma && size <= d_target + 0.5 * sigma) break;
    }
    if (steps_taken) *steps_taken = done;
    if (last_size) *last_size = size;
    if (phi_out || mask) {
        double *f = phi_out ? phi_out : field;
        if ((rc = mc_ch_field(g, state, f, workspace, G.total, hip_stream))) return rc;
        if (mask) {
            const long long n_pore = llround(porosity * (double)n);
            if ((rc = mc_rank_threshold(f, (int64_t)n, n_pore, mask, rank_ws, rank_ws_bytes((int64_t)n), hip_stream)))
                return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return MC_OK;
}

}  // extern "C"
