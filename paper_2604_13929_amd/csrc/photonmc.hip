// photonmc.hip -- MI355X (gfx950) kernels and the C ABI declared in photonmc.h.
//
// Kernels
//   k_fill_i64     zero the tallies and the queue counter (a fill kernel, so the
//                  sequence stays capturable in a HIP graph without memset nodes)
//   k_pack         uint8 mask -> 4x4x4 bit bricks (one uint64 per brick)
//   k_walk         persistent photon walk: one photon per lane, wavefronts take
//                  photon ids from a global queue in chunks and refill idle lanes
//   k_trace        one traced photon per lane, same step function, records
//   k_reduce       per-depth, per-phase exact integer sums of the fluence tally
//   k_finalize     the estimators in FP64 from those sums and the scalar channels
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "internal.hpp"
#include "spinodal.h"

using namespace pmc;

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

namespace pmc {
namespace host {

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_err[0] = 0; }

}  // namespace host
}  // namespace pmc

using namespace pmc::host;

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_i64(int64_t *__restrict__ p, uint64_t n, int64_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One thread per 4x4x4 brick; bit (dz*16 + dy*4 + dx) is 1 for a pore voxel.
// Voxels outside the volume (ragged edges) stay 0 and are never addressed.
__global__ void k_pack(const uint8_t *__restrict__ mask, int32_t nx, int32_t ny, int32_t nz, int32_t nxb,
                       int32_t nyb, uint64_t nbricks, uint64_t *__restrict__ bricks)
{
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbricks) return;
    const int32_t bx = (int32_t)(b % (uint64_t)nxb);
    const int32_t by = (int32_t)((b / (uint64_t)nxb) % (uint64_t)nyb);
    const int32_t bz = (int32_t)(b / ((uint64_t)nxb * (uint64_t)nyb));
    uint64_t bits = 0;
    for (int dz = 0; dz < 4; ++dz) {
        const int32_t z = bz * 4 + dz;
        if (z >= nz) break;
        for (int dy = 0; dy < 4; ++dy) {
            const int32_t y = by * 4 + dy;
            if (y >= ny) break;
            const uint8_t *row = mask + ((uint64_t)z * ny + y) * (uint64_t)nx;
            for (int dx = 0; dx < 4; ++dx) {
                const int32_t x = bx * 4 + dx;
                if (x >= nx) break;
                if (row[x]) bits |= 1ull << ((dz << 4) | (dy << 2) | dx);
            }
        }
    }
    bricks[b] = bits;
}

// Staged quanta -> the caller's [nz][ny][nx] tally in Q31 units: F += S << shift.
// The walk has already added there what the staging words could not hold (whole
// 2^32-quanta carries and deposits of 2^31 quanta or more).
__global__ void k_unstage(const uint32_t *__restrict__ S, int64_t *__restrict__ F, int32_t nx, int32_t ny, int32_t nz,
                          int32_t lnx, int32_t lny, int32_t planes)
{
    const uint64_t n = (uint64_t)nx * ny * nz;
    const PlaneDims P = plane_dims(nx, ny, nz);
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t x = (int32_t)(v % (uint64_t)nx);
        const int32_t y = (int32_t)((v / (uint64_t)nx) % (uint64_t)ny);
        const int32_t z = (int32_t)(v / ((uint64_t)nx * ny));
        if (planes)
            F[v] += (int64_t)((uint64_t)S[plane_index(P, nx, ny, 0u, x, y, z)] + S[plane_index(P, nx, ny, 1u, x, y, z)] +
                              S[plane_index(P, nx, ny, 2u, x, y, z)])
                    << kDepositShift;
        else
            F[v] += (int64_t)S[stage_index(lnx, lny, x, y, z)] << kDepositShift;
    }
}

// ---------------------------------------------------------------------------
// Sinks: where a step's side effects go
// ---------------------------------------------------------------------------
// Fluence deposits straight to the caller's [nz][ny][nx] tally (Q31 units), one
// device-scope atomic per voxel visit.
struct DirectDeposit {
    template <typename R>
    __device__ __forceinline__ void flush(const Job &J, const Photon<R> &p, uint64_t a)
    {
        if (a != 0ull)
            __hip_atomic_fetch_add((unsigned long long *)(J.fluence + voxel_index(J, p)),
                                   (unsigned long long)a << kDepositShift, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Fluence deposits logged in LDS for a staging tally of uint32 quanta in lines of
// 16 words (one 64-byte line): the plane layout where its three tables fit (see
// stage_word), else lines of 2x2x4 voxels.  Each lane appends its deposits to its
// own kLogK slots; once some lane has filled them, the wavefront issues the log
// with lanes transposed, so that one atomic instruction carries the kLogK slots of
// each of 64/kLogK lanes: deposits of one photon that fall in the same line travel
// as one memory-side request.  A 2x2x4 line holds twice the voxels a line of int64
// words would (0.40 against 0.48 requests per photon-step over oracle trajectories
// of the 256^3 workload), and 16-lane groups of 32-bit atomics on one line run at
// 26.5 G requests/s against 23.7 for 8-lane groups of 64-bit atomics.
// A flush would cut the run of deposits a photon is still making into one line in
// two requests.  So the newest entries of a lane's log that lie in the line of its
// current voxel (its next deposit's line, unless an interaction turns it to
// another plane table), up to kLogHold of them, are held back: they stay in the
// lane's ring of slots and go out with the deposits that follow them.
// A word cannot hold a voxel's sum: the flush reads back each word's previous
// value and, where an add wrapped it past 2^32, adds the lost 2^32 quanta to the
// caller's int64 tally, so the total stays exact (a quantum of 2^8 Q31 units makes
// that about one carry per 2000 photon-steps).  A log entry is a 32-bit word
// index and a value below 2^31 (its top bit marks a held entry); a photon's
// deposit in one voxel of 2^31 quanta or more (256 voxel lengths at full weight)
// goes to the int64 tally directly.  At 16 slots a 256-thread workgroup's log
// takes 33 KB, so four workgroups fit per CU.
#ifndef MC_LOG_K
#define MC_LOG_K 16
#endif
#ifndef MC_LOG_HOLD
#define MC_LOG_HOLD 6
#endif
constexpr int kLogK = MC_LOG_K;
constexpr int kLogHold = MC_LOG_HOLD;   // 0: no entries held back
static_assert(kLogK == 16 || kLogK == 32, "the transposed flush needs kLogK dividing 64, at least 16");
static_assert(kLogHold >= 0 && kLogHold < kLogK, "a lane must keep a free slot after a flush");
constexpr int kLogStride = 65;  // 64 lanes + 1: the transposed reads hit distinct banks
constexpr uint32_t kNoLine = 0xFFFFFFFFu;

template <int kLogSlots>
struct LoggedDepositK {
    uint32_t *lidx;             // this wavefront's log: [slot][kLogStride]
    uint32_t *lval;
    uint32_t lane;
    uint32_t head, count;       // this lane's ring of kLogSlots slots
    template <typename R>
    __device__ __forceinline__ void flush(const Job &J, const Photon<R> &p, uint64_t a)
    {
        if (a != 0ull) {
            if (a >> 31) {
                __hip_atomic_fetch_add((unsigned long long *)(J.fluence + voxel_index(J, p)),
                                       (unsigned long long)a << kDepositShift, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint32_t s = log_slot<kLogStride, kLogSlots>(lane, head, count);
                lidx[s] = stage_word(J, p);
                lval[s] = (uint32_t)a;
                ++count;
            }
        }
    }
};

// The carry of a staging word that wrapped: 2^32 quanta into the voxel's int64 word.
__device__ __forceinline__ void stage_carry(const Job &J, uint32_t idx)
{
    __hip_atomic_fetch_add((unsigned long long *)(J.fluence + stage_voxel(J, idx)), 1ull << (32 + kDepositShift),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Issue the wavefront's log.  HOLD: each lane first marks the newest run of entries
// in its log that lies in `line` (kNoLine: none), the issue skips them, and they
// stay as the lane's whole ring.  The FP64 transport, bound by its VALU, holds
// nothing.
template <int K, bool HOLD>
__device__ __forceinline__ void flush_log(uint32_t *lidx, uint32_t *lval, const Job &J, uint32_t lane,
                                          uint32_t line, uint32_t &head, uint32_t &count)
{
    constexpr bool kHold = HOLD && kLogHold > 0;
    const uint32_t held =
        kHold ? log_mark_run<kLogStride, K, (kHold ? kLogHold : 1)>(lidx, lval, lane, head, count, line) : 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // in two halves, each issuing its adds before it looks at what they returned
    // (half the returned words live at a time keeps the walk within 128 VGPRs)
#pragma unroll
    for (int h = 0; h < K; h += K / 2) {
        uint32_t old[K / 2];
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const uint32_t src = (uint32_t)(h + i) * (64 / K) + lane / K;
            const uint32_t e = (lane % K) * kLogStride + src;
            const uint32_t v = lval[e];
            old[i] = 0u;
            if (v != 0u && (!kHold || v < kLogHeld))
                old[i] = __hip_atomic_fetch_add(J.stage + lidx[e], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const uint32_t src = (uint32_t)(h + i) * (64 / K) + lane / K;
            const uint32_t e = (lane % K) * kLogStride + src;
            const uint32_t v = lval[e];
            if (v != 0u && (!kHold || v < kLogHeld)) {
                if (old[i] > 0xFFFFFFFFu - v) stage_carry(J, lidx[e]);
                lval[e] = 0u;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (kHold) {
        log_keep_run<kLogStride, K, (kHold ? kLogHold : 1)>(lval, lane, head, count, held);
    } else {
        head = 0u;
        count = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <class Deposit>
struct TallySink : Deposit {
    template <typename R> __device__ __forceinline__ void segment(const Photon<R> &, const Job &, R, bool) {}
    template <typename R> __device__ __forceinline__ void deflect(Photon<R> &, const Job &, R) {}
};

// Likelihood-ratio (perturbation Monte Carlo) scores of the track-length
// estimator.  The sampled path density is mu_s^k exp(-mu_t l_solid) prod p_HG;
// its log-derivatives give the scores S_mus = k/mu_s - l_solid,
// S_mua = -l_solid and S_g = sum_i d ln p_HG(cos_i)/dg.  A segment of length d
// starting with those scores adds w (S d - [solid] d^2/2) to the mu_s and mu_a
// bins (the d^2/2 is the survival inside the segment) and w S_g d to the g bin,
// per (parameter, phase, depth), in fixed point 2^-MC_GRAD_FIXED_BITS of a Q31
// weight x voxel, each segment's value rounded to nearest.  Roulette decisions
// carry no score: survival 1/m with weight x m is unbiased.
constexpr double kGradScale = 1.0 / (double)(1ll << MC_GRAD_FIXED_BITS);

// The block keeps its score bins in LDS as int32 words (half the space of int64
// bins: four 256-thread walk workgroups still fit per CU at nz = 256) and moves a
// word to the global (hi, lo) int64 pairs before it can overflow.  A value of
// magnitude >= kGradDirect goes to the global pair directly; any other is added
// to its word, and a lane whose add leaves the word at magnitude >= kGradSpill
// swaps the word for 0 and adds what it took to the global pair.  A lane that
// sees the threshold swaps before its next add, so at most one add per thread of
// the block lands on a word between its crossing and the swap: |word| < kGradSpill
// + 512 * kGradDirect = 2^28 + 2^30.  Every transfer is exact, so the totals are
// the integer sums of the segments' fixed-point values whatever the order.  The
// global pairs are few (6 nz, a hot address each), so the direct path must stay
// rare: at 2^-20 a value reaches 2^21 only where (w / 2^31) |S| d reaches 1024
// voxels, while under implicit capture (w / 2^31) l_solid peaks at 1 / (e mu_a),
// 37 voxels at mu_a = 0.01.
constexpr long long kGradDirect = 1ll << 21;
constexpr int kGradSpill = 1 << 28;

__device__ __forceinline__ void grad_global_add(unsigned long long *grad, int32_t i, long long v)
{
    atomicAdd(&grad[2 * i], (unsigned long long)(v >> 32));
    atomicAdd(&grad[2 * i + 1], (unsigned long long)v & 0xFFFFFFFFull);
}

__device__ __forceinline__ void grad_bin_add(int *bins, unsigned long long *grad, int32_t i, long long v)
{
    if (v == 0) return;
    if (v >= kGradDirect || v <= -kGradDirect) {
        grad_global_add(grad, i, v);
        return;
    }
    const long long nv = (long long)atomicAdd(&bins[i], (int)v) + v;
    if (nv >= kGradSpill || nv <= -kGradSpill) grad_global_add(grad, i, (long long)atomicExch(&bins[i], 0));
}

__device__ __forceinline__ double hg_score(double ct, double g)
{
    return -2.0 * g / (1.0 - g * g) + 3.0 * (ct - g) / (1.0 + g * g - 2.0 * g * ct);
}

template <class Deposit>
struct GradSink : Deposit {
    int *bins;                 // LDS [3][2][nz] int32 words
    unsigned long long *grad;  // global [3][2][nz] (hi, lo) pairs
    int32_t nz;
    double inv_mu_s;           // 1/mu_s, 0 when mu_s = 0
    template <typename R>
    __device__ __forceinline__ void segment(const Photon<R> &p, const Job &, R d, bool solid)
    {
        if (p.iz < 0 || p.iz >= nz) return;                  // air pads carry no bins
        const double dd = (double)d, ls = p.l_tot - p.l_void;  // solid path before this segment
        const double sq = solid ? 0.5 * dd * dd : 0.0;
        const double sw = (double)p.w * kGradScale;
        const int32_t base = (solid ? 0 : nz) + p.iz;
        const long long vs = __double2ll_rn(sw * (((double)p.k * inv_mu_s - ls) * dd - sq));
        const long long va = __double2ll_rn(sw * (-ls * dd - sq));
        const long long vg = __double2ll_rn(sw * (p.score_g * dd));
        grad_bin_add(bins, grad, base, vs);
        grad_bin_add(bins, grad, 2 * nz + base, va);
        grad_bin_add(bins, grad, 4 * nz + base, vg);
    }
    template <typename R> __device__ __forceinline__ void deflect(Photon<R> &p, const Job &J, R ct)
    {
        p.score_g += hg_score((double)ct, (double)J.g);
    }
};

// Terminal outcome of one photon into the block's channel accumulators (LDS).
template <typename R>
__device__ __forceinline__ void account(unsigned long long *acc, const Photon<R> &p, int32_t ev, int32_t nz)
{
    if (ev == EV_ESC_R || ev == EV_ESC_T) {
        atomicAdd(&acc[ev == EV_ESC_R ? MC_S_R : MC_S_T], (unsigned long long)p.w);
        atomicAdd(&acc[MC_S_ESC_W], (unsigned long long)p.w);
        atomicAdd(&acc[MC_S_ESC_N], 1ull);
        if (p.l_void > (double)nz) {
            atomicAdd(&acc[MC_S_ESC_W_GTL], (unsigned long long)p.w);
            atomicAdd(&acc[MC_S_ESC_N_GTL], 1ull);
        }
        // w * l_void can reach 2^51 per photon: sum the two 32-bit halves separately
        const unsigned long long vp = __double2ull_rn((double)p.w * p.l_void);
        atomicAdd(&acc[MC_S_ESC_W_VOID_PATH], vp & 0xFFFFFFFFull);
        if (vp >> 32) atomicAdd(&acc[MC_S_ESC_W_VOID_PATH_HI], vp >> 32);
    } else if (ev == EV_LOST) {
        atomicAdd(&acc[MC_S_LOST], (unsigned long long)p.w);
    } else if (ev == EV_GATED) {
        atomicAdd(&acc[MC_S_GATED], (unsigned long long)p.w);
    }
    if (p.absorbed) atomicAdd(&acc[MC_S_A], (unsigned long long)p.absorbed);
    if (p.rr) atomicAdd(&acc[MC_S_RR], (unsigned long long)p.rr);  // two's complement: signed sum
    atomicAdd(&acc[MC_S_STEPS], (unsigned long long)p.steps);
    atomicAdd(&acc[MC_S_INTERACTIONS], (unsigned long long)p.k);
    atomicAdd(&acc[MC_S_LAUNCHED], 1ull);
}

// In-pore path histogram of the escaping photons of a walk (Sec. 3.5 (c)), kept
// per workgroup in LDS (weights 64-bit, counts 32-bit) and added to w and n once.
struct EscHist {
    unsigned long long *w;    // [nbins] escaped Q31 weight
    unsigned long long *n;    // [nbins] escaped photons
    double width;
    int32_t nbins;            // 1 .. kEscMaxBins
};

// ---------------------------------------------------------------------------
// Persistent walk
// ---------------------------------------------------------------------------
// Each wavefront owns a private range [q_next, q_end) of queue positions and
// takes `chunk` more with one atomic when it runs dry.  Idle lanes are refilled
// together once at least `refill` of them are idle (or all are), so launches
// run converged.  A lane whose segment ends at an interaction point waits there
// until `defer` lanes of its wavefront wait (or no lane can advance); then the
// waiting lanes run their interactions together, so that code runs with many
// lanes active instead of a few in every iteration.  A photon's own sequence of
// steps is the same either way.  A wavefront exits when the queue is exhausted,
// its range is empty and none of its lanes is alive; every photon terminates
// (escape, weight 0, roulette, or the step cap), and a waiting lane is served
// at the latest once no lane can advance, so every wavefront exits.
template <bool GRAD, bool LOGGED> struct SinkOf {
    using Deposit = typename std::conditional<LOGGED, LoggedDepositK<GRAD ? 16 : kLogK>, DirectDeposit>::type;
    using type = typename std::conditional<GRAD, GradSink<Deposit>, TallySink<Deposit>>::type;
};

// LOGGED: deposits go through the log into J.stage (see LoggedDepositK).  GENERAL: the
// step that also knows the paper's boundary model (see walk.hpp).
// ESC: also bin the in-pore path of every escaping photon (EscHist).
template <int BLOCK, typename R, bool GRAD, bool LOGGED, bool GENERAL, bool ESC>
__global__ __launch_bounds__(BLOCK) void k_walk(const Job J, unsigned long long *__restrict__ queue, int32_t chunk,
                                                int32_t refill, int32_t defer, unsigned long long *__restrict__ grad,
                                                const EscHist eh)
{
    constexpr int kWaves = BLOCK / 64;
    constexpr int K = GRAD ? 16 : kLogK;   // log slots per lane (the gradient bins share the LDS)
    constexpr bool kFP32 = std::is_same<R, float>::value;
    __shared__ unsigned long long acc[MC_NSCALARS];
    __shared__ uint32_t s_lidx[LOGGED ? kWaves * K * kLogStride : 1];
    __shared__ uint32_t s_lval[LOGGED ? kWaves * K * kLogStride : 1];
    extern __shared__ unsigned long long s_dyn[];   // GRAD: int32 bins [3][2][nz]; ESC: weights [nbins], then counts
    unsigned long long *esc_w = s_dyn;
    unsigned int *esc_n = reinterpret_cast<unsigned int *>(s_dyn + (ESC ? eh.nbins : 0));
    const uint32_t lane = __lane_id();
    uint32_t *lidx = s_lidx + (threadIdx.x >> 6) * (LOGGED ? K * kLogStride : 0);
    uint32_t *lval = s_lval + (threadIdx.x >> 6) * (LOGGED ? K * kLogStride : 0);
    if (threadIdx.x < MC_NSCALARS) acc[threadIdx.x] = 0ull;
    int *gbins = reinterpret_cast<int *>(s_dyn);
    if (GRAD)
        for (int32_t i = threadIdx.x; i < 6 * J.nz; i += BLOCK) gbins[i] = 0;
    if (ESC)
        for (int32_t i = threadIdx.x; i < eh.nbins; i += BLOCK) {
            esc_w[i] = 0ull;
            esc_n[i] = 0u;
        }
    if (LOGGED)
        for (int i = 0; i < K; ++i) lval[i * kLogStride + lane] = 0u;
    __syncthreads();

    typename SinkOf<GRAD, LOGGED>::type sink;
    if constexpr (LOGGED) {
        sink.lidx = lidx;
        sink.lval = lval;
        sink.lane = lane;
        sink.head = 0u;
        sink.count = 0u;
    }
    if constexpr (GRAD) {
        sink.bins = gbins;
        sink.grad = grad;
        sink.nz = J.nz;
        sink.inv_mu_s = J.mu_s > 0.0 ? 1.0 / J.mu_s : 0.0;
    }
    Photon<R> p;
    bool alive = false;
    bool waiting = false;   // alive, at an interaction point, interaction not yet run
    uint64_t q_next = 0, q_end = 0;
    bool exhausted = false;
    const uint64_t total = J.n_photons;

    auto retire = [&](int32_t ev) {
        account(acc, p, ev, J.nz);
        if (ESC && (ev == EV_ESC_R || ev == EV_ESC_T)) {
            const int b = escape_path_bin(p.l_void, eh.width, eh.nbins);
            atomicAdd(&esc_w[b], (unsigned long long)p.w);
            atomicAdd(&esc_n[b], 1u);
        }
        alive = false;
    };

    for (;;) {
        const uint64_t idle = __ballot(!alive);
        if (idle != 0ull) {
            const int32_t nidle = __popcll(idle);
            if (!exhausted && (nidle >= refill || idle == ~0ull)) {
                if (q_next >= q_end) {
                    unsigned long long base = 0ull;
                    if (lane == 0) base = atomicAdd(queue, (unsigned long long)chunk);
                    base = __shfl(base, 0);
                    if (base >= total) {
                        exhausted = true;
                    } else {
                        q_next = base;
                        q_end = base + (uint64_t)chunk < total ? base + (uint64_t)chunk : total;
                    }
                }
                if (q_next < q_end) {
                    const uint64_t avail = q_end - q_next;
                    const uint32_t rank = (uint32_t)__popcll(idle & __lanemask_lt());
                    if (!alive && rank < avail) {
                        launch<GENERAL>(p, J, (uint32_t)(J.photon_begin + q_next + rank));
                        alive = true;
                    }
                    q_next += (uint64_t)nidle < avail ? (uint64_t)nidle : avail;
                }
            }
            if (exhausted && q_next >= q_end && !__any(alive)) break;
        }
        if (alive && !waiting) {
            const int32_t ev = advance<GENERAL>(p, J, sink);
            if (ev == EV_AT_INTERACTION) {
                waiting = true;
            } else {
                const int32_t fin = finish(p, J, sink, ev);
                if (is_terminal(fin)) retire(fin);
            }
        }
        const uint64_t wait_mask = __ballot(waiting);
        if (wait_mask != 0ull &&
            (__popcll(wait_mask) >= defer || __ballot(alive && !waiting) == 0ull)) {
            if (waiting) {
                const int32_t fin = finish(p, J, sink, interact(p, J, sink));
                waiting = false;
                if (is_terminal(fin)) retire(fin);
            }
        }
        // a lane logs at most one deposit per iteration (an advance that reaches an
        // interaction point logs none), so issue the log once some lane has filled it
        if constexpr (LOGGED) {
            if (__ballot(sink.count >= (uint32_t)K) != 0ull)
                flush_log<K, kFP32>(lidx, lval, J, lane, alive ? stage_word(J, p) >> 4 : kNoLine, sink.head,
                                    sink.count);
        }
    }
    if constexpr (LOGGED) flush_log<K, kFP32>(lidx, lval, J, lane, kNoLine, sink.head, sink.count);
    __syncthreads();
    if (threadIdx.x < MC_NSCALARS) {
        const unsigned long long v = acc[threadIdx.x];
        if (v) atomicAdd((unsigned long long *)&J.scalars[threadIdx.x], v);
    }
    if (ESC)
        for (int32_t i = threadIdx.x; i < eh.nbins; i += BLOCK)
            if (esc_n[i]) {
                atomicAdd(&eh.w[i], esc_w[i]);
                atomicAdd(&eh.n[i], (unsigned long long)esc_n[i]);
            }
    if (GRAD) {
        // what the words still hold, signed, into the (hi, lo) pairs: total = sum(hi) * 2^32 + sum(lo)
        for (int32_t i = threadIdx.x; i < 6 * J.nz; i += BLOCK) {
            const long long v = (long long)gbins[i];
            if (v) grad_global_add(grad, i, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Trace
// ---------------------------------------------------------------------------
struct TraceSink {
    mc_trace_rec *rec;
    int32_t max_rec, n;
    template <typename R>
    __device__ __forceinline__ void segment(const Photon<R> &p, const Job &, R d, bool)
    {
        if (n < max_rec) {
            mc_trace_rec &r = rec[n];
            r.ix = p.ix; r.iy = p.iy; r.iz = p.iz; r.event = -1;
            r.fx = p.fx; r.fy = p.fy; r.fz = p.fz;
            r.ux = p.ux; r.uy = p.uy; r.uz = p.uz;
            r.d = d; r.s_rem = p.s_rem; r.w = p.w; r.k = p.k;
        }
    }
    template <typename R> __device__ __forceinline__ void deflect(const Photon<R> &, const Job &, R) {}
    template <typename R> __device__ __forceinline__ void flush(const Job &, const Photon<R> &, uint64_t) {}
    __device__ __forceinline__ void post(int32_t ev)
    {
        if (n < max_rec) rec[n].event = ev;
        ++n;
    }
};

template <typename R, bool GENERAL>
__global__ void k_trace(const Job J, const uint64_t *__restrict__ ids, int32_t n, int32_t max_rec,
                        mc_trace_rec *__restrict__ recs, mc_photon_rec *__restrict__ out)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    TraceSink sink{recs + (int64_t)i * max_rec, max_rec, 0};
    for (int32_t j = 0; j < max_rec; ++j) sink.rec[j].event = -1;
    Photon<R> p;
    launch<GENERAL>(p, J, (uint32_t)ids[i]);
    int32_t ev;
    for (;;) {
        ev = step<GENERAL>(p, J, sink);
        sink.post(ev);
        if (is_terminal(ev)) break;
    }
    if (out) {
        mc_photon_rec o;
        o.R = ev == EV_ESC_R ? (int64_t)p.w : 0;
        o.T = ev == EV_ESC_T ? (int64_t)p.w : 0;
        o.A = (int64_t)p.absorbed;
        o.RR = p.rr;
        o.lost = ev == EV_LOST ? (int64_t)p.w : 0;
        o.w_final = p.w;
        o.fate = (uint32_t)ev;
        o.steps = p.steps;
        o.interactions = p.k;
        o.path_void = p.l_void;
        o.path_solid = p.l_tot - p.l_void;
        out[i] = o;
    }
}

// ---------------------------------------------------------------------------
// Reduction
// ---------------------------------------------------------------------------
// bins[z][8]: solid (hi, lo), pore (hi, lo), n_solid, n_pore, max, unused.
// A voxel value v >= 0 is split as v = hi * 2^32 + lo; the halves are summed
// separately, so no partial sum overflows and the totals are exact.
constexpr int kReduceBlock = 256;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

__global__ __launch_bounds__(kReduceBlock) void k_reduce(const int64_t *__restrict__ F, const uint8_t *__restrict__ mask,
                                                         uint64_t layer, uint64_t per_block,
                                                         unsigned long long *__restrict__ bins)
{
    const uint64_t z = blockIdx.y;
    const uint64_t begin = (uint64_t)blockIdx.x * per_block;
    const uint64_t end = begin + per_block < layer ? begin + per_block : layer;
    const int64_t *f = F + z * layer;
    const uint8_t *m = mask + z * layer;
    unsigned long long s_hi = 0, s_lo = 0, p_hi = 0, p_lo = 0, n_s = 0, n_p = 0, mx = 0;
    for (uint64_t i = begin + threadIdx.x; i < end; i += kReduceBlock) {
        const unsigned long long v = (unsigned long long)f[i];
        const unsigned long long hi = v >> 32, lo = v & 0xFFFFFFFFull;
        if (m[i]) { p_hi += hi; p_lo += lo; ++n_p; }
        else      { s_hi += hi; s_lo += lo; ++n_s; }
        mx = v > mx ? v : mx;
    }
    __shared__ unsigned long long part[kReduceBlock / 64][7];
    const int w = threadIdx.x >> 6;
    unsigned long long vals[7] = {s_hi, s_lo, p_hi, p_lo, n_s, n_p, mx};
#pragma unroll
    for (int c = 0; c < 6; ++c) vals[c] = wave_sum(vals[c]);
    vals[6] = wave_max(vals[6]);
    if (__lane_id() == 0)
        for (int c = 0; c < 7; ++c) part[w][c] = vals[c];
    __syncthreads();
    if (threadIdx.x < 7) {
        unsigned long long t = 0;
        for (int i = 0; i < kReduceBlock / 64; ++i)
            t = threadIdx.x == 6 ? (part[i][6] > t ? part[i][6] : t) : t + part[i][threadIdx.x];
        unsigned long long *dst = bins + z * kBinW + threadIdx.x;
        if (threadIdx.x == 6) atomicMax(dst, t);
        else if (t) atomicAdd(dst, t);
    }
}

__device__ __forceinline__ double join(unsigned long long hi, unsigned long long lo)
{
    return (double)hi * 4294967296.0 + (double)lo;
}

// One block: per-depth profiles in parallel, totals by thread 0 in z order.
__global__ void k_finalize(const unsigned long long *__restrict__ bins, const int64_t *__restrict__ S, int32_t nx,
                           int32_t ny, int32_t nz, double *__restrict__ q, double *__restrict__ depth)
{
    const double n_ph = (double)S[MC_S_LAUNCHED];
    const double launched_w = n_ph * 2147483648.0;
    const double face = (double)nx * (double)ny;
    const double norm = face / launched_w;  // Phi/S0 per unit of F
    const double nan = __builtin_nan("");
    if (depth) {
        for (int32_t z = threadIdx.x; z < nz; z += blockDim.x) {
            const unsigned long long *b = bins + (uint64_t)z * kBinW;
            const double fs = join(b[0], b[1]), fp = join(b[2], b[3]);
            depth[z] = (fs + fp) * norm / face;
            depth[nz + z] = b[4] ? fs * norm / (double)b[4] : nan;
            depth[2 * nz + z] = b[5] ? fp * norm / (double)b[5] : nan;
        }
    }
    if (threadIdx.x != 0) return;
    unsigned long long s_hi = 0, s_lo = 0, p_hi = 0, p_lo = 0, n_s = 0, n_p = 0, mx = 0;
    for (int32_t z = 0; z < nz; ++z) {
        const unsigned long long *b = bins + (uint64_t)z * kBinW;
        s_hi += b[0]; s_lo += b[1]; p_hi += b[2]; p_lo += b[3]; n_s += b[4]; n_p += b[5];
        mx = b[6] > mx ? b[6] : mx;
    }
    const double fs = join(s_hi, s_lo), fp = join(p_hi, p_lo);
    const double nvox = (double)(n_s + n_p);
    for (int i = 0; i < MC_NSUMMARY; ++i) q[i] = 0.0;
    q[MC_Q_PHI3D] = n_s ? fs * norm / (double)n_s : nan;
    q[MC_Q_PHI1D] = (fs + fp) * norm / nvox;
    q[MC_Q_PHI_PORE] = n_p ? fp * norm / (double)n_p : nan;
    q[MC_Q_R_CONTRAST] = q[MC_Q_PHI_PORE] / q[MC_Q_PHI3D];
    q[MC_Q_POROSITY] = (double)n_p / nvox;
    q[MC_Q_RATIO] = q[MC_Q_PHI3D] / q[MC_Q_PHI1D];
    // with no pore voxel the pore term of the identity is absent
    q[MC_Q_IDENTITY_RHS] =
        n_p ? 1.0 / (q[MC_Q_POROSITY] * q[MC_Q_R_CONTRAST] + (1.0 - q[MC_Q_POROSITY])) : 1.0;
    q[MC_Q_R] = (double)S[MC_S_R] / launched_w;
    q[MC_Q_T] = (double)S[MC_S_T] / launched_w;
    q[MC_Q_A] = (double)S[MC_S_A] / launched_w;
    q[MC_Q_RR] = (double)S[MC_S_RR] / launched_w;
    q[MC_Q_LOST] = (double)S[MC_S_LOST] / launched_w;
    const int64_t sum = S[MC_S_R] + S[MC_S_T] + S[MC_S_A] + S[MC_S_RR] + S[MC_S_LOST] + S[MC_S_GATED];
    q[MC_Q_CLOSURE_EXACT] = (sum == S[MC_S_LAUNCHED] * (int64_t)2147483648ll) ? 1.0 : 0.0;
    const unsigned long long *b0 = bins, *bl = bins + (uint64_t)(nz - 1) * kBinW;
    const double f0 = join(b0[0], b0[1]) + join(b0[2], b0[3]);
    const double fl = join(bl[0], bl[1]) + join(bl[2], bl[3]);
    q[MC_Q_FRONT_BACK] = fl > 0.0 ? f0 / fl : __builtin_inf();
    q[MC_Q_L_OPT] = q[MC_Q_PHI1D] * (double)nz;
    q[MC_Q_ESC_FRAC] = (double)S[MC_S_ESC_W] / launched_w;
    q[MC_Q_PW_VOID_GTL] = S[MC_S_ESC_W] ? (double)S[MC_S_ESC_W_GTL] / (double)S[MC_S_ESC_W] : nan;
    q[MC_Q_PN_VOID_GTL] = S[MC_S_ESC_N] ? (double)S[MC_S_ESC_N_GTL] / (double)S[MC_S_ESC_N] : nan;
    const double void_path = join((unsigned long long)S[MC_S_ESC_W_VOID_PATH_HI],
                                  (unsigned long long)S[MC_S_ESC_W_VOID_PATH]);
    q[MC_Q_MEAN_VOID_PATH] = S[MC_S_ESC_W] ? void_path / (double)S[MC_S_ESC_W] : nan;
    q[MC_Q_STEPS_PER_PHOTON] = (double)S[MC_S_STEPS] / n_ph;
    q[MC_Q_INTERACTIONS_PER_PHOTON] = (double)S[MC_S_INTERACTIONS] / n_ph;
    // an overflowing voxel tally makes the run invalid; weight stopped by the step or
    // path cap leaves it valid but incomplete
    q[MC_Q_STATUS] = mx >= (1ull << 62) ? (double)MC_EOVERFLOW : (S[MC_S_LOST] > 0 ? (double)MC_WARN_LOST : 0.0);
    q[MC_Q_N_SOLID] = (double)n_s;
    q[MC_Q_LAUNCHED] = n_ph;
    q[MC_Q_GATED] = (double)S[MC_S_GATED] / launched_w;
}

// Jacobian of <Phi>_3D, <Phi>_1D and Phi(z) with respect to (mu_s, mu_a, g)
// from the gradient bins, normalised as the forward estimators (Phi/S0).
__device__ __forceinline__ double join_signed(unsigned long long hi, unsigned long long lo)
{
    return (double)(long long)hi * 4294967296.0 + (double)lo;
}

__global__ void k_grad_finalize(const unsigned long long *__restrict__ grad, const unsigned long long *__restrict__ bins,
                                const int64_t *__restrict__ S, int32_t nx, int32_t ny, int32_t nz,
                                double *__restrict__ jac)
{
    const double face = (double)nx * (double)ny;
    const double norm = face / ((double)S[MC_S_LAUNCHED] * 2147483648.0) / kGradScale;
    const int32_t row = 2 + nz;
    for (int32_t i = threadIdx.x; i < 3 * nz; i += blockDim.x) {
        const int32_t p = i / nz, z = i % nz;
        const unsigned long long *gs = grad + 2 * ((2 * p) * nz + z), *gp = grad + 2 * ((2 * p + 1) * nz + z);
        jac[p * row + 2 + z] = (join_signed(gs[0], gs[1]) + join_signed(gp[0], gp[1])) * norm / face;
    }
    if (threadIdx.x >= 3) return;
    const int32_t p = threadIdx.x;
    unsigned long long n_s = 0, n_p = 0, s_hi = 0, s_lo = 0, t_hi = 0, t_lo = 0;
    for (int32_t z = 0; z < nz; ++z) {
        n_s += bins[(uint64_t)z * kBinW + 4];
        n_p += bins[(uint64_t)z * kBinW + 5];
        const unsigned long long *gs = grad + 2 * ((2 * p) * nz + z), *gp = grad + 2 * ((2 * p + 1) * nz + z);
        s_hi += gs[0]; s_lo += gs[1];
        t_hi += gs[0] + gp[0]; t_lo += gs[1] + gp[1];
    }
    jac[p * row + 0] = n_s ? join_signed(s_hi, s_lo) * norm / (double)n_s : __builtin_nan("");
    jac[p * row + 1] = join_signed(t_hi, t_lo) * norm / (double)(n_s + n_p);
}

// ---------------------------------------------------------------------------
// Roofline probe: random 64-bit scatter-adds, the walk's deposit pattern
// without the walk.  Addresses come from a 64-bit mixer of (thread, i), scaled
// to the table (a multiple of 64 entries) by the high half of a 64 x 64-bit
// product.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// A uniform pick in [0, units) from 64 random bits.
__device__ __forceinline__ uint64_t pick(uint64_t x, uint64_t units) { return __umul64hi(x, units); }

// The FP32 transport's square root, sine and cosine of a turn, and logarithm over
// all 2^24 uniforms the walk draws (u = i 2^-24 for the turn and the square root,
// (i + 1) 2^-24 for the logarithm), against FP64: the largest absolute sine and
// cosine errors and relative logarithm and square-root errors, as the bit
// patterns of non-negative doubles (ordered as integers), maxima over the grid.
__global__ __launch_bounds__(256) void k_probe_math(unsigned long long *__restrict__ out)
{
    __shared__ double m[4][256];
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;   // the grid is exactly 2^24 threads
    const float u = (float)i * 0x1.0p-24f, v = (float)(i + 1u) * 0x1.0p-24f;
    float sf, cf;
    r_sincos_turn(u, &sf, &cf);
    double sd, cd;
    r_sincos_turn((double)u, &sd, &cd);
    const double ld = log((double)v), qd = sqrt((double)u);
    double e[4];
    e[0] = fabs((double)sf - sd);
    e[1] = fabs((double)cf - cd);
    e[2] = v < 1.0f ? fabs((double)r_log_unit(v) - ld) / fabs(ld) : fabs((double)r_log_unit(v));
    e[3] = i ? fabs((double)r_sqrt(u) - qd) / qd : fabs((double)r_sqrt(u));
    for (int j = 0; j < 4; ++j) m[j][threadIdx.x] = e[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < (unsigned)st)
            for (int j = 0; j < 4; ++j) m[j][threadIdx.x] = fmax(m[j][threadIdx.x], m[j][threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x < 4) atomicMax(&out[threadIdx.x], (unsigned long long)__double_as_longlong(m[threadIdx.x][0]));
}

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(unsigned long long *__restrict__ table, uint64_t n, uint64_t per_thread)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t wave = t >> 6, lane = t & 63;
    unsigned long long sink = 0;   // the returning modes use what the atomics return
    for (uint64_t i = 0; i < per_thread; ++i) {
        const uint64_t a = pick(mix64(t * per_thread + i), n);
        if (MODE == 0) {
            __hip_atomic_fetch_add(table + a, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE == 1) {
            __hip_atomic_fetch_add(table + a, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (MODE == 2) {
            table[a] = i;
        } else if (MODE == 3) {
            // 32-bit atomic add at a random 32-bit slot
            unsigned int *t32 = (unsigned int *)table;
            __hip_atomic_fetch_add(t32 + ((a << 1) | (i & 1)), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE == 4) {
            // the 64 lanes of a wavefront hit 64 consecutive slots of one random block
            const uint64_t blk = pick(mix64(wave * per_thread + i), n / 64) * 64;
            __hip_atomic_fetch_add(table + blk + lane, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE >= 5 && MODE <= 7) {
            // groups of G lanes hit G consecutive slots (G * 8 bytes) of a random aligned block
            constexpr uint64_t G = MODE == 5 ? 16 : (MODE == 6 ? 8 : 4);
            const uint64_t grp = (t >> (MODE == 5 ? 4 : (MODE == 6 ? 3 : 2)));
            const uint64_t blk = pick(mix64(grp * per_thread + i), n / G) * G;
            __hip_atomic_fetch_add(table + blk + (lane & (G - 1)), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE == 8) {
            // 64-bit atomic add returning the old value, random slot
            sink += __hip_atomic_fetch_add(table + a, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE == 9) {
            // 32-bit atomic add returning the old value, random slot
            unsigned int *t32 = (unsigned int *)table;
            sink += __hip_atomic_fetch_add(t32 + ((a << 1) | (i & 1)), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (MODE == 10 || MODE == 11) {
            // groups of 16 lanes on the 16 consecutive 32-bit slots of a random 64-byte line,
            // without (10) or with (11) the old value returned
            unsigned int *t32 = (unsigned int *)table;
            const uint64_t blk = pick(mix64((t >> 4) * per_thread + i), n / 8) * 8;
            unsigned int *p32 = t32 + 2 * blk + (lane & 15);
            if (MODE == 10) __hip_atomic_fetch_add(p32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else sink += __hip_atomic_fetch_add(p32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // groups of 8 lanes on one random 64-byte line, 64-bit, the old value returned
            const uint64_t blk = pick(mix64((t >> 3) * per_thread + i), n / 8) * 8;
            sink += __hip_atomic_fetch_add(table + blk + (lane & 7), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // never true for the counts these modes add (the sums stay far below 2^64 - 1); it keeps
    // the returned values live
    if (sink == ~0ull) table[0] = sink;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace pmc {
namespace host {

Dims dims_of(const mc_volume *v)
{
    Dims d;
    d.nxb = (v->nx + 3) / 4;
    d.nyb = (v->ny + 3) / 4;
    d.nzb = (v->nz + 3) / 4;
    d.nbricks = (uint64_t)d.nxb * d.nyb * d.nzb;
    d.nvox = (uint64_t)v->nx * v->ny * v->nz;
    d.lnx = (v->nx + 1) / 2;
    d.lny = (v->ny + 1) / 2;
    d.lnz = (v->nz + 3) / 4;
    d.line_words = (uint64_t)d.lnx * d.lny * d.lnz * 16;
    const uint64_t plane_words = plane_dims(v->nx, v->ny, v->nz).words;
    d.planes = plane_words * sizeof(uint32_t) <= kPlaneStageMaxBytes;
    d.stage_words = d.planes ? plane_words : d.line_words;
    d.logged = d.stage_words <= (1ull << 32);
    return d;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

size_t stage_offset(const Dims &d) { return kHeaderBytes + align256(d.nbricks * sizeof(uint64_t)); }

size_t run_workspace_bytes(const Dims &d)
{
    return stage_offset(d) + (d.logged ? align256(d.stage_words * sizeof(uint32_t)) : 0);
}

int check_volume(const mc_volume *v)
{
    if (!v) return fail(MC_EINVAL, "volume is NULL");
    if (v->nx < 1 || v->ny < 1 || v->nz < 1 || v->nx > 65535 || v->ny > 65535 || v->nz > 65535)
        return fail(MC_EINVAL, "volume dimensions %d x %d x %d outside [1, 65535]", v->nx, v->ny, v->nz);
    if ((uint64_t)v->nx * v->ny * v->nz >= (1ull << 34))
        return fail(MC_EINVAL, "volume has 2^34 or more voxels");
    if (!v->mask) return fail(MC_EINVAL, "mask pointer is NULL");
    return MC_OK;
}

int make_job(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons, uint64_t seed,
             uint32_t stream_id, Job *J)
{
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!opt) return fail(MC_EINVAL, "optics is NULL");
    if (!(opt->mu_s >= 0.0f) || !(opt->mu_a >= 0.0f) || !isfinite(opt->mu_s) || !isfinite(opt->mu_a))
        return fail(MC_EINVAL, "mu_s and mu_a must be finite and >= 0");
    if (!(fabsf(opt->g) < 1.0f)) return fail(MC_EINVAL, "|g| must be < 1");
    if (opt->roulette_m < 2) return fail(MC_EINVAL, "roulette_m must be >= 2");
    if (!(opt->w_roulette >= 0.0f) || !(opt->w_roulette <= 1.0f)) return fail(MC_EINVAL, "w_roulette must be in [0, 1]");
    const double w_th = floor((double)opt->w_roulette * 2147483648.0);
    if (w_th * (double)opt->roulette_m > 2147483648.0)
        return fail(MC_EINVAL, "w_roulette * roulette_m must not exceed 1 (a survivor would outweigh a launched photon)");
    if (opt->source != 0 && opt->source != 1) return fail(MC_EINVAL, "source must be 0 or 1");
    const bool gate_on = opt->gate > 0.0 && !isinf(opt->gate);
    if (isnan(opt->gate)) return fail(MC_EINVAL, "gate is NaN");
    if (opt->reserved != 0) return fail(MC_EINVAL, "mc_optics.reserved must be 0");
    if (opt->boundary == MC_BOUNDARY_PLAIN) {
        if (opt->lateral != MC_LATERAL_PERIODIC || (opt->n_solid != 0.0f && opt->n_solid != 1.0f) || gate_on)
            return fail(MC_EINVAL, "the plain boundary model has periodic laterals, index 1 and no time gate");
    } else if (opt->boundary == MC_BOUNDARY_PAPER) {
        if (opt->lateral != MC_LATERAL_PERIODIC && opt->lateral != MC_LATERAL_MIRROR)
            return fail(MC_EINVAL, "lateral must be MC_LATERAL_PERIODIC or MC_LATERAL_MIRROR");
        if (opt->n_solid != 0.0f && !(opt->n_solid >= 1.0f && isfinite(opt->n_solid)))
            return fail(MC_EINVAL, "n_solid must be finite and >= 1 (0 selects 1)");
    } else {
        return fail(MC_EINVAL, "boundary must be MC_BOUNDARY_PLAIN or MC_BOUNDARY_PAPER");
    }
    if (n_photons == 0) return fail(MC_EINVAL, "n_photons is 0");
    if (photon_begin >= (1ull << 32) || n_photons > (1ull << 32) - photon_begin)
        return fail(MC_EINVAL, "photon ids must be < 2^32");
    memset(J, 0, sizeof *J);
    const Dims d = dims_of(vol);
    J->nx = vol->nx;
    J->ny = vol->ny;
    J->nz = vol->nz;
    J->nxb = d.nxb;
    J->nyb = d.nyb;
    J->lnx = d.lnx;
    J->lny = d.lny;
    const PlaneDims pd = plane_dims(vol->nx, vol->ny, vol->nz);
    J->stage_off1 = pd.off1;
    J->stage_off2 = pd.off2;
    const double mu_s = opt->mu_s, mu_a = opt->mu_a, mu_t = mu_s + mu_a;
    J->mu_t = mu_t;
    J->mu_s = mu_s;
    J->g = opt->g;
    J->path_cap = opt->path_cap > 0.0f ? opt->path_cap : kInf;
    J->s_q = mu_t > 0.0 ? (uint64_t)llround(mu_s / mu_t * 4294967296.0) : 0ull;
    J->w_th = (uint32_t)w_th;
    J->t_m = (uint32_t)llround(16777216.0 / (double)opt->roulette_m);
    J->m = opt->roulette_m;
    J->key0 = (uint32_t)seed;
    J->key1 = (uint32_t)(seed >> 32);
    J->stream_id = stream_id;
    J->source = opt->source;
    J->max_steps = opt->max_steps ? opt->max_steps : (1u << 24);
    J->photon_begin = photon_begin;
    J->n_photons = n_photons;
    J->queue_begin = 0;
    J->paper = opt->boundary == MC_BOUNDARY_PAPER ? 1 : 0;
    J->lateral = opt->lateral;
    J->n_solid = opt->n_solid == 0.0f ? 1.0f : opt->n_solid;
    J->fresnel = J->n_solid != 1.0f ? 1 : 0;
    J->gate = gate_on ? opt->gate : (double)kInf;
    return MC_OK;
}

int device_info(DeviceInfo *out)
{
    static std::mutex mu;
    static DeviceInfo cache[64];
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0 || dev >= 64) return fail(MC_EHIP, "device index %d out of range", dev);
    if (cache[dev].cus == 0) HIP_TRY(hipDeviceGetAttribute(&cache[dev].cus, hipDeviceAttributeMultiprocessorCount, dev));
    *out = cache[dev];
    return MC_OK;
}

mc_tune resolve_tune(const mc_tune *t, int32_t defer_default)
{
    mc_tune r;
    mc_tune_default(&r);
    if (defer_default > 0) r.defer = defer_default;
    if (t) {
        if (t->block > 0) r.block = t->block;
        if (t->waves_per_cu > 0) r.waves_per_cu = t->waves_per_cu;
        if (t->chunk > 0) r.chunk = t->chunk;
        if (t->refill > 0) r.refill = t->refill;
        if (t->defer > 0) r.defer = t->defer;
    }
    return r;
}

int check_tune(const mc_tune &t)
{
    if (t.block != 64 && t.block != 128 && t.block != 256 && t.block != 512)
        return fail(MC_EINVAL, "tune: block size %d not one of 64, 128, 256, 512", t.block);
    if (t.chunk < 1 || t.refill < 1 || t.refill > 64 || t.waves_per_cu < 1 || t.waves_per_cu > 32 || t.defer < 1 ||
        t.defer > 64)
        return fail(MC_EINVAL,
                    "tune out of range (chunk >= 1, refill and defer in [1, 64], waves_per_cu in [1, 32])");
    return MC_OK;
}

int fill(int64_t *p, uint64_t n, hipStream_t s)
{
    if (n == 0) return MC_OK;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, (int64_t)0);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int pack(const mc_volume *vol, uint64_t *bricks, hipStream_t s)
{
    const Dims d = dims_of(vol);
    const uint64_t blocks = (d.nbricks + 255) / 256;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, vol->mask, vol->nx, vol->ny, vol->nz, d.nxb,
                       d.nyb, d.nbricks, bricks);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

thread_local Timing g_timing;

Timing &timing() { return g_timing; }

int time_begin(hipStream_t s)
{
    if (!g_timing.start) {
        HIP_TRY(hipEventCreate(&g_timing.start));
        HIP_TRY(hipEventCreate(&g_timing.stop));
    }
    HIP_TRY(hipEventRecord(g_timing.start, s));
    return MC_OK;
}

int time_end(hipStream_t s)
{
    HIP_TRY(hipEventRecord(g_timing.stop, s));
    g_timing.armed = true;
    return MC_OK;
}

int enqueue_reduce(const mc_volume *vol, const int64_t *fluence, const int64_t *scalars, double *summary,
                   double *depth, unsigned long long *bins, hipStream_t s)
{
    int rc = fill((int64_t *)bins, (uint64_t)vol->nz * kBinW, s);
    if (rc) return rc;
    const uint64_t layer = (uint64_t)vol->nx * vol->ny;
    const uint64_t per_block = 8192;
    const uint64_t gx = (layer + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)gx, (unsigned)vol->nz), dim3(kReduceBlock), 0, s, fluence, vol->mask,
                       layer, per_block, bins);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, bins, scalars, vol->nx, vol->ny, vol->nz, summary, depth);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

template <typename R, bool GRAD, bool LOGGED, bool GENERAL, bool ESC>
void enqueue_walk(int block, int blocks, const Job &J, unsigned long long *queue, const mc_tune &t,
                  unsigned long long *grad, const EscHist &eh, hipStream_t s)
{
    const size_t lds = GRAD ? (size_t)6 * J.nz * sizeof(int)
                            : (ESC ? (size_t)eh.nbins * (sizeof(unsigned long long) + sizeof(unsigned int)) : 0);
    switch (block) {
    case 64:
        hipLaunchKernelGGL((k_walk<64, R, GRAD, LOGGED, GENERAL, ESC>), dim3(blocks), dim3(64), lds, s, J, queue, t.chunk,
                           t.refill, t.defer, grad, eh);
        break;
    case 128:
        hipLaunchKernelGGL((k_walk<128, R, GRAD, LOGGED, GENERAL, ESC>), dim3(blocks), dim3(128), lds, s, J, queue,
                           t.chunk, t.refill, t.defer, grad, eh);
        break;
    case 256:
        hipLaunchKernelGGL((k_walk<256, R, GRAD, LOGGED, GENERAL, ESC>), dim3(blocks), dim3(256), lds, s, J, queue,
                           t.chunk, t.refill, t.defer, grad, eh);
        break;
    default:
        hipLaunchKernelGGL((k_walk<512, R, GRAD, LOGGED, GENERAL, ESC>), dim3(blocks), dim3(512), lds, s, J, queue,
                           t.chunk, t.refill, t.defer, grad, eh);
        break;
    }
}

template <typename R, bool GRAD, bool ESC>
void enqueue_walk_dep(bool logged, int block, int blocks, const Job &J, unsigned long long *queue, const mc_tune &t,
                      unsigned long long *grad, const EscHist &eh, hipStream_t s)
{
    if (J.paper) {
        if (logged) enqueue_walk<R, GRAD, true, true, ESC>(block, blocks, J, queue, t, grad, eh, s);
        else enqueue_walk<R, GRAD, false, true, ESC>(block, blocks, J, queue, t, grad, eh, s);
    } else {
        if (logged) enqueue_walk<R, GRAD, true, false, ESC>(block, blocks, J, queue, t, grad, eh, s);
        else enqueue_walk<R, GRAD, false, false, ESC>(block, blocks, J, queue, t, grad, eh, s);
    }
}

int launch_walk(const Job &J, unsigned long long *queue, const mc_tune &t, hipStream_t s, int flags,
                unsigned long long *grad, bool logged, const EscHist *esc)
{
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    const int waves_per_block = t.block / 64;
    const int blocks = std::max(1, di.cus * t.waves_per_cu / waves_per_block);
    const bool timed = (flags & MC_TIMED) != 0;
    if (timed && (rc = time_begin(s))) return rc;
    const EscHist none = {nullptr, nullptr, 1.0, 0};
    if (grad) {
        if (flags & MC_FP64) enqueue_walk_dep<double, true, false>(logged, t.block, blocks, J, queue, t, grad, none, s);
        else enqueue_walk_dep<float, true, false>(logged, t.block, blocks, J, queue, t, grad, none, s);
    } else if (esc) {
        if (flags & MC_FP64) enqueue_walk_dep<double, false, true>(logged, t.block, blocks, J, queue, t, nullptr, *esc, s);
        else enqueue_walk_dep<float, false, true>(logged, t.block, blocks, J, queue, t, nullptr, *esc, s);
    } else {
        if (flags & MC_FP64) enqueue_walk_dep<double, false, false>(logged, t.block, blocks, J, queue, t, nullptr, none, s);
        else enqueue_walk_dep<float, false, false>(logged, t.block, blocks, J, queue, t, nullptr, none, s);
    }
    HIP_TRY(hipGetLastError());
    if (timed && (rc = time_end(s))) return rc;
    return MC_OK;
}

// Zero the tallies (unless accumulating), pack the mask, walk, and for the
// logged deposit path add the staged quanta to the caller's tally.
int run_walk(const mc_volume *vol, Job J, int flags, const mc_tune &t, char *ws, unsigned long long *grad_bins,
             hipStream_t s, const EscHist *esc)
{
    const Dims d = dims_of(vol);
    const bool logged = d.logged && !(flags & MC_DIRECT_DEPOSIT);
    unsigned long long *queue = (unsigned long long *)ws;
    uint64_t *bricks = (uint64_t *)(ws + kHeaderBytes);
    uint32_t *stage = (uint32_t *)(ws + stage_offset(d));
    int rc;
    if (!(flags & MC_ACCUMULATE)) {
        if ((rc = fill(J.fluence, d.nvox, s))) return rc;
        if ((rc = fill(J.scalars, MC_NSCALARS, s))) return rc;
        if (grad_bins && (rc = fill((int64_t *)grad_bins, (uint64_t)12 * vol->nz, s))) return rc;
        if (esc && (rc = fill((int64_t *)esc->w, (uint64_t)esc->nbins, s))) return rc;
        if (esc && (rc = fill((int64_t *)esc->n, (uint64_t)esc->nbins, s))) return rc;
    }
    // the staging words as int64 pairs: a line is 16 words, so the count is even
    const bool planes = d.planes && !(flags & (MC_LINE_STAGING | MC_FP64));
    if (logged && (rc = fill((int64_t *)stage, (planes ? d.stage_words : d.line_words) / 2, s))) return rc;
    if ((rc = fill((int64_t *)queue, kHeaderBytes / 8, s))) return rc;
    if ((rc = pack(vol, bricks, s))) return rc;
    J.bricks = bricks;
    J.stage = logged ? stage : nullptr;
    J.stage_planes = logged && planes;
    if ((rc = launch_walk(J, queue, t, s, flags, grad_bins, logged, esc))) return rc;
    if (logged) return unstage(stage, J.fluence, vol, planes, s);
    return MC_OK;
}

int unstage(const uint32_t *stage, int64_t *fluence, const mc_volume *vol, bool planes, hipStream_t s)
{
    const Dims d = dims_of(vol);
    const uint64_t blocks = std::min<uint64_t>((d.nvox + 255) / 256, 16384);
    hipLaunchKernelGGL(k_unstage, dim3((unsigned)blocks), dim3(256), 0, s, stage, fluence, vol->nx, vol->ny, vol->nz,
                       d.lnx, d.lny, (int32_t)planes);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // namespace host
}  // namespace pmc

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int mc_abi_version(void) { return MC_ABI_VERSION; }

size_t mc_sizeof(const char *type_name)
{
    if (!type_name) return 0;
    if (!strcmp(type_name, "mc_volume")) return sizeof(mc_volume);
    if (!strcmp(type_name, "mc_optics")) return sizeof(mc_optics);
    if (!strcmp(type_name, "mc_ch_grid")) return sizeof(mc_ch_grid);
    if (!strcmp(type_name, "mc_tune")) return sizeof(mc_tune);
    if (!strcmp(type_name, "mc_trace_rec")) return sizeof(mc_trace_rec);
    if (!strcmp(type_name, "mc_photon_rec")) return sizeof(mc_photon_rec);
    if (!strcmp(type_name, "mc_job")) return sizeof(mc_job);
    if (!strcmp(type_name, "mc_escape_bins")) return sizeof(mc_escape_bins);
    return 0;
}

const char *mc_last_error(void) { return g_err; }

const char *mc_strerror(int status)
{
    switch (status) {
    case MC_OK: return "ok";
    case MC_WARN_LOST: return "warning: weight stopped by the step or path cap";
    case MC_EINVAL: return "invalid argument";
    case MC_EOVERFLOW: return "a voxel tally reached 2^62";
    case MC_EHIP: return "HIP runtime error";
    case MC_ENOSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

void mc_tune_default(mc_tune *t)
{
    if (!t) return;
    t->block = 256;
    t->waves_per_cu = 16;
    t->chunk = 256;
    t->refill = 16;
    t->defer = 4;
}

size_t mc_run_workspace_bytes(const mc_volume *vol)
{
    if (check_volume(vol)) return 0;
    return run_workspace_bytes(dims_of(vol));
}

int mc_run(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons, uint64_t seed,
           uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars, void *workspace, size_t workspace_bytes,
           const mc_tune *tune, void *hip_stream)
{
    clear_error();
    Job J;
    int rc = make_job(vol, opt, photon_begin, n_photons, seed, stream_id, &J);
    if (rc) return rc;
    if (!fluence || !scalars || !workspace) return fail(MC_EINVAL, "fluence, scalars and workspace must be non-NULL");
    const size_t need = mc_run_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    const mc_tune t = resolve_tune(tune, (J.paper || (flags & MC_FP64)) ? kDeferVALUBound : 0);
    if ((rc = check_tune(t))) return rc;
    J.fluence = fluence;
    J.scalars = scalars;
    return run_walk(vol, J, flags, t, (char *)workspace, nullptr, (hipStream_t)hip_stream);
}

int mc_run_escape_histogram(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons,
                            uint64_t seed, uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars,
                            void *workspace, size_t workspace_bytes, const mc_tune *tune, double bin_width,
                            int32_t nbins, int64_t *hist_w, int64_t *hist_n, void *hip_stream)
{
    clear_error();
    if (!hist_w || !hist_n) return fail(MC_EINVAL, "hist_w and hist_n must be non-NULL");
    if (nbins < 1 || nbins > kEscMaxBins) return fail(MC_EINVAL, "nbins must be in [1, %d]", kEscMaxBins);
    if (!(bin_width > 0.0) || !isfinite(bin_width)) return fail(MC_EINVAL, "bin_width must be finite and > 0");
    Job J;
    int rc = make_job(vol, opt, photon_begin, n_photons, seed, stream_id, &J);
    if (rc) return rc;
    if (!fluence || !scalars || !workspace) return fail(MC_EINVAL, "fluence, scalars and workspace must be non-NULL");
    const size_t need = mc_run_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    const mc_tune t = resolve_tune(tune, (J.paper || (flags & MC_FP64)) ? kDeferVALUBound : 0);
    if ((rc = check_tune(t))) return rc;
    J.fluence = fluence;
    J.scalars = scalars;
    const EscHist esc = {(unsigned long long *)hist_w, (unsigned long long *)hist_n, bin_width, nbins};
    return run_walk(vol, J, flags, t, (char *)workspace, nullptr, (hipStream_t)hip_stream, &esc);
}

int mc_walk_elapsed_ms(float *ms)
{
    if (!ms) return fail(MC_EINVAL, "ms is NULL");
    if (!g_timing.armed) return fail(MC_EINVAL, "no timed walk has been enqueued on this thread");
    HIP_TRY(hipEventSynchronize(g_timing.stop));
    HIP_TRY(hipEventElapsedTime(ms, g_timing.start, g_timing.stop));
    return MC_OK;
}

size_t mc_reduce_workspace_bytes(const mc_volume *vol)
{
    if (check_volume(vol)) return 0;
    return (size_t)vol->nz * kBinW * sizeof(uint64_t);
}

int mc_reduce(const mc_volume *vol, const int64_t *fluence, const int64_t *scalars, double *summary, double *depth,
              void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    int rc = check_volume(vol);
    if (rc) return rc;
    if (!fluence || !scalars || !summary || !workspace) return fail(MC_EINVAL, "NULL argument");
    const size_t need = mc_reduce_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return enqueue_reduce(vol, fluence, scalars, summary, depth, (unsigned long long *)workspace,
                          (hipStream_t)hip_stream);
}

int mc_trace(const mc_volume *vol, const mc_optics *opt, const uint64_t *photon_ids, int32_t n, int32_t max_steps,
             uint64_t seed, uint32_t stream_id, int flags, mc_trace_rec *recs, mc_photon_rec *outcome,
             void *workspace, size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    Job J;
    int rc = make_job(vol, opt, 0, 1, seed, stream_id, &J);
    if (rc) return rc;
    if (n < 0 || max_steps < 0) return fail(MC_EINVAL, "n and max_steps must be >= 0");
    if (n == 0) return MC_OK;
    if (!photon_ids || !workspace || (max_steps > 0 && !recs)) return fail(MC_EINVAL, "NULL argument");
    const size_t need = mc_run_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t s = (hipStream_t)hip_stream;
    uint64_t *bricks = (uint64_t *)((char *)workspace + kHeaderBytes);
    J.bricks = bricks;
    if ((rc = pack(vol, bricks, s))) return rc;
    const dim3 grid((unsigned)((n + 63) / 64));
    if (flags & MC_FP64) {
        if (J.paper)
            hipLaunchKernelGGL((k_trace<double, true>), grid, dim3(64), 0, s, J, photon_ids, n, max_steps, recs, outcome);
        else
            hipLaunchKernelGGL((k_trace<double, false>), grid, dim3(64), 0, s, J, photon_ids, n, max_steps, recs, outcome);
    } else {
        if (J.paper)
            hipLaunchKernelGGL((k_trace<float, true>), grid, dim3(64), 0, s, J, photon_ids, n, max_steps, recs, outcome);
        else
            hipLaunchKernelGGL((k_trace<float, false>), grid, dim3(64), 0, s, J, photon_ids, n, max_steps, recs, outcome);
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

size_t mc_grad_workspace_bytes(const mc_volume *vol)
{
    if (check_volume(vol)) return 0;
    return mc_run_workspace_bytes(vol) + mc_reduce_workspace_bytes(vol) + MC_NSUMMARY * sizeof(double);
}

int mc_grad(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons, uint64_t seed,
            uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars, int64_t *grad_bins, double *jac,
            double *summary, double *depth, void *workspace, size_t workspace_bytes, const mc_tune *tune,
            void *hip_stream)
{
    clear_error();
    Job J;
    int rc = make_job(vol, opt, photon_begin, n_photons, seed, stream_id, &J);
    if (rc) return rc;
    if (vol->nz > MC_GRAD_MAX_NZ) return fail(MC_EINVAL, "mc_grad supports nz <= %d (got %d)", MC_GRAD_MAX_NZ, vol->nz);
    if (!fluence || !scalars || !grad_bins || !workspace)
        return fail(MC_EINVAL, "fluence, scalars, grad_bins and workspace must be non-NULL");
    const size_t need = mc_grad_workspace_bytes(vol);
    if (workspace_bytes < need) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    const mc_tune t = resolve_tune(tune, kDeferVALUBound);
    if ((rc = check_tune(t))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    char *ws = (char *)workspace;
    unsigned long long *bins = (unsigned long long *)(ws + mc_run_workspace_bytes(vol));
    double *scratch_q = (double *)(ws + mc_run_workspace_bytes(vol) + mc_reduce_workspace_bytes(vol));
    J.fluence = fluence;
    J.scalars = scalars;
    if ((rc = run_walk(vol, J, flags, t, ws, (unsigned long long *)grad_bins, s))) return rc;
    if (jac || summary || depth) {
        if ((rc = enqueue_reduce(vol, fluence, scalars, summary ? summary : scratch_q, depth, bins, s))) return rc;
    }
    if (jac) {
        hipLaunchKernelGGL(k_grad_finalize, dim3(1), dim3(256), 0, s, (const unsigned long long *)grad_bins, bins,
                           scalars, vol->nx, vol->ny, vol->nz, jac);
        HIP_TRY(hipGetLastError());
    }
    return MC_OK;
}

int mc_probe_math(double *max_err, void *hip_stream)
{
    clear_error();
    if (!max_err) return fail(MC_EINVAL, "max_err is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = fill((int64_t *)max_err, 4, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_probe_math, dim3(1u << 16), dim3(256), 0, s, (unsigned long long *)max_err);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

int mc_probe_scatter(int64_t *table, uint64_t n_entries, uint64_t n_ops, int mode, int waves_per_cu,
                     void *hip_stream)
{
    clear_error();
    if (!table || n_entries < 64 || n_entries % 64 != 0)
        return fail(MC_EINVAL, "table must be non-NULL with an entry count that is a multiple of 64");
    if (mode < 0 || mode > 12) return fail(MC_EINVAL, "mode must be in [0, 12]");
    if (waves_per_cu == 0) waves_per_cu = 16;
    if (waves_per_cu < 4 || waves_per_cu > 32 || waves_per_cu % 4)
        return fail(MC_EINVAL, "waves_per_cu must be 0 (16) or a multiple of 4 in [4, 32]");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    const uint64_t threads = (uint64_t)di.cus * (uint64_t)waves_per_cu * 64;
    const uint64_t per_thread = std::max<uint64_t>(1, n_ops / threads);
    const unsigned blocks = (unsigned)(threads / 256);
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long *t = (unsigned long long *)table;
    const uint64_t m = n_entries;
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe<0>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 5: hipLaunchKernelGGL(k_probe<5>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 6: hipLaunchKernelGGL(k_probe<6>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 7: hipLaunchKernelGGL(k_probe<7>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 8: hipLaunchKernelGGL(k_probe<8>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 9: hipLaunchKernelGGL(k_probe<9>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 10: hipLaunchKernelGGL(k_probe<10>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    case 11: hipLaunchKernelGGL(k_probe<11>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    default: hipLaunchKernelGGL(k_probe<12>, dim3(blocks), dim3(256), 0, s, t, m, per_thread); break;
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // extern "C"

