// batch.hip -- many masks of uneven size, porosity and optics in one
// persistent launch; a captured HIP graph of the whole batched step; and the
// launch-shape autotuner with its on-disk cache.
//
// The job table is ordered longest-first (photons x depth as the cost
// estimate) and concatenated into one photon queue; a wavefront's chunk may
// straddle two jobs, so every lane carries its own job index and reads that
// job's constants from a copy of the table staged in LDS.  Each job draws its
// own Philox streams (seed, stream id), so job k of a batch is bitwise the same
// as a plain run of that job.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace pmc;
using namespace pmc::host;

static_assert(sizeof(Job) % 8 == 0, "job table is staged in 8-byte words");

namespace {

// Writes up to 8 job descriptors, passed by value, into the device table.
struct JobPack {
    Job j[8];
};

__global__ void k_write_jobs(JobPack pack, Job *__restrict__ dst, int32_t count)
{
    const int32_t w = (int32_t)(sizeof(Job) / 8);
    const uint64_t *src = (const uint64_t *)pack.j;
    uint64_t *d = (uint64_t *)dst;
    for (int32_t i = threadIdx.x; i < count * w; i += blockDim.x) d[i] = src[i];
}

// The escape-path histogram of one job (table order), NULL w: none.  Read only
// when a photon escapes, so it stays in global memory, not in the LDS job table.
// The walk adds into kEscReplicas copies in the workspace, a workgroup's copy
// chosen by its index: a batch runs its jobs longest first, so at any time most
// of the chip's escapes go to a few bins of one job, and one 64-byte line takes
// only ~1e8 atomics per second at the memory side.  k_esc_fold adds the copies
// into the caller's bins after the walk.
constexpr int kEscReplicas = 16;
struct BatchEsc {
    unsigned long long *w;    // [nbins] escaped Q31 weight (the caller's)
    unsigned long long *n;    // [nbins] escaped photons (the caller's)
    unsigned long long *rw;   // [kEscReplicas][kEscMaxBins] copies of w (workspace)
    unsigned long long *rn;   // [kEscReplicas][kEscMaxBins] copies of n (workspace)
    double width;
    int32_t nbins;
    int32_t pad;
};
static_assert(sizeof(BatchEsc) % 8 == 0, "histogram table is written in 8-byte words");
constexpr size_t kEscReplicaWords = 2ull * kEscReplicas * kEscMaxBins;   // per job: copies of w and n

struct EscPack {
    BatchEsc e[16];
};

__global__ void k_write_esc(EscPack pack, BatchEsc *__restrict__ dst, int32_t count)
{
    const int32_t w = (int32_t)(sizeof(BatchEsc) / 8);
    const uint64_t *src = (const uint64_t *)pack.e;
    uint64_t *d = (uint64_t *)dst;
    for (int32_t i = threadIdx.x; i < count * w; i += blockDim.x) d[i] = src[i];
}

// One workgroup per job: bin b of the caller's histogram += the sum of its copies.
__global__ __launch_bounds__(256) void k_esc_fold(const BatchEsc *__restrict__ esc)
{
    const BatchEsc e = esc[blockIdx.x];
    if (e.w == nullptr) return;
    for (int32_t b = threadIdx.x; b < e.nbins; b += blockDim.x) {
        unsigned long long sw = 0ull, sn = 0ull;
        for (int r = 0; r < kEscReplicas; ++r) {
            sw += e.rw[(size_t)r * kEscMaxBins + b];
            sn += e.rn[(size_t)r * kEscMaxBins + b];
        }
        e.w[b] += sw;
        e.n[b] += sn;
    }
}

struct BatchTallySink {
    template <typename R> __device__ __forceinline__ void segment(const Photon<R> &, const Job &, R, bool) {}
    template <typename R> __device__ __forceinline__ void deflect(Photon<R> &, const Job &, R) {}
    template <typename R> __device__ __forceinline__ void flush(const Job &J, const Photon<R> &p, uint64_t a)
    {
        if (a != 0ull)
            __hip_atomic_fetch_add((unsigned long long *)(J.fluence + voxel_index(J, p)),
                                   (unsigned long long)a << kDepositShift, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Line-coalesced deposits for the batch: as the plain walk's log (8-byte
// entries, 16 slots per lane, issued transposed once some lane has filled its
// slots, the run of entries in the line a photon still deposits into held back,
// uint32 staging words in each job's own layout, planes or lines, carries of
// wrapped words into the job's int64 tally), with the job index in the top 6 bits
// of the 32-bit entry index, which leaves 26 bits for the word index into the
// job's staging tally (the batch logs only when every job's staging tally is that
// small).  A deposit of 2^31 quanta or more goes to the job's tally directly.  The
// log's 33 KB of LDS per 256-thread workgroup, with the job table and the per-job
// channels, still lets three workgroups share a CU.
constexpr int kBLogK = 16;
constexpr int kBLogStride = 65;
#ifndef MC_LOG_HOLD
#define MC_LOG_HOLD 6
#endif
constexpr int kBLogHold = MC_LOG_HOLD;
constexpr uint32_t kBNoLine = 0xFFFFFFFFu;
constexpr int kJobShift = 26;
constexpr uint32_t kIdxMask = (1u << kJobShift) - 1u;
constexpr uint64_t kBatchLogWords = 1ull << kJobShift;   // largest staging tally a logged batch job may have

struct BatchLoggedSink {
    uint32_t *lidx;
    uint32_t *lval;
    uint32_t lane;
    uint32_t head, count;       // this lane's ring of kBLogK slots
    uint32_t tag;               // job << kJobShift
    template <typename R> __device__ __forceinline__ void segment(const Photon<R> &, const Job &, R, bool) {}
    template <typename R> __device__ __forceinline__ void deflect(Photon<R> &, const Job &, R) {}
    template <typename R> __device__ __forceinline__ void flush(const Job &J, const Photon<R> &p, uint64_t a)
    {
        if (a != 0ull) {
            if (a >> 31) {
                __hip_atomic_fetch_add((unsigned long long *)(J.fluence + voxel_index(J, p)),
                                       (unsigned long long)a << kDepositShift, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            } else {
                const uint32_t s = log_slot<kBLogStride, kBLogK>(lane, head, count);
                lidx[s] = stage_word(J, p) | tag;
                lval[s] = (uint32_t)a;
                ++count;
            }
        }
    }
};

// Issue the wavefront's log; HOLD: the newest run of each lane's log that lies in
// `line` (job bits included; kBNoLine: none) stays as the lane's ring.  The FP64
// transport holds nothing.
template <bool HOLD>
__device__ __forceinline__ void flush_batch_log(uint32_t *lidx, uint32_t *lval, const Job *jobs, uint32_t lane,
                                                uint32_t line, uint32_t &head, uint32_t &count)
{
    const uint32_t held = HOLD ? log_mark_run<kBLogStride, kBLogK, kBLogHold>(lidx, lval, lane, head, count, line) : 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // in two halves, each issuing its adds before it looks at what they returned
#pragma unroll
    for (int h = 0; h < kBLogK; h += kBLogK / 2) {
        uint32_t old[kBLogK / 2];
#pragma unroll
        for (int i = 0; i < kBLogK / 2; ++i) {
            const uint32_t src = (uint32_t)(h + i) * (64 / kBLogK) + lane / kBLogK;
            const uint32_t e = (lane % kBLogK) * kBLogStride + src;
            const uint32_t v = lval[e];
            old[i] = 0u;
            if (v != 0u && (!HOLD || v < kLogHeld)) {
                const uint32_t w = lidx[e];
                old[i] = __hip_atomic_fetch_add(jobs[w >> kJobShift].stage + (w & kIdxMask), v, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            }
        }
#pragma unroll
        for (int i = 0; i < kBLogK / 2; ++i) {
            const uint32_t src = (uint32_t)(h + i) * (64 / kBLogK) + lane / kBLogK;
            const uint32_t e = (lane % kBLogK) * kBLogStride + src;
            const uint32_t v = lval[e];
            if (v != 0u && (!HOLD || v < kLogHeld)) {
                if (old[i] > 0xFFFFFFFFu - v) {
                    // the word wrapped: its lost 2^32 quanta go to the voxel's int64 word
                    const uint32_t w = lidx[e];
                    const Job &J = jobs[w >> kJobShift];
                    __hip_atomic_fetch_add((unsigned long long *)(J.fluence + stage_voxel(J, w & kIdxMask)),
                                           1ull << (32 + kDepositShift), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                lval[e] = 0u;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (HOLD) {
        log_keep_run<kBLogStride, kBLogK, kBLogHold>(lval, lane, head, count, held);
    } else {
        head = 0u;
        count = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename R>
__device__ __forceinline__ void account_job(unsigned long long *acc, const Photon<R> &p, int32_t ev, int32_t nz)
{
    if (ev == EV_ESC_R || ev == EV_ESC_T) {
        atomicAdd(&acc[ev == EV_ESC_R ? MC_S_R : MC_S_T], (unsigned long long)p.w);
        atomicAdd(&acc[MC_S_ESC_W], (unsigned long long)p.w);
        atomicAdd(&acc[MC_S_ESC_N], 1ull);
        if (p.l_void > (double)nz) {
            atomicAdd(&acc[MC_S_ESC_W_GTL], (unsigned long long)p.w);
            atomicAdd(&acc[MC_S_ESC_N_GTL], 1ull);
        }
        const unsigned long long vp = __double2ull_rn((double)p.w * p.l_void);
        atomicAdd(&acc[MC_S_ESC_W_VOID_PATH], vp & 0xFFFFFFFFull);
        if (vp >> 32) atomicAdd(&acc[MC_S_ESC_W_VOID_PATH_HI], vp >> 32);
    } else if (ev == EV_LOST) {
        atomicAdd(&acc[MC_S_LOST], (unsigned long long)p.w);
    } else if (ev == EV_GATED) {
        atomicAdd(&acc[MC_S_GATED], (unsigned long long)p.w);
    }
    if (p.absorbed) atomicAdd(&acc[MC_S_A], (unsigned long long)p.absorbed);
    if (p.rr) atomicAdd(&acc[MC_S_RR], (unsigned long long)p.rr);
    atomicAdd(&acc[MC_S_STEPS], (unsigned long long)p.steps);
    atomicAdd(&acc[MC_S_INTERACTIONS], (unsigned long long)p.k);
    atomicAdd(&acc[MC_S_LAUNCHED], 1ull);
}

// Same queue discipline as the plain walk: a wavefront-private range of queue
// positions refilled by one atomic, idle lanes refilled together, interactions
// run together once `defer` lanes wait at one (or no lane can advance), exit
// once the queue is exhausted and no lane is alive.
// LOGGED: deposits go through the log into each job's staging tally.  GENERAL:
// some job uses the paper's boundary model (each job's own flags select its
// physics).  esc: per-job escape-path histograms (Sec. 3.5 (c)), or NULL.
template <int BLOCK, typename R, bool LOGGED, bool GENERAL>
__global__ __launch_bounds__(BLOCK) void k_walk_batch(const Job *__restrict__ jobs, int32_t n_jobs,
                                                      unsigned long long *__restrict__ queue, int32_t chunk,
                                                      int32_t refill, int32_t defer,
                                                      const BatchEsc *__restrict__ esc)
{
    constexpr int kWaves = BLOCK / 64;
    constexpr bool kFP32 = std::is_same<R, float>::value;
    __shared__ Job s_jobs[MC_MAX_BATCH_JOBS];
    __shared__ unsigned long long acc[MC_MAX_BATCH_JOBS][MC_NSCALARS];
    __shared__ uint32_t s_lidx[LOGGED ? kWaves * kBLogK * kBLogStride : 1];
    __shared__ uint32_t s_lval[LOGGED ? kWaves * kBLogK * kBLogStride : 1];
    const uint32_t lane = __lane_id();
    uint32_t *lidx = s_lidx + (threadIdx.x >> 6) * (LOGGED ? kBLogK * kBLogStride : 0);
    uint32_t *lval = s_lval + (threadIdx.x >> 6) * (LOGGED ? kBLogK * kBLogStride : 0);
    if (LOGGED)
        for (int i = 0; i < kBLogK; ++i) lval[i * kBLogStride + lane] = 0u;
    {
        const uint64_t *src = (const uint64_t *)jobs;
        uint64_t *dst = (uint64_t *)s_jobs;
        const int32_t words = n_jobs * (int32_t)(sizeof(Job) / 8);
        for (int32_t i = threadIdx.x; i < words; i += BLOCK) dst[i] = src[i];
        unsigned long long *a = &acc[0][0];
        for (int32_t i = threadIdx.x; i < n_jobs * MC_NSCALARS; i += BLOCK) a[i] = 0ull;
    }
    __syncthreads();

    const uint64_t total = s_jobs[n_jobs - 1].queue_begin + s_jobs[n_jobs - 1].n_photons;
    typename std::conditional<LOGGED, BatchLoggedSink, BatchTallySink>::type sink;
    if constexpr (LOGGED) {
        sink.lidx = lidx;
        sink.lval = lval;
        sink.lane = lane;
        sink.head = 0u;
        sink.count = 0u;
    }
    Photon<R> p;
    int32_t job = 0;
    bool alive = false;
    bool waiting = false;   // alive, at an interaction point, interaction not yet run
    uint64_t q_next = 0, q_end = 0;
    bool exhausted = false;

    auto retire = [&](int32_t ev, int32_t nz) {
        account_job(acc[job], p, ev, nz);
        if (esc != nullptr && (ev == EV_ESC_R || ev == EV_ESC_T)) {
            const BatchEsc &e = esc[job];
            if (e.w != nullptr) {
                const size_t b = (size_t)(blockIdx.x % kEscReplicas) * kEscMaxBins +
                                 (size_t)escape_path_bin(p.l_void, e.width, e.nbins);
                __hip_atomic_fetch_add(e.rw + b, (unsigned long long)p.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(e.rn + b, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
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
                        const uint64_t q = q_next + rank;
                        int32_t lo = 0, hi = n_jobs - 1;  // last job whose range starts at or before q
                        while (lo < hi) {
                            const int32_t mid = (lo + hi + 1) >> 1;
                            if (s_jobs[mid].queue_begin <= q) lo = mid;
                            else hi = mid - 1;
                        }
                        job = lo;
                        const Job &J = s_jobs[job];
                        launch<GENERAL>(p, J, (uint32_t)(J.photon_begin + (q - J.queue_begin)));
                        alive = true;
                    }
                    q_next += (uint64_t)nidle < avail ? (uint64_t)nidle : avail;
                }
            }
            if (exhausted && q_next >= q_end && !__any(alive)) break;
        }
        if constexpr (LOGGED) sink.tag = (uint32_t)job << kJobShift;
        if (alive && !waiting) {
            const Job &J = s_jobs[job];
            const int32_t ev = advance<GENERAL>(p, J, sink);
            if (ev == EV_AT_INTERACTION) {
                waiting = true;
            } else {
                const int32_t fin = finish(p, J, sink, ev);
                if (is_terminal(fin)) retire(fin, J.nz);
            }
        }
        const uint64_t wait_mask = __ballot(waiting);
        if (wait_mask != 0ull &&
            (__popcll(wait_mask) >= defer || __ballot(alive && !waiting) == 0ull)) {
            if (waiting) {
                const Job &J = s_jobs[job];
                const int32_t fin = finish(p, J, sink, interact(p, J, sink));
                waiting = false;
                if (is_terminal(fin)) retire(fin, J.nz);
            }
        }
        // a lane logs at most one deposit per iteration, so issue the log once some
        // lane has filled it
        if constexpr (LOGGED) {
            if (__ballot(sink.count >= (uint32_t)kBLogK) != 0ull)
                flush_batch_log<kFP32>(lidx, lval, s_jobs, lane,
                                       alive ? (stage_word(s_jobs[job], p) | sink.tag) >> 4 : kBNoLine, sink.head,
                                       sink.count);
        }
    }
    if constexpr (LOGGED) flush_batch_log<kFP32>(lidx, lval, s_jobs, lane, kBNoLine, sink.head, sink.count);
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n_jobs * MC_NSCALARS; i += BLOCK) {
        const unsigned long long v = acc[i / MC_NSCALARS][i % MC_NSCALARS];
        if (v) atomicAdd((unsigned long long *)&s_jobs[i / MC_NSCALARS].scalars[i % MC_NSCALARS], v);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t jobs_off, esc_off, bricks_off[MC_MAX_BATCH_JOBS], bins_off[MC_MAX_BATCH_JOBS],
        stage_off[MC_MAX_BATCH_JOBS], esc_rep_off[MC_MAX_BATCH_JOBS], total;
    bool logged;   // every job's staging tally fits the log's 26-bit indices
    bool planes[MC_MAX_BATCH_JOBS];   // the job's staging tally may take the plane layout
};

Layout layout_of(const mc_job *jobs, int32_t n)
{
    Layout L;
    size_t off = kHeaderBytes;
    L.jobs_off = off;
    off += align_up(sizeof(Job) * MC_MAX_BATCH_JOBS);
    L.esc_off = off;
    off += align_up(sizeof(BatchEsc) * MC_MAX_BATCH_JOBS);
    L.logged = true;
    for (int32_t i = 0; i < n; ++i) L.logged = L.logged && dims_of(&jobs[i].vol).line_words <= kBatchLogWords;
    for (int32_t i = 0; i < n; ++i) {
        const Dims d = dims_of(&jobs[i].vol);
        L.planes[i] = d.planes && d.stage_words <= kBatchLogWords;
        L.bricks_off[i] = off;
        off += align_up(d.nbricks * sizeof(uint64_t));
        L.bins_off[i] = off;
        off += align_up((size_t)jobs[i].vol.nz * kBinW * sizeof(uint64_t));
        L.stage_off[i] = off;
        if (L.logged) off += align_up((L.planes[i] ? d.stage_words : d.line_words) * sizeof(uint32_t));
        L.esc_rep_off[i] = off;
        off += align_up(kEscReplicaWords * sizeof(uint64_t));
    }
    L.total = off;
    return L;
}

// A validated batch: device job descriptors in queue (longest-first) order.
struct Prepared {
    std::vector<Job> table;       // queue order
    std::vector<int32_t> order;   // table index -> caller's job index
    Layout L;
    uint64_t total_photons = 0;
    bool general = false;         // some job uses the paper boundary model
    bool planes[MC_MAX_BATCH_JOBS] = {};   // caller's job index -> staged in the plane layout
};

// MC_LINE_STAGING or MC_FP64 in flags keeps every job's staging tally in the line layout.
int prepare(const mc_job *jobs, int32_t n, char *ws, size_t ws_bytes, int flags, Prepared *P)
{
    if (!jobs || n < 1 || n > MC_MAX_BATCH_JOBS)
        return fail(MC_EINVAL, "a batch holds 1 to %d jobs (got %d)", MC_MAX_BATCH_JOBS, n);
    if (!ws) return fail(MC_EINVAL, "workspace is NULL");
    char msg[512];
    for (int32_t i = 0; i < n; ++i) {
        int rc = check_volume(&jobs[i].vol);
        if (rc) {
            snprintf(msg, sizeof msg, "%s", mc_last_error());
            return fail(rc, "job %d: %s", i, msg);
        }
    }
    P->L = layout_of(jobs, n);
    if (ws_bytes < P->L.total) return fail(MC_ENOSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, P->L.total);
    P->order.resize(n);
    for (int32_t i = 0; i < n; ++i) P->order[i] = i;
    // longest first; ties keep the caller's order
    std::stable_sort(P->order.begin(), P->order.end(), [&](int32_t a, int32_t b) {
        const double ca = (double)jobs[a].n_photons * jobs[a].vol.nz, cb = (double)jobs[b].n_photons * jobs[b].vol.nz;
        return ca > cb;
    });
    P->table.resize(n);
    uint64_t q = 0;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t i = P->order[t];
        const mc_job &jb = jobs[i];
        Job &J = P->table[t];
        int rc = make_job(&jb.vol, &jb.opt, jb.photon_begin, jb.n_photons, jb.seed, jb.stream_id, &J);
        if (rc) {
            snprintf(msg, sizeof msg, "%s", mc_last_error());
            return fail(rc, "job %d: %s", i, msg);
        }
        if (!jb.fluence || !jb.scalars) return fail(MC_EINVAL, "job %d: fluence and scalars must be non-NULL", i);
        if (J.max_steps > (1u << 26)) return fail(MC_EINVAL, "job %d: batch jobs allow max_steps <= 2^26", i);
        J.bricks = (const uint64_t *)(ws + P->L.bricks_off[i]);
        J.fluence = jb.fluence;
        J.stage = P->L.logged ? (uint32_t *)(ws + P->L.stage_off[i]) : nullptr;
        J.stage_planes = P->L.logged && P->L.planes[i] && !(flags & (MC_LINE_STAGING | MC_FP64));
        P->planes[i] = J.stage_planes != 0;
        J.scalars = jb.scalars;
        J.queue_begin = q;
        q += jb.n_photons;
        P->general = P->general || J.paper;
    }
    P->total_photons = q;
    return MC_OK;
}

template <typename R, bool LOGGED, bool GENERAL>
void enqueue_batch_walk(int block, int blocks, const Job *table, int32_t n, unsigned long long *queue,
                        const mc_tune &t, const BatchEsc *esc, hipStream_t s)
{
    switch (block) {
    case 64:
        hipLaunchKernelGGL((k_walk_batch<64, R, LOGGED, GENERAL>), dim3(blocks), dim3(64), 0, s, table, n, queue, t.chunk,
                           t.refill, t.defer, esc);
        break;
    case 128:
        hipLaunchKernelGGL((k_walk_batch<128, R, LOGGED, GENERAL>), dim3(blocks), dim3(128), 0, s, table, n, queue, t.chunk,
                           t.refill, t.defer, esc);
        break;
    case 256:
        hipLaunchKernelGGL((k_walk_batch<256, R, LOGGED, GENERAL>), dim3(blocks), dim3(256), 0, s, table, n, queue, t.chunk,
                           t.refill, t.defer, esc);
        break;
    default:
        hipLaunchKernelGGL((k_walk_batch<512, R, LOGGED, GENERAL>), dim3(blocks), dim3(512), 0, s, table, n, queue, t.chunk,
                           t.refill, t.defer, esc);
        break;
    }
}

int enqueue_table(const Prepared &P, char *ws, hipStream_t s)
{
    Job *dst = (Job *)(ws + P.L.jobs_off);
    const int32_t n = (int32_t)P.table.size();
    for (int32_t i = 0; i < n; i += 8) {
        JobPack pack;
        memset(&pack, 0, sizeof pack);
        const int32_t c = std::min(8, n - i);
        for (int32_t k = 0; k < c; ++k) pack.j[k] = P.table[i + k];
        hipLaunchKernelGGL(k_write_jobs, dim3(1), dim3(256), 0, s, pack, dst + i, c);
        HIP_TRY(hipGetLastError());
    }
    return MC_OK;
}

// The walk alone (table written, tallies zeroed and masks packed beforehand);
// with_esc: the histogram table in the workspace is written and in use.
int enqueue_walk_only(const Prepared &P, char *ws, const mc_tune &t, int flags, hipStream_t s, bool with_esc = false)
{
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    if ((rc = fill((int64_t *)ws, kHeaderBytes / 8, s))) return rc;
    const int blocks = std::max(1, di.cus * t.waves_per_cu / (t.block / 64));
    const Job *table = (const Job *)(ws + P.L.jobs_off);
    const BatchEsc *esc = with_esc ? (const BatchEsc *)(ws + P.L.esc_off) : nullptr;
    unsigned long long *queue = (unsigned long long *)ws;
    const int32_t n = (int32_t)P.table.size();
    const bool f64 = (flags & MC_FP64) != 0;
    if (P.general) {
        if (P.L.logged) {
            if (f64) enqueue_batch_walk<double, true, true>(t.block, blocks, table, n, queue, t, esc, s);
            else enqueue_batch_walk<float, true, true>(t.block, blocks, table, n, queue, t, esc, s);
        } else {
            if (f64) enqueue_batch_walk<double, false, true>(t.block, blocks, table, n, queue, t, esc, s);
            else enqueue_batch_walk<float, false, true>(t.block, blocks, table, n, queue, t, esc, s);
        }
    } else {
        if (P.L.logged) {
            if (f64) enqueue_batch_walk<double, true, false>(t.block, blocks, table, n, queue, t, esc, s);
            else enqueue_batch_walk<float, true, false>(t.block, blocks, table, n, queue, t, esc, s);
        } else {
            if (f64) enqueue_batch_walk<double, false, false>(t.block, blocks, table, n, queue, t, esc, s);
            else enqueue_batch_walk<float, false, false>(t.block, blocks, table, n, queue, t, esc, s);
        }
    }
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

// The histogram table in queue order, from the caller's per-job bins (validated).
int enqueue_esc_table(const Prepared &P, const mc_escape_bins *bins, char *ws, hipStream_t s)
{
    BatchEsc *dst = (BatchEsc *)(ws + P.L.esc_off);
    const int32_t n = (int32_t)P.table.size();
    for (int32_t i = 0; i < n; i += 16) {
        EscPack pack;
        memset(&pack, 0, sizeof pack);
        const int32_t c = std::min(16, n - i);
        for (int32_t k = 0; k < c; ++k) {
            const int32_t job = P.order[i + k];
            const mc_escape_bins &b = bins[job];
            if (!b.hist_w) continue;
            unsigned long long *rep = (unsigned long long *)(ws + P.L.esc_rep_off[job]);
            pack.e[k].w = (unsigned long long *)b.hist_w;
            pack.e[k].n = (unsigned long long *)b.hist_n;
            pack.e[k].rw = rep;
            pack.e[k].rn = rep + (size_t)kEscReplicas * kEscMaxBins;
            pack.e[k].width = b.bin_width;
            pack.e[k].nbins = b.nbins;
        }
        hipLaunchKernelGGL(k_write_esc, dim3(1), dim3(256), 0, s, pack, dst + i, c);
        HIP_TRY(hipGetLastError());
    }
    return MC_OK;
}

// The whole batched step: table, zeroed tallies, packed masks, one walk, reductions.
// bins: per-job escape-path histograms (caller's job order, validated), or NULL.
int enqueue_batch(const mc_job *jobs, const Prepared &P, char *ws, const mc_tune &t, int flags, hipStream_t s,
                  const mc_escape_bins *bins = nullptr)
{
    int rc = enqueue_table(P, ws, s);
    if (rc) return rc;
    const int32_t n = (int32_t)P.table.size();
    if (bins) {
        if ((rc = enqueue_esc_table(P, bins, ws, s))) return rc;
        for (int32_t i = 0; i < n; ++i) {
            if (!bins[i].hist_w) continue;
            if ((rc = fill((int64_t *)(ws + P.L.esc_rep_off[i]), kEscReplicaWords, s))) return rc;
            if (jobs[i].accumulate) continue;
            if ((rc = fill(bins[i].hist_w, (uint64_t)bins[i].nbins, s))) return rc;
            if ((rc = fill(bins[i].hist_n, (uint64_t)bins[i].nbins, s))) return rc;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        const mc_job &jb = jobs[i];
        const Dims d = dims_of(&jb.vol);
        if (!jb.accumulate) {
            if ((rc = fill(jb.fluence, d.nvox, s))) return rc;
            if ((rc = fill(jb.scalars, MC_NSCALARS, s))) return rc;
        }
        // the staging words as int64 pairs: a line is 16 words, so the count is even
        if (P.L.logged &&
            (rc = fill((int64_t *)(ws + P.L.stage_off[i]), (P.planes[i] ? d.stage_words : d.line_words) / 2, s)))
            return rc;
        if ((rc = pack(&jb.vol, (uint64_t *)(ws + P.L.bricks_off[i]), s))) return rc;
    }
    const bool timed = (flags & MC_TIMED) != 0;
    if (timed && (rc = time_begin(s))) return rc;
    if ((rc = enqueue_walk_only(P, ws, t, flags, s, bins != nullptr))) return rc;
    if (timed && (rc = time_end(s))) return rc;
    if (bins) {
        hipLaunchKernelGGL(k_esc_fold, dim3(n), dim3(256), 0, s, (const BatchEsc *)(ws + P.L.esc_off));
        HIP_TRY(hipGetLastError());
    }
    if (P.L.logged) {
        for (int32_t i = 0; i < n; ++i) {
            const mc_job &jb = jobs[i];
            if ((rc = unstage((const uint32_t *)(ws + P.L.stage_off[i]), jb.fluence, &jb.vol, P.planes[i], s)))
                return rc;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        const mc_job &jb = jobs[i];
        if (!jb.summary) continue;
        if ((rc = enqueue_reduce(&jb.vol, jb.fluence, jb.scalars, jb.summary, jb.depth,
                                 (unsigned long long *)(ws + P.L.bins_off[i]), s)))
            return rc;
    }
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate descent over waves per CU, block size, chunk, refill
// threshold and interaction deferral, each trial a timed walk over a scaled-down copy of the
// batch (every job keeps at least one photon).  Results never depend on the
// launch shape, so tuning only changes speed.
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;

std::string cache_path()
{
    const char *env = getenv("PHOTONMC_TUNE_CACHE");
    if (env && *env) return env;
    const char *home = getenv("HOME");
    if (!home || !*home) return "";
    std::string dir = std::string(home) + "/.cache";
    mkdir(dir.c_str(), 0755);
    return dir + "/photonmc_tune.txt";
}

bool cache_get(const std::string &key, mc_tune *t)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    const std::string path = cache_path();
    if (path.empty()) return false;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[400];
        mc_tune r;
        if (sscanf(line, "%399s %d %d %d %d %d", k, &r.block, &r.waves_per_cu, &r.chunk, &r.refill, &r.defer) == 6 &&
            key == k &&
            check_tune(r) == MC_OK) {
            *t = r;  // the last entry for a key wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_put(const std::string &key, const mc_tune &t)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), t.block, t.waves_per_cu, t.chunk, t.refill, t.defer);
    fclose(f);
}

std::string shape_key(const char *kind, const Prepared &P, int flags)
{
    // a failed query only weakens the cache key (unknown arch / 0 CUs)
    int dev = 0;
    hipDeviceProp_t prop;
    memset(&prop, 0, sizeof prop);
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        memset(&prop, 0, sizeof prop);
        snprintf(prop.gcnArchName, sizeof prop.gcnArchName, "unknown");
    }
    uint64_t vox = 0;
    for (const Job &J : P.table) vox += (uint64_t)J.nx * J.ny * J.nz;
    char buf[400];
    snprintf(buf, sizeof buf, "%s|%s|cu%d|%s%s|jobs%zu|vox2^%d|ph2^%d", kind, prop.gcnArchName,
             prop.multiProcessorCount, (flags & MC_FP64) ? "f64" : "f32", P.general ? "|paper" : "", P.table.size(),
             (int)log2((double)vox + 1.0),
             (int)log2((double)P.total_photons + 1.0));
    for (char *c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    return buf;
}

int time_trial(const std::function<int(const mc_tune &)> &enqueue, const mc_tune &t, hipStream_t s, float *ms)
{
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    int rc = MC_OK;
    if (hipEventRecord(a, s) != hipSuccess) rc = fail(MC_EHIP, "event record failed");
    if (!rc) rc = enqueue(t);
    if (!rc && hipEventRecord(b, s) != hipSuccess) rc = fail(MC_EHIP, "event record failed");
    if (!rc && hipEventSynchronize(b) != hipSuccess) rc = fail(MC_EHIP, "event sync failed");
    if (!rc && hipEventElapsedTime(ms, a, b) != hipSuccess) rc = fail(MC_EHIP, "elapsed time failed");
    if (hipEventDestroy(a) != hipSuccess && !rc) rc = fail(MC_EHIP, "event destroy failed");
    if (hipEventDestroy(b) != hipSuccess && !rc) rc = fail(MC_EHIP, "event destroy failed");
    return rc;
}

// Coordinate descent from the default shape.  A trial's time varies by about 1 %
// between launches, so a candidate replaces the best only when it is faster by
// more than kTuneMargin, and the final choice must beat the default again in two
// more alternating trials, else the default stays.
constexpr float kTuneMargin = 0.01f;

int tune_descent(const std::function<int(const mc_tune &)> &enqueue, hipStream_t s, mc_tune *best_out)
{
    mc_tune best, dflt;
    mc_tune_default(&dflt);
    best = dflt;
    float best_ms = 0.0f;
    int rc = time_trial(enqueue, best, s, &best_ms);  // also warms the code objects
    if (rc) return rc;
    if ((rc = time_trial(enqueue, best, s, &best_ms))) return rc;
    auto consider = [&](mc_tune cand) -> int {
        if (check_tune(cand) != MC_OK) return MC_OK;
        float ms = 0.0f;
        int r = time_trial(enqueue, cand, s, &ms);
        if (r) return r;
        if (ms < best_ms * (1.0f - kTuneMargin)) {
            best_ms = ms;
            best = cand;
        }
        return MC_OK;
    };
    for (int w : {4, 8, 12, 16, 24, 32}) {
        mc_tune c = best;
        c.waves_per_cu = w;
        if ((rc = consider(c))) return rc;
    }
    for (int b : {64, 128, 256, 512}) {
        mc_tune c = best;
        c.block = b;
        if ((rc = consider(c))) return rc;
    }
    for (int ch : {32, 128, 256, 1024, 4096}) {
        mc_tune c = best;
        c.chunk = ch;
        if ((rc = consider(c))) return rc;
    }
    for (int rf : {1, 8, 16, 32, 48}) {
        mc_tune c = best;
        c.refill = rf;
        if ((rc = consider(c))) return rc;
    }
    for (int df : {1, 8, 16, 24, 32, 40, 48}) {
        mc_tune c = best;
        c.defer = df;
        if ((rc = consider(c))) return rc;
    }
    bool keep = memcmp(&best, &dflt, sizeof best) != 0;
    for (int k = 0; k < 2 && keep; ++k) {
        float ms_d = 0.0f, ms_b = 0.0f;
        if ((rc = time_trial(enqueue, dflt, s, &ms_d))) return rc;
        if ((rc = time_trial(enqueue, best, s, &ms_b))) return rc;
        keep = ms_b < ms_d;
    }
    clear_error();
    *best_out = keep ? best : dflt;
    return MC_OK;
}

// Scaled-down copy of a prepared batch for tuning trials.
Prepared scaled(const Prepared &P, double fraction)
{
    Prepared S = P;
    uint64_t q = 0;
    for (Job &J : S.table) {
        J.n_photons = std::max<uint64_t>(1, (uint64_t)((double)J.n_photons * fraction));
        J.queue_begin = q;
        q += J.n_photons;
    }
    S.total_photons = q;
    return S;
}

int autotune_prepared(const mc_job *jobs, const Prepared &P, char *ws, int flags, hipStream_t s, mc_tune *out)
{
    for (size_t i = 0; i < P.table.size(); ++i)
        if (jobs[i].accumulate)
            return fail(MC_EINVAL, "job %zu accumulates: tuning trials would add to its tallies; pass a tune", i);
    // trials of about 2^25 photons in total: long enough that the tail of a launch and
    // the spread between trials do not decide the shape
    const double fraction = std::min(1.0, 33554432.0 / (double)P.total_photons);
    Prepared S = scaled(P, fraction);
    int rc = enqueue_table(S, ws, s);
    if (rc) return rc;
    for (size_t i = 0; i < S.table.size(); ++i)
        if ((rc = pack(&jobs[S.order[i]].vol, (uint64_t *)(ws + S.L.bricks_off[S.order[i]]), s))) return rc;
    auto trial = [&](const mc_tune &t) { return enqueue_walk_only(S, ws, t, flags & MC_FP64, s); };
    return tune_descent(trial, s, out);
}

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t mc_batch_workspace_bytes(const mc_job *jobs, int32_t n_jobs)
{
    if (!jobs || n_jobs < 1 || n_jobs > MC_MAX_BATCH_JOBS) return 0;
    for (int32_t i = 0; i < n_jobs; ++i)
        if (check_volume(&jobs[i].vol)) return 0;
    return layout_of(jobs, n_jobs).total;
}

int mc_autotune_batch(const mc_job *jobs, int32_t n_jobs, int flags, void *workspace, size_t workspace_bytes,
                      mc_tune *out, void *hip_stream)
{
    clear_error();
    if (!out) return fail(MC_EINVAL, "out is NULL");
    Prepared P;
    int rc = prepare(jobs, n_jobs, (char *)workspace, workspace_bytes, flags, &P);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const std::string key = shape_key("batch", P, flags);
    if ((rc = autotune_prepared(jobs, P, (char *)workspace, flags, s, out))) return rc;
    cache_put(key, *out);
    return MC_OK;
}

}  // extern "C"

namespace {

int run_batch(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune, void *workspace,
              size_t workspace_bytes, void *hip_stream, const mc_escape_bins *bins)
{
    Prepared P;
    int rc = prepare(jobs, n_jobs, (char *)workspace, workspace_bytes, flags, &P);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    mc_tune t;
    if (tune) {
        t = resolve_tune(tune);
    } else {
        const std::string key = shape_key("batch", P, flags);
        if (!cache_get(key, &t)) {
            if ((rc = autotune_prepared(jobs, P, (char *)workspace, flags, s, &t))) return rc;
            cache_put(key, t);
        }
    }
    if ((rc = check_tune(t))) return rc;
    return enqueue_batch(jobs, P, (char *)workspace, t, flags, s, bins);
}

}  // namespace

extern "C" {

int mc_run_batch(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune, void *workspace,
                 size_t workspace_bytes, void *hip_stream)
{
    clear_error();
    return run_batch(jobs, n_jobs, flags, tune, workspace, workspace_bytes, hip_stream, nullptr);
}

int mc_run_batch_escape_histogram(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune,
                                  const mc_escape_bins *bins, void *workspace, size_t workspace_bytes,
                                  void *hip_stream)
{
    clear_error();
    if (!bins) return fail(MC_EINVAL, "bins is NULL");
    if (jobs && n_jobs >= 1 && n_jobs <= MC_MAX_BATCH_JOBS) {
        for (int32_t i = 0; i < n_jobs; ++i) {
            const mc_escape_bins &b = bins[i];
            if (b.reserved != 0) return fail(MC_EINVAL, "job %d: bins.reserved must be 0", i);
            if (!b.hist_w) continue;
            if (!b.hist_n) return fail(MC_EINVAL, "job %d: hist_n is NULL while hist_w is not", i);
            if (b.nbins < 1 || b.nbins > kEscMaxBins)
                return fail(MC_EINVAL, "job %d: nbins must be in [1, %d]", i, kEscMaxBins);
            if (!(b.bin_width > 0.0) || !isfinite(b.bin_width))
                return fail(MC_EINVAL, "job %d: bin_width must be finite and > 0", i);
        }
    }
    return run_batch(jobs, n_jobs, flags, tune, workspace, workspace_bytes, hip_stream, bins);
}

int mc_batch_graph_create(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune, void *workspace,
                          size_t workspace_bytes, mc_graph *out)
{
    clear_error();
    if (!out) return fail(MC_EINVAL, "out is NULL");
    if (flags & MC_TIMED) return fail(MC_EINVAL, "MC_TIMED cannot be captured; time the graph launch instead");
    Prepared P;
    int rc = prepare(jobs, n_jobs, (char *)workspace, workspace_bytes, flags, &P);
    if (rc) return rc;
    const mc_tune t = resolve_tune(tune);
    if ((rc = check_tune(t))) return rc;
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    GraphHandle *h = new GraphHandle;
    rc = MC_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(MC_EHIP, "hipStreamBeginCapture failed");
    } else {
        const int erc = enqueue_batch(jobs, P, (char *)workspace, t, flags, cs);
        const hipError_t e = hipStreamEndCapture(cs, &h->graph);
        if (erc) rc = erc;
        else if (e != hipSuccess) rc = fail(MC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        else if (hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess)
            rc = fail(MC_EHIP, "hipGraphInstantiate failed");
    }
    if (hipStreamDestroy(cs) != hipSuccess && !rc) rc = fail(MC_EHIP, "hipStreamDestroy failed");
    if (rc) {
        // already failing: the first error is the one reported
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        delete h;
        return rc;
    }
    *out = (mc_graph)h;
    return MC_OK;
}

int mc_graph_launch(mc_graph g, void *hip_stream)
{
    clear_error();
    if (!g) return fail(MC_EINVAL, "graph is NULL");
    HIP_TRY(hipGraphLaunch(((GraphHandle *)g)->exec, (hipStream_t)hip_stream));
    return MC_OK;
}

int mc_graph_destroy(mc_graph g)
{
    clear_error();
    if (!g) return MC_OK;
    GraphHandle *h = (GraphHandle *)g;
    int rc = MC_OK;
    if (h->exec && hipGraphExecDestroy(h->exec) != hipSuccess) rc = fail(MC_EHIP, "hipGraphExecDestroy failed");
    if (h->graph && hipGraphDestroy(h->graph) != hipSuccess && !rc) rc = fail(MC_EHIP, "hipGraphDestroy failed");
    delete h;
    return rc;
}

}  // extern "C"
