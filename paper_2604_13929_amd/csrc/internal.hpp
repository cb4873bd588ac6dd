// Host-side helpers shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "photonmc.h"
#include "walk.hpp"

struct EscHist;  // the escape-path histogram of a walk (photonmc.hip)

namespace pmc {
namespace host {

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return ::pmc::host::fail(MC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kHeaderBytes = 256;  // queue counter(s) at the start of a run workspace
constexpr int kBinW = 8;              // int64 words per depth bin of the reduction
constexpr int kEscMaxBins = 512;      // escape-path bins; 6 KB of LDS leaves four walk workgroups per CU
// A walk stages its deposits in the plane layout (three tables) where those fit in
// this many bytes, else in the line layout (one table): tripled, the 256^3 tally
// stays within the 256 MiB Infinity Cache, beyond which memory-side atomics slow
// down.
#ifndef MC_PLANE_STAGE_MAX_BYTES
#define MC_PLANE_STAGE_MAX_BYTES (192ull << 20)
#endif
constexpr uint64_t kPlaneStageMaxBytes = MC_PLANE_STAGE_MAX_BYTES;

struct Dims {
    int32_t nxb, nyb, nzb;       // 4x4x4 mask bricks
    uint64_t nbricks, nvox;
    int32_t lnx, lny, lnz;       // staging lines of 2x2x4 voxels (line layout)
    uint64_t line_words;         // uint32 words of the line layout
    bool planes;                 // the single-run walk stages in the plane layout
    uint64_t stage_words;        // uint32 words of the single-run walk's staging tally
    bool logged;                 // the staging tally fits 32-bit indices
};
size_t run_workspace_bytes(const Dims &d);
size_t stage_offset(const Dims &d);
Dims dims_of(const mc_volume *v);
int check_volume(const mc_volume *v);
int make_job(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons, uint64_t seed,
             uint32_t stream_id, Job *J);

struct DeviceInfo {
    int cus = 0;
};
int device_info(DeviceInfo *out);

// The launch shape: the caller's fields where > 0, else the defaults, with defer_default
// (when > 0) in place of the plain walk's default defer.
mc_tune resolve_tune(const mc_tune *t, int32_t defer_default = 0);
// The default defer of a walk: the gradient walk, the paper's boundary model and the FP64
// transport are bound by their VALU and run their interactions in larger groups.
constexpr int32_t kDeferVALUBound = 8;
int check_tune(const mc_tune &t);

// asynchronous building blocks on a stream
int fill(int64_t *p, uint64_t n, hipStream_t s);
int pack(const mc_volume *vol, uint64_t *bricks, hipStream_t s);
int unstage(const uint32_t *stage, int64_t *fluence, const mc_volume *vol, bool planes, hipStream_t s);
// zero (unless accumulating), pack, walk and move the staged tally into the caller's
// fluence, with the queue, packed mask and staging tally in the workspace ws
int run_walk(const mc_volume *vol, Job J, int flags, const mc_tune &t, char *ws, unsigned long long *grad_bins,
             hipStream_t s, const EscHist *esc = nullptr);
int enqueue_reduce(const mc_volume *vol, const int64_t *fluence, const int64_t *scalars, double *summary,
                   double *depth, unsigned long long *bins, hipStream_t s);

// the walk-kernel timer (MC_TIMED)
struct Timing {
    hipEvent_t start = nullptr, stop = nullptr;
    bool armed = false;
};
Timing &timing();
int time_begin(hipStream_t s);
int time_end(hipStream_t s);

}  // namespace host
}  // namespace pmc
