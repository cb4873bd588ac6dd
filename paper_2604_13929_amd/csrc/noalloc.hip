// noalloc.hip -- mc_run_noalloc (photonmc.h): mc_run for callers that cannot
// allocate device memory.  The run's queue counter and packed mask live in a
// fixed file-scope device array instead of a caller's workspace; the fluence is
// deposited with one atomic per voxel visit straight into the caller's tally, so
// no staging tally is needed.  Every GPU the library runs on holds its own copy of
// the array until the process ends; host code reaches a device's copy only through
// the address hipGetSymbolAddress returns for it on that device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

using namespace pmc;
using namespace pmc::host;

namespace {

constexpr size_t kScratchBytes = kHeaderBytes + ((size_t)16 << 20);   // the queue counter and 2^21 mask bricks
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's copy of `scratch`, looked up once per device with
// that device current.
int scratch_address(void **out)
{
    static std::mutex mu;
    static void *cache[64];
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MC_EHIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!cache[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(MC_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        cache[dev] = ptr;
    }
    *out = cache[dev];
    return MC_OK;
}

}  // namespace

extern "C" {

size_t mc_run_noalloc_max_bricks(void) { return (kScratchBytes - kHeaderBytes) / sizeof(uint64_t); }

int mc_run_noalloc(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons,
                   uint64_t seed, uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars,
                   const mc_tune *tune, void *hip_stream)
{
    clear_error();
    Job J;
    int rc = make_job(vol, opt, photon_begin, n_photons, seed, stream_id, &J);
    if (rc) return rc;
    if (!fluence || !scalars) return fail(MC_EINVAL, "fluence and scalars must be non-NULL");
    if (flags & ~(MC_ACCUMULATE | MC_FP64 | MC_DIRECT_DEPOSIT))
        return fail(MC_EINVAL, "mc_run_noalloc takes MC_ACCUMULATE, MC_FP64 and MC_DIRECT_DEPOSIT only (no MC_TIMED)");
    const Dims d = dims_of(vol);
    if (d.nbricks > mc_run_noalloc_max_bricks())
        return fail(MC_ENOSPACE, "volume needs %llu mask bricks of 4x4x4 voxels; the fixed scratch holds %zu",
                    (unsigned long long)d.nbricks, mc_run_noalloc_max_bricks());
    const mc_tune t = resolve_tune(tune, (J.paper || (flags & MC_FP64)) ? kDeferVALUBound : 0);
    if ((rc = check_tune(t))) return rc;
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    J.fluence = fluence;
    J.scalars = scalars;
    // the queue counter and the packed mask sit where mc_run's workspace holds them;
    // MC_DIRECT_DEPOSIT leaves the staging tally out, so they are all the walk uses
    return run_walk(vol, J, flags | MC_DIRECT_DEPOSIT, t, (char *)ws, nullptr, (hipStream_t)hip_stream);
}

}  // extern "C"
