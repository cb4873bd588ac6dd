/*
 * photonmc.h -- C ABI of the MI355X (gfx950) photon-migration library.
 *
 * The library simulates weighted photon packets through a voxelised binary
 * solid/pore mask, as in "Three-dimensional photon transport in spinodal
 * photocatalytic aerogels":
 *   - Sec. 2.5 (Three-dimensional Monte Carlo simulation) and App. B: pores are
 *     transparent (mu_a = mu_s = 0), solid voxels absorb and scatter; a planar
 *     collimated source covers the z = 0 face and points along +z; the axial
 *     faces are open; weighted photons with implicit capture and Russian
 *     roulette; absorptance from an absorbed-energy counter and reflectance /
 *     transmittance from escape records (Eq. RTA, Eq. closure);
 *   - Sec. 2.6 (Fluence estimators): solid-weighted <Phi>_3D (Eq. Phi_MC3D),
 *     volume average <Phi>_1D (Eq. Phi_MC1D), pore average and the contrast
 *     ratio r (Eq. r_def), and the identity of Eq. dilution;
 *   - Sec. 3.5 (c): in-pore path length of every escaping photon.
 * Two boundary models (mc_optics.boundary):
 *   - MC_BOUNDARY_PLAIN: lateral faces periodic, refractive index 1 everywhere,
 *     photons start on the z = 0 face and escape when they cross z = 0 or z = Nz;
 *   - MC_BOUNDARY_PAPER (Sec. 2.5 "Source and boundary conditions", "Photon
 *     budget, time gate and statistics", App. B): a one-voxel air pad (index 1,
 *     untallied) on each axial face, photons start on the pad's outer face and
 *     escape through the outer face of either pad; lateral faces specular
 *     mirrors or periodic; the solid has index n_solid and every face between
 *     media of different index reflects (total internal reflection, or with the
 *     unpolarised Fresnel reflectance against one uniform of the photon's own
 *     Fresnel stream) or refracts (Snell's law); optional time gate (Eq. tend)
 *     on the optical path sum(n d), the cut weight going to its own channel.
 *
 * Conventions
 *   - All buffers named "device" are HIP device pointers owned by the caller.
 *     The library never allocates device memory; scratch space is passed in
 *     as a workspace whose size a *_workspace_bytes() query returns.
 *   - Every entry point is asynchronous on the given HIP stream (NULL: the
 *     legacy default stream) and returns after enqueueing, except where noted.
 *     Pointers must stay valid until the enqueued work has finished.
 *   - Status: 0 ok, > 0 warning, < 0 error.  No entry point throws.  On error
 *     nothing is enqueued and mc_last_error() (thread-local) explains why.
 *   - Weights are integers in units of 2^-31 of a launched photon (Q31).  The
 *     fluence tally is int64, in Q31 weight x voxel length; each track segment's
 *     deposit w d is rounded to a whole multiple of MC_DEPOSIT_QUANTUM Q31 units
 *     (2^-23 of a launched photon x voxel) before it is added.  Integer atomics
 *     make every result independent of scheduling: a run is bitwise
 *     reproducible and a run split into photon ranges sums to the whole.
 *   - Coordinates: voxel (x, y, z), x fastest; z = 0 is the illuminated face.
 */
#ifndef PHOTONMC_H
#define PHOTONMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_ABI_VERSION 4

/* status codes */
#define MC_OK 0
#define MC_WARN_LOST 1      /* some weight hit the step / path cap (scalar MC_S_LOST > 0) */
#define MC_EINVAL (-1)      /* invalid argument */
#define MC_EOVERFLOW (-2)   /* a voxel tally reached 2^62 (reported by the reduction) */
#define MC_EHIP (-3)        /* a HIP runtime call failed */
#define MC_ENOSPACE (-4)    /* workspace too small */

/* flags */
#define MC_ACCUMULATE 1     /* add to the tallies instead of zeroing them first */
#define MC_TIMED 2          /* time the walk kernel with HIP events on the run's stream (mc_walk_elapsed_ms) */
#define MC_FP64 4           /* geometry and scattering in FP64 instead of FP32 (reference transport); its
                               walk is bound by the VALU, so it stages deposits in the line layout, whose
                               index costs less VALU work than the plane layout's */
#define MC_DIRECT_DEPOSIT 8 /* one atomic per voxel visit into the caller's tally, not the line-coalesced
                               deposit log into a staging tally of uint32 words (the log is used when that
                               staging tally has <= 2^32 words) */
#define MC_LINE_STAGING 16  /* stage the logged deposits in one table of 2 x 2 x 4-voxel lines even where
                               the three tables of 4 x 4-voxel planes fit (the workspace sizes allow for
                               the planes; the two layouts give identical tallies); for mc_run_batch,
                               in every job.  Implied by MC_FP64. */

#define MC_DEPOSIT_QUANTUM 256 /* Q31 units: every tally value is a multiple of it */
#define MC_GRAD_FIXED_BITS 20  /* mc_grad's score bins count units of 2^-20 Q31 weight x voxel */

/* Scalar tally channels: int64 words in a caller-owned device array of
 * MC_NSCALARS entries.  Weight channels are Q31.  For every run
 * R + T + A + RR + LOST + GATED == LAUNCHED * 2^31 exactly.  One set of tallies holds
 * fewer than 2^32 photons (so LAUNCHED * 2^31 < 2^63). */
enum {
    MC_S_R = 0,            /* weight escaped through z = 0 (reflectance) */
    MC_S_T,                /* weight escaped through z = Nz (transmittance) */
    MC_S_A,                /* weight absorbed at interaction sites */
    MC_S_RR,               /* net weight removed by Russian roulette (signed) */
    MC_S_LOST,             /* weight of photons stopped by the step / path cap */
    MC_S_ESC_W,            /* escaped weight, both faces */
    MC_S_ESC_W_GTL,        /* escaped weight whose in-pore path exceeds Nz */
    MC_S_ESC_W_VOID_PATH,  /* sum of escaped weight x in-pore path (Q31 x voxel), low 32 bits of each
                              photon's term (summed as unsigned) */
    MC_S_ESC_N,            /* escaped photons */
    MC_S_ESC_N_GTL,        /* escaped photons whose in-pore path exceeds Nz */
    MC_S_STEPS,            /* photon-steps (one segment inside one voxel) */
    MC_S_INTERACTIONS,     /* interaction events */
    MC_S_LAUNCHED,         /* photons launched */
    MC_S_ESC_W_VOID_PATH_HI, /* high parts (term >> 32) of the same sum: total = HI * 2^32 + LO */
    MC_S_GATED,            /* weight of photons stopped by the time gate (paper boundary model) */
    MC_NSCALARS = 16
};

/* Reduced results (doubles, caller-owned device array of MC_NSUMMARY). Phi is
 * reported as Phi/S0, dimensionless (Eq. Phi_norm without the physical units). */
enum {
    MC_Q_PHI3D = 0,        /* <Phi>_3D, solid-weighted (Eq. Phi_MC3D) */
    MC_Q_PHI1D,            /* <Phi>_1D, volume average (Eq. Phi_MC1D) */
    MC_Q_PHI_PORE,         /* pore average */
    MC_Q_R_CONTRAST,       /* r = <Phi>_pore / <Phi>_3D (Eq. r_def) */
    MC_Q_POROSITY,         /* achieved porosity N_pore / N_vox */
    MC_Q_RATIO,            /* <Phi>_3D / <Phi>_1D */
    MC_Q_IDENTITY_RHS,     /* 1 / [phi r + (1 - phi)] (Eq. dilution) */
    MC_Q_R,                /* reflectance R */
    MC_Q_T,                /* transmittance T */
    MC_Q_A,                /* absorptance A */
    MC_Q_RR,               /* roulette balance */
    MC_Q_LOST,             /* lost fraction */
    MC_Q_CLOSURE_EXACT,    /* 1.0 if R+T+A+RR+LOST == LAUNCHED * 2^31 exactly, else 0.0 */
    MC_Q_FRONT_BACK,       /* Phi(z = 0) / Phi(z = Nz - 1) */
    MC_Q_L_OPT,            /* <Phi>_1D * Nz, in voxels */
    MC_Q_ESC_FRAC,         /* escaped weight / launched weight */
    MC_Q_PW_VOID_GTL,      /* escaped-weight fraction with in-pore path > Nz */
    MC_Q_PN_VOID_GTL,      /* escaped-photon fraction with in-pore path > Nz */
    MC_Q_MEAN_VOID_PATH,   /* escaped-weight-weighted mean in-pore path, voxels */
    MC_Q_STEPS_PER_PHOTON,
    MC_Q_INTERACTIONS_PER_PHOTON,
    MC_Q_STATUS,           /* MC_EOVERFLOW if a voxel tally reached 2^62, else MC_WARN_LOST if weight
                              was stopped by the step / path cap (scalar MC_S_LOST > 0), else 0 */
    MC_Q_N_SOLID,          /* solid voxel count */
    MC_Q_LAUNCHED,         /* photons the tallies hold */
    MC_Q_GATED,            /* weight fraction stopped by the time gate */
    MC_NSUMMARY = 32
};

/* The volume: a binary mask in device memory, uint8[nz][ny][nx], 1 = pore,
 * 0 = solid (the paper's m; s = 1 - m).  Limits: 1 <= nx, ny, nz <= 65535,
 * nx*ny*nz < 2^34. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;
    const uint8_t *mask;
} mc_volume;

/* boundary models (mc_optics.boundary) */
#define MC_BOUNDARY_PLAIN 0
#define MC_BOUNDARY_PAPER 1
#define MC_LATERAL_PERIODIC 0
#define MC_LATERAL_MIRROR 1

/* Optical properties of the solid phase (per voxel length); pores are 0.  A
 * zero-initialised tail (boundary .. gate) selects the plain model. */
typedef struct {
    float mu_s;            /* scattering coefficient, >= 0 */
    float mu_a;            /* absorption coefficient, >= 0 */
    float g;               /* Henyey-Greenstein anisotropy, |g| < 1 */
    float w_roulette;      /* roulette threshold as a fraction of a launched photon (1e-4) */
    uint32_t roulette_m;   /* roulette survival 1/m, m >= 2 (10); w_roulette * m <= 1 */
    float path_cap;        /* stop a photon after this total path, voxels (<= 0: none) */
    int32_t source;        /* 0: collimated normal incidence (the paper's); 1: Lambertian (test) */
    uint32_t max_steps;    /* stop a photon after this many steps (0: 2^24) */
    int32_t boundary;      /* MC_BOUNDARY_PLAIN (0) or MC_BOUNDARY_PAPER (1) */
    int32_t lateral;       /* paper model: MC_LATERAL_PERIODIC (0) or MC_LATERAL_MIRROR (1); plain: 0 */
    float n_solid;         /* paper model: refractive index of the solid, >= 1 (0: 1); plain: 0 or 1 */
    int32_t reserved;      /* 0 */
    double gate;           /* paper model: optical path limit c t_end in voxels, sum of n x segment length
                              over the walk, pads included (<= 0 or +inf: none); plain: <= 0 or +inf */
} mc_optics;

/* Launch shape of the persistent walk.  Any value <= 0 selects the default.
 * Results do not depend on it. */
typedef struct {
    int32_t block;         /* threads per workgroup: 64, 128, 256, 512 */
    int32_t waves_per_cu;  /* resident waves per compute unit the grid is sized for */
    int32_t chunk;         /* photons a wavefront takes from the queue at once */
    int32_t refill;        /* refill a wavefront once this many of its lanes are idle */
    int32_t defer;         /* run a wavefront's interactions once this many of its lanes wait at an
                              interaction point (or no lane can advance); 1: at once; at most 64.
                              Default 4 for the plain walk; 8 for the gradient walk, the paper's
                              boundary model and the FP64 transport, whose walks are bound by their
                              VALU rather than by their deposit requests */
} mc_tune;

/* Fill *t with the library defaults (those of the plain walk). */
void mc_tune_default(mc_tune *t);

/* Workspace (device bytes) an mc_run on this volume needs. */
size_t mc_run_workspace_bytes(const mc_volume *vol);

/*
 * Run photons [photon_begin, photon_begin + n_photons) of the stream
 * (seed, stream_id) through the volume (Sec. 2.5, App. B).
 *   fluence  device int64[nz][ny][nx], Q31 weight x voxel (track-length estimator)
 *   scalars  device int64[MC_NSCALARS]
 *   workspace, workspace_bytes  device scratch of >= mc_run_workspace_bytes(vol)
 *   tune     launch shape, or NULL for defaults
 * Tallies are zeroed first unless flags has MC_ACCUMULATE.  Photon p draws
 * Philox4x32-10 block k (k = 0 launch, k >= 1 its k-th interaction) with
 * key (seed lo, seed hi) and counter (k, p, stream_id, 0); photon ids must be
 * < 2^32.  Errors: MC_EINVAL for a bad volume or optics, n_photons == 0,
 * photon_begin + n_photons > 2^32; MC_ENOSPACE; MC_EHIP.
 */
int mc_run(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons,
           uint64_t seed, uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars,
           void *workspace, size_t workspace_bytes, const mc_tune *tune, void *hip_stream);

/*
 * mc_run for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same walk
 * and the same tallies, bit for bit, with no workspace argument.  The queue counter
 * and the packed mask live in a fixed scratch array of 16 MiB + 256 bytes that the
 * library holds on every GPU it runs on until the process ends; the call
 * allocates nothing.  The fluence is deposited with one atomic per voxel visit straight into
 * the caller's tally (MC_DIRECT_DEPOSIT), since the line-coalesced log would need a
 * scratch tally as large as the fluence, so it runs slower than mc_run.
 *   limit   the mask's 4x4x4 bricks, ceil(nx/4) ceil(ny/4) ceil(nz/4), at most
 *           mc_run_noalloc_max_bricks() = 2^21 (e.g. 512 x 512 x 512 voxels);
 *           larger volumes: MC_ENOSPACE, nothing enqueued
 *   flags   MC_ACCUMULATE, MC_FP64 (MC_DIRECT_DEPOSIT is implied); MC_TIMED is
 *           refused (its events would be allocated)
 * Every call on one GPU uses that GPU's one scratch array (each call clears the
 * queue counter and repacks the mask first), so calls that overlap on one GPU, on
 * any streams, race and give wrong results: serialise them.  Other arguments and
 * errors as mc_run.
 */
int mc_run_noalloc(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons,
                   uint64_t seed, uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars,
                   const mc_tune *tune, void *hip_stream);
/* The largest brick count mc_run_noalloc accepts. */
size_t mc_run_noalloc_max_bricks(void);

/*
 * mc_run that also histograms the in-pore path of every escaping photon (fate R
 * or T) of the run (Sec. 3.5 (c)), with the bins of mc_escape_path_histogram
 * (analytics.h): bin b holds b * bin_width <= path < (b + 1) * bin_width, the
 * last bin everything beyond.  The tallies are those of mc_run with the same
 * arguments, bit for bit.
 *   bin_width   finite, > 0 (voxels);  nbins  1 .. 512
 *   hist_w, hist_n  device int64[nbins]: escaped Q31 weight and photon count per
 *                   bin; zeroed first unless flags has MC_ACCUMULATE
 * Errors as mc_run, and MC_EINVAL for NULL histograms or a bad bin_width / nbins.
 */
int mc_run_escape_histogram(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin,
                            uint64_t n_photons, uint64_t seed, uint32_t stream_id, int flags, int64_t *fluence,
                            int64_t *scalars, void *workspace, size_t workspace_bytes, const mc_tune *tune,
                            double bin_width, int32_t nbins, int64_t *hist_w, int64_t *hist_n, void *hip_stream);

/* Duration in milliseconds of the walk kernel of the last mc_run on this thread
 * that carried MC_TIMED (two HIP events recorded on its stream around the walk
 * launch only).  Waits for that walk to finish.  MC_EINVAL if none. */
int mc_walk_elapsed_ms(float *ms);

/* Workspace (device bytes) an mc_reduce on this volume needs. */
size_t mc_reduce_workspace_bytes(const mc_volume *vol);

/*
 * Reduce the tallies of a run (Sec. 2.6): per-depth, per-phase integer sums of
 * the fluence (exact, two 64-bit halves), then the estimators in FP64.
 *   summary  device double[MC_NSUMMARY]
 *   depth    device double[3][nz]: Phi/S0 lateral mean, solid mean, pore mean per
 *            depth (NaN where a layer has no voxel of that phase); may be NULL
 * The photon count is the tallies' own MC_S_LAUNCHED.  The outcome of the run is
 * known only on the device, so the reduction writes it to summary[MC_Q_STATUS]:
 * MC_EOVERFLOW when a voxel tally reached 2^62 (the estimators are then invalid),
 * otherwise MC_WARN_LOST when weight was stopped by the step or path cap (the
 * estimators then miss that weight's further path), otherwise MC_OK.  The return
 * value covers only the arguments and the launch.
 */
int mc_reduce(const mc_volume *vol, const int64_t *fluence, const int64_t *scalars, double *summary,
              double *depth, void *workspace, size_t workspace_bytes, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Gradients by the likelihood-ratio (perturbation Monte Carlo) method; not in
 * the paper.  The sampled path density of a photon with k interactions is
 * mu_s^k exp(-mu_t l_solid) prod_i p_HG(cos_i; g) (implicit capture supplies
 * the ratio to the sampling density), so the scores are S_mus = k/mu_s - l_solid,
 * S_mua = -l_solid, S_g = sum_i d ln p_HG(cos_i; g)/dg.  A track segment of
 * length d adds w (S d - [solid] d^2/2) to the mu_s and mu_a bins and w S_g d to
 * the g bin of its (phase, depth).
 * ------------------------------------------------------------------------- */
#define MC_GRAD_MAX_NZ 2048

/* Workspace (device bytes) an mc_grad on this volume needs. */
size_t mc_grad_workspace_bytes(const mc_volume *vol);

/*
 * The walk of mc_run (same photons, same tallies) that also accumulates the
 * score bins, then optionally the reduction and the Jacobian:
 *   grad_bins  device int64[3][2][nz][2]: (mu_s, mu_a, g) x (solid, pore) x depth x
 *              (hi, lo); value = hi * 2^32 + lo (lo summed as unsigned) in units of
 *              2^-MC_GRAD_FIXED_BITS Q31 weight x voxel
 *   jac        device double[3][2 + nz] or NULL: d<Phi>_3D, d<Phi>_1D, dPhi(z)/S0
 *              with respect to mu_s, mu_a, g (per voxel units)
 *   summary, depth  as mc_reduce, or NULL
 * nz <= MC_GRAD_MAX_NZ.  flags: MC_ACCUMULATE (also accumulates grad_bins),
 * MC_FP64, MC_TIMED.  Errors as mc_run.
 */
int mc_grad(const mc_volume *vol, const mc_optics *opt, uint64_t photon_begin, uint64_t n_photons, uint64_t seed,
            uint32_t stream_id, int flags, int64_t *fluence, int64_t *scalars, int64_t *grad_bins, double *jac,
            double *summary, double *depth, void *workspace, size_t workspace_bytes, const mc_tune *tune,
            void *hip_stream);

/* One trace record per step of a traced photon: the state at the start of the
 * step (exact values of the transport precision, widened to double) and how the
 * step ended. */
typedef struct {
    double fx, fy, fz;     /* offsets inside the voxel, [0, 1] */
    double ux, uy, uz;     /* direction */
    double d;              /* segment length */
    double s_rem;          /* remaining free path (solid length) at the start of the step */
    uint32_t w;            /* weight, Q31 */
    uint32_t k;            /* interactions so far */
    int32_t ix, iy, iz;
    int32_t event;         /* 0/1/2 face crossing on x/y/z, 3 scatter, 4 escape z<0, 5 escape z>Nz,
                              6 weight absorbed to zero, 7 roulette kill, 8 cap, 9 time gate,
                              10/11/12 reflection (mirror, Fresnel or total internal) on an x/y/z face;
                              -1 unused.  In the paper model iz = -1 and iz = Nz are the air pads. */
} mc_trace_rec;

/* Per-photon outcome of a traced photon. */
typedef struct {
    int64_t R, T, A, RR, lost;     /* this photon's share of each weight channel */
    uint32_t w_final, fate;        /* final weight and final event */
    uint32_t steps, interactions;
    double path_void, path_solid;
} mc_photon_rec;

/*
 * Trace photons one per lane through the same walk as mc_run (no tallies); flags
 * may hold MC_FP64:
 *   photon_ids  device uint64[n] (each < 2^32)
 *   recs        device mc_trace_rec[n][max_steps] (all records written; unused ones event -1)
 *   outcome     device mc_photon_rec[n], or NULL
 */
int mc_trace(const mc_volume *vol, const mc_optics *opt, const uint64_t *photon_ids, int32_t n,
             int32_t max_steps, uint64_t seed, uint32_t stream_id, int flags, mc_trace_rec *recs,
             mc_photon_rec *outcome, void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * Roofline probe (measurement only, not part of the walk): n_ops random scatter
 * operations over a device table of n_entries int64 (a multiple of 64), spread
 * over waves_per_cu resident waves per compute unit (0: 16; else a multiple of 4 in
 * [4, 32]).  mode 0: device-scope 64-bit atomic add (what the walk's fluence
 * deposit does); 1: workgroup-scope 64-bit atomic add; 2: plain 64-bit store;
 * 3: device-scope 32-bit atomic add; 4: 64-bit atomic add with the 64 lanes of a
 * wavefront on 64 consecutive entries; 5, 6, 7: 64-bit atomic add with groups of
 * 16, 8, 4 lanes on 16, 8, 4 consecutive entries of a random aligned block (128, 64,
 * 32 bytes); 8: mode 0 returning the old value; 9: mode 3 returning the old value;
 * 10, 11: 32-bit atomic add with groups of 16 lanes on the 16 words of a random
 * 64-byte line, without / with the old value returned; 12: mode 6 returning the old
 * value.  The table's contents afterwards are meaningless.
 */
int mc_probe_scatter(int64_t *table, uint64_t n_entries, uint64_t n_ops, int mode, int waves_per_cu,
                     void *hip_stream);

/*
 * Accuracy of the FP32 transport's hardware functions on the inputs the walk
 * gives them (the interaction step of Sec. 2.5 / App. B: the azimuth's sine and
 * cosine, the square roots of the deflection, the free path's logarithm), over all
 * 2^24 uniforms, against FP64.  max_err: device double[4], written with the
 * largest absolute sine error, absolute cosine error, relative logarithm error and
 * relative square-root error.  Asynchronous on the stream.
 */
int mc_probe_math(double *max_err, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batched runs: many volumes of uneven size, porosity and optics in one
 * persistent launch.  Every job draws its own Philox streams (seed, stream_id),
 * so job k of a batch is bitwise identical to mc_run of that job alone, for any
 * launch shape.
 * ------------------------------------------------------------------------- */
#define MC_MAX_BATCH_JOBS 64

typedef struct {
    mc_volume vol;
    mc_optics opt;
    uint64_t photon_begin, n_photons, seed;
    uint32_t stream_id;
    int32_t accumulate;    /* nonzero: add to this job's tallies instead of zeroing them */
    int64_t *fluence;      /* device int64[nz][ny][nx] */
    int64_t *scalars;      /* device int64[MC_NSCALARS] */
    double *summary;       /* device double[MC_NSUMMARY]: also reduce this job; NULL: no reduction */
    double *depth;         /* device double[3][nz] or NULL (as mc_reduce) */
} mc_job;

/* Workspace (device bytes) a batch of these jobs needs; 0 for an invalid batch. */
size_t mc_batch_workspace_bytes(const mc_job *jobs, int32_t n_jobs);

/*
 * Run 1..MC_MAX_BATCH_JOBS jobs: zero (unless accumulate) and pack every job,
 * one persistent walk over all photons of all jobs (queued longest job first),
 * then the reduction of every job that has a summary buffer.  flags: MC_FP64,
 * MC_TIMED (times the walk kernel).  tune NULL: the launch shape cached for
 * this batch's shape class (device, precision, job count, total voxels and
 * photons, each rounded to a power of two) is used, or found by
 * mc_autotune_batch first and cached (file $PHOTONMC_TUNE_CACHE, else
 * ~/.cache/photonmc_tune.txt; MC_EINVAL if a job accumulates then, as the
 * tuning trials write to the tallies).  Errors: MC_EINVAL (a job is invalid;
 * the message names it), MC_ENOSPACE, MC_EHIP.
 */
int mc_run_batch(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune, void *workspace,
                 size_t workspace_bytes, void *hip_stream);

/* The in-pore path histogram of one batch job's escaping photons (Sec. 3.5 (c)),
 * with the bins of mc_run_escape_histogram. */
typedef struct {
    double bin_width;      /* finite, > 0 (voxels) */
    int32_t nbins;         /* 1 .. 512; the last bin takes every longer path */
    int32_t reserved;      /* must be 0 */
    int64_t *hist_w;       /* device int64[nbins]: escaped Q31 weight per bin; NULL: no histogram for this job */
    int64_t *hist_n;       /* device int64[nbins]: escaped photons per bin */
} mc_escape_bins;

/*
 * mc_run_batch that also histograms, per job, the in-pore path of every escaping
 * photon (fate R or T) over the whole run (Sec. 3.5 (c)), so that no per-photon
 * record is needed.  bins: host array [n_jobs], entry i for jobs[i]; a job whose
 * hist_w is NULL keeps no histogram.  A job's histogram is zeroed first unless
 * the job accumulates.  Job k's tallies are those of mc_run_batch and its
 * histogram equals, bin for bin, mc_run_escape_histogram of job k alone, for any
 * launch shape.  The walk adds each escaping photon into one of 16 copies of
 * its job's bins in the workspace (a workgroup's copy by its index, so that the
 * few bins most photons fall in are not one hot address), and a kernel after
 * the walk adds the copies into hist_w / hist_n.  tune NULL: as mc_run_batch.  Errors as
 * mc_run_batch, and MC_EINVAL for a NULL bins array, a histogram entry with
 * hist_n NULL, a nonzero reserved field or a bad bin_width / nbins (the message
 * names the job).
 */
int mc_run_batch_escape_histogram(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune,
                                  const mc_escape_bins *bins, void *workspace, size_t workspace_bytes,
                                  void *hip_stream);

/*
 * Find a fast launch shape for this batch by timed trials on a scaled-down copy
 * of it (about 2^25 photons per trial; coordinate descent from the default shape
 * over waves per CU, block size, chunk, refill and defer, a candidate taken only
 * when over 1 % faster, and the result kept only if it beats the default again in
 * two more trials), store it in the tune cache and return it.
 * Synchronises the stream.  Overwrites the jobs' tallies with meaningless
 * values (MC_EINVAL if a job accumulates).
 */
int mc_autotune_batch(const mc_job *jobs, int32_t n_jobs, int flags, void *workspace, size_t workspace_bytes,
                      mc_tune *out, void *hip_stream);

/* A captured HIP graph of a whole batched step (what mc_run_batch enqueues, with
 * a fixed tune), replayable with one launch.  All buffers named by the jobs and
 * the workspace are baked in and must outlive the graph. */
typedef struct mc_graph_s *mc_graph;
int mc_batch_graph_create(const mc_job *jobs, int32_t n_jobs, int flags, const mc_tune *tune, void *workspace,
                          size_t workspace_bytes, mc_graph *out);
int mc_graph_launch(mc_graph graph, void *hip_stream);
int mc_graph_destroy(mc_graph graph);

/* ---------------------------------------------------------------------------
 * The paper's reference model and comparison metrics.  The host functions take
 * host pointers and return at once; mc_rms_w is a kernel on the stream.
 * ------------------------------------------------------------------------- */

/*
 * Time gate of Eq. tend (Sec. 2.5, "Photon budget, time gate and statistics"):
 *   t_end = max(5 n_eff / (mu_a c), 6 L^2 / D_phys),
 *   D_phys = (c / n_eff) / (3 (mu_a,eff + mu_s,eff')),
 * with the effective-medium scaling of Eq. EMA_scaling, mu_eff = (1 - porosity) mu,
 * and the reduced scattering coefficient mu_s' = mu_s (1 - g).
 *   mu_s, mu_a  solid (shell) coefficients per unit length, >= 0;  |g| < 1
 *   porosity    in [0, 1];  thickness L > 0 in the same length unit
 *   n_eff >= 1; c > 0, the speed of light in length per time unit
 *   t_end       host double: the gate in time units, +inf when mu_a = 0 (the first
 *               term is then unbounded).  With c = 1 and voxel units it is c t_end
 *               in voxels, the optical path limit that mc_optics.gate takes.
 * Host function.  Errors: MC_EINVAL for a NULL pointer or an argument out of range.
 */
int mc_time_gate(double mu_s, double mu_a, double g, double porosity, double thickness, double n_eff, double c,
                 double *t_end);

/*
 * Collimated-source diffusion approximation (Sec. 2.4: Eq. DA_total with the
 * particular solution of Eq. DA_diff_eq, the constants of Eq. Cpm for the
 * extrapolated boundaries Phi_diff(-z_b) = Phi_diff(L + z_b) = 0, Eq. Phi_diff, and
 * Eq. Lopt_DA) on a slab of nz voxel layers, in voxel units with S0 = 1:
 *   effective coefficients (Eq. EMA_scaling)  mu_a,eff = (1 - porosity) mu_a,
 *   mu_s,eff' = (1 - porosity) mu_s (1 - g);  D = 1 / (3 (mu_a,eff + mu_s,eff')),
 *   kappa = sqrt(mu_a,eff / D), mu_t = mu_a,eff + mu_s,eff', z_b = (2/3) / mu_s,eff',
 *   L = nz.
 *   profile  host double[nz] or NULL: the mean of Phi_DA / S0 over depth [z, z + 1)
 *            of layer z (each term of Eq. DA_total integrated in closed form), the
 *            quantity a depth profile of mc_reduce estimates
 *   l_opt    host double or NULL: L_opt of Eq. Lopt_DA in voxels, the integral over
 *            [0, L], i.e. the sum of the profile (so <Phi>_DA / S0 = l_opt / nz)
 * Host function.  Errors: MC_EINVAL for nz < 1, |g| >= 1, porosity outside [0, 1),
 * effective coefficients that are not finite and > 0, kappa = mu_t (the particular
 * solution is degenerate), kappa (L + 2 z_b) > 700 (sinh overflows), or both
 * outputs NULL.
 */
int mc_da_profile(double mu_s, double mu_a, double g, double porosity, int32_t nz, double *profile, double *l_opt);

/*
 * Discrepancy between a depth profile p and a reference q (Sec. 2.7, Eq. RMSw, and
 * the two variants of App. B / Table S1), over the depths where q is finite and
 * positive and p is finite:
 *   out[0]  RMS_w = [sum_z q (p - q)^2 / q^2 / sum_z q]^(1/2)      (Eq. RMSw)
 *   out[1]  unweighted: [mean_z ((p - q) / q)^2]^(1/2)
 *   out[2]  log-ratio: [mean_z ln(p / q)^2]^(1/2), over those depths where p > 0 too
 * profile, reference  device double[n], n >= 1;  out  device double[3] (NaN where
 * no depth qualifies).  Fractions, not percent.  Sums in a fixed order: the result
 * is reproducible.  Errors: MC_EINVAL (NULL argument, n < 1), MC_EHIP.
 */
int mc_rms_w(const double *profile, const double *reference, int32_t n, double *out, void *hip_stream);

/* Text for a status code. */
const char *mc_strerror(int status);
/* Message of the last error on this thread ("" if none). */
const char *mc_last_error(void);
/* Library ABI version (MC_ABI_VERSION). */
int mc_abi_version(void);
/* sizeof one of the ABI structs by name ("mc_volume", "mc_optics", "mc_tune",
 * "mc_trace_rec", "mc_photon_rec", "mc_job", "mc_escape_bins"), 0 for an unknown name; lets a
 * binding check its layouts. */
size_t mc_sizeof(const char *type_name);

#ifdef __cplusplus
}
#endif
#endif /* PHOTONMC_H */
