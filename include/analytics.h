/*
 * analytics.h -- C ABI of the morphology and fluence analytics of "Three-
 * dimensional photon transport in spinodal photocatalytic aerogels" (Sec. 3.5),
 * part of libphotonmc.so.  Conventions as in photonmc.h: caller-owned device
 * buffers, asynchronous on the given HIP stream, status 0 ok / < 0 error with
 * mc_last_error().  Volumes are mc_volume masks (1 = pore, 0 = solid).
 */
#ifndef ANALYTICS_H
#define ANALYTICS_H

#include <stddef.h>
#include <stdint.h>

#include "photonmc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Sec. 3.5 (a): chord-length histogram along one axis (0 = x, 1 = y, 2 = z; the
 * paper uses the beam axis z).  A chord is a maximal run of voxels of one phase on
 * a line; chords cut by the faces count with their in-volume length.
 *   hist  device int64[2][n_axis + 1]: hist[phase][len], phase 0 solid, 1 pore (written). */
int mc_chord_histogram(const mc_volume *vol, int32_t axis, int64_t *hist, void *hip_stream);

/* Sec. 3.5 (b): depth-normalised phase contrast from mc_reduce's depth[3][nz]
 * (lateral mean, solid mean, pore mean per depth): c_solid(z) = solid / lateral
 * mean and c_pore(z) likewise over z0 <= z < nz, skipping depths whose lateral
 * mean is not positive or that lack the phase.
 *   out  device double[5]: solid mean, solid sample sd, pore mean, pore sample sd,
 *        depths with a positive lateral mean. */
int mc_phase_contrast(const double *depth, int32_t nz, int32_t z0, double *out, void *hip_stream);

/* Sec. 3.5 (c): in-pore path of escaping photons (fate 4 or 5) from per-photon
 * outcome records (mc_trace with max_steps = 0): bin b of width bin_width holds
 * b * bin_width <= path < (b + 1) * bin_width, the last bin everything beyond.
 *   rec         device mc_photon_rec[n]
 *   thresholds  HOST double[nthr], nthr <= 8
 *   hist_w, hist_n   device int64[nbins]: escaped Q31 weight and photon count
 *   above_w, above_n device int64[nthr]: weight and count with path > threshold (may be NULL if nthr = 0)
 * Outputs are written (zeroed first). */
int mc_escape_path_histogram(const mc_photon_rec *rec, int64_t n, double bin_width, int32_t nbins,
                             const double *thresholds, int32_t nthr, int64_t *hist_w, int64_t *hist_n,
                             int64_t *above_w, int64_t *above_n, void *hip_stream);

/* Sec. 3.5, co-localisation: for each slice z0 <= z < nz the k = ceil(frac * nx * ny)
 * voxels of highest fluence (ties to the lower linear index) and how many of them
 * are solid; 0 < frac <= 1, nx * ny < 2^31.
 *   fluence  device int64[nz][ny][nx] (mc_run's tally; any int64 values)
 *   top_count, top_solid  device int64[nz - z0] (written) */
int mc_bright_colocalization(const mc_volume *vol, const int64_t *fluence, int32_t z0, double frac,
                             int64_t *top_count, int64_t *top_solid, void *hip_stream);

/* Local pore size (Sec. 3.5, co-localisation): the exact Euclidean distance from
 * every pore voxel centre to the nearest solid voxel centre inside the volume (no
 * periodic images), 0 in the solid, +inf everywhere if there is no solid voxel.
 * Squared distances are 32-bit integers: needs nx^2 + ny^2 + nz^2 < 2^30 - 1 (an
 * extent up to 32 767 on one axis), MC_EINVAL otherwise.
 *   dist  device double[nz][ny][nx] (written) */
size_t mc_pore_distance_workspace_bytes(const mc_volume *vol);
int mc_pore_distance(const mc_volume *vol, double *dist, void *workspace, size_t workspace_bytes,
                     void *hip_stream);

/* Sec. 3.5, co-localisation: Spearman rank correlation, per slice z0 <= z < nz, between
 * the fluence and the local pore size (the distance of mc_pore_distance) over the
 * pore voxels of that slice.  Ties take the average of their ranks; rho is the
 * Pearson correlation of the two rank vectors, NaN where a slice has fewer than two
 * pore voxels or either rank vector is constant.
 *   fluence      device int64[nz][ny][nx] (mc_run's tally)
 *   rho          device double[nz - z0] (written)
 *   n_pore       device int64[nz - z0]: pore voxels per slice (written)
 * Needs nx * ny * (nz - z0) < 2^31 and the distance transform's extent limit.
 * Unlike the other calls this one synchronises
 * the stream once: the number of pore voxels sizes the sorts, and the largest
 * fluence and squared distance fix their bit ranges.  The workspace query
 * asks the HIP runtime for the current device's sort configuration and returns 0
 * (with mc_last_error) for invalid arguments or when no device answers; the
 * workspace it sizes is for the current device. */
size_t mc_pore_spearman_workspace_bytes(const mc_volume *vol, int32_t z0);
int mc_pore_spearman(const mc_volume *vol, const int64_t *fluence, int32_t z0, double *rho, int64_t *n_pore,
                     void *workspace, size_t workspace_bytes, void *hip_stream);

/* Sec. 3.1, Fig. 2b: radial power spectral density of the binary mask itself
 * (values 0 and 1), with the shells and conventions of mc_ch_psd (spinodal.h):
 * psd[s], s = 0 .. max(nx,ny,nz)/2, sums |m_hat_k|^2 of the unnormalised forward
 * transform over s - 1/2 <= |k| max(nx,ny,nz) / (2 pi) < s + 1/2, the k = 0 mode
 * excluded; the dominant pore-plus-strut size is max(nx,ny,nz) / (2 s_peak).
 * The grid limits are those of the Cahn-Hilliard transforms: nx even, every extent
 * a product of powers of 2 and 3 up to 1024.
 *   psd  device double[max(nx,ny,nz)/2 + 1] (written) */
size_t mc_mask_psd_workspace_bytes(const mc_volume *vol);
int mc_mask_psd(const mc_volume *vol, double *psd, void *workspace, size_t workspace_bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ANALYTICS_H */
