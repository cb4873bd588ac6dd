/*
 * spinodal.h -- C ABI of the MI355X (gfx950) Cahn-Hilliard spinodal mask
 * generator, part of libphotonmc.so.
 *
 * It integrates the Cahn-Hilliard equation of "Three-dimensional photon
 * transport in spinodal photocatalytic aerogels" (Sec. 2.2, Eq. CH) with the
 * double well f(phi) = phi^2 (1 - phi)^2 and unit mobility by the semi-implicit
 * Fourier spectral step of Eq. CH_spectral,
 *     phihat^{n+1}_k = (phihat^n_k - dt k^2 [f'(phi^n)]^_k) / (1 + dt kappa k^4),
 * in double precision on a periodic voxel grid, measures the radial power
 * spectral density whose peak App. A uses as its stopping criterion, and
 * binarises the final field by rank (App. A, Binarisation).
 *
 * Conventions (as in photonmc.h): every buffer is caller-owned device memory;
 * calls are asynchronous on the given HIP stream unless noted; status 0 ok,
 * < 0 error (MC_EINVAL, MC_EHIP, MC_ENOSPACE), message in mc_last_error().
 *
 * Layouts
 *   real field   double[nz][ny][nx], x fastest;
 *   spectrum     complex double (re, im interleaved) [nz][ny][nx/2 + 1]: the
 *                unnormalised forward transform along x (real to complex), y and
 *                z, the layout of numpy.fft.rfftn on a C-ordered array;
 *   wavenumbers  k = 2 pi m / N per axis, m the signed frequency index.
 * Limits: nx even, 2 <= nx <= 1024, 1 <= ny, nz <= 1024, every extent a product
 * of powers of 2 and 3; nx*ny*nz < 2^31.
 */
#ifndef SPINODAL_H
#define SPINODAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;      /* 0 */
    double kappa;          /* gradient coefficient kappa_CH, voxel units (Eq. kappa_cal), > 0 */
    double dt;             /* time step, dimensionless CH units (App. A), > 0 */
} mc_ch_grid;

/* The grid constants for a target dominant size d_target (voxels, > 0):
 * kappa_CH = (1/2) (d_target / (8 pi))^2 (Eq. kappa_cal) and the time step of App. A,
 * dt = min(0.5 / (kappa_CH k_max^4), 1) with k_max = pi per voxel.  Writes g->kappa
 * and g->dt of a host struct (the extents are left as they are).  Host function.
 * MC_EINVAL for a NULL grid or a d_target that is not finite and > 0. */
int mc_ch_grid_from_target(double d_target, mc_ch_grid *g);

/* App. A's dominant structural size from a radial PSD (mc_ch_psd, or mc_mask_psd of
 * analytics.h): the peak shell s_peak, the first s >= 1 holding the largest psd[s]
 * (shell 0 is the mean, excluded), and size = n_max / (2 s_peak) voxels, half the
 * peak wavelength (one pore and one strut per period).
 *   psd         device double[n_bins], n_bins >= 2;  n_max = max(nx, ny, nz) >= 1
 *   peak_shell  device int32 or NULL;  size  device double or NULL (not both NULL)
 * Asynchronous on the stream.  MC_EINVAL, MC_EHIP. */
int mc_psd_peak(const double *psd, int32_t n_bins, int32_t n_max, int32_t *peak_shell, double *size,
                void *hip_stream);

/* Device workspace of the mc_ch_* calls: one spectrum-sized work array plus
 * transform tables and reduction space.  0 when the grid is invalid. */
size_t mc_ch_workspace_bytes(const mc_ch_grid *g);

/* state = forward transform of the real field phi0 (the initial condition; App. A
 * uses 0.5 + N(0, 0.05^2) noise clipped to [0, 1], supplied by the caller). */
int mc_ch_init(const mc_ch_grid *g, const double *phi0, double *state, void *workspace, size_t workspace_bytes,
               void *hip_stream);

/* n_steps steps of Eq. CH_spectral on the spectrum `state` (in place).  flags may
 * hold MC_TIMED: HIP events around the step kernels, read by mc_ch_elapsed_ms(). */
int mc_ch_steps(const mc_ch_grid *g, int32_t n_steps, double *state, void *workspace, size_t workspace_bytes,
                int flags, void *hip_stream);

/* phi = inverse transform of `state` (normalised by 1/(nx ny nz), as numpy.fft.irfftn). */
int mc_ch_field(const mc_ch_grid *g, const double *state, double *phi, void *workspace, size_t workspace_bytes,
                void *hip_stream);

/* Radial power spectral density: psd[s], s = 0 .. max(nx,ny,nz)/2, the sum of
 * |phihat_k|^2 over the modes of the full spectrum with
 * s - 1/2 <= |k| max(nx,ny,nz) / (2 pi) < s + 1/2, the k = 0 mode excluded (each
 * mode of the half spectrum stored with 0 < kx index < nx/2 stands for itself and
 * its conjugate).  Sums are in double; their order of addition is not fixed, so
 * they are reproducible to rounding.  The dominant size of App. A is
 * max(nx,ny,nz) / (2 s_peak). */
int mc_ch_psd(const mc_ch_grid *g, const double *state, double *psd, void *workspace, size_t workspace_bytes,
              void *hip_stream);

/* Milliseconds between the HIP events of the last mc_ch_steps call that carried
 * MC_TIMED (waits for it); < 0 if none. */
double mc_ch_elapsed_ms(void);

/* Rank binarisation (App. A): mask[i] = 1 for the n_pore largest field values,
 * ties going to the lower linear index, 0 elsewhere; exact for any values
 * (-0.0 and +0.0 compare equal; NaN is not allowed).  field and mask are device
 * arrays of n >= 1 elements, 0 <= n_pore <= n, n < 2^40. */
size_t mc_rank_threshold_workspace_bytes(int64_t n);
int mc_rank_threshold(const double *field, int64_t n, int64_t n_pore, uint8_t *mask, void *workspace,
                      size_t workspace_bytes, void *hip_stream);

/*
 * App. A's loop, synchronous on the stream: from phi0, run check_every steps at
 * a time until the dominant size (above) lies in [d_target - sigma/2,
 * d_target + sigma/2] or max_steps steps have run; then write the field to
 * phi_out (may be NULL) and, when mask is not NULL, binarise it with n_pore =
 * round(porosity * N) pore voxels.  Writes the steps taken and the last dominant
 * size (voxels).  Workspace: mc_ch_workspace_bytes + a real field +
 * mc_rank_threshold_workspace_bytes(N), see mc_ch_generate_workspace_bytes.
 */
size_t mc_ch_generate_workspace_bytes(const mc_ch_grid *g);
int mc_ch_generate(const mc_ch_grid *g, const double *phi0, double d_target, double sigma, int32_t check_every,
                   int32_t max_steps, double porosity, double *state, double *phi_out, uint8_t *mask,
                   int32_t *steps_taken, double *last_size, void *workspace, size_t workspace_bytes,
                   void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPINODAL_H */
