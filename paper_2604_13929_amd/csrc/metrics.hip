// metrics.hip -- the paper's reference model and comparison metrics, declared in
// photonmc.h:
//   mc_time_gate   the diffusion-aware time gate of Eq. tend (host arithmetic)
//   mc_da_profile  the collimated-source diffusion approximation of Sec. 2.4,
//                  averaged over each voxel layer in closed form (host arithmetic)
//   mc_rms_w       Eq. RMSw and its unweighted and log-ratio variants (Sec. 2.7,
//                  App. B, Table S1) between two device depth profiles, in one
//                  workgroup on the stream
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "internal.hpp"

using namespace pmc::host;

namespace {

// cosh(a) - cosh(b) = 2 sinh((a + b)/2) sinh((a - b)/2): no cancellation when a ~ b
double cosh_diff(double a, double b) { return 2.0 * sinh(0.5 * (a + b)) * sinh(0.5 * (a - b)); }

constexpr int kRmsBlock = 256;

// Sums over the depths in a fixed tree order, so the result does not depend on
// scheduling.  s[0] sum ref (p - ref)^2 / ref^2, s[1] sum ref, s[2] sum ((p - ref)/ref)^2
// and s[3] its count, s[4] sum ln(p/ref)^2 and s[5] its count.
__global__ __launch_bounds__(kRmsBlock) void k_rms_w(const double *__restrict__ p, const double *__restrict__ q,
                                                     int32_t n, double *__restrict__ out)
{
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t z = threadIdx.x; z < n; z += kRmsBlock) {
        const double ref = q[z], v = p[z];
        if (!(ref > 0.0) || !isfinite(ref) || !isfinite(v)) continue;
        const double rel = (v - ref) / ref;
        s[0] += ref * rel * rel;
        s[1] += ref;
        s[2] += rel * rel;
        s[3] += 1.0;
        if (v > 0.0) {
            const double l = log(v / ref);
            s[4] += l * l;
            s[5] += 1.0;
        }
    }
    __shared__ double part[6][kRmsBlock];
    for (int c = 0; c < 6; ++c) part[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int h = kRmsBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int c = 0; c < 6; ++c) part[c][threadIdx.x] += part[c][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nan = __builtin_nan("");
        out[0] = part[1][0] > 0.0 ? sqrt(part[0][0] / part[1][0]) : nan;
        out[1] = part[3][0] > 0.0 ? sqrt(part[2][0] / part[3][0]) : nan;
        out[2] = part[5][0] > 0.0 ? sqrt(part[4][0] / part[5][0]) : nan;
    }
}

}  // namespace

extern "C" {

int mc_time_gate(double mu_s, double mu_a, double g, double porosity, double thickness, double n_eff, double c,
                 double *t_end)
{
    clear_error();
    if (!t_end) return fail(MC_EINVAL, "t_end is NULL");
    if (!(mu_s >= 0.0) || !(mu_a >= 0.0) || !isfinite(mu_s) || !isfinite(mu_a))
        return fail(MC_EINVAL, "mu_s and mu_a must be finite and >= 0");
    if (!(fabs(g) < 1.0)) return fail(MC_EINVAL, "|g| must be < 1");
    if (!(porosity >= 0.0 && porosity <= 1.0)) return fail(MC_EINVAL, "porosity must be in [0, 1]");
    if (!(thickness > 0.0) || !isfinite(thickness)) return fail(MC_EINVAL, "thickness must be finite and > 0");
    if (!(n_eff >= 1.0) || !isfinite(n_eff)) return fail(MC_EINVAL, "n_eff must be finite and >= 1");
    if (!(c > 0.0) || !isfinite(c)) return fail(MC_EINVAL, "c must be finite and > 0");
    // Eq. EMA_scaling: the effective coefficients scale with the solid fraction
    const double mu_a_eff = (1.0 - porosity) * mu_a;
    const double mu_s_red_eff = (1.0 - porosity) * mu_s * (1.0 - g);
    // without absorption the first term is unbounded: no gate (+inf)
    const double absorb = mu_a > 0.0 ? 5.0 * n_eff / (mu_a * c) : (double)INFINITY;
    // 6 L^2 / D_phys with D_phys = (c / n_eff) / (3 (mu_a,eff + mu_s,eff'))
    const double diffuse = 6.0 * thickness * thickness * 3.0 * (mu_a_eff + mu_s_red_eff) * n_eff / c;
    *t_end = absorb > diffuse ? absorb : diffuse;
    return MC_OK;
}

int mc_da_profile(double mu_s, double mu_a, double g, double porosity, int32_t nz, double *profile, double *l_opt)
{
    clear_error();
    if (!profile && !l_opt) return fail(MC_EINVAL, "profile and l_opt are both NULL");
    if (nz < 1) return fail(MC_EINVAL, "nz must be >= 1");
    if (!(fabs(g) < 1.0)) return fail(MC_EINVAL, "|g| must be < 1");
    if (!(porosity >= 0.0 && porosity < 1.0)) return fail(MC_EINVAL, "porosity must be in [0, 1)");
    // Eq. EMA_scaling, and the reduced scattering coefficient mu_s' = mu_s (1 - g)
    const double mua = (1.0 - porosity) * mu_a;
    const double musr = (1.0 - porosity) * mu_s * (1.0 - g);
    if (!(mua > 0.0) || !(musr > 0.0) || !isfinite(mua) || !isfinite(musr))
        return fail(MC_EINVAL, "the effective mu_a and mu_s (1 - g) must be finite and > 0");
    const double D = 1.0 / (3.0 * (mua + musr));
    const double kappa = sqrt(mua / D);
    const double mu_t = mua + musr;
    const double z_b = (2.0 / 3.0) / musr;
    const double L = (double)nz, L_e = L + 2.0 * z_b;
    if (fabs(kappa - mu_t) <= 1e-12 * mu_t)
        return fail(MC_EINVAL, "kappa equals mu_t (mu_s' = 2 mu_a): the particular solution is degenerate");
    if (kappa * L_e > 700.0) return fail(MC_EINVAL, "kappa (L + 2 z_b) > 700: sinh overflows");
    // Eq. DA_diff_eq's particular solution A e^{-mu_t z}, Eq. Cpm's constants (S0 = 1)
    const double A = musr / (D * (kappa * kappa - mu_t * mu_t));
    const double sh = sinh(kappa * L_e);
    const double c_plus = -A * exp(-mu_t * (L + z_b)) / sh;
    const double c_minus = -A * exp(mu_t * z_b) / sh;
    // the mean of Eq. DA_total (ballistic + Eq. Phi_diff) over [z, z + 1): each term integrated exactly
    const double decay = -expm1(-mu_t) / mu_t;  // (1 - e^{-mu_t}) / mu_t
    double sum = 0.0;
    for (int32_t iz = 0; iz < nz; ++iz) {
        const double z0 = (double)iz, z1 = z0 + 1.0;
        const double expo = exp(-mu_t * z0) * decay;
        const double up = cosh_diff(kappa * (z1 + z_b), kappa * (z0 + z_b)) / kappa;
        const double down = cosh_diff(kappa * (L + z_b - z0), kappa * (L + z_b - z1)) / kappa;
        const double v = (1.0 + A) * expo + c_plus * up + c_minus * down;
        if (profile) profile[iz] = v;
        sum += v;
    }
    // Eq. Lopt_DA: (1/S0) times the integral over [0, L], the sum of the layer means
    if (l_opt) *l_opt = sum;
    return MC_OK;
}

int mc_rms_w(const double *profile, const double *reference, int32_t n, double *out, void *hip_stream)
{
    clear_error();
    if (!profile || !reference || !out) return fail(MC_EINVAL, "NULL argument");
    if (n < 1) return fail(MC_EINVAL, "n must be >= 1");
    hipLaunchKernelGGL(k_rms_w, dim3(1), dim3(kRmsBlock), 0, (hipStream_t)hip_stream, profile, reference, n, out);
    HIP_TRY(hipGetLastError());
    return MC_OK;
}

}  // extern "C"
