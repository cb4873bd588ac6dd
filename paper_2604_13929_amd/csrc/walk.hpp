// Photon state and one step of the voxel walk, device side (gfx950, wave64).
//
// Physics (paper, Sec. 2.5 and App. B): transparent pores, absorbing and
// scattering solid, planar collimated source on z = 0 along +z, open axial
// faces, weighted photons with implicit capture and Russian roulette.  The
// readings fixed here where the paper is silent: periodic lateral faces,
// index 1 everywhere, track-length fluence per voxel, absorption at
// interaction sites on an integer Q31 weight, HG deflection by inverse CDF,
// the MCML direction update (Wang, Jacques & Zheng 1995), one Philox block per
// event, the face axis taken as the first minimum in x, y, z order, an
// interaction winning a tie against a face, in-voxel offsets clamped to [0,1].
//
// The paper's own boundary model (Sec. 2.5 "Source and boundary conditions",
// App. B) is the GENERAL step: one-voxel air pads (layers iz = -1 and iz = nz,
// index 1, untallied) on the axial faces, specular mirrors or periodic lateral
// faces, a solid of index n_solid with reflection or refraction at every face
// between media of different index (total internal reflection, else the
// unpolarised Fresnel reflectance against a uniform of the photon's Fresnel
// stream: Philox tag 4, block j >> 2, word j & 3 for its j-th decision; Snell's
// law scales the tangential components by n1/n2), and the time gate of
// Eq. tend on the optical path sum(n d).  With n_solid = 1, periodic faces and
// no gate, the general step reproduces the plain step's tallies exactly.
//
// Position is an integer voxel index plus an offset in [0,1] per axis.  The
// geometry and scattering arithmetic is templated on R: float (the default
// transport) or double (a reference transport whose trajectories follow an
// FP64 evaluation of the same steps).  The remaining free path and the path
// sums are FP64 in both, since they accumulate over many segments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "philox.hpp"

namespace pmc {

constexpr float kInf = __builtin_inff();
constexpr uint32_t kW1 = 0x80000000u;  // launched weight, 2^31

// events (same codes as the trace records of the public header)
enum : int32_t {
    EV_FACE_X = 0, EV_FACE_Y = 1, EV_FACE_Z = 2, EV_SCATTER = 3,
    EV_ESC_R = 4, EV_ESC_T = 5, EV_DEAD_ABSORB = 6, EV_DEAD_ROULETTE = 7, EV_LOST = 8, EV_GATED = 9,
    EV_REFLECT_X = 10, EV_REFLECT_Y = 11, EV_REFLECT_Z = 12
};

__host__ __device__ __forceinline__ bool is_terminal(int32_t ev) { return ev >= EV_ESC_R && ev <= EV_GATED; }

// Bin of an escaping photon's in-pore path pv (Sec. 3.5 (c)): b * width <= pv <
// (b + 1) * width, the last bin everything beyond.  The walk's own histogram and
// the binning of traced records both use this one definition.
__device__ __forceinline__ int escape_path_bin(double pv, double width, int nbins)
{
    const double q = floor(pv / width);
    return q >= (double)(nbins - 1) ? nbins - 1 : (q > 0.0 ? (int)q : 0);
}

// Per-job constants.  Everything integer that decides an outcome is computed
// on the host in FP64 (survival factor, roulette threshold and odds).
struct Job {
    const uint64_t *bricks;   // 4x4x4 bit bricks, 1 = pore
    int64_t *fluence;         // [nz][ny][nx]
    uint32_t *stage;          // staging tally of the logged deposits (plane or line layout), or NULL
    int64_t *scalars;         // [MC_NSCALARS]
    int32_t nx, ny, nz;
    int32_t nxb, nyb;         // bricks along x and y
    int32_t lnx, lny;         // staging lines along x and y (line layout)
    int32_t stage_planes;     // 1: the staging tally is in the plane layout
    uint32_t stage_off1;      // plane layout: first words of tables 1 and 2
    uint32_t stage_off2;
    double mu_t;              // mu_s + mu_a of the solid, summed in FP64 on the host
    double mu_s;              // mu_s of the solid (the gradient walk's score)
    float g;
    float path_cap;           // +inf when off
    uint64_t s_q;             // round(mu_s / mu_t * 2^32), <= 2^32
    uint32_t w_th;            // roulette threshold (Q31)
    uint32_t t_m;             // survive roulette iff (r >> 8) < t_m
    uint32_t m;               // roulette multiplier
    uint32_t key0, key1;      // Philox key = seed
    uint32_t stream_id;
    int32_t source;           // 0 collimated, 1 Lambertian
    uint32_t max_steps;
    uint64_t photon_begin;    // first photon id
    uint64_t n_photons;
    uint64_t queue_begin;     // this job's offset in the launch-wide queue
    int32_t paper;            // paper boundary model: air pads, mirrors or periodic, index, gate
    int32_t lateral;          // paper model: 1 mirrors, 0 periodic
    float n_solid;            // refractive index of the solid (1 in the plain model)
    int32_t fresnel;          // n_solid != 1
    double gate;              // optical path limit (paper model), +inf when off
};

template <typename R>
struct Photon {
    int32_t ix, iy, iz;
    R fx, fy, fz;
    R ux, uy, uz;
    R iux, iuy, iuz;          // 1/|u| per axis (+inf where u = 0), kept with the direction
    double s_rem;             // remaining free path, in solid path length
    double l_void, l_tot;     // path inside pores, total path
    double score_g;           // sum of d ln p_HG / dg over the deflections so far (gradient walk)
    uint32_t w, k, steps, pid;
    uint64_t absorbed;        // weight absorbed by this photon so far
    int64_t rr;               // roulette balance of this photon
    uint64_t acc;             // deposit in the current voxel not yet flushed, in quanta
    uint32_t brick;           // index of the cached brick
    uint32_t solid;           // current voxel is solid
    uint64_t bits;            // cached brick
    double l_opt;             // optical path sum(n d), pads included (paper model's gate)
    uint32_t nf;              // Fresnel decisions drawn so far
    U4 fr;                    // words of the current Fresnel block not drawn yet, next in fr.x
};

// precision-generic helpers.  The FP32 transport takes the hardware square root,
// sine and cosine (of 2 pi u, the unit being the turn) and base-2 logarithm: on
// this path's inputs they stay within 1.3e-7 of FP64 (sine and cosine, absolute,
// over all 2^24 uniforms) and 1.7e-7 relative (logarithm, square root), against
// 5e-8 and 1.6e-7 for the library's sincospif and logf; the FP64 transport takes
// the correctly rounded library functions.
__device__ __forceinline__ float r_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double r_sqrt(double x) { return sqrt(x); }
// sin and cos of 2 pi u for u in [0, 1)
__device__ __forceinline__ void r_sincos_turn(float u, float *s, float *c)
{
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ void r_sincos_turn(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }
// ln u for u in (0, 1]
__device__ __forceinline__ float r_log_unit(float u) { return __builtin_amdgcn_logf(u) * 0.693147180559945309f; }
__device__ __forceinline__ double r_log_unit(double u) { return log(u); }
__device__ __forceinline__ uint64_t r_to_u64(float x) { return __float2ull_rn(x); }
__device__ __forceinline__ uint64_t r_to_u64(double x) { return __double2ull_rn(x); }
template <typename R> __device__ __forceinline__ R r_inf() { return (R)kInf; }
template <typename R> __device__ __forceinline__ R clamp01(R x) { return fmin(fmax(x, (R)0), (R)1); }
template <typename R> __device__ __forceinline__ R u01(uint32_t r) { return (R)(r >> 8) * (R)0x1.0p-24; }
// 1/x: the hardware reciprocal in the FP32 transport (within 1 ulp), the correctly
// rounded quotient in the FP64 reference transport
__device__ __forceinline__ float r_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double r_rcp(double x) { return 1.0 / x; }
// a/b: a times the hardware reciprocal in FP32, the correctly rounded quotient in FP64
__device__ __forceinline__ float r_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double r_div(double a, double b) { return a / b; }
// 1/sqrt(x): the hardware reciprocal square root in FP32 (within 1 ulp)
__device__ __forceinline__ float r_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double r_rsqrt(double x) { return 1.0 / sqrt(x); }
// 1/|u| per axis, +inf on an axis the photon does not move along
template <typename R> __device__ __forceinline__ R inv_abs(R u) { return u != (R)0 ? r_rcp(fabs(u)) : r_inf<R>(); }

// The face distances divide by |u| every step; the quotients are computed once per
// direction (at launch, deflection and refraction) and kept in the photon state.
template <typename R> __device__ __forceinline__ void set_direction(Photon<R> &p, R ux, R uy, R uz)
{
    p.ux = ux;
    p.uy = uy;
    p.uz = uz;
    p.iux = inv_abs(ux);
    p.iuy = inv_abs(uy);
    p.iuz = inv_abs(uz);
}

__device__ __forceinline__ uint32_t brick_of(const Job &J, int32_t ix, int32_t iy, int32_t iz)
{
    return ((uint32_t)(iz >> 2) * (uint32_t)J.nyb + (uint32_t)(iy >> 2)) * (uint32_t)J.nxb + (uint32_t)(ix >> 2);
}

__device__ __forceinline__ uint32_t bit_of(int32_t ix, int32_t iy, int32_t iz)
{
    return ((uint32_t)(iz & 3) << 4) | ((uint32_t)(iy & 3) << 2) | (uint32_t)(ix & 3);
}

// Refresh the solid flag of the current voxel, reloading the brick only when
// the photon has left the cached one.  The air pads (iz outside [0, nz)) are
// not solid (GENERAL walks only; the plain walk never stands in a pad).
template <bool GENERAL, typename R>
__device__ __forceinline__ void lookup(Photon<R> &p, const Job &J)
{
    if (GENERAL && (p.iz < 0 || p.iz >= J.nz)) {
        p.solid = 0u;
        return;
    }
    const uint32_t b = brick_of(J, p.ix, p.iy, p.iz);
    if (b != p.brick) {
        p.bits = J.bricks[b];
        p.brick = b;
    }
    p.solid = (uint32_t)((p.bits >> bit_of(p.ix, p.iy, p.iz)) & 1ull) ^ 1u;
}

template <typename R>
__device__ __forceinline__ uint64_t voxel_index(const Job &J, const Photon<R> &p)
{
    return ((uint64_t)p.iz * (uint64_t)J.ny + (uint64_t)p.iy) * (uint64_t)J.nx + (uint64_t)p.ix;
}

// A segment's track-length deposit w d is rounded to a whole number of quanta of
// 2^kDepositShift Q31 weight x voxel (2^-23 of a launched photon x voxel); the
// tallies hold Q31 units, so every tally value is a multiple of the quantum.
constexpr int kDepositShift = 8;

// Index in the staging tally of the logged deposits: uint32 words in lines of
// 2 x 2 x 4 voxels (x, y, z), one line = 16 words = one 64-byte memory-side atomic
// request, so that successive deposits of a photon tend to share a line.
__host__ __device__ __forceinline__ uint32_t stage_index(int32_t lnx, int32_t lny, int32_t ix, int32_t iy, int32_t iz)
{
    const uint32_t line = ((uint32_t)(iz >> 2) * (uint32_t)lny + (uint32_t)(iy >> 1)) * (uint32_t)lnx + (uint32_t)(ix >> 1);
    return (line << 4) | ((uint32_t)(iz & 3) << 2) | ((uint32_t)(iy & 1) << 1) | (uint32_t)(ix & 1);
}

// Plane layout of the staging tally: three tables whose lines are 4 x 4 voxels
// one voxel thin, across x (table 0: 1 x 4 x 4), across y (table 1: 4 x 1 x 4)
// and across z (table 2: 4 x 4 x 1), each padded to whole lines along its
// 4-voxel axes.  A deposit goes into the table across the axis of the photon's
// smallest direction component, so that the line extends along the two axes
// the photon moves along most: over oracle trajectories of the 256^3 workload
// this gives 0.375 requests per photon-step against 0.401 for the one table of
// 2 x 2 x 4 lines.  A voxel's total is the sum of its three words.
struct PlaneDims {
    uint32_t px, py, pz;      // 4-voxel groups along x, y, z
    uint32_t off1, off2;      // first words of tables 1 and 2
    uint64_t words;           // words of the three tables
};

__host__ __device__ __forceinline__ PlaneDims plane_dims(int32_t nx, int32_t ny, int32_t nz)
{
    PlaneDims P;
    P.px = ((uint32_t)nx + 3u) >> 2;
    P.py = ((uint32_t)ny + 3u) >> 2;
    P.pz = ((uint32_t)nz + 3u) >> 2;
    const uint64_t t0 = (uint64_t)nx * P.py * P.pz * 16, t1 = (uint64_t)P.px * ny * P.pz * 16;
    P.off1 = (uint32_t)t0;
    P.off2 = (uint32_t)(t0 + t1);
    P.words = t0 + t1 + (uint64_t)P.px * P.py * nz * 16;
    return P;
}

// Word of voxel (ix, iy, iz) in plane table t; valid where P.words <= 2^32.
__host__ __device__ __forceinline__ uint32_t plane_index(const PlaneDims &P, int32_t nx, int32_t ny, uint32_t t,
                                                         int32_t ix, int32_t iy, int32_t iz)
{
    const uint32_t x = (uint32_t)ix, y = (uint32_t)iy, z = (uint32_t)iz;
    const uint32_t zh = t == 2u ? z : z >> 2;
    const uint32_t yh = t == 1u ? y : y >> 2;
    const uint32_t xh = t == 0u ? x : x >> 2;
    const uint32_t ly = t == 1u ? (uint32_t)ny : P.py;
    const uint32_t lx = t == 0u ? (uint32_t)nx : P.px;
    const uint32_t hi = t == 2u ? (y & 3u) : (z & 3u);
    const uint32_t lo = t == 0u ? (y & 3u) : (x & 3u);
    const uint32_t first = t == 0u ? 0u : (t == 1u ? P.off1 : P.off2);
    return first + ((((zh * ly + yh) * lx + xh)) << 4) + (hi << 2) + lo;
}

// The plane table of a deposit: the one across the axis of the smallest |u|.
template <typename R>
__device__ __forceinline__ uint32_t plane_table(R ux, R uy, R uz)
{
    const R ax = fabs(ux), ay = fabs(uy), az = fabs(uz);
    return (ax <= ay && ax <= az) ? 0u : (ay <= az ? 1u : 2u);
}

// The plane layout's dimensions from a job: the table offsets are stored in it
// (the batch reads its jobs from LDS, per lane).
__host__ __device__ __forceinline__ PlaneDims plane_dims_of(const Job &J)
{
    PlaneDims P;
    P.px = ((uint32_t)J.nx + 3u) >> 2;
    P.py = ((uint32_t)J.ny + 3u) >> 2;
    P.pz = ((uint32_t)J.nz + 3u) >> 2;
    P.off1 = J.stage_off1;
    P.off2 = J.stage_off2;
    P.words = 0;   // unused here
    return P;
}

// The staging word of a photon's deposit in its current voxel.
template <typename R>
__device__ __forceinline__ uint32_t stage_word(const Job &J, const Photon<R> &p)
{
    if (J.stage_planes)
        return plane_index(plane_dims_of(J), J.nx, J.ny, plane_table(p.ux, p.uy, p.uz), p.ix, p.iy, p.iz);
    return stage_index(J.lnx, J.lny, p.ix, p.iy, p.iz);
}

// The voxel, as an index of the [nz][ny][nx] tally, of a plane-layout word.
__host__ __device__ __forceinline__ uint64_t plane_voxel(const Job &J, uint32_t idx)
{
    const PlaneDims P = plane_dims_of(J);
    const uint32_t t = idx < P.off1 ? 0u : (idx < P.off2 ? 1u : 2u);
    const uint32_t r = idx - (t == 0u ? 0u : (t == 1u ? P.off1 : P.off2));
    const uint32_t line = r >> 4, hi = (r >> 2) & 3u, lo = r & 3u;
    uint64_t x, y, z;
    if (t == 0u) {
        const uint32_t q = line / (uint32_t)J.nx;
        x = line - q * (uint32_t)J.nx;
        y = (uint64_t)(q % P.py) * 4 + lo;
        z = (uint64_t)(q / P.py) * 4 + hi;
    } else if (t == 1u) {
        const uint32_t q = line / P.px;
        x = (uint64_t)(line - q * P.px) * 4 + lo;
        y = q % (uint32_t)J.ny;
        z = (uint64_t)(q / (uint32_t)J.ny) * 4 + hi;
    } else {
        const uint32_t q = line / P.px;
        x = (uint64_t)(line - q * P.px) * 4 + lo;
        y = (uint64_t)(q % P.py) * 4 + hi;
        z = q / P.py;
    }
    return (z * (uint64_t)J.ny + y) * (uint64_t)J.nx + x;
}

// The voxel, as an index of the [nz][ny][nx] tally, of a staging word.
__host__ __device__ __forceinline__ uint64_t stage_voxel(const Job &J, uint32_t idx)
{
    if (J.stage_planes) return plane_voxel(J, idx);
    const uint32_t line = idx >> 4, off = idx & 15u;
    const uint32_t t = line / (uint32_t)J.lnx;
    const uint64_t x = (uint64_t)(line - t * (uint32_t)J.lnx) * 2 + (off & 1u);
    const uint32_t bz = t / (uint32_t)J.lny;
    const uint64_t y = (uint64_t)(t - bz * (uint32_t)J.lny) * 2 + ((off >> 1) & 1u);
    const uint64_t z = (uint64_t)bz * 4 + (off >> 2);
    return (z * (uint64_t)J.ny + y) * (uint64_t)J.nx + x;
}

// The walks' deposit logs (LDS, one per wavefront): slot s of lane l is element
// s * STRIDE + l of two arrays, a staging word index and a value.  A lane's slots
// form a ring of K: its entries, oldest first, sit in slots (head + j) mod K for
// j < count.  A logged value is below 2^31: the top bit marks an entry held back
// from the next issue.
constexpr uint32_t kLogHeld = 0x80000000u;

// The slot of a lane's next entry.
template <int STRIDE, int K>
__device__ __forceinline__ uint32_t log_slot(uint32_t lane, uint32_t head, uint32_t count)
{
    return ((head + count) & (uint32_t)(K - 1)) * STRIDE + lane;
}

// Mark the newest entries of this lane's log that lie in `line` (the staging line of
// its next deposit; kNoLine-like values match nothing), at most CAP of them, stopping
// at the first that does not; returns how many.
template <int STRIDE, int K, int CAP>
__device__ __forceinline__ uint32_t log_mark_run(const uint32_t *lidx, uint32_t *lval, uint32_t lane, uint32_t head,
                                                 uint32_t count, uint32_t line)
{
    uint32_t n = 0;
    bool run = true;
#pragma unroll
    for (int k = 0; k < CAP; ++k) {
        const uint32_t e = ((head + count - 1u - (uint32_t)k) & (uint32_t)(K - 1)) * STRIDE + lane;
        run = run && (uint32_t)k < count && (lidx[e] >> 4) == line;
        if (run) {
            lval[e] |= kLogHeld;
            ++n;
        }
    }
    return n;
}

// After an issue that skipped them: unmark this lane's n held entries (the newest n
// of its count) and make them the whole ring.
template <int STRIDE, int K, int CAP>
__device__ __forceinline__ void log_keep_run(uint32_t *lval, uint32_t lane, uint32_t &head, uint32_t &count,
                                             uint32_t n)
{
#pragma unroll
    for (int k = 0; k < CAP; ++k)
        if ((uint32_t)k < n) lval[((head + count - 1u - (uint32_t)k) & (uint32_t)(K - 1)) * STRIDE + lane] &= ~kLogHeld;
    head = (head + count - n) & (uint32_t)(K - 1);
    count = n;
}

template <typename R>
__device__ __forceinline__ double free_path(const Job &J, uint32_t r)
{
    // tau = -ln U, U in (0,1]; the interaction lies tau / mu_t into the solid.  The
    // FP32 transport takes the logarithm and the quotient in FP32 (the remaining path
    // is then kept in FP64 as it is consumed); the FP64 transport takes both in FP64.
    if (!(J.mu_t > 0.0)) return (double)kInf;
    if constexpr (std::is_same<R, float>::value) {
        const float u = (float)((r >> 8) + 1u) * 0x1.0p-24f;
        return (double)(-r_log_unit(u) * r_rcp((float)J.mu_t));
    } else {
        const double u = (double)((r >> 8) + 1u) * 0x1.0p-24;
        return -r_log_unit(u) / J.mu_t;
    }
}

// Launch photon `pid` (Philox block k = 0): uniform position on the z = 0 face
// from 24-bit uniforms scaled by the face size in integer arithmetic, normal
// incidence (or Lambertian for the test source), first free path.
template <bool GENERAL, typename R>
__device__ __forceinline__ void launch(Photon<R> &p, const Job &J, uint32_t pid)
{
    const U4 r = philox4x32_10(U4{0u, pid, J.stream_id, 0u}, J.key0, J.key1);
    const uint64_t X = (uint64_t)(r.x >> 8) * (uint64_t)J.nx;
    const uint64_t Y = (uint64_t)(r.y >> 8) * (uint64_t)J.ny;
    p.ix = (int32_t)(X >> 24);
    p.iy = (int32_t)(Y >> 24);
    p.iz = (GENERAL && J.paper) ? -1 : 0;  // paper model: the outer face of the top air pad
    p.fx = (R)(uint32_t)(X & 0xFFFFFFu) * (R)0x1.0p-24;
    p.fy = (R)(uint32_t)(Y & 0xFFFFFFu) * (R)0x1.0p-24;
    p.fz = (R)0;
    if (J.source == 1) {
        const U4 s = philox4x32_10(U4{0u, pid, J.stream_id, 1u}, J.key0, J.key1);
        const R ct = r_sqrt(u01<R>(s.x));
        const R st = r_sqrt(fmax((R)0, ((R)1 - ct) * ((R)1 + ct)));
        R sp, cp;
        r_sincos_turn(u01<R>(s.y), &sp, &cp);
        set_direction(p, st * cp, st * sp, ct);
    } else {
        set_direction(p, (R)0, (R)0, (R)1);
    }
    p.s_rem = free_path<R>(J, r.z);
    p.l_void = 0.0;
    p.l_tot = 0.0;
    p.score_g = 0.0;
    p.w = kW1;
    p.k = 0u;
    p.steps = 0u;
    p.pid = pid;
    p.absorbed = 0ull;
    p.rr = 0;
    p.acc = 0ull;
    p.brick = 0xFFFFFFFFu;
    p.l_opt = 0.0;
    p.nf = 0u;
    lookup<GENERAL>(p, J);
}

// Henyey-Greenstein deflection and the MCML direction update.  sin(theta) is
// formed from (1 - cos)(1 + cos), each factor written without cancellation:
//   1 - cos = (1-g)(1-xi)(t+1-g)/den,  1 + cos = (1+g) xi (1+g+t)/den,
// with den = 1 - g + 2 g xi and t = (1 - g^2)/den.  The transverse norm of the
// old direction is sqrt(ux^2 + uy^2) (= sqrt(1 - uz^2) for a unit vector).
// Returns cos(theta) (the gradient walk scores it).
template <typename R>
__device__ __forceinline__ R scatter(Photon<R> &p, const Job &J, uint32_t r0, uint32_t r1)
{
    const R g = (R)J.g, xi = u01<R>(r0);
    R ct, st2;
    if (g != (R)0) {
        const R den = (R)1 - g + (R)2 * g * xi;
        const R t = r_div((R)1 - g * g, den);
        ct = r_div((R)1 + g * g - t * t, (R)2 * g);
        const R om = r_div(((R)1 - g) * ((R)1 - xi) * (t + (R)1 - g), den);
        const R op = r_div(((R)1 + g) * xi * ((R)1 + g + t), den);
        st2 = om * op;
    } else {
        ct = (R)2 * xi - (R)1;
        st2 = (R)4 * xi * ((R)1 - xi);
    }
    ct = fmin(fmax(ct, (R)-1), (R)1);
    const R st = r_sqrt(fmax(st2, (R)0));
    R sp, cp;
    r_sincos_turn(u01<R>(r1), &sp, &cp);
    const R ux = p.ux, uy = p.uy, uz = p.uz;
    const R tn = r_sqrt(ux * ux + uy * uy);
    R nx, ny, nz;
    if (tn == (R)0) {
        nx = st * cp;
        ny = st * sp;
        nz = (uz >= (R)0 ? ct : -ct);
    } else {
        const R it = r_rcp(tn);
        nx = st * (ux * uz * cp - uy * sp) * it + ux * ct;
        ny = st * (uy * uz * cp + ux * sp) * it + uy * ct;
        nz = -st * cp * tn + uz * ct;
    }
    const R inrm = r_rsqrt(nx * nx + ny * ny + nz * nz);
    set_direction(p, nx * inrm, ny * inrm, nz * inrm);
    return ct;
}

// Unpolarised Fresnel reflectance from index n1 into n2 at incidence cosine ci:
// the mean of the s and p power coefficients.  Returns 1 on total internal
// reflection; otherwise *ct is the cosine of the refracted direction.
// The FP32 transport forms both quotients from one reciprocal of the product of
// their denominators.
template <typename R>
__device__ __forceinline__ R fresnel(R n1, R n2, R ci, R *ct)
{
    const R eta = r_div(n1, n2);
    const R st2 = eta * eta * ((R)1 - ci * ci);
    if (st2 >= (R)1) {
        *ct = (R)0;
        return (R)1;
    }
    const R c = r_sqrt((R)1 - st2);
    R rs, rp;
    if constexpr (std::is_same<R, float>::value) {
        const R ds = n1 * ci + n2 * c, dp = n1 * c + n2 * ci;
        const R inv = r_rcp(ds * dp);
        rs = (n1 * ci - n2 * c) * dp * inv;
        rp = (n1 * c - n2 * ci) * ds * inv;
    } else {
        rs = (n1 * ci - n2 * c) / (n1 * ci + n2 * c);
        rp = (n1 * c - n2 * ci) / (n1 * c + n2 * ci);
    }
    *ct = c;
    return (R)0.5 * (rs * rs + rp * rp);
}

// Uniform of the photon's next Fresnel decision: word j & 3 of block j >> 2 of
// its tag-4 Philox stream, a block drawn once per four decisions.  The unused
// words wait in p.fr and move down one place per draw (a variable word index
// would force the photon state out of registers).
template <typename R>
__device__ __forceinline__ R fresnel_uniform(Photon<R> &p, const Job &J)
{
    const uint32_t j = p.nf++;
    if ((j & 3u) == 0u) p.fr = philox4x32_10(U4{j >> 2, p.pid, J.stream_id, 4u}, J.key0, J.key1);
    const uint32_t w = p.fr.x;
    p.fr.x = p.fr.y;
    p.fr.y = p.fr.z;
    p.fr.z = p.fr.w;
    return u01<R>(w);
}

// An event a walk kernel sees between advance() and interact(): the photon stands
// at an interaction point, its interaction not yet drawn.  Never recorded.
constexpr int32_t EV_AT_INTERACTION = 13;

// One photon-step is advance() and, when the segment ends at an interaction point,
// interact(), then finish().  step() runs them back to back; the walk kernels may
// run a lane's interact() some iterations after its advance() (the lane waits
// meanwhile), which changes nothing in the photon's history.
//
// advance(): the segment inside the current voxel up to a face, an interaction
// point or an escape (and, in the GENERAL walk, a reflection or the time gate).
// The Sink receives every segment (deposits and gradient scores are taken only
// inside the slab) and the flushed per-voxel deposits.
template <bool GENERAL, typename R, class Sink>
__device__ __forceinline__ int32_t advance(Photon<R> &p, const Job &J, Sink &sink)
{
    const R dx = p.ux != (R)0 ? (p.ux > (R)0 ? (R)1 - p.fx : p.fx) * p.iux : r_inf<R>();
    const R dy = p.uy != (R)0 ? (p.uy > (R)0 ? (R)1 - p.fy : p.fy) * p.iuy : r_inf<R>();
    const R dz = p.uz != (R)0 ? (p.uz > (R)0 ? (R)1 - p.fz : p.fz) * p.iuz : r_inf<R>();
    int32_t axis = 0;
    R d_face = dx;
    R ua = p.ux;              // direction component normal to the face reached
    if (dy < d_face) { axis = 1; d_face = dy; ua = p.uy; }
    if (dz < d_face) { axis = 2; d_face = dz; ua = p.uz; }
    const bool solid = p.solid != 0u;
    bool interact = solid && (p.s_rem <= (double)d_face);
    R d = interact ? (R)p.s_rem : d_face;
    bool in_slab = true, gated = false;
    double n_here = 1.0;
    if constexpr (GENERAL) {
        in_slab = p.iz >= 0 && p.iz < J.nz;
        n_here = solid ? (double)J.n_solid : 1.0;
        // the optical path may reach the gate, not pass it
        if (p.l_opt + n_here * (double)d > J.gate) {
            gated = true;
            interact = false;
            d = (R)fmax((J.gate - p.l_opt) / n_here, 0.0);
        }
    }

    sink.segment(p, J, d, solid);
    if (in_slab) {
        // track-length deposit, rounded to whole quanta per segment, accumulated while in this voxel
        p.acc += r_to_u64((R)p.w * d * (R)(1.0 / (1 << kDepositShift)));
        if (solid) p.s_rem = fmax(p.s_rem - (double)d, 0.0);
        else p.l_void += (double)d;
        p.l_tot += (double)d;
    }
    if constexpr (GENERAL) p.l_opt += n_here * (double)d;
    p.steps += 1u;

    int32_t ev;
    if ((GENERAL && gated) || interact) {
        p.fx = clamp01(p.fx + p.ux * d);
        p.fy = clamp01(p.fy + p.uy * d);
        p.fz = clamp01(p.fz + p.uz * d);
        ev = (GENERAL && gated) ? EV_GATED : EV_AT_INTERACTION;
    } else if constexpr (!GENERAL) {
        // the two other axes advance; the face axis is set on the face the photon enters
        // (every component written with a value select, so no lane branches on the axis)
        const R ax = clamp01(p.fx + p.ux * d), ay = clamp01(p.fy + p.uy * d), az = clamp01(p.fz + p.uz * d);
        const bool up = ua > (R)0;
        const R enter = up ? (R)0 : (R)1;
        p.fx = axis == 0 ? enter : ax;
        p.fy = axis == 1 ? enter : ay;
        p.fz = axis == 2 ? enter : az;
        sink.flush(J, p, p.acc);
        p.acc = 0ull;
        const int32_t sgn = up ? 1 : -1;
        const int32_t jx = p.ix + sgn, jy = p.iy + sgn;
        // lateral faces are periodic
        const int32_t wx = jx == J.nx ? 0 : (jx < 0 ? J.nx - 1 : jx);
        const int32_t wy = jy == J.ny ? 0 : (jy < 0 ? J.ny - 1 : jy);
        p.ix = axis == 0 ? wx : p.ix;
        p.iy = axis == 1 ? wy : p.iy;
        p.iz = axis == 2 ? p.iz + sgn : p.iz;
        ev = axis;
        if (p.iz < 0) ev = EV_ESC_R;
        else if (p.iz >= J.nz) ev = EV_ESC_T;
        if (!is_terminal(ev)) lookup<false>(p, J);
    } else {
        if (axis != 0) p.fx = clamp01(p.fx + p.ux * d);
        if (axis != 1) p.fy = clamp01(p.fy + p.uy * d);
        if (axis != 2) p.fz = clamp01(p.fz + p.uz * d);
        const int32_t sgn = ua > (R)0 ? 1 : -1;
        int32_t jx = p.ix, jy = p.iy, jz = p.iz;
        bool reflect = false, out = false;
        if (axis == 0) {
            jx += sgn;
            if (jx < 0 || jx >= J.nx) {
                if (J.lateral) reflect = true;             // specular mirror
                else jx = jx < 0 ? J.nx - 1 : 0;           // periodic
            }
        } else if (axis == 1) {
            jy += sgn;
            if (jy < 0 || jy >= J.ny) {
                if (J.lateral) reflect = true;
                else jy = jy < 0 ? J.ny - 1 : 0;
            }
        } else {
            jz += sgn;
            out = J.paper ? (jz < -1 || jz > J.nz) : (jz < 0 || jz >= J.nz);
        }
        // the neighbour's medium, from the cached brick when it holds it
        uint32_t nb = p.brick;
        uint64_t nbits = p.bits;
        bool next_solid = false;
        if (!reflect && !out && jz >= 0 && jz < J.nz) {
            nb = brick_of(J, jx, jy, jz);
            if (nb != p.brick) nbits = J.bricks[nb];
            next_solid = ((nbits >> bit_of(jx, jy, jz)) & 1ull) == 0ull;
        }
        if (!reflect && !out && J.fresnel && next_solid != solid) {
            const R n1 = solid ? (R)J.n_solid : (R)1, n2 = next_solid ? (R)J.n_solid : (R)1;
            R ct;
            const R rf = fresnel(n1, n2, fabs(ua), &ct);
            if (rf >= (R)1 || fresnel_uniform(p, J) < rf) {
                reflect = true;
            } else {
                const R eta = r_div(n1, n2);
                set_direction(p, axis == 0 ? (R)sgn * ct : eta * p.ux, axis == 1 ? (R)sgn * ct : eta * p.uy,
                              axis == 2 ? (R)sgn * ct : eta * p.uz);
            }
        }
        // Every component is written with a value select: stores chosen by axis would
        // be merged into one store through a selected address, which keeps the photon
        // state in memory.
        if (reflect) {
            // stay in this voxel on the face, normal component reversed (|u| unchanged)
            const R face = sgn > 0 ? (R)1 : (R)0;
            p.ux = axis == 0 ? -p.ux : p.ux;
            p.uy = axis == 1 ? -p.uy : p.uy;
            p.uz = axis == 2 ? -p.uz : p.uz;
            p.fx = axis == 0 ? face : p.fx;
            p.fy = axis == 1 ? face : p.fy;
            p.fz = axis == 2 ? face : p.fz;
            ev = EV_REFLECT_X + axis;
        } else {
            if (in_slab) sink.flush(J, p, p.acc);
            p.acc = 0ull;
            if (out) {
                ev = jz < 0 ? EV_ESC_R : EV_ESC_T;
            } else {
                const R face = sgn > 0 ? (R)0 : (R)1;
                p.ix = jx; p.iy = jy; p.iz = jz;
                p.fx = axis == 0 ? face : p.fx;
                p.fy = axis == 1 ? face : p.fy;
                p.fz = axis == 2 ? face : p.fz;
                if (jz >= 0 && jz < J.nz) {
                    p.brick = nb;
                    p.bits = nbits;
                }
                p.solid = next_solid ? 1u : 0u;
                ev = axis;
            }
        }
    }
    return ev;
}

// interact(): the interaction at the point advance() stopped at, with Philox block k
// of the photon: implicit capture on the integer weight, Henyey-Greenstein
// deflection (the Sink sees the cosine), Russian roulette, the next free path.
template <typename R, class Sink>
__device__ __forceinline__ int32_t interact(Photon<R> &p, const Job &J, Sink &sink)
{
    p.k += 1u;
    const U4 r = philox4x32_10(U4{p.k, p.pid, J.stream_id, 0u}, J.key0, J.key1);
    // implicit capture on the integer weight, round half up
    const uint32_t w_new = (uint32_t)(((uint64_t)p.w * J.s_q + 0x80000000ull) >> 32);
    p.absorbed += (uint64_t)(p.w - w_new);
    p.w = w_new;
    if (w_new == 0u) return EV_DEAD_ABSORB;
    const R ct = scatter(p, J, r.x, r.y);
    sink.deflect(p, J, ct);
    int32_t ev = EV_SCATTER;
    if (p.w < J.w_th) {
        if ((r.w >> 8) < J.t_m) {
            p.rr -= (int64_t)(J.m - 1u) * (int64_t)p.w;
            p.w *= J.m;
        } else {
            p.rr += (int64_t)p.w;
            ev = EV_DEAD_ROULETTE;
        }
    }
    p.s_rem = free_path<R>(J, r.z);
    return ev;
}

// finish(): the step and path caps, and the deposit a photon that ends inside a
// voxel (absorbed, roulette, cap, gate) leaves there.
template <typename R, class Sink>
__device__ __forceinline__ int32_t finish(Photon<R> &p, const Job &J, Sink &sink, int32_t ev)
{
    if (!is_terminal(ev) && (p.steps >= J.max_steps || p.l_tot > (double)J.path_cap)) ev = EV_LOST;
    if (is_terminal(ev) && p.acc != 0ull) {
        sink.flush(J, p, p.acc);
        p.acc = 0ull;
    }
    return ev;
}

// One whole photon-step.  Returns the event.
template <bool GENERAL, typename R, class Sink>
__device__ __forceinline__ int32_t step(Photon<R> &p, const Job &J, Sink &sink)
{
    int32_t ev = advance<GENERAL>(p, J, sink);
    if (ev == EV_AT_INTERACTION) ev = interact(p, J, sink);
    return finish(p, J, sink, ev);
}

}  // namespace pmc
