/*
 * oracle.c -- plain FP64 reference of the photon-migration hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the HIP path.  It is deliberately slow and scalar: one photon at a time, in
 * the order the method states its steps, in double precision.
 *
 * What it follows (paper: "Three-dimensional photon transport in spinodal
 * photocatalytic aerogels"):
 *   - Sec. 2.5 (Three-dimensional Monte Carlo simulation): pores carry
 *     mu_a = mu_s = 0, solid voxels carry the shell coefficients; a planar
 *     collimated source covers the whole z = 0 face and propagates along +z;
 *     the axial faces are open and escaping weight is recorded on each face;
 *     the solver uses weighted photons with implicit capture and Russian
 *     roulette; absorptance comes from an absorbed-energy counter and R, T
 *     from the escape records, so R + T + A = 1 is a measurement (Eq. RTA,
 *     Eq. closure).
 *   - App. B (Monte Carlo solver configuration): source, tallies, fixed seed.
 *   - Sec. 3.5 (c) / Fig. 4c (per-photon path statistics): cumulative in-pore path
 *     of every escaping photon, and the weight fraction whose in-pore path
 *     exceeds the slab thickness L.
 *
 * Where the paper is silent the reading below is used (each is listed with
 * its reason in the design notes of the repository):
 *   - lateral faces periodic, n = 1 everywhere (no Fresnel, no air pad);
 *   - fluence is the track-length estimator: weight x segment length, per voxel;
 *   - absorption happens at interaction sites: w' = w * mu_s/mu_t, realised on
 *     an integer weight in units of 2^-31 with a survival factor quantised to
 *     S_q = round(mu_s/mu_t * 2^32) and round-half-up;
 *   - Russian roulette below w_th = floor(w_roulette * 2^31): survive with
 *     probability 1/m (integer compare on 24 random bits), weight times m;
 *   - free path tau = -ln U, U in (0,1] from 24 random bits;
 *   - Henyey-Greenstein polar angle by inverse CDF, azimuth 2*pi*U, direction
 *     update by the rotation formulas of Wang, Jacques & Zheng (MCML, 1995);
 *   - one Philox4x32-10 block (Salmon, Moraes, Dror & Shaw, SC'11) per event:
 *     key = (seed lo, seed hi), counter = (event k, photon id, stream id, tag);
 *     k = 0 is the launch, k >= 1 the k-th interaction.  tag 0 transport,
 *     tag 1 source extras (Lambertian test source);
 *   - ties: the face axis is the first minimum in x, y, z order; an interaction
 *     wins a tie against a face; in-voxel offsets are clamped to [0, 1].
 *
 * The paper's own boundary model (boundary = 1; Sec. 2.5 "Source and boundary
 * conditions" and "Photon budget, time gate and statistics", App. B):
 *   - a one-voxel air pad (index 1, no attenuation, no tally) on each axial
 *     face: layers iz = -1 and iz = nz.  Photons start on the outer face of the
 *     top pad and escape when they leave through the outer face of either pad;
 *   - lateral faces are specular mirrors (lateral = 1) or periodic (lateral = 0);
 *   - the solid has refractive index n_solid, pores and air have 1.  At every
 *     face between two media of different index the photon is reflected or
 *     refracted: total internal reflection when Snell's law has no solution,
 *     otherwise reflection with the Fresnel reflectance for unpolarised light
 *     (mean of the s and p power coefficients).  Reading: the choice is made
 *     against one uniform of its own Philox stream, tag 4, counter
 *     (j >> 2, photon, stream, 4), word j & 3 for the photon's j-th Fresnel
 *     decision.  Refraction scales the tangential direction components by
 *     n1/n2 and sets the normal one to cos(theta_t) with its sign kept;
 *   - time gate (Eq. tend): the photon's optical path sum(n d), pads included,
 *     may not exceed `gate` (c t_end in voxels).  The segment that reaches it is
 *     cut there, its part deposited, and the photon's weight goes to its own
 *     channel (gated), so the integer closure stays exact.
 * Path statistics (in-pore path, solid path) count slab voxels only.
 *
 * Gradients (likelihood-ratio / perturbation Monte Carlo) are not in the
 * paper; the oracle computes them from the path density
 *   mu_s^k * exp(-mu_t * l_solid) * prod_i p_HG(cos_i; g)
 * whose log-derivatives are the per-photon scores
 *   S_mus = k/mu_s - l_solid,  S_mua = -l_solid,
 *   S_g   = sum_i [-2g/(1-g^2) + 3(cos_i - g)/(1 + g^2 - 2 g cos_i)];
 * a segment of length d in a voxel adds w*(S*d - [solid] d^2/2) to the mu_s and
 * mu_a bins (survival inside the segment) and w*S_g*d to the g bin.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_W1 2147483648.0 /* launched weight 2^31 */
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the published definition (Salmon et al., SC'11):      */
/* each round multiplies counter words 0 and 2 by two fixed odd constants,   */
/* takes the 64-bit products apart into high and low halves, xors the high   */
/* halves with the other counter words and the round key, and permutes; the  */
/* key is advanced by the two Weyl increments between rounds.                */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t a_hi = (uint32_t)(prod_a >> 32), a_lo = (uint32_t)prod_a;
        uint32_t b_hi = (uint32_t)(prod_b >> 32), b_lo = (uint32_t)prod_b;
        uint32_t n0 = b_hi ^ c1 ^ k0;
        uint32_t n1 = b_lo;
        uint32_t n2 = a_hi ^ c3 ^ k1;
        uint32_t n3 = a_lo;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in [0,1) and in (0,1] from the top 24 bits of a word */
static double u_closed_open(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }
static double u_open_closed(uint32_t r) { return (double)((r >> 8) + 1u) * (1.0 / 16777216.0); }

typedef struct {
    int32_t nx, ny, nz;
    const uint8_t *mask;     /* [nz][ny][nx], 1 = pore, 0 = solid */
    double mu_s, mu_a, g;    /* solid coefficients per voxel; pores are 0 */
    double w_roulette;       /* roulette threshold as a fraction of the launch weight */
    uint32_t roulette_m;     /* survival 1/m */
    double path_cap;         /* total path cap in voxels (<= 0: none) */
    int32_t source;          /* 0 collimated normal incidence, 1 Lambertian (test source) */
    uint64_t seed;
    uint32_t stream_id;
    uint32_t max_steps;      /* step cap (photon counted as lost beyond it) */
    int32_t boundary;        /* 0: periodic laterals, index 1, no pads, no gate; 1: the paper's model */
    int32_t lateral;         /* boundary 1: 0 periodic, 1 specular mirrors */
    double n_solid;          /* boundary 1: refractive index of the solid (>= 1) */
    double gate;             /* boundary 1: optical path limit c t_end in voxels (INFINITY: none) */
} orc_problem;

/* integer channels */
enum {
    ORC_R, ORC_T, ORC_A, ORC_RR, ORC_LOST,
    ORC_ESC_W, ORC_ESC_W_GTL, ORC_ESC_N, ORC_ESC_N_GTL,
    ORC_STEPS, ORC_INTERACTIONS, ORC_GATED, ORC_NI
};
/* floating channels */
enum { ORC_ESC_W_VOID_PATH, ORC_PATH_TOTAL, ORC_PATH_SOLID, ORC_PATH_VOID, ORC_ND };

/* one record per step, for trajectory parity */
typedef struct {
    int32_t ix, iy, iz;
    int32_t event;           /* how the step ended, see below */
    double fx, fy, fz;       /* state at the start of the step */
    double ux, uy, uz;
    double d;                /* segment length */
    double tie_gap;          /* smallest gap between competing distances */
    int64_t w;               /* weight at the start of the step (units of 2^-31) */
    uint32_t k;              /* interactions so far */
    uint32_t pad;
} orc_rec;

/* events */
enum { EV_FACE_X = 0, EV_FACE_Y = 1, EV_FACE_Z = 2, EV_SCATTER = 3, EV_ESC_R = 4,
       EV_ESC_T = 5, EV_DEAD_ABSORB = 6, EV_DEAD_ROULETTE = 7, EV_LOST = 8, EV_GATED = 9,
       EV_REFLECT_X = 10, EV_REFLECT_Y = 11, EV_REFLECT_Z = 12 };

static int terminal(int ev) { return ev >= EV_ESC_R && ev <= EV_GATED; }

/* per-photon summary */
typedef struct {
    int64_t R, T, A, RR, lost;   /* this photon's share of each channel */
    int64_t w_final;
    uint64_t steps, interactions;
    double path_void, path_solid;
    double min_gap;              /* smallest tie gap over the whole walk (see orc_rec) */
    double max_visit;            /* largest weight x path deposited between two face crossings (one
                                    stay in a voxel), weight units 2^-31 x voxel: a diagnostic output */
    int32_t fate;                /* final event */
    int32_t pad;
} orc_photon;

typedef struct {
    int64_t ich[ORC_NI];
    double dch[ORC_ND];
} orc_sums;

/* what one walk writes into */
typedef struct {
    double *fluence;      /* [nvox] or NULL */
    double *grad;         /* [3][2][nz] or NULL */
    double *depth;        /* [2][nz] forward bins (phase-resolved depth sums) or NULL */
    orc_rec *trace;       /* [max_rec] or NULL */
    int32_t max_rec;
    orc_photon *summary;  /* or NULL */
    orc_sums *sums;
} orc_sink;

static void draw(const orc_problem *P, uint64_t photon, uint32_t k, uint32_t tag, uint32_t r[4])
{
    uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    uint32_t ctr[4] = {k, (uint32_t)photon, P->stream_id, tag};
    orc_philox(ctr, key, r);
}

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* d ln p_HG(mu; g) / dg */
static double hg_score(double mu, double g)
{
    return -2.0 * g / (1.0 - g * g) + 3.0 * (mu - g) / (1.0 + g * g - 2.0 * g * mu);
}

/* State of one photon between steps. */
typedef struct {
    int64_t ix, iy, iz;
    double fx, fy, fz;
    double ux, uy, uz;
    double tau;              /* optical depth left to the next interaction */
    int64_t w;               /* weight, units of 2^-31 */
    uint32_t k;              /* interactions so far */
    uint32_t pad;
    uint64_t steps;
    double l_void, l_solid;
    double score_s, score_a, score_g;   /* LR scores (see the header comment) */
    double l_opt;            /* optical path sum(n d) so far, pads included (time gate) */
    uint32_t nf;             /* Fresnel decisions drawn so far */
    uint32_t pad2;
} orc_state;

/* Launch: uniform position over the z = 0 face (integer voxel + offset from 24-bit
 * uniforms), direction +z (or Lambertian for the test source), weight 2^31, and the
 * optical depth of the first flight. */
static void launch(const orc_problem *P, uint64_t photon, orc_state *st)
{
    uint32_t r[4];
    draw(P, photon, 0, 0, r);
    memset(st, 0, sizeof *st);
    uint64_t X = (uint64_t)(r[0] >> 8) * (uint64_t)P->nx;
    uint64_t Y = (uint64_t)(r[1] >> 8) * (uint64_t)P->ny;
    st->ix = (int64_t)(X >> 24);
    st->iy = (int64_t)(Y >> 24);
    st->iz = P->boundary ? -1 : 0;   /* paper model: outer face of the top air pad */
    st->fx = (double)(X & 0xFFFFFFu) / 16777216.0;
    st->fy = (double)(Y & 0xFFFFFFu) / 16777216.0;
    st->fz = 0.0;
    st->ux = 0.0; st->uy = 0.0; st->uz = 1.0;
    if (P->source == 1) {
        uint32_t s[4];
        draw(P, photon, 0, 1, s);
        double ct = sqrt(u_closed_open(s[0]));
        double stt = sqrt(1.0 - ct * ct);
        double psi = 2.0 * ORC_PI * u_closed_open(s[1]);
        st->ux = stt * cos(psi);
        st->uy = stt * sin(psi);
        st->uz = ct;
    }
    st->tau = -log(u_open_closed(r[2]));
    st->w = (int64_t)ORC_W1;
}

/*
 * Fresnel reflectance for unpolarised light going from index n1 into n2 at
 * incidence cosine cos_i (> 0): the mean of the s and p power reflection
 * coefficients.  Returns 1 (and *cos_t = 0) for total internal reflection.
 */
double orc_fresnel(double n1, double n2, double cos_i, double *cos_t)
{
    const double eta = n1 / n2;
    const double sin_t2 = eta * eta * (1.0 - cos_i * cos_i);
    if (sin_t2 >= 1.0) {
        if (cos_t) *cos_t = 0.0;
        return 1.0;
    }
    const double ct = sqrt(1.0 - sin_t2);
    const double rs = (n1 * cos_i - n2 * ct) / (n1 * cos_i + n2 * ct);
    const double rp = (n1 * ct - n2 * cos_i) / (n1 * ct + n2 * cos_i);
    if (cos_t) *cos_t = ct;
    return 0.5 * (rs * rs + rp * rp);
}

/* uniform for the photon's j-th Fresnel decision (tag-4 stream, four words per block) */
static double fresnel_uniform(const orc_problem *P, uint64_t photon, uint32_t j)
{
    uint32_t r[4];
    draw(P, photon, j >> 2, 4, r);
    return u_closed_open(r[j & 3u]);
}

static int is_solid(const orc_problem *P, int64_t ix, int64_t iy, int64_t iz)
{
    if (iz < 0 || iz >= P->nz) return 0;   /* air pad */
    return P->mask[(iz * P->ny + iy) * P->nx + ix] == 0;
}

static void escape(const orc_problem *P, orc_state *st, orc_sink *S, orc_photon *me, int top)
{
    const int64_t w = st->w;
    if (top) { S->sums->ich[ORC_R] += w; me->R += w; }
    else     { S->sums->ich[ORC_T] += w; me->T += w; }
    S->sums->ich[ORC_ESC_W] += w;
    S->sums->ich[ORC_ESC_N] += 1;
    if (st->l_void > (double)P->nz) {
        S->sums->ich[ORC_ESC_W_GTL] += w;
        S->sums->ich[ORC_ESC_N_GTL] += 1;
    }
    S->sums->dch[ORC_ESC_W_VOID_PATH] += (double)w * st->l_void;
}

/*
 * One step from state st: the segment inside the current voxel up to a face, an
 * interaction, the time gate or an escape.  Updates st, the sink and the photon's
 * own shares me; returns the event, and sets *gap to how close the step came to a
 * different decision (|s_int - d_face|, the gaps between face distances, and in the
 * paper model the gate margin and the Fresnel uniform's distance to the reflectance).
 */
static int step(const orc_problem *P, uint64_t photon, orc_state *st, orc_sink *S, orc_photon *me, double *gap_out)
{
    const int64_t nx = P->nx, ny = P->ny, nz = P->nz;
    const int paper = (P->boundary == 1);
    const double mu_t_solid = P->mu_s + P->mu_a;
    /* survival factor of one interaction, as an integer fraction of 2^32 */
    uint64_t S_q = 0;
    if (mu_t_solid > 0.0) S_q = (uint64_t)llround(P->mu_s / mu_t_solid * 4294967296.0);
    const int64_t w_th = (int64_t)floor(P->w_roulette * ORC_W1);
    const uint32_t T_m = (uint32_t)llround(16777216.0 / (double)P->roulette_m);

    const int in_slab = (st->iz >= 0 && st->iz < nz);
    const int64_t v = in_slab ? (st->iz * ny + st->iy) * nx + st->ix : -1;
    const int solid = in_slab && P->mask[v] == 0;
    const double mu_t = solid ? mu_t_solid : 0.0;
    const double n_here = (paper && solid) ? P->n_solid : 1.0;

    /* distance to each face along the direction of travel */
    double dist[3];
    double f[3] = {st->fx, st->fy, st->fz};
    double u[3] = {st->ux, st->uy, st->uz};
    for (int a = 0; a < 3; ++a) {
        if (u[a] > 0.0) dist[a] = (1.0 - f[a]) / u[a];
        else if (u[a] < 0.0) dist[a] = f[a] / (-u[a]);
        else dist[a] = INFINITY;
    }
    int axis = 0;
    if (dist[1] < dist[axis]) axis = 1;
    if (dist[2] < dist[axis]) axis = 2;
    const double d_face = dist[axis];
    const double s_int = (mu_t > 0.0) ? st->tau / mu_t : INFINITY;
    int interact = (s_int <= d_face);
    double d = interact ? s_int : d_face;

    double gap = fabs(s_int - d_face);
    for (int a = 0; a < 3; ++a)
        if (a != axis && isfinite(dist[a])) {
            double ga = fabs(dist[a] - d_face);
            if (ga < gap) gap = ga;
        }
    /* Time gate of Eq. tend.  A photon's time of flight is its optical path over
     * c, t = sum(n_i d_i) / c (light moves at c/n in a medium of index n), so the
     * condition t <= t_end reads sum(n d) <= c t_end = gate, written here on the
     * optical path after this segment.  Reading: the photon may reach the gate
     * but not pass it; the segment that would pass it is cut where t = t_end. */
    int gated = 0;
    if (paper && isfinite(P->gate)) {
        const double gg = fabs(st->l_opt + n_here * d - P->gate) / n_here;
        if (gg < gap) gap = gg;
        if (st->l_opt + n_here * d > P->gate) {
            const double t_left = (P->gate - st->l_opt) / n_here;
            gated = 1;
            interact = 0;
            d = t_left > 0.0 ? t_left : 0.0;
        }
    }
    orc_rec *rec = NULL;
    if (S->trace && (int64_t)st->steps < S->max_rec) {
        rec = &S->trace[st->steps];
        rec->ix = (int32_t)st->ix; rec->iy = (int32_t)st->iy; rec->iz = (int32_t)st->iz;
        rec->fx = st->fx; rec->fy = st->fy; rec->fz = st->fz;
        rec->ux = st->ux; rec->uy = st->uy; rec->uz = st->uz;
        rec->w = st->w; rec->k = st->k; rec->d = d;
        rec->event = -1;
    }

    /* track-length deposit (slab voxels only) */
    const int64_t w = st->w;
    if (in_slab) {
        if (S->fluence) S->fluence[v] += (double)w * d;
        if (S->depth) S->depth[(solid ? 0 : 1) * nz + st->iz] += (double)w * d;
        if (S->grad) {
            const int ph = solid ? 0 : 1;
            const double sq = solid ? 0.5 * d * d : 0.0;
            S->grad[(0 * 2 + ph) * nz + st->iz] += (double)w * (st->score_s * d - sq);
            S->grad[(1 * 2 + ph) * nz + st->iz] += (double)w * (st->score_a * d - sq);
            S->grad[(2 * 2 + ph) * nz + st->iz] += (double)w * (st->score_g * d);
        }
        if (solid) {
            st->l_solid += d;
            st->score_s -= d;
            st->score_a -= d;
        } else {
            st->l_void += d;
        }
    }
    st->l_opt += n_here * d;

    int event;
    int done = 0;
    if (interact || gated) {
        st->fx = clamp01(st->fx + st->ux * d);
        st->fy = clamp01(st->fy + st->uy * d);
        st->fz = clamp01(st->fz + st->uz * d);
        if (interact) {
            st->tau = 0.0;
            event = EV_SCATTER;
        } else {
            st->tau -= mu_t * d;
            if (st->tau < 0.0) st->tau = 0.0;
            event = EV_GATED;
        }
    } else {
        if (axis != 0) st->fx = clamp01(st->fx + st->ux * d);
        if (axis != 1) st->fy = clamp01(st->fy + st->uy * d);
        if (axis != 2) st->fz = clamp01(st->fz + st->uz * d);
        st->tau -= mu_t * d;
        if (st->tau < 0.0) st->tau = 0.0;
        event = axis;
    }
    st->steps += 1;

    if (gated) {
        S->sums->ich[ORC_GATED] += st->w;
        done = 1;
    } else if (!interact && !paper) {
        /* cross the face: periodic laterals, open axial faces */
        if (axis == 0) {
            if (st->ux > 0.0) { st->ix += 1; st->fx = 0.0; if (st->ix == nx) st->ix = 0; }
            else              { st->ix -= 1; st->fx = 1.0; if (st->ix < 0) st->ix = nx - 1; }
        } else if (axis == 1) {
            if (st->uy > 0.0) { st->iy += 1; st->fy = 0.0; if (st->iy == ny) st->iy = 0; }
            else              { st->iy -= 1; st->fy = 1.0; if (st->iy < 0) st->iy = ny - 1; }
        } else {
            if (st->uz > 0.0) { st->iz += 1; st->fz = 0.0; }
            else              { st->iz -= 1; st->fz = 1.0; }
            if (st->iz < 0 || st->iz >= nz) {
                /* escape through an open axial face */
                const int top = (st->iz < 0);
                escape(P, st, S, me, top);
                event = top ? EV_ESC_R : EV_ESC_T;
                done = 1;
            }
        }
    } else if (!interact) {
        /* paper model: mirror, Fresnel reflection / refraction, or crossing */
        int64_t j[3] = {st->ix, st->iy, st->iz};
        const double sgn = (axis == 0 ? st->ux : axis == 1 ? st->uy : st->uz) > 0.0 ? 1.0 : -1.0;
        j[axis] += (int64_t)sgn;
        int reflect = 0, out = 0;
        if (axis < 2) {
            const int64_t n_ax = axis == 0 ? nx : ny;
            if (j[axis] < 0 || j[axis] >= n_ax) {
                if (P->lateral == 1) reflect = 1;                   /* specular mirror */
                else j[axis] = (j[axis] < 0) ? n_ax - 1 : 0;        /* periodic */
            }
        } else if (j[2] < -1 || j[2] > nz) {
            out = 1;                                                /* through a pad's outer face */
        }
        double uu[3] = {st->ux, st->uy, st->uz};
        if (!reflect && !out) {
            const double n_next = is_solid(P, j[0], j[1], j[2]) ? P->n_solid : 1.0;
            if (n_next != n_here) {
                const double cos_i = fabs(uu[axis]);
                double cos_t;
                const double R = orc_fresnel(n_here, n_next, cos_i, &cos_t);
                if (R >= 1.0) {
                    reflect = 1;                                    /* total internal reflection */
                } else {
                    const double U = fresnel_uniform(P, photon, st->nf);
                    st->nf += 1;
                    const double gf = fabs(U - R);
                    if (gf < gap) gap = gf;
                    if (U < R) {
                        reflect = 1;
                    } else {
                        const double eta = n_here / n_next;
                        for (int a = 0; a < 3; ++a) uu[a] = (a == axis) ? sgn * cos_t : eta * uu[a];
                    }
                }
            }
        }
        if (reflect) {
            uu[axis] = -uu[axis];
            f[0] = st->fx; f[1] = st->fy; f[2] = st->fz;
            f[axis] = sgn > 0.0 ? 1.0 : 0.0;
            st->fx = f[0]; st->fy = f[1]; st->fz = f[2];
            event = EV_REFLECT_X + axis;
        } else if (out) {
            escape(P, st, S, me, j[2] < 0);
            event = j[2] < 0 ? EV_ESC_R : EV_ESC_T;
            done = 1;
        } else {
            st->ix = j[0]; st->iy = j[1]; st->iz = j[2];
            f[0] = st->fx; f[1] = st->fy; f[2] = st->fz;
            f[axis] = sgn > 0.0 ? 0.0 : 1.0;
            st->fx = f[0]; st->fy = f[1]; st->fz = f[2];
        }
        st->ux = uu[0]; st->uy = uu[1]; st->uz = uu[2];
    } else {
        /* interaction: absorb, scatter, roulette, new free path */
        st->k += 1;
        uint32_t r[4];
        draw(P, photon, st->k, 0, r);
        const int64_t w_new = (int64_t)(((uint64_t)st->w * S_q + 2147483648ull) >> 32);
        S->sums->ich[ORC_A] += st->w - w_new;
        me->A += st->w - w_new;
        st->w = w_new;
        if (w_new == 0) {
            event = EV_DEAD_ABSORB;
            done = 1;
        } else {
            /* Henyey-Greenstein polar angle, inverse CDF */
            const double g = P->g, xi = u_closed_open(r[0]);
            double ct;
            if (g != 0.0) {
                const double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
                ct = (1.0 + g * g - t * t) / (2.0 * g);
            } else {
                ct = 2.0 * xi - 1.0;
            }
            if (ct < -1.0) ct = -1.0;
            if (ct > 1.0) ct = 1.0;
            const double stt = sqrt(1.0 - ct * ct);
            const double psi = 2.0 * ORC_PI * u_closed_open(r[1]);
            const double cp = cos(psi), sp = sin(psi);
            st->score_g += hg_score(ct, g);
            if (P->mu_s > 0.0) st->score_s += 1.0 / P->mu_s;
            /* rotate the direction (MCML).  The transverse norm is
             * sqrt(1 - uz^2) = sqrt(ux^2 + uy^2) for a unit vector; the
             * axis-aligned form is used only when the direction lies on the
             * z axis. */
            const double ux = st->ux, uy = st->uy, uz = st->uz;
            const double tn = sqrt(ux * ux + uy * uy);
            double nux, nuy, nuz;
            if (tn == 0.0) {
                nux = stt * cp;
                nuy = stt * sp;
                nuz = (uz >= 0.0 ? 1.0 : -1.0) * ct;
            } else {
                nux = stt * (ux * uz * cp - uy * sp) / tn + ux * ct;
                nuy = stt * (uy * uz * cp + ux * sp) / tn + uy * ct;
                nuz = -stt * cp * tn + uz * ct;
            }
            const double nrm = sqrt(nux * nux + nuy * nuy + nuz * nuz);
            st->ux = nux / nrm; st->uy = nuy / nrm; st->uz = nuz / nrm;
            /* Russian roulette on the integer weight */
            if (st->w < w_th) {
                if ((r[3] >> 8) < T_m) {
                    const int64_t m = (int64_t)P->roulette_m;
                    S->sums->ich[ORC_RR] -= (m - 1) * st->w;
                    me->RR -= (m - 1) * st->w;
                    st->w *= m;
                } else {
                    S->sums->ich[ORC_RR] += st->w;
                    me->RR += st->w;
                    event = EV_DEAD_ROULETTE;
                    done = 1;
                }
            }
            st->tau = -log(u_open_closed(r[2]));
        }
    }

    if (!done) {
        const double path = st->l_void + st->l_solid;
        if (st->steps >= P->max_steps || (P->path_cap > 0.0 && path > P->path_cap)) {
            S->sums->ich[ORC_LOST] += st->w;
            me->lost += st->w;
            event = EV_LOST;
        }
    }
    if (gap_out) *gap_out = gap;
    if (rec) {
        rec->event = event;
        rec->tie_gap = gap;
    }
    return event;
}

/* Walk one photon from launch to termination. */
static void walk(const orc_problem *P, uint64_t photon, orc_sink *S)
{
    orc_state st;
    launch(P, photon, &st);
    orc_photon me;
    memset(&me, 0, sizeof me);
    me.min_gap = INFINITY;
    int event;
    double visit = 0.0;   /* deposited during the current stay in a voxel */
    for (;;) {
        double gap;
        const double w0 = (double)st.w, path0 = st.l_void + st.l_solid;
        event = step(P, photon, &st, S, &me, &gap);
        if (gap < me.min_gap) me.min_gap = gap;
        visit += w0 * ((st.l_void + st.l_solid) - path0);
        if (visit > me.max_visit) me.max_visit = visit;
        if (event == EV_FACE_X || event == EV_FACE_Y || event == EV_FACE_Z) visit = 0.0;
        if (terminal(event)) break;
    }
    S->sums->ich[ORC_STEPS] += (int64_t)st.steps;
    S->sums->ich[ORC_INTERACTIONS] += (int64_t)st.k;
    S->sums->dch[ORC_PATH_TOTAL] += st.l_void + st.l_solid;
    S->sums->dch[ORC_PATH_SOLID] += st.l_solid;
    S->sums->dch[ORC_PATH_VOID] += st.l_void;
    if (S->summary) {
        me.w_final = st.w;
        me.steps = st.steps;
        me.interactions = st.k;
        me.path_void = st.l_void;
        me.path_solid = st.l_solid;
        me.fate = event;
        *S->summary = me;
    }
}

/* ------------------------------------------------------------------------- */
/* Multi-threaded driver over a photon-id range.                             */
/* ------------------------------------------------------------------------- */
typedef struct {
    const orc_problem *P;
    uint64_t begin, end;      /* photon ids */
    int nbatch;
    double *fluence;          /* private [nbatch][nvox] or NULL */
    double *grad;             /* private [nbatch][3][2][nz] or NULL */
    double *depth;            /* private [nbatch][2][nz] or NULL */
    orc_sums *sums;           /* private [nbatch] */
} orc_task;

static void *run_task(void *arg)
{
    orc_task *T = (orc_task *)arg;
    const int64_t nvox = (int64_t)T->P->nx * T->P->ny * T->P->nz;
    for (uint64_t p = T->begin; p < T->end; ++p) {
        const int b = (int)(p % (uint64_t)T->nbatch);
        orc_sink S;
        memset(&S, 0, sizeof S);
        S.fluence = T->fluence ? T->fluence + (int64_t)b * nvox : NULL;
        S.grad = T->grad ? T->grad + (int64_t)b * 6 * T->P->nz : NULL;
        S.depth = T->depth ? T->depth + (int64_t)b * 2 * T->P->nz : NULL;
        S.sums = &T->sums[b];
        walk(T->P, p, &S);
    }
    return NULL;
}

static int valid(const orc_problem *P)
{
    if (!P || !P->mask || P->nx <= 0 || P->ny <= 0 || P->nz <= 0) return 0;
    if (!(P->mu_s >= 0.0) || !(P->mu_a >= 0.0) || !(fabs(P->g) < 1.0)) return 0;
    if (P->roulette_m < 2 || P->max_steps == 0) return 0;
    if (P->boundary == 0) {
        /* the plain model has no index, mirrors or gate */
        if (P->lateral != 0 || P->n_solid != 1.0 || !isinf(P->gate)) return 0;
    } else if (P->boundary == 1) {
        if (P->lateral != 0 && P->lateral != 1) return 0;
        if (!(P->n_solid >= 1.0) || !isfinite(P->n_solid)) return 0;
        if (!(P->gate > 0.0)) return 0;
    } else {
        return 0;
    }
    /* a surviving photon's weight w_th * m must not exceed the launch weight, so that
     * every weight stays <= 2^31 and w * S_q fits in 64 bits */
    if (!(P->w_roulette >= 0.0) || floor(P->w_roulette * ORC_W1) * (double)P->roulette_m > ORC_W1) return 0;
    return 1;
}

/*
 * Run photons [begin, begin + n) split over nthreads threads.  Each photon
 * belongs to batch (id mod nbatch); every output is per batch:
 *   fluence [nbatch][nz][ny][nx]  (weight x voxel, weight in units of 2^-31) or NULL
 *   grad    [nbatch][3][2][nz]    LR bins (param mu_s, mu_a, g; phase solid, pore) or NULL
 *   depth   [nbatch][2][nz]       phase-resolved depth sums of the fluence or NULL
 *   ich     [nbatch][ORC_NI], dch [nbatch][ORC_ND]
 * Outputs are added to (the caller zeroes them).  Returns 0, or -1 on bad input.
 */
int orc_run(const orc_problem *P, uint64_t begin, uint64_t n, int nthreads, int nbatch,
            double *fluence, double *grad, double *depth, int64_t *ich, double *dch)
{
    if (!valid(P) || nbatch < 1 || !ich || !dch) return -1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > n) nthreads = (int)(n ? n : 1);
    const int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    orc_task *tasks = (orc_task *)calloc((size_t)nthreads, sizeof(orc_task));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!tasks || !th) { free(tasks); free(th); return -1; }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        orc_task *T = &tasks[t];
        T->P = P;
        T->begin = begin + n * (uint64_t)t / (uint64_t)nthreads;
        T->end = begin + n * (uint64_t)(t + 1) / (uint64_t)nthreads;
        T->nbatch = nbatch;
        T->sums = (orc_sums *)calloc((size_t)nbatch, sizeof(orc_sums));
        if (fluence) T->fluence = (double *)calloc((size_t)(nbatch * nvox), sizeof(double));
        if (grad) T->grad = (double *)calloc((size_t)nbatch * 6 * P->nz, sizeof(double));
        if (depth) T->depth = (double *)calloc((size_t)nbatch * 2 * P->nz, sizeof(double));
        if (!T->sums || (fluence && !T->fluence) || (grad && !T->grad) || (depth && !T->depth)) rc = -1;
    }
    if (rc == 0) {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_task, &tasks[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
        /* combine thread-private results in thread order */
        for (int t = 0; t < nthreads; ++t) {
            orc_task *T = &tasks[t];
            for (int b = 0; b < nbatch; ++b) {
                for (int c = 0; c < ORC_NI; ++c) ich[b * ORC_NI + c] += T->sums[b].ich[c];
                for (int c = 0; c < ORC_ND; ++c) dch[b * ORC_ND + c] += T->sums[b].dch[c];
            }
            if (fluence)
                for (int64_t i = 0; i < nbatch * nvox; ++i) fluence[i] += T->fluence[i];
            if (grad)
                for (int64_t i = 0; i < (int64_t)nbatch * 6 * P->nz; ++i) grad[i] += T->grad[i];
            if (depth)
                for (int64_t i = 0; i < (int64_t)nbatch * 2 * P->nz; ++i) depth[i] += T->depth[i];
        }
    }
    for (int t = 0; t < nthreads; ++t) {
        free(tasks[t].sums);
        free(tasks[t].fluence);
        free(tasks[t].grad);
        free(tasks[t].depth);
    }
    free(tasks);
    free(th);
    return rc;
}

/*
 * Trace the given photons one by one: the first max_rec steps of each
 * (out[n][max_rec], unused records keep event = -1 as set by the caller) and
 * a per-photon summary (summary[n]).
 */
int orc_trace(const orc_problem *P, const uint64_t *ids, int32_t n, int32_t max_rec,
              orc_rec *out, orc_photon *summary)
{
    if (!valid(P) || !ids || n < 0 || max_rec < 0) return -1;
    for (int32_t i = 0; i < n; ++i) {
        orc_sums sums;
        memset(&sums, 0, sizeof sums);
        orc_sink S;
        memset(&S, 0, sizeof S);
        S.trace = out ? out + (int64_t)i * max_rec : NULL;
        S.max_rec = max_rec;
        S.summary = summary ? &summary[i] : NULL;
        S.sums = &sums;
        walk(P, ids[i], &S);
    }
    return 0;
}

/*
 * One step of photon `photon` from the state *st (updated in place); returns the
 * event and the step's tie gap.  Lets a test restart the reference walk from any
 * state another implementation reports.  Tallies of the step are discarded.
 */
int orc_step(const orc_problem *P, uint64_t photon, orc_state *st, double *gap)
{
    if (!valid(P) || !st) return -1;
    orc_sums sums;
    memset(&sums, 0, sizeof sums);
    orc_sink S;
    memset(&S, 0, sizeof S);
    S.sums = &sums;
    orc_photon me;
    memset(&me, 0, sizeof me);
    return step(P, photon, st, &S, &me, gap);
}

int orc_sizeof_state(void) { return (int)sizeof(orc_state); }
int orc_sizeof_rec(void) { return (int)sizeof(orc_rec); }
int orc_sizeof_photon(void) { return (int)sizeof(orc_photon); }
int orc_sizeof_problem(void) { return (int)sizeof(orc_problem); }
