/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the growing-tissue D2Q9 lattice
 * Boltzmann method of arXiv 2303.02210.  TEST INFRASTRUCTURE ONLY (see the
 * header): the product path never calls this code.
 *
 * The update is the paper's Appendix A algorithm, steps 1-7, applied to every
 * site of the live window, followed by the front heights, the width w(t) and
 * the rear-wall rule of Appendix A's last paragraph.  The paper works on the
 * triangular D2Q7 lattice; this oracle uses the square D2Q9 lattice with the
 * textbook weights (4/9, 1/9, 1/36) and sound speed c_s^2 = 1/3, so the
 * steady state of Eq. 3 reads w_i rho (1 + 3 e.u* + 9/2 (e.u*)^2 - 3/2 |u*|^2)
 * and the zero-sum noise of Eq. 4 subtracts the mean over 9 directions.
 *
 * Direction numbering: 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
 * Reverse pairs: 1<->3, 2<->4, 5<->7, 6<->8.  x is periodic (columns), y is
 * the growth axis (rows); the rear wall sits half a lattice unit below the
 * first live row.
 *
 * The paper's own lattice, D2Q7 (Sec. II), is the second option: six unit
 * directions at multiples of pi/3 plus rest, weights 1/2 (rest) and 1/12,
 * c_s^2 = 1/4, so Eq. 3 reads w_i rho (1 + 4 e.u* + 8 (e.u*)^2 - 2 |u*|^2) and
 * Eq. 4 subtracts the mean over 7 directions.  Its rows are horizontal with
 * odd rows shifted by half a unit (see the header).
 *
 * Compile with -ffp-contract=off: every product and sum below is rounded on
 * its own, in the order written.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------- */
/* Lattice                                                                   */
/* ----------------------------------------------------------------------- */
static const int32_t CX[9]  = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int32_t CY[9]  = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int32_t OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

static double weight(int i)
{
    if (i == 0) return 4.0 / 9.0;
    if (i <= 4) return 1.0 / 9.0;
    return 1.0 / 36.0;
}

/* D2Q7: 0 rest, 1 E, 2 NE, 3 NW, 4 W, 5 SW, 6 SE */
static const int32_t OPP7[7] = {0, 4, 5, 6, 1, 2, 3};
static const double SQRT3_2 = 0.86602540378443864676;   /* sin(pi/3) */

static double weight7(int i)
{
    return (i == 0) ? 1.0 / 2.0 : 1.0 / 12.0;
}

int orc_q(const orc_params *p)
{
    return p->lattice == ORC_LATTICE_D2Q7 ? 7 : 9;
}


void orc_lattice(int32_t cx[9], int32_t cy[9], int32_t opp[9], double w[9])
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = OPP[i];
        w[i] = weight(i);
    }
}

/* ----------------------------------------------------------------------- */
/* Philox4x32-10, from its definition in Salmon et al., SC'11: each round    */
/* multiplies counter words 0 and 2 by two fixed odd constants, swaps the    */
/* halves and xors in the key; the key is bumped by two Weyl constants       */
/* between rounds.                                                           */
/* ----------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random streams: the fourth counter word is 4*stream + call. */
enum { STREAM_NOISE = 0, STREAM_INIT = 1, STREAM_DIVISION = 2, STREAM_SELECTION = 4 };

static double u24(uint32_t k24)
{
    /* (k + 1/2) 2^-24: exact in double, strictly inside (0, 1) */
    return ((double)k24 + 0.5) * (1.0 / 16777216.0);
}

void orc_noise_bits(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                    int64_t y_abs, uint32_t k_out[9])
{
    uint32_t key[2] = {seed, replica};
    uint32_t ctr[4] = {(uint32_t)x, (uint32_t)y_abs, (uint32_t)t, 4u * STREAM_NOISE + 0u};
    uint32_t a[4], b[4];
    orc_philox4x32_10(ctr, key, a);
    ctr[3] = 4u * STREAM_NOISE + 1u;
    orc_philox4x32_10(ctr, key, b);
    /* eight draws from the top 24 bits of the eight words ... */
    for (int i = 0; i < 4; ++i) {
        k_out[i] = a[i] >> 8;
        k_out[4 + i] = b[i] >> 8;
    }
    /* ... and the ninth from the low bytes of the first three words */
    k_out[8] = ((a[0] & 0xFFu) << 16) | ((a[1] & 0xFFu) << 8) | (a[2] & 0xFFu);
}

void orc_noise_uniforms(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                        int64_t y_abs, double u_out[9])
{
    uint32_t k[9];
    orc_noise_bits(seed, replica, t, x, y_abs, k);
    for (int i = 0; i < 9; ++i) u_out[i] = u24(k[i]);
}

double orc_init_uniform(uint32_t seed, uint32_t replica, int32_t x, int64_t y_abs)
{
    uint32_t key[2] = {seed, replica};
    uint32_t ctr[4] = {(uint32_t)x, (uint32_t)y_abs, 0u, 4u * STREAM_INIT + 0u};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return u24(r[0] >> 8);
}

void orc_division_draws(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                        int64_t y_abs, double *U_out, uint64_t *axes_out)
{
    uint32_t key[2] = {seed, replica};
    uint32_t ctr[4] = {(uint32_t)x, (uint32_t)y_abs, (uint32_t)t, 4u * STREAM_DIVISION + 0u};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    /* 26 + 26 bits of the first two words; n + 1/2 is exact in double */
    uint64_t n = ((uint64_t)(r[0] >> 6) << 26) | (uint64_t)(r[1] >> 6);
    *U_out = ((double)n + 0.5) * (1.0 / 4503599627370496.0);
    *axes_out = ((uint64_t)r[3] << 32) | (uint64_t)r[2];
}

/* The selection procedure of Sec. II (ORC_DIVISION_SELECTION): attempt a of
 * step t is one Philox call with the attempt number in the first two counter
 * words. */
void orc_selection_draws(uint32_t seed, uint32_t replica, int64_t t, int64_t a,
                         double *U_site, double *U_acc, uint32_t *axis_bits)
{
    uint32_t key[2] = {seed, replica};
    uint32_t ctr[4] = {(uint32_t)a, (uint32_t)((uint64_t)a >> 32), (uint32_t)t,
                       4u * STREAM_SELECTION + 0u};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    uint64_t n = ((uint64_t)(r[0] >> 6) << 26) | (uint64_t)(r[1] >> 6);
    *U_site = ((double)n + 0.5) * (1.0 / 4503599627370496.0);
    *U_acc = ((double)r[2] + 0.5) * (1.0 / 4294967296.0);
    *axis_bits = r[3];
}

double orc_selection_round_uniform(uint32_t seed, uint32_t replica, int64_t t)
{
    uint32_t key[2] = {seed, replica};
    uint32_t ctr[4] = {0u, 0u, (uint32_t)t, 4u * STREAM_SELECTION + 1u};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    return ((double)r[0] + 0.5) * (1.0 / 4294967296.0);
}

/* ----------------------------------------------------------------------- */
/* Poisson counts for the division laws                                      */
/* ----------------------------------------------------------------------- */
double orc_exp_neg(double lam)
{
    /* e^-lam = (e^-m)^16 with m = lam / 16 <= 1/2: the Taylor series of e^-m
     * through the m^17 term, by Horner's rule
     *   e^-m = 1 - (m/1)(1 - (m/2)(1 - (m/3)(... (1 - m/17)))),
     * then squared four times */
    double m = lam * 0.0625;
    double r = 1.0;
    for (int n = 17; n >= 1; --n) {
        double q = m / (double)n;
        r = 1.0 - q * r;
    }
    for (int i = 0; i < 4; ++i) r = r * r;
    return r;
}

int orc_poisson_k(double U, double lam)
{
    /* smallest k with U <= P(0) + ... + P(k), P(k) = e^-lam lam^k / k! */
    double pk = orc_exp_neg(lam);
    double cdf = pk;
    int k = 0;
    while (U > cdf && k < 32) {
        k = k + 1;
        pk = pk * lam / (double)k;
        cdf = cdf + pk;
    }
    return k;
}

/* ----------------------------------------------------------------------- */
/* Eq. 3 on D2Q9                                                             */
/* ----------------------------------------------------------------------- */
void orc_fss(double rho, double ux, double uy, double out[9])
{
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        /* e_i . u*, written as a sum of the signed velocity components */
        double cu;
        if (CX[i] == 0 && CY[i] == 0) cu = 0.0;
        else if (CY[i] == 0) cu = (CX[i] > 0) ? ux : -ux;
        else if (CX[i] == 0) cu = (CY[i] > 0) ? uy : -uy;
        else cu = ((CX[i] > 0) ? ux : -ux) + ((CY[i] > 0) ? uy : -uy);
        double wr = weight(i) * rho;
        out[i] = wr * (((1.0 + 3.0 * cu) + 4.5 * (cu * cu)) - 1.5 * usq);
    }
}

/* Eq. 3 on D2Q7.  e_i . u* from the components: a = ux/2, b = sqrt(3)/2 uy;
 * E: ux, NE: a + b, NW: b - a, and the reverse directions their negatives. */
void orc_fss7(double rho, double ux, double uy, double out[7])
{
    double usq = ux * ux + uy * uy;
    double a = 0.5 * ux;
    double b = SQRT3_2 * uy;
    double cu[7];
    cu[0] = 0.0;
    cu[1] = ux;
    cu[2] = a + b;
    cu[3] = b - a;
    cu[4] = -cu[1];
    cu[5] = -cu[2];
    cu[6] = -cu[3];
    for (int i = 0; i < 7; ++i) {
        double wr = weight7(i) * rho;
        out[i] = wr * (((1.0 + 4.0 * cu[i]) + 8.0 * (cu[i] * cu[i])) - 2.0 * usq);
    }
}

/* Eq. 3 at rest on either lattice: w_i rho */
static void fss_rest(const orc_params *p, double rho, double out[9])
{
    if (p->lattice == ORC_LATTICE_D2Q7) orc_fss7(rho, 0.0, 0.0, out);
    else orc_fss(rho, 0.0, 0.0, out);
}

/* ----------------------------------------------------------------------- */
/* Window storage                                                            */
/* ----------------------------------------------------------------------- */
struct orc_state {
    orc_params p;
    double    *f;      /* [9][H][L]; window row j holds absolute row y_wall + j */
    double    *fn;     /* next populations                                       */
    int32_t   *h;      /* [L] front heights (absolute rows)                      */
    int64_t    t;
    int64_t    y_wall;
    int64_t    h_hi;
    double     mass, src_total, fix_total, retired, hbar, W;
    uint32_t   status;
    double     lam;        /* division laws: lam of the next step              */
    int64_t    divisions;  /* cumulative divisions                             */
    int32_t   *divmap;     /* [H][L] divisions per window site since cleared   */
    int32_t   *sel;        /* selection procedure: the last step's divisions,
                              [H][L][axes] (NULL under the per-site form)    */
};

static size_t idx(const orc_params *p, int i, int32_t j, int32_t x)
{
    return ((size_t)i * (size_t)p->H + (size_t)j) * (size_t)p->L + (size_t)x;
}

static int params_valid(const orc_params *p)
{
    if (p->L < 1 || p->H < 2) return 0;
    if (!(p->tau > 0.5)) return 0;
    if (!(p->rho_c > 0.0)) return 0;
    if (!(p->sigma >= 0.0) || !(p->growth_rate >= 0.0)) return 0;
    if (!(p->mu >= 0.0 && p->mu <= 1.0)) return 0;
    if (!(p->init_amp >= 0.0 && p->init_amp < 1.0)) return 0;
    if (!(p->rho_init >= 0.0)) return 0;
    if (p->init_rows < 0 || p->init_rows > p->H) return 0;
    if (p->growth < ORC_GROWTH_NONE || p->growth > ORC_GROWTH_DIVISION_DENSITY) return 0;
    if ((p->growth == ORC_GROWTH_DIVISION || p->growth == ORC_GROWTH_DIVISION_DENSITY) &&
        !(p->rho_cell > 0.0))
        return 0;
    if (p->growth == ORC_GROWTH_DIVISION_DENSITY && !(p->rho0 > p->rho_c)) return 0;
    if (p->region < ORC_REGION_ALL || p->region > ORC_REGION_REAR_BAND) return 0;
    if (p->region != ORC_REGION_ALL && p->region_width < 0) return 0;
    if (p->ybc < ORC_Y_WALL_FIXED || p->ybc > ORC_Y_PERIODIC) return 0;
    if (p->ybc == ORC_Y_WALL_FOLLOW && (p->wall_min_gap < 0 || !(p->wall_w_factor >= 0.0))) return 0;
    if (p->lattice != ORC_LATTICE_D2Q9 && p->lattice != ORC_LATTICE_D2Q7) return 0;
    /* a periodic D2Q7 column of rows must keep the row parity across the seam */
    if (p->lattice == ORC_LATTICE_D2Q7 && p->ybc == ORC_Y_PERIODIC && p->H % 2 != 0) return 0;
    return 1;
}

/* ----------------------------------------------------------------------- */
/* Step 1: streaming, pulled to the receiving site                           */
/* ----------------------------------------------------------------------- */
/* D2Q7 pull sources: the upstream neighbour of (x, y) along -e_i.  With odd
 * rows shifted by +1/2, the neighbour half a unit to the left in the row
 * below or above is at column x - 1 + par, and half a unit to the right at
 * x + par, par = y mod 2.  Row offsets and those column choices: */
static void pull_source7(int i, int par, int32_t *dx, int32_t *dy)
{
    switch (i) {
    case 1: *dx = -1; *dy = 0; break;            /* E from the left            */
    case 2: *dx = par - 1; *dy = -1; break;      /* NE from below-left         */
    case 3: *dx = par; *dy = -1; break;          /* NW from below-right        */
    case 4: *dx = 1; *dy = 0; break;             /* W from the right           */
    case 5: *dx = par; *dy = 1; break;           /* SW from above-right        */
    case 6: *dx = par - 1; *dy = 1; break;       /* SE from above-left         */
    default: *dx = 0; *dy = 0; break;            /* rest                       */
    }
}

static void pull_site7(const orc_params *p, const double *f, int32_t x, int32_t j, int64_t y_abs,
                       double fstar[7])
{
    const int par = (int)(y_abs & 1);
    for (int i = 0; i < 7; ++i) {
        int32_t dx, dy;
        pull_source7(i, par, &dx, &dy);
        int32_t xs = ((x + dx) % p->L + p->L) % p->L;   /* periodic in x */
        int32_t js = j + dy;
        if (p->ybc == ORC_Y_PERIODIC) {
            js = (js % p->H + p->H) % p->H;
            fstar[i] = f[idx(p, i, js, xs)];
        } else if (js < 0) {
            /* rear wall: what left this site towards it comes back reversed */
            fstar[i] = f[idx(p, OPP7[i], j, x)];
        } else if (js >= p->H) {
            fstar[i] = 0.0;
        } else {
            fstar[i] = f[idx(p, i, js, xs)];
        }
    }
}

void orc_pull_site(const orc_params *p, const double *f, int32_t x, int32_t j, double fstar[9])
{
    orc_pull_site_abs(p, f, x, j, j, fstar);
}

void orc_pull_site_abs(const orc_params *p, const double *f, int32_t x, int32_t j, int64_t y_abs,
                       double fstar[9])
{
    if (p->lattice == ORC_LATTICE_D2Q7) {
        pull_site7(p, f, x, j, y_abs, fstar);
        return;
    }
    for (int i = 0; i < 9; ++i) {
        int32_t xs = ((x - CX[i]) % p->L + p->L) % p->L;   /* periodic in x */
        int32_t js = j - CY[i];
        if (p->ybc == ORC_Y_PERIODIC) {
            js = (js % p->H + p->H) % p->H;
            fstar[i] = f[idx(p, i, js, xs)];
        } else if (js < 0) {
            /* rear wall, half a unit below row 0: what left this site
             * towards the wall comes straight back (bounce-back) */
            fstar[i] = f[idx(p, OPP[i], j, x)];
        } else if (js >= p->H) {
            /* nothing lies beyond the top of the window */
            fstar[i] = 0.0;
        } else {
            fstar[i] = f[idx(p, i, js, xs)];
        }
    }
}

static int in_region(const orc_params *p, int64_t y_abs, int32_t h_prev_x, int64_t y_wall)
{
    if (p->region == ORC_REGION_FRONT_BAND)
        return y_abs >= (int64_t)h_prev_x - (int64_t)p->region_width;
    if (p->region == ORC_REGION_REAR_BAND)
        return y_abs < y_wall + (int64_t)p->region_width;
    return 1;
}

static double sum9(const double v[9])
{
    double s = v[0];
    for (int i = 1; i < 9; ++i) s = s + v[i];
    return s;
}

static double sum7(const double v[7])
{
    double s = v[0];
    for (int i = 1; i < 7; ++i) s = s + v[i];
    return s;
}

/* density of a site's populations on either lattice, summed in index order */
static double sumq(const orc_params *p, const double *v)
{
    return p->lattice == ORC_LATTICE_D2Q7 ? sum7(v) : sum9(v);
}

static int division_law(const orc_params *p)
{
    return p->growth == ORC_GROWTH_DIVISION || p->growth == ORC_GROWTH_DIVISION_DENSITY;
}

/* Division laws: whether a tissue site of density rho may divide, and its
 * acceptance probability q (1 for the uniform draw; Eq. 5 for the density
 * law: 1 - rho / rho0 above rho_c, none otherwise). */
static int division_eligible(const orc_params *p, double rho, int in_reg, double *q)
{
    *q = 1.0;
    if (!division_law(p) || !in_reg) return 0;
    if (p->growth == ORC_GROWTH_DIVISION_DENSITY) {
        *q = 1.0 - rho / p->rho0;
        return rho > p->rho_c && *q > 0.0;
    }
    return 1;
}

/* The site's weight in the normaliser of the next step's rate: 1 per
 * eligible site, or its acceptance probability in units of 2^-24 (integers,
 * so that the sum does not depend on its order). */
static int64_t division_weight(const orc_params *p, double q)
{
    return p->growth == ORC_GROWTH_DIVISION ? 1 : (int64_t)(q * 16777216.0);
}

/* A site's density in units of 2^-24, truncated (the mass m_tot of the
 * division laws is summed in these integers). */
static int64_t mass_fx(double rho)
{
    return (int64_t)(rho * 16777216.0);
}

/* Expected divisions per unit weight: n_s = g m_tot / rho_cell divisions
 * (Sec. II) shared by the total weight of the eligible sites. */
static double division_lam(const orc_params *p, int64_t mfx, int64_t wsum)
{
    if (!division_law(p) || wsum <= 0) return 0.0;
    double m_tot = (double)mfx * (1.0 / 16777216.0);
    double ns = p->growth_rate * m_tot / p->rho_cell;
    double wt = (p->growth == ORC_GROWTH_DIVISION) ? (double)wsum
                                                   : (double)wsum * (1.0 / 16777216.0);
    return ns / wt;
}

/* ----------------------------------------------------------------------- */
/* Steps 2-7 at one site of the D2Q7 lattice                                 */
/* ----------------------------------------------------------------------- */
static int update_site7(const orc_params *p, const double fstar_in[7], int64_t t, int32_t x,
                        int64_t y_abs, int32_t h_prev_x, int64_t y_wall, int force, double lam,
                        const int32_t *given, double out[7], double *S_out, double *dfix_out,
                        int32_t *ndiv_out, int64_t *wfx_out)
{
    double fs[7];
    for (int i = 0; i < 7; ++i) fs[i] = fstar_in[i];
    *S_out = 0.0;
    *dfix_out = 0.0;
    *ndiv_out = 0;
    *wfx_out = 0;

    /* step 2: density and momentum (Eq. 1) with e_i = (cos, sin)((i-1) pi/3):
     * j_x = (f1 - f4) + (f2 - f3 - f5 + f6)/2, j_y = sqrt(3)/2 (f2 + f3 - f5 - f6) */
    double rho_star = sum7(fs);
    double jx = (fs[1] - fs[4]) + 0.5 * (((fs[2] - fs[3]) + fs[6]) - fs[5]);
    double jy = SQRT3_2 * (((fs[2] + fs[3]) - fs[5]) - fs[6]);

    int tissue = (force < 0) ? (rho_star >= p->rho_c) : (force > 0);
    if (!tissue) {
        /* step 5, second case: reverse every direction (1-4, 2-5, 3-6) */
        for (int i = 0; i < 7; ++i) out[i] = fs[OPP7[i]];
        return 0;
    }

    /* step 3: the expected injection shared by the six moving directions */
    double S = 0.0;
    if (p->growth == ORC_GROWTH_BULK && in_region(p, y_abs, h_prev_x, y_wall))
        S = p->growth_rate * rho_star;
    double s6 = S / 6.0;
    for (int i = 1; i < 7; ++i) fs[i] = fs[i] + s6;
    /* step 3, division laws: as on D2Q9, with three axes; each division's
     * axis is one base-3 digit of the 64 random bits */
    double q;
    if (given) {
        /* the selection procedure chose this site's divisions per axis */
        int k = given[0] + given[1] + given[2];
        double half = p->rho_cell * 0.5;
        for (int a = 0; a < 3; ++a) {
            double amount = (double)given[a] * half;
            fs[a + 1] = fs[a + 1] + amount;
            fs[OPP7[a + 1]] = fs[OPP7[a + 1]] + amount;
        }
        S = (double)k * p->rho_cell;
        *ndiv_out = k;
    } else if (division_eligible(p, rho_star, in_region(p, y_abs, h_prev_x, y_wall), &q)) {
        *wfx_out = division_weight(p, q);
        double l = lam * q;
        if (l > 8.0) l = 8.0;
        if (l > 0.0) {
            double U;
            uint64_t axes;
            orc_division_draws(p->seed, p->replica, t, x, y_abs, &U, &axes);
            int k = orc_poisson_k(U, l);
            int count[3] = {0, 0, 0};
            uint64_t digits = axes;
            for (int d = 0; d < k; ++d) {
                count[digits % 3u] += 1;
                digits = digits / 3u;
            }
            double half = p->rho_cell * 0.5;
            for (int a = 0; a < 3; ++a) {
                /* axis a joins direction a + 1 and its reverse a + 4 */
                double amount = (double)count[a] * half;
                fs[a + 1] = fs[a + 1] + amount;
                fs[OPP7[a + 1]] = fs[OPP7[a + 1]] + amount;
            }
            S = (double)k * p->rho_cell;
            *ndiv_out = k;
        }
    }
    double rho = rho_star + S;
    *S_out = S;

    /* step 4 and step 5, first case */
    double kmu = 1.0 - p->mu;
    double ux = (jx / rho) * kmu;
    double uy = (jy / rho) * kmu;
    double fss[7];
    orc_fss7(rho, ux, uy, fss);
    double omega = 1.0 / p->tau;
    for (int i = 0; i < 7; ++i) out[i] = fs[i] - omega * (fs[i] - fss[i]);

    /* step 6: Eq. 4 over seven directions (the first seven noise draws) */
    if (rho > p->rho_c && p->sigma > 0.0) {
        double u[9], eta[7];
        orc_noise_uniforms(p->seed, p->replica, t, x, y_abs, u);
        for (int i = 0; i < 7; ++i) eta[i] = p->sigma * (2.0 * u[i] - 1.0);
        double m = sum7(eta) / 7.0;
        for (int i = 0; i < 7; ++i) out[i] = out[i] + (eta[i] - m);
    }

    /* step 7, as on D2Q9 with the D2Q7 reverse directions */
    int any_negative = 0;
    for (int i = 0; i < 7; ++i) if (out[i] < 0.0) any_negative = 1;
    if (any_negative) {
        double before = sum7(out);
        if (out[0] < 0.0) {
            double rho_pre = sum7(out);
            out[0] = 0.0;
            double rest = sum7(out);
            if (rest > 0.0) {
                double r = rho_pre / rest;
                for (int i = 0; i < 7; ++i) out[i] = out[i] * r;
            }
        }
        for (int i = 1; i < 7; ++i) {
            if (out[i] < 0.0) {
                out[OPP7[i]] = out[OPP7[i]] + (-out[i]);
                out[i] = 0.0;
            }
        }
        *dfix_out = sum7(out) - before;
    }
    return 1;
}

/* ----------------------------------------------------------------------- */
/* Steps 2-7 at one site                                                     */
/* ----------------------------------------------------------------------- */
/* given: the selection procedure's divisions of this site per axis (D2Q9:
 * 4, D2Q7: 3 counts), or NULL for the per-site Poisson draw */
static int update_site(const orc_params *p, const double fstar_in[9], int64_t t,
                       int32_t x, int64_t y_abs, int32_t h_prev_x, int64_t y_wall,
                       int force, double lam, const int32_t *given, double out[9],
                       double *S_out, double *dfix_out, int32_t *ndiv_out, int64_t *wfx_out)
{
    if (p->lattice == ORC_LATTICE_D2Q7)
        return update_site7(p, fstar_in, t, x, y_abs, h_prev_x, y_wall, force, lam, given, out,
                            S_out, dfix_out, ndiv_out, wfx_out);
    double fs[9];
    for (int i = 0; i < 9; ++i) fs[i] = fstar_in[i];
    *S_out = 0.0;
    *dfix_out = 0.0;
    *ndiv_out = 0;
    *wfx_out = 0;

    /* step 2: density and momentum of the streamed populations (Eq. 1) */
    double rho_star = sum9(fs);
    double jx = ((((fs[1] - fs[3]) + fs[5]) - fs[6]) - fs[7]) + fs[8];
    double jy = ((((fs[2] - fs[4]) + fs[5]) + fs[6]) - fs[7]) - fs[8];

    /* step 5's test, taken on the streamed density: tissue or void */
    int tissue = (force < 0) ? (rho_star >= p->rho_c) : (force > 0);

    if (!tissue) {
        /* step 5, second case: reverse every direction (bounce-back front) */
        for (int i = 0; i < 9; ++i) out[i] = fs[OPP[i]];
        return 0;
    }

    /* step 3: mass from proliferation, in expectation: S = g rho* shared
     * equally by the eight moving directions (pairs of opposite directions
     * receive equal amounts, so no momentum is added) */
    double S = 0.0;
    if (p->growth == ORC_GROWTH_BULK && in_region(p, y_abs, h_prev_x, y_wall))
        S = p->growth_rate * rho_star;
    double s8 = S * 0.125;
    for (int i = 1; i < 9; ++i) fs[i] = fs[i] + s8;
    /* step 3, division laws: the paper injects rho_cell / 2 into both
     * directions of a randomly oriented axis at n_s sites drawn with
     * replacement (accepted with probability q under Eq. 5).  Drawing each
     * site's number of divisions from a Poisson law with mean lam q, site by
     * site and independently, gives the same expected divisions per site;
     * lam spreads n_s over the eligible sites' total weight. */
    double q;
    static const int AXIS[4] = {1, 2, 5, 6};
    if (given) {
        /* the selection procedure chose this site's divisions per axis */
        int k = given[0] + given[1] + given[2] + given[3];
        double half = p->rho_cell * 0.5;
        for (int a = 0; a < 4; ++a) {
            double amount = (double)given[a] * half;
            fs[AXIS[a]] = fs[AXIS[a]] + amount;
            fs[OPP[AXIS[a]]] = fs[OPP[AXIS[a]]] + amount;
        }
        S = (double)k * p->rho_cell;
        *ndiv_out = k;
    } else if (division_eligible(p, rho_star, in_region(p, y_abs, h_prev_x, y_wall), &q)) {
        *wfx_out = division_weight(p, q);
        double l = lam * q;
        if (l > 8.0) l = 8.0;
        if (l > 0.0) {
            double U;
            uint64_t axes;
            orc_division_draws(p->seed, p->replica, t, x, y_abs, &U, &axes);
            int k = orc_poisson_k(U, l);
            /* two bits per division choose the axis: 1-3, 2-4, 5-7 or 6-8 */
            int count[4] = {0, 0, 0, 0};
            for (int d = 0; d < k; ++d) count[(axes >> (2 * d)) & 3u] += 1;
            double half = p->rho_cell * 0.5;
            for (int a = 0; a < 4; ++a) {
                double amount = (double)count[a] * half;
                fs[AXIS[a]] = fs[AXIS[a]] + amount;
                fs[OPP[AXIS[a]]] = fs[OPP[AXIS[a]]] + amount;
            }
            S = (double)k * p->rho_cell;
            *ndiv_out = k;
        }
    }
    double rho = rho_star + S;
    *S_out = S;

    /* step 4: u* = (1 - mu) u and the steady state of Eq. 3 */
    double kmu = 1.0 - p->mu;
    double ux = (jx / rho) * kmu;
    double uy = (jy / rho) * kmu;
    double fss[9];
    orc_fss(rho, ux, uy, fss);

    /* step 5, first case: relax towards the steady state (Eq. 2) */
    double omega = 1.0 / p->tau;
    for (int i = 0; i < 9; ++i) out[i] = fs[i] - omega * (fs[i] - fss[i]);

    /* step 6: zero-sum uniform noise of Eq. 4, only where rho > rho_c */
    if (rho > p->rho_c && p->sigma > 0.0) {
        double u[9], eta[9];
        orc_noise_uniforms(p->seed, p->replica, t, x, y_abs, u);
        for (int i = 0; i < 9; ++i) eta[i] = p->sigma * (2.0 * u[i] - 1.0);
        double m = sum9(eta) / 9.0;
        for (int i = 0; i < 9; ++i) out[i] = out[i] + (eta[i] - m);
    }

    /* step 7: remove negative populations */
    int any_negative = 0;
    for (int i = 0; i < 9; ++i) if (out[i] < 0.0) any_negative = 1;
    if (any_negative) {
        double before = sum9(out);
        if (out[0] < 0.0) {
            /* zero the rest population, then rescale all nine so that the
             * site keeps the density it had before the zeroing */
            double rho_pre = sum9(out);
            out[0] = 0.0;
            double rest = sum9(out);
            if (rest > 0.0) {
                double r = rho_pre / rest;
                for (int i = 0; i < 9; ++i) out[i] = out[i] * r;
            }
        }
        for (int i = 1; i < 9; ++i) {
            if (out[i] < 0.0) {
                /* the magnitude goes to the reverse direction */
                out[OPP[i]] = out[OPP[i]] + (-out[i]);
                out[i] = 0.0;
            }
        }
        *dfix_out = sum9(out) - before;
    }
    return 1;
}

int orc_update_site(const orc_params *p, const double fstar_in[9], int64_t t,
                    int32_t x, int64_t y_abs, int32_t h_prev_x, int64_t y_wall,
                    int force, double lam, double out[9], double *S_out,
                    double *dfix_out, int32_t *ndiv_out, int64_t *wfx_out)
{
    return update_site(p, fstar_in, t, x, y_abs, h_prev_x, y_wall, force, lam, NULL, out, S_out,
                       dfix_out, ndiv_out, wfx_out);
}

/* ----------------------------------------------------------------------- */
/* Diagnostics: h(x), its mean and the width w(t)                            */
/* ----------------------------------------------------------------------- */
/* w(t) of Sec. III: the population standard deviation of h over the L
 * columns.  Heights are integers, so the sums are taken exactly in integers
 * (relative to the wall row, which leaves the variance unchanged):
 *   hbar = y_wall + S1 / L,   w = sqrt(L S2 - S1^2) / L,
 * with S1 = sum d, S2 = sum d^2, d = h - y_wall.  This makes both results
 * independent of summation order. */
static void width_of(const orc_state *s, double *hbar, double *W)
{
    const int32_t L = s->p.L;
    int64_t S1 = 0, S2 = 0;
    for (int32_t x = 0; x < L; ++x) {
        int64_t d = (int64_t)s->h[x] - s->y_wall;
        S1 += d;
        S2 += d * d;
    }
    int64_t num = (int64_t)L * S2 - S1 * S1;
    *hbar = (double)s->y_wall + (double)S1 / (double)L;
    *W = sqrt((double)num) / (double)L;
}

static double window_mass(const orc_state *s)
{
    const orc_params *p = &s->p;
    double m = 0.0;
    for (int32_t j = 0; j < p->H; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            double v[9];
            for (int i = 0; i < orc_q(p); ++i) v[i] = s->f[idx(p, i, j, x)];
            m += sumq(p, v);
        }
    return m;
}

/* Window mass in units of 2^-24, site by site (see mass_fx). */
static int64_t window_mass_fx(const orc_state *s)
{
    const orc_params *p = &s->p;
    int64_t m = 0;
    for (int32_t j = 0; j < p->H; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            double v[9];
            for (int i = 0; i < orc_q(p); ++i) v[i] = s->f[idx(p, i, j, x)];
            m += mass_fx(sumq(p, v));
        }
    return m;
}

/* Division laws on a state given as populations (the initial state, or one
 * set from outside): its sites count as eligible by their own density, with
 * the current front heights. */
static void division_rates_from_state(orc_state *s)
{
    const orc_params *p = &s->p;
    int64_t wsum = 0;
    for (int32_t j = 0; j < p->H; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            double v[9];
            for (int i = 0; i < orc_q(p); ++i) v[i] = s->f[idx(p, i, j, x)];
            double rho = sumq(p, v), q;
            int64_t y_abs = s->y_wall + j;
            if (rho >= p->rho_c &&
                division_eligible(p, rho, in_region(p, y_abs, s->h[x], s->y_wall), &q))
                wsum += division_weight(p, q);
        }
    s->lam = division_lam(p, window_mass_fx(s), wsum);
}

static void check_front(orc_state *s)
{
    const orc_params *p = &s->p;
    int64_t hmax = s->h[0];
    for (int32_t x = 1; x < p->L; ++x) if (s->h[x] > hmax) hmax = s->h[x];
    if (hmax > s->h_hi) s->h_hi = hmax;
    if (p->ybc != ORC_Y_PERIODIC && hmax >= s->y_wall + (int64_t)p->H)
        s->status |= ORC_ST_DOMAIN_FULL;
    if (!isfinite(s->mass)) s->status |= ORC_ST_NONFINITE;
}

/* ----------------------------------------------------------------------- */
/* Life cycle                                                                */
/* ----------------------------------------------------------------------- */
size_t orc_state_bytes(const orc_params *p)
{
    return 2u * (size_t)orc_q(p) * (size_t)p->L * (size_t)p->H * sizeof(double) +
           (size_t)p->L * sizeof(int32_t);
}

orc_state *orc_create(const orc_params *p)
{
    if (!p || !params_valid(p)) return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *p;
    size_t n = (size_t)orc_q(p) * (size_t)p->L * (size_t)p->H;
    s->f = (double *)calloc(n, sizeof(double));
    s->fn = (double *)calloc(n, sizeof(double));
    s->h = (int32_t *)calloc((size_t)p->L, sizeof(int32_t));
    s->divmap = (int32_t *)calloc((size_t)p->L * (size_t)p->H, sizeof(int32_t));
    if (!s->f || !s->fn || !s->h || !s->divmap) { orc_destroy(s); return NULL; }
    if (division_law(p) && p->division_mode == ORC_DIVISION_SELECTION) {
        size_t na = p->lattice == ORC_LATTICE_D2Q7 ? 3 : 4;
        s->sel = (int32_t *)calloc((size_t)p->L * (size_t)p->H * na, sizeof(int32_t));
        if (!s->sel) { orc_destroy(s); return NULL; }
    }

    /* Appendix A initialisation: u = 0, rho uniform around rho_init in the
     * first init_rows rows, f_i = f_i^SS(rho, 0); empty above */
    for (int32_t j = 0; j < p->init_rows; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            double U = orc_init_uniform(p->seed, p->replica, x, j);
            double rho = p->rho_init * (1.0 + p->init_amp * (2.0 * U - 1.0));
            double fss[9];
            fss_rest(p, rho, fss);
            for (int i = 0; i < orc_q(p); ++i) s->f[idx(p, i, j, x)] = fss[i];
        }
    s->t = 0;
    s->y_wall = 0;
    /* initial front: one above the highest site whose density reaches rho_c */
    for (int32_t x = 0; x < p->L; ++x) {
        int32_t hx = 0;
        for (int32_t j = 0; j < p->H; ++j) {
            double v[9];
            for (int i = 0; i < orc_q(p); ++i) v[i] = s->f[idx(p, i, j, x)];
            if (sumq(p, v) >= p->rho_c) hx = j + 1;
        }
        s->h[x] = hx;
    }
    s->h_hi = 0;
    s->mass = window_mass(s);
    width_of(s, &s->hbar, &s->W);
    division_rates_from_state(s);
    check_front(s);
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->f);
    free(s->fn);
    free(s->h);
    free(s->divmap);
    free(s->sel);
    free(s);
}

/* Rear wall of the active portion (Appendix A, last paragraph): after a step,
 * the wall moves up to at least max(gap, factor * w) below the mean front;
 * rows it passes leave the simulation and their mass is booked as retired. */
static void advance_wall(orc_state *s)
{
    const orc_params *p = &s->p;
    double gap = s->W * p->wall_w_factor;
    if (gap < (double)p->wall_min_gap) gap = (double)p->wall_min_gap;
    int64_t target = (int64_t)floor(s->hbar - gap);
    if (target <= s->y_wall) return;
    int64_t k = target - s->y_wall;
    if (k >= p->H) k = p->H - 1;
    double gone = 0.0;
    for (int32_t j = 0; j < (int32_t)k; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            double v[9];
            for (int i = 0; i < orc_q(p); ++i) v[i] = s->f[idx(p, i, j, x)];
            gone += sumq(p, v);
        }
    for (int i = 0; i < orc_q(p); ++i)
        for (int32_t j = 0; j < p->H; ++j)
            for (int32_t x = 0; x < p->L; ++x) {
                int32_t src = j + (int32_t)k;
                s->f[idx(p, i, j, x)] = (src < p->H) ? s->f[idx(p, i, src, x)] : 0.0;
            }
    /* the division map moves with the window */
    for (int32_t j = 0; j < p->H; ++j)
        for (int32_t x = 0; x < p->L; ++x) {
            int32_t src = j + (int32_t)k;
            s->divmap[(size_t)j * p->L + x] = (src < p->H) ? s->divmap[(size_t)src * p->L + x] : 0;
        }
    s->y_wall += k;
    s->retired += gone;
    s->mass = s->mass - gone;
    /* columns with no tissue left in the window sit at the wall */
    for (int32_t x = 0; x < p->L; ++x)
        if (s->h[x] < s->y_wall) s->h[x] = (int32_t)s->y_wall;
}

/* Step 3 as Sec. II states it (ORC_DIVISION_SELECTION), before any site is
 * updated.  The streamed state's total mass m_tot gives n_s = g m_tot /
 * rho_cell divisions (rounded to an integer stochastically: floor(n_s), plus
 * one with probability n_s - floor(n_s), so that g m_tot is added on
 * average).  Sites are drawn uniformly, with replacement, from the occupied
 * sites (tissue: streamed density >= rho_c) of the proliferating region, and
 * a drawn site divides with probability p_div: 1 for the uniform law, Eq. 5
 * on its streamed density for the density law.  Draws go on until n_s
 * divisions have happened; each division picks its axis at random.
 * counts[naxes * (j * L + x) + a] receives the divisions of window site
 * (x, j) along axis a.  Returns n_s over the occupied sites' total
 * acceptance probability (a site's expected divisions per unit of p_div),
 * or 0 if none may divide. */
static double selection_divisions(orc_state *s, int32_t *counts)
{
    const orc_params *p = &s->p;
    const int naxes = p->lattice == ORC_LATTICE_D2Q7 ? 3 : 4;
    const size_t nsites = (size_t)p->L * (size_t)p->H;
    memset(counts, 0, nsites * (size_t)naxes * sizeof(int32_t));
    int64_t *occ = (int64_t *)malloc(nsites * sizeof(int64_t));
    double *pdiv = (double *)malloc(nsites * sizeof(double));
    size_t nocc = 0;
    double m_tot = 0.0, wtot = 0.0;
    for (int32_t j = 0; j < p->H; ++j) {
        int64_t y_abs = s->y_wall + j;
        for (int32_t x = 0; x < p->L; ++x) {
            double fstar[9], q;
            orc_pull_site_abs(p, s->f, x, j, y_abs, fstar);
            double rho = sumq(p, fstar);
            m_tot += rho;
            if (rho < p->rho_c || !in_region(p, y_abs, s->h[x], s->y_wall)) continue;
            occ[nocc] = (int64_t)j * p->L + x;
            pdiv[nocc] = division_eligible(p, rho, 1, &q) ? q : 0.0;
            wtot += pdiv[nocc];
            nocc += 1;
        }
    }
    double ns = p->growth_rate * m_tot / p->rho_cell;
    double base = floor(ns);
    int64_t n = (int64_t)base;
    if (orc_selection_round_uniform(p->seed, p->replica, s->t) < ns - base) n += 1;
    int64_t done = 0;
    for (int64_t a = 0; done < n && nocc > 0 && wtot > 0.0; ++a) {
        double Us, Ua;
        uint32_t bits;
        orc_selection_draws(p->seed, p->replica, s->t, a, &Us, &Ua, &bits);
        size_t c = (size_t)(Us * (double)nocc);
        if (c >= nocc) c = nocc - 1;
        if (!(Ua < pdiv[c])) continue;
        /* the axis: uniform over the lattice's axes */
        int axis = (int)(((uint64_t)bits * (uint64_t)naxes) >> 32);
        counts[(size_t)naxes * (size_t)occ[c] + (size_t)axis] += 1;
        done += 1;
    }
    free(occ);
    free(pdiv);
    return wtot > 0.0 ? ns / wtot : 0.0;
}

int orc_step(orc_state *s, int64_t nsteps)
{
    const orc_params *p = &s->p;
    const int selection = s->sel != NULL;
    const int naxes = p->lattice == ORC_LATTICE_D2Q7 ? 3 : 4;
    int32_t *counts = s->sel;
    for (int64_t n = 0; n < nsteps; ++n) {
        if (s->status & ORC_ST_DOMAIN_FULL) break;
        double src = 0.0, fix = 0.0;
        int64_t wsum = 0;
        double lam_sel = selection ? selection_divisions(s, counts) : 0.0;
        int32_t *h_new = (int32_t *)malloc((size_t)p->L * sizeof(int32_t));
        for (int32_t x = 0; x < p->L; ++x) h_new[x] = (int32_t)s->y_wall;
        for (int32_t j = 0; j < p->H; ++j) {
            int64_t y_abs = s->y_wall + j;
            for (int32_t x = 0; x < p->L; ++x) {
                double fstar[9], out[9], S, dfix;
                int32_t ndiv;
                int64_t wfx;
                orc_pull_site_abs(p, s->f, x, j, y_abs, fstar);
                const int32_t *given =
                    counts ? counts + (size_t)naxes * ((size_t)j * p->L + x) : NULL;
                int tissue = update_site(p, fstar, s->t, x, y_abs, s->h[x], s->y_wall, -1,
                                         s->lam, given, out, &S, &dfix, &ndiv, &wfx);
                for (int i = 0; i < orc_q(p); ++i) s->fn[idx(p, i, j, x)] = out[i];
                src += S;
                fix += dfix;
                s->divisions += ndiv;
                s->divmap[(size_t)j * p->L + x] += ndiv;
                wsum += wfx;
                if (tissue && y_abs + 1 > h_new[x]) h_new[x] = (int32_t)(y_abs + 1);
            }
        }
        double *tmp = s->f; s->f = s->fn; s->fn = tmp;
        memcpy(s->h, h_new, (size_t)p->L * sizeof(int32_t));
        free(h_new);
        s->t += 1;
        s->src_total += src;
        s->fix_total += fix;
        s->mass = window_mass(s);
        width_of(s, &s->hbar, &s->W);
        if (p->ybc == ORC_Y_WALL_FOLLOW) {
            advance_wall(s);
            width_of(s, &s->hbar, &s->W);
        }
        /* division laws: the next step shares g m_tot / rho_cell divisions
         * over the weight of the sites eligible at this step (the sites
         * eligible at the next step are known only as it runs).  The
         * selection procedure reports the mean divisions per unit weight
         * its step used instead. */
        if (selection)
            s->lam = lam_sel;
        else
            s->lam = division_lam(p, window_mass_fx(s), wsum);
        check_front(s);
    }
    return (s->status & ORC_ST_DOMAIN_FULL) ? -4 : 0;
}

void orc_diagnostics(const orc_state *s, orc_diag *d)
{
    d->mass = s->mass;
    d->src_total = s->src_total;
    d->fix_total = s->fix_total;
    d->retired = s->retired;
    d->hbar = s->hbar;
    d->W = s->W;
    d->step = s->t;
    d->y_wall = s->y_wall;
    d->h_hi = s->h_hi;
    d->status = s->status;
    d->lam = s->lam;
    d->divisions = s->divisions;
}

void orc_front_heights(const orc_state *s, int32_t *h_out)
{
    memcpy(h_out, s->h, (size_t)s->p.L * sizeof(int32_t));
}

void orc_get_populations(const orc_state *s, double *f_out)
{
    memcpy(f_out, s->f, (size_t)orc_q(&s->p) * (size_t)s->p.L * (size_t)s->p.H * sizeof(double));
}

void orc_set_populations(orc_state *s, const double *f_in)
{
    memcpy(s->f, f_in, (size_t)orc_q(&s->p) * (size_t)s->p.L * (size_t)s->p.H * sizeof(double));
    s->mass = window_mass(s);
    division_rates_from_state(s);
}

void orc_set_front_heights(orc_state *s, const int32_t *h_in)
{
    memcpy(s->h, h_in, (size_t)s->p.L * sizeof(int32_t));
    width_of(s, &s->hbar, &s->W);
    division_rates_from_state(s);
}

void orc_set_step(orc_state *s, int64_t t)
{
    s->t = t;
}

void orc_set_lam(orc_state *s, double lam)
{
    s->lam = lam;
}

void orc_division_map(const orc_state *s, int32_t *out)
{
    memcpy(out, s->divmap, (size_t)s->p.L * (size_t)s->p.H * sizeof(int32_t));
}

int orc_selection_counts(const orc_state *s, int32_t *out)
{
    if (!s->sel) return 0;
    size_t na = s->p.lattice == ORC_LATTICE_D2Q7 ? 3 : 4;
    memcpy(out, s->sel, (size_t)s->p.L * (size_t)s->p.H * na * sizeof(int32_t));
    return (int)na;
}

void orc_clear_division_map(orc_state *s)
{
    memset(s->divmap, 0, (size_t)s->p.L * (size_t)s->p.H * sizeof(int32_t));
}
