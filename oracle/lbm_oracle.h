/*
 * lbm_oracle.h -- plain FP64 CPU oracle for the growing-tissue lattice
 * Boltzmann method (Killeen, Partridge, Bertrand, Lee, "Modeling growing
 * confluent tissues using a lattice Boltzmann method", arXiv 2303.02210), on
 * the square D2Q9 lattice or on the paper's own triangular D2Q7 lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously correct
 * reference the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never calls it.  It shares no code, header, table or helper
 * with the HIP library: every constant below is restated here from the paper
 * (and from the textbook D2Q9 lattice the paper cites for its equilibrium).
 *
 * Everything is double precision and evaluated in one fixed order (the order
 * each formula is written in), with no fused multiply-add.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* growth law (Sec. II, mass injection between streaming and redistribution):
 * none; the expectation of the paper's injection spread over every tissue
 * site (bulk); or the paper's discrete cell divisions, at tissue sites drawn
 * uniformly (division) or accepted with the density-dependent probability of
 * Eq. 5 (division_density) */
enum { ORC_GROWTH_NONE = 0, ORC_GROWTH_BULK = 1, ORC_GROWTH_DIVISION = 2,
       ORC_GROWTH_DIVISION_DENSITY = 3 };
/* proliferating region: everywhere, a band of width ell below the front, or a
 * band of width d above the rear wall (Appendix B) */
enum { ORC_REGION_ALL = 0, ORC_REGION_FRONT_BAND = 1, ORC_REGION_REAR_BAND = 2 };
/* boundary along the growth axis: fixed bounce-back rear wall, rear wall that
 * follows the front (Appendix A, last paragraph), or periodic (test mode) */
enum { ORC_Y_WALL_FIXED = 0, ORC_Y_WALL_FOLLOW = 1, ORC_Y_PERIODIC = 2 };
/* how the division laws choose their sites in step 3:
 *   ORC_DIVISION_PER_SITE  each eligible site draws a Poisson number of
 *                          divisions of mean lam q, lam = n_s over the total
 *                          weight of the sites eligible at the previous step
 *                          (the data-parallel form the GPU library computes)
 *   ORC_DIVISION_SELECTION the procedure as Sec. II states it: n_s =
 *                          g m_tot / rho_cell with m_tot the total mass of
 *                          the streamed state, sites drawn uniformly with
 *                          replacement from the occupied (tissue) sites of the
 *                          region, each draw accepted with probability
 *                          p_div (1, or Eq. 5), until n_s divisions happened
 *                          (n_s rounded stochastically to an integer) */
enum { ORC_DIVISION_PER_SITE = 0, ORC_DIVISION_SELECTION = 1 };
/* status bits */
enum { ORC_ST_DOMAIN_FULL = 1u, ORC_ST_NONFINITE = 2u };
/* lattice: square D2Q9 (populations [9][H][L]) or the paper's triangular D2Q7
 * (Sec. II; populations [7][H][L]).  D2Q7 rows are horizontal lines sqrt(3)/2
 * apart and odd rows are shifted half a lattice unit along +x, so site (x, y)
 * sits at (x + (y mod 2)/2, y sqrt(3)/2); directions e_i = (cos, sin) of
 * (i - 1) pi/3: 0 rest, 1 E, 2 NE, 3 NW, 4 W, 5 SW, 6 SE; reverse pairs 1-4,
 * 2-5, 3-6.  Parity is that of the absolute row. */
enum { ORC_LATTICE_D2Q9 = 0, ORC_LATTICE_D2Q7 = 1 };

typedef struct {
    int32_t  L, H;           /* columns (periodic x), rows (growth axis y)   */
    double   tau;            /* relaxation time, Eq. 2                        */
    double   mu;             /* friction, u* = (1 - mu) u, below Eq. 3        */
    double   rho_c;          /* threshold density, Appendix A step 5          */
    double   rho_init;       /* initial mean density, Appendix A              */
    double   init_amp;       /* rho ~ U[(1-a), (1+a)] rho_init (paper: 0.1)   */
    int32_t  init_rows;      /* tissue initially fills rows [0, init_rows)    */
    int32_t  growth;         /* ORC_GROWTH_*                                  */
    double   growth_rate;    /* g, mass added per unit tissue mass per step   */
    int32_t  region;         /* ORC_REGION_*                                  */
    int32_t  region_width;   /* ell (front band) or d (rear band)             */
    double   sigma;          /* noise amplitude, Eq. 4                        */
    int32_t  ybc;            /* ORC_Y_*                                       */
    int32_t  wall_min_gap;   /* rear wall kept >= max(gap, factor*w) behind   */
    double   wall_w_factor;  /*   the mean front height (Appendix A)          */
    uint32_t seed;           /* Philox key word 0                             */
    uint32_t replica;        /* Philox key word 1                             */
    double   rho_cell;       /* mass of one cell (division laws), Sec. II     */
    double   rho0;           /* density above which division stops, Eq. 5     */
    int32_t  lattice;        /* ORC_LATTICE_*                                 */
    int32_t  division_mode;  /* ORC_DIVISION_*                                */
} orc_params;

typedef struct {
    double   mass;           /* total mass of the live window after the step */
    double   src_total;      /* cumulative injected mass                      */
    double   fix_total;      /* cumulative mass change of the negative fix    */
    double   retired;        /* cumulative mass in rows the rear wall left    */
    double   hbar, W;        /* mean and standard deviation of h(x)           */
    int64_t  step;           /* steps taken                                   */
    int64_t  y_wall;         /* absolute row of the first live row            */
    int64_t  h_hi;           /* largest front height seen so far              */
    uint32_t status;         /* ORC_ST_* bits                                 */
    double   lam;            /* division laws: expected divisions per drawn
                                site (unit weight) at the next step           */
    int64_t  divisions;      /* cumulative number of cell divisions           */
} orc_diag;

typedef struct orc_state orc_state;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The nine noise draws of one site: 24-bit integers k_0..k_8, and the
 * uniforms U_i = (k_i + 1/2) 2^-24 on (0, 1). */
void orc_noise_bits(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                    int64_t y_abs, uint32_t k_out[9]);
void orc_noise_uniforms(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                        int64_t y_abs, double u_out[9]);
/* Uniform of the initial-density draw at (x, y). */
double orc_init_uniform(uint32_t seed, uint32_t replica, int32_t x, int64_t y_abs);

/* Draws of the selection procedure (ORC_DIVISION_SELECTION) at step t:
 * attempt a gives the uniform that picks the site (U_site, 52 bits), the
 * acceptance uniform (U_acc, 32 bits) and 32 bits for the axis; the rounding
 * of a fractional n_s uses U_round. */
void orc_selection_draws(uint32_t seed, uint32_t replica, int64_t t, int64_t a,
                         double *U_site, double *U_acc, uint32_t *axis_bits);
double orc_selection_round_uniform(uint32_t seed, uint32_t replica, int64_t t);

/* Division draws of one site at step t: a uniform U = (n + 1/2) 2^-52 on
 * (0, 1) from 52 random bits (the Poisson count) and 64 bits of division
 * axes, two per division. */
void orc_division_draws(uint32_t seed, uint32_t replica, int64_t t, int32_t x,
                        int64_t y_abs, double *U_out, uint64_t *axes_out);
/* e^-lam for 0 <= lam <= 8 from basic arithmetic only (so that any two IEEE
 * implementations agree bit for bit). */
double orc_exp_neg(double lam);
/* Poisson(lam) count by inversion of its distribution function at U,
 * capped at 32. */
int orc_poisson_k(double U, double lam);

/* Lattice constants as used by the oracle (for the closed-form pins). */
void orc_lattice(int32_t cx[9], int32_t cy[9], int32_t opp[9], double w[9]);

/* Eq. 3 with D2Q9 coefficients: steady-state populations for rho and the
 * (already friction-damped) velocity u*. */
void orc_fss(double rho, double ux_star, double uy_star, double out[9]);

/* Stream (Appendix A step 1) for one site: f*_i(x, j) pulled from the window
 * f[9][H][L] (j = row inside the window). */
void orc_pull_site(const orc_params *p, const double *f, int32_t x, int32_t j,
                   double fstar[9]);
/* The same for window row j holding absolute row y_abs (D2Q7 pulls depend on
 * the absolute row's parity; orc_pull_site takes y_abs = j). */
void orc_pull_site_abs(const orc_params *p, const double *f, int32_t x, int32_t j,
                       int64_t y_abs, double fstar[9]);
/* Eq. 3 on D2Q7: w_i rho (1 + 4 e.u* + 8 (e.u*)^2 - 2 |u*|^2), w = 1/2, 1/12. */
void orc_fss7(double rho, double ux_star, double uy_star, double out[7]);
/* Populations per site of the lattice p names (9 or 7). */
int orc_q(const orc_params *p);

/* Steps 2-7 of Appendix A at one site, given its streamed populations.
 * force: -1 classify by density, 0 force the void branch, 1 force tissue.
 * lam: the division laws' expected divisions per unit weight at this step.
 * Returns 1 if the site was classified tissue.  S_out: injected mass,
 * dfix_out: mass change of the negative-value fix, ndiv_out: divisions at
 * the site, wfx_out: the site's weight for the division laws' normaliser
 * (1 per eligible site, or 2^24 x its acceptance probability; 0 if not
 * eligible). */
int orc_update_site(const orc_params *p, const double fstar[9], int64_t t,
                    int32_t x, int64_t y_abs, int32_t h_prev_x, int64_t y_wall,
                    int force, double lam, double out[9], double *S_out,
                    double *dfix_out, int32_t *ndiv_out, int64_t *wfx_out);

size_t     orc_state_bytes(const orc_params *p);
orc_state *orc_create(const orc_params *p);        /* NULL if p invalid */
int        orc_step(orc_state *s, int64_t nsteps); /* 0, or -4 domain full */
void       orc_destroy(orc_state *s);
void       orc_diagnostics(const orc_state *s, orc_diag *out);
void       orc_front_heights(const orc_state *s, int32_t *h_out);
/* populations of the live window, [9][H][L], window row j = y_wall + j */
void       orc_get_populations(const orc_state *s, double *f_out);
void       orc_set_populations(orc_state *s, const double *f_in);
/* replace h (used as h_prev by the front band) */
void       orc_set_front_heights(orc_state *s, const int32_t *h_in);
/* set the step counter (the noise of the next step is drawn at counter t) */
void       orc_set_step(orc_state *s, int64_t t);
/* division laws: set lam of the next step (it otherwise comes from the
 * previous step, or from the state's own densities after a set) */
void       orc_set_lam(orc_state *s, double lam);
/* Divisions per site of the window ([H][L], row j = absolute row y_wall + j)
 * since creation or the last clear; rows the wall retires leave the map. */
void       orc_division_map(const orc_state *s, int32_t *out);
void       orc_clear_division_map(orc_state *s);
/* Selection procedure: the last step's divisions per window site and axis,
 * [H][L][axes]; returns the number of axes (4 on D2Q9, 3 on D2Q7; D2Q9 axes
 * E-W, N-S, NE-SW, NW-SE; D2Q7 E-W, NE-SW, NW-SE), or 0 (nothing written)
 * under the per-site form. */
int        orc_selection_counts(const orc_state *s, int32_t *out);

#ifdef __cplusplus
}
#endif
#endif
