/*
 * lbmgrow.h -- C ABI of the MI355X (gfx950) growing-tissue lattice Boltzmann
 * library.
 *
 * The method is the lattice Boltzmann model of a growing tissue of Killeen,
 * Partridge, Bertrand and Lee (arXiv 2303.02210), run on the square D2Q9
 * lattice: per step and per site, stream, take moments (Eq. 1), add the
 * proliferation mass, relax towards the friction-damped steady state (Eqs. 2
 * and 3) or -- below the threshold density -- reverse every direction (the
 * two-step bounce-back front of Sec. II), add zero-sum noise (Eq. 4) and
 * remove negative populations (Appendix A, steps 1-7).  Per column the
 * library keeps the interface height h(x, t) used for the width w(t) of
 * Sec. III, and optionally moves the rear wall with the front (Appendix A).
 *
 * Conventions shared by every call:
 *   - Lattice: x = column, periodic, 0 <= x < L; y = row along the growth
 *     direction.  Directions: 0 rest, 1 E(+x), 2 N(+y), 3 W, 4 S, 5 NE, 6 NW,
 *     7 SW, 8 SE; reverse pairs 1-3, 2-4, 5-7, 6-8.
 *   - Populations on the host are float64 arrays [9][H][L] (direction,
 *     window row, column); window row j is absolute row y_wall + j.
 *   - Device memory is never allocated by the library: the caller passes one
 *     device workspace of at least lbm_workspace_bytes() bytes that must stay
 *     valid until lbm_destroy.  Every device operation is enqueued on the
 *     caller's HIP stream.
 *   - Every call returns LBM_OK (0) or a negative lbm_status.  Calls marked
 *     "synchronizes" wait for the stream; others only enqueue work.  Faults
 *     found on the device (front reached the top row, non-finite mass) are
 *     latched in a device status word and returned by the next synchronizing
 *     call; after any error a handle only accepts lbm_destroy,
 *     lbm_diagnostics and lbm_last_error (everything else: LBM_E_STATE).
 *   - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef LBMGROW_H
#define LBMGROW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 4u

typedef struct lbm_handle lbm_handle;
typedef struct lbm_batch lbm_batch;

typedef enum {
    LBM_OK = 0,
    LBM_E_INVALID = -1,      /* bad argument or parameter                     */
    LBM_E_NOMEM = -2,        /* workspace or host buffer too small            */
    LBM_E_DEVICE = -3,       /* a HIP runtime call failed                     */
    LBM_E_DOMAIN_FULL = -4,  /* the front reached the last row of the window  */
    LBM_E_NONFINITE = -5,    /* total mass became NaN or infinite             */
    LBM_E_UNSUPPORTED = -6,  /* valid request the library does not implement */
    LBM_E_STATE = -7         /* handle is in an error state                   */
} lbm_status;

/* Storage / arithmetic of the populations. */
typedef enum {
    LBM_FP64 = 0,            /* float64 storage and arithmetic                */
    LBM_FP32 = 1,            /* float32 storage and arithmetic                */
    LBM_FP16_OFFSET = 2,     /* float16 of f_i - W_i, float32 arithmetic      */
    LBM_BF16_OFFSET = 3      /* bfloat16 of f_i - W_i, float32 arithmetic     */
} lbm_precision;

/* Growth law (Sec. II, mass injection between streaming and redistribution). */
typedef enum {
    LBM_GROWTH_NONE = 0,
    LBM_GROWTH_BULK = 1,     /* every tissue site of the region gains g rho*
                                (the expectation of the paper's injection)    */
    LBM_GROWTH_DIVISION = 2, /* discrete divisions: rho_cell / 2 on both
                                directions of a random axis, at a Poisson
                                number per tissue site of the region, n_s =
                                g m_tot / rho_cell per step in expectation    */
    LBM_GROWTH_DIVISION_DENSITY = 3  /* as DIVISION, each site weighted by
                                the probability 1 - rho / rho0 of Eq. 5 (rho
                                the streamed density; none at or below rho_c) */
} lbm_growth;

/* Proliferating region. */
typedef enum {
    LBM_REGION_ALL = 0,        /* all tissue sites                              */
    LBM_REGION_FRONT_BAND = 1, /* tissue with y >= h_prev(x) - region_width     */
    LBM_REGION_REAR_BAND = 2   /* tissue with y <  y_wall + region_width (App. B) */
} lbm_region;

/* Boundary along the growth axis. */
typedef enum {
    LBM_Y_WALL_FIXED = 0,    /* bounce-back wall below row 0, empty above top */
    LBM_Y_WALL_FOLLOW = 1,   /* wall follows the front (Appendix A)           */
    LBM_Y_PERIODIC = 2       /* periodic rows (test mode)                     */
} lbm_ybc;

/* Lattice (Sec. II).  D2Q9: the square lattice, directions 0 rest, 1 E, 2 N,
 * 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.  D2Q7: the paper's own triangular
 * lattice, weights 1/2 and 1/12, c_s^2 = 1/4, directions 0 rest, 1 E, 2 NE,
 * 3 NW, 4 W, 5 SW, 6 SE; its rows are horizontal lines sqrt(3)/2 apart with
 * odd (absolute) rows shifted half a unit along +x.  Population arrays are
 * [Q][H][L] with Q = 9 or 7. */
typedef enum {
    LBM_LATTICE_D2Q9 = 0,
    LBM_LATTICE_D2Q7 = 1
} lbm_lattice;

/* lbm_params.flags */
#define LBM_FLAG_DIVISION_MAP 2u   /* keep a per-site count of the divisions
                                      (read with lbm_division_map)            */
#define LBM_FLAG_WINDOW 1u   /* sweep only rows that can hold mass: rows at or
                                below the highest front seen plus one (the rest
                                are exactly zero); results are unchanged      */
#define LBM_FLAG_STOCHASTIC_ROUND 4u  /* FP16 / BF16 offset storage only: a
                                tissue site's stored offsets are rounded
                                stochastically (to the neighbour above their
                                magnitude with probability equal to the
                                distance from the one below, in ulps) instead
                                of to nearest, so that increments smaller than
                                half an ulp survive on average.  Draws one
                                Philox call per tissue site (stream 3).
                                LBM_E_INVALID with FP32 / FP64 storage or
                                with kernel_vb 2 (the LDS-staged form).      */

#define LBM_FLAG_BATCH_TABLE 8u   /* in a batch, always step this member
                                through the batch's shared tile table        */
#define LBM_FLAG_BATCH_OWN 16u    /* in a batch, step this member by its own
                                launches inside the batch's graph (ignored
                                for members that move their wall or window
                                or grow by a division law).  Without either
                                flag members of at least 2^22 sites that do
                                neither step by their own launches.  Results
                                are the same either way.                     */

/*
 * Model and run parameters.  Set abi_version = LBM_ABI_VERSION and
 * struct_size = sizeof(lbm_params).
 *   L, H          columns (periodic) and rows of the live window;
 *                 2 <= L <= 2^24, H >= 4 and L * H * Q <= 2^31 populations
 *                 (Q = 9 on D2Q9, 7 on D2Q7); they must fit the workspace.
 *   lattice       lbm_lattice.  D2Q7 runs every form but the LDS-staged one
 *                 (kernel_vb 2) and needs an even H when periodic.
 *   precision     lbm_precision.
 *   tau           relaxation time of Eq. 2, tau > 1/2.
 *   mu            friction: the steady state uses u* = (1 - mu) u (below
 *                 Eq. 3); 0 <= mu <= 1.
 *   rho_c         threshold density of the bounce-back front (Appendix A,
 *                 step 5); rho_c > 0.
 *   rho_init, init_amp, init_rows
 *                 initial state (Appendix A): rows [0, init_rows) at rest with
 *                 rho uniform on [(1 - a), (1 + a)] rho_init, a = init_amp in
 *                 [0, 1); rows above empty.
 *   growth, growth_rate
 *                 lbm_growth and the rate g >= 0 (mass per unit tissue mass per
 *                 step; Sec. II).  The division laws draw each eligible site's
 *                 divisions from a Poisson law of mean lam q (q = 1, or Eq. 5's
 *                 probability), lam = n_s over the total q of the sites eligible
 *                 at the previous step; m_tot is the window mass then.  They
 *                 run the per-step device bookkeeping (as the follow wall does).
 *   rho_cell, rho0
 *                 division laws: the mass of one cell (> 0), and the density
 *                 at which division stops (Eq. 5; > rho_c).
 *   region, region_width
 *                 lbm_region and its width (>= 0).
 *   sigma         noise amplitude of Eq. 4, sigma >= 0.
 *   ybc           lbm_ybc.
 *   wall_min_gap, wall_w_factor
 *                 follow mode: after each step the wall moves up to
 *                 floor(hbar - max(wall_min_gap, wall_w_factor * w)) (Appendix
 *                 A uses 50 and 10).
 *   rho_ref       offset base of the 16-bit storages: populations are stored
 *                 as f_i - W_i with W_i = w_i rho_ref rounded to the storage
 *                 type, so that an empty site decodes to exactly 0.
 *   seed, replica Philox4x32-10 key words of all random draws.
 *   flags         LBM_FLAG_* bits.
 *   kernel_vb, kernel_ty
 *                 launch shape (results do not depend on it): 0 = library
 *                 default; kernel_vb 1 = one column per lane, 2 = population
 *                 rows staged through LDS by asynchronous global-to-LDS
 *                 loads (16-bit storages need an even width), 4 / 8 / 16 =
 *                 that many bytes of columns per lane (used when the width
 *                 splits evenly); kernel_ty = rows per thread (1..64).
 *                 Batches run staged members in the 4-byte (float64: 8-byte)
 *                 vector form.
 *   kernel_order  order in which a step's row strips of tiles are handed to
 *                 the GPU (results do not depend on it): 0 = library
 *                 default (4 for the D2Q9 step without a division law at
 *                 up to 4 rows per thread, 1 otherwise), 1 = from the wall
 *                 up, 2 = spread over the height
 *                 (the tiles in flight then mix tissue and empty rows),
 *                 3 = from the wall up on half of the chip's dies and from
 *                 the top down on the other half, 4 = two sweeps side by
 *                 side, one up the lower half and one up the upper half.
 */
typedef struct {
    uint32_t abi_version;
    uint32_t struct_size;
    int32_t  L, H;
    int32_t  precision;
    int32_t  growth;
    double   tau, mu, rho_c;
    double   rho_init, init_amp;
    int32_t  init_rows;
    int32_t  region;
    double   growth_rate;
    int32_t  region_width;
    int32_t  ybc;
    double   sigma;
    int32_t  wall_min_gap;
    int32_t  flags;
    double   wall_w_factor;
    double   rho_ref;
    uint32_t seed, replica;
    int32_t  kernel_vb;
    int32_t  kernel_ty;
    double   rho_cell;
    double   rho0;
    int32_t  lattice;
    int32_t  kernel_order;
} lbm_params;

/* Diagnostics after the last enqueued step (all reductions in float64). */
typedef struct {
    double   mass;        /* total mass in the live window                    */
    double   src_total;   /* mass injected by growth since creation           */
    double   fix_total;   /* mass added by the negative-population fix        */
    double   retired;     /* mass in rows the rear wall has left behind       */
    double   hbar, W;     /* mean and standard deviation of h(x) (Sec. III)   */
    int64_t  step;        /* steps taken                                      */
    int64_t  y_wall;      /* absolute row of window row 0                     */
    int64_t  h_hi;        /* highest front height seen since creation         */
    uint32_t status;      /* LBM_ST_* bits latched on the device              */
    uint32_t reserved;
    double   lam;         /* division laws: lam of the next step              */
    int64_t  divisions;   /* division laws: cell divisions since creation     */
    int64_t  rows_swept;  /* window rows updated since creation: L * rows_swept
                             site updates (H per step without the sweep
                             window, fewer with it)                           */
} lbm_diag;

#define LBM_ST_DOMAIN_FULL 1u
#define LBM_ST_NONFINITE   2u
#define LBM_ST_SYNC_LOST   4u   /* a multi-step batch launch's grid barrier
                                   gave up waiting (LBM_E_DEVICE)           */

/* Library version string, e.g. "lbmgrow 1.1 gfx950 src 0123456789abcdef":
 * the last word is the first 16 hex digits of the SHA-256 of the sources
 * the library was compiled from (this header and the kernel and host
 * sources), so a build can be matched to its source tree. */
const char *lbm_version(void);

/* Device workspace size for p; 0 if p is invalid. */
size_t lbm_workspace_bytes(const lbm_params *p);

/*
 * Create a simulation in dev_ws (device pointer, ws_bytes >= the size above,
 * 256-byte aligned) on hip_stream (a hipStream_t; NULL = the null stream).
 * Enqueues the initial state of Appendix A.  The handle is host memory owned
 * by the library until lbm_destroy.  Errors: LBM_E_INVALID (parameters,
 * null/unaligned pointers), LBM_E_NOMEM (ws_bytes too small), LBM_E_DEVICE.
 */
int lbm_create(const lbm_params *p, void *dev_ws, size_t ws_bytes, void *hip_stream,
               lbm_handle **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): lbm_create
 * without a workspace.  The caller passes only the population storage (two
 * buffers, the simulation's state); everything else the kernels use (front
 * heights, per-block tallies, device state, diagnostics record, batch
 * descriptor; a division map if flagged) lives in a static device array of
 * the library, 16 MiB per device, held until the process ends.  The call
 * allocates no device memory.
 *   dev_pops == NULL: size query, *pops_bytes = bytes the population storage
 *                     needs for p (nothing is created).
 *   otherwise:        dev_pops (device, 256-byte aligned, *pops_bytes bytes,
 *                     caller owned, valid until lbm_destroy) receives the
 *                     initial state on hip_stream; *out is a handle used
 *                     like any other (step, front heights, diagnostics,
 *                     populations, checkpoints, batches).
 * One such handle may be live per device at a time, since all of them would
 * share the device's array; lbm_destroy of it synchronizes its stream and
 * frees the array for the next one.
 * Errors: LBM_E_INVALID (parameters, null/unaligned pointers), LBM_E_NOMEM
 * (*pops_bytes too small; the lattice needs more than 16 MiB of scratch, e.g.
 * a division map of more than about 4M sites; or another live handle on the
 * device holds the array), LBM_E_DEVICE.
 */
int lbm_create_static(const lbm_params *p, void *dev_pops, size_t *pops_bytes, void *hip_stream,
                      lbm_handle **out);

/* Enqueue nsteps >= 0 steps (Appendix A steps 1-7 on every site, then the
 * front heights and, in follow mode, the wall).  Does not synchronize. */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Copy h(x) of the current state (L int32, absolute rows) to host_h and the
 * step count to *step_out (may be NULL).  Synchronizes; returns a latched
 * device fault if there is one. */
int lbm_front_heights(lbm_handle *h, int32_t *host_h, int64_t *step_out);

/* Enqueue a copy of h(x) of the current state into dst (L int32; device
 * memory or pinned host memory).  Does not synchronize: the caller
 * synchronizes the stream before reading dst. */
int lbm_front_heights_async(lbm_handle *h, int32_t *dst);

/* Fill *out.  Synchronizes. */
int lbm_diagnostics(lbm_handle *h, lbm_diag *out);

/* Populations of the live window decoded to float64 [Q][H][L].
 * Synchronizes. */
int lbm_get_populations(lbm_handle *h, double *host_f);

/* Replace the populations (encoded to the storage type with round to nearest
 * even).  Front heights are left unchanged.  Synchronizes. */
int lbm_set_populations(lbm_handle *h, const double *host_f);

/* Replace h(x) (L int32, absolute rows), e.g. as h_prev of the front band.
 * Synchronizes. */
int lbm_set_front_heights(lbm_handle *h, const int32_t *host_h);

/* Divisions per site of the live window since creation or the last clear
 * (Sec. IV: the proliferation counts near h_max and h_min), [H][L] int32,
 * row j = absolute row y_wall + j; rows the rear wall retires leave the
 * map.  clear != 0 zeroes it afterwards.  Needs LBM_FLAG_DIVISION_MAP
 * (LBM_E_INVALID otherwise).  Not part of checkpoints.  Synchronizes. */
int lbm_division_map(lbm_handle *h, int32_t *host_counts, int clear);

/* Checkpoint: size of the host blob, save, and restore into a handle created
 * with the same parameters.  A restored run continues bit for bit like the
 * uninterrupted one (all draws are keyed by step and site).  Synchronize. */
size_t lbm_state_bytes(const lbm_handle *h);
int lbm_get_state(lbm_handle *h, void *host_blob, size_t bytes);
int lbm_set_state(lbm_handle *h, const void *host_blob, size_t bytes);

/* Bandwidth reference for measurements: enqueue a copy of `bytes` bytes from
 * src to dst (device memory, both 16-byte aligned, not overlapping; bytes a
 * multiple of 16) by a streaming kernel of this library (16-byte nontemporal
 * loads and stores).  A benchmark times it beside the step kernel as the HBM
 * ceiling a plain read-and-write stream reaches.  LBM_E_INVALID on bad
 * arguments, LBM_E_DEVICE if the launch fails.  Does not synchronize. */
int lbm_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Human-readable description of the last error on h (never NULL). */
const char *lbm_last_error(const lbm_handle *h);

/* Release the handle.  Never frees the workspace.  Does not synchronize. */
int lbm_destroy(lbm_handle *h);

/*
 * Batches: many handles of any size and precision advanced together.  Per
 * step there is one kernel launch per group of members sharing a storage
 * type and kernel form, over the flattened table of all their tiles (plus,
 * for a group whose members follow the front, sweep a window or divide, a
 * launch of their between-step bookkeeping, and for a windowed group one
 * that rebuilds its table from the members' live rows); large members that
 * do none of that are stepped by their own kernels instead
 * (LBM_FLAG_BATCH_OWN), inside the same graph; a run of K steps is captured
 * in a HIP graph and replayed while the membership stays the same.  Every
 * member keeps its own workspace, state and status, and its populations come
 * out bit for bit as with lbm_step on the handle alone.
 *   lbm_tiles            tiles (thread blocks per step) of a simulation
 *                        with parameters p; 0 if p is invalid.
 *   lbm_batch_workspace_bytes  device workspace for up to max_members whose
 *                        tiles add up to at most max_tiles.
 *   lbm_batch_create     empty batch in dev_ws (256-byte aligned, caller
 *                        owned, valid until lbm_batch_destroy) on hip_stream;
 *                        members must use the same stream.
 *   lbm_batch_add/remove membership changes (take effect at the next step);
 *                        a handle belongs to at most one batch, and
 *                        lbm_destroy removes it from its batch.
 *   lbm_batch_step       nsteps >= 0 steps of every member; does not
 *                        synchronize; LBM_E_STATE if a member is in an error
 *                        state (remove it and step again).
 *   lbm_batch_persistent on = 1: each group whose members neither move their
 *                        wall or window nor grow by a division law runs
 *                        all nsteps of a lbm_batch_step in one cooperative
 *                        launch (a fixed grid of resident blocks striding
 *                        over its tile table, a grid-wide barrier between
 *                        steps); the other groups launch per step as
 *                        before; the run is enqueued directly, not through
 *                        a graph, every group on the batch's stream in
 *                        turn.  on = 0 (the default) restores per-step
 *                        launches.  A barrier that waits past about a
 *                        second gives up and latches LBM_ST_SYNC_LOST in
 *                        the members of that launch.  Results are the same
 *                        either way.
 *   lbm_batch_destroy    releases the batch, not its members.
 * Errors: LBM_E_INVALID (null/foreign handles, stream mismatch, full batch),
 * LBM_E_NOMEM (workspace too small, or members' tiles beyond max_tiles at
 * the next step), LBM_E_DEVICE.
 */
int64_t lbm_tiles(const lbm_params *p);
size_t lbm_batch_workspace_bytes(int max_members, int64_t max_tiles);
int lbm_batch_create(void *dev_ws, size_t ws_bytes, int max_members, int64_t max_tiles,
                     void *hip_stream, lbm_batch **out);
int lbm_batch_add(lbm_batch *b, lbm_handle *h);
int lbm_batch_remove(lbm_batch *b, lbm_handle *h);
int lbm_batch_step(lbm_batch *b, int64_t nsteps);
int lbm_batch_persistent(lbm_batch *b, int on);
int lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBMGROW_H */
