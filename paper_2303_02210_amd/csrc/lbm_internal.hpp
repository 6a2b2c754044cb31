// lbm_internal.hpp -- kernel argument blocks and launchers shared by the
// kernels (lbm_kernels.hip) and the C-ABI implementation (lbm_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace lbm {

template <class S>
struct Real;
template <>
struct Real<double> { using type = double; };
template <>
struct Real<float> { using type = float; };
template <>
struct Real<__half> { using type = float; };
template <>
struct Real<__hip_bfloat16> { using type = float; };

enum : int { kModeFixed = 0, kModeDevice = 1, kModePeriodic = 2 };
enum : int { kGrowthNone = 0, kGrowthBulk = 1, kGrowthDivision = 2, kGrowthDivisionDensity = 3 };

// Per-block tallies, kPartialSlots doubles per block: [0] mass of the block's
// sites after the step, [1] injected mass and [2] mass change of the negative
// fix (both accumulated over steps), [3] unused.
constexpr int kPartialSlots = 4;
// Division-law tallies of one step (integers, so their sum does not depend on
// the order of the additions): blocks add theirs atomically to one of
// kDivSlots slots of kDivSlotWords words (one 64-byte line each, to spread
// the atomics), words [0] mass in units of 2^-24, [1] weight of the eligible
// sites, [2] divisions.  The kernel that turns them into the next step's rate
// clears them again.
constexpr int kDivSlots = 64, kDivSlotWords = 8;
constexpr double kFx = 16777216.0;      // 2^24: fixed-point unit of masses and weights
enum : int { kRegionAll = 0, kRegionFrontBand = 1, kRegionRearBand = 2 };
enum : uint32_t { kStDomainFull = 1u, kStNonFinite = 2u, kStSyncLost = 4u };

// A grid-wide barrier of a multi-step batch launch: arrivals of the current
// round, the round number, and a flag set when a wait ran out (zeroed
// before the first launch; the barrier leaves `count` at 0).
struct GridBar {
    uint32_t count;
    uint32_t gen;
    uint32_t err;
    uint32_t pad;
};

// Population layout.  Each row holds the padded width Lp = n_tiles * TW
// columns as n_tiles consecutive tiles; a tile stores the nq directions (9 on
// D2Q9, 7 on D2Q7) of TW consecutive columns one after the other
// ([tile][direction][column in tile]).  A wavefront's reads of one row are
// then a few contiguous runs instead of nq streams far apart.  TW is a power
// of two (64, 128 or 256 columns).
struct Tiles {
    int64_t rs;    // elements per row: nq * Lp
    int32_t tws;   // log2(TW)
    int32_t nq;    // populations per site
    __host__ __device__ int64_t col(int x) const
    {
        return ((int64_t)(x >> tws) * nq << tws) + (x & ((1 << tws) - 1));
    }
    __host__ __device__ int64_t at(int q, int64_t r, int x) const
    {
        return r * rs + col(x) + ((int64_t)q << tws);
    }
};

// Geometry of the LDS-staged form of the step for element size ES bytes.
// One wavefront owns SEG consecutive columns: each of its lanes copies one
// dword (two for float64) of every population row it needs into LDS, so a
// population row segment is 256 (float64: 512) bytes and a lane updates V
// sites.  Rows are held RING deep per wave; NW waves form a block.
struct StagedGeom {
    int es;
    __host__ __device__ constexpr StagedGeom(int e) : es(e) {}
    __host__ __device__ constexpr int dwords() const { return es == 8 ? 2 : 1; }
    __host__ __device__ constexpr int segb() const { return 256 * dwords(); }
    __host__ __device__ constexpr int seg() const { return segb() / es; }
    __host__ __device__ constexpr int sites() const { return seg() / 64; }
    __host__ __device__ constexpr int stage_bytes() const { return 9 * segb() + 256; }
    __host__ __device__ constexpr int loads() const { return 9 * dwords() + 1; }
    __host__ __device__ constexpr int ring() const { return es == 8 ? 3 : 4; }
    __host__ __device__ constexpr int waves() const { return es == 8 ? 2 : 4; }
};

// Device-resident run state (in the workspace).
struct DevState {
    int64_t  y_wall;        // absolute row of window row 0
    int64_t  y_valid_top;   // rows at or above this read as empty
    int64_t  n_rows;        // window rows the next step sweeps
    int64_t  h_hi;          // highest front height seen (device-driven modes)
    double   retired_total; // mass of rows left behind by the wall
    double   retired_last;  // ... by the last wall move
    uint32_t status;        // kSt* bits
    uint32_t pad;
    double   lam;           // division laws: expected divisions per unit weight this step
    double   p0;            // uniform division law: e^-min(lam, 8), no division at a site
    int64_t  divisions;     // divisions so far
    int64_t  rows_swept;    // sweep window: window rows the steps so far swept
    alignas(64) unsigned long long div_acc[kDivSlots][kDivSlotWords];
};

// Diagnostics record written by diag_kernel (layout of lbm_diag).
struct DiagOut {
    double   mass, src_total, fix_total, retired, hbar, W;
    int64_t  step, y_wall, h_hi;
    uint32_t status, reserved;
    double   lam;
    int64_t  divisions;
    int64_t  rows_swept;
};

template <class S>
struct StepArgs {
    using R = typename Real<S>::type;
    const S *fin;
    S *fout;
    const int32_t *h_prev;
    int32_t *h_next;
    int32_t *h_clear;       // slot to reset to the wall row (fixed modes), or null
    int32_t *colmax;        // per-column highest front
    double *partials;       // [nblocks][kPartialSlots]: mass, injected, fix, spare
    int32_t *divmap;        // [H][L] divisions per site (physical rows), or null
    DevState *st;
    int32_t L, H, ty;
    Tiles tl;
    int32_t mode, growth, region, region_width;
    int32_t noise;
    int32_t sround;         // 16-bit storage: stochastic rounding of tissue sites
    int32_t xcd_rows;       // row strips per run of tiles given to one XCD (0: none)
    int32_t strip_mul;      // > 1: each XCD visits its runs in the spread order (m mul) mod M;
                            // -1: XCDs 4-7 visit theirs from the top down
    uint32_t t, seed, replica;
    R omega, kmu, rho_c, g, sigma;
    R w[9];
    R Wd[9];
    double rho_cell, rho0;  // division laws: cell mass, density where division stops
    // A batch member stepped by its own launches inside the batch's graph:
    // its buffers, front-height slots and step counter come from its member
    // descriptor (a BatchRep<S>) in device memory, at step clock_k of the
    // run, so that a replayed graph steps on; null: from the fields above.
    const void *clock;
    int32_t clock_k;
};

template <class S>
struct InitArgs {
    using R = typename Real<S>::type;
    S *f;
    int32_t *h0;
    int32_t *colmax;
    double *partials;
    int32_t L, H, ty;
    Tiles tl;
    int32_t init_rows;
    int32_t cpt;            // columns per thread
    uint32_t seed, replica;
    double rho_init, init_amp, rho_c;
    double w[9];
    R Wd[9];
};

template <class S>
struct MassArgs {
    using R = typename Real<S>::type;
    const S *f;
    double *partials;
    DevState *st;           // (division laws: the tallies are added to its slots)
    const int32_t *h;       // front heights (division laws' front band)
    int32_t L, H, ty;
    int32_t cpt;            // columns per thread
    Tiles tl;
    int32_t growth, region, region_width;
    double rho_c, rho0;
    R Wd[9];
};

template <class S>
struct FinalizeArgs {
    using R = typename Real<S>::type;
    const S *f;             // state just written
    int32_t *h_next;        // its front heights
    int32_t *h_clear;       // slot of the step after next
    const int32_t *colmax;  // per-column highest front since creation
    DevState *st;
    int32_t L, H;
    Tiles tl;
    int32_t follow, window, min_gap;
    double w_factor;
    R Wd[9];
    int32_t *divmap;        // per-site divisions: rows the wall retires are cleared
    // division laws: the rate of the next step from the step's tallies
    int32_t growth;
    double g, rho_cell;
};

struct DiagArgs {
    const double *partials;
    int32_t nblocks;
    const int32_t *h_cur;
    const int32_t *colmax;
    int32_t L;
    DevState *st;
    DiagOut *out;
};

// One member of a batch: its static step and finalize parameters plus what
// the per-step fields are derived from.  Lives in the member's workspace.
template <class S>
struct BatchRep {
    StepArgs<S> a;          // per-step fields (fin, fout, h_*, t) unused
    FinalizeArgs<S> fa;     // per-step fields (f, h_next, h_clear) unused
    S *f[2];                // the two population buffers
    int32_t *hs[3];         // the three front-height slots
    int64_t t0;             // steps taken when the current batch run started
    int32_t cur0;           // buffer holding the state at that point
    int32_t gx;             // tiles along x
    int32_t ty;             // rows per tile
    int32_t nblocks;        // tiles in all
    int32_t device_driven;  // follow wall / sweep window: finalize each step
    int32_t window;         // sweep window: only tiles of live rows run
    int32_t last_live;      // tiles run by the last windowed launch
    int32_t pad2;
};

// Entry of a batch tile table: a run of n tiles of one member stacked in y
// (member index in its group, number of the run's lowest tile inside the
// member; tiles are numbered row strip major, x fastest).  A run is updated
// as one tile n row strips tall.
struct TileRef {
    int32_t rep;
    int32_t local0;
    int32_t n;
    int32_t pad;
};
// Rows per batch run (a member's row strips are grouped to about this many).
constexpr int kRowsPerRun = 4;
// Blocks of a windowed group's step launch.
constexpr int kWindowGrid = 8192;
__host__ __device__ inline int run_strips(int ty) { return ty >= kRowsPerRun ? 1 : kRowsPerRun / ty; }
// Runs of ry strips covering the first `strips` row strips of a member gx
// tiles wide.
__host__ __device__ inline int64_t run_count(int64_t strips, int gx, int ty, int ry = 0)
{
    if (ry <= 0) ry = run_strips(ty);
    return (strips + ry - 1) / ry * gx;
}
// Run l of those: its lowest tile and its height in strips.
__host__ __device__ inline TileRef run_ref(int rep, int64_t l, int64_t strips, int gx, int ty,
                                           int ry = 0)
{
    if (ry <= 0) ry = run_strips(ty);
    const int64_t by0 = (l / gx) * ry;
    const int64_t bx = l % gx;
    const int64_t n = strips - by0 < ry ? strips - by0 : ry;
    return TileRef{rep, (int32_t)(by0 * gx + bx), (int32_t)n, 0};
}

template <class S>
hipError_t launch_step(const StepArgs<S> &a, dim3 grid, int nt, int rb, hipStream_t s);
// The step on the D2Q7 lattice: vb bytes of columns per lane (4, 8, 16), or
// vb = 0 for one column per lane with rb rows' loads at once.
template <class S>
hipError_t launch_step7(const StepArgs<S> &a, dim3 grid, int nt, int vb, int rb, hipStream_t s);
// A batch group: n members with the same storage type and kernel form (div:
// the members grow by the division laws).
// reps: device array of member descriptors; table: the group's tiles;
// count: device word holding how many table entries the next launch runs.
// grid: blocks launched (each runs table entries blockIdx.x + i * grid).
// K steps (k .. k + K - 1) in one launch: with bar, a cooperative launch
// whose blocks meet at a grid-wide barrier between steps (grid must not
// exceed batch_coop_grid); without, K must be 1.
template <class S>
hipError_t launch_step_batch(BatchRep<S> *const *reps, const TileRef *table, const int32_t *count,
                             int grid, int vec, int nt, int vb_or_rb, int div, int sr, int k,
                             int K, GridBar *bar, hipStream_t s);
// Blocks of that kernel that fit the device at once (0 on failure).
template <class S>
int batch_coop_grid(int vec, int nt, int vb_or_rb, int div, int sr, int device);
// A windowed group whose tile table is rebuilt before each step: its n
// members' descriptors (BatchRep<S> pointers of one storage type) and where
// its table and entry count go.
struct PlanJob {
    void *const *reps;
    TileRef *table;
    int32_t *count;
    int32_t n;
    int32_t pad;
};
// Rebuild the tables of njobs windowed groups of storage type S (one block
// each) from their members' live rows.
template <class S>
hipError_t launch_plan_batch(const PlanJob *jobs, int njobs, hipStream_t s);
// Between-step work of the n members of a group (one block each).
template <class S>
hipError_t launch_finalize_batch(BatchRep<S> *const *reps, int n, int k, hipStream_t s);
template <class S>
hipError_t launch_batch_advance(BatchRep<S> *const *reps, int n, int K, hipStream_t s);
template <class S>
hipError_t launch_step_vec(const StepArgs<S> &a, dim3 grid, int nt, int vb, hipStream_t s);
// LDS-staged form: grid.x blocks of StagedGeom(sizeof(S)).waves() waves.
template <class S>
hipError_t launch_step_staged(const StepArgs<S> &a, dim3 grid, hipStream_t s);
template <class S>
hipError_t launch_init(const InitArgs<S> &a, dim3 grid, int nt, hipStream_t s);
template <class S>
hipError_t launch_mass(const MassArgs<S> &a, dim3 grid, int nt, hipStream_t s);
template <class S>
hipError_t launch_finalize(const FinalizeArgs<S> &a, hipStream_t s);
hipError_t launch_diag(const DiagArgs &a, hipStream_t s);
// Division laws: the rate of the next step from the tallies of a state set
// from outside (creation, lbm_set_populations), nothing retired.
hipError_t launch_rates(int growth, double g, double rho_cell, DevState *st, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// The static scratch of lbm_create_static: a file-scope device array of
// kStaticScratchBytes per device.  static_scratch_of finds the device the
// stream belongs to and that device's address of the array (looked up once
// per device, with the device current, and kept).
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch_of(hipStream_t s, int *device, void **ptr);
// Streaming copy of n 16-byte vectors (the benchmark's bandwidth reference).
hipError_t launch_stream_copy(void *dst, const void *src, int64_t n16, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_state_set(DevState *st, int64_t y_wall, int64_t y_valid_top, int64_t n_rows,
                            int64_t h_hi, hipStream_t s);

}  // namespace lbm
