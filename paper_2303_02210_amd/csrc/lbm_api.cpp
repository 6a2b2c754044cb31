// lbm_api.cpp -- C ABI of the gfx950 growing-tissue lattice Boltzmann library
// (declared in include/lbmgrow.h): parameter checks, workspace layout, launch
// configuration, host<->device transfers and error latching.
#include "lbmgrow.h"
#include "lbm_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// D2Q9 weights (rest, axes, diagonals).
const double kW[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
// D2Q7 weights (Sec. II): 1/2 at rest, 1/12 on each of the six directions.
const double kW7[9] = {1.0 / 2.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
                       1.0 / 12.0, 1.0 / 12.0, 0.0, 0.0};

int lattice_q(const lbm_params *p) { return p->lattice == LBM_LATTICE_D2Q7 ? 7 : 9; }
const double *lattice_w(const lbm_params *p) { return p->lattice == LBM_LATTICE_D2Q7 ? kW7 : kW; }

// ---- host float16 / bfloat16 conversions, round to nearest even --------------
uint16_t f32_to_f16(float f)
{
    uint32_t x;
    std::memcpy(&x, &f, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t ax = x & 0x7FFFFFFFu;
    if (ax >= 0x7F800000u) return (uint16_t)(sign | (ax > 0x7F800000u ? 0x7E00u : 0x7C00u));
    if (ax >= 0x477FF000u) return (uint16_t)(sign | 0x7C00u);      // rounds to infinity
    if (ax < 0x38800000u) {                                         // below 2^-14: subnormal
        float af;
        std::memcpy(&af, &ax, 4);
        const long r = std::lrintf(af * 16777216.0f);                 // multiples of 2^-24
        return (uint16_t)(sign | (uint32_t)r);
    }
    const uint32_t e = (ax >> 23) - 127u + 15u;
    const uint32_t m = ax & 0x7FFFFFu;
    uint32_t h = (e << 10) | (m >> 13);
    const uint32_t rem = m & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1u;
    return (uint16_t)(sign | h);
}

float f16_to_f32(uint16_t h)
{
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
    const uint32_t e = (h >> 10) & 0x1Fu;
    const uint32_t m = h & 0x3FFu;
    uint32_t x;
    if (e == 0) {
        const float v = (float)m * (1.0f / 16777216.0f);
        std::memcpy(&x, &v, 4);
        x |= sign;
    } else if (e == 31) {
        x = sign | 0x7F800000u | (m << 13);
    } else {
        x = sign | ((e - 15u + 127u) << 23) | (m << 13);
    }
    float f;
    std::memcpy(&f, &x, 4);
    return f;
}

uint16_t f32_to_bf16(float f)
{
    uint32_t x;
    std::memcpy(&x, &f, 4);
    if ((x & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((x >> 16) | 0x40u);
    x += 0x7FFFu + ((x >> 16) & 1u);
    return (uint16_t)(x >> 16);
}

float bf16_to_f32(uint16_t b)
{
    const uint32_t x = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &x, 4);
    return f;
}

size_t elem_bytes(int prec)
{
    switch (prec) {
    case LBM_FP64: return 8;
    case LBM_FP32: return 4;
    default: return 2;
    }
}

// Storage offset W_i = w_i rho_ref rounded to the storage type (0 when the
// storage holds f_i itself).
double offset_base(int prec, double w, double rho_ref)
{
    const float v = (float)(w * rho_ref);
    if (prec == LBM_FP16_OFFSET) return (double)f16_to_f32(f32_to_f16(v));
    if (prec == LBM_BF16_OFFSET) return (double)bf16_to_f32(f32_to_bf16(v));
    return 0.0;
}

struct Layout {
    size_t esize = 0;
    int64_t lp = 0;          // padded width (whole tiles)
    Tiles tl{};
    size_t nelem = 0;        // population elements per buffer
    size_t fbytes = 0;
    size_t off_f[2] = {0, 0};
    size_t off_h[3] = {0, 0, 0};
    size_t off_colmax = 0, off_partials = 0, off_state = 0, off_diag = 0, off_rep = 0;
    size_t off_divmap = 0;   // [H][L] int32 per-site divisions (0: not kept)
    size_t total = 0;
    int nt = 256, ty = 16, gx = 1, gy = 1, nblocks = 1, rb = 2;
    bool vec = false;   // vector kernel: vb bytes (cpt columns) per thread
    bool staged = false;  // LDS-staged kernel (same tiles as the vector form)
    int cpt = 1, vb = 16;
};

bool params_ok(const lbm_params *p, std::string *why)
{
    auto bad = [&](const char *m) {
        if (why) *why = m;
        return false;
    };
    if (!p) return bad("null params");
    if (p->abi_version != LBM_ABI_VERSION) return bad("abi_version mismatch");
    if (p->struct_size != sizeof(lbm_params)) return bad("struct_size mismatch");
    if (p->L < 2 || p->H < 4) return bad("L must be >= 2 and H >= 4");
    if (p->lattice != LBM_LATTICE_D2Q9 && p->lattice != LBM_LATTICE_D2Q7) return bad("bad lattice");
    // one padded row of populations is addressed with 32-bit byte offsets
    // (and with L bounded first, the product below cannot overflow)
    if (p->L > (1 << 24)) return bad("L must be <= 2^24");
    if ((int64_t)p->L * (int64_t)p->H * lattice_q(p) > (int64_t)1 << 31) return bad("lattice too large");
    if (p->precision < LBM_FP64 || p->precision > LBM_BF16_OFFSET) return bad("bad precision");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return bad("tau must be > 1/2");
    if (!(p->mu >= 0.0 && p->mu <= 1.0)) return bad("mu must be in [0, 1]");
    if (!(p->rho_c > 0.0) || !std::isfinite(p->rho_c)) return bad("rho_c must be > 0");
    if (!(p->rho_init >= 0.0) || !std::isfinite(p->rho_init)) return bad("rho_init must be >= 0");
    if (!(p->init_amp >= 0.0 && p->init_amp < 1.0)) return bad("init_amp must be in [0, 1)");
    if (p->init_rows < 0 || p->init_rows > p->H) return bad("init_rows out of range");
    if (p->growth < LBM_GROWTH_NONE || p->growth > LBM_GROWTH_DIVISION_DENSITY) return bad("bad growth");
    if (p->growth >= LBM_GROWTH_DIVISION && (!(p->rho_cell > 0.0) || !std::isfinite(p->rho_cell)))
        return bad("rho_cell must be > 0");
    if (p->growth == LBM_GROWTH_DIVISION_DENSITY && (!(p->rho0 > p->rho_c) || !std::isfinite(p->rho0)))
        return bad("rho0 must be > rho_c");
    if (!(p->growth_rate >= 0.0) || !std::isfinite(p->growth_rate)) return bad("growth_rate must be >= 0");
    if (p->region < LBM_REGION_ALL || p->region > LBM_REGION_REAR_BAND) return bad("bad region");
    if (p->region_width < 0) return bad("region_width must be >= 0");
    if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) return bad("sigma must be >= 0");
    if (p->ybc < LBM_Y_WALL_FIXED || p->ybc > LBM_Y_PERIODIC) return bad("bad ybc");
    if (p->ybc == LBM_Y_WALL_FOLLOW && (p->wall_min_gap < 0 || !(p->wall_w_factor >= 0.0)))
        return bad("bad wall follow parameters");
    if ((p->flags & ~(LBM_FLAG_WINDOW | LBM_FLAG_DIVISION_MAP | LBM_FLAG_STOCHASTIC_ROUND |
                      LBM_FLAG_BATCH_TABLE | LBM_FLAG_BATCH_OWN)) != 0)
        return bad("unknown flags");
    if ((p->flags & LBM_FLAG_BATCH_TABLE) && (p->flags & LBM_FLAG_BATCH_OWN))
        return bad("LBM_FLAG_BATCH_TABLE and LBM_FLAG_BATCH_OWN exclude each other");
    if ((p->flags & LBM_FLAG_STOCHASTIC_ROUND) &&
        p->precision != LBM_FP16_OFFSET && p->precision != LBM_BF16_OFFSET)
        return bad("stochastic rounding needs FP16 or BF16 offset storage");
    if ((p->flags & LBM_FLAG_STOCHASTIC_ROUND) && p->kernel_vb == 2)
        return bad("the LDS-staged form has no stochastic rounding");
    if (!(p->kernel_vb == 0 || p->kernel_vb == 1 || p->kernel_vb == 2 || p->kernel_vb == 4 ||
          p->kernel_vb == 8 || p->kernel_vb == 16))
        return bad("kernel_vb must be 0, 1, 2, 4, 8 or 16");
    if (p->kernel_ty < 0 || p->kernel_ty > 64) return bad("kernel_ty must be in [0, 64]");
    if (p->kernel_order < 0 || p->kernel_order > 4) return bad("kernel_order must be in [0, 4]");
    if ((p->flags & LBM_FLAG_WINDOW) && p->ybc == LBM_Y_PERIODIC)
        return bad("the sweep window needs a rear wall");
    if (p->lattice == LBM_LATTICE_D2Q7 && p->kernel_vb == 2)
        return bad("the D2Q7 step has no LDS-staged form (kernel_vb 2)");
    if (p->lattice == LBM_LATTICE_D2Q7 && p->ybc == LBM_Y_PERIODIC && p->H % 2 != 0)
        return bad("a periodic D2Q7 lattice needs an even number of rows");
    if ((p->precision == LBM_FP16_OFFSET || p->precision == LBM_BF16_OFFSET) &&
        (!(p->rho_ref >= 0.0) || !std::isfinite(p->rho_ref)))
        return bad("rho_ref must be >= 0");
    return true;
}

// A multiplier m coprime to M near M (3 - sqrt 5)/2: the sequence (k m) mod M
// then visits 0..M-1 with consecutive entries far apart and every stretch of
// it spread evenly over the range (the golden-ratio sequence).
int spread_multiplier(int M)
{
    if (M <= 2) return 0;
    int m = (int)std::lround(0.3819660112501051 * M);
    if (m < 1) m = 1;
    auto gcd = [](int a, int b) {
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        return a;
    };
    while (gcd(m, M) != 1) ++m;
    return m;
}

int pick_ty(int gx, int H, int pref, bool forced)
{
    if (forced) return pref;
    // rows per thread: the preferred count, fewer if that would leave the
    // device with under 2048 blocks (8 per CU)
    int t = pref;
    while (t > 1 && (int64_t)gx * ((H + t - 1) / t) < 2048) t /= 2;
    return t;
}

Layout make_layout(const lbm_params *p)
{
    Layout l;
    l.esize = elem_bytes(p->precision);
    // tile width: the largest of 256, 128, 64 columns that divides the width
    // rounded up to 64 (no padding beyond that)
    const int64_t l64 = (int64_t)align_up((size_t)p->L, 64);
    int tws = (l64 % 256 == 0) ? 8 : ((l64 % 128 == 0) ? 7 : 6);
    l.lp = (int64_t)align_up((size_t)p->L, (size_t)1 << tws);
    l.tl.tws = tws;
    l.tl.nq = lattice_q(p);
    l.tl.rs = (int64_t)l.tl.nq * l.lp;
    l.nelem = (size_t)l.tl.rs * (size_t)p->H;
    l.fbytes = align_up(l.nelem * l.esize, kAlign);
    // vector kernel when the columns split evenly into lanes; bytes per lane
    // and rows per thread as measured best on MI355X for a 4096 x 4096
    // lattice: float64 16 B / 1 row, float32 4 B / 1 row, 16-bit 4 B / 2 rows
    // (4 rows with a division law)
    l.vb = l.esize == 8 ? 16 : 4;
    int ty_pref = l.esize == 2 ? (p->growth >= LBM_GROWTH_DIVISION ? 4 : 2) : 1;
    bool scalar = false;
    if (p->kernel_vb == 1) scalar = true;                 // one column per lane
    // D2Q7 measured best at 4096 x 4096 in the vector form with 8 B per lane
    // for float64 and 4 B otherwise
    if (p->lattice == LBM_LATTICE_D2Q7 && p->kernel_vb == 0) l.vb = l.esize == 8 ? 8 : 4;
    else if (p->kernel_vb == 2) l.staged = true;          // rows staged through LDS
    else if (p->kernel_vb > 1) l.vb = p->kernel_vb;       // 4, 8 or 16 bytes per lane
    // the staged form moves 16-bit populations in pairs of columns
    if (l.staged && l.esize == 2 && p->L % 2 != 0) l.staged = false;
    if (l.staged) {
        // tiles of the vector form with one dword (float64: one site) per lane
        const StagedGeom G((int)l.esize);
        l.vb = G.sites() * (int)l.esize;
        ty_pref = 32;
    }
    if ((size_t)l.vb < l.esize) l.vb = (int)l.esize;
    if (p->kernel_ty > 0) ty_pref = p->kernel_ty;
    const int V = (int)(l.vb / l.esize);
    l.vec = !scalar && (p->L % V) == 0;
    l.cpt = l.vec ? V : 1;
    const int lanes = (p->L + l.cpt - 1) / l.cpt;
    l.nt = lanes <= 64 ? 64 : (lanes <= 128 ? 128 : 256);
    if (l.staged) l.nt = 64 * StagedGeom((int)l.esize).waves();
    l.gx = (lanes + l.nt - 1) / l.nt;
    // D2Q7, measured best at 4096 x 4096: float64 1 row per thread, the others
    // 2 rows (one column per lane, used when the width does not split into
    // vectors: float64 1 row, float32 2, 16-bit 4)
    if (p->lattice == LBM_LATTICE_D2Q7 && p->kernel_ty <= 0)
        ty_pref = l.esize == 8 ? 1 : (l.vec || l.esize == 4 ? 2 : 4);
    const bool pref_rows = l.vec || p->kernel_ty > 0 || p->lattice == LBM_LATTICE_D2Q7;
    l.ty = pick_ty(l.gx, p->H, pref_rows ? ty_pref : 2, p->kernel_ty > 0);
    l.gy = (p->H + l.ty - 1) / l.ty;
    l.rb = 2;
    l.nblocks = l.gx * l.gy;
    size_t o = 0;
    l.off_f[0] = o; o += l.fbytes;
    l.off_f[1] = o; o += l.fbytes;
    const size_t hb = align_up((size_t)p->L * 4, kAlign);
    for (int k = 0; k < 3; ++k) { l.off_h[k] = o; o += hb; }
    l.off_colmax = o; o += hb;
    l.off_partials = o; o += align_up((size_t)l.nblocks * kPartialSlots * 8, kAlign);
    l.off_state = o; o += align_up(sizeof(DevState), kAlign);
    l.off_diag = o; o += align_up(sizeof(DiagOut), kAlign);
    l.off_rep = o; o += align_up(sizeof(BatchRep<double>), kAlign);
    if (p->flags & LBM_FLAG_DIVISION_MAP) {
        l.off_divmap = o;
        o += align_up((size_t)p->L * (size_t)p->H * 4, kAlign);
    }
    l.total = o;
    return l;
}

}  // namespace

struct lbm_handle {
    lbm_params p{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;             // the two population buffers (and, unless
    size_t ws_bytes = 0;            // static, the scratch after them)
    char *scratch = nullptr;        // front heights, tallies, device state, ...
    int static_device = -1;         // device whose static scratch this handle holds
    Layout lay;
    int cur = 0;
    int64_t t = 0;
    int mode = kModeFixed;
    bool device_driven = false;
    bool moves = false;             // the wall follows or the sweep window is on
    int err = LBM_OK;
    std::string msg = "no error";
    double Wd[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    lbm_batch *batch = nullptr;     // batch this handle belongs to
    bool rep_ok = false;            // device descriptor matches (rep_t0, rep_cur0)
    int64_t rep_t0 = 0;
    int rep_cur0 = 0;

    // everything after the population buffers lives in the scratch area, at
    // its offset from the first front-height slot
    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(scratch + (off - lay.off_h[0])); }
    void *fbuf(int k) const { return ws + lay.off_f[k]; }
    int32_t *hslot(int64_t step) const { return at<int32_t>(lay.off_h[step % 3]); }
    int32_t *colmax() const { return at<int32_t>(lay.off_colmax); }
    double *partials() const { return at<double>(lay.off_partials); }
    DevState *st() const { return at<DevState>(lay.off_state); }
    DiagOut *diag() const { return at<DiagOut>(lay.off_diag); }
    int32_t *divmap() const { return lay.off_divmap ? at<int32_t>(lay.off_divmap) : nullptr; }

    int fail(int code, const std::string &m)
    {
        if (err == LBM_OK) {
            err = code;
            msg = m;
        }
        return code;
    }
    int hip(hipError_t e, const char *what)
    {
        if (e == hipSuccess) return LBM_OK;
        return fail(LBM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
};

namespace {

template <class S>
int do_init(lbm_handle *h)
{
    using R = typename Real<S>::type;
    const lbm_params &p = h->p;
    const Layout &l = h->lay;
    hipStream_t s = h->stream;
    int rc;
    // zero both population buffers' bookkeeping and every small array
    if ((rc = h->hip(launch_fill_i32(h->hslot(0), (int64_t)(l.off_partials - l.off_h[0]) / 4, 0, s),
                     "fill")))
        return rc;
    if ((rc = h->hip(launch_fill_f64(h->partials(), (int64_t)l.nblocks * kPartialSlots, 0.0, s), "fill")))
        return rc;
    if (h->divmap() &&
        (rc = h->hip(launch_fill_i32(h->divmap(), (int64_t)p.L * p.H, 0, s), "fill")))
        return rc;
    // the device state, division tallies and counts included
    if ((rc = h->hip(launch_fill_i32(reinterpret_cast<int32_t *>(h->st()),
                                     (int64_t)(sizeof(DevState) / 4), 0, s),
                     "fill")))
        return rc;
    if ((rc = h->hip(launch_state_set(h->st(), 0, p.H, p.H, 0, s), "state")))
        return rc;
    InitArgs<S> a{};
    a.f = reinterpret_cast<S *>(h->fbuf(0));
    a.h0 = h->hslot(0);
    a.colmax = h->colmax();
    a.partials = h->partials();
    a.L = p.L;
    a.H = p.H;
    a.ty = l.ty;
    a.tl = l.tl;
    a.init_rows = p.init_rows;
    a.cpt = l.cpt;
    a.seed = p.seed;
    a.replica = p.replica;
    a.rho_init = p.rho_init;
    a.init_amp = p.init_amp;
    a.rho_c = p.rho_c;
    for (int i = 0; i < 9; ++i) {
        a.w[i] = kW[i];
        a.Wd[i] = (R)h->Wd[i];
    }
    for (int i = 0; i < 9; ++i) a.w[i] = lattice_w(&p)[i];
    if ((rc = h->hip(launch_init<S>(a, dim3(l.gx, l.gy), l.nt, s), "init kernel"))) return rc;
    h->cur = 0;
    h->t = 0;
    // empty second buffer: rows never written read as empty through the
    // device window bookkeeping, but clear it so snapshots are clean
    // (a fill kernel rather than a memset: callers may capture this in a graph)
    return h->hip(launch_fill_i32(reinterpret_cast<int32_t *>(h->fbuf(1)), (int64_t)(l.fbytes / 4), 0, s),
                  "clear");
}

template <class S>
void fill_step_args(const lbm_handle *h, StepArgs<S> &a)
{
    using R = typename Real<S>::type;
    const lbm_params &p = h->p;
    const Layout &l = h->lay;
    a = StepArgs<S>{};
    a.partials = h->partials();
    a.divmap = h->divmap();
    a.colmax = h->colmax();
    a.st = h->st();
    a.L = p.L;
    a.H = p.H;
    a.ty = l.ty;
    a.tl = l.tl;
    a.mode = h->mode;
    a.growth = p.growth;
    a.region = p.region;
    a.region_width = p.region_width;
    a.noise = p.sigma > 0.0;
    a.sround = (p.flags & LBM_FLAG_STOCHASTIC_ROUND) != 0;
    a.xcd_rows = 1;   // one row strip of tiles per run (measured best)
    // default: two sweeps for the D2Q9 step without a division law in blocks
    // of up to 4 rows, from the wall up otherwise (measured best on each)
    const int order = p.kernel_order ? p.kernel_order
                      : (l.tl.nq == 9 && p.growth < LBM_GROWTH_DIVISION && l.ty <= 4) ? 4 : 1;
    a.strip_mul = (order == 2) ? spread_multiplier(l.gy / 8)
                  : (order == 3) ? -1
                  : (order == 4) ? -2 : 0;
    a.seed = p.seed;
    a.replica = p.replica;
    a.omega = (R)(1.0 / p.tau);
    a.kmu = (R)(1.0 - p.mu);
    a.rho_c = (R)p.rho_c;
    a.g = (R)p.growth_rate;
    a.sigma = (R)p.sigma;
    a.rho_cell = p.rho_cell;
    a.rho0 = p.rho0;
    for (int i = 0; i < 9; ++i) {
        a.w[i] = (R)lattice_w(&p)[i];
        a.Wd[i] = (R)h->Wd[i];
    }
}

template <class S>
void fill_finalize_args(const lbm_handle *h, FinalizeArgs<S> &fa)
{
    using R = typename Real<S>::type;
    const lbm_params &p = h->p;
    fa = FinalizeArgs<S>{};
    fa.st = h->st();
    fa.divmap = h->divmap();
    fa.colmax = h->colmax();
    fa.L = p.L;
    fa.H = p.H;
    fa.tl = h->lay.tl;
    fa.follow = p.ybc == LBM_Y_WALL_FOLLOW;
    fa.window = (p.flags & LBM_FLAG_WINDOW) != 0;
    fa.min_gap = p.wall_min_gap;
    fa.w_factor = p.wall_w_factor;
    for (int i = 0; i < 9; ++i) fa.Wd[i] = (R)h->Wd[i];
    fa.growth = p.growth;
    fa.g = p.growth_rate;
    fa.rho_cell = p.rho_cell;
}

template <class S>
int do_step(lbm_handle *h, int64_t n)
{
    const Layout &l = h->lay;
    StepArgs<S> a;
    fill_step_args<S>(h, a);
    FinalizeArgs<S> fa;
    fill_finalize_args<S>(h, fa);

    const dim3 grid(l.gx, l.gy);
    for (int64_t k = 0; k < n; ++k) {
        a.fin = reinterpret_cast<const S *>(h->fbuf(h->cur));
        a.fout = reinterpret_cast<S *>(h->fbuf(h->cur ^ 1));
        a.h_prev = h->hslot(h->t);
        a.h_next = h->hslot(h->t + 1);
        a.h_clear = h->moves ? nullptr : h->hslot(h->t + 2);
        a.t = (uint32_t)h->t;
        int rc = h->hip(l.tl.nq == 7 ? launch_step7<S>(a, grid, l.nt, l.vec ? l.vb : 0, l.rb, h->stream)
                        : l.staged ? launch_step_staged<S>(a, grid, h->stream)
                        : l.vec    ? launch_step_vec<S>(a, grid, l.nt, l.vb, h->stream)
                                   : launch_step<S>(a, grid, l.nt, l.rb, h->stream),
                        "step kernel");
        if (rc) return rc;
        if (h->device_driven && !h->moves) {
            // division law, wall and window fixed: only the next rate
            rc = h->hip(launch_rates(h->p.growth, h->p.growth_rate, h->p.rho_cell, h->st(),
                                     h->stream),
                        "rates kernel");
            if (rc) return rc;
        } else if (h->device_driven) {
            fa.f = a.fout;
            fa.h_next = h->hslot(h->t + 1);
            fa.h_clear = h->hslot(h->t + 2);
            rc = h->hip(launch_finalize<S>(fa, h->stream), "finalize kernel");
            if (rc) return rc;
        }
        h->cur ^= 1;
        h->t += 1;
    }
    return LBM_OK;
}

template <class S>
int do_mass(lbm_handle *h)
{
    using R = typename Real<S>::type;
    MassArgs<S> a{};
    a.f = reinterpret_cast<const S *>(h->fbuf(h->cur));
    a.partials = h->partials();
    a.st = h->st();
    a.L = h->p.L;
    a.H = h->p.H;
    a.ty = h->lay.ty;
    a.cpt = h->lay.cpt;
    a.tl = h->lay.tl;
    a.h = h->hslot(h->t);
    a.growth = h->p.growth;
    a.region = h->p.region;
    a.region_width = h->p.region_width;
    a.rho_c = h->p.rho_c;
    a.rho0 = h->p.rho0;
    for (int i = 0; i < 9; ++i) a.Wd[i] = (R)h->Wd[i];
    int rc = h->hip(launch_mass<S>(a, dim3(h->lay.gx, h->lay.gy), h->lay.nt, h->stream),
                    "mass kernel");
    if (rc || h->p.growth < LBM_GROWTH_DIVISION) return rc;
    // division laws: the next step's rate from this state
    return h->hip(launch_rates(h->p.growth, h->p.growth_rate, h->p.rho_cell, h->st(), h->stream),
                  "rates kernel");
}

#define LBM_DISPATCH(prec, fn, ...)                                   \
    ((prec) == LBM_FP64   ? fn<double>(__VA_ARGS__)                    \
     : (prec) == LBM_FP32 ? fn<float>(__VA_ARGS__)                     \
     : (prec) == LBM_FP16_OFFSET ? fn<__half>(__VA_ARGS__)             \
                                 : fn<__hip_bfloat16>(__VA_ARGS__))

int usable(lbm_handle *h)
{
    if (!h) return LBM_E_INVALID;
    if (h->err != LBM_OK) return LBM_E_STATE;
    return LBM_OK;
}

int sync_and_check(lbm_handle *h)
{
    uint32_t status = 0;
    int rc = h->hip(hipMemcpyAsync(&status, &h->st()->status, sizeof(status),
                                   hipMemcpyDeviceToHost, h->stream),
                    "status copy");
    if (rc) return rc;
    if ((rc = h->hip(hipStreamSynchronize(h->stream), "synchronize"))) return rc;
    if (status & kStDomainFull) return h->fail(LBM_E_DOMAIN_FULL, "front reached the top row of the window");
    if (status & kStNonFinite) return h->fail(LBM_E_NONFINITE, "total mass is not finite");
    if (status & kStSyncLost) return h->fail(LBM_E_DEVICE, "a batch launch's grid barrier gave up");
    return LBM_OK;
}

double decode_one(int prec, const char *base, size_t idx, double Wd)
{
    switch (prec) {
    case LBM_FP64: {
        double v;
        std::memcpy(&v, base + idx * 8, 8);
        return v;
    }
    case LBM_FP32: {
        float v;
        std::memcpy(&v, base + idx * 4, 4);
        return (double)v;
    }
    case LBM_FP16_OFFSET: {
        uint16_t v;
        std::memcpy(&v, base + idx * 2, 2);
        return (double)(f16_to_f32(v) + (float)Wd);
    }
    default: {
        uint16_t v;
        std::memcpy(&v, base + idx * 2, 2);
        return (double)(bf16_to_f32(v) + (float)Wd);
    }
    }
}

void encode_one(int prec, char *base, size_t idx, double f, double Wd)
{
    switch (prec) {
    case LBM_FP64:
        std::memcpy(base + idx * 8, &f, 8);
        break;
    case LBM_FP32: {
        const float v = (float)f;
        std::memcpy(base + idx * 4, &v, 4);
        break;
    }
    case LBM_FP16_OFFSET: {
        const uint16_t v = f32_to_f16((float)f - (float)Wd);
        std::memcpy(base + idx * 2, &v, 2);
        break;
    }
    default: {
        const uint16_t v = f32_to_bf16((float)f - (float)Wd);
        std::memcpy(base + idx * 2, &v, 2);
        break;
    }
    }
}

int read_state(lbm_handle *h, DevState *out)
{
    int rc = h->hip(hipMemcpyAsync(out, h->st(), sizeof(DevState), hipMemcpyDeviceToHost, h->stream),
                    "state copy");
    if (rc) return rc;
    return h->hip(hipStreamSynchronize(h->stream), "synchronize");
}

// State blob: header, current populations, current h slot, column maxima,
// block partials and the device state.
struct BlobHeader {
    uint64_t magic;
    lbm_params p;
    int64_t t;
    uint64_t fbytes, hbytes, pbytes;
};
constexpr uint64_t kMagic = 0x31626C6D62676C6Cull;

// One live handle per device may use that device's static scratch; the host
// side of those handles is static too, so creating one allocates nothing.
std::mutex g_static_mu;
bool g_static_taken[kMaxDevices] = {};
lbm_handle g_static_handles[kMaxDevices];

bool claim_static(int dev)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (dev < 0 || dev >= kMaxDevices || g_static_taken[dev]) return false;
    g_static_taken[dev] = true;
    return true;
}

void release_static(int dev)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (dev >= 0 && dev < kMaxDevices) g_static_taken[dev] = false;
}

// The handle over populations `pops` (two buffers) and scratch `scr` (the
// rest of the layout, from the first front-height slot on): initial state
// and, for the division laws, the first step's rate.
int create_handle(const lbm_params *p, const Layout &lay, char *pops, size_t pops_bytes,
                  char *scr, int static_device, void *hip_stream, lbm_handle **out)
{
    lbm_handle *h;
    if (static_device >= 0) {
        h = &g_static_handles[static_device];
        *h = lbm_handle();
    } else if (!(h = new (std::nothrow) lbm_handle())) {
        return LBM_E_NOMEM;
    }
    h->p = *p;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->ws = pops;
    h->ws_bytes = pops_bytes;
    h->scratch = scr;
    h->static_device = static_device;
    h->lay = lay;
    // Work between steps: the full finalize when the wall or the window
    // moves; otherwise, under a division law, only the next rate from the
    // step's tallies (rates_kernel).
    h->moves = p->ybc == LBM_Y_WALL_FOLLOW || (p->flags & LBM_FLAG_WINDOW);
    h->device_driven = h->moves || p->growth >= LBM_GROWTH_DIVISION;
    h->mode = p->ybc == LBM_Y_PERIODIC ? kModePeriodic : (h->device_driven ? kModeDevice : kModeFixed);
    for (int i = 0; i < 9; ++i) h->Wd[i] = offset_base(p->precision, lattice_w(p)[i], p->rho_ref);
    int rc = LBM_DISPATCH(p->precision, do_init, h);
    if (rc == LBM_OK && h->device_driven) {
        // rows the first step must sweep: the initial front (at most
        // init_rows) plus one; every row above is empty
        int64_t nr = (p->flags & LBM_FLAG_WINDOW) ? std::min<int64_t>(p->H, p->init_rows + 2) : p->H;
        if (nr < 1) nr = 1;
        rc = h->hip(launch_state_set(h->st(), 0, p->H, nr, 0, h->stream), "state");
    }
    if (rc == LBM_OK && p->growth >= LBM_GROWTH_DIVISION)
        rc = LBM_DISPATCH(p->precision, do_mass, h);   // the first step's division rate
    if (rc != LBM_OK) {
        if (static_device < 0) delete h;
        return rc;
    }
    *out = h;
    return LBM_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

#ifndef LBM_SOURCE_HASH
#define LBM_SOURCE_HASH "unknown"
#endif
const char *lbm_version(void) { return "lbmgrow 1.1 gfx950 src " LBM_SOURCE_HASH; }

size_t lbm_workspace_bytes(const lbm_params *p)
{
    if (!params_ok(p, nullptr)) return 0;
    return make_layout(p).total;
}

int lbm_create(const lbm_params *p, void *dev_ws, size_t ws_bytes, void *hip_stream,
               lbm_handle **out)
{
    if (!out) return LBM_E_INVALID;
    *out = nullptr;
    if (!params_ok(p, nullptr)) return LBM_E_INVALID;
    if (!dev_ws || (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0) return LBM_E_INVALID;
    const Layout lay = make_layout(p);
    if (ws_bytes < lay.total) return LBM_E_NOMEM;
    char *ws = reinterpret_cast<char *>(dev_ws);
    return create_handle(p, lay, ws, ws_bytes, ws + lay.off_h[0], -1, hip_stream, out);
}

int lbm_create_static(const lbm_params *p, void *dev_pops, size_t *pops_bytes, void *hip_stream,
                      lbm_handle **out)
{
    if (!pops_bytes) return LBM_E_INVALID;
    if (!params_ok(p, nullptr)) return LBM_E_INVALID;
    const Layout lay = make_layout(p);
    const size_t need = lay.off_h[0];                 // the two population buffers
    if (lay.total - lay.off_h[0] > kStaticScratchBytes) return LBM_E_NOMEM;
    if (!dev_pops) {                                  // size query
        *pops_bytes = need;
        return LBM_OK;
    }
    if (!out) return LBM_E_INVALID;
    *out = nullptr;
    if ((reinterpret_cast<uintptr_t>(dev_pops) % kAlign) != 0) return LBM_E_INVALID;
    if (*pops_bytes < need) return LBM_E_NOMEM;
    int dev = -1;
    void *scr = nullptr;
    if (static_scratch_of(reinterpret_cast<hipStream_t>(hip_stream), &dev, &scr) != hipSuccess)
        return LBM_E_DEVICE;
    if (!claim_static(dev)) return LBM_E_NOMEM;       // another live handle holds it
    const int rc = create_handle(p, lay, reinterpret_cast<char *>(dev_pops), *pops_bytes,
                                 reinterpret_cast<char *>(scr), dev, hip_stream, out);
    if (rc != LBM_OK) release_static(dev);
    return rc;
}

int lbm_step(lbm_handle *h, int64_t nsteps)
{
    int rc = usable(h);
    if (rc) return rc;
    if (nsteps < 0) return LBM_E_INVALID;
    return LBM_DISPATCH(h->p.precision, do_step, h, nsteps);
}

int lbm_front_heights(lbm_handle *h, int32_t *host_h, int64_t *step_out)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_h) return LBM_E_INVALID;
    rc = h->hip(hipMemcpyAsync(host_h, h->hslot(h->t), (size_t)h->p.L * 4, hipMemcpyDeviceToHost,
                               h->stream),
                "front heights copy");
    if (rc) return rc;
    if (step_out) *step_out = h->t;
    return sync_and_check(h);
}

int lbm_front_heights_async(lbm_handle *h, int32_t *dst)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!dst) return LBM_E_INVALID;
    return h->hip(hipMemcpyAsync(dst, h->hslot(h->t), (size_t)h->p.L * 4, hipMemcpyDefault,
                                 h->stream),
                  "front heights copy");
}

int lbm_diagnostics(lbm_handle *h, lbm_diag *out)
{
    if (!h || !out) return LBM_E_INVALID;
    DiagArgs a{};
    a.partials = h->partials();
    a.nblocks = h->lay.nblocks;
    a.h_cur = h->hslot(h->t);
    a.colmax = h->colmax();
    a.L = h->p.L;
    a.st = h->st();
    a.out = h->diag();
    int rc = h->hip(launch_diag(a, h->stream), "diag kernel");
    if (rc) return rc;
    DiagOut d{};
    rc = h->hip(hipMemcpyAsync(&d, h->diag(), sizeof(d), hipMemcpyDeviceToHost, h->stream),
                "diag copy");
    if (rc) return rc;
    if ((rc = h->hip(hipStreamSynchronize(h->stream), "synchronize"))) return rc;
    out->mass = d.mass;
    out->src_total = d.src_total;
    out->fix_total = d.fix_total;
    out->retired = d.retired;
    out->hbar = d.hbar;
    out->W = d.W;
    out->step = h->t;
    out->y_wall = d.y_wall;
    out->h_hi = d.h_hi;
    out->status = d.status;
    out->reserved = 0;
    out->lam = d.lam;
    out->divisions = d.divisions;
    // a run without the sweep window sweeps all H rows every step
    out->rows_swept = (h->p.flags & LBM_FLAG_WINDOW) ? d.rows_swept : h->t * (int64_t)h->p.H;
    if (d.status & kStDomainFull) h->fail(LBM_E_DOMAIN_FULL, "front reached the top row of the window");
    if (d.status & kStNonFinite) h->fail(LBM_E_NONFINITE, "total mass is not finite");
    if (d.status & kStSyncLost) h->fail(LBM_E_DEVICE, "a batch launch's grid barrier gave up");
    return LBM_OK;
}

int lbm_get_populations(lbm_handle *h, double *host_f)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_f) return LBM_E_INVALID;
    const Layout &l = h->lay;
    const lbm_params &p = h->p;
    std::vector<char> raw(l.nelem * l.esize);
    rc = h->hip(hipMemcpyAsync(raw.data(), h->fbuf(h->cur), raw.size(), hipMemcpyDeviceToHost,
                               h->stream),
                "populations copy");
    if (rc) return rc;
    DevState st{};
    if ((rc = read_state(h, &st))) return rc;
    const bool ring = h->mode == kModeDevice;
    for (int q = 0; q < l.tl.nq; ++q)
        for (int j = 0; j < p.H; ++j) {
            const int64_t y = st.y_wall + j;
            const bool valid = h->mode == kModePeriodic || y < st.y_valid_top;
            const int64_t r = ring ? (y % p.H) : j;
            for (int x = 0; x < p.L; ++x) {
                const size_t o = ((size_t)q * p.H + j) * p.L + x;
                host_f[o] = valid ? decode_one(p.precision, raw.data(), (size_t)l.tl.at(q, r, x),
                                               h->Wd[q])
                                  : 0.0;
            }
        }
    return LBM_OK;
}

int lbm_set_populations(lbm_handle *h, const double *host_f)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_f) return LBM_E_INVALID;
    const Layout &l = h->lay;
    const lbm_params &p = h->p;
    DevState st{};
    if ((rc = read_state(h, &st))) return rc;
    std::vector<char> raw(l.nelem * l.esize, 0);
    const bool ring = h->mode == kModeDevice;
    for (int q = 0; q < l.tl.nq; ++q)
        for (int j = 0; j < p.H; ++j) {
            const int64_t y = st.y_wall + j;
            const int64_t r = ring ? (y % p.H) : j;
            for (int x = 0; x < p.L; ++x)
                encode_one(p.precision, raw.data(), (size_t)l.tl.at(q, r, x),
                           host_f[((size_t)q * p.H + j) * p.L + x], h->Wd[q]);
        }
    rc = h->hip(hipMemcpyAsync(h->fbuf(h->cur), raw.data(), raw.size(), hipMemcpyHostToDevice,
                               h->stream),
                "populations copy");
    if (rc) return rc;
    // every row of the window is now live
    const int64_t hi = st.y_wall + p.H;
    if ((rc = h->hip(launch_state_set(h->st(), st.y_wall, st.y_wall + p.H, p.H,
                                      h->device_driven ? hi : st.h_hi, h->stream),
                     "state")))
        return rc;
    if ((rc = LBM_DISPATCH(p.precision, do_mass, h))) return rc;
    return h->hip(hipStreamSynchronize(h->stream), "synchronize");
}

int lbm_set_front_heights(lbm_handle *h, const int32_t *host_h)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_h) return LBM_E_INVALID;
    rc = h->hip(hipMemcpyAsync(h->hslot(h->t), host_h, (size_t)h->p.L * 4, hipMemcpyHostToDevice,
                               h->stream),
                "front heights copy");
    if (rc) return rc;
    // the division laws' eligible sites may depend on the front (front band)
    if (h->p.growth >= LBM_GROWTH_DIVISION && (rc = LBM_DISPATCH(h->p.precision, do_mass, h)))
        return rc;
    return h->hip(hipStreamSynchronize(h->stream), "synchronize");
}

int lbm_division_map(lbm_handle *h, int32_t *host_counts, int clear)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_counts || !h->divmap()) return LBM_E_INVALID;
    const lbm_params &p = h->p;
    std::vector<int32_t> raw((size_t)p.L * p.H);
    rc = h->hip(hipMemcpyAsync(raw.data(), h->divmap(), raw.size() * 4, hipMemcpyDeviceToHost,
                               h->stream),
                "division map copy");
    if (rc) return rc;
    if (clear && (rc = h->hip(launch_fill_i32(h->divmap(), (int64_t)p.L * p.H, 0, h->stream),
                              "fill")))
        return rc;
    DevState st{};
    if ((rc = read_state(h, &st))) return rc;   // (synchronizes the stream)
    // window row j holds absolute row y_wall + j at physical row (y_wall + j) mod H
    const bool ring = h->mode == kModeDevice;
    for (int j = 0; j < p.H; ++j) {
        const int64_t r = ring ? (st.y_wall + j) % p.H : j;
        std::memcpy(host_counts + (size_t)j * p.L, raw.data() + (size_t)r * p.L, (size_t)p.L * 4);
    }
    return LBM_OK;
}

size_t lbm_state_bytes(const lbm_handle *h)
{
    if (!h) return 0;
    const Layout &l = h->lay;
    return sizeof(BlobHeader) + l.nelem * l.esize + 2 * (size_t)h->p.L * 4 +
           (size_t)l.nblocks * kPartialSlots * 8 + sizeof(DevState);
}

int lbm_get_state(lbm_handle *h, void *host_blob, size_t bytes)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_blob) return LBM_E_INVALID;
    if (bytes < lbm_state_bytes(h)) return LBM_E_NOMEM;
    const Layout &l = h->lay;
    char *b = reinterpret_cast<char *>(host_blob);
    BlobHeader hd{};
    hd.magic = kMagic;
    hd.p = h->p;
    hd.t = h->t;
    hd.fbytes = (uint64_t)(l.nelem * l.esize);
    hd.hbytes = (uint64_t)h->p.L * 4;
    hd.pbytes = (uint64_t)l.nblocks * kPartialSlots * 8;
    std::memcpy(b, &hd, sizeof hd);
    size_t o = sizeof hd;
    struct Piece {
        const void *src;
        size_t n;
    } pieces[] = {{h->fbuf(h->cur), hd.fbytes},
                  {h->hslot(h->t), hd.hbytes},
                  {h->colmax(), hd.hbytes},
                  {h->partials(), hd.pbytes},
                  {h->st(), sizeof(DevState)}};
    for (const Piece &pc : pieces) {
        if ((rc = h->hip(hipMemcpyAsync(b + o, pc.src, pc.n, hipMemcpyDeviceToHost, h->stream),
                         "state copy")))
            return rc;
        o += pc.n;
    }
    return h->hip(hipStreamSynchronize(h->stream), "synchronize");
}

int lbm_set_state(lbm_handle *h, const void *host_blob, size_t bytes)
{
    int rc = usable(h);
    if (rc) return rc;
    if (!host_blob) return LBM_E_INVALID;
    if (bytes < lbm_state_bytes(h)) return LBM_E_NOMEM;
    const Layout &l = h->lay;
    const char *b = reinterpret_cast<const char *>(host_blob);
    BlobHeader hd;
    std::memcpy(&hd, b, sizeof hd);
    // (how a batch steps the run does not change its state)
    lbm_params saved = hd.p, mine = h->p;
    saved.flags &= ~(int32_t)(LBM_FLAG_BATCH_TABLE | LBM_FLAG_BATCH_OWN);
    mine.flags &= ~(int32_t)(LBM_FLAG_BATCH_TABLE | LBM_FLAG_BATCH_OWN);
    if (hd.magic != kMagic || std::memcmp(&saved, &mine, sizeof(lbm_params)) != 0 ||
        hd.fbytes != (uint64_t)(l.nelem * l.esize))
        return LBM_E_INVALID;
    h->t = hd.t;
    size_t o = sizeof hd;
    struct Piece {
        void *dst;
        size_t n;
    } pieces[] = {{h->fbuf(h->cur), hd.fbytes},
                  {h->hslot(h->t), hd.hbytes},
                  {h->colmax(), hd.hbytes},
                  {h->partials(), hd.pbytes},
                  {h->st(), sizeof(DevState)}};
    for (const Piece &pc : pieces) {
        if ((rc = h->hip(hipMemcpyAsync(pc.dst, b + o, pc.n, hipMemcpyHostToDevice, h->stream),
                         "state copy")))
            return rc;
        o += pc.n;
    }
    // the next step's front-height slot starts at the wall row
    DevState st;
    std::memcpy(&st, b + o - sizeof(DevState), sizeof st);
    if ((rc = h->hip(launch_fill_i32(h->hslot(h->t + 1), h->p.L, (int32_t)st.y_wall, h->stream),
                     "fill")))
        return rc;
    if (!h->device_driven &&
        (rc = h->hip(launch_fill_i32(h->hslot(h->t + 2), h->p.L, 0, h->stream), "fill")))
        return rc;
    return h->hip(hipStreamSynchronize(h->stream), "synchronize");
}

int lbm_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (!dst || !src || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) % 16) != 0 ||
        (reinterpret_cast<uintptr_t>(src) % 16) != 0)
        return LBM_E_INVALID;
    const char *d = reinterpret_cast<const char *>(dst), *sp = reinterpret_cast<const char *>(src);
    if (d < sp + bytes && sp < d + bytes && bytes > 0) return LBM_E_INVALID;   // overlap
    return launch_stream_copy(dst, src, (int64_t)(bytes / 16),
                              reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess
               ? LBM_OK
               : LBM_E_DEVICE;
}

const char *lbm_last_error(const lbm_handle *h)
{
    if (!h) return "null handle";
    return h->msg.c_str();
}

int lbm_destroy(lbm_handle *h)
{
    if (!h) return LBM_E_INVALID;
    if (h->batch) lbm_batch_remove(h->batch, h);
    if (h->static_device >= 0) {
        // the next handle on this device reuses the scratch: let this
        // handle's work finish first
        (void)hipStreamSynchronize(h->stream);
        const int dev = h->static_device;
        *h = lbm_handle();
        release_static(dev);
        return LBM_OK;
    }
    delete h;
    return LBM_OK;
}

}  // extern "C"
// ============================================================================
// Batches
// ============================================================================
namespace {

constexpr int kMaxGroups = 16;

// Members of at least this many sites that neither move their wall or
// window nor grow by a division law are stepped by their own launches inside
// the batch's graph (LBM_FLAG_BATCH_OWN / LBM_FLAG_BATCH_TABLE override it):
// a step of such a member keeps the GPU busy long enough for its launch to
// cost nothing, and the solo kernels run it faster than the shared table.
constexpr int64_t kOwnSites = (int64_t)1 << 22;

bool steps_on_its_own(const lbm_handle *h)
{
    if (h->device_driven) return false;
    if (h->p.flags & LBM_FLAG_BATCH_TABLE) return false;
    if (h->p.flags & LBM_FLAG_BATCH_OWN) return true;
    return (int64_t)h->p.L * h->p.H >= kOwnSites;
}

struct BatchGroup {
    // kernel form; form: 0 one column per lane, 1 vector, 2 the D2Q7 step;
    // own: the members are stepped by their own launches (no tile table)
    int prec = 0, form = 0, nt = 0, vbrb = 0, ty = 0, windowed = 0, div = 0, sr = 0, own = 0;
    std::vector<lbm_handle *> m;
    int64_t tiles = 0;                           // tiles over all members
    int grid = 0;                                // blocks per step launch
    int ndev = 0;                                // members finalized each step
    void **reps = nullptr;                       // device: descriptor pointers
    int32_t *count = nullptr;                    // device: table entries to run
    TileRef *table = nullptr;                    // device: the group's tiles
    PlanJob *job = nullptr;                      // device: its table's plan (windowed)
    GridBar *bar = nullptr;                      // device: barrier of multi-step launches
    int coop_grid = 0;                           // blocks of a multi-step launch (0: none)
};

size_t batch_slot_bytes(int max_members)
{
    return align_up((size_t)max_members * sizeof(void *), kAlign) + kAlign;
}

// Workspace: one slot per group (its descriptor pointers, then in the last
// kAlign bytes its table's entry count and plan job), then the tile tables.
constexpr size_t kPlanJobOffset = 64;   // within the last kAlign bytes of a slot
constexpr size_t kGridBarOffset = 128;
static_assert(kPlanJobOffset + sizeof(PlanJob) <= kGridBarOffset &&
                  kGridBarOffset + sizeof(GridBar) <= kAlign,
              "plan job and barrier fit the slot's tail");
size_t batch_table_offset(int max_members) { return kMaxGroups * batch_slot_bytes(max_members); }

template <class S>
int write_rep(lbm_handle *h)
{
    BatchRep<S> r{};
    fill_step_args<S>(h, r.a);
    fill_finalize_args<S>(h, r.fa);
    r.f[0] = reinterpret_cast<S *>(h->fbuf(0));
    r.f[1] = reinterpret_cast<S *>(h->fbuf(1));
    for (int k = 0; k < 3; ++k) r.hs[k] = h->at<int32_t>(h->lay.off_h[k]);
    r.t0 = h->t;
    r.cur0 = h->cur;
    r.gx = h->lay.gx;
    r.ty = h->lay.ty;
    r.nblocks = h->lay.nblocks;
    r.device_driven = h->device_driven ? 1 : 0;
    r.window = (h->p.flags & LBM_FLAG_WINDOW) ? 1 : 0;
    r.last_live = h->lay.nblocks;   // first windowed launch clears every idle tile
    int rc = h->hip(hipMemcpyAsync(h->at<char>(h->lay.off_rep), &r, sizeof r, hipMemcpyHostToDevice,
                                   h->stream),
                    "batch descriptor copy");
    if (rc) return rc;
    // the copy reads r: wait for it before r goes out of scope
    rc = h->hip(hipStreamSynchronize(h->stream), "synchronize");
    if (rc) return rc;
    h->rep_ok = true;
    h->rep_t0 = h->t;
    h->rep_cur0 = h->cur;
    return LBM_OK;
}

// n steps of a member with its own launches: its solo kernel, the per-step
// inputs read from its descriptor at steps 0..n-1 of the run.  The steps of
// one member go back to back, so a member whose state is not much larger
// than the 256 MB last-level cache finds part of it there at the next step.
template <class S>
hipError_t enqueue_own_member(lbm_handle *h, int n, hipStream_t s)
{
    const Layout &l = h->lay;
    StepArgs<S> a;
    fill_step_args<S>(h, a);
    a.clock = h->at<char>(l.off_rep);
    const dim3 grid(l.gx, l.gy);
    for (int k = 0; k < n; ++k) {
        a.clock_k = k;
        const hipError_t e =
            l.tl.nq == 7 ? launch_step7<S>(a, grid, l.nt, l.vec ? l.vb : 0, l.rb, s)
            : l.staged   ? launch_step_staged<S>(a, grid, s)
            : l.vec      ? launch_step_vec<S>(a, grid, l.nt, l.vb, s)
                         : launch_step<S>(a, grid, l.nt, l.rb, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// n steps of a table group: per step its table (windowed groups), the step,
// and the between-step work of its device-driven members.  (Building the
// next step's table inside the between-step launch, by its last block to
// finish, measured slower: that hand-over needs device-wide cache write-backs.)
// persist: a group with neither (coop_grid set) runs all n steps in one
// cooperative launch.
template <class S>
hipError_t enqueue_group(const BatchGroup &g, int n, bool persist, hipStream_t s)
{
    BatchRep<S> *const *reps = reinterpret_cast<BatchRep<S> *const *>(g.reps);
    if (persist && g.coop_grid > 0)
        return launch_step_batch<S>(reps, g.table, g.count, g.coop_grid, g.form, g.nt, g.vbrb,
                                    g.div, g.sr, 0, n, g.bar, s);
    for (int k = 0; k < n; ++k) {
        hipError_t e = hipSuccess;
        if (g.windowed && (e = launch_plan_batch<S>(g.job, 1, s)) != hipSuccess) return e;
        e = launch_step_batch<S>(reps, g.table, g.count, g.grid, g.form, g.nt, g.vbrb, g.div, g.sr,
                                 k, 1, nullptr, s);
        if (e != hipSuccess) return e;
        if (g.ndev && (e = launch_finalize_batch<S>(reps, (int)g.m.size(), k, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}
template <class S>
hipError_t enqueue_group_advance(const BatchGroup &g, int K, hipStream_t s)
{
    return launch_batch_advance<S>(reinterpret_cast<BatchRep<S> *const *>(g.reps),
                                   (int)g.m.size(), K, s);
}

#define LBM_DISPATCH_COOP(prec, ...)                                  \
    ((prec) == LBM_FP64   ? batch_coop_grid<double>(__VA_ARGS__)       \
     : (prec) == LBM_FP32 ? batch_coop_grid<float>(__VA_ARGS__)        \
     : (prec) == LBM_FP16_OFFSET ? batch_coop_grid<__half>(__VA_ARGS__) \
                                 : batch_coop_grid<__hip_bfloat16>(__VA_ARGS__))

#define LBM_DISPATCH_HIP(prec, fn, ...)                               \
    ((prec) == LBM_FP64   ? fn<double>(__VA_ARGS__)                    \
     : (prec) == LBM_FP32 ? fn<float>(__VA_ARGS__)                     \
     : (prec) == LBM_FP16_OFFSET ? fn<__half>(__VA_ARGS__)             \
                                 : fn<__hip_bfloat16>(__VA_ARGS__))

}  // namespace

struct lbm_batch {
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int max_members = 0;
    int64_t max_tiles = 0;
    std::vector<lbm_handle *> members;
    std::vector<BatchGroup> groups;
    // multi-step launches (lbm_batch_persistent): the run is enqueued
    // directly instead of through a graph
    bool persistent = false;
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_n = -1;

    void drop_graph()
    {
        // An executable graph may still be running from the last
        // lbm_batch_step (which does not synchronize): let it finish before
        // destroying it.  (teardown: a failure here leaves nothing to undo)
        if (gexec) {
            (void)hipStreamSynchronize(stream);
            (void)hipGraphExecDestroy(gexec);
        }
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_n = -1;
    }

    // Group members by storage type and kernel form; upload the tables.
    int rebuild()
    {
        groups.clear();
        for (lbm_handle *h : members) {
            const int vbrb = h->lay.vec ? h->lay.vb : h->lay.rb;
            const int win = (h->p.flags & LBM_FLAG_WINDOW) ? 1 : 0;
            const int div = h->p.growth >= LBM_GROWTH_DIVISION ? 1 : 0;
            const int sr = (h->p.flags & LBM_FLAG_STOCHASTIC_ROUND) ? 1 : 0;
            const int form = h->lay.tl.nq == 7 ? (h->lay.vec ? 3 : 2) : (h->lay.vec ? 1 : 0);
            const int own = steps_on_its_own(h) ? 1 : 0;
            BatchGroup *g = nullptr;
            for (BatchGroup &c : groups)
                if (c.own ? (own && c.prec == h->p.precision)
                          : (!own && c.prec == h->p.precision && c.form == form &&
                             c.nt == h->lay.nt && c.vbrb == vbrb && c.ty == h->lay.ty &&
                             c.windowed == win && c.div == div && c.sr == sr))
                    g = &c;
            if (!g) {
                if ((int)groups.size() == kMaxGroups) return LBM_E_INVALID;
                groups.emplace_back();
                g = &groups.back();
                g->prec = h->p.precision;
                g->form = form;
                g->nt = h->lay.nt;
                g->vbrb = vbrb;
                g->ty = h->lay.ty;
                g->windowed = win;
                g->div = div;
                g->sr = sr;
                g->own = own;
            }
            g->m.push_back(h);
        }
        const size_t slot = batch_slot_bytes(max_members);
        TileRef *table = reinterpret_cast<TileRef *>(ws + batch_table_offset(max_members));
        int64_t used = 0;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            BatchGroup &g = groups[gi];
            char *base = ws + gi * slot;
            g.reps = reinterpret_cast<void **>(base);
            g.count = reinterpret_cast<int32_t *>(base + slot - kAlign);
            g.job = reinterpret_cast<PlanJob *>(base + slot - kAlign + kPlanJobOffset);
            g.bar = reinterpret_cast<GridBar *>(base + slot - kAlign + kGridBarOffset);
            g.coop_grid = 0;
            std::vector<void *> reps(g.m.size());
            g.tiles = 0;
            g.ndev = 0;
            for (size_t i = 0; i < g.m.size(); ++i) {
                reps[i] = g.m[i]->at<char>(g.m[i]->lay.off_rep);
                if (!g.own) g.tiles += g.m[i]->lay.nblocks;
                g.ndev += g.m[i]->device_driven ? 1 : 0;
            }
            if (used + g.tiles > max_tiles || g.tiles > INT32_MAX) return LBM_E_NOMEM;
            g.table = table + used;
            used += g.tiles;
            std::vector<TileRef> tab;
            int32_t cnt = 0;
            if (g.own) {
                g.grid = 0;
            } else if (g.windowed) {
                g.grid = (int)std::min<int64_t>(g.tiles, kWindowGrid);
            } else {
                // every tile, member by member, in runs stacked in y
                for (size_t i = 0; i < g.m.size(); ++i) {
                    const Layout &ml = g.m[i]->lay;
                    const int64_t nr = run_count(ml.gy, ml.gx, ml.ty);
                    for (int64_t l = 0; l < nr; ++l)
                        tab.push_back(run_ref((int)i, l, ml.gy, ml.gx, ml.ty));
                }
                cnt = (int32_t)tab.size();
                g.grid = cnt;
                if (g.ndev == 0) {
                    // (on the device of the batch's stream)
                    int dev = 0;
                    hipDevice_t d;
                    if (stream && hipStreamGetDevice(stream, &d) == hipSuccess) dev = (int)d;
                    else if (hipGetDevice(&dev) != hipSuccess) return LBM_E_DEVICE;
                    const int cg = LBM_DISPATCH_COOP(g.prec, g.form, g.nt, g.vbrb, g.div, g.sr, dev);
                    g.coop_grid = std::min(cg, g.grid);
                }
            }
            const PlanJob job{g.reps, g.table, g.count, (int32_t)g.m.size(), 0};
            const GridBar bar0{0, 0, 0, 0};
            if (hipMemcpyAsync(g.reps, reps.data(), reps.size() * sizeof(void *),
                               hipMemcpyHostToDevice, stream) != hipSuccess ||
                hipMemcpyAsync(g.bar, &bar0, sizeof bar0, hipMemcpyHostToDevice, stream) != hipSuccess ||
                (g.windowed && hipMemcpyAsync(g.job, &job, sizeof job, hipMemcpyHostToDevice,
                                              stream) != hipSuccess) ||
                hipMemcpyAsync(g.count, &cnt, sizeof cnt, hipMemcpyHostToDevice, stream) != hipSuccess ||
                (!tab.empty() && hipMemcpyAsync(g.table, tab.data(), tab.size() * sizeof(TileRef),
                                                hipMemcpyHostToDevice, stream) != hipSuccess) ||
                hipStreamSynchronize(stream) != hipSuccess)
                return LBM_E_DEVICE;
        }
        dirty = false;
        drop_graph();
        return LBM_OK;
    }

    // n steps on stream st of a table group, or (g == nullptr) of every
    // member stepped by its own launches, all n steps of one member and then
    // the next.
    hipError_t enqueue_part(const BatchGroup *g, int n, hipStream_t st)
    {
        hipError_t e = hipSuccess;
        if (g) return LBM_DISPATCH_HIP(g->prec, enqueue_group, *g, n, persistent, st);
        for (const BatchGroup &o : groups) {
            if (!o.own) continue;
            for (lbm_handle *h : o.m)
                if ((e = LBM_DISPATCH_HIP(o.prec, enqueue_own_member, h, n, st)) != hipSuccess)
                    return e;
        }
        return e;
    }

    // A run of n steps on the batch's stream: the members stepped by their
    // own launches (all n steps of one, then the next), each table group's
    // n steps, then the descriptors' step counters.  (Capturing the groups
    // as parallel branches on side streams, forked and joined by events,
    // measured faster on small windowed runs, but with it the host process
    // crashed inside lbm_batch_step, a segmentation fault whose cause was not
    // found; the groups run in turn.)
    hipError_t enqueue(int64_t n)
    {
        hipError_t e = hipSuccess;
        bool own = false;
        for (const BatchGroup &g : groups) own = own || g.own;
        if (own && (e = enqueue_part(nullptr, (int)n, stream)) != hipSuccess) return e;
        for (const BatchGroup &g : groups)
            if (!g.own && (e = enqueue_part(&g, (int)n, stream)) != hipSuccess) return e;
        for (const BatchGroup &g : groups)
            if ((e = LBM_DISPATCH_HIP(g.prec, enqueue_group_advance, g, (int)n, stream)) !=
                hipSuccess)
                return e;
        return e;
    }
};

extern "C" {

size_t lbm_batch_workspace_bytes(int max_members, int64_t max_tiles)
{
    if (max_members < 1 || max_tiles < 1) return 0;
    return batch_table_offset(max_members) +
           align_up((size_t)max_tiles * sizeof(TileRef), kAlign);
}

int64_t lbm_tiles(const lbm_params *p)
{
    if (!params_ok(p, nullptr)) return 0;
    return make_layout(p).nblocks;
}

int lbm_batch_create(void *dev_ws, size_t ws_bytes, int max_members, int64_t max_tiles,
                     void *hip_stream, lbm_batch **out)
{
    if (!out) return LBM_E_INVALID;
    *out = nullptr;
    if (!dev_ws || max_members < 1 || max_tiles < 1 ||
        (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) != 0)
        return LBM_E_INVALID;
    if (ws_bytes < lbm_batch_workspace_bytes(max_members, max_tiles)) return LBM_E_NOMEM;
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_E_NOMEM;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = reinterpret_cast<char *>(dev_ws);
    b->ws_bytes = ws_bytes;
    b->max_members = max_members;
    b->max_tiles = max_tiles;
    *out = b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch *b, lbm_handle *h)
{
    if (!b || !h || h->batch || h->stream != b->stream) return LBM_E_INVALID;
    if ((int)b->members.size() >= b->max_members) return LBM_E_INVALID;
    b->members.push_back(h);
    h->batch = b;
    h->rep_ok = false;
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_remove(lbm_batch *b, lbm_handle *h)
{
    if (!b || !h || h->batch != b) return LBM_E_INVALID;
    b->members.erase(std::find(b->members.begin(), b->members.end(), h));
    h->batch = nullptr;
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0 || nsteps > INT32_MAX) return LBM_E_INVALID;
    if (nsteps == 0 || b->members.empty()) return LBM_OK;
    for (lbm_handle *h : b->members)
        if (h->err != LBM_OK) return LBM_E_STATE;
    int rc;
    if (b->dirty && (rc = b->rebuild())) return rc;
    // descriptors of members stepped on their own (or new) since the last run
    for (lbm_handle *h : b->members)
        if (!h->rep_ok || h->rep_t0 != h->t || h->rep_cur0 != h->cur)
            if ((rc = LBM_DISPATCH(h->p.precision, write_rep, h))) return rc;
    hipError_t e = hipSuccess;
    if (b->persistent) {
        // one cooperative launch per group covers the run: no graph
        e = b->enqueue(nsteps);
    } else {
        if (b->graph_n != nsteps) {
            b->drop_graph();
            // capture the run; streams that cannot be captured (the null
            // stream) get the same launches directly
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const hipError_t ec = b->enqueue(nsteps);
                hipGraph_t g = nullptr;
                const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
                if (ec == hipSuccess && e2 == hipSuccess && g &&
                    hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) == hipSuccess) {
                    b->graph = g;
                    b->graph_n = nsteps;
                } else {
                    if (g) (void)hipGraphDestroy(g);
                    b->gexec = nullptr;
                    (void)hipGetLastError();
                }
            } else {
                (void)hipGetLastError();
            }
        }
        e = b->gexec ? hipGraphLaunch(b->gexec, b->stream) : b->enqueue(nsteps);
    }
    if (e != hipSuccess) return LBM_E_DEVICE;
    for (lbm_handle *h : b->members) {
        h->t += nsteps;
        h->cur ^= (int)(nsteps & 1);
        h->rep_t0 += nsteps;
        h->rep_cur0 = (int)((h->rep_cur0 + nsteps) & 1);
    }
    return LBM_OK;
}

int lbm_batch_persistent(lbm_batch *b, int on)
{
    if (!b || (on != 0 && on != 1)) return LBM_E_INVALID;
    if (b->persistent != (on != 0)) {
        b->persistent = on != 0;
        b->drop_graph();
    }
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return LBM_E_INVALID;
    for (lbm_handle *h : b->members) h->batch = nullptr;
    b->drop_graph();
    delete b;
    return LBM_OK;
}

}  // extern "C"
