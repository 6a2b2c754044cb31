// lbm_step.hpp -- gfx950 kernels of the growing-tissue D2Q9 lattice
// Boltzmann library.
//
// One fused kernel advances the whole lattice by one step (the paper's
// Appendix A, steps 1-7, on every site): pull-streaming with the rear-wall
// bounce-back, moments (Eq. 1), the two-step bounce-back front (Sec. II),
// the growth source, the friction-damped steady state (Eq. 3) and BGK
// relaxation (Eq. 2), the zero-sum noise (Eq. 4) and the negative-population
// fix, then the store, per-column front heights (atomic max) and per-block
// float64 mass tallies.  Populations are stored row by row in tiles of TW
// columns holding the 9 directions one after the other (see Tiles), so a
// wavefront reads and writes a few contiguous runs per row.  Threads own
// columns and march over `ty` rows.
//
// The arithmetic follows one fixed order with no contraction (this file is
// compiled with -ffp-contract=off), so the float64 instantiation reproduces a
// plain sequential float64 evaluation of the same formulas bit for bit.
#pragma once
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include <climits>
#include <type_traits>

namespace lbm {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Population buffers always live in global memory; saying so lets the
// compiler use global (not flat) loads and stores for pointers that were read
// from memory (batch descriptors).
#define LBM_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ const T LBM_GLOBAL *as_global(const T *p)
{
    return (const T LBM_GLOBAL *)p;
}
template <class T>
__device__ __forceinline__ T LBM_GLOBAL *as_global(T *p)
{
    return (T LBM_GLOBAL *)p;
}

// Storage types as they sit in memory: the 16-bit formats are accessed as
// raw 16-bit words (their C++ classes cannot be assigned through
// address-space-qualified pointers) and converted bit for bit.
template <class S>
using MemT = typename std::conditional<sizeof(S) == 2, uint16_t, S>::type;

template <class S>
__device__ __forceinline__ S from_mem(MemT<S> v)
{
    if constexpr (sizeof(S) == 2) {
        S r;
        __builtin_memcpy(&r, &v, 2);
        return r;
    } else {
        return v;
    }
}
template <class S>
__device__ __forceinline__ MemT<S> to_mem(S v)
{
    if constexpr (sizeof(S) == 2) {
        uint16_t r;
        __builtin_memcpy(&r, &v, 2);
        return r;
    } else {
        return v;
    }
}

template <class R>
__device__ __forceinline__ R sum9(const R v[9])
{
    R s = v[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s = s + v[i];
    return s;
}

// The first q of nine values summed in index order (q = 9 on D2Q9, 7 on D2Q7).
template <class R>
__device__ __forceinline__ R sumq(const R v[9], int q)
{
    R s = v[0];
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (i < q) s = s + v[i];
    return s;
}

// Barrier for LDS traffic only: waits for this wave's LDS operations, not
// for its global stores (__syncthreads would also wait for every store in
// flight, which a tile that goes on to other work must not do).
__device__ __forceinline__ void lds_barrier()
{
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Wavefront reductions by DPP lane moves, which stay in the vector ALU (a
// shuffle through ds_bpermute costs an LDS round trip per 32 bits and level):
// neighbours, pairs of neighbours, the mirrored half of each group of 8 and of
// each row of 16 lanes, after which every lane of a row holds the row's
// result; the four rows' results are then read from lanes 0, 16, 32 and 48.
// The order of the operations is fixed, so float sums are deterministic.
// Every lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_move(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t read_lane(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

struct OpAdd {
    template <class T>
    __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
    template <class T>
    __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
};

// Every lane gets the result over its row of 16 lanes (8-byte T: double or
// long long).
template <class T, class Op = OpAdd>
__device__ __forceinline__ T row_reduce(T v, Op op = Op())
{
    static_assert(sizeof(T) == 8, "64-bit lanes");
    constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
    v = op(v, __builtin_bit_cast(T, dpp_move<kXor1>(__builtin_bit_cast(uint64_t, v))));
    v = op(v, __builtin_bit_cast(T, dpp_move<kXor2>(__builtin_bit_cast(uint64_t, v))));
    v = op(v, __builtin_bit_cast(T, dpp_move<kHalfMirror>(__builtin_bit_cast(uint64_t, v))));
    v = op(v, __builtin_bit_cast(T, dpp_move<kMirror>(__builtin_bit_cast(uint64_t, v))));
    return v;
}

// The result over the whole wavefront, in every lane.
template <class T, class Op = OpAdd>
__device__ __forceinline__ T wave_reduce(T v, Op op = Op())
{
    v = row_reduce(v, op);
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const T r0 = __builtin_bit_cast(T, read_lane(u, 0));
    const T r1 = __builtin_bit_cast(T, read_lane(u, 16));
    const T r2 = __builtin_bit_cast(T, read_lane(u, 32));
    const T r3 = __builtin_bit_cast(T, read_lane(u, 48));
    return op(op(op(r0, r1), r2), r3);
}

__device__ __forceinline__ double wave_sum(double v) { return wave_reduce(v); }

// Division-law state of a thread: this step's mean per unit weight and, for
// the uniform law, the chance e^-lam of no division (both read once from the
// device state), and the tallies of its sites: the weight of the eligible
// ones and the divisions they made.
struct DivTally {
    long long w = 0, n = 0;
    double lam = 0.0, p0 = 1.0;
};

__device__ __forceinline__ DivTally div_begin(const DevState *st)
{
    DivTally d;
    d.lam = st->lam;
    d.p0 = st->p0;
    return d;
}

__device__ __forceinline__ DivTally div_site(const DivTally &d)
{
    DivTally s;
    s.lam = d.lam;
    s.p0 = d.p0;
    return s;
}

// The per-site division map (if kept): a site's divisions at its physical
// row y mod H.  Each site is updated by one lane per step, so no atomics.
template <class S>
__device__ __forceinline__ void count_divisions(const StepArgs<S> &a, int64_t y, uint32_t x,
                                                long long n)
{
    if (n > 0 && a.divmap) a.divmap[(y % a.H) * a.L + x] += (int32_t)n;
}

// Deterministic block sums of a tile's tallies (fixed tree), one LDS round:
// the three masses end in thread 0; with the division laws, thread 0 also
// adds the block's fixed-point mass, weight and divisions to one of the
// step's slots in the device state.  Called by every thread of the block.
template <int NT, bool DIV>
__device__ __forceinline__ void block_tallies(double &a, double &b, double &c, long long mfx,
                                              const DivTally &dv, DevState *st, int block)
{
    constexpr int NW = NT / 64;
    __shared__ double red[3][NW];
    __shared__ long long redi[3][NW];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    long long i0 = 0, i1 = 0, i2 = 0;
    if constexpr (DIV) {
        i0 = wave_reduce(mfx);
        i1 = wave_reduce(dv.w);
        i2 = wave_reduce(dv.n);
    }
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
        if constexpr (DIV) {
            redi[0][wave] = i0;
            redi[1][wave] = i1;
            redi[2][wave] = i2;
        }
    }
    lds_barrier();
    if (threadIdx.x == 0) {
        a = red[0][0];
        b = red[1][0];
        c = red[2][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            a += red[0][w];
            b += red[1][w];
            c += red[2][w];
        }
        if constexpr (DIV) {
            long long t[3] = {0, 0, 0};
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                t[0] += redi[0][w];
                t[1] += redi[1][w];
                t[2] += redi[2][w];
            }
            unsigned long long *slot = st->div_acc[block & (kDivSlots - 1)];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (t[k] != 0) atomicAdd(slot + k, (unsigned long long)t[k]);
        }
    }
    lds_barrier();   // the arrays are free again (a batch block goes on to more tiles)
}

template <int NT>
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c)
{
    block_tallies<NT, false>(a, b, c, 0, DivTally(), nullptr, 0);
}

// ---------------------------------------------------------------------------
// Steps 3-7 of the update at a tissue site (streamed density rho_s >= rho_c),
// given its streamed populations fs.  S_acc / x_acc collect the injected mass
// and the mass change of the negative-population fix.
// ---------------------------------------------------------------------------
template <class S, bool DIV>
__device__ __forceinline__ void tissue_update(const StepArgs<S> &a, uint32_t t, typename Codec<S>::R fs[9],
                                              typename Codec<S>::R rho_s,
                                              typename Codec<S>::R out[9], uint32_t x, int64_t y,
                                              int64_t y_wall, int32_t hp, double &s_acc,
                                              double &x_acc, DivTally &dv)
{
    using R = typename Codec<S>::R;
    // ---- step 2 (rest): momentum ----------------------------------------------
    const R jx = ((((fs[1] - fs[3]) + fs[5]) - fs[6]) - fs[7]) + fs[8];
    const R jy = ((((fs[2] - fs[4]) + fs[5]) + fs[6]) - fs[7]) - fs[8];
    // ---- step 3: growth source.  Bulk law: its expectation, shared by the 8
    // moving directions (opposite pairs receive equal amounts: no momentum) --
    bool in_reg = true;
    if (a.region == kRegionFrontBand) in_reg = (y >= (int64_t)hp - a.region_width);
    else if (a.region == kRegionRearBand) in_reg = (y < y_wall + a.region_width);
    R S_ = (a.growth == kGrowthBulk && in_reg) ? a.g * rho_s : R(0);
    const R s8 = S_ * R(0.125);
#pragma unroll
    for (int i = 1; i < 9; ++i) fs[i] = fs[i] + s8;
    // Division laws (Sec. II; Eq. 5): a Poisson number of divisions with mean
    // lam q, each putting rho_cell / 2 on both directions of a drawn axis
    if constexpr (DIV) if (in_reg) {
        double q = 1.0;
        bool elig = true;
        if (a.growth == kGrowthDivisionDensity) {
            q = 1.0 - (double)rho_s / a.rho0;
            elig = rho_s > a.rho_c && q > 0.0;
        }
        if (elig) {
            const bool uniform = a.growth == kGrowthDivision;
            dv.w += uniform ? 1 : (long long)(q * kFx);
            double l = dv.lam * q;
            if (l > 8.0) l = 8.0;
            if (l > 0.0) {
                double U;
                uint64_t axes;
                division_draws(a.seed, a.replica, t, x, (uint32_t)y, U, axes);
                // (uniform law: one mean for every site, its e^-lam precomputed)
                const int k = uniform ? poisson_k_from(U, l, dv.p0) : poisson_k_small(U, l);
                int count[4] = {0, 0, 0, 0};
                for (int d = 0; d < k; ++d) count[(axes >> (2 * d)) & 3u] += 1;
                const double half = a.rho_cell * 0.5;
                constexpr int axis[4] = {1, 2, 5, 6};
                constexpr int rev[4] = {3, 4, 7, 8};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double amount = (double)count[c] * half;
                    fs[axis[c]] = fs[axis[c]] + (R)amount;
                    fs[rev[c]] = fs[rev[c]] + (R)amount;
                }
                S_ = (R)((double)k * a.rho_cell);
                dv.n += k;
            }
        }
    }
    const R rho = rho_s + S_;
    s_acc += (double)S_;

    // ---- step 4: u* = (1 - mu) u and the steady state of Eq. 3 ---------------
    const R ux = (jx / rho) * a.kmu;
    const R uy = (jy / rho) * a.kmu;
    const R usq = ux * ux + uy * uy;
    const R u15 = R(1.5) * usq;
    const R nux = -ux, nuy = -uy;
    R cu[9];
    cu[0] = R(0);
    cu[1] = ux;
    cu[2] = uy;
    cu[3] = nux;
    cu[4] = nuy;
    cu[5] = ux + uy;
    cu[6] = nux + uy;
    cu[7] = nux + nuy;
    cu[8] = ux + nuy;
    // ---- step 5 (tissue): relax towards f^SS (Eq. 2) --------------------------
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R c = cu[i];
        const R fss = (a.w[dclass9(i)] * rho) * (((R(1) + R(3) * c) + R(4.5) * (c * c)) - u15);
        out[i] = fs[i] - a.omega * (fs[i] - fss);
    }
    // ---- step 6: zero-sum noise where rho > rho_c (Eq. 4) ----------------------
    if (a.noise && rho > a.rho_c) {
        R v[9];
        noise_factors<R>(a.seed, a.replica, t, x, (uint32_t)y, v);
        R eta[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) eta[i] = a.sigma * v[i];
        const R m = sum9(eta) / R(9);
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i] = out[i] + (eta[i] - m);
    }
    // ---- step 7: negative populations --------------------------------------------
    bool neg = false;
#pragma unroll
    for (int i = 0; i < 9; ++i) neg = neg || (out[i] < R(0));
    if (neg) {
        const R before = sum9(out);
        if (out[0] < R(0)) {
            const R rho_pre = sum9(out);
            out[0] = R(0);
            const R rest = sum9(out);
            if (rest > R(0)) {
                const R r = rho_pre / rest;
#pragma unroll
                for (int i = 0; i < 9; ++i) out[i] = out[i] * r;
            }
        }
        constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if (out[i] < R(0)) {
                out[opp[i]] = out[opp[i]] + (-out[i]);
                out[i] = R(0);
            }
        }
        x_acc += (double)(sum9(out) - before);
    }
}

// Steps 2-7 at one site from its nine streamed raw (stored) values v, with
// validity already applied to fs (the decoded values).  The void branch of
// step 5 only reverses directions, so it forwards the stored values as they
// are.  Writes the stored result to so[9]; returns true for tissue.
// The division laws' fixed-point mass of a site: its density in units of
// 2^-24, truncated (summed as integers, so in any order).
__device__ __forceinline__ long long mass_fx(double rho)
{
    const double v = rho * kFx;
    return fabs(v) < 2147483648.0 ? (long long)(int)v : (long long)v;
}

// (the same for a float density: scaling by 2^24 is exact in float too)
__device__ __forceinline__ long long mass_fx(float rho)
{
    const float v = rho * 16777216.0f;
    return fabsf(v) < 2147483648.0f ? (long long)(int)v : mass_fx((double)rho);
}

// A tissue site's N outputs encoded for storage (so) and the values stored
// (kept): rounded to nearest, or (SR, 16-bit storages) stochastically with
// the site's rounding bits.
template <class S, int N, bool SR>
__device__ __forceinline__ void encode_site(const StepArgs<S> &a, uint32_t t, uint32_t x,
                                            int64_t y, const typename Codec<S>::R out[N],
                                            const typename Codec<S>::R Wd[N], S so[N],
                                            typename Codec<S>::R kept[N])
{
    if constexpr (SR && sizeof(S) == 2) {
        uint32_t r[9];
        round_bits(a.seed, a.replica, t, x, (uint32_t)y, r);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            so[i] = Codec<S>::enc_sr(out[i], Wd[i], r[i]);
            kept[i] = Codec<S>::dec(so[i], Wd[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            so[i] = Codec<S>::enc(out[i], Wd[i]);
            kept[i] = Codec<S>::dec(so[i], Wd[i]);
        }
    }
}

template <class S, bool DIV, bool SR = false>
__device__ __forceinline__ bool site_step(const StepArgs<S> &a, uint32_t t, const S v[9],
                                          typename Codec<S>::R fs[9], const typename Codec<S>::R Wd[9],
                                          S so[9], uint32_t x, int64_t y, int64_t y_wall, int32_t hp,
                                          double &m_acc, double &s_acc, double &x_acc,
                                          long long &mfx_acc, DivTally &dv)
{
    using R = typename Codec<S>::R;
    // ---- step 2: density ---------------------------------------------------------
    const R rho_s = sum9(fs);
    if (rho_s >= a.rho_c) {
        R out[9];
        tissue_update<S, DIV>(a, t, fs, rho_s, out, x, y, y_wall, hp, s_acc, x_acc, dv);
        R kept[9];
        encode_site<S, 9, SR>(a, t, x, y, out, Wd, so, kept);
        const R m = sum9(kept);
        m_acc += (double)m;
        if constexpr (DIV) mfx_acc += mass_fx(m);
        return true;
    }
    // ---- step 5 (void): reverse every direction ------------------------------------
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
    for (int i = 0; i < 9; ++i) so[i] = v[opp[i]];
    m_acc += (double)rho_s;
    if constexpr (DIV) {
        // the stored (reversed) values, summed in their stored order
        R m = fs[opp[0]];
#pragma unroll
        for (int i = 1; i < 9; ++i) m = m + fs[opp[i]];
        mfx_acc += mass_fx(m);
    }
    return false;
}

// Where one window row pulls its nine populations from (all wave-uniform):
// the physical row and plane of each pull, and whether the source is live.
struct RowSrc {
    int rm, r0, rp;        // physical rows y-1, y, y+1
    bool below;            // y-1 is behind the rear wall: reflect in place
    bool vm, v0, vp;       // source rows hold live data
};

__device__ __forceinline__ RowSrc row_sources(int mode, int j, int r0, int H, int64_t y,
                                              int64_t y_top)
{
    RowSrc s;
    s.r0 = r0;
    s.rm = (r0 == 0) ? H - 1 : r0 - 1;
    s.rp = (r0 == H - 1) ? 0 : r0 + 1;
    if (mode == kModePeriodic) {
        s.below = false;
        s.vm = s.v0 = s.vp = true;
    } else {
        s.below = (j == 0);
        s.v0 = y < y_top;
        s.vm = !s.below && (y - 1 < y_top);
        s.vp = (y + 1 < y_top) && (j + 1 < H);
    }
    return s;
}

// ---------------------------------------------------------------------------
// The fused step.  Each thread owns one column; a block of NT threads covers
// NT consecutive columns and `ty` rows, visited in batches of RB rows whose
// 9*RB loads are all issued before any of them is used.  Blocks are
// renumbered so that each XCD (dispatch goes round-robin over the 8 XCDs)
// works on one contiguous part of the lattice, keeping the cache lines that
// neighbouring blocks share in one L2.
// ---------------------------------------------------------------------------
// Block-to-tile order.  Dispatch goes round-robin over the 8 XCDs (block
// `lin` runs on XCD lin % 8), each with its own L2.  XCD x gets the runs x,
// x + 8, x + 16, ... of ch consecutive tiles: neighbouring tiles, which share
// the cache lines at their edges, mostly meet in one L2, and every XCD gets
// its share of each part of the lattice (tissue rows cost far more than
// empty ones; one XCD must not get them all).  ch <= 0: dispatch order.
// mul > 1 spreads each XCD's runs over the lattice: its m-th run is run
// (m mul) mod M of its M runs (mul coprime to M), so that the tiles in flight
// at any moment come from all heights -- tissue rows and empty rows are then
// worked on side by side instead of one after the other.  mul = -1 mirrors
// the order on XCDs 4-7 (they start at the top), so that while half the
// XCDs work through the tissue rows near the wall the other half stream the
// rows above and the shared HBM stays busy.  mul = -2 runs two sweeps side
// by side on every XCD: its even runs climb the lower half, its odd runs the
// upper half, each in order.
__device__ __forceinline__ int xcd_order(int lin, int nb, int ch, int mul = 0)
{
    if (ch <= 0) return lin;
    const int full = nb - nb % (8 * ch);
    if (lin >= full) return lin;
    const int k = lin >> 3;
    int m = k / ch;
    const int M = full / (8 * ch);
    if (mul > 1) m = (int)(((int64_t)m * mul) % M);
    else if (mul == -1 && (lin & 4)) m = M - 1 - m;
    else if (mul == -2) m = (m & 1) ? (M + 1) / 2 + (m >> 1) : (m >> 1);
    return (m * 8 + (lin & 7)) * ch + k % ch;
}

// Per-step inputs of one tile: the buffers and front-height slots of this
// step and the step counter.
template <class S>
struct StepIO {
    const S *fin;
    S *fout;
    const int32_t *h_prev;
    int32_t *h_next;
    int32_t *h_clear;
    uint32_t t;
};

// A batch member's per-step inputs at step k of a run: buffers and slots by
// the parity and the step count the member descriptor holds.
template <class S>
__device__ __forceinline__ StepIO<S> batch_io(const BatchRep<S> *R, int k)
{
    const int64_t tt = R->t0 + k;
    const bool cur = ((R->cur0 + k) & 1) != 0;
    // (selects, not indexing: the descriptor stays in registers)
    const int s = (int)(tt % 3);
    int32_t *const h0 = R->hs[0], *const h1 = R->hs[1], *const h2 = R->hs[2];
    StepIO<S> io;
    io.fin = cur ? R->f[1] : R->f[0];
    io.fout = cur ? R->f[0] : R->f[1];
    io.h_prev = s == 0 ? h0 : (s == 1 ? h1 : h2);
    io.h_next = s == 0 ? h1 : (s == 1 ? h2 : h0);
    io.h_clear = R->device_driven ? nullptr : (s == 0 ? h2 : (s == 1 ? h0 : h1));
    io.t = (uint32_t)tt;
    return io;
}

// The per-step inputs of a launch: from the arguments, or (a batch member
// stepped by its own launches in the batch's graph) from its descriptor.
template <class S>
__device__ __forceinline__ StepIO<S> step_io(const StepArgs<S> &a)
{
    if (a.clock) return batch_io(reinterpret_cast<const BatchRep<S> *>(a.clock), a.clock_k);
    return StepIO<S>{a.fin, a.fout, a.h_prev, a.h_next, a.h_clear, a.t};
}


template <class S, int NT, int RB, bool DIV, bool SR = false>
__device__ __forceinline__ void step_scalar_tile(const StepArgs<S> &a, const StepIO<S> &io, int bx,
                                                 int by, int nbx, int nstrips = 1)
{
    using R = typename Codec<S>::R;

    const int L = a.L, H = a.H;
    const int xr = bx * NT + threadIdx.x;
    const bool active = xr < L;
    const uint32_t x = active ? (uint32_t)xr : (uint32_t)(L - 1);   // loads stay in bounds
    const uint32_t xm = (x == 0) ? (uint32_t)(L - 1) : x - 1;
    const uint32_t xp = (x == (uint32_t)(L - 1)) ? 0u : x + 1;

    int64_t y_wall = 0, y_top = H, nrows = H;
    if (a.mode == kModeDevice) {
        y_wall = a.st->y_wall;
        y_top = a.st->y_valid_top;
        nrows = a.st->n_rows;
    }
    const int j0 = by * a.ty;
    const int jend = (int)min((int64_t)(j0 + nstrips * a.ty), nrows);

    double m_acc = 0.0, s_acc = 0.0, x_acc = 0.0;
    long long mfx_acc = 0;     // division laws: fixed-point mass
    DivTally dv;
    if constexpr (DIV) dv = div_begin(a.st);
    int64_t ymax = -1;
    const int32_t hp = (a.region == kRegionFrontBand) ? io.h_prev[x] : 0;
    R Wd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Wd[i] = a.Wd[dclass9(i)];

    const Tiles tl = a.tl;
    const int64_t cx = tl.col(x), cxm = tl.col(xm), cxp = tl.col(xp);
    const int tws = tl.tws;
    const MemT<S> LBM_GLOBAL *__restrict__ F = as_global(reinterpret_cast<const MemT<S> *>(io.fin));
    MemT<S> LBM_GLOBAL *__restrict__ G = as_global(reinterpret_cast<MemT<S> *>(io.fout));
    int rnext = (a.mode == kModeDevice) ? (int)((y_wall + j0) % H) : j0;

    for (int jb = j0; jb < jend; jb += RB) {
        S raw[RB][9];
        RowSrc src[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int j = jb + k;
            const int64_t y = y_wall + j;
            src[k] = row_sources(a.mode, j, rnext, H, y, y_top);
            rnext = src[k].rp;
            if (j < jend) {
                const RowSrc &s = src[k];
                // ---- step 1: pull-stream; the wall reflects in place -----
                const MemT<S> LBM_GLOBAL *row0 = F + (int64_t)s.r0 * tl.rs;
                const MemT<S> LBM_GLOBAL *rowm = F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs;
                const MemT<S> LBM_GLOBAL *rowp = F + (int64_t)s.rp * tl.rs;
                const int qn2 = s.below ? 4 : 2, qn5 = s.below ? 7 : 5, qn6 = s.below ? 8 : 6;
                const int64_t cn5 = s.below ? cx : cxm, cn6 = s.below ? cx : cxp;
                raw[k][0] = from_mem<S>(row0[cx + (0 << tws)]);
                raw[k][1] = from_mem<S>(row0[cxm + (1 << tws)]);
                raw[k][3] = from_mem<S>(row0[cxp + (3 << tws)]);
                raw[k][2] = from_mem<S>(rowm[cx + (qn2 << tws)]);
                raw[k][5] = from_mem<S>(rowm[cn5 + (qn5 << tws)]);
                raw[k][6] = from_mem<S>(rowm[cn6 + (qn6 << tws)]);
                raw[k][4] = from_mem<S>(rowp[cx + (4 << tws)]);
                raw[k][7] = from_mem<S>(rowp[cxp + (7 << tws)]);
                raw[k][8] = from_mem<S>(rowp[cxm + (8 << tws)]);
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int j = jb + k;
            if (j >= jend) break;
            const int64_t y = y_wall + j;
            const RowSrc &s = src[k];
            S v[9];
            R fs[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                v[i] = raw[k][i];
                fs[i] = Codec<S>::dec(v[i], Wd[i]);
            }
            // sources that hold no live data stream in nothing
            if (!s.v0) {
                v[0] = Codec<S>::enc(R(0), Wd[0]);
                v[1] = v[3] = Codec<S>::enc(R(0), Wd[1]);
                fs[0] = fs[1] = fs[3] = R(0);
            }
            if (!s.below && !s.vm) {
                v[2] = Codec<S>::enc(R(0), Wd[2]);
                v[5] = v[6] = Codec<S>::enc(R(0), Wd[5]);
                fs[2] = fs[5] = fs[6] = R(0);
            }
            if (!s.vp) {
                v[4] = Codec<S>::enc(R(0), Wd[4]);
                v[7] = v[8] = Codec<S>::enc(R(0), Wd[7]);
                fs[4] = fs[7] = fs[8] = R(0);
            }
            S so[9];
            double m_site = 0.0, s_site = 0.0, x_site = 0.0;
            long long mfx_site = 0;
            DivTally dv_site = div_site(dv);
            const bool tissue = site_step<S, DIV, SR>(a, io.t, v, fs, Wd, so, x, y, y_wall, hp, m_site,
                                             s_site, x_site, mfx_site, dv_site);
            MemT<S> LBM_GLOBAL *rowg = G + (int64_t)s.r0 * tl.rs + cx;
            if (active) {
#pragma unroll
                for (int i = 0; i < 9; ++i) rowg[i << tws] = to_mem<S>(so[i]);
                m_acc += m_site;
                mfx_acc += mfx_site;
                dv.w += dv_site.w;
                dv.n += dv_site.n;
                if constexpr (DIV) count_divisions(a, y, x, dv_site.n);
                if (tissue) {
                    // (the source and the step-7 change are zero at void sites)
                    s_acc += s_site;
                    x_acc += x_site;
                    ymax = y;
                    if (a.mode != kModePeriodic && j + 1 >= H) atomicOr(&a.st->status, kStDomainFull);
                }
            }
        }
    }

    // ---- front heights -----------------------------------------------------
    if (active) {
        if (ymax >= 0) {
            const int32_t hv = (int32_t)(ymax + 1);
            atomicMax(io.h_next + x, hv);
            atomicMax(a.colmax + x, hv);
        }
        if (io.h_clear && by == 0) io.h_clear[x] = 0;
    }

    // ---- per-block tallies (fixed order: deterministic) ------------------------
    block_tallies<NT, DIV>(m_acc, s_acc, x_acc, mfx_acc, dv, a.st, by * nbx + bx);
    double *pb = a.partials + kPartialSlots * (by * nbx + bx);
    if (threadIdx.x == 0) {
        pb[0] = m_acc;
        pb[1] += s_acc;
        pb[2] += x_acc;
        // a batch run taller than one strip keeps its tallies in its lowest
        // tile's slots; the per-step slots of the strips above it hold nothing
        for (int i = 1; i < nstrips; ++i) {
            double *q = a.partials + kPartialSlots * ((by + i) * nbx + bx);
            q[0] = 0.0;
        }
    }
}

template <class S, int NT, int RB, bool DIV, bool SR>
__global__ __launch_bounds__(NT) void step_kernel(StepArgs<S> a)
{
    const int nbx = gridDim.x;
    const int lin = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y, nbx * a.xcd_rows,
                              a.strip_mul);
    const StepIO<S> io = step_io(a);
    step_scalar_tile<S, NT, RB, DIV, SR>(a, io, lin % nbx, lin / nbx, nbx);
}

// ---------------------------------------------------------------------------
// 16-byte vector form of the step.  Each lane owns V = 16 / sizeof(S)
// consecutive columns, so every plane row is read and written with aligned
// 16-byte accesses (nontemporal: each value is used once per step).  The
// populations that move along x arrive from the neighbouring column: inside
// a wavefront that is the neighbouring lane's first or last element (one
// cross-lane shuffle per plane), at the wavefront's two edges and across the
// periodic seam it is a single wave-uniform load.  Needs L % V == 0.
// ---------------------------------------------------------------------------
// Raw per-lane vectors of ND dwords (8 or 16 bytes).
template <int ND>
struct RawVec;
template <>
struct RawVec<1> {
    typedef uint32_t type __attribute__((ext_vector_type(1)));
};
template <>
struct RawVec<2> {
    typedef uint32_t type __attribute__((ext_vector_type(2)));
};
template <>
struct RawVec<4> {
    typedef uint32_t type __attribute__((ext_vector_type(4)));
};

template <class S, int ND>
__device__ __forceinline__ S get_el(const typename RawVec<ND>::type &v, int i)
{
    if constexpr (sizeof(S) == 8) {
        const uint64_t b = (uint64_t)v[2 * i] | ((uint64_t)v[2 * i + 1] << 32);
        return __longlong_as_double((long long)b);
    } else if constexpr (sizeof(S) == 4) {
        return __uint_as_float(v[i]);
    } else {
        // (a select chain, so that i may also be a runtime index)
        uint32_t w = v[0];
#pragma unroll
        for (int d = 1; d < ND; ++d) w = ((i >> 1) == d) ? v[d] : w;
        const unsigned short b = (unsigned short)((w >> (16 * (i & 1))) & 0xFFFFu);
        S r;
        __builtin_memcpy(&r, &b, 2);
        return r;
    }
}

template <class S, int ND>
__device__ __forceinline__ void put_el(typename RawVec<ND>::type &v, int i, S s)
{
    if constexpr (sizeof(S) == 8) {
        const uint64_t b = (uint64_t)__double_as_longlong(s);
        v[2 * i] = (uint32_t)b;
        v[2 * i + 1] = (uint32_t)(b >> 32);
    } else if constexpr (sizeof(S) == 4) {
        v[i] = __float_as_uint(s);
    } else {
        unsigned short b;
        __builtin_memcpy(&b, &s, 2);
        const int sh = 16 * (i & 1);
        const uint32_t m = 0xFFFFu << sh, bb = (uint32_t)b << sh;
#pragma unroll
        for (int d = 0; d < ND; ++d) v[d] = ((i >> 1) == d) ? ((v[d] & ~m) | bb) : v[d];
    }
}

template <int ND, class T>
__device__ __forceinline__ typename RawVec<ND>::type vload(const T LBM_GLOBAL *p)
{
    return __builtin_nontemporal_load(
        reinterpret_cast<const typename RawVec<ND>::type LBM_GLOBAL *>(p));
}
template <int ND, class T>
__device__ __forceinline__ void vstore(T LBM_GLOBAL *p, const typename RawVec<ND>::type &v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<typename RawVec<ND>::type LBM_GLOBAL *>(p));
}

// Nontemporal store of a lane's vector through a buffer resource.  A lane
// whose offset lies beyond the resource's range stores nothing, so lanes
// past the last column need no branch around the store (a branch would make
// the compiler treat the stores as possibly not issued, and then wait for
// them before the next row's loads could be used).
constexpr uint32_t kBufWord3 = 0x00020000u;   // raw buffer, 32-bit data format
constexpr int kAuxNT = 2;                     // nontemporal cache policy
constexpr uint32_t kOffNone = 0x7FFFFFFFu;    // offset beyond any row
template <int ND>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff,
                                       const typename RawVec<ND>::type &v)
{
    if constexpr (ND == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(v[0], r, off, soff, kAuxNT);
    } else if constexpr (ND == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, soff, kAuxNT);
    } else {
        __builtin_amdgcn_raw_buffer_store_b128(v, r, off, soff, kAuxNT);
    }
}

// Loads through a buffer resource: the per-lane byte offset in a register,
// the per-plane offset in a scalar register.
template <int ND>
__device__ __forceinline__ typename RawVec<ND>::type bload(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                           uint32_t soff)
{
    typename RawVec<ND>::type v;
    if constexpr (ND == 1) {
        v[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, kAuxNT);
    } else if constexpr (ND == 2) {
        v = __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, kAuxNT);
    } else {
        v = __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, kAuxNT);
    }
    return v;
}
// One element at a wave-uniform byte offset.
template <class S>
__device__ __forceinline__ S bload_el(__amdgpu_buffer_rsrc_t r, uint32_t soff)
{
    if constexpr (sizeof(S) == 8) {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, 0, soff, 0);
        return __longlong_as_double((long long)((uint64_t)v[0] | ((uint64_t)v[1] << 32)));
    } else if constexpr (sizeof(S) == 4) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, 0, soff, 0));
    } else {
        const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, 0, soff, 0);
        S v;
        __builtin_memcpy(&v, &b, 2);
        return v;
    }
}
// A row's resource.  Every lane of a wavefront works on the same row, so
// base and bytes are wave-uniform.  UNIFORM (the 16-bit storages, which also
// load through resources) says so with one readfirstlane per word, which
// keeps the resource in scalar registers where the compiler would otherwise
// be unable to prove it uniform and wrap every access through it in a loop
// over the distinct values of the lanes.  readfirstlane returns int: each
// word goes back through uint32_t, so that a low word with bit 31 set is not
// sign-extended into the high one.
template <bool UNIFORM = false>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, int64_t bytes)
{
    if constexpr (UNIFORM) {
        const uint64_t b = reinterpret_cast<uint64_t>(base);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
        const uint64_t ub = ((uint64_t)hi << 32) | (uint64_t)lo;
        return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(ub), 0,
                                                 __builtin_amdgcn_readfirstlane((int)bytes),
                                                 (int)kBufWord3);
    }
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, (int)kBufWord3);
}

// Lane i's copy of lane i - 1's (wave_shr:1) or lane i + 1's (wave_shl:1)
// dword, by a DPP move within the vector ALU; lanes 0 and 63 get no
// neighbour's value (their callers take an edge value instead).
__device__ __forceinline__ uint32_t lane_from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, false);
}

// The left lane's last element (inside the wave) or the edge value.
template <class S, int ND>
__device__ __forceinline__ S from_left(const typename RawVec<ND>::type &own, S edge, bool use_edge)
{
    constexpr int NV = ND * 4 / (int)sizeof(S);
    typename RawVec<ND>::type t;
    t[ND - 1] = lane_from_left(own[ND - 1]);
    if constexpr (sizeof(S) == 8) t[ND - 2] = lane_from_left(own[ND - 2]);
    const S n = get_el<S, ND>(t, NV - 1);
    return use_edge ? edge : n;
}
// The right lane's first element (inside the wave) or the edge value.
template <class S, int ND>
__device__ __forceinline__ S from_right(const typename RawVec<ND>::type &own, S edge, bool use_edge)
{
    typename RawVec<ND>::type t;
    t[0] = lane_from_right(own[0]);
    if constexpr (sizeof(S) == 8) t[1] = lane_from_right(own[1]);
    const S n = get_el<S, ND>(t, 0);
    return use_edge ? edge : n;
}

// ND dwords per lane; WPE: waves per SIMD the register allocation aims for.
template <class S, int NT, int ND, bool DIV, bool SR = false>
__device__ __forceinline__ void step_vec_tile(const StepArgs<S> &a, const StepIO<S> &io, int bx,
                                              int by, int nbx, int nstrips = 1)
{
    using R = typename Codec<S>::R;
    using VT = typename RawVec<ND>::type;
    constexpr int V = ND * 4 / (int)sizeof(S);

    const int L = a.L, H = a.H;
    const int lane = threadIdx.x & 63;
    const int xv = (bx * NT + (int)threadIdx.x) * V;          // first column of this lane
    // first column of the wave.  It is uniform; the 16-bit storages, which
    // load through buffer resources, tell the compiler so (their wave-edge
    // loads then take a scalar offset instead of a loop over the lanes'
    // values); the wider types, loading through plain pointers, measured
    // slower with it (float32 78.6% -> 68.9% of 8 TB/s at 4096^2)
    const int x0 = sizeof(S) == 2 ? __builtin_amdgcn_readfirstlane(xv - lane * V) : xv - lane * V;
    const bool active = xv < L;
    // wave-uniform edge columns: left of the wave and right of it (periodic)
    const int xl = (x0 == 0 || x0 >= L) ? L - 1 : x0 - 1;     // (a wave past L reads in bounds)
    const int xr = (x0 + 64 * V < L) ? x0 + 64 * V : 0;
    const bool edge_l = (lane == 0);
    const bool edge_r = (lane == 63) || (xv + V >= L);

    int64_t y_wall = 0, y_top = H, nrows = H;
    if (a.mode == kModeDevice) {
        y_wall = a.st->y_wall;
        y_top = a.st->y_valid_top;
        nrows = a.st->n_rows;
    }
    const int j0 = by * a.ty;
    const int jend = (int)min((int64_t)(j0 + nstrips * a.ty), nrows);

    double m_acc = 0.0, s_acc = 0.0, x_acc = 0.0;
    long long mfx_acc = 0;     // division laws: fixed-point mass
    DivTally dv;
    if constexpr (DIV) dv = div_begin(a.st);
    int32_t jmax[V], hp[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        jmax[i] = -1;
        hp[i] = (a.region == kRegionFrontBand && active) ? io.h_prev[xv + i] : 0;
    }
    R Wd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Wd[i] = a.Wd[dclass9(i)];
    // bits of an exactly empty population of each direction (0 for float64
    // and float32, -W_i for the 16-bit offsets), as one dword of a vector
    uint32_t epat[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if constexpr (sizeof(S) == 2) {
            const uint32_t b = to_mem<S>(Codec<S>::enc(R(0), Wd[i]));
            epat[i] = b | (b << 16);
        } else {
            epat[i] = 0u;
        }
    }

    const Tiles tl = a.tl;
    const int tws = tl.tws;
    // lanes past the last column read (and never store) the last vector, so
    // every access stays inside the row
    const int64_t cv = tl.col(active ? xv : L - V), cl = tl.col(xl), cr = tl.col(xr);
    const MemT<S> LBM_GLOBAL *__restrict__ F = as_global(reinterpret_cast<const MemT<S> *>(io.fin));
    MemT<S> LBM_GLOBAL *__restrict__ G = as_global(reinterpret_cast<MemT<S> *>(io.fout));
    int r0 = (a.mode == kModeDevice) ? (int)((y_wall + j0) % H) : j0;

    // ---- step 1: pull-stream.  The loads of one window row: the nine
    // vectors and the six values at the wavefront's edges -------------------
    struct Fetch {
        VT A[9];
        S e[6];   // E, W, NE, NW, SW, SE sources beyond the wave's edges
    };
    constexpr uint32_t EB = sizeof(MemT<S>);
    const uint32_t loff = (uint32_t)(cv * EB);        // this lane's vector in a row
    const int64_t rowbytes = tl.rs * EB;
    const auto pl = [&](int q) { return ((uint32_t)q << tws) * EB; };
    // (16-bit storage loads through buffer resources, which need fewer
    // registers; the wider types measured faster with plain global loads)
    auto fetch = [&](int j, int r, Fetch &f) {
        const RowSrc s = row_sources(a.mode, j, r, H, y_wall + j, y_top);
        if constexpr (sizeof(S) != 2) {
            const MemT<S> LBM_GLOBAL *row0 = F + (int64_t)s.r0 * tl.rs;
            const MemT<S> LBM_GLOBAL *rowm = F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs;
            const MemT<S> LBM_GLOBAL *rowp = F + (int64_t)s.rp * tl.rs;
            const int qn2 = s.below ? 4 : 2, qn5 = s.below ? 7 : 5, qn6 = s.below ? 8 : 6;
            f.A[0] = vload<ND>(row0 + cv + (0 << tws));
            f.A[1] = vload<ND>(row0 + cv + (1 << tws));
            f.A[3] = vload<ND>(row0 + cv + (3 << tws));
            f.A[2] = vload<ND>(rowm + cv + (qn2 << tws));
            f.A[5] = vload<ND>(rowm + cv + (qn5 << tws));
            f.A[6] = vload<ND>(rowm + cv + (qn6 << tws));
            f.A[4] = vload<ND>(rowp + cv + (4 << tws));
            f.A[7] = vload<ND>(rowp + cv + (7 << tws));
            f.A[8] = vload<ND>(rowp + cv + (8 << tws));
            f.e[0] = from_mem<S>(row0[cl + (1 << tws)]);
            f.e[1] = from_mem<S>(row0[cr + (3 << tws)]);
            f.e[2] = from_mem<S>(rowm[cl + (5 << tws)]);
            f.e[3] = from_mem<S>(rowm[cr + (6 << tws)]);
            f.e[4] = from_mem<S>(rowp[cr + (7 << tws)]);
            f.e[5] = from_mem<S>(rowp[cl + (8 << tws)]);
            return;
        }
        const __amdgpu_buffer_rsrc_t R0 =
            row_rsrc<true>((const void *)(F + (int64_t)s.r0 * tl.rs), rowbytes);
        const __amdgpu_buffer_rsrc_t Rm =
            row_rsrc<true>((const void *)(F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs), rowbytes);
        const __amdgpu_buffer_rsrc_t Rp =
            row_rsrc<true>((const void *)(F + (int64_t)s.rp * tl.rs), rowbytes);
        // directions feeding N, NE, NW: the row below, or this site reflected
        const int qn2 = s.below ? 4 : 2, qn5 = s.below ? 7 : 5, qn6 = s.below ? 8 : 6;
        f.A[0] = bload<ND>(R0, loff, pl(0));
        f.A[1] = bload<ND>(R0, loff, pl(1));
        f.A[3] = bload<ND>(R0, loff, pl(3));
        f.A[2] = bload<ND>(Rm, loff, pl(qn2));
        f.A[5] = bload<ND>(Rm, loff, pl(qn5));
        f.A[6] = bload<ND>(Rm, loff, pl(qn6));
        f.A[4] = bload<ND>(Rp, loff, pl(4));
        f.A[7] = bload<ND>(Rp, loff, pl(7));
        f.A[8] = bload<ND>(Rp, loff, pl(8));
        f.e[0] = bload_el<S>(R0, (uint32_t)(cl * EB) + pl(1));
        f.e[1] = bload_el<S>(R0, (uint32_t)(cr * EB) + pl(3));
        f.e[2] = bload_el<S>(Rm, (uint32_t)(cl * EB) + pl(5));
        f.e[3] = bload_el<S>(Rm, (uint32_t)(cr * EB) + pl(6));
        f.e[4] = bload_el<S>(Rp, (uint32_t)(cr * EB) + pl(7));
        f.e[5] = bload_el<S>(Rp, (uint32_t)(cl * EB) + pl(8));
    };
    // The update of window row j (physical row r) from the loads in cur:
    // the stored results go to O; returns where the row pulled from.
    Fetch cur;
    VT O[9];
    auto update_row = [&](int j, int r) -> RowSrc {
        const int64_t y = y_wall + j;
        const RowSrc s = row_sources(a.mode, j, r, H, y, y_top);
        const VT A0 = cur.A[0], A1 = cur.A[1], A2 = cur.A[2], A3 = cur.A[3], A4 = cur.A[4];
        const VT A5 = cur.A[5], A6 = cur.A[6], A7 = cur.A[7], A8 = cur.A[8];
        const S e1 = cur.e[0], e3 = cur.e[1], e5 = cur.e[2], e6 = cur.e[3], e7 = cur.e[4];
        const S e8 = cur.e[5];
        // neighbours across lanes (E-type: from x-1, W-type: from x+1)
        const S n1 = from_left<S, ND>(A1, e1, edge_l);
        const S n8 = from_left<S, ND>(A8, e8, edge_l);
        const S n5 = from_left<S, ND>(A5, e5, edge_l);
        const S n3 = from_right<S, ND>(A3, e3, edge_r);
        const S n7 = from_right<S, ND>(A7, e7, edge_r);
        const S n6 = from_right<S, ND>(A6, e6, edge_r);

        // A neighbourhood whose every pulled value is exactly empty updates to
        // empty (the void rule only reverses directions, and opposite
        // directions share a weight): when that holds for the whole
        // wavefront, the per-site update is skipped.
        bool busy = false;
        {
            const VT *Av[9] = {&A0, &A1, &A2, &A3, &A4, &A5, &A6, &A7, &A8};
#pragma unroll
            for (int q = 0; q < 9; ++q)
#pragma unroll
                for (int d = 0; d < ND; ++d) busy = busy || ((*Av[q])[d] != epat[q]);
            const S ev[6] = {e1, e3, e5, e6, e7, e8};
            constexpr int eq[6] = {1, 3, 5, 6, 7, 8};
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                typename RawVec<ND>::type t;
#pragma unroll
                for (int d = 0; d < ND; ++d) t[d] = epat[eq[i]];
                busy = busy || (to_mem<S>(ev[i]) != to_mem<S>(get_el<S, ND>(t, 0)));
            }
        }
        uint32_t tmask = 0;
        if (__builtin_amdgcn_ballot_w64(busy) == 0) {
#pragma unroll
            for (int q = 0; q < 9; ++q)
#pragma unroll
                for (int d = 0; d < ND; ++d) O[q][d] = epat[q];
        } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            S v[9];
            v[0] = get_el<S, ND>(A0, k);
            v[1] = (k == 0) ? n1 : get_el<S, ND>(A1, k - 1);
            v[3] = (k == V - 1) ? n3 : get_el<S, ND>(A3, k + 1);
            v[2] = get_el<S, ND>(A2, k);
            if (s.below) {
                v[5] = get_el<S, ND>(A5, k);
                v[6] = get_el<S, ND>(A6, k);
            } else {
                v[5] = (k == 0) ? n5 : get_el<S, ND>(A5, k - 1);
                v[6] = (k == V - 1) ? n6 : get_el<S, ND>(A6, k + 1);
            }
            v[4] = get_el<S, ND>(A4, k);
            v[7] = (k == V - 1) ? n7 : get_el<S, ND>(A7, k + 1);
            v[8] = (k == 0) ? n8 : get_el<S, ND>(A8, k - 1);
            R fs[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) fs[i] = Codec<S>::dec(v[i], Wd[i]);
            // sources that hold no live data stream in nothing
            if (!s.v0) {
                v[0] = Codec<S>::enc(R(0), Wd[0]);
                v[1] = v[3] = Codec<S>::enc(R(0), Wd[1]);
                fs[0] = fs[1] = fs[3] = R(0);
            }
            if (!s.below && !s.vm) {
                v[2] = Codec<S>::enc(R(0), Wd[2]);
                v[5] = v[6] = Codec<S>::enc(R(0), Wd[5]);
                fs[2] = fs[5] = fs[6] = R(0);
            }
            if (!s.vp) {
                v[4] = Codec<S>::enc(R(0), Wd[4]);
                v[7] = v[8] = Codec<S>::enc(R(0), Wd[7]);
                fs[4] = fs[7] = fs[8] = R(0);
            }
            S so[9];
            double m_site = 0.0, s_site = 0.0, x_site = 0.0;
            const uint32_t x = (uint32_t)(xv + k);
            int32_t hpk = hp[0];
#pragma unroll
            for (int d = 1; d < V; ++d) hpk = (k == d) ? hp[d] : hpk;
            long long mfx_site = 0;
            DivTally dv_site = div_site(dv);
            const bool tissue = site_step<S, DIV, SR>(a, io.t, v, fs, Wd, so, x, y, y_wall, hpk, m_site,
                                             s_site, x_site, mfx_site, dv_site);
#pragma unroll
            for (int i = 0; i < 9; ++i) put_el<S, ND>(O[i], k, so[i]);
            if (active) {
                m_acc += m_site;
                mfx_acc += mfx_site;
                dv.w += dv_site.w;
                dv.n += dv_site.n;
                if constexpr (DIV) count_divisions(a, y, x, dv_site.n);
                if (tissue) {
                    // (the source and the step-7 change are zero at void sites)
                    s_acc += s_site;
                    x_acc += x_site;
                    tmask |= 1u << k;
                    if (a.mode != kModePeriodic && j + 1 >= H) atomicOr(&a.st->status, kStDomainFull);
                }
            }
        }
        }
#pragma unroll
        for (int k = 0; k < V; ++k)
            if ((tmask >> k) & 1u) jmax[k] = j;
        return s;
    };
    const uint32_t soff = active ? loff : kOffNone;
    auto store_row = [&](const RowSrc &s) {
        const __amdgpu_buffer_rsrc_t rr =
            row_rsrc<sizeof(S) == 2>((const void *)(G + (int64_t)s.r0 * tl.rs), rowbytes);
#pragma unroll
        for (int i = 0; i < 9; ++i) bstore<ND>(rr, soff, pl(i), O[i]);
    };
    // Each row's stores go out after the next row's loads: the memory counter
    // retires in issue order, so waiting for those loads never waits for
    // these stores.  (The first row is updated ahead of the loop, so every
    // update inside it follows the same sequence of memory operations.)
    if (j0 < jend) {
        fetch(j0, r0, cur);
        RowSrc s = update_row(j0, r0);
        for (int j = j0 + 1; j < jend; ++j) {
            __asm__ volatile("" ::: "memory");
            fetch(j, s.rp, cur);
            __asm__ volatile("" ::: "memory");
            store_row(s);
            s = update_row(j, s.rp);
        }
        store_row(s);
    }

    // ---- front heights -----------------------------------------------------
    if (active) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (jmax[k] >= 0) {
                const int32_t hv = (int32_t)(y_wall + jmax[k] + 1);
                atomicMax(io.h_next + xv + k, hv);
                atomicMax(a.colmax + xv + k, hv);
            }
            if (io.h_clear && by == 0) io.h_clear[xv + k] = 0;
        }
    }

    // ---- per-block tallies (fixed order: deterministic) ------------------------
    block_tallies<NT, DIV>(m_acc, s_acc, x_acc, mfx_acc, dv, a.st, by * nbx + bx);
    double *pb = a.partials + kPartialSlots * (by * nbx + bx);
    if (threadIdx.x == 0) {
        pb[0] = m_acc;
        pb[1] += s_acc;
        pb[2] += x_acc;
        // a batch run taller than one strip keeps its tallies in its lowest
        // tile's slots; the per-step slots of the strips above it hold nothing
        for (int i = 1; i < nstrips; ++i) {
            double *q = a.partials + kPartialSlots * ((by + i) * nbx + bx);
            q[0] = 0.0;
        }
    }
}

// Waves per SIMD the vector form's register allocation aims for (1 = no
// target), as measured fastest on a 4096 x 4096 lattice: the 16-bit storages
// at 4 bytes per lane fit 96 registers, so 5 waves share a SIMD (faster than
// 4); with the division laws they take 4 (at 5 they spill heavily), and
// float32 at 4 bytes per lane takes 6 (the few registers spilled belong to
// the rarely taken division branch).
template <class S, int ND, bool DIV>
constexpr int vec_waves()
{
    if constexpr (ND != 1) return 1;
    else if constexpr (sizeof(S) == 2) return DIV ? 4 : 5;
    else if constexpr (sizeof(S) == 4) return DIV ? 6 : 1;
    else return 1;
}

template <class S, int NT, int ND, bool DIV, bool SR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(vec_waves<S, ND, DIV || SR>())))
void step_kernel_vec(StepArgs<S> a)
{
    const int nbx = gridDim.x;
    const int lin = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y, nbx * a.xcd_rows,
                              a.strip_mul);
    const StepIO<S> io = step_io(a);
    step_vec_tile<S, NT, ND, DIV, SR>(a, io, lin % nbx, lin / nbx, nbx);
}

// ---------------------------------------------------------------------------
// LDS-staged form of the step.  Each wavefront owns one segment of SEG
// consecutive columns and marches up its block's rows.  The nine population
// rows that the update of row y pulls from (rest, E, W from row y; N, NE, NW
// from y - 1, or at the wall row its own S, SW, SE; S, SW, SE from y + 1)
// are copied from HBM straight into LDS by asynchronous global-to-LDS loads
// of one dword per lane, RING - 1 rows ahead of the row being updated: HBM
// reads stay in flight while a row computes, and they hold no registers.  A
// tenth load per row brings the six values that the segment's two edge
// columns pull from the neighbouring segments; every other neighbour along x
// is a plain LDS read one element over.  A wavefront reads only what it
// loaded itself, so waves never wait for each other: each waits on its own
// vector-memory counter, which retires loads and stores in issue order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_load_dword(const void *g, void *l)
{
    __builtin_amdgcn_global_load_lds((const void LBM_GLOBAL *)g,
                                     (__attribute__((address_space(3))) void *)l, 4, 0, 0);
}

// Wait until at most N of this wave's vector-memory operations are pending
// (the counter holds at most 63).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    constexpr int n = N < 63 ? N : 63;
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
    __asm__ volatile("" ::: "memory");
}

// wait_vm<A * M + B * MS>() for the runtime pair (a, b), 0 <= a < D, 0 <= b <= D.
template <int M, int MS, int D, int A = 0, int B = 0>
__device__ __forceinline__ void wait_vm_ab(int a, int b)
{
    if constexpr (A < D) {
        if constexpr (B <= D) {
            if (a == A && b == B) {
                wait_vm<A * M + B * MS>();
                return;
            }
            wait_vm_ab<M, MS, D, A, B + 1>(a, b);
        } else {
            wait_vm_ab<M, MS, D, A + 1, 0>(a, b);
        }
    }
}

// Nine LDS reads at byte addresses ad[] into v[], complete on return.  The
// reads are written in assembly (and wait for themselves) because the
// compiler, seeing an LDS read after an asynchronous global-to-LDS load,
// would otherwise wait for every such load in flight, including the rows
// being fetched ahead.
template <class S>
__device__ __forceinline__ void lds_read9(const uint32_t ad[9], S v[9])
{
    if constexpr (sizeof(S) == 8) {
        uint64_t r[9];
        __asm__ volatile(
            "ds_read_b64 %0, %9\n\tds_read_b64 %1, %10\n\tds_read_b64 %2, %11\n\t"
            "ds_read_b64 %3, %12\n\tds_read_b64 %4, %13\n\tds_read_b64 %5, %14\n\t"
            "ds_read_b64 %6, %15\n\tds_read_b64 %7, %16\n\tds_read_b64 %8, %17\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
              "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8])
            : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]), "v"(ad[6]),
              "v"(ad[7]), "v"(ad[8]));
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = __longlong_as_double((long long)r[i]);
    } else {
        uint32_t r[9];
        if constexpr (sizeof(S) == 4) {
            __asm__ volatile(
                "ds_read_b32 %0, %9\n\tds_read_b32 %1, %10\n\tds_read_b32 %2, %11\n\t"
                "ds_read_b32 %3, %12\n\tds_read_b32 %4, %13\n\tds_read_b32 %5, %14\n\t"
                "ds_read_b32 %6, %15\n\tds_read_b32 %7, %16\n\tds_read_b32 %8, %17\n\t"
                "s_waitcnt lgkmcnt(0)"
                : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
                  "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8])
                : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]),
                  "v"(ad[6]), "v"(ad[7]), "v"(ad[8]));
#pragma unroll
            for (int i = 0; i < 9; ++i) v[i] = __uint_as_float(r[i]);
        } else {
            __asm__ volatile(
                "ds_read_u16 %0, %9\n\tds_read_u16 %1, %10\n\tds_read_u16 %2, %11\n\t"
                "ds_read_u16 %3, %12\n\tds_read_u16 %4, %13\n\tds_read_u16 %5, %14\n\t"
                "ds_read_u16 %6, %15\n\tds_read_u16 %7, %16\n\tds_read_u16 %8, %17\n\t"
                "s_waitcnt lgkmcnt(0)"
                : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]),
                  "=&v"(r[6]), "=&v"(r[7]), "=&v"(r[8])
                : "v"(ad[0]), "v"(ad[1]), "v"(ad[2]), "v"(ad[3]), "v"(ad[4]), "v"(ad[5]),
                  "v"(ad[6]), "v"(ad[7]), "v"(ad[8]));
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint16_t b = (uint16_t)r[i];
                __builtin_memcpy(&v[i], &b, 2);
            }
        }
    }
}

// 32-bit LDS address of a pointer into shared memory.
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

template <class S, bool DIV>
__device__ __forceinline__ void step_staged_tile(const StepArgs<S> &a, const StepIO<S> &io, int bx,
                                                 int by, int nbx, unsigned char *lds_block)
{
    using R = typename Codec<S>::R;
    constexpr StagedGeom G(sizeof(S));
    constexpr int ES = (int)sizeof(S);
    constexpr int P = G.dwords(), SEGB = G.segb(), SEG = G.seg(), V = G.sites();
    constexpr int STAGE = G.stage_bytes(), RING = G.ring(), D = RING - 1;
    constexpr int NT = 64 * G.waves();
    constexpr int HALO = 9 * SEGB;                 // edge values: dword(s) per lane
    constexpr int HS = 4 * (ES == 8 ? 2 : 1);      // bytes per edge value slot

    const int L = a.L, H = a.H;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c0 = (bx * G.waves() + wave) * SEG;  // first column of this wave
    const bool live = c0 < L;                      // (wave-uniform)

    int64_t y_wall = 0, y_top = H, nrows = H;
    if (a.mode == kModeDevice) {
        y_wall = a.st->y_wall;
        y_top = a.st->y_valid_top;
        nrows = a.st->n_rows;
    }
    const int j0 = by * a.ty;
    const int n = live ? (int)max((int64_t)0, min((int64_t)a.ty, nrows - j0)) : 0;

    const Tiles tl = a.tl;
    const int tws = tl.tws;
    const int x_end = min(c0 + SEG, L);            // one past the last column
    const int iR = x_end - 1 - c0;                 // local index of that column
    const int xl = (c0 == 0) ? L - 1 : c0 - 1;     // left of the segment (periodic)
    const int xr = (x_end == L) ? 0 : x_end;       // right of it

    // byte offsets of this lane's dwords inside a population row (lanes past
    // the last column reread a column in range and never use it)
    int32_t dofs[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        if constexpr (ES == 8) {
            const int xe = min(c0 + 32 * p + (lane >> 1), L - 1);
            dofs[p] = (int32_t)(tl.col(xe) * 8 + 4 * (lane & 1));
        } else if constexpr (ES == 4) {
            dofs[p] = (int32_t)(tl.col(min(c0 + lane, L - 1)) * 4);
        } else {
            dofs[p] = (int32_t)(tl.col(min(c0 + 2 * lane, L - 2)) * 2);
        }
    }
    // the tenth load: lane h (or lanes 2h, 2h + 1 for float64) brings edge
    // value h: 0-2 from the left column (E, NE, SE), 3-5 from the right
    // (W, NW, SW); the remaining lanes repeat value 0
    int hv = (ES == 8) ? (lane >> 1) : lane;
    hv = hv < 6 ? hv : 0;
    const int hplane = (hv == 0) ? 1 : (hv == 1) ? 5 : (hv == 2) ? 8 : (hv == 3) ? 3 : (hv == 4) ? 6 : 7;
    const int hrow = (hv == 0 || hv == 3) ? 0 : (hv == 1 || hv == 4) ? -1 : 1;
    const int xh = hv < 3 ? xl : xr;
    const int32_t hofs =
        (int32_t)((tl.col(ES == 2 ? (xh & ~1) : xh) + ((int64_t)hplane << tws)) * ES +
                  (ES == 8 ? 4 * (lane & 1) : 0));

    double m_acc = 0.0, s_acc = 0.0, x_acc = 0.0;
    long long mfx_acc = 0;     // division laws: fixed-point mass
    DivTally dv;
    if constexpr (DIV) dv = div_begin(a.st);
    int32_t jmax[V], hp[V];
    const int xs = c0 + V * lane;                  // this lane's first site
    const bool active = live && xs < L;            // (L even for 16-bit storage)
#pragma unroll
    for (int v = 0; v < V; ++v) {
        jmax[v] = -1;
        hp[v] = (a.region == kRegionFrontBand && active) ? io.h_prev[xs + v] : 0;
    }
    R Wd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Wd[i] = a.Wd[dclass9(i)];

    const unsigned char *Fb = reinterpret_cast<const unsigned char *>(io.fin);
    unsigned char LBM_GLOBAL *Gb = as_global(reinterpret_cast<unsigned char *>(io.fout));
    const int64_t sofs = tl.col(active ? xs : 0) * ES;   // this lane's store offset in a row
    const int64_t rowb = tl.rs * ES;
    constexpr int64_t kOne = 1;
    unsigned char *ring = lds_block + wave * (RING * STAGE);

    int r_issue = (a.mode == kModeDevice) ? (int)((y_wall + j0) % H) : j0;
    int r_comp = r_issue;
    auto issue = [&](int k, unsigned char *st) {
        const int j = j0 + k;
        const RowSrc s = row_sources(a.mode, j, r_issue, H, y_wall + j, y_top);
        r_issue = s.rp;
        const unsigned char *b0 = Fb + (int64_t)s.r0 * rowb;
        const unsigned char *bm = Fb + (int64_t)(s.below ? s.r0 : s.rm) * rowb;
        const unsigned char *bp = Fb + (int64_t)s.rp * rowb;
        auto ld = [&](int slot, const unsigned char *base, int plane) {
            const unsigned char *pb = base + ((int64_t)plane << tws) * ES;
#pragma unroll
            for (int p = 0; p < P; ++p) lds_load_dword(pb + dofs[p], st + slot * SEGB + p * 256);
        };
        ld(0, b0, 0);
        ld(1, b0, 1);
        ld(3, b0, 3);
        ld(2, bm, s.below ? 4 : 2);
        ld(5, bm, s.below ? 7 : 5);
        ld(6, bm, s.below ? 8 : 6);
        ld(4, bp, 4);
        ld(7, bp, 7);
        ld(8, bp, 8);
        const unsigned char *bh = hrow == 0 ? b0 : (hrow < 0 ? bm : bp);
        lds_load_dword(bh + hofs, st + HALO);
        __asm__ volatile("" ::: "memory");
    };

    for (int k = 0; k < D && k < n; ++k) issue(k, ring + k * STAGE);
    // One row: start loading row k + D into the slot row k - 1 used, then
    // update row k.
    auto row = [&](int k, unsigned char *wr, const unsigned char *st) {
        if (k + D < n) issue(k + D, wr);

        const int j = j0 + k;
        const int64_t y = y_wall + j;
        const RowSrc s = row_sources(a.mode, j, r_comp, H, y, y_top);
        r_comp = s.rp;
        S out9[V][9];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int i = V * lane + v;
            const bool le = (i == 0), re = (i == iR);
            // LDS byte offset of slot q at local column c; edge values
            const auto at = [&](int q, int c) { return q * SEGB + c * ES; };
            constexpr int hl = ES == 2 ? 2 : 0;   // 16-bit: left value is the upper half
            const uint32_t sb = lds_addr(st);
            uint32_t ad[9];
            ad[0] = sb + at(0, i);
            ad[2] = sb + at(2, i);
            ad[4] = sb + at(4, i);
            ad[1] = sb + (le ? HALO + 0 * HS + hl : at(1, i - 1));
            ad[8] = sb + (le ? HALO + 2 * HS + hl : at(8, i - 1));
            ad[3] = sb + (re ? HALO + 3 * HS : at(3, i + 1));
            ad[7] = sb + (re ? HALO + 5 * HS : at(7, i + 1));
            ad[5] = sb + (s.below ? at(5, i) : (le ? HALO + 1 * HS + hl : at(5, i - 1)));
            ad[6] = sb + (s.below ? at(6, i) : (re ? HALO + 4 * HS : at(6, i + 1)));
            S vv[9];
            lds_read9<S>(ad, vv);
            R fs[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) fs[q] = Codec<S>::dec(vv[q], Wd[q]);
            // sources that hold no live data stream in nothing
            if (!s.v0) {
                vv[0] = Codec<S>::enc(R(0), Wd[0]);
                vv[1] = vv[3] = Codec<S>::enc(R(0), Wd[1]);
                fs[0] = fs[1] = fs[3] = R(0);
            }
            if (!s.below && !s.vm) {
                vv[2] = Codec<S>::enc(R(0), Wd[2]);
                vv[5] = vv[6] = Codec<S>::enc(R(0), Wd[5]);
                fs[2] = fs[5] = fs[6] = R(0);
            }
            if (!s.vp) {
                vv[4] = Codec<S>::enc(R(0), Wd[4]);
                vv[7] = vv[8] = Codec<S>::enc(R(0), Wd[7]);
                fs[4] = fs[7] = fs[8] = R(0);
            }
            double m_site = 0.0, s_site = 0.0, x_site = 0.0;
            long long mfx_site = 0;
            DivTally dv_site = div_site(dv);
            const bool tissue = site_step<S, DIV>(a, io.t, vv, fs, Wd, out9[v], (uint32_t)(c0 + i),
                                                  y, y_wall, hp[v], m_site, s_site, x_site,
                                                  mfx_site, dv_site);
            if (active) {
                m_acc += m_site;
                mfx_acc += mfx_site;
                dv.w += dv_site.w;
                dv.n += dv_site.n;
                if constexpr (DIV) count_divisions(a, y, (uint32_t)(c0 + i), dv_site.n);
                if (tissue) {
                    // (the source and the step-7 change are zero at void sites)
                    s_acc += s_site;
                    x_acc += x_site;
                    jmax[v] = j;
                    if (a.mode != kModePeriodic && j + 1 >= H) atomicOr(&a.st->status, kStDomainFull);
                }
            }
        }
        if (active) {
            unsigned char LBM_GLOBAL *g = Gb + (int64_t)s.r0 * rowb + sofs;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                unsigned char LBM_GLOBAL *gq = g + ((kOne * q) << tws) * ES;
                if constexpr (ES == 2) {
                    uint32_t w = 0;
                    __builtin_memcpy(&w, &out9[0][q], 2);
                    uint16_t hi;
                    __builtin_memcpy(&hi, &out9[1][q], 2);
                    w |= (uint32_t)hi << 16;
                    __builtin_nontemporal_store(w, reinterpret_cast<uint32_t LBM_GLOBAL *>(gq));
                } else {
                    __builtin_nontemporal_store(out9[0][q], reinterpret_cast<S LBM_GLOBAL *>(gq));
                }
            }
        }
    };
    for (int k = 0; k < n; ++k) {
        // stage k has landed once no more than the loads of the stages issued
        // after it and the stores issued after it are pending
        wait_vm_ab<G.loads(), 9, D>(min(D - 1, n - 1 - k), min(k, D));
        row(k, ring + ((k + D) % RING) * STAGE, ring + (k % RING) * STAGE);
    }

    // ---- front heights -----------------------------------------------------
    if (active) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (xs + v < L) {
                if (jmax[v] >= 0) {
                    const int32_t hv2 = (int32_t)(y_wall + jmax[v] + 1);
                    atomicMax(io.h_next + xs + v, hv2);
                    atomicMax(a.colmax + xs + v, hv2);
                }
                if (io.h_clear && by == 0) io.h_clear[xs + v] = 0;
            }
        }
    }

    // ---- per-block tallies (fixed order: deterministic) ------------------------
    block_tallies<NT, DIV>(m_acc, s_acc, x_acc, mfx_acc, dv, a.st, by * nbx + bx);
    double *pp = a.partials + kPartialSlots * (by * nbx + bx);
    if (threadIdx.x == 0) {
        pp[0] = m_acc;
        pp[1] += s_acc;
        pp[2] += x_acc;
    }
}

template <class S, bool DIV>
__global__ __launch_bounds__(64 * StagedGeom(sizeof(S)).waves()) void step_kernel_staged(StepArgs<S> a)
{
    constexpr StagedGeom G(sizeof(S));
    __shared__ __attribute__((aligned(16))) unsigned char lds[G.waves() * G.ring() * G.stage_bytes()];
    const int nbx = gridDim.x;
    const int lin = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y, nbx * a.xcd_rows,
                              a.strip_mul);
    const StepIO<S> io = step_io(a);
    step_staged_tile<S, DIV>(a, io, lin % nbx, lin / nbx, nbx, lds);
}

// ---------------------------------------------------------------------------
// Initial state (Appendix A): rows [0, init_rows) at rest, rho uniform on
// [(1 - a), (1 + a)] rho_init, f_i = w_i rho; everything above empty.  Same
// thread layout as the step so that partials[.][0] holds the initial mass.
// ---------------------------------------------------------------------------
template <class S, int NT>
__global__ __launch_bounds__(NT) void init_kernel(InitArgs<S> a)
{
    using R = typename Codec<S>::R;
    const int j0 = blockIdx.y * a.ty;
    double m_acc = 0.0, z1 = 0.0, z2 = 0.0;
    for (int c = 0; c < a.cpt; ++c) {
        const int x = (blockIdx.x * NT + threadIdx.x) * a.cpt + c;
        if (x >= a.L) break;
        int ymax = -1;
        const int jend = min(j0 + a.ty, a.H);
        for (int j = j0; j < jend; ++j) {
            double rho = 0.0;
            if (j < a.init_rows) {
                const double U = init_uniform(a.seed, a.replica, (uint32_t)x, (uint32_t)j);
                rho = a.rho_init * (1.0 + a.init_amp * (2.0 * U - 1.0));
            }
            R kept[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (i >= a.tl.nq) break;
                const R f = (R)(a.w[i] * rho);
                const S s = Codec<S>::enc(f, a.Wd[i]);
                a.f[a.tl.at(i, j, x)] = s;
                kept[i] = Codec<S>::dec(s, a.Wd[i]);
            }
            const R r = sumq(kept, a.tl.nq);
            m_acc += (double)r;
            if (r >= (R)a.rho_c) ymax = j;
        }
        if (ymax >= 0) {
            atomicMax(a.h0 + x, ymax + 1);
            atomicMax(a.colmax + x, ymax + 1);
        }
    }
    block_sum3<NT>(m_acc, z1, z2);
    if (threadIdx.x == 0) {
        double *p = a.partials + kPartialSlots * (blockIdx.y * gridDim.x + blockIdx.x);
        p[0] = m_acc;
        p[1] = 0.0;
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

// Mass of the current state into partials[.][0] (after populations are
// replaced from the host).  Rows at or above y_valid_top read as empty.
template <class S, int NT>
__global__ __launch_bounds__(NT) void mass_kernel(MassArgs<S> a)
{
    using R = typename Codec<S>::R;
    const int j0 = blockIdx.y * a.ty;
    double m_acc = 0.0, z1 = 0.0, z2 = 0.0;
    long long mfx = 0;
    DivTally dv;
    const int64_t y_wall = a.st->y_wall, y_top = a.st->y_valid_top;
    for (int c = 0; c < a.cpt; ++c) {
        const int x = (blockIdx.x * NT + threadIdx.x) * a.cpt + c;
        if (x >= a.L) break;
        const int jend = min(j0 + a.ty, a.H);
        for (int j = j0; j < jend; ++j) {
            const int64_t y = y_wall + j;
            if (y >= y_top) break;
            const int r = (int)(y % a.H);
            R v[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (i < a.tl.nq) v[i] = Codec<S>::dec(a.f[a.tl.at(i, r, x)], a.Wd[i]);
            const R rho = sumq(v, a.tl.nq);
            m_acc += (double)rho;
            if (a.growth >= kGrowthDivision) {
                // the division laws' tallies of a state given as populations:
                // its sites count as eligible by their own density
                mfx += mass_fx((double)rho);
                bool in_reg = true;
                if (a.region == kRegionFrontBand) in_reg = y >= (int64_t)a.h[x] - a.region_width;
                else if (a.region == kRegionRearBand) in_reg = y < y_wall + a.region_width;
                if (rho >= (R)a.rho_c && in_reg) {
                    if (a.growth == kGrowthDivision) {
                        dv.w += 1;
                    } else {
                        const double q = 1.0 - (double)rho / a.rho0;
                        if (rho > (R)a.rho_c && q > 0.0) dv.w += (long long)(q * kFx);
                    }
                }
            }
        }
    }
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    if (a.growth >= kGrowthDivision) block_tallies<NT, true>(m_acc, z1, z2, mfx, dv, a.st, blk);
    else block_sum3<NT>(m_acc, z1, z2);
    if (threadIdx.x == 0) a.partials[kPartialSlots * blk] = m_acc;
}

// ---------------------------------------------------------------------------
// Small single-block kernels.
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 1024;
constexpr int kRedWaves = kRedThreads / 64;

// Deterministic reductions of one block of kRedThreads threads: N values at
// once, one LDS round, results in every thread.  The 16 waves' results are
// combined by each row of 16 lanes reading them one per lane.
template <int N, class T, class Op = OpAdd>
__device__ __forceinline__ void block_reduce(T (&v)[N], T (*sh)[kRedWaves], Op op = Op())
{
    static_assert(kRedWaves == 16, "one wave's result per lane of a row");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_reduce(v[k], op);
    __syncthreads();   // (sh may still be read by an earlier reduction)
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][wave] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = row_reduce(sh[k][lane & 15], op);
}

// Division laws: this thread's share of the step's tallies from the device
// state's slots, which it clears for the next step (words: fixed-point mass,
// weight, divisions).
__device__ __forceinline__ void take_div_slots(DevState *st, long long &mfx, long long &wsum,
                                               long long &ndiv)
{
    if (threadIdx.x < kDivSlots) {
        unsigned long long *slot = st->div_acc[threadIdx.x];
        mfx += (long long)slot[0];
        wsum += (long long)slot[1];
        ndiv += (long long)slot[2];
        slot[0] = slot[1] = slot[2] = 0ull;
    }
}

// The next step's mean per unit weight and, for the uniform law, its chance
// of no division at a site (thread 0).
__device__ __forceinline__ void set_division_rate(DevState *st, int growth, double lam,
                                                  long long ndiv)
{
    st->lam = lam;
    st->p0 = growth == kGrowthDivision ? exp_neg(lam < 8.0 ? lam : 8.0) : 1.0;
    st->divisions += ndiv;
}

// This thread's share of the front-height sums relative to the wall row,
// S1 = sum (h - y_wall) and S2 = sum (h - y_wall)^2, and of the highest entry
// of colmax (four columns' loads in flight at a time).
__device__ __forceinline__ void height_sums(const int32_t *h, const int32_t *colmax, int L,
                                            int64_t y_wall, long long &s1, long long &s2,
                                            long long &cm)
{
    constexpr int U = 4;
    for (int x0 = threadIdx.x; x0 < L; x0 += U * kRedThreads) {
        int32_t hv[U], cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = x0 + u * kRedThreads;
            hv[u] = x < L ? h[x] : 0;
            cv[u] = x < L ? colmax[x] : INT_MIN;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (x0 + u * kRedThreads < L) {
                const long long d = (long long)hv[u] - y_wall;
                s1 += d;
                s2 += d * d;
                cm = (long long)cv[u] > cm ? (long long)cv[u] : cm;
            }
        }
    }
}

// hbar and w of Sec. III from the exact integer sums (so the result does not
// depend on the order of summation): hbar = y_wall + S1 / L,
// w = sqrt(L S2 - S1^2) / L.
__device__ __forceinline__ void height_stats(long long S1, long long S2, int L, int64_t y_wall,
                                             double &hbar, double &W)
{
    const long long num = (long long)L * S2 - S1 * S1;
    hbar = (double)y_wall + (double)S1 / (double)L;
    W = sqrt((double)num) / (double)L;
}

// Between steps when the device drives the window (rear wall that follows the
// front, and/or the exact sweep window): wall rule of Appendix A, retired
// mass, highest front so far, rows the next step must sweep, and the next
// front-height slot reset to the wall row.
template <class S>
__device__ __forceinline__ void finalize_body(const FinalizeArgs<S> &a)
{
    using R = typename Codec<S>::R;
    __shared__ long long shi[5][kRedWaves];
    __shared__ double shd[1][kRedWaves];
    DevState *st = a.st;
    const int64_t y_wall = st->y_wall;
    const int64_t nrows_done = st->n_rows;
    // front-height sums, division-law tallies (integers: order-free) and the
    // highest front so far, in two block reductions
    long long si[5] = {0, 0, 0, 0, 0};   // S1, S2, mass (2^-24), weight, divisions
    long long cm[1] = {LLONG_MIN};
    height_sums(a.h_next, a.colmax, a.L, y_wall, si[0], si[1], cm[0]);
    if (a.growth >= kGrowthDivision) take_div_slots(st, si[2], si[3], si[4]);
    block_reduce(si, shi);
    block_reduce(cm, shi, OpMax());
    double hbar, W;
    height_stats(si[0], si[1], a.L, y_wall, hbar, W);

    int64_t k = 0;
    if (a.follow) {
        double gap = a.w_factor * W;
        if (gap < (double)a.min_gap) gap = (double)a.min_gap;
        const int64_t target = (int64_t)floor(hbar - gap);
        if (target > y_wall) k = target - y_wall;
        if (k > a.H - 1) k = a.H - 1;
    }
    double gone[1] = {0.0};
    long long gone_fx[1] = {0};
    if (k > 0) {
        const int64_t n = k * (int64_t)a.L;
        for (int64_t e = threadIdx.x; e < n; e += kRedThreads) {
            const int64_t y = y_wall + e / a.L;
            const int x = (int)(e % a.L);
            const int r = (int)(y % a.H);
            R v[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (i < a.tl.nq) v[i] = Codec<S>::dec(a.f[a.tl.at(i, r, x)], a.Wd[i]);
            const R m = sumq(v, a.tl.nq);
            gone[0] += (double)m;
            gone_fx[0] += mass_fx((double)m);
        }
        block_reduce(gone, shd);
        block_reduce(gone_fx, shi);
        // the division map forgets the rows the wall leaves behind
        if (a.divmap)
            for (int64_t e = threadIdx.x; e < n; e += kRedThreads)
                a.divmap[((y_wall + e / a.L) % a.H) * a.L + e % a.L] = 0;
    }
    // division laws: the next step's rate from this step's tallies, less the
    // rows the wall leaves behind
    const double lam_next =
        a.growth >= kGrowthDivision
            ? division_lam(a.growth == kGrowthDivision, a.g, a.rho_cell, si[2] - gone_fx[0], si[3])
            : 0.0;
    const int64_t y_new = y_wall + k;
    // highest front so far and the rows the next step must sweep
    const long long hi = st->h_hi > cm[0] ? st->h_hi : cm[0];
    for (int x = threadIdx.x; x < a.L; x += kRedThreads) {
        if (a.h_next[x] < y_new) a.h_next[x] = (int32_t)y_new;
        a.h_clear[x] = (int32_t)y_new;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (a.growth >= kGrowthDivision) set_division_rate(st, a.growth, lam_next, si[4]);
        st->retired_last = gone[0];
        st->retired_total += gone[0];
        st->y_valid_top = y_wall + nrows_done;
        st->rows_swept += nrows_done;
        st->y_wall = y_new;
        st->h_hi = hi;
        int64_t nr = a.H;
        if (a.window) {
            nr = (int64_t)hi + 2 - y_new;
            if (nr > a.H) nr = a.H;
            if (nr < 1) nr = 1;
        }
        st->n_rows = nr;
    }
}

template <class S>
__global__ __launch_bounds__(kRedThreads) void finalize_kernel(FinalizeArgs<S> a)
{
    finalize_body<S>(a);
}

// ---------------------------------------------------------------------------
// Batches: one launch advances every member of a group by one step.  The
// 1-D grid enumerates all members' tiles; a block finds its member by binary
// search over the prefix sums of tile counts and runs the same tile body as
// the solo kernels, so each member's populations come out bit for bit as in
// a solo run.  Per-step buffers and slots follow from the member's step count.
// ---------------------------------------------------------------------------
// A member descriptor, read through the constant address space: it does not
// change while a step runs and its address is the same for the whole block,
// so its fields are fetched by scalar loads into scalar registers, as kernel
// arguments are (the tile bodies then need no vector registers for them).
template <class T>
__device__ __forceinline__ T load_descriptor(const void *p)
{
    static_assert(sizeof(T) % 4 == 0, "descriptor is read as dwords");
    using C = const __attribute__((address_space(4))) uint32_t;
    C *src = (C *)p;
    T out;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return out;
}

// Grid-wide barrier between the steps of a multi-step batch launch (its
// blocks are all resident: the launch is cooperative).  Every thread makes
// its writes visible device-wide, the block's first thread counts the
// block in and waits for the round to change, and every thread then sees
// the other blocks' writes.  (The device-scope fences write each XCD's
// cache back, so a barrier costs far more than the step boundary of a
// graph-replayed launch.)  The wait is bounded: past kBarrierSpins polls
// (about a second) a block gives up, flags the barrier and returns false; a
// block that finds the flag set returns false at once, so every block of
// the launch leaves soon after the first gives up.
constexpr uint32_t kBarrierSpins = 1u << 22;
__device__ __forceinline__ bool grid_barrier(GridBar *b)
{
    __shared__ int ok;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 0;
        if (__hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            const uint32_t g = __hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t arrived =
                __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == gridDim.x - 1) {
                __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&b->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                ok = 1;
            } else {
                for (uint32_t spins = 0;; ++spins) {
                    if (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != g) {
                        ok = 1;
                        break;
                    }
                    if (spins >= kBarrierSpins ||
                        __hip_atomic_load(&b->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        __hip_atomic_fetch_or(&b->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
            }
        }
    }
    __syncthreads();
    __threadfence();
    return ok != 0;
}

// After a barrier gave up: every member of the launch latches kStSyncLost.
template <class S>
__device__ void batch_sync_lost(BatchRep<S> *const *reps, const TileRef *table, int total)
{
    for (int c = threadIdx.x; c < total; c += blockDim.x)
        atomicOr(&reps[table[c].rep]->a.st->status, kStSyncLost);
}

// Each table entry is a run of tiles of one member stacked in y, which a
// block updates as one tall tile after fetching the member's descriptor.
// Windowed groups launch a fixed grid that strides over the entries.  A
// multi-step launch (bar set) runs steps k .. k + K - 1 with a grid-wide
// barrier between them.
template <class S, int NT, int ND, bool VEC, bool DIV, bool SR>
__global__ __launch_bounds__(NT) void step_batch(BatchRep<S> *const *reps, const TileRef *table,
                                                 const int32_t *count, int k, int K, GridBar *bar)
{
    const int total = *count;
    for (int s = 0; s < K; ++s) {
        for (int c = blockIdx.x; c < total; c += gridDim.x) {
            const TileRef e = table[xcd_order(c, total, 2)];
            const BatchRep<S> R = load_descriptor<BatchRep<S>>(reps[e.rep]);
            const StepIO<S> io = batch_io(&R, k + s);
            const int bx = e.local0 % R.gx, by = e.local0 / R.gx;
            if constexpr (VEC) step_vec_tile<S, NT, ND, DIV, SR>(R.a, io, bx, by, R.gx, e.n);
            else step_scalar_tile<S, NT, ND, DIV, SR>(R.a, io, bx, by, R.gx, e.n);
        }
        if (s + 1 < K && !grid_barrier(bar)) {
            batch_sync_lost(reps, table, total);
            return;
        }
    }
}

// Tile table of a windowed group: each member contributes the tiles of its
// live rows (the first n_rows window rows, as set by its last finalize).
// One block: tile counts, exclusive scan, then the entries.
__device__ __forceinline__ int live_tiles(int32_t gx, int32_t ty, int32_t nblocks, int window,
                                          int64_t n_rows)
{
    if (!window) return nblocks;
    const int64_t strips = (n_rows + ty - 1) / ty;
    const int64_t c = strips * gx;
    return c < nblocks ? (int)c : nblocks;
}

// A member's live tiles, from the rows its last between-step work set.
template <class S>
__device__ __forceinline__ int member_live(const BatchRep<S> *R)
{
    return live_tiles(R->gx, R->ty, R->nblocks, R->window, R->a.st->n_rows);
}

// One block: the tile table of a windowed group for its next step.
template <class S>
__device__ void plan_group(const PlanJob &J)
{
    BatchRep<S> *const *reps = reinterpret_cast<BatchRep<S> *const *>(J.reps);
    const int n = J.n;
    TileRef *table = J.table;
    int32_t *count = J.count;
    __shared__ int32_t pre[kRedThreads + 1];
    __shared__ int32_t live_sh[kRedThreads];
    __shared__ int32_t carry;
    __shared__ long long tot_sh[1][kRedWaves];
    // When every live tile of the group fits the launch's grid, each run is
    // one tile (a block then walks the shortest chain of row loads); runs of
    // about kRowsPerRun rows otherwise.
    long long tot[1] = {0};
    int live_first = 0;   // this thread's member of the first chunk
    for (int i = threadIdx.x; i < n; i += kRedThreads) {
        const int lv = member_live(reps[i]);
        if (i < kRedThreads) live_first = lv;
        tot[0] += lv;
    }
    block_reduce(tot, tot_sh);
    const int ry = tot[0] <= kWindowGrid ? 1 : 0;   // 0: the default height
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kRedThreads) {
        const int i = base + threadIdx.x;
        int c = 0, live = 0;
        if (i < n) {
            const BatchRep<S> *R = reps[i];
            live = base == 0 ? live_first : member_live(R);
            c = (int)run_count(live / R->gx, R->gx, R->ty, ry);    // runs of this member
        }
        live_sh[threadIdx.x] = live;
        // inclusive scan of this chunk (Hillis-Steele)
        pre[threadIdx.x] = c;
        __syncthreads();
        for (int off = 1; off < kRedThreads; off <<= 1) {
            const int v = threadIdx.x >= off ? pre[threadIdx.x - off] : 0;
            __syncthreads();
            pre[threadIdx.x] += v;
            __syncthreads();
        }
        __syncthreads();
        // entries of this chunk's members, filled by the whole block
        const int m_end = min(n - base, kRedThreads);
        for (int m = 0; m < m_end; ++m) {
            const int cm = pre[m] - (m ? pre[m - 1] : 0);
            const int s0 = carry + (m ? pre[m - 1] : 0);
            const int live = live_sh[m];
            const BatchRep<S> *Rm = reps[base + m];
            for (int l = threadIdx.x; l < cm; l += kRedThreads)
                table[s0 + l] = run_ref(base + m, l, live / Rm->gx, Rm->gx, Rm->ty, ry);
            // tiles that ran last step but not this one: their mass tally
            // would otherwise stay behind (a solo launch writes 0 there)
            BatchRep<S> *R = reps[base + m];
            const int last = R->last_live;
            for (int b = live + threadIdx.x; b < last; b += kRedThreads)
                R->a.partials[kPartialSlots * b] = 0.0;
            __syncthreads();
            if (threadIdx.x == 0) R->last_live = live;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += pre[m_end - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

// The same table for a group of at most 64 members, by one wavefront (one
// lane per member): no block-wide barriers, which dominate the latency of
// the block-wide form on the small groups of a served trace.
template <class S>
__device__ void plan_group_wave(const PlanJob &J)
{
    BatchRep<S> *const *reps = reinterpret_cast<BatchRep<S> *const *>(J.reps);
    const int n = J.n;
    const int lane = threadIdx.x;
    int live = 0, gx = 1, ty = 1;
    if (lane < n) {
        const BatchRep<S> *R = reps[lane];
        live = member_live(R);
        gx = R->gx;
        ty = R->ty;
    }
    const long long tot = wave_reduce((long long)live);
    const int ry = tot <= kWindowGrid ? 1 : 0;   // as in plan_group
    const int c = lane < n ? (int)run_count(live / gx, gx, ty, ry) : 0;
    int incl = c;   // inclusive scan over the lanes
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const int excl = incl - c;
    for (int m = 0; m < n; ++m) {
        const int cm = __shfl(c, m, 64), s0 = __shfl(excl, m, 64), lv = __shfl(live, m, 64);
        const int gm = __shfl(gx, m, 64), tm = __shfl(ty, m, 64);
        for (int l = lane; l < cm; l += 64) J.table[s0 + l] = run_ref(m, l, lv / gm, gm, tm, ry);
        // tiles that ran last step but not this one (as in plan_group)
        BatchRep<S> *R = reps[m];
        const int last = R->last_live;
        for (int b = lv + lane; b < last; b += 64) R->a.partials[kPartialSlots * b] = 0.0;
        if (lane == 0) R->last_live = lv;
    }
    // (the cross-lane read with every lane active: lane 63 must take part)
    const int total = __shfl(incl, 63, 64);
    if (lane == 0) *J.count = total;
}

// One block per windowed group (the first step of a run).
template <class S>
__global__ __launch_bounds__(kRedThreads) void plan_batch(const PlanJob *jobs)
{
    const PlanJob &J = jobs[blockIdx.x];
    if (J.n <= 64) {
        if (threadIdx.x < 64) plan_group_wave<S>(J);
        return;
    }
    plan_group<S>(J);
}

// One block per member of a group: the between-step work of the
// device-driven ones.
template <class S>
__global__ __launch_bounds__(kRedThreads) void finalize_batch(BatchRep<S> *const *reps, int k)
{
    const BatchRep<S> *R = reps[blockIdx.x];
    if (!R->device_driven) return;
    FinalizeArgs<S> fa = R->fa;
    const int64_t tt = R->t0 + k;
    const int cur = (R->cur0 + k) & 1;
    fa.f = R->f[cur ^ 1];
    fa.h_next = R->hs[(tt + 1) % 3];
    fa.h_clear = R->hs[(tt + 2) % 3];
    finalize_body<S>(fa);
}

template <class S>
__global__ void batch_advance(BatchRep<S> *const *reps, int n, int K)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        BatchRep<S> *R = reps[i];
        R->t0 += K;
        R->cur0 = (R->cur0 + K) & 1;
    }
}

// Calls f(DIV, SR) with std::bool_constant arguments for the run's growth
// law and rounding (stochastic rounding exists for the 16-bit storages).
template <class S, class F>
void by_variant(bool div, bool sr, F &&f)
{
    if constexpr (sizeof(S) == 2) {
        if (sr) {
            if (div) f(std::true_type{}, std::true_type{});
            else f(std::false_type{}, std::true_type{});
            return;
        }
    }
    if (div) f(std::true_type{}, std::false_type{});
    else f(std::false_type{}, std::false_type{});
}

}  // namespace lbm

#include "lbm_d2q7.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Launchers (host side)
// ---------------------------------------------------------------------------
template <class S, int RB>
void launch_step_rb(const StepArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    by_variant<S>(a.growth >= kGrowthDivision, a.sround != 0, [&](auto d, auto r) {
        constexpr bool DIV = decltype(d)::value, SR = decltype(r)::value;
        if (nt == 256) hipLaunchKernelGGL((step_kernel<S, 256, RB, DIV, SR>), grid, dim3(256), 0, s, a);
        else if (nt == 128) hipLaunchKernelGGL((step_kernel<S, 128, RB, DIV, SR>), grid, dim3(128), 0, s, a);
        else hipLaunchKernelGGL((step_kernel<S, 64, RB, DIV, SR>), grid, dim3(64), 0, s, a);
    });
}

template <class S, int ND>
void launch_vec_nt(const StepArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    by_variant<S>(a.growth >= kGrowthDivision, a.sround != 0, [&](auto d, auto r) {
        constexpr bool DIV = decltype(d)::value, SR = decltype(r)::value;
        if (nt == 256) hipLaunchKernelGGL((step_kernel_vec<S, 256, ND, DIV, SR>), grid, dim3(256), 0, s, a);
        else if (nt == 128) hipLaunchKernelGGL((step_kernel_vec<S, 128, ND, DIV, SR>), grid, dim3(128), 0, s, a);
        else hipLaunchKernelGGL((step_kernel_vec<S, 64, ND, DIV, SR>), grid, dim3(64), 0, s, a);
    });
}

// vb: bytes per lane (4, 8 or 16).
template <class S>
hipError_t launch_step_vec(const StepArgs<S> &a, dim3 grid, int nt, int vb, hipStream_t s)
{
    if (vb == 4) {
        if constexpr (sizeof(S) <= 4) launch_vec_nt<S, 1>(a, grid, nt, s);
        else return hipErrorInvalidValue;
    } else if (vb == 8) {
        launch_vec_nt<S, 2>(a, grid, nt, s);
    } else {
        launch_vec_nt<S, 4>(a, grid, nt, s);
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_step_staged(const StepArgs<S> &a, dim3 grid, hipStream_t s)
{
    constexpr StagedGeom G(sizeof(S));
    if (a.growth >= kGrowthDivision)
        hipLaunchKernelGGL((step_kernel_staged<S, true>), grid, dim3(64 * G.waves()), 0, s, a);
    else
        hipLaunchKernelGGL((step_kernel_staged<S, false>), grid, dim3(64 * G.waves()), 0, s, a);
    return hipGetLastError();
}

template <class S>
hipError_t launch_step(const StepArgs<S> &a, dim3 grid, int nt, int rb, hipStream_t s)
{
    if (rb >= 2) launch_step_rb<S, 2>(a, grid, nt, s);
    else launch_step_rb<S, 1>(a, grid, nt, s);
    return hipGetLastError();
}

template <class S>
hipError_t launch_init(const InitArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    if (nt == 256) hipLaunchKernelGGL((init_kernel<S, 256>), grid, dim3(256), 0, s, a);
    else if (nt == 128) hipLaunchKernelGGL((init_kernel<S, 128>), grid, dim3(128), 0, s, a);
    else hipLaunchKernelGGL((init_kernel<S, 64>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

template <class S>
hipError_t launch_mass(const MassArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    if (nt == 256) hipLaunchKernelGGL((mass_kernel<S, 256>), grid, dim3(256), 0, s, a);
    else if (nt == 128) hipLaunchKernelGGL((mass_kernel<S, 128>), grid, dim3(128), 0, s, a);
    else hipLaunchKernelGGL((mass_kernel<S, 64>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
}

template <class S>
hipError_t launch_finalize(const FinalizeArgs<S> &a, hipStream_t s)
{
    hipLaunchKernelGGL((finalize_kernel<S>), dim3(1), dim3(kRedThreads), 0, s, a);
    return hipGetLastError();
}

// The batch kernel of one form (nullptr if the form does not exist).
template <class S, int NT, bool DIV, bool SR>
const void *batch_kernel_div(int vec, int vb_or_rb)
{
    if (vec == 2)   // the D2Q7 step, one column per lane
        return vb_or_rb >= 2 ? (const void *)&step_batch7<S, NT, 2, false, DIV, SR>
                             : (const void *)&step_batch7<S, NT, 1, false, DIV, SR>;
    if (vec == 3) {   // the D2Q7 vector form
        if (vb_or_rb == 4) {
            if constexpr (sizeof(S) <= 4) return (const void *)&step_batch7<S, NT, 1, true, DIV, SR>;
            return nullptr;
        }
        return vb_or_rb == 8 ? (const void *)&step_batch7<S, NT, 2, true, DIV, SR>
                             : (const void *)&step_batch7<S, NT, 4, true, DIV, SR>;
    }
    if (vec) {
        if (vb_or_rb == 4) {
            if constexpr (sizeof(S) <= 4) return (const void *)&step_batch<S, NT, 1, true, DIV, SR>;
            return nullptr;
        }
        return vb_or_rb == 8 ? (const void *)&step_batch<S, NT, 2, true, DIV, SR>
                             : (const void *)&step_batch<S, NT, 4, true, DIV, SR>;
    }
    return vb_or_rb >= 2 ? (const void *)&step_batch<S, NT, 2, false, DIV, SR>
                         : (const void *)&step_batch<S, NT, 1, false, DIV, SR>;
}

template <class S>
const void *batch_kernel(int vec, int nt, int vb_or_rb, int div, int sr)
{
    const void *f = nullptr;
    by_variant<S>(div != 0, sr != 0, [&](auto d, auto r) {
        constexpr bool D = decltype(d)::value, R = decltype(r)::value;
        f = nt == 256   ? batch_kernel_div<S, 256, D, R>(vec, vb_or_rb)
            : nt == 128 ? batch_kernel_div<S, 128, D, R>(vec, vb_or_rb)
                        : batch_kernel_div<S, 64, D, R>(vec, vb_or_rb);
    });
    return f;
}

template <class S>
hipError_t launch_step_batch(BatchRep<S> *const *reps, const TileRef *table, const int32_t *count,
                             int grid, int vec, int nt, int vb_or_rb, int div, int sr, int k,
                             int K, GridBar *bar, hipStream_t s)
{
    if (grid <= 0 || K <= 0) return hipSuccess;
    if (K > 1 && !bar) return hipErrorInvalidValue;
    const void *f = batch_kernel<S>(vec, nt, vb_or_rb, div, sr);
    if (!f) return hipErrorInvalidValue;
    void *args[] = {(void *)&reps, (void *)&table, (void *)&count, (void *)&k, (void *)&K,
                    (void *)&bar};
    return bar ? hipLaunchCooperativeKernel(f, dim3(grid), dim3(nt), args, 0, s)
               : hipLaunchKernel(f, dim3(grid), dim3(nt), args, 0, s);
}

template <class S>
int batch_coop_grid(int vec, int nt, int vb_or_rb, int div, int sr, int device)
{
    const void *f = batch_kernel<S>(vec, nt, vb_or_rb, div, sr);
    int per_cu = 0, cus = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, nt, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return per_cu * cus;
}

template <class S>
hipError_t launch_plan_batch(const PlanJob *jobs, int njobs, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((plan_batch<S>), dim3(njobs), dim3(kRedThreads), 0, s, jobs);
    return hipGetLastError();
}

template <class S>
hipError_t launch_finalize_batch(BatchRep<S> *const *reps, int n, int k, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((finalize_batch<S>), dim3(n), dim3(kRedThreads), 0, s, reps, k);
    return hipGetLastError();
}

template <class S>
hipError_t launch_batch_advance(BatchRep<S> *const *reps, int n, int K, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((batch_advance<S>), dim3((n + 255) / 256), dim3(256), 0, s, reps, n, K);
    return hipGetLastError();
}

}  // namespace lbm
