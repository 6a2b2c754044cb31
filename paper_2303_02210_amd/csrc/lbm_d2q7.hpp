// lbm_d2q7.hpp -- the fused step on the paper's own triangular D2Q7 lattice
// (Sec. II): six unit directions at multiples of pi/3 plus rest, weights 1/2
// and 1/12, c_s^2 = 1/4, so the steady state of Eq. 3 is
// w_i rho (1 + 4 e.u* + 8 (e.u*)^2 - 2 |u*|^2) and the noise of Eq. 4
// subtracts the mean over seven directions.
//
// Geometry: rows are horizontal lines sqrt(3)/2 apart and odd rows sit half a
// unit to the right, so site (x, y) is at (x + (y mod 2)/2, y sqrt(3)/2)
// (parity of the absolute row).  Directions: 0 rest, 1 E, 2 NE, 3 NW, 4 W,
// 5 SW, 6 SE; reverse pairs 1-4, 2-5, 3-6.  The upstream neighbour half a
// unit to the left in the row below or above is column x - 1 + par, half a
// unit to the right column x + par (par = y mod 2).
//
// Two forms: one column per lane, each lane loading its seven pulls directly
// (the lanes of a wave read contiguous runs of each row), and a vector form
// with several columns per lane; both with the same row bookkeeping,
// rear-wall reflection, tallies and front heights as the D2Q9 forms.
// Included by lbm_step.hpp after the shared pieces.
#pragma once

namespace lbm {

constexpr int kOpp7[7] = {0, 4, 5, 6, 1, 2, 3};
constexpr double kSin60 = 0.86602540378443864676;   // sqrt(3)/2

template <class R>
__device__ __forceinline__ R sum7(const R v[7])
{
    R s = v[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) s = s + v[i];
    return s;
}

// Steps 2-7 of Appendix A at a D2Q7 tissue site (streamed density rho_s >=
// rho_c), in the same order of operations as the D2Q9 form.
template <class S, bool DIV>
__device__ __forceinline__ void tissue_update7(const StepArgs<S> &a, uint32_t t,
                                               typename Codec<S>::R fs[7],
                                               typename Codec<S>::R rho_s,
                                               typename Codec<S>::R out[7], uint32_t x, int64_t y,
                                               int64_t y_wall, int32_t hp, double &s_acc,
                                               double &x_acc, DivTally &dv)
{
    using R = typename Codec<S>::R;
    // ---- step 2 (rest): momentum, e_i = (cos, sin)((i - 1) pi/3) ------------
    const R jx = (fs[1] - fs[4]) + R(0.5) * (((fs[2] - fs[3]) + fs[6]) - fs[5]);
    const R jy = R(kSin60) * (((fs[2] + fs[3]) - fs[5]) - fs[6]);
    // ---- step 3: growth source, its expectation shared by six directions ----
    bool in_reg = true;
    if (a.region == kRegionFrontBand) in_reg = (y >= (int64_t)hp - a.region_width);
    else if (a.region == kRegionRearBand) in_reg = (y < y_wall + a.region_width);
    R S_ = (a.growth == kGrowthBulk && in_reg) ? a.g * rho_s : R(0);
    const R s6 = S_ / R(6);
#pragma unroll
    for (int i = 1; i < 7; ++i) fs[i] = fs[i] + s6;
    // Division laws: as on D2Q9, with three axes, each division's axis one
    // base-3 digit of the 64 random bits
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
                const int k = uniform ? poisson_k_from(U, l, dv.p0) : poisson_k_small(U, l);
                int count[3] = {0, 0, 0};
                for (int d = 0; d < k; ++d) {
                    count[axes % 3u] += 1;
                    axes = axes / 3u;
                }
                const double half = a.rho_cell * 0.5;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double amount = (double)count[c] * half;
                    fs[c + 1] = fs[c + 1] + (R)amount;
                    fs[c + 4] = fs[c + 4] + (R)amount;
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
    const R u2 = R(2) * usq;
    const R ah = R(0.5) * ux;
    const R bh = R(kSin60) * uy;
    R cu[7];
    cu[0] = R(0);
    cu[1] = ux;
    cu[2] = ah + bh;
    cu[3] = bh - ah;
    cu[4] = -cu[1];
    cu[5] = -cu[2];
    cu[6] = -cu[3];
    // ---- step 5 (tissue): relax towards f^SS (Eq. 2) --------------------------
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const R c = cu[i];
        const R fss = (a.w[dclass7(i)] * rho) * (((R(1) + R(4) * c) + R(8) * (c * c)) - u2);
        out[i] = fs[i] - a.omega * (fs[i] - fss);
    }
    // ---- step 6: zero-sum noise where rho > rho_c (Eq. 4), seven draws -------
    if (a.noise && rho > a.rho_c) {
        R v[9];
        noise_factors<R>(a.seed, a.replica, t, x, (uint32_t)y, v);
        R eta[7];
#pragma unroll
        for (int i = 0; i < 7; ++i) eta[i] = a.sigma * v[i];
        const R m = sum7(eta) / R(7);
#pragma unroll
        for (int i = 0; i < 7; ++i) out[i] = out[i] + (eta[i] - m);
    }
    // ---- step 7: negative populations --------------------------------------------
    bool neg = false;
#pragma unroll
    for (int i = 0; i < 7; ++i) neg = neg || (out[i] < R(0));
    if (neg) {
        const R before = sum7(out);
        if (out[0] < R(0)) {
            const R rho_pre = sum7(out);
            out[0] = R(0);
            const R rest = sum7(out);
            if (rest > R(0)) {
                const R r = rho_pre / rest;
#pragma unroll
                for (int i = 0; i < 7; ++i) out[i] = out[i] * r;
            }
        }
#pragma unroll
        for (int i = 1; i < 7; ++i) {
            if (out[i] < R(0)) {
                out[kOpp7[i]] = out[kOpp7[i]] + (-out[i]);
                out[i] = R(0);
            }
        }
        x_acc += (double)(sum7(out) - before);
    }
}

// Steps 2-7 at one D2Q7 site from its seven streamed stored values v (fs: the
// decoded values, validity applied).  Writes the stored result to so[7];
// returns true for tissue.
template <class S, bool DIV, bool SR = false>
__device__ __forceinline__ bool site_step7(const StepArgs<S> &a, uint32_t t, const S v[7],
                                           typename Codec<S>::R fs[7],
                                           const typename Codec<S>::R Wd[7], S so[7], uint32_t x,
                                           int64_t y, int64_t y_wall, int32_t hp, double &m_acc,
                                           double &s_acc, double &x_acc, long long &mfx_acc,
                                           DivTally &dv)
{
    using R = typename Codec<S>::R;
    const R rho_s = sum7(fs);
    if (rho_s >= a.rho_c) {
        R out[7];
        tissue_update7<S, DIV>(a, t, fs, rho_s, out, x, y, y_wall, hp, s_acc, x_acc, dv);
        R kept[7];
        encode_site<S, 7, SR>(a, t, x, y, out, Wd, so, kept);
        const R m = sum7(kept);
        m_acc += (double)m;
        if constexpr (DIV) mfx_acc += mass_fx(m);
        return true;
    }
    // ---- step 5 (void): reverse every direction ------------------------------------
#pragma unroll
    for (int i = 0; i < 7; ++i) so[i] = v[kOpp7[i]];
    m_acc += (double)rho_s;
    if constexpr (DIV) {
        R m = fs[kOpp7[0]];
#pragma unroll
        for (int i = 1; i < 7; ++i) m = m + fs[kOpp7[i]];
        mfx_acc += mass_fx(m);
    }
    return false;
}

// The D2Q7 step over one tile: NT columns (one per lane) by `ty` rows,
// visited RB rows at a time with all 7 RB loads issued before any is used.
template <class S, int NT, int RB, bool DIV, bool SR = false>
__device__ __forceinline__ void step_tile7(const StepArgs<S> &a, const StepIO<S> &io, int bx,
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
    long long mfx_acc = 0;
    DivTally dv;
    if constexpr (DIV) dv = div_begin(a.st);
    int64_t ymax = -1;
    const int32_t hp = (a.region == kRegionFrontBand) ? io.h_prev[x] : 0;
    R Wd[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) Wd[i] = a.Wd[dclass7(i)];

    const Tiles tl = a.tl;
    const int64_t cx = tl.col(x), cxm = tl.col(xm), cxp = tl.col(xp);
    const int tws = tl.tws;
    const MemT<S> LBM_GLOBAL *__restrict__ F = as_global(reinterpret_cast<const MemT<S> *>(io.fin));
    MemT<S> LBM_GLOBAL *__restrict__ G = as_global(reinterpret_cast<MemT<S> *>(io.fout));
    int rnext = (a.mode == kModeDevice) ? (int)((y_wall + j0) % H) : j0;

    for (int jb = j0; jb < jend; jb += RB) {
        S raw[RB][7];
        RowSrc src[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int j = jb + k;
            const int64_t y = y_wall + j;
            src[k] = row_sources(a.mode, j, rnext, H, y, y_top);
            rnext = src[k].rp;
            if (j < jend) {
                const RowSrc &s = src[k];
                const bool odd = (y & 1) != 0;
                // ---- step 1: pull-stream; the wall reflects NE / NW in place -----
                const MemT<S> LBM_GLOBAL *row0 = F + (int64_t)s.r0 * tl.rs;
                const MemT<S> LBM_GLOBAL *rowm = F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs;
                const MemT<S> LBM_GLOBAL *rowp = F + (int64_t)s.rp * tl.rs;
                const int qn2 = s.below ? 5 : 2, qn3 = s.below ? 6 : 3;
                const int64_t c2 = s.below ? cx : (odd ? cx : cxm);   // from below-left
                const int64_t c3 = s.below ? cx : (odd ? cxp : cx);   // from below-right
                const int64_t c5 = odd ? cxp : cx;                    // from above-right
                const int64_t c6 = odd ? cx : cxm;                    // from above-left
                raw[k][0] = from_mem<S>(row0[cx + (0 << tws)]);
                raw[k][1] = from_mem<S>(row0[cxm + (1 << tws)]);
                raw[k][4] = from_mem<S>(row0[cxp + (4 << tws)]);
                raw[k][2] = from_mem<S>(rowm[c2 + (qn2 << tws)]);
                raw[k][3] = from_mem<S>(rowm[c3 + (qn3 << tws)]);
                raw[k][5] = from_mem<S>(rowp[c5 + (5 << tws)]);
                raw[k][6] = from_mem<S>(rowp[c6 + (6 << tws)]);
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int j = jb + k;
            if (j >= jend) break;
            const int64_t y = y_wall + j;
            const RowSrc &s = src[k];
            S v[7];
            R fs[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                v[i] = raw[k][i];
                fs[i] = Codec<S>::dec(v[i], Wd[i]);
            }
            // sources that hold no live data stream in nothing
            if (!s.v0) {
                v[0] = Codec<S>::enc(R(0), Wd[0]);
                v[1] = v[4] = Codec<S>::enc(R(0), Wd[1]);
                fs[0] = fs[1] = fs[4] = R(0);
            }
            if (!s.below && !s.vm) {
                v[2] = v[3] = Codec<S>::enc(R(0), Wd[2]);
                fs[2] = fs[3] = R(0);
            }
            if (!s.vp) {
                v[5] = v[6] = Codec<S>::enc(R(0), Wd[5]);
                fs[5] = fs[6] = R(0);
            }
            S so[7];
            double m_site = 0.0, s_site = 0.0, x_site = 0.0;
            long long mfx_site = 0;
            DivTally dv_site = div_site(dv);
            const bool tissue = site_step7<S, DIV, SR>(a, io.t, v, fs, Wd, so, x, y, y_wall, hp,
                                                   m_site, s_site, x_site, mfx_site, dv_site);
            MemT<S> LBM_GLOBAL *rowg = G + (int64_t)s.r0 * tl.rs + cx;
            if (active) {
#pragma unroll
                for (int i = 0; i < 7; ++i) rowg[i << tws] = to_mem<S>(so[i]);
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
        for (int i = 1; i < nstrips; ++i) a.partials[kPartialSlots * ((by + i) * nbx + bx)] = 0.0;
    }
}

// The D2Q7 step with ND dwords (V = 4 ND / sizeof(S) consecutive columns) per
// lane: per row the seven vector loads and six wave-edge values, the +-x
// neighbours across lanes by DPP moves, and the same load/store ordering,
// empty-wavefront skip and tallies as the D2Q9 vector form.  Which diagonal
// pulls take the neighbouring column depends on the row's parity
// (wave-uniform): NE and SE from x - 1 on even rows, NW and SW from x + 1 on
// odd rows, the others from x itself.
template <class S, int NT, int ND, bool DIV, bool SR = false>
__device__ __forceinline__ void step_vec_tile7(const StepArgs<S> &a, const StepIO<S> &io, int bx,
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
    long long mfx_acc = 0;
    DivTally dv;
    if constexpr (DIV) dv = div_begin(a.st);
    int32_t jmax[V], hp[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        jmax[i] = -1;
        hp[i] = (a.region == kRegionFrontBand && active) ? io.h_prev[xv + i] : 0;
    }
    R Wd[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) Wd[i] = a.Wd[dclass7(i)];
    uint32_t epat[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        if constexpr (sizeof(S) == 2) {
            const uint32_t b = to_mem<S>(Codec<S>::enc(R(0), Wd[i]));
            epat[i] = b | (b << 16);
        } else {
            epat[i] = 0u;
        }
    }

    const Tiles tl = a.tl;
    const int tws = tl.tws;
    const int64_t cv = tl.col(active ? xv : L - V), cl = tl.col(xl), cr = tl.col(xr);
    const MemT<S> LBM_GLOBAL *__restrict__ F = as_global(reinterpret_cast<const MemT<S> *>(io.fin));
    MemT<S> LBM_GLOBAL *__restrict__ G = as_global(reinterpret_cast<MemT<S> *>(io.fout));
    int r0 = (a.mode == kModeDevice) ? (int)((y_wall + j0) % H) : j0;

    struct Fetch {
        VT A[7];
        S e[6];   // E, W, NE, NW, SW, SE sources beyond the wave's edges
    };
    constexpr uint32_t EB = sizeof(MemT<S>);
    const uint32_t loff = (uint32_t)(cv * EB);
    const int64_t rowbytes = tl.rs * EB;
    const auto pl = [&](int q) { return ((uint32_t)q << tws) * EB; };
    auto fetch = [&](int j, int r, Fetch &f) {
        const RowSrc s = row_sources(a.mode, j, r, H, y_wall + j, y_top);
        // NE / NW pull from the row below, or from this site reflected (SW / SE)
        const int qn2 = s.below ? 5 : 2, qn3 = s.below ? 6 : 3;
        if constexpr (sizeof(S) != 2) {
            const MemT<S> LBM_GLOBAL *row0 = F + (int64_t)s.r0 * tl.rs;
            const MemT<S> LBM_GLOBAL *rowm = F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs;
            const MemT<S> LBM_GLOBAL *rowp = F + (int64_t)s.rp * tl.rs;
            f.A[0] = vload<ND>(row0 + cv + (0 << tws));
            f.A[1] = vload<ND>(row0 + cv + (1 << tws));
            f.A[4] = vload<ND>(row0 + cv + (4 << tws));
            f.A[2] = vload<ND>(rowm + cv + (qn2 << tws));
            f.A[3] = vload<ND>(rowm + cv + (qn3 << tws));
            f.A[5] = vload<ND>(rowp + cv + (5 << tws));
            f.A[6] = vload<ND>(rowp + cv + (6 << tws));
            f.e[0] = from_mem<S>(row0[cl + (1 << tws)]);
            f.e[1] = from_mem<S>(row0[cr + (4 << tws)]);
            f.e[2] = from_mem<S>(rowm[cl + (2 << tws)]);
            f.e[3] = from_mem<S>(rowm[cr + (3 << tws)]);
            f.e[4] = from_mem<S>(rowp[cr + (5 << tws)]);
            f.e[5] = from_mem<S>(rowp[cl + (6 << tws)]);
            return;
        }
        const __amdgpu_buffer_rsrc_t R0 =
            row_rsrc<true>((const void *)(F + (int64_t)s.r0 * tl.rs), rowbytes);
        const __amdgpu_buffer_rsrc_t Rm =
            row_rsrc<true>((const void *)(F + (int64_t)(s.below ? s.r0 : s.rm) * tl.rs), rowbytes);
        const __amdgpu_buffer_rsrc_t Rp =
            row_rsrc<true>((const void *)(F + (int64_t)s.rp * tl.rs), rowbytes);
        f.A[0] = bload<ND>(R0, loff, pl(0));
        f.A[1] = bload<ND>(R0, loff, pl(1));
        f.A[4] = bload<ND>(R0, loff, pl(4));
        f.A[2] = bload<ND>(Rm, loff, pl(qn2));
        f.A[3] = bload<ND>(Rm, loff, pl(qn3));
        f.A[5] = bload<ND>(Rp, loff, pl(5));
        f.A[6] = bload<ND>(Rp, loff, pl(6));
        f.e[0] = bload_el<S>(R0, (uint32_t)(cl * EB) + pl(1));
        f.e[1] = bload_el<S>(R0, (uint32_t)(cr * EB) + pl(4));
        f.e[2] = bload_el<S>(Rm, (uint32_t)(cl * EB) + pl(2));
        f.e[3] = bload_el<S>(Rm, (uint32_t)(cr * EB) + pl(3));
        f.e[4] = bload_el<S>(Rp, (uint32_t)(cr * EB) + pl(5));
        f.e[5] = bload_el<S>(Rp, (uint32_t)(cl * EB) + pl(6));
    };
    Fetch cur;
    VT O[7];
    auto update_row = [&](int j, int r) -> RowSrc {
        const int64_t y = y_wall + j;
        const bool odd = (y & 1) != 0;
        const RowSrc s = row_sources(a.mode, j, r, H, y, y_top);
        const VT A0 = cur.A[0], A1 = cur.A[1], A2 = cur.A[2], A3 = cur.A[3];
        const VT A4 = cur.A[4], A5 = cur.A[5], A6 = cur.A[6];
        // neighbours across lanes: from x - 1 (E, NE, SE) and x + 1 (W, NW, SW)
        const S n1 = from_left<S, ND>(A1, cur.e[0], edge_l);
        const S n4 = from_right<S, ND>(A4, cur.e[1], edge_r);
        const S n2 = from_left<S, ND>(A2, cur.e[2], edge_l);
        const S n3 = from_right<S, ND>(A3, cur.e[3], edge_r);
        const S n5 = from_right<S, ND>(A5, cur.e[4], edge_r);
        const S n6 = from_left<S, ND>(A6, cur.e[5], edge_l);

        // an exactly empty neighbourhood over the whole wavefront: skip
        bool busy = false;
        {
            const VT *Av[7] = {&A0, &A1, &A2, &A3, &A4, &A5, &A6};
#pragma unroll
            for (int q = 0; q < 7; ++q)
#pragma unroll
                for (int d = 0; d < ND; ++d) busy = busy || ((*Av[q])[d] != epat[q]);
            constexpr int eq[6] = {1, 4, 2, 3, 5, 6};
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                typename RawVec<ND>::type t;
#pragma unroll
                for (int d = 0; d < ND; ++d) t[d] = epat[eq[i]];
                busy = busy || (to_mem<S>(cur.e[i]) != to_mem<S>(get_el<S, ND>(t, 0)));
            }
        }
        uint32_t tmask = 0;
        if (__builtin_amdgcn_ballot_w64(busy) == 0) {
#pragma unroll
            for (int q = 0; q < 7; ++q)
#pragma unroll
                for (int d = 0; d < ND; ++d) O[q][d] = epat[q];
        } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            S v[7];
            const S left1 = (k == 0) ? n1 : get_el<S, ND>(A1, k == 0 ? 0 : k - 1);
            const S right4 = (k == V - 1) ? n4 : get_el<S, ND>(A4, k == V - 1 ? k : k + 1);
            const S left2 = (k == 0) ? n2 : get_el<S, ND>(A2, k == 0 ? 0 : k - 1);
            const S right3 = (k == V - 1) ? n3 : get_el<S, ND>(A3, k == V - 1 ? k : k + 1);
            const S right5 = (k == V - 1) ? n5 : get_el<S, ND>(A5, k == V - 1 ? k : k + 1);
            const S left6 = (k == 0) ? n6 : get_el<S, ND>(A6, k == 0 ? 0 : k - 1);
            v[0] = get_el<S, ND>(A0, k);
            v[1] = left1;
            v[4] = right4;
            if (s.below) {
                v[2] = get_el<S, ND>(A2, k);
                v[3] = get_el<S, ND>(A3, k);
            } else {
                v[2] = odd ? get_el<S, ND>(A2, k) : left2;
                v[3] = odd ? right3 : get_el<S, ND>(A3, k);
            }
            v[5] = odd ? right5 : get_el<S, ND>(A5, k);
            v[6] = odd ? get_el<S, ND>(A6, k) : left6;
            R fs[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) fs[i] = Codec<S>::dec(v[i], Wd[i]);
            if (!s.v0) {
                v[0] = Codec<S>::enc(R(0), Wd[0]);
                v[1] = v[4] = Codec<S>::enc(R(0), Wd[1]);
                fs[0] = fs[1] = fs[4] = R(0);
            }
            if (!s.below && !s.vm) {
                v[2] = v[3] = Codec<S>::enc(R(0), Wd[2]);
                fs[2] = fs[3] = R(0);
            }
            if (!s.vp) {
                v[5] = v[6] = Codec<S>::enc(R(0), Wd[5]);
                fs[5] = fs[6] = R(0);
            }
            S so[7];
            double m_site = 0.0, s_site = 0.0, x_site = 0.0;
            const uint32_t x = (uint32_t)(xv + k);
            int32_t hpk = hp[0];
#pragma unroll
            for (int d = 1; d < V; ++d) hpk = (k == d) ? hp[d] : hpk;
            long long mfx_site = 0;
            DivTally dv_site = div_site(dv);
            const bool tissue = site_step7<S, DIV, SR>(a, io.t, v, fs, Wd, so, x, y, y_wall, hpk,
                                                   m_site, s_site, x_site, mfx_site, dv_site);
#pragma unroll
            for (int i = 0; i < 7; ++i) put_el<S, ND>(O[i], k, so[i]);
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
        for (int i = 0; i < 7; ++i) bstore<ND>(rr, soff, pl(i), O[i]);
    };
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

    block_tallies<NT, DIV>(m_acc, s_acc, x_acc, mfx_acc, dv, a.st, by * nbx + bx);
    double *pb = a.partials + kPartialSlots * (by * nbx + bx);
    if (threadIdx.x == 0) {
        pb[0] = m_acc;
        pb[1] += s_acc;
        pb[2] += x_acc;
        for (int i = 1; i < nstrips; ++i) a.partials[kPartialSlots * ((by + i) * nbx + bx)] = 0.0;
    }
}

template <class S, int NT, int ND, bool DIV, bool SR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(vec_waves<S, ND, DIV || SR>())))
void step_kernel_vec7(StepArgs<S> a)
{
    const int nbx = gridDim.x;
    const int lin = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y, nbx * a.xcd_rows,
                              a.strip_mul);
    const StepIO<S> io = step_io(a);
    step_vec_tile7<S, NT, ND, DIV, SR>(a, io, lin % nbx, lin / nbx, nbx);
}

template <class S, int NT, int RB, bool DIV, bool SR>
__global__ __launch_bounds__(NT) void step_kernel7(StepArgs<S> a)
{
    const int nbx = gridDim.x;
    const int lin = xcd_order(blockIdx.y * nbx + blockIdx.x, nbx * gridDim.y, nbx * a.xcd_rows,
                              a.strip_mul);
    const StepIO<S> io = step_io(a);
    step_tile7<S, NT, RB, DIV, SR>(a, io, lin % nbx, lin / nbx, nbx);
}

// Batches: as step_batch, with a D2Q7 tile body (VEC: ND dwords per lane,
// else one column per lane with ND rows' loads at once).
template <class S, int NT, int ND, bool VEC, bool DIV, bool SR>
__global__ __launch_bounds__(NT) void step_batch7(BatchRep<S> *const *reps, const TileRef *table,
                                                  const int32_t *count, int k, int K, GridBar *bar)
{
    const int total = *count;
    for (int s = 0; s < K; ++s) {
        for (int c = blockIdx.x; c < total; c += gridDim.x) {
            const TileRef e = table[xcd_order(c, total, 2)];
            const BatchRep<S> R = load_descriptor<BatchRep<S>>(reps[e.rep]);
            const StepIO<S> io = batch_io(&R, k + s);
            const int bx = e.local0 % R.gx, by = e.local0 / R.gx;
            if constexpr (VEC) step_vec_tile7<S, NT, ND, DIV, SR>(R.a, io, bx, by, R.gx, e.n);
            else step_tile7<S, NT, ND, DIV, SR>(R.a, io, bx, by, R.gx, e.n);
        }
        if (s + 1 < K && !grid_barrier(bar)) {
            batch_sync_lost(reps, table, total);
            return;
        }
    }
}

template <class S, int RB, bool DIV, bool SR>
void launch_step7_rb(const StepArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    if (nt == 256) hipLaunchKernelGGL((step_kernel7<S, 256, RB, DIV, SR>), grid, dim3(256), 0, s, a);
    else if (nt == 128) hipLaunchKernelGGL((step_kernel7<S, 128, RB, DIV, SR>), grid, dim3(128), 0, s, a);
    else hipLaunchKernelGGL((step_kernel7<S, 64, RB, DIV, SR>), grid, dim3(64), 0, s, a);
}

template <class S, int ND, bool DIV, bool SR>
void launch_vec7_nt(const StepArgs<S> &a, dim3 grid, int nt, hipStream_t s)
{
    if (nt == 256) hipLaunchKernelGGL((step_kernel_vec7<S, 256, ND, DIV, SR>), grid, dim3(256), 0, s, a);
    else if (nt == 128) hipLaunchKernelGGL((step_kernel_vec7<S, 128, ND, DIV, SR>), grid, dim3(128), 0, s, a);
    else hipLaunchKernelGGL((step_kernel_vec7<S, 64, ND, DIV, SR>), grid, dim3(64), 0, s, a);
}

template <class S, bool DIV, bool SR>
void launch_vec7(const StepArgs<S> &a, dim3 grid, int nt, int vb, hipStream_t s)
{
    if (vb == 4) {
        if constexpr (sizeof(S) <= 4) launch_vec7_nt<S, 1, DIV, SR>(a, grid, nt, s);
    } else if (vb == 8) {
        launch_vec7_nt<S, 2, DIV, SR>(a, grid, nt, s);
    } else {
        launch_vec7_nt<S, 4, DIV, SR>(a, grid, nt, s);
    }
}

// vb: bytes per lane of the vector form (4, 8 or 16), 0 for one column per
// lane with rb rows' loads at once.
template <class S>
hipError_t launch_step7(const StepArgs<S> &a, dim3 grid, int nt, int vb, int rb, hipStream_t s)
{
    if (vb == 4 && sizeof(S) > 4) return hipErrorInvalidValue;
    by_variant<S>(a.growth >= kGrowthDivision, a.sround != 0, [&](auto d, auto r) {
        constexpr bool DIV = decltype(d)::value, SR = decltype(r)::value;
        if (vb > 0) launch_vec7<S, DIV, SR>(a, grid, nt, vb, s);
        else if (rb >= 2) launch_step7_rb<S, 2, DIV, SR>(a, grid, nt, s);
        else launch_step7_rb<S, 1, DIV, SR>(a, grid, nt, s);
    });
    return hipGetLastError();
}

}  // namespace lbm
