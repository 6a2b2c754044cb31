// lbm_common.hip -- small non-templated kernels of the gfx950 library: fills,
// device-state set-up and the diagnostics reduction; the static scratch of
// handles created without a workspace.
#include "lbm_step.hpp"

#include <mutex>

namespace lbm {

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_f64_kernel(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void state_set_kernel(DevState *st, int64_t y_wall, int64_t y_valid_top,
                                 int64_t n_rows, int64_t h_hi)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->y_wall = y_wall;
        st->y_valid_top = y_valid_top;
        st->n_rows = n_rows;
        st->h_hi = h_hi;
        st->retired_total = 0.0;
        st->retired_last = 0.0;
        st->status = 0u;
        st->lam = 0.0;
        st->p0 = 1.0;
    }
}

// Division laws: the next step's rate from the tallies in the device state's
// slots (one lane per slot), which it clears, and the divisions they count.
// Used after a state is set from outside (its creation or
// lbm_set_populations: no divisions counted) and between the steps of a run
// whose wall and sweep window stay put (nothing retired, so the rate is the
// one the full between-step kernel would compute from the same integers).
__global__ __launch_bounds__(kDivSlots) void rates_kernel(int growth, double g, double rho_cell,
                                                          DevState *st)
{
    static_assert(kDivSlots == 64, "one wavefront, one lane per slot");
    long long mfx = 0, wsum = 0, ndiv = 0;
    take_div_slots(st, mfx, wsum, ndiv);
    mfx = wave_reduce(mfx);
    wsum = wave_reduce(wsum);
    ndiv = wave_reduce(ndiv);
    if (threadIdx.x == 0)
        set_division_rate(st, growth, division_lam(growth == kGrowthDivision, g, rho_cell, mfx, wsum),
                          ndiv);
}

hipError_t launch_rates(int growth, double g, double rho_cell, DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(rates_kernel, dim3(1), dim3(kDivSlots), 0, s, growth, g, rho_cell, st);
    return hipGetLastError();
}

// Diagnostics of the current state.
__global__ __launch_bounds__(kRedThreads) void diag_kernel(DiagArgs a)
{
    __shared__ double shd[3][kRedWaves];
    __shared__ long long shi[2][kRedWaves];
    double v[3] = {0.0, 0.0, 0.0};   // mass, injected, fix
    for (int b = threadIdx.x; b < a.nblocks; b += kRedThreads) {
        const double *p = a.partials + kPartialSlots * b;
        v[0] += p[0];
        v[1] += p[1];
        v[2] += p[2];
    }
    block_reduce(v, shd);
    const double m = v[0], s = v[1], fx = v[2];
    const int64_t y_wall = a.st->y_wall;
    long long si[2] = {0, 0};
    long long hm[1] = {LLONG_MIN};
    height_sums(a.h_cur, a.colmax, a.L, y_wall, si[0], si[1], hm[0]);
    block_reduce(si, shi);
    block_reduce(hm, shi, OpMax());
    double hbar, W;
    height_stats(si[0], si[1], a.L, y_wall, hbar, W);
    const long long hi = hm[0];
    if (threadIdx.x == 0) {
        DiagOut *o = a.out;
        const double mass = m - a.st->retired_last;
        uint32_t st = a.st->status;
        if (!isfinite(mass)) {
            st |= kStNonFinite;
            a.st->status = st;
        }
        o->mass = mass;
        o->src_total = s;
        o->fix_total = fx;
        o->retired = a.st->retired_total;
        o->hbar = hbar;
        o->W = W;
        o->y_wall = y_wall;
        o->h_hi = hi;
        o->status = st;
        o->lam = a.st->lam;
        o->divisions = a.st->divisions;
        o->rows_swept = a.st->rows_swept;
    }
}

hipError_t launch_diag(const DiagArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(kRedThreads), 0, s, a);
    return hipGetLastError();
}

// Streaming copy: each thread moves kCopyUnroll 16-byte vectors with
// nontemporal loads and stores, all its loads in flight before the first
// store; a block covers kCopyUnroll x kCopyThreads consecutive vectors, so
// every access is coalesced.  One vector per thread in blocks of 512
// measured fastest (6.4-6.6 TB/s over 0.3-2 GB each way, against 6.2-6.3 for
// four per thread and 5.9-6.1 without the nontemporal hints).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 512, kCopyUnroll = 1;

__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(u32x4 *dst, const u32x4 *src,
                                                                   int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kCopyThreads;
        if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kCopyThreads;
        if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
}

hipError_t launch_stream_copy(void *dst, const void *src, int64_t n16, hipStream_t s)
{
    if (n16 <= 0) return hipSuccess;
    const int64_t per_block = kCopyThreads * kCopyUnroll;
    const int64_t blocks = (n16 + per_block - 1) / per_block;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s,
                       reinterpret_cast<u32x4 *>(dst), reinterpret_cast<const u32x4 *>(src), n16);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Scratch of the handle created by lbm_create_static (one live such handle
// per device): its front-height slots, tallies, device state, diagnostics
// record and batch descriptor.  Each device holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in: only the
// address from hipGetSymbolAddress may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_of(hipStream_t s, int *device, void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    int dev = cur;
    if (s) {
        hipDevice_t d;
        if ((e = hipStreamGetDevice(s, &d)) != hipSuccess) return e;
        dev = (int)d;
    }
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        // look the array up with its device current
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *device = dev;
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_state_set(DevState *st, int64_t y_wall, int64_t y_valid_top, int64_t n_rows,
                            int64_t h_hi, hipStream_t s)
{
    hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, st, y_wall, y_valid_top,
                       n_rows, h_hi);
    return hipGetLastError();
}

}  // namespace lbm
