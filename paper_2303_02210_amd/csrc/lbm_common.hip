// lbm_common.hip -- small non-templated kernels of the gfx950 library: fills,
// device-state set-up and the diagnostics reduction.
#include "lbm_step.hpp"

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
    }
}

// Diagnostics of the current state.
__global__ __launch_bounds__(kRedThreads) void diag_kernel(DiagArgs a)
{
    __shared__ double shd[kRedThreads / 64];
    __shared__ long long shi[kRedThreads / 64];
    double m = 0.0, s = 0.0, fx = 0.0;
    for (int b = threadIdx.x; b < a.nblocks; b += kRedThreads) {
        m += a.partials[4 * b + 0];
        s += a.partials[4 * b + 1];
        fx += a.partials[4 * b + 2];
    }
    m = block_sum_d(m, shd);
    s = block_sum_d(s, shd);
    fx = block_sum_d(fx, shd);
    const int64_t y_wall = a.st->y_wall;
    double hbar, W;
    long long hmax;
    height_stats(a.h_cur, a.L, y_wall, shi, hbar, W, hmax);
    long long hi = LLONG_MIN;
    for (int x = threadIdx.x; x < a.L; x += kRedThreads)
        hi = (long long)a.colmax[x] > hi ? (long long)a.colmax[x] : hi;
    hi = block_max_i(hi, shi);
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
    }
}

hipError_t launch_diag(const DiagArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(diag_kernel, dim3(1), dim3(kRedThreads), 0, s, a);
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

hipError_t launch_state_set(DevState *st, int64_t y_wall, int64_t y_valid_top, int64_t n_rows,
                            int64_t h_hi, hipStream_t s)
{
    hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, st, y_wall, y_valid_top,
                       n_rows, h_hi);
    return hipGetLastError();
}

}  // namespace lbm
