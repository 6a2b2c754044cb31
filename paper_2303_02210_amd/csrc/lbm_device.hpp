// lbm_device.hpp -- device-side building blocks of the gfx950 growing-tissue
// lattice Boltzmann library: the D2Q9 lattice, the Philox4x32-10 counter-based
// generator and the population storage codecs.
//
// Lattice (square D2Q9; the paper's Eq. 3 and Eq. 4 written for it): weights
// 4/9 (rest), 1/9 (axes), 1/36 (diagonals), c_s^2 = 1/3.  Directions:
// 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace lbm {

// Direction classes: the directions of a class share their weight, so their
// storage offsets and empty patterns are equal too.  Kernels read one value
// per class (D2Q9: rest 0, axes 1, diagonals 5; D2Q7: rest 0, the six
// neighbours 1), which keeps three (two) scalar registers live instead of
// nine (seven).
__host__ __device__ constexpr int dclass9(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 5); }
__host__ __device__ constexpr int dclass7(int i) { return i == 0 ? 0 : 1; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Ten rounds of: two 32x32->64 multiplications of
// counter words 0 and 2, halves swapped and xored with counter words 1, 3 and
// the key; the key advances by the two Weyl increments between rounds.
//
// SCALAR_KEYS: the key (seed, replica) is wave-uniform at every call site, a
// run's constant; pinning it to two scalar registers at the call makes each
// round's key a scalar add there, where the compiler would otherwise keep all
// twenty round keys of a kernel live across its row loop.  In the float
// kernels those twenty ran out of scalar registers (spilled to vector lanes
// and reloaded at every call, with a few vector spills to scratch); pinned,
// they measured 1-1.6 points of 8 TB/s faster on every 16-bit form and level
// on float32, but 2.5 points slower on the float64 step, which keeps the
// unpinned form.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t v[4];
};

template <bool SCALAR_KEYS = false>
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
    if constexpr (SCALAR_KEYS) asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    U4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Counter word 3 is 4 * stream + call.
enum : uint32_t { kStreamNoise = 0, kStreamInit = 1, kStreamDivision = 2, kStreamRound = 3 };

// Nine 24-bit draws for the noise of site (x, y) at step t: the top 24 bits of
// the eight words of calls 0 and 1, and the low bytes of call 0's words 0-2.
// Returned as the exact factors v_i = (2 k_i + 1 - 2^24) 2^-24 in (-1, 1), so
// that eta~_i = sigma v_i is uniform on (-sigma, sigma).
template <class R>
__device__ __forceinline__ void noise_factors(uint32_t seed, uint32_t replica, uint32_t t,
                                              uint32_t x, uint32_t y, R v[9])
{
    constexpr bool pin = sizeof(R) == 4;     // float arithmetic (see philox10)
    const U4 a = philox10<pin>(x, y, t, 4u * kStreamNoise + 0u, seed, replica);
    const U4 b = philox10<pin>(x, y, t, 4u * kStreamNoise + 1u, seed, replica);
    uint32_t k[9];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        k[i] = a.v[i] >> 8;
        k[4 + i] = b.v[i] >> 8;
    }
    k[8] = ((a.v[0] & 0xFFu) << 16) | ((a.v[1] & 0xFFu) << 8) | (a.v[2] & 0xFFu);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int n = (int)(2u * k[i] + 1u) - (1 << 24);   // odd, |n| < 2^24: exact
        v[i] = (R)n * (R)(1.0 / 16777216.0);
    }
}

// ---------------------------------------------------------------------------
// Discrete cell divisions (Sec. II; Eq. 5).  Each eligible site draws its
// number of divisions from a Poisson law: a uniform U = (n + 1/2) 2^-52 from
// 52 random bits inverts the distribution function, whose terms use only
// basic IEEE arithmetic (so every implementation draws the same count), and
// two further random bits per division pick its axis.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void division_draws(uint32_t seed, uint32_t replica, uint32_t t,
                                               uint32_t x, uint32_t y, double &U, uint64_t &axes)
{
    const U4 a = philox10(x, y, t, 4u * kStreamDivision + 0u, seed, replica);
    const uint64_t n = ((uint64_t)(a.v[0] >> 6) << 26) | (uint64_t)(a.v[1] >> 6);
    U = ((double)n + 0.5) * (1.0 / 4503599627370496.0);
    axes = ((uint64_t)a.v[3] << 32) | (uint64_t)a.v[2];
}

// e^-lam, 0 <= lam <= 8: (e^-m)^16 with m = lam / 16 and e^-m from its
// Taylor series through m^17 by Horner's rule.
__device__ __forceinline__ double exp_neg(double lam)
{
    const double m = lam * 0.0625;
    double r = 1.0;
#pragma unroll
    for (int n = 17; n >= 1; --n) {
        const double q = m / (double)n;
        r = 1.0 - q * r;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) r = r * r;
    return r;
}

// Smallest k with U <= P(0) + ... + P(k) for the Poisson law of mean lam,
// capped at 32, given p0 = exp_neg(lam).
__device__ __forceinline__ int poisson_k_from(double U, double lam, double p0)
{
    double pk = p0;
    double cdf = pk;
    int k = 0;
    while (U > cdf && k < 32) {
        k = k + 1;
        pk = pk * lam / (double)k;
        cdf = cdf + pk;
    }
    return k;
}

__device__ __forceinline__ int poisson_k(double U, double lam)
{
    return poisson_k_from(U, lam, exp_neg(lam));
}

// poisson_k(U, lam) without the exponential when U is plainly below P(0):
// e^-lam > 1 - lam, and exp_neg's relative error (under 1e-14) is far inside
// the margin 2^-40, so U < (1 - lam)(1 - 2^-40) implies U < exp_neg(lam) and
// the count is 0.  At small means nearly every site takes this exit.
__device__ __forceinline__ int poisson_k_small(double U, double lam)
{
    if (U < (1.0 - lam) * (1.0 - 0x1p-40)) return 0;
    return poisson_k(U, lam);
}

// Expected divisions per unit weight: n_s = g m_tot / rho_cell divisions
// (Sec. II) shared by the eligible sites' total weight; m_tot and the weight
// are integers in units of 2^-24 (the uniform law weighs each site 1).
__host__ __device__ inline double division_lam(bool uniform, double g, double rho_cell,
                                               long long mfx, long long wsum)
{
    if (wsum <= 0) return 0.0;
    const double m_tot = (double)mfx * (1.0 / 16777216.0);
    const double ns = g * m_tot / rho_cell;
    const double wt = uniform ? (double)wsum : (double)wsum * (1.0 / 16777216.0);
    return ns / wt;
}

// Uniform (k + 1/2) 2^-24 of the initial density at (x, y).
__device__ __forceinline__ double init_uniform(uint32_t seed, uint32_t replica, uint32_t x,
                                               uint32_t y)
{
    const U4 a = philox10(x, y, 0u, 4u * kStreamInit + 0u, seed, replica);
    return ((double)(a.v[0] >> 8) + 0.5) * (1.0 / 16777216.0);
}

// ---------------------------------------------------------------------------
// Storage codecs.  FP64 / FP32 store f_i as is.  The 16-bit storages keep
// s_i = f_i - W_i with W_i = w_i rho_ref rounded to the storage type; an empty
// site stores -W_i exactly and decodes to exactly 0.
// ---------------------------------------------------------------------------
template <class S>
struct Codec;

template <>
struct Codec<double> {
    using R = double;
    __device__ __forceinline__ static R dec(double s, R) { return s; }
    __device__ __forceinline__ static double enc(R f, R) { return f; }
};

template <>
struct Codec<float> {
    using R = float;
    __device__ __forceinline__ static R dec(float s, R) { return s; }
    __device__ __forceinline__ static float enc(R f, R) { return f; }
};

// Stochastic rounding of a float32 offset o to a 16-bit storage, with r a
// 14-bit random number: the magnitude moves to the representable neighbour
// above it with probability equal to its distance from the one below, in
// units of the storage's ulp, so the stored value equals o on average.  The
// result is a float32 that the storage holds exactly.
//   BF16: 16 mantissa bits are dropped; 4 r is added to the magnitude's bits
//   before they are cut (probabilities exact to 2^-14).
//   FP16, |o| >= 2^-14: 13 bits are dropped; r / 2 is added (exact).
//   FP16, |o| < 2^-14 (subnormal, steps of 2^-24): floor(|o| 2^24 + r 2^-14).
__device__ __forceinline__ float sround_bf16(float o, uint32_t r)
{
    const uint32_t b = __float_as_uint(o);
    const uint32_t mag = ((b & 0x7FFFFFFFu) + ((r & 0x3FFFu) << 2)) & 0xFFFF0000u;
    return __uint_as_float((b & 0x80000000u) | mag);
}

__device__ __forceinline__ float sround_f16(float o, uint32_t r)
{
    const uint32_t b = __float_as_uint(o);
    uint32_t mag = b & 0x7FFFFFFFu;
    if (mag >= 0x38800000u) {
        mag = (mag + ((r & 0x3FFFu) >> 1)) & ~0x1FFFu;
    } else {
        const float m = __uint_as_float(mag) * 16777216.0f;                  // exact
        const float q = floorf(m + (float)(r & 0x3FFFu) * (1.0f / 16384.0f));  // integer < 2^10
        mag = __float_as_uint(q * (1.0f / 16777216.0f));                     // exact
    }
    return __uint_as_float((b & 0x80000000u) | mag);
}

// The fourteen-bit numbers of one site's stochastic rounding: two from each
// word of one Philox call (bits 0-13 and 14-27) and a ninth from the four
// words' top nibbles.
__device__ __forceinline__ void round_bits(uint32_t seed, uint32_t replica, uint32_t t,
                                           uint32_t x, uint32_t y, uint32_t r[9])
{
    const U4 a = philox10<true>(x, y, t, 4u * kStreamRound + 0u, seed, replica);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[2 * k] = a.v[k] & 0x3FFFu;
        r[2 * k + 1] = (a.v[k] >> 14) & 0x3FFFu;
    }
    r[8] = ((a.v[0] >> 28) | ((a.v[1] >> 28) << 4) | ((a.v[2] >> 28) << 8) |
            ((a.v[3] >> 28) << 12)) >> 2;
}

template <>
struct Codec<__half> {
    using R = float;
    __device__ __forceinline__ static R dec(__half s, R W) { return __half2float(s) + W; }
    __device__ __forceinline__ static __half enc(R f, R W) { return __float2half_rn(f - W); }
    __device__ __forceinline__ static __half enc_sr(R f, R W, uint32_t r)
    {
        return __float2half_rn(sround_f16(f - W, r));
    }
};

template <>
struct Codec<__hip_bfloat16> {
    using R = float;
    __device__ __forceinline__ static R dec(__hip_bfloat16 s, R W)
    {
        return __bfloat162float(s) + W;
    }
    __device__ __forceinline__ static __hip_bfloat16 enc(R f, R W)
    {
        return __float2bfloat16(f - W);
    }
    __device__ __forceinline__ static __hip_bfloat16 enc_sr(R f, R W, uint32_t r)
    {
        return __float2bfloat16(sround_bf16(f - W, r));
    }
};

}  // namespace lbm
