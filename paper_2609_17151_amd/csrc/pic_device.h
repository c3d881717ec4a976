// Device helpers of the MI355X PIC-MCC library: counter-based random numbers,
// Box-Muller, scattering rotation, wave/block scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten multiply-xor rounds
// on a 128-bit counter under a 64-bit key bumped by the Weyl constants.
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64 product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// odd 24-bit integer 2*(x>>9)+1: the uniform below is this times 2^-24
__device__ __forceinline__ uint32_t odd24(uint32_t x) { return ((x >> 9) << 1) | 1u; }

// uniform in (0,1) with 23 random bits (exact in binary32 and binary64)
__device__ __forceinline__ double u01d(uint32_t x) { return (double)odd24(x) * 0x1p-24; }

// Box-Muller pair from two uniforms; the angle 2 pi ub as sincospi(2 ub),
// whose argument 2 ub is exact (no argument reduction)
__device__ __forceinline__ void box_muller_d(double ua, double ub, double& g0, double& g1)
{
    const double r = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    g0 = r * c;
    g1 = r * s;
}

// Direction after scattering by (chi, phi = 2 pi u_phi) about the unit
// direction d (Vahedi & Surendra form with the x axis as reference; the y
// axis when d is within 1e-6 of x), in FP64: only the few particles that
// collide in a step take this path, so its cost is small, and the new
// velocity is rounded to binary32 once, at the end.
__device__ __forceinline__ void scatter_dir_d(double dx, double dy, double dz, double cos_chi, double u_phi,
                                              double& ox, double& oy, double& oz)
{
    const double sin_chi = sqrt(fmax(0.0, 1.0 - cos_chi * cos_chi));
    double sp, cp;
    sincospi(2.0 * u_phi, &sp, &cp);
    double a = dx, b = dy, c = dz;
    double st = sqrt(fmax(0.0, 1.0 - a * a));
    const bool alt = !(st > 1e-6);
    if (alt) {
        a = dy;
        b = dz;
        c = dx;
        st = sqrt(fmax(0.0, 1.0 - a * a));
    }
    const double A = sin_chi / st;
    const double na = a * cos_chi + sin_chi * cp * st;
    const double nb = b * cos_chi + A * (sp * c - cp * a * b);
    const double nc = c * cos_chi - A * (sp * b + cp * a * c);
    ox = alt ? nc : na;
    oy = alt ? na : nb;
    oz = alt ? nb : nc;
}

// inclusive scan of one 32-bit value over a 64-wide wave
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ float wave_sum_f32(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

}  // namespace pic
