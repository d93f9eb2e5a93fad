// mtpt_rng.h -- device-side random-walk normals for the MTPT step (gfx950).
//
// The paper asks only for standard-normal jumps (Sec. 3, random-walk update).
// This library draws them counter-based, so that a particle's jump at a step
// depends only on (seed, step, pid) and never on launch order:
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
//     key     = (seed & 0xffffffff, seed >> 32)
//     counter = (pid, call, step & 0xffffffff, step >> 32)
//   u1 = (2 k1 + 1) 2^-53 with k1 = word1 << 20 | word0 >> 12, u2 likewise from
//   words 3 and 2; Box-Muller z0 = r cos(2 pi u2), z1 = r sin(2 pi u2),
//   r = sqrt(-2 ln u1).  Call 0 gives dimensions 0 and 1, call 1 dimension 2.
// ln, sin and cos are evaluated from their series by Horner with a fixed
// operation order: each multiply-add an IEEE fused multiply-add, nothing
// else contracted; FP64 division and square root are IEEE correctly rounded.
// So the jumps are reproducible bit for bit by any implementation of the
// same recipe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtpt {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r != 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32->64 product gives both halves
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
        c = make_uint4(static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
                       static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0));
    }
    return c;
}

__device__ __forceinline__ double unit_open(uint32_t low, uint32_t high)
{
    const uint64_t k = (static_cast<uint64_t>(high) << 20) | (low >> 12);
    return static_cast<double>(2ull * k + 1ull) * 0x1p-53;
}

// reciprocals of the odd numbers 3..23 and of the factorials 2!..19!,
// folded at compile time (each factorial exact in FP64, one IEEE division)
constexpr double inv_u(int v) { return 1.0 / static_cast<double>(v); }
constexpr double inv_fact(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k)
        f = f * static_cast<double>(k);
    return 1.0 / f;
}

// fma(a, b, c) = a b + c rounded once (IEEE), with the constant addend c
// taken from scalar registers.  Left to itself the compiler turns a fused
// multiply-add with a constant addend into two vector moves of the constant
// and a v_fmac; v_fma_f64 reads the scalar pair directly.  c must be the
// same in every lane (here always a compile-time constant): a scalar operand
// holds one value per wave.  Arithmetic only: the instruction's inputs are
// read before its result is written.
__device__ __forceinline__ double fma_sc(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// ln(u), u in (0,1): u = m 2^e, m folded into [sqrt(1/2), sqrt(2)];
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), series through s^23 by Horner.
// Each multiply-add is one IEEE fused multiply-add; nothing else is fused.
__device__ __forceinline__ double ln_unit(double u)
{
#pragma clang fp contract(off)
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(u));
    int e = static_cast<int>((b >> 52) & 0x7ffu) - 1023;
    double m = __longlong_as_double(static_cast<long long>((b & 0x000fffffffffffffull) |
                                                           0x3ff0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double t = inv_u(23);
#pragma unroll
    for (int k = 10; k >= 1; --k)
        t = fma_sc(z, t, inv_u(2 * k + 1));
    const double s2 = s + s;
    const double lm = __builtin_fma(s2, z * t, s2);
    const double ed = static_cast<double>(e);
    const double r = __builtin_fma(ed, 5.497923018708371e-14, lm);   // ln 2 minus its 42-bit head
    return __builtin_fma(ed, 0.6931471805598903, r);                // 42-bit head of ln 2
}

// sin and cos of 2 pi u, u in (0,1): quadrant from 4u, in-quadrant angle
// folded to [0, pi/4], Taylor series through y^19 / y^18 in z = y^2 by
// Horner with fused multiply-adds (coefficients +-1/n!).
__device__ __forceinline__ void sincos_2pi_unit(double u, double* sn, double* cs)
{
#pragma clang fp contract(off)
    const double v = 4.0 * u;
    const int q = static_cast<int>(v);
    const double f = v - static_cast<double>(q);
    const bool fold = f > 0.5;
    const double y = (fold ? (1.0 - f) : f) * 1.5707963267948966;
    const double z = y * y;
    double ts = -inv_fact(19), tc = -inv_fact(18);
#pragma unroll
    for (int k = 8; k >= 1; --k) {
        const double sg = (k & 1) ? -1.0 : 1.0;
        ts = fma_sc(z, ts, sg * inv_fact(2 * k + 1));
        tc = fma_sc(z, tc, sg * inv_fact(2 * k));
    }
    ts = __builtin_fma(z, ts, 1.0);
    tc = __builtin_fma(z, tc, 1.0);
    const double sy = y * ts;
    const double cy = tc;
    const double sp = fold ? cy : sy;
    const double cp = fold ? sy : cy;
    switch (q & 3) {
    case 0: *sn = sp;  *cs = cp;  break;
    case 1: *sn = cp;  *cs = -sp; break;
    case 2: *sn = -sp; *cs = -cp; break;
    default: *sn = -cp; *cs = sp; break;
    }
}

__device__ __forceinline__ void normal_pair(uint64_t seed, int64_t step, uint32_t pid,
                                            uint32_t call, double* z0, double* z1)
{
#pragma clang fp contract(off)
    const uint64_t st = static_cast<uint64_t>(step);
    const uint4 w = philox4x32_10(make_uint4(pid, call, static_cast<uint32_t>(st),
                                             static_cast<uint32_t>(st >> 32)),
                                  static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double u1 = unit_open(w.x, w.y);
    const double u2 = unit_open(w.z, w.w);
    const double r = __builtin_sqrt(-2.0 * ln_unit(u1));
    double sn, cs;
    sincos_2pi_unit(u2, &sn, &cs);
    *z0 = r * cs;
    *z1 = r * sn;
}

}  // namespace mtpt
