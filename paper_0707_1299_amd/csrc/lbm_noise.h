// Thermal noise of the fluctuating step and of the Brownian colloid update.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds that multiply counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57,
// mix the high halves of the products with the other counter words and the
// key, and advance the key by 0x9E3779B9, 0xBB67AE85 between rounds.
// Normals: Box-Muller on pairs of 32-bit outputs, u = (x + 1/2) 2^-32,
// z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1)
// (FP64 with the library functions, FP32 with the hardware instructions).
//
// Modes: the fifteen non-conserved D3Q19 polynomials of the orthogonal basis
// of Duenweg, Schiller and Ladd (2007), mutually w-orthogonal and orthogonal
// to 1 and c: bulk, five shear, nine ghosts (see emode).
#pragma once

#include "lbm_device.h"

namespace lbm {

struct Philox4 {
    uint32_t v[4];
};

// Three-way XOR in one VALU instruction (v_bitop3_b32 with truth table 0x96: the
// output bit is set where an odd number of the three input bits are).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Both callers pass a per-lane word 0 and wave-uniform words 1..3, so in the first
// round the new word 0 is wave-uniform: it stays a plain XOR, which the compiler
// keeps on the scalar unit; every other XOR of three words is one v_bitop3.
__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one multiply (v_mad_u64_u32) giving both halves
        const uint64_t p0 = uint64_t(c0) * 0xD2511F53u, p1 = uint64_t(c2) * 0xCD9E8D57u;
        const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
        const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
        c0 = r == 0 ? hi1 ^ c1 ^ k0 : xor3(hi1, c1, k0);
        c1 = lo1;
        c2 = xor3(hi0, c3, k1);
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

template <class T> __device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, T& z0, T& z1)
{
    constexpr T two_m32 = T(2.3283064365386962890625e-10);   // 2^-32
    const T u0 = (T(a) + T(0.5)) * two_m32, u1 = (T(b) + T(0.5)) * two_m32;
    const T r = sqrt(T(-2) * log(u0));
    const T t = T(2.0 * 3.14159265358979323846) * u1;
    z0 = r * cos(t);
    z1 = r * sin(t);
}

// FP32: the hardware transcendentals fit Box-Muller directly: v_log_f32 is log2 and
// v_sin_f32 / v_cos_f32 take their argument in revolutions, i.e. sin(2 pi u) = v_sin(u)
// for u in (0, 1), with no range reduction.
template <> __device__ __forceinline__ void box_muller<float>(uint32_t a, uint32_t b, float& z0, float& z1)
{
    constexpr float two_m32 = 2.3283064365386962890625e-10f;
    const float u0 = (float(a) + 0.5f) * two_m32, u1 = (float(b) + 0.5f) * two_m32;
    const float r = __builtin_amdgcn_sqrtf(-2.0f * 0.69314718055994530942f * __builtin_amdgcn_logf(u0));
    z0 = r * __builtin_amdgcn_cosf(u1);
    z1 = r * __builtin_amdgcn_sinf(u1);
}

// Square root of a noise amplitude: the library's in FP64; in FP32 the hardware
// instruction (1 ulp), where the library's correctly rounded form costs about ten
// more instructions.
__device__ __forceinline__ double noise_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float noise_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// The fifteen mode polynomials at velocity i (integers on D3Q19).
__host__ __device__ constexpr int emode(int k, int i)
{
    const int x = cvel(i, 0), y = cvel(i, 1), z = cvel(i, 2);
    const int c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return c2 - 1;                          // bulk
    case 1: return 3 * x * x - c2;                  // shear
    case 2: return y * y - z * z;
    case 3: return x * y;
    case 4: return x * z;
    case 5: return y * z;
    case 6: return (3 * c2 - 5) * x;                // ghosts
    case 7: return (3 * c2 - 5) * y;
    case 8: return (3 * c2 - 5) * z;
    case 9: return (y * y - z * z) * x;
    case 10: return (z * z - x * x) * y;
    case 11: return (x * x - y * y) * z;
    case 12: return 3 * c2 * c2 - 6 * c2 + 1;
    case 13: return (2 * c2 - 3) * (3 * x * x - c2);
    default: return (2 * c2 - 3) * (y * y - z * z);
    }
}

// Parity under c -> -c: bulk, shear (0..5) and the ghosts 12..14 are even, the
// ghosts 6..11 odd; velocities 2j+1 and 2j+2 are opposite, so e_k at the second
// of a pair is +-e_k at the first.
__host__ __device__ constexpr bool mode_even(int k) { return k < 6 || k >= 12; }

constexpr bool modes_have_parity()
{
    for (int k = 0; k < 15; ++k)
        for (int i = 1; i < NQ; i += 2)
            if (emode(k, i + 1) != (mode_even(k) ? emode(k, i) : -emode(k, i))) return false;
    for (int k = 0; k < 15; ++k)
        if (!mode_even(k) && emode(k, 0) != 0) return false;
    return true;
}
static_assert(modes_have_parity(), "mode parity table");

// The bulk and shear modes are quadratic in c: sum_{k<6} e_k(c) a_k equals
// -a0 + c_x^2 (a0 + 2 a1) + c_y^2 (a0 - a1 + a2) + c_z^2 (a0 - a1 - a2)
//   + c_x c_y a3 + c_x c_z a4 + c_y c_z a5,
// so their noise adds to the rest term and the second-moment pieces of the
// post-collision bracket.  Checked on every velocity for unit amplitudes.
constexpr bool stress_modes_fold()
{
    for (int k = 0; k < 6; ++k)
        for (int i = 0; i < NQ; ++i) {
            const int a[6] = {k == 0, k == 1, k == 2, k == 3, k == 4, k == 5};
            const int x = cvel(i, 0), y = cvel(i, 1), z = cvel(i, 2);
            const int folded = -a[0] + x * x * (a[0] + 2 * a[1]) + y * y * (a[0] - a[1] + a[2]) +
                               z * z * (a[0] - a[1] - a[2]) + x * y * a[3] + x * z * a[4] + y * z * a[5];
            if (folded != emode(k, i)) return false;
        }
    return true;
}
static_assert(stress_modes_fold(), "stress-mode noise folded into the bracket pieces");

// b_k = sum_i w_i e_k(c_i)^2
__host__ __device__ constexpr double mode_norm(int k)
{
    double b = 0.0;
    for (int i = 0; i < NQ; ++i) b += wgt(i) * double(emode(k, i) * emode(k, i));
    return b;
}

// Counter words of the node noise: call j of step t for node n of box b.
__device__ __forceinline__ Philox4 node_draw(uint32_t n, uint32_t b, unsigned long long t, uint32_t j, uint32_t k0,
                                             uint32_t k1)
{
    return philox4x32_10(n, b, uint32_t(t), ((uint32_t(t >> 32) & 0x0FFFFFFFu) << 4) | j, k0, k1);
}

// ... and of the particle noise of point p (stream word 2^32 - 1, never a box index).
__device__ __forceinline__ Philox4 particle_draw(uint32_t p, unsigned long long t, uint32_t k0, uint32_t k1)
{
    return philox4x32_10(p, 0xFFFFFFFFu, uint32_t(t), (uint32_t(t >> 32) & 0x0FFFFFFFu) << 4, k0, k1);
}

}  // namespace lbm
