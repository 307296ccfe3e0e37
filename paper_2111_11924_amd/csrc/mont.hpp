// Montgomery arithmetic for gfx950 in a redundant 2^LB radix (LB = 28 or 27).
//
// The operation is Montgomery multiplication (paper, Sec. 3.2, Algorithm 3):
// t = a b R^-1 mod m with R = 2^(LB*NL), reached word by word (CIOS: one
// multiplier limb b_i per step, one reduction multiple m_i = t_0 n' mod 2^LB per
// step, then a one-limb shift).  Limbs hold LB bits in 32-bit registers and
// every column is accumulated in 64 bits, so a partial product is exactly one
// v_mad_u64_u32 and no carry is resolved inside the loop: with a, b, m, n
// limbs below 2^LB a column collects at most 2*NL products below 2^(2LB), which
// stays below 2^64 for the sizes instantiated here (checked by static_assert).
// Carries are propagated once, after the last step.
//
// Lazy reduction: with 4m < R and a, b < 2m (more generally a*b < R*m) the
// result is below 2m, so no conditional subtraction is needed between the
// multiplications of an exponentiation; the final value is brought into [0, m)
// once at the end (canonicalize).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmk {

template <int LB>
struct Radix {
    static constexpr uint32_t MASK = (1u << LB) - 1u;
};

// Number of LB-bit limbs for a modulus of `bits` bits: R = 2^(LB*NL) > 4m.
constexpr int limbs_for(int bits, int lb) { return (bits + 2 + lb - 1) / lb; }

// Number of 4-limb groups of an NL-limb number (multiplier staging unit).
constexpr int groups_of(int nl) { return (nl + 3) / 4; }

// r = a * b * R^-1 mod m, result in [0, 2m) as NL normalised LB-bit limbs.
// a: NL limbs in registers; b: staged in LDS as groups_of(NL) uint4 values,
// group g of this lane at bl[g * 64] (bl = base + lane), limb 4g+u in
// component u; n: modulus limbs; n0 = -m^-1 mod 2^LB.  r may alias a.
// Bounds: every limb below 2^LB and a*b < R*m.
template <int NL, int LB>
__device__ __forceinline__ void mont_mul(uint32_t (&r)[NL], const uint32_t (&a)[NL],
                                         const uint4 *bl, const uint32_t (&n)[NL], uint32_t n0) {
    static_assert(2.0 * NL * (double)(1ull << LB) * (double)(1ull << LB) < 18446744073709551615.0,
                  "column sums may overflow 64 bits");
    constexpr uint32_t MASK = Radix<LB>::MASK;
    // keep the surrounding step logic (loads of the next operand, table stores)
    // out of the product: mixing them in only lengthens live ranges
    __builtin_amdgcn_sched_barrier(0);
    uint64_t t[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) t[j] = 0;
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) {
        const uint4 bq = bl[g * 64];
        const uint32_t bg[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (4 * g + u >= NL) break;
            const uint32_t bi = bg[u];
#pragma unroll
            for (int j = 0; j < NL; ++j) t[j] += (uint64_t)a[j] * bi;
            const uint32_t m = ((uint32_t)t[0] * n0) & MASK;
#pragma unroll
            for (int j = 0; j < NL; ++j) t[j] += (uint64_t)m * n[j];
            // t[0] is now a multiple of 2^LB: divide the whole accumulator by 2^LB
            const uint64_t c = t[0] >> LB;
#pragma unroll
            for (int j = 0; j < NL - 1; ++j) t[j] = t[j + 1];
            t[NL - 1] = 0;
            t[0] += c;
        }
    }
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const uint64_t v = t[j] + c;
        r[j] = (uint32_t)v & MASK;
        c = v >> LB;
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Stage a register number as the multiplier of the next mont_mul.
template <int NL>
__device__ __forceinline__ void stage_regs(uint4 *bl, const uint32_t (&x)[NL]) {
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) {
        const uint32_t x0 = x[4 * g];
        const uint32_t x1 = 4 * g + 1 < NL ? x[4 * g + 1] : 0u;
        const uint32_t x2 = 4 * g + 2 < NL ? x[4 * g + 2] : 0u;
        const uint32_t x3 = 4 * g + 3 < NL ? x[4 * g + 3] : 0u;
        bl[g * 64] = make_uint4(x0, x1, x2, x3);
    }
}

// Stage groups_of(NL) uint4 values read from global memory at src[g * stride].
template <int NL>
__device__ __forceinline__ void stage_global(uint4 *bl, const uint4 *src, int stride) {
    uint4 v[groups_of(NL)];
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) v[g] = src[(size_t)g * stride];
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) bl[g * 64] = v[g];
}

// Stage the constant 1 (leaves Montgomery form: MM(x, 1) = x R^-1).
template <int NL>
__device__ __forceinline__ void stage_one(uint4 *bl) {
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) bl[g * 64] = make_uint4(g == 0 ? 1u : 0u, 0u, 0u, 0u);
}

// x < 2m  ->  x mod m (canonical).  Subtract m, keep the difference when no
// borrow comes out of the top limb.
template <int NL, int LB>
__device__ __forceinline__ void canonicalize(uint32_t (&x)[NL], const uint32_t (&n)[NL]) {
    constexpr uint32_t MASK = Radix<LB>::MASK;
    uint32_t d[NL];
    int32_t borrow = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int32_t v = (int32_t)x[j] - (int32_t)n[j] - borrow;
        d[j] = (uint32_t)v & MASK;
        borrow = v < 0 ? 1 : 0;
    }
    const bool keep = borrow == 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) x[j] = keep ? d[j] : x[j];
}

// Limb j of an LB-bit-radix number read out of little-endian 32-bit words w[0..S)
// (bits [LB*j, LB*j+LB)); words past S read as zero.
template <int S, int LB>
__device__ __forceinline__ uint32_t radix_limb(const uint32_t (&w)[S], int j) {
    const int bit = LB * j;
    const int k = bit >> 5, sh = bit & 31;
    const uint32_t lo = k < S ? w[k] : 0u;
    const uint32_t hi = (k + 1) < S ? w[k + 1] : 0u;
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return (uint32_t)(v >> sh) & Radix<LB>::MASK;
}

// Word k (32 bits) of a number given as NL limbs of LB bits.
template <int NL, int LB>
__device__ __forceinline__ uint32_t radix_word(const uint32_t (&x)[NL], int k) {
    const int bit = 32 * k;
    const int j = bit / LB, sh = bit % LB;
    // at most three limbs contribute to one 32-bit word when LB >= 16; only the
    // low 32 bits of the 64-bit sum are kept, so bits shifted past 64 do not matter
    const uint64_t l0 = j < NL ? x[j] : 0u;
    const uint64_t l1 = (j + 1) < NL ? x[j + 1] : 0u;
    const uint64_t l2 = (j + 2) < NL ? x[j + 2] : 0u;
    const uint64_t v = (l0 >> sh) | (l1 << (LB - sh)) | (l2 << (2 * LB - sh));
    return (uint32_t)v;
}

}  // namespace pmk
