// Montgomery arithmetic for gfx950 in a redundant 2^LB radix (LB = 28 or 27).
//
// The operation is Montgomery multiplication (paper, Sec. 3.2, Algorithm 3):
// t = a b R^-1 mod m with R = 2^(LB*NL), reached word by word with one
// reduction digit m_k = t_k n' mod 2^LB per word.  Limbs hold LB bits in 32-bit
// registers and every column is accumulated in 64 bits, so a partial product is
// exactly one v_mad_u64_u32 and no carry flag is ever handled: a column collects
// at most 2*NL products below 2^(2LB) plus a carry, which stays below 2^64 for
// the sizes instantiated here (checked by static_assert).
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

// Column alignment (a source that defines PMK_COLUMN_ALIGN to 1 before the
// includes): each column of mont_mul / mont_sqr starts at an 8-byte boundary
// (the assembler pads with s_nop), which keeps more of the 8-byte
// v_mad_u64_u32 at addresses 0 modulo 8, where the unrolled products run
// faster, in kernels whose code around the products would otherwise leave them
// at 4 modulo 8.
#ifndef PMK_COLUMN_ALIGN
#define PMK_COLUMN_ALIGN 0
#endif
__device__ __forceinline__ void column_align() {
    if constexpr (PMK_COLUMN_ALIGN) asm volatile(".p2align 3");
}

// Product-scanning Montgomery multiplication (the "finely integrated product
// scanning" order of Koc, Acar and Kaliski): column k of the double-length
// result collects every a_i b_j and m_i n_j with i + j = k in one 64-bit
// accumulator (one v_mad_u64_u32 each); for the low NL columns the reduction
// digit m_k = acc n0 mod 2^LB is chosen so the column becomes a multiple of
// 2^LB; only the carry acc >> LB moves on.  The high NL columns are the result.
//
// r = a * b * R^-1 mod m in [0, 2m) as NL normalised LB-bit limbs, for limbs of
// a, b, n below 2^LB, n0 = -m^-1 mod 2^LB and a*b < R*m.  r may alias a or b:
// limb k-NL of r is written at column k, after the last column that reads
// limb k-NL of a or b.
template <int NL, int LB>
__device__ __forceinline__ void mont_mul(uint32_t (&r)[NL], const uint32_t (&a)[NL],
                                         const uint32_t (&b)[NL], const uint32_t (&n)[NL],
                                         uint32_t n0) {
    static_assert((2.0 * NL + 1) * (double)(1ull << LB) * (double)(1ull << LB) < 18446744073709551615.0,
                  "column sums may overflow 64 bits");
    constexpr uint32_t MASK = Radix<LB>::MASK;
    uint32_t m[NL];
    uint64_t carry = 0;
    __builtin_amdgcn_sched_barrier(0);
    column_align();
#pragma unroll
    for (int k = 0; k < 2 * NL - 1; ++k) {
        const int lo = k - NL + 1 > 0 ? k - NL + 1 : 0;
        // two interleaved accumulators halve the length of the dependent chain
        uint64_t acc0 = carry, acc1 = 0;
        int t = 0;
#pragma unroll
        for (int i = lo; i <= (k < NL ? k : NL - 1); ++i, ++t) {
            if (t & 1)
                acc1 += (uint64_t)a[i] * b[k - i];
            else
                acc0 += (uint64_t)a[i] * b[k - i];
        }
#pragma unroll
        for (int i = lo; i < (k < NL ? k : NL); ++i, ++t) {
            if (t & 1)
                acc1 += (uint64_t)m[i] * n[k - i];
            else
                acc0 += (uint64_t)m[i] * n[k - i];
        }
        uint64_t acc = acc0 + acc1;
        if (k < NL) {
            m[k] = ((uint32_t)acc * n0) & MASK;
            acc += (uint64_t)m[k] * n[0];  // now a multiple of 2^LB
        } else {
            r[k - NL] = (uint32_t)acc & MASK;
        }
        carry = acc >> LB;
        // keep the schedule column by column: interleaving columns only adds
        // live accumulators and pushes the register count past 3 waves per SIMD
        __builtin_amdgcn_sched_barrier(0);
        column_align();
    }
    r[NL - 1] = (uint32_t)carry;
}

// Montgomery squaring r = a^2 R^-1 mod m, same order and bounds as mont_mul,
// with each cross product a_i a_j (i < j) formed once and doubled: about
// NL^2/2 fewer multiply-adds than mont_mul(a, a).
template <int NL, int LB>
__device__ __forceinline__ void mont_sqr(uint32_t (&r)[NL], const uint32_t (&a)[NL],
                                         const uint32_t (&n)[NL], uint32_t n0) {
    constexpr uint32_t MASK = Radix<LB>::MASK;
    uint32_t m[NL];
    uint64_t carry = 0;
    __builtin_amdgcn_sched_barrier(0);
    column_align();
#pragma unroll
    for (int k = 0; k < 2 * NL - 1; ++k) {
        const int lo = k - NL + 1 > 0 ? k - NL + 1 : 0;
        uint64_t x0 = 0, x1 = 0;
        int t = 0;
#pragma unroll
        for (int i = lo; i < k - i; ++i, ++t) {
            if (t & 1)
                x1 += (uint64_t)a[i] * a[k - i];
            else
                x0 += (uint64_t)a[i] * a[k - i];
        }
        uint64_t y0 = ((x0 + x1) << 1) + carry, y1 = 0;
        if ((k & 1) == 0) y1 += (uint64_t)a[k / 2] * a[k / 2];
        t = 0;
#pragma unroll
        for (int i = lo; i < (k < NL ? k : NL); ++i, ++t) {
            if (t & 1)
                y1 += (uint64_t)m[i] * n[k - i];
            else
                y0 += (uint64_t)m[i] * n[k - i];
        }
        uint64_t acc = y0 + y1;
        if (k < NL) {
            m[k] = ((uint32_t)acc * n0) & MASK;
            acc += (uint64_t)m[k] * n[0];
        } else {
            r[k - NL] = (uint32_t)acc & MASK;
        }
        carry = acc >> LB;
        __builtin_amdgcn_sched_barrier(0);
        column_align();
    }
    r[NL - 1] = (uint32_t)carry;
}

// Load an NL-limb number stored as groups_of(NL) uint4 values at src[g * stride].
template <int NL>
__device__ __forceinline__ void load_groups(uint32_t (&x)[NL], const uint4 *src, int stride) {
#pragma unroll
    for (int g = 0; g < groups_of(NL); ++g) {
        const uint4 v = src[(size_t)g * stride];
        const uint32_t c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (4 * g + u < NL) x[4 * g + u] = c[u];
    }
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

// The same, reading word k from src[k * stride] (memory instead of registers).
template <int S, int LB>
__device__ __forceinline__ uint32_t radix_limb_mem(const uint32_t *src, size_t stride, int j) {
    const int bit = LB * j;
    const int k = bit >> 5, sh = bit & 31;
    const uint32_t lo = k < S ? src[(size_t)k * stride] : 0u;
    const uint32_t hi = (k + 1) < S ? src[(size_t)(k + 1) * stride] : 0u;
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return (uint32_t)(v >> sh) & Radix<LB>::MASK;
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
