// Montgomery multiplication with one bignum spread over a group of L adjacent
// lanes (L = 2, 4 or 8), for the numbers whose limbs do not fit one lane's
// registers (full-size 3072- to 8192-bit moduli, 3072/4096-bit CRT halves).
//
// Same arithmetic as mont.hpp (Sec. 3.2, Algorithm 3; LB-bit limbs, 64-bit
// column accumulators, no carry handling inside the loop), in operand-scanning
// order (CIOS): lane `pos` of a group owns limbs [pos K, pos K + K) of a, n and
// of the running accumulator t.  Step i adds a b_i (b_i read from LDS, one
// address per group: a broadcast), forms the reduction digit m_i from the
// group's lowest accumulator limb (broadcast from lane 0 by DPP: a quad
// permutation, plus a row shift for groups of 8), adds m_i n, and divides t by
// 2^LB: every lane hands its lowest limb to the lane below (DPP), lane 0 folds
// the carry of its lowest limb into the next one.  Carries between lanes are settled once, after the last step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mont.hpp"

namespace pmk {

// LDS words through pointers of the LDS address space.  The kernels hand an
// opaque copy (empty asm) of a pointer to their loops so that addresses are
// formed at each use; made from a generic pointer, that copy no longer tells
// the compiler that it points into LDS, and its accesses would become flat
// memory operations (a global-memory wait per access).
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ lds_u32 *as_lds(uint32_t *p) { return (lds_u32 *)p; }
__device__ __forceinline__ const lds_u32 *as_lds(const uint32_t *p) { return (const lds_u32 *)p; }
template <typename T>
__device__ __forceinline__ T *opaque_lds(T *p) {
    asm volatile("" : "+v"(p));
    return p;
}
// Flat = true keeps the generic form (flat accesses) instead: measured faster
// for the 8192-bit CRT halves only (150.8 against 172.4 ms for 100 KB, while
// every other lane-group kernel ran as fast or faster with LDS pointers; A/B
// on one box)
template <bool Flat>
using lds_word = typename std::conditional<Flat, uint32_t, lds_u32>::type;
template <bool Flat>
__device__ __forceinline__ lds_word<Flat> *lds_k(uint32_t *p) { return (lds_word<Flat> *)p; }
template <bool Flat>
__device__ __forceinline__ const lds_word<Flat> *lds_k(const uint32_t *p) { return (const lds_word<Flat> *)p; }

// quad_perm DPP selectors (four 2-bit lane indices inside each quad)
constexpr int qperm(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }

template <int Ctrl>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, 0xF, 0xF, false);
}

// DPP row shifts (within 16-lane rows): lane i receives lane i + n (shl) or
// lane i - n (shr); lanes whose source lies outside the row receive 0.
template <int N>
__device__ __forceinline__ uint32_t row_shl(uint32_t v) { return dpp<0x100 + N>(v); }
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t v) { return dpp<0x110 + N>(v); }

// Groups of L = 2, 4 or 8 adjacent lanes (aligned, so a group never crosses a
// 16-lane row).  pos = lane % L.
// value held by lane 0 of the group
template <int L>
__device__ __forceinline__ uint32_t grp_first(uint32_t v, int pos) {
    static_assert(L == 2 || L == 4 || L == 8, "groups of 2, 4 or 8 lanes");
    if constexpr (L == 2) return dpp<qperm(0, 0, 2, 2)>(v);
    if constexpr (L == 4) return dpp<qperm(0, 0, 0, 0)>(v);
    const uint32_t q = dpp<qperm(0, 0, 0, 0)>(v);  // lane 0 of each quad
    const uint32_t u = row_shr<4>(q);              // upper quad: the lower quad's lane 0
    return pos < 4 ? q : u;
}
// value held by the group's last lane
template <int L>
__device__ __forceinline__ uint32_t grp_last(uint32_t v, int pos) {
    if constexpr (L == 2) return dpp<qperm(1, 1, 3, 3)>(v);
    if constexpr (L == 4) return dpp<qperm(3, 3, 3, 3)>(v);
    const uint32_t q = dpp<qperm(3, 3, 3, 3)>(v);  // lane 3 of each quad
    const uint32_t l = row_shl<4>(q);              // lower quad: the upper quad's lane 3
    return pos < 4 ? l : q;
}
// value of the next lane of the group (the last lane gets 0)
template <int L>
__device__ __forceinline__ uint32_t grp_next(uint32_t v, int pos) {
    uint32_t x;
    if constexpr (L == 2) x = dpp<qperm(1, 1, 3, 3)>(v);
    else if constexpr (L == 4) x = dpp<qperm(1, 2, 3, 3)>(v);
    else x = row_shl<1>(v);
    return pos == L - 1 ? 0u : x;
}
// value of the previous lane of the group (lane 0 gets 0)
template <int L>
__device__ __forceinline__ uint32_t grp_prev(uint32_t v, int pos) {
    uint32_t x;
    if constexpr (L == 2) x = dpp<qperm(0, 0, 2, 2)>(v);
    else if constexpr (L == 4) x = dpp<qperm(0, 0, 1, 2)>(v);
    else x = row_shr<1>(v);
    return pos == 0 ? 0u : x;
}
template <int L>
__device__ __forceinline__ uint64_t grp_next64(uint64_t v, int pos) {
    return ((uint64_t)grp_next<L>((uint32_t)(v >> 32), pos) << 32) | grp_next<L>((uint32_t)v, pos);
}
template <int L>
__device__ __forceinline__ uint64_t grp_prev64(uint64_t v, int pos) {
    return ((uint64_t)grp_prev<L>((uint32_t)(v >> 32), pos) << 32) | grp_prev<L>((uint32_t)v, pos);
}

// r = a b R^-1 mod m (R = 2^(LB NLT)), result below 2m, normalised.  K = NLT/L
// limbs per lane; b_i at bl[i * bstride] in LDS; r may alias a.
template <int NLT, int LB, int L, bool Flat = false>
__device__ __forceinline__ void mont_mul_lanes(uint32_t (&r)[NLT / L], const uint32_t (&a)[NLT / L],
                                               const uint32_t *bl, int bstride,
                                               const uint32_t (&n)[NLT / L], uint32_t n0, int pos) {
    constexpr int K = NLT / L;
    static_assert(K * L == NLT, "limbs must split evenly over the lanes");
    static_assert((2.0 * NLT + 1) * (double)(1ull << LB) * (double)(1ull << LB) < 18446744073709551615.0,
                  "column sums may overflow 64 bits");
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const lds_word<Flat> *b3 = opaque_lds(lds_k<Flat>(bl));  // b_i addresses: base + immediate at each use
    uint64_t t[K];
#pragma unroll
    for (int j = 0; j < K; ++j) t[j] = 0;
    // with few limbs per lane a step is short and its read of b_i would stall
    // it: b_(i+1) is read one step ahead; with many (K > 20) the step hides
    // the read and the extra register only adds pressure
    constexpr bool kAhead = K <= 20;
    uint32_t bn = kAhead ? (uint32_t)b3[0] : 0u;
    __builtin_amdgcn_sched_barrier(0);
    // NLT = L K steps, as L blocks of K unrolled steps: t shifts by one limb
    // per step, so after K steps its registers are back in place and the
    // block's code serves every block (code size K steps, not NLT)
#pragma unroll 1
    for (int blk = 0; blk < L; ++blk) {
        const lds_word<Flat> *bb = b3 + blk * K * bstride;
#pragma unroll
        for (int ii = 0; ii < K; ++ii) {
            uint32_t bi;
            if constexpr (kAhead) {
                bi = bn;
                // the next step's limb, read while this step runs (the steps
                // are kept apart by scheduling barriers); after the last step
                // limb 0 again, unused
                bn = bb[ii + 1 < K ? (ii + 1) * bstride : (blk + 1 < L ? K * bstride : -blk * K * bstride)];
            } else {
                bi = bb[ii * bstride];
            }
#pragma unroll
            for (int j = 0; j < K; ++j) t[j] += (uint64_t)a[j] * bi;
            const uint32_t m = (grp_first<L>((uint32_t)t[0], pos) * n0) & MASK;
#pragma unroll
            for (int j = 0; j < K; ++j) t[j] += (uint64_t)m * n[j];
            // lane 0's lowest column is now a multiple of 2^LB: its carry moves up;
            // every other lane's lowest column moves down to the lane below
            const uint64_t c = pos == 0 ? t[0] >> LB : 0;
            const uint64_t in = grp_next64<L>(t[0], pos);
#pragma unroll
            for (int j = 0; j < K - 1; ++j) t[j] = t[j + 1];
            t[K - 1] = in;
            t[0] += c;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // settle carries: within each lane, then L-1 rounds across lane boundaries
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t v = t[j] + c;
        r[j] = (uint32_t)v & MASK;
        c = v >> LB;
    }
#pragma unroll
    for (int s = 1; s < L; ++s) {
        uint64_t cin = grp_prev64<L>(c, pos);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t v = (uint64_t)r[j] + cin;
            r[j] = (uint32_t)v & MASK;
            cin = v >> LB;
        }
        c = cin;
    }
}

// x < 2m -> x mod m for a lane-distributed number: the borrow of x - m crosses
// the lanes in L rounds; the group keeps x - m when the top lane ends without
// a borrow.
template <int K, int LB, int L>
__device__ __forceinline__ void canonicalize_lanes(uint32_t (&x)[K], const uint32_t (&n)[K], int pos) {
    constexpr uint32_t MASK = Radix<LB>::MASK;
    uint32_t d[K];
    uint32_t bin = 0, bout = 0;
#pragma unroll
    for (int s = 0; s < L; ++s) {
        int32_t borrow = (int32_t)bin;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int32_t v = (int32_t)x[j] - (int32_t)n[j] - borrow;
            d[j] = (uint32_t)v & MASK;
            borrow = v < 0 ? 1 : 0;
        }
        bout = (uint32_t)borrow;
        bin = grp_prev<L>(bout, pos);
    }
    const bool keep = grp_last<L>(bout, pos) == 0;
#pragma unroll
    for (int j = 0; j < K; ++j) x[j] = keep ? d[j] : x[j];
}

}  // namespace pmk
