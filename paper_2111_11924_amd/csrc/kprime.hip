// Batched primality testing for key generation: the primes p, q of every key
// pair of Algorithm 1's initialisation (Sec. 1.1 step 1; Sec. 3.1).  One lane
// per candidate, the candidate's modulus held per lane (candidates differ, so
// unlike the encryption and CRT kernels nothing is wave-uniform):
//   sieve_kernel         trial division by the odd primes below 4096;
//   miller_rabin_kernel  Miller-Rabin with caller-drawn bases: for each base a,
//                        with m - 1 = 2^s d (d odd), a^d = 1 or a^(2^j d) = -1
//                        for some j < s, else m is composite.
// The exponentiation is the fixed-window Montgomery one of the CRT kernels
// (window table per wavefront, digits per lane), in the radix of the key
// class's CRT halves.
#include "kernels_impl.hpp"

namespace pmk {

constexpr int kSievePrimes = 563;  // odd primes 3 .. 4093

__constant__ uint16_t c_small_primes[kSievePrimes];

namespace {

bool primes_ready[16] = {};

// odd primes below 4096 (host side, by a sieve of Eratosthenes)
int small_primes(uint16_t *out) {
    bool comp[4096] = {};
    int n = 0;
    for (int i = 3; i < 4096; i += 2) {
        if (comp[i]) continue;
        out[n++] = (uint16_t)i;
        for (int j = i * i; j < 4096; j += 2 * i) comp[j] = true;
    }
    return n;
}

}  // namespace

// flags[i] = 1 if no odd prime below 4096 divides candidate i (SH words)
template <int SH>
__global__ __launch_bounds__(256) void sieve_kernel(const uint32_t *__restrict__ cand, uint32_t count,
                                                    uint32_t *__restrict__ flags) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t *m = cand + (size_t)i * SH;
    uint32_t w[SH];
#pragma unroll
    for (int k = 0; k < SH; ++k) w[k] = m[k];
    uint32_t ok = 1;
    for (int t = 0; t < kSievePrimes && ok; ++t) {
        const uint32_t p = c_small_primes[t];
        const uint32_t r32 = (uint32_t)((1ull << 32) % p);  // 2^32 mod p
        uint32_t r = 0;
#pragma unroll
        for (int k = SH - 1; k >= 0; --k) r = (r * r32 + w[k] % p) % p;  // r < p < 2^12: no overflow
        ok = r != 0;
    }
    flags[i] = ok;
}

// x = 2x mod m for 0 <= x < m (radix-LB limbs)
template <int NL, int LB>
PMK_DEV void mod_double_limbs(uint32_t (&x)[NL], const uint32_t (&m)[NL]) {
    constexpr uint32_t MASK = Radix<LB>::MASK;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const uint32_t v = (x[j] << 1) + c;
        x[j] = v & MASK;
        c = v >> LB;
    }
    canonicalize<NL, LB>(x, m);
}

// limbs of x equal to table entry e (memory), lane-wise
template <int NL>
PMK_DEV bool equals_entry(const uint32_t (&x)[NL], const uint32_t *tbl, uint32_t e, int lane) {
    const uint32_t *t = fresh(tbl) + (size_t)e * NL * kTile + lane;
    uint32_t diff = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) diff |= x[j] ^ t[(size_t)j * kTile];
    return diff == 0;
}

// bits [pos, pos + w) of the candidate's words (zero past its end)
template <int SH>
PMK_DEV uint32_t bits_at(const uint32_t *m, int pos, int w) {
    const int k = pos >> 5, sh = pos & 31;
    const uint32_t lo = k < SH ? m[k] : 0u;
    const uint32_t hi = k + 1 < SH ? m[k + 1] : 0u;
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & ((1u << w) - 1u);
}

// Table slot entries: [0, 2^win) the window table, then R mod m, R^2 mod m and
// m - (R mod m) (the Montgomery forms of 1 and -1, and the entry constant).
template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void miller_rabin_kernel(
    const uint32_t *__restrict__ cand, uint32_t count, const uint32_t *__restrict__ bases, int rounds, int win,
    uint32_t *table, uint64_t slot_words, uint32_t *__restrict__ result) {
    code_align<code_id(kCodeMillerRabin, CB, 0)>();
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, SH = G.SH;
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const int lane = threadIdx.x, T = 1 << win;
    const uint32_t e_one = (uint32_t)T, e_rr = e_one + 1, e_neg = e_one + 2;
    uint32_t *tbl = table + (size_t)blockIdx.x * slot_words;
    const uint32_t nunits = (count + kTile - 1) / kTile;
    for (uint32_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        const uint32_t i0 = u * kTile + lane;
        const uint32_t i = i0 < count ? i0 : count - 1;
        const uint32_t *m32 = fresh_v(cand + (size_t)i * SH);
        uint32_t n[NL], acc[NL], b[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) n[j] = radix_limb_mem<SH, LB>(m32, 1, j);
        uint32_t x = m32[0];  // -m^-1 mod 2^LB by Newton's iteration on 32 bits
#pragma unroll
        for (int t = 0; t < 5; ++t) x *= 2u - m32[0] * x;
        const uint32_t n0 = (0u - x) & MASK;
        // R mod m and R^2 mod m by doubling from 1; -1 in Montgomery form
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = j == 0 ? 1u : 0u;
        for (int t = 0; t < LB * NL; ++t) mod_double_limbs<NL, LB>(acc, n);
        store_entry(tbl, e_one, lane, acc);
        {
            int32_t br = 0;
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const int32_t v = (int32_t)n[j] - (int32_t)acc[j] - br;
                b[j] = (uint32_t)v & MASK;
                br = v < 0 ? 1 : 0;
            }
            store_entry(tbl, e_neg, lane, b);
        }
        for (int t = 0; t < LB * NL; ++t) mod_double_limbs<NL, LB>(acc, n);
        store_entry(tbl, e_rr, lane, acc);
        // m - 1 = 2^s d
        int s = 1;
        while (s < 32 * SH && !((m32[s >> 5] >> (s & 31)) & 1u)) ++s;
        const int ndig = (32 * SH - s + win - 1) / win;  // digits of d (leading ones may be 0)
        const int smax = (int)wave_max((uint32_t)s);
        uint32_t pass_all = 1;
        for (int rd = 0; rd < rounds; ++rd) {
            const uint32_t *a32 = fresh_v(bases + ((size_t)i * rounds + rd) * SH);
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<SH, LB>(a32, 1, j);
            load_entry(b, tbl, e_rr, lane);
            mont_mul<NL, LB>(acc, acc, b, n, n0);  // a~
            store_entry(tbl, 1, lane, acc);
#pragma unroll
            for (int j = 0; j < NL; ++j) b[j] = acc[j];
            load_entry(acc, tbl, e_one, lane);
            store_entry(tbl, 0, lane, acc);
            load_entry(acc, tbl, 1, lane);
            for (int e = 2; e < T; ++e) {  // T[e] = T[e-1] a~
                mont_mul<NL, LB>(acc, acc, b, n, n0);
                store_entry(tbl, e, lane, acc);
            }
            // a^d: digits of d from the top (d's bit k is m's bit s + k)
            load_entry(acc, tbl, bits_at<SH>(m32, s + (ndig - 1) * win, win), lane);
            for (int k = ndig - 2; k >= 0; --k) {
                for (int q = 0; q < win; ++q) mont_sqr<NL, LB>(acc, acc, n, n0);
                load_entry(b, tbl, bits_at<SH>(m32, s + k * win, win), lane);
                mont_mul<NL, LB>(acc, acc, b, n, n0);
            }
            canonicalize<NL, LB>(acc, n);
            bool pass = equals_entry(acc, tbl, e_one, lane) || equals_entry(acc, tbl, e_neg, lane);
            bool dead = false;
            // a^(2^j d), j = 1 .. s-1: -1 passes, 1 (without -1 before it) is composite
            for (int j = 1; j < smax; ++j) {
                mont_sqr<NL, LB>(acc, acc, n, n0);
                canonicalize<NL, LB>(acc, n);
                if (j < s && !pass && !dead) {
                    if (equals_entry(acc, tbl, e_neg, lane))
                        pass = true;
                    else if (equals_entry(acc, tbl, e_one, lane))
                        dead = true;
                }
            }
            pass_all &= pass ? 1u : 0u;
        }
        if (i0 < count) result[i0] = pass_all;
    }
}

namespace {

template <int CB>
int launch_mr(const uint32_t *cand, uint32_t count, const uint32_t *bases, int rounds, int win, uint32_t *table,
              uint64_t slot_words, uint32_t grid, uint32_t *result, hipStream_t s) {
    hipLaunchKernelGGL(miller_rabin_kernel<CB>, dim3(grid), dim3(64), 0, s, cand, count, bases, rounds, win, table,
                       slot_words, result);
    return (int)hipGetLastError();
}

template <int SH>
int launch_sieve(const uint32_t *cand, uint32_t count, uint32_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(sieve_kernel<SH>, dim3((count + 255) / 256), dim3(256), 0, s, cand, count, flags);
    return (int)hipGetLastError();
}

template <int CB>
uint32_t mr_slots(int num_cus) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)miller_rabin_kernel<CB>, 64, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return (uint32_t)nb * (uint32_t)num_cus;
}

}  // namespace

int prime_class_ok(int cls) { return cls >= 3 && cls <= 6; }

uint64_t mr_slot_words(int cls, int win) {
    const Geom g = make_geom(kClassBits[cls]);
    return (uint64_t)((1 << win) + 3) * g.nlh * kTile;
}

uint32_t mr_wave_slots(int cls, int num_cus) {
    switch (cls) {
        case 3: return mr_slots<1024>(num_cus);
        case 4: return mr_slots<2048>(num_cus);
        case 5: return mr_slots<3072>(num_cus);
        case 6: return mr_slots<4096>(num_cus);
        default: return 0;
    }
}

int launch_sieve_class(int cls, const uint32_t *cand, uint32_t count, uint32_t *flags, int device, void *stream) {
    if (device < 0 || device >= 16) return (int)hipErrorInvalidValue;
    if (!primes_ready[device]) {
        uint16_t p[kSievePrimes];
        if (small_primes(p) != kSievePrimes) return (int)hipErrorInvalidValue;
        const hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_small_primes), p, sizeof p);
        if (e != hipSuccess) return (int)e;
        primes_ready[device] = true;
    }
    hipStream_t s = (hipStream_t)stream;
    switch (cls) {
        case 3: return launch_sieve<make_geom(1024).SH>(cand, count, flags, s);
        case 4: return launch_sieve<make_geom(2048).SH>(cand, count, flags, s);
        case 5: return launch_sieve<make_geom(3072).SH>(cand, count, flags, s);
        case 6: return launch_sieve<make_geom(4096).SH>(cand, count, flags, s);
        default: return (int)hipErrorInvalidValue;
    }
}

int launch_mr_class(int cls, const uint32_t *cand, uint32_t count, const uint32_t *bases, int rounds, int win,
                    uint32_t *table, uint64_t slot_words, uint32_t grid, uint32_t *result, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (cls) {
        case 3: return launch_mr<1024>(cand, count, bases, rounds, win, table, slot_words, grid, result, s);
        case 4: return launch_mr<2048>(cand, count, bases, rounds, win, table, slot_words, grid, result, s);
        case 5: return launch_mr<3072>(cand, count, bases, rounds, win, table, slot_words, grid, result, s);
        case 6: return launch_mr<4096>(cand, count, bases, rounds, win, table, slot_words, grid, result, s);
        default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace pmk
