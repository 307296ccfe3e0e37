// HIP kernels of the PMKRSA hot path for gfx950 (wave64).
//
//   pack      chunk bytes -> 32-bit limbs in [tile][word][lane] tiles
//             (Sec. 3.1: the message as a vector of chunk integers)
//   encrypt   c = m^e mod N, left-to-right binary exponentiation
//             (Sec. 1.1 step 2; Algorithm 2 in its left-to-right form)
//   halves    m_p = c^dp mod p and m_q = c^dq mod q, fixed-window
//             exponentiation (Sec. 2.1, equation CRT-RSA; Algorithm 2 with
//             w-bit digits instead of bits)
//   garner    h = qinv (m_p - m_q) mod p, m = m_q + h q (Sec. 2.1)
//   unpack    32-bit limbs -> big-endian bytes of each block
//
// Every bignum operation is one lane's work (64 bignums per wavefront); the
// Montgomery products (Sec. 3.2, Algorithm 3) are in mont.hpp.  A tile holds up
// to 64 chunks under one key, so modulus, exponent and window digits are
// wave-uniform.  The exponentiation kernels are persistent: each 64-thread block
// owns a scratch slot for its window table and walks tiles blockIdx.x,
// +gridDim.x, ...
#include <hip/hip_runtime.h>

#include "mont.hpp"
#include "pmk_internal.hpp"

namespace pmk {

#define PMK_DEV __device__ __forceinline__

PMK_DEV uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// word k (little-endian order) of the big-endian integer stored in
// src[base .. base+len): bytes [base+len-4k-4, base+len-4k); bytes before base are 0
PMK_DEV uint32_t be_word(const uint8_t *src, uint64_t base, int64_t len, int k) {
    const int64_t hi = len - 4 * (int64_t)k;
    if (hi <= 0) return 0u;
    const int64_t lo = hi - 4;
    if (lo >= 0 && ((base + (uint64_t)lo) & 3u) == 0)
        return bswap32(*reinterpret_cast<const uint32_t *>(src + base + lo));
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t pos = lo + b;
        if (pos >= 0) w |= (uint32_t)src[base + pos] << (8 * (3 - b));
    }
    return w;
}

// store word k (little-endian order) of a value into its big-endian byte field
// dst[base .. base+len)
PMK_DEV void be_store(uint8_t *dst, uint64_t base, int64_t len, int k, uint32_t w) {
    const int64_t hi = len - 4 * (int64_t)k;
    if (hi <= 0) return;
    const int64_t lo = hi - 4;
    if (lo >= 0 && ((base + (uint64_t)lo) & 3u) == 0) {
        *reinterpret_cast<uint32_t *>(dst + base + lo) = bswap32(w);
        return;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t pos = lo + b;
        if (pos >= 0) dst[base + pos] = (uint8_t)(w >> (8 * (3 - b)));
    }
}

// ------------------------------------------------------------------ pack / unpack
// One 256-thread block per tile of 64 chunks.  Reads walk each chunk's bytes in
// order (coalesced), the tile is transposed in LDS, writes are whole rows of 64
// lanes (coalesced).

template <int S>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *__restrict__ src,
                                                   const ChunkDesc *__restrict__ desc,
                                                   const uint32_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ tile_key, int stride,
                                                   int off_kbytes, uint32_t *__restrict__ x32, int decrypt) {
    __shared__ uint32_t tile[S * (kTile + 1)];
    const uint32_t t = blockIdx.x;
    const int64_t kb = keys[(size_t)tile_key[t] * stride + off_kbytes];
    for (int i = threadIdx.x; i < S * kTile; i += blockDim.x) {
        const int c = i / S, k = i % S;
        const ChunkDesc d = desc[(size_t)t * kTile + c];
        uint32_t w = 0;
        if (d.msg_len) w = decrypt ? be_word(src, d.ct_off, kb, k) : be_word(src, d.msg_off, d.msg_len, k);
        tile[k * (kTile + 1) + c] = w;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S * kTile; i += blockDim.x) {
        const int k = i / kTile, lane = i % kTile;
        x32[((size_t)t * S + k) * kTile + lane] = tile[k * (kTile + 1) + lane];
    }
}

template <int S>
__global__ __launch_bounds__(256) void unpack_kernel(const uint32_t *__restrict__ y32,
                                                     const ChunkDesc *__restrict__ desc,
                                                     const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ tile_key, int stride,
                                                     int off_kbytes, uint8_t *__restrict__ dst, int decrypt) {
    __shared__ uint32_t tile[S * (kTile + 1)];
    const uint32_t t = blockIdx.x;
    const int64_t kb = keys[(size_t)tile_key[t] * stride + off_kbytes];
    for (int i = threadIdx.x; i < S * kTile; i += blockDim.x) {
        const int k = i / kTile, lane = i % kTile;
        tile[k * (kTile + 1) + lane] = y32[((size_t)t * S + k) * kTile + lane];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S * kTile; i += blockDim.x) {
        const int c = i / S, k = i % S;
        const ChunkDesc d = desc[(size_t)t * kTile + c];
        if (!d.msg_len) continue;
        const uint32_t w = tile[k * (kTile + 1) + c];
        if (decrypt)
            be_store(dst, d.msg_off, d.msg_len, k, w);
        else
            be_store(dst, d.ct_off, kb, k, w);
    }
}

// ------------------------------------------------------------------ helpers
template <int NL>
PMK_DEV void load_limbs(uint32_t (&x)[NL], const uint32_t *p) {
#pragma unroll
    for (int j = 0; j < NL; ++j) x[j] = p[j];
}

// An opaque copy of a wave-uniform pointer.  Table addresses are otherwise
// loop-invariant, and the compiler hoists all NL per-limb addresses of every
// access out of the loops, where they occupy registers for the whole kernel;
// through this copy they are formed at each access from the scalar base.
template <typename T>
PMK_DEV T *fresh(T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Window-table entries live in global memory as [entry][limb][lane] words, one
// scratch slot per resident wave: every access of a wave is 64 consecutive words.
template <int NL>
PMK_DEV void store_entry(uint32_t *tbl, uint32_t e, int lane, const uint32_t (&x)[NL]) {
    uint32_t *t = fresh(tbl) + (size_t)e * NL * kTile + lane;
#pragma unroll
    for (int j = 0; j < NL; ++j) t[(size_t)j * kTile] = x[j];
}
template <int NL>
PMK_DEV void load_entry(uint32_t (&x)[NL], const uint32_t *tbl, uint32_t e, int lane) {
    const uint32_t *t = fresh(tbl) + (size_t)e * NL * kTile + lane;
#pragma unroll
    for (int j = 0; j < NL; ++j) x[j] = t[(size_t)j * kTile];
}
// x = table entry e (e > 0) or, for e = 0, the Montgomery one of the key record
template <int NL>
PMK_DEV void load_digit(uint32_t (&x)[NL], const uint32_t *tbl, uint32_t e, int lane, const uint32_t *one) {
    if (e) {
        load_entry(x, tbl, e, lane);
    } else {
        load_limbs(x, one);
    }
}

PMK_DEV uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// ------------------------------------------------------------------ encryption
// One lane per chunk: x~ = MM(x, R^2), then for the exponent bits below the top
// one: square, and multiply by x~ where the bit is set; MM(., 1) leaves
// Montgomery form.
template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void encrypt_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ tile_key, uint32_t ntiles,
    const uint32_t *__restrict__ x32, uint32_t *__restrict__ y32, uint32_t *__restrict__ table) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlf, LB = G.lbf, S = G.S;
    const int lane = threadIdx.x;
    uint32_t *tbl = table + (size_t)blockIdx.x * 2 * NL * kTile;

    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t *kr = keys + (size_t)tile_key[tile] * G.stride;  // wave-uniform
        uint32_t n[NL];
        load_limbs(n, kr + G.off_nf);
        const uint32_t n0 = kr[G.off_n0f];
        const uint32_t e0 = kr[G.off_e], e1 = kr[G.off_e + 1];
        const int top = (int)kr[G.off_ebits] - 1;

        uint32_t acc[NL], b[NL];
        {
            uint32_t w[S];
#pragma unroll
            for (int k = 0; k < S; ++k) w[k] = x32[((size_t)tile * S + k) * kTile + lane];
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[j] = radix_limb<S, LB>(w, j);
        }
        load_limbs(b, kr + G.off_rrf);
        mont_mul<NL, LB>(acc, acc, b, n, n0);  // x~ = x R mod N
        store_entry(tbl, 1, lane, acc);
        for (int bit = top - 1; bit >= 0; --bit) {
            mont_sqr<NL, LB>(acc, acc, n, n0);
            const uint32_t eb = bit >= 32 ? (e1 >> (bit - 32)) & 1u : (e0 >> bit) & 1u;
            if (eb) {
                load_entry(b, tbl, 1, lane);
                mont_mul<NL, LB>(acc, acc, b, n, n0);
            }
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
        mont_mul<NL, LB>(acc, acc, b, n, n0);  // leave Montgomery form
        canonicalize<NL, LB>(acc, n);
#pragma unroll
        for (int k = 0; k < S; ++k)
            y32[((size_t)tile * S + k) * kTile + lane] = radix_word<NL, LB>(acc, k);
    }
}

// ------------------------------------------------------------------ CRT halves
// Job tile jt = 2 t + h works on tile t's chunks modulo p (h = 0) or q (h = 1).
// Reduction and entry into Montgomery form at once:
// x~ = MM(c_lo, R^2) + MM(c_hi, R^3) = c R mod p (below 4p), with
// c = c_hi 2^(LB NL) + c_lo.  Table T[k] = x~^k (T[0] = R mod p), then
// fixed windows from the top: WIN squarings and one multiply by T[digit].
PMK_DEV uint32_t digit_of(const uint32_t *d, int SH, int k, int w) {
    const int pos = k * w;
    const int wd = pos >> 5, sh = pos & 31;
    const uint32_t lo = d[wd];
    const uint32_t hi = (wd + 1) < SH ? d[wd + 1] : 0u;
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & ((1u << w) - 1u);
}

template <int CB, int WIN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void halves_kernel(
    const uint32_t *__restrict__ keys, const ChunkDesc *__restrict__ desc,
    const uint32_t *__restrict__ tile_key, uint32_t ntiles, const uint32_t *__restrict__ x32,
    uint32_t *__restrict__ half, uint32_t *__restrict__ table, uint32_t *__restrict__ err) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S, SH = G.SH;
    constexpr int T = 1 << WIN;
    constexpr int NW = (32 * SH + WIN - 1) / WIN;  // digits of the exponent
    const int lane = threadIdx.x;
    const uint32_t njobs = 2 * ntiles;
    uint32_t *tbl = table + (size_t)blockIdx.x * T * NL * kTile;

    for (uint32_t jt = blockIdx.x; jt < njobs; jt += gridDim.x) {
        const uint32_t tile = jt >> 1;
        const int h = jt & 1;
        const uint32_t *kr = keys + (size_t)tile_key[tile] * G.stride;  // wave-uniform
        const uint32_t *hr = kr + G.off_half[0] + h * G.h_size;
        uint32_t n[NL];
        load_limbs(n, hr + G.h_m);
        const uint32_t n0 = hr[G.h_m0];
        const uint32_t *dexp = hr + G.h_d;
        const uint32_t *one_h = hr + G.h_one;

        uint32_t acc[NL], b[NL];
        {
            uint32_t w[S];
#pragma unroll
            for (int k = 0; k < S; ++k) w[k] = x32[((size_t)tile * S + k) * kTile + lane];
            if (h == 0 && desc[(size_t)tile * kTile + lane].msg_len) {
                // C must lie in Z_N: compare with N, most significant word first
                const uint32_t *n32 = kr + G.off_n32;
                int cmp = 0;
#pragma unroll
                for (int k = S - 1; k >= 0; --k) cmp = cmp ? cmp : (w[k] > n32[k]) - (w[k] < n32[k]);
                if (cmp >= 0) atomicOr(err, 1u);
            }
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[j] = radix_limb<S, LB>(w, j + NL);
            store_entry(tbl, 0, lane, acc);  // c_hi, parked in entry 0 until it is used
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[j] = radix_limb<S, LB>(w, j);
        }
        load_limbs(b, hr + G.h_rr);

        // One call site each for the product and the square keeps the loop's
        // code within the instruction cache.  Phases:
        //   0  MM(c_lo, R^2) = c_lo R mod p            (parked in T[1])
        //   1  MM(c_hi, R^3) = c_hi R^2 mod p; x~ = sum (below 4p), T[1] = x~
        //   2  T[e] = T[e-1] x~ for e = 2 .. T-1
        //   3  per digit below the top one: WIN squarings, then times T[digit]
        //   4  MM(., 1): leave Montgomery form
        int phase = 0, e = 2, digit = NW - 2, sq = 0;
        for (;;) {
            if (phase == 3) {
                if (sq < WIN) {
                    mont_sqr<NL, LB>(acc, acc, n, n0);
                    ++sq;
                    continue;
                }
                load_digit(b, tbl, digit_of(dexp, SH, digit, WIN), lane, one_h);
            }
            mont_mul<NL, LB>(acc, acc, b, n, n0);
            if (phase == 4) break;
            if (phase == 0) {
                store_entry(tbl, 1, lane, acc);
                load_entry(acc, tbl, 0, lane);
                load_limbs(b, hr + G.h_rrr);
                phase = 1;
                continue;
            }
            if (phase == 1) {
                load_entry(b, tbl, 1, lane);
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    const uint32_t v = acc[j] + b[j] + c;
                    acc[j] = v & Radix<LB>::MASK;
                    c = v >> LB;
                }
                store_entry(tbl, 1, lane, acc);
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // x~, the multiplier of phase 2
                phase = 2;
            } else if (phase == 2) {
                store_entry(tbl, e, lane, acc);
                ++e;
            } else {  // phase 3: the digit's multiply is done
                --digit;
                sq = 0;
            }
            if (phase == 2 && e == T) {
                // table complete: start from the top digit
                load_digit(acc, tbl, digit_of(dexp, SH, NW - 1, WIN), lane, one_h);
                phase = 3;
            }
            if (phase == 3 && digit < 0) {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                phase = 4;
            }
        }
        canonicalize<NL, LB>(acc, n);
        uint32_t *dst = half + ((size_t)jt * NL) * kTile + lane;
#pragma unroll
        for (int j = 0; j < NL; ++j) dst[(size_t)j * kTile] = acc[j];
    }
}

// ------------------------------------------------------------------ Garner
// One lane per chunk: h = MM(m_p + p - m_q, qinv R mod p) = qinv (m_p - m_q) mod p,
// canonical; m = m_q + h q by schoolbook columns.
template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void garner_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ tile_key,
    const uint32_t *__restrict__ half, uint32_t *__restrict__ y32) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S;
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const uint32_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t *kr = keys + (size_t)tile_key[tile] * G.stride;  // wave-uniform
    const uint32_t *hp = kr + G.off_half[0];
    const uint32_t *hq = kr + G.off_half[1];
    const uint32_t *mp_src = half + ((size_t)(2 * tile) * NL) * kTile + lane;
    const uint32_t *mq_src = half + ((size_t)(2 * tile + 1) * NL) * kTile + lane;

    uint32_t p[NL], mq[NL], a[NL], b[NL];
    load_limbs(p, hp + G.h_m);
#pragma unroll
    for (int j = 0; j < NL; ++j) mq[j] = mq_src[(size_t)j * kTile];
    {
        // a = m_p + p - m_q, in (0, 2p): limb-wise with signed carries
        int32_t c = 0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int32_t v = (int32_t)mp_src[(size_t)j * kTile] + (int32_t)p[j] - (int32_t)mq[j] + c;
            a[j] = (uint32_t)v & MASK;
            c = v >> LB;  // arithmetic shift: -1, 0 or 1
        }
    }
    load_limbs(b, kr + G.off_qinvr);
    mont_mul<NL, LB>(a, a, b, p, hp[G.h_m0]);
    canonicalize<NL, LB>(a, p);  // h

    uint32_t q[NL];
    load_limbs(q, hq + G.h_m);
    uint32_t m[2 * NL];
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < 2 * NL; ++k) {  // m = m_q + h q, column by column
        uint64_t acc = c + (k < NL ? mq[k] : 0u);
#pragma unroll
        for (int i = (k - NL + 1 > 0 ? k - NL + 1 : 0); i <= (k < NL ? k : NL - 1); ++i)
            acc += (uint64_t)a[i] * q[k - i];
        m[k] = (uint32_t)acc & MASK;
        c = acc >> LB;
    }
#pragma unroll
    for (int k = 0; k < S; ++k) y32[((size_t)tile * S + k) * kTile + lane] = radix_word<2 * NL, LB>(m, k);
}

// ------------------------------------------------------------------ launchers
namespace {

template <int CB>
constexpr int kWin = window_for(CB / 2);

template <int CB>
int occupancy_blocks(const void *fn) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

template <int CB>
uint32_t slots_for(int decrypt, int num_cus) {
    const void *fn = decrypt ? (const void *)halves_kernel<CB, kWin<CB>> : (const void *)encrypt_kernel<CB>;
    return (uint32_t)(occupancy_blocks<CB>(fn) * num_cus);
}

template <int CB>
int do_pack(const ClassRun &r, const uint8_t *src, int decrypt, hipStream_t s) {
    constexpr Geom G = make_geom(CB);
    hipLaunchKernelGGL(pack_kernel<G.S>, dim3(r.ntiles), dim3(256), 0, s, src, r.desc, r.keys, r.tile_key,
                       G.stride, G.off_kbytes, r.x32, decrypt);
    return (int)hipGetLastError();
}

template <int CB>
int do_unpack(const ClassRun &r, uint8_t *dst, int decrypt, hipStream_t s) {
    constexpr Geom G = make_geom(CB);
    hipLaunchKernelGGL(unpack_kernel<G.S>, dim3(r.ntiles), dim3(256), 0, s, r.y32, r.desc, r.keys, r.tile_key,
                       G.stride, G.off_kbytes, dst, decrypt);
    return (int)hipGetLastError();
}

template <int CB>
int do_encrypt(const ClassRun &r, hipStream_t s) {
    const uint32_t grid = r.ntiles < r.slots_enc ? r.ntiles : r.slots_enc;
    hipLaunchKernelGGL(encrypt_kernel<CB>, dim3(grid), dim3(64), 0, s, r.keys, r.tile_key, r.ntiles, r.x32,
                       r.y32, r.table);
    return (int)hipGetLastError();
}

template <int CB>
int do_halves(const ClassRun &r, hipStream_t s) {
    const uint32_t jobs = 2 * r.ntiles;
    const uint32_t grid = jobs < r.slots_dec ? jobs : r.slots_dec;
    hipLaunchKernelGGL((halves_kernel<CB, kWin<CB>>), dim3(grid), dim3(64), 0, s, r.keys, r.desc, r.tile_key,
                       r.ntiles, r.x32, r.half, r.table, r.err);
    return (int)hipGetLastError();
}

template <int CB>
int do_garner(const ClassRun &r, hipStream_t s) {
    hipLaunchKernelGGL(garner_kernel<CB>, dim3(r.ntiles), dim3(64), 0, s, r.keys, r.tile_key, r.half, r.y32);
    return (int)hipGetLastError();
}

#define PMK_DISPATCH(cls, CALL)           \
    switch (cls) {                        \
        case 0: { constexpr int CB = 128; CALL; } \
        case 1: { constexpr int CB = 256; CALL; } \
        case 2: { constexpr int CB = 512; CALL; } \
        case 3: { constexpr int CB = 1024; CALL; } \
        case 4: { constexpr int CB = 2048; CALL; } \
        default: return (int)hipErrorInvalidValue; \
    }

}  // namespace

int launch_pack(const ClassRun &r, const uint8_t *src, int decrypt, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, return do_pack<CB>(r, src, decrypt, (hipStream_t)stream));
}
int launch_unpack(const ClassRun &r, uint8_t *dst, int decrypt, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, return do_unpack<CB>(r, dst, decrypt, (hipStream_t)stream));
}
int launch_encrypt(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, return do_encrypt<CB>(r, (hipStream_t)stream));
}
int launch_decrypt_halves(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, return do_halves<CB>(r, (hipStream_t)stream));
}
int launch_garner(const ClassRun &r, void *stream) {
    if (r.ntiles == 0) return 0;
    PMK_DISPATCH(r.cls, return do_garner<CB>(r, (hipStream_t)stream));
}

uint64_t table_words_per_slot(int cls, int decrypt) {
    const Geom g = make_geom(kClassBits[cls]);
    if (!decrypt) return (uint64_t)2 * g.nlf * kTile;
    return (uint64_t)(1u << window_for(kClassBits[cls] / 2)) * g.nlh * kTile;
}

uint32_t wave_slots(int cls, int decrypt, int num_cus) {
    PMK_DISPATCH(cls, return slots_for<CB>(decrypt, num_cus));
}

}  // namespace pmk
