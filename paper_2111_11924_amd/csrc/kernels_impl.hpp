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
// Every CRT half (up to 2048 bits) and every full-size number up to 2048 bits
// is one lane's work (64 bignums per wavefront, Montgomery products in
// mont.hpp); full-size 3072- and 4096-bit numbers (encryption) are spread over
// 4 lanes (mont_lanes.hpp).  A tile holds 64 chunks under one key, so the
// modulus and exponent are wave-uniform.
// The exponentiation kernels are persistent: each 64-thread block owns a
// scratch slot for its window table and walks tiles blockIdx.x, +gridDim.x, ...
#pragma once
#include <hip/hip_runtime.h>

#include "mont.hpp"
#include "mont_lanes.hpp"
#include "pmk_internal.hpp"

namespace pmk {

#ifndef PMK_DEV
#define PMK_DEV __device__ __forceinline__
#endif

// ------------------------------------------------------------------ code alignment
// v_mad_u64_u32 is an 8-byte instruction.  In the long straight-line
// Montgomery products, runs of it at addresses 4 modulo 8 ran about 20 %
// slower than at 0 modulo 8 (CRT halves of 3072/4096-bit keys: 22.1 / 53.1 ms
// against 18.0 / 43.7 ms); short loops of it measure the same either way.  Where the
// multiply-adds of a kernel land depends on all the code before them, so the
// build reads them out of each compiled kernel and lists, in PMK_CODE_PAD, the
// kernels (code_id) with over 60 % of them at 4 modulo 8; each of those starts with
// one 4-byte s_nop, which moves all its code by 4 bytes.  Kernel kinds, the
// same numbers as the build's table:
enum CodeKind : uint32_t {
    kCodeEncrypt = 1, kCodeHalves = 2, kCodeJoint = 3, kCodeLanes = 4, kCodeJointLanes = 5, kCodeGarner = 6,
    kCodeGarnerLds = 7, kCodeBatchWide = 8, kCodeMpPart = 9, kCodeMpGarner = 10, kCodeMillerRabin = 11
};
#ifndef PMK_CODE_PAD
#define PMK_CODE_PAD 0u
#endif
constexpr uint32_t kCodePad[] = {PMK_CODE_PAD};
constexpr uint32_t code_id(CodeKind kind, int a, int b) { return (uint32_t)kind * 1000000u + (uint32_t)a * 10u + (uint32_t)b; }
constexpr bool code_padded(uint32_t id) {
    for (uint32_t x : kCodePad)
        if (x == id) return true;
    return false;
}
template <uint32_t ID>
PMK_DEV void code_align() {
    if constexpr (code_padded(ID)) asm volatile("s_nop 0");
}

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

template <int S, int CPT>
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *__restrict__ src,
                                                   const ChunkDesc *__restrict__ desc,
                                                   const uint32_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ tile_key, int stride,
                                                   int off_kbytes, uint32_t *__restrict__ x32, int decrypt) {
    __shared__ uint32_t tile[S * (CPT + 1)];
    const uint32_t t = blockIdx.x;
    const int64_t kb = keys[(size_t)tile_key[t] * stride + off_kbytes];
    for (int i = threadIdx.x; i < S * CPT; i += blockDim.x) {
        const int c = i / S, k = i % S;
        const ChunkDesc d = desc[(size_t)t * CPT + c];
        uint32_t w = 0;
        if (d.msg_len) w = decrypt ? be_word(src, d.ct_off, kb, k) : be_word(src, d.msg_off, d.msg_len, k);
        tile[k * (CPT + 1) + c] = w;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S * CPT; i += blockDim.x) {
        const int k = i / CPT, c = i % CPT;
        x32[((size_t)t * S + k) * CPT + c] = tile[k * (CPT + 1) + c];
    }
}

// Output forms of unpack_kernel.
enum UnpackMode {
    kOutCipher = 0,    // encryption: kb-byte blocks at ct_off
    kOutChunks = 1,    // decryption: msg_len bytes at msg_off, range-checked
    kOutBlocks = 2     // decryption: the whole m as a kb-byte block at ct_off, range-checked
};

// x (word k at x[k * CPT]) < n (word k at n[k]), most significant word first
template <int S, int CPT>
PMK_DEV bool below(const uint32_t *x, const uint32_t *n) {
    for (int k = S - 1; k >= 0; --k) {
        const uint32_t a = x[(size_t)k * CPT], b = n[k];
        if (a != b) return a < b;
    }
    return false;
}

// Decryption output keeps to the range of the scheme, as the oracle does: a
// chunk whose ciphertext block is not below its modulus (a ciphertext lies in
// Z_N, Sec. 1.1) -- checked against the packed input words chk and, for
// blinded decryption, chk2 -- or whose plaintext does not fit its msg_len bytes
// (no encryption of a chunk of that length has it) is written as zero bytes and
// sets bit 0 of *err (PMK_ERANGE), and its byte of slot_err when given.  The
// full-block form checks the range only.
template <int S, int CPT>
__global__ __launch_bounds__(256) void unpack_kernel(const uint32_t *__restrict__ y32,
                                                     const ChunkDesc *__restrict__ desc,
                                                     const uint32_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ tile_key, int stride,
                                                     int off_kbytes, int off_n32, uint8_t *__restrict__ dst, int mode,
                                                     const uint32_t *__restrict__ chk,
                                                     const uint32_t *__restrict__ chk2, uint32_t *err,
                                                     uint8_t *slot_err) {
    __shared__ uint32_t tile[S * (CPT + 1)];
    __shared__ uint32_t bad[CPT];
    const uint32_t t = blockIdx.x;
    const uint32_t *kr = keys + (size_t)tile_key[t] * stride;
    const int64_t kb = kr[off_kbytes];
    for (int i = threadIdx.x; i < S * CPT; i += blockDim.x) {
        const int k = i / CPT, c = i % CPT;
        tile[k * (CPT + 1) + c] = y32[((size_t)t * S + k) * CPT + c];
    }
    __syncthreads();
    if (mode != kOutCipher && threadIdx.x < CPT) {
        const int c = threadIdx.x;
        const uint32_t len = desc[(size_t)t * CPT + c].msg_len;
        uint32_t out = 0;
        if (len) {
            if (mode == kOutChunks) {
                // word len/4 keeps its low len%4 bytes; every byte above them must be 0
                const int full = (int)(len / 4), rem = (int)(len % 4);
                for (int k = full; k < S; ++k) {
                    const uint32_t w = tile[k * (CPT + 1) + c];
                    out |= (k == full && rem) ? w >> (8 * rem) : w;
                }
            }
            const uint32_t *n32 = kr + off_n32;
            if (chk && !below<S, CPT>(chk + (size_t)t * S * CPT + c, n32)) out = 1;
            if (chk2 && !below<S, CPT>(chk2 + (size_t)t * S * CPT + c, n32)) out = 1;
            if (out) {
                atomicOr(err, 1u);
                if (slot_err) slot_err[(size_t)t * CPT + c] = 1;  // names the chunk (request server)
            }
        }
        bad[c] = out;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S * CPT; i += blockDim.x) {
        const int c = i / S, k = i % S;
        const ChunkDesc d = desc[(size_t)t * CPT + c];
        if (!d.msg_len) continue;
        const uint32_t w = mode != kOutCipher && bad[c] ? 0u : tile[k * (CPT + 1) + c];
        if (mode == kOutChunks)
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
// wave-uniform values (key material of a key-uniform tile): readfirstlane keeps
// them in scalar registers even where the compiler cannot prove the load uniform
PMK_DEV uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
template <int NL>
PMK_DEV void load_uniform(uint32_t (&x)[NL], const uint32_t *p) {
#pragma unroll
    for (int j = 0; j < NL; ++j) x[j] = uni(p[j]);
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
// the same for a per-lane (VGPR) pointer or value
template <typename T>
PMK_DEV T *fresh_v(T *p) {
    asm volatile("" : "+v"(p));
    return p;
}
PMK_DEV int fresh_i(int x) {
    asm volatile("" : "+v"(x));
    return x;
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

// The CRT-halves table of the one-lane classes uses 16-byte rows instead:
// [entry][group of 4 limbs][lane] uint4 values, so one digit's entry can be
// copied into LDS by global_load_lds_dwordx4 (lane i's 16 bytes land at
// dst + 16 i) while the digit's squarings run, without holding registers.
template <int NL>
PMK_DEV void store_row4(uint32_t *tbl, uint32_t e, int lane, const uint32_t (&x)[NL]) {
    constexpr int G4 = (NL + 3) / 4;
    uint4 *t = reinterpret_cast<uint4 *>(fresh(tbl)) + (size_t)e * G4 * kTile + lane;
#pragma unroll
    for (int g = 0; g < G4; ++g) {
        uint4 v;
        v.x = x[4 * g];
        v.y = 4 * g + 1 < NL ? x[4 * g + 1] : 0u;
        v.z = 4 * g + 2 < NL ? x[4 * g + 2] : 0u;
        v.w = 4 * g + 3 < NL ? x[4 * g + 3] : 0u;
        t[(size_t)g * kTile] = v;
    }
}
template <int NL>
PMK_DEV void load_row4(uint32_t (&x)[NL], const uint32_t *tbl, uint32_t e, int lane) {
    constexpr int G4 = (NL + 3) / 4;
    const uint4 *t = reinterpret_cast<const uint4 *>(fresh(tbl)) + (size_t)e * G4 * kTile + lane;
#pragma unroll
    for (int g = 0; g < G4; ++g) {
        const uint4 v = t[(size_t)g * kTile];
        x[4 * g] = v.x;
        if (4 * g + 1 < NL) x[4 * g + 1] = v.y;
        if (4 * g + 2 < NL) x[4 * g + 2] = v.z;
        if (4 * g + 3 < NL) x[4 * g + 3] = v.w;
    }
}
// start copying entry e of this wave's table into lds[G4 * 64 * 4] (asynchronous)
template <int NL>
PMK_DEV void prefetch_row4(uint32_t *lds, const uint32_t *tbl, uint32_t e, int lane) {
    constexpr int G4 = (NL + 3) / 4;
    const uint4 *t = reinterpret_cast<const uint4 *>(fresh(tbl)) + (size_t)e * G4 * kTile + lane;
#pragma unroll
    for (int g = 0; g < G4; ++g)
        __builtin_amdgcn_global_load_lds((const void *)(t + (size_t)g * kTile),
                                         (__attribute__((address_space(3))) void *)(lds + g * kTile * 4), 16, 0, 0);
}
// wait for the copy, then read this lane's limbs out of LDS
template <int NL>
PMK_DEV void take_row4(uint32_t (&x)[NL], const uint32_t *lds, int lane) {
    constexpr int G4 = (NL + 3) / 4;
    __builtin_amdgcn_s_waitcnt(0);
    const uint4 *t = reinterpret_cast<const uint4 *>(lds) + lane;
#pragma unroll
    for (int g = 0; g < G4; ++g) {
        const uint4 v = t[g * kTile];
        x[4 * g] = v.x;
        if (4 * g + 1 < NL) x[4 * g + 1] = v.y;
        if (4 * g + 2 < NL) x[4 * g + 2] = v.z;
        if (4 * g + 3 < NL) x[4 * g + 3] = v.w;
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
// Montgomery form.  `tbl` is the calling wave's scratch slot.
template <int CB>
PMK_DEV void encrypt_unit(const ClassRun r, uint32_t tile, uint32_t *tbl) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlf, LB = G.lbf, S = G.S;
    const int lane = threadIdx.x;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;  // wave-uniform
    uint32_t n[NL];
    load_uniform(n, kr + G.off_nf);
    const uint32_t n0 = uni(kr[G.off_n0f]);
    const uint32_t e0 = uni(kr[G.off_e]), e1 = uni(kr[G.off_e + 1]);
    const int top = (int)uni(kr[G.off_ebits]) - 1;

    uint32_t acc[NL], b[NL];
    {
        uint32_t w[S];
#pragma unroll
        for (int k = 0; k < S; ++k) w[k] = r.x32[((size_t)tile * S + k) * kTile + lane];
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
    // leave Montgomery form: MM(x~^e, 1) = x^e; with a final factor v,
    // MM(x~^e, v) = x^e v mod N (blinded encryption: m^e r^e = (m r)^e)
    if (r.fin32) {
        const uint32_t *v = r.fin32 + (size_t)tile * S * kTile + lane;
#pragma unroll
        for (int j = 0; j < NL; ++j) b[j] = radix_limb_mem<S, LB>(v, kTile, j);
    } else {
#pragma unroll
        for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
    }
    mont_mul<NL, LB>(acc, acc, b, n, n0);
    canonicalize<NL, LB>(acc, n);
#pragma unroll
    for (int k = 0; k < S; ++k) r.y32[((size_t)tile * S + k) * kTile + lane] = radix_word<NL, LB>(acc, k);
}

// ------------------------------------------------------------------ CRT halves
// Job tile jt = 2 t + h works on tile t's chunks modulo p (h = 0) or q (h = 1).
// Reduction and entry into Montgomery form at once:
// x~ = MM(c_lo, R^2) + MM(c_hi, R^3) = c R mod p (below 4p), with
// c = c_hi 2^(LB NL) + c_lo.  Then sliding windows of at most r.win bits over
// a table of the odd powers x~^(2j+1), and a last product by 1.
PMK_DEV uint32_t digit_of(const uint32_t *d, int SH, int k, int w) {
    const int pos = k * w;
    const int wd = pos >> 5, sh = pos & 31;
    const uint32_t lo = d[wd];
    const uint32_t hi = (wd + 1) < SH ? d[wd + 1] : 0u;
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & ((1u << w) - 1u);
}

// Bits of a wave-uniform exponent of SH words (scalar registers and branches).
PMK_DEV uint32_t exp_bit(const uint32_t *d, int k) { return (uni(d[k >> 5]) >> (k & 31)) & 1u; }
// bits [l, l + len) of d, len <= 32
PMK_DEV uint32_t exp_bits(const uint32_t *d, int SH, int l, int len) {
    const int wd = l >> 5, sh = l & 31;
    const uint32_t lo = uni(d[wd]);
    const uint32_t hi = (wd + 1) < SH ? uni(d[wd + 1]) : 0u;
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & (uint32_t)((1ull << len) - 1u);
}
PMK_DEV int exp_top_bit(const uint32_t *d, int SH) {  // index of the highest set bit, -1 for d = 0
    for (int k = SH - 1; k >= 0; --k) {
        const uint32_t v = uni(d[k]);
        if (v) return 32 * k + 31 - __builtin_clz(v);
    }
    return -1;
}
// One step of the left-to-right sliding-window schedule, from bit i down: the
// zero bits above the next set bit j, then the window [l, j] of at most w bits
// that ends in a set bit at l.  The step squares nsq = (i - j) + (j - l + 1)
// times, then multiplies by the odd power x^v (table index v >> 1), v = d[l..j].
// Without a set bit left (j < 0) it squares i + 1 times and has no product.
struct WinStep {
    // packed into one scalar register: nsq in bits 0-12, idx in 13-17, the
    // product flag in 18, next + 1 in 19-31 (exponents of up to 8191 bits)
    uint32_t v;
    PMK_DEV static WinStep make(int nsq, uint32_t idx, bool mul, int next) {
        return WinStep{(uint32_t)nsq | (idx << 13) | ((uint32_t)mul << 18) | ((uint32_t)(next + 1) << 19)};
    }
    PMK_DEV int nsq() const { return (int)(v & 0x1FFFu); }
    PMK_DEV uint32_t idx() const { return (v >> 13) & 0x1Fu; }
    PMK_DEV bool mul() const { return (v >> 18) & 1u; }
    PMK_DEV int next() const { return (int)(v >> 19) - 1; }
};
PMK_DEV WinStep win_step(const uint32_t *d, int SH, int i, int w) {
    int j = i;
    while (j >= 0 && !exp_bit(d, j)) --j;
    if (j < 0) return WinStep::make(i + 1, 0u, false, -1);
    int l = j - w + 1 > 0 ? j - w + 1 : 0;
    while (!exp_bit(d, l)) ++l;
    return WinStep::make(i - l + 1, exp_bits(d, SH, l, j - l + 1) >> 1, true, l - 1);
}

// The three exponent words that end at bit i (words below bit 0 read as 0).
// Plain loads, issued one step ahead: nothing waits for them until the next
// step is planned, so their latency hides behind the current step's squarings.
struct ExpWords {
    uint32_t w0, w1, w2;
};
PMK_DEV ExpWords exp_words(const uint32_t *d, int i) {
    const int k = i >> 5;
    return ExpWords{k >= 2 ? d[k - 2] : 0u, k >= 1 ? d[k - 1] : 0u, d[k]};
}
// win_step from the 64 bits [i - 63, i] of preloaded words; bit by bit from
// memory when the zero run or the window reaches below them
PMK_DEV WinStep win_step_words(const uint32_t *d, int SH, int i, int w, ExpWords x) {
    const int sh = 31 - (i & 31);  // puts bit i at bit 63
    const uint64_t top = ((uint64_t)uni(x.w2) << 32) | uni(x.w1);
    const uint64_t v = sh ? (top << sh) | (uni(x.w0) >> (32 - sh)) : top;
    if (v == 0) return i < 64 ? WinStep::make(i + 1, 0u, false, -1) : win_step(d, SH, i, w);
    const int z = __builtin_clzll(v);
    if (z > 64 - w) return win_step(d, SH, i, w);
    const int j = i - z;                        // next set bit
    const int len = j - w + 1 >= 0 ? w : j + 1;  // window [j - len + 1, j]
    uint32_t val = (uint32_t)((v << z) >> (64 - len));
    const int tz = __builtin_ctz(val);
    val >>= tz;
    const int l = j - len + 1 + tz;
    return WinStep::make(i - l + 1, val >> 1, true, l - 1);
}
// the step after st, and the loads for the one after that
PMK_DEV void win_advance(WinStep &st, ExpWords &nx, const uint32_t *d, int SH, int w) {
    st = st.next() >= 0 ? win_step_words(d, SH, st.next(), w, nx) : WinStep::make(0, 0u, false, -1);
    if (st.next() >= 0) nx = exp_words(d, st.next());
}
// the first window (it starts at the top set bit top >= 0), with the loads for the step after it
PMK_DEV WinStep win_first(ExpWords &nx, const uint32_t *d, int SH, int top, int w) {
    const WinStep first = win_step(d, SH, top, w);
    if (first.next() >= 0) nx = exp_words(d, first.next());
    return first;
}

// Sliding windows (odd-power table, 2^(w-1) entries) where they measured
// faster: the one-lane classes up to 2048 bits (three waves per SIMD) and the
// lane-group classes; the 3072/4096-bit one-lane halves (two waves per SIMD)
// measured 6 % slower and 0 % faster with them and keep fixed windows (2^w
// entries, T[0] = R mod p).
template <int CB>
constexpr bool kSlidingHalves = lanes_half(CB) > 1 || make_geom(CB).nlh <= 40;

template <int CB>
PMK_DEV void halves_unit(const ClassRun r, uint32_t jt, uint32_t *tbl, uint32_t *lds) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S, SH = G.SH;
    const int win = r.win;
    const int lane = threadIdx.x;
    const uint32_t tile = jt >> 1;
    const int h = jt & 1;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;  // wave-uniform
    const uint32_t *hr = kr + G.off_half[0] + h * G.h_size;
    uint32_t n[NL];
    load_uniform(n, hr + G.h_m);
    const uint32_t n0 = uni(hr[G.h_m0]);
    const uint32_t *dexp = hr + G.h_d;
    const uint32_t *one_h = hr + G.h_one;

    uint32_t acc[NL], b[NL];
    if constexpr (S <= 64) {
        uint32_t w[S];
#pragma unroll
        for (int k = 0; k < S; ++k) w[k] = r.x32[((size_t)tile * S + k) * kTile + lane];
        if (h == 0 && r.desc[(size_t)tile * kTile + lane].msg_len) {
            // C must lie in Z_N: compare with N, most significant word first
            const uint32_t *n32 = kr + G.off_n32;
            int cmp = 0;
#pragma unroll
            for (int k = S - 1; k >= 0; --k) cmp = cmp ? cmp : (w[k] > n32[k]) - (w[k] < n32[k]);
            if (cmp >= 0) atomicOr(r.err, 1u);
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = radix_limb<S, LB>(w, j + NL);
        store_row4(tbl, 0, lane, acc);  // c_hi, parked in entry 0 until it is used
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = radix_limb<S, LB>(w, j);
    } else {
        // 3072/4096 bits: the ciphertext words are read from the tile in memory
        // (staging up to 128 words in registers would spill)
        const uint32_t *w = fresh_v(r.x32 + (size_t)tile * S * kTile + lane);
        if (h == 0 && r.desc[(size_t)tile * kTile + lane].msg_len) {
            // C must lie in Z_N: compare with N, most significant word first
            const uint32_t *n32 = kr + G.off_n32;
            int cmp = 0;
#pragma unroll 1
            for (int k = S - 1; k >= 0 && cmp == 0; --k) {
                const uint32_t x = w[(size_t)k * kTile], y = n32[k];
                cmp = (x > y) - (x < y);
            }
            if (cmp >= 0) atomicOr(r.err, 1u);
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w, kTile, j + NL);
        store_row4(tbl, 0, lane, acc);  // c_hi, parked in entry 0 until it is used
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w, kTile, j);
    }
    load_limbs(b, hr + G.h_rr);

    if constexpr (kSlidingHalves<CB>) {
        const int TH = 1 << (win - 1);  // odd powers x~, x~^3, ..., x~^(2 TH - 1)
        // One call site each for the product and the square keeps the loop's
        // code within the instruction cache.  Phases:
        //   0  MM(c_lo, R^2) = c_lo R mod p            (parked in entry 1)
        //   1  MM(c_hi, R^3) = c_hi R^2 mod p; x~ = sum (below 4p) -> entry 0
        //   2  x~^2 (the step between odd powers)
        //   5  entry e = x~^(2e+1) = entry e-1 times x~^2, e = 1 .. TH-1
        //   3  per window step: its squarings (while the step's odd power is
        //      copied into LDS), then times that power
        //   4  MM(., 1): leave Montgomery form
        int phase = 0, e = 1, sq = 0;
        WinStep st = WinStep::make(0, 0u, false, -1);
        ExpWords nx{0u, 0u, 0u};
        for (;;) {
            if (phase == 3) {
                if (sq < st.nsq()) {
                    if (sq == 0 && st.mul()) prefetch_row4<NL>(lds, tbl, st.idx(), lane);
                    mont_sqr<NL, LB>(acc, acc, n, n0);
                    ++sq;
                    continue;
                }
                if (st.mul()) {
                    take_row4(b, lds, lane);
                } else {  // trailing zero bits done
#pragma unroll
                    for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                    phase = 4;
                }
            }
            mont_mul<NL, LB>(acc, acc, b, n, n0);
            if (phase == 4) break;
            if (phase == 0) {
                store_row4(tbl, 1, lane, acc);
                load_row4(acc, tbl, 0, lane);
                load_limbs(b, hr + G.h_rrr);
                phase = 1;
                // table-building steps leave nothing in flight: the wait the
                // compiler puts where the window loop joins them would otherwise
                // also wait for the window's prefetch
                __builtin_amdgcn_s_waitcnt(0);
                continue;
            }
            if (phase == 1) {
                load_row4(b, tbl, 1, lane);
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    const uint32_t v = acc[j] + b[j] + c;
                    acc[j] = v & Radix<LB>::MASK;
                    c = v >> LB;
                }
                store_row4(tbl, 0, lane, acc);
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // next: x~ x~
                phase = 2;
                __builtin_amdgcn_s_waitcnt(0);
                continue;
            }
            if (phase == 2) {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // x~^2, the multiplier of phase 5
                load_row4(acc, tbl, 0, lane);
                phase = 5;
                __builtin_amdgcn_s_waitcnt(0);
                continue;
            }
            if (phase == 5) {
                store_row4(tbl, e, lane, acc);
                ++e;
                __builtin_amdgcn_s_waitcnt(0);
                if (e < TH) continue;
                // table complete: the first window starts at the top set bit
                // (no squarings of 1); d = 0 gives the Montgomery one
                const int top = exp_top_bit(dexp, SH);
                if (top < 0) {
                    load_limbs(acc, one_h);
                    st = WinStep::make(0, 0u, false, -1);
                } else {
                    st = win_first(nx, dexp, SH, top, win);
                    load_row4(acc, tbl, st.idx(), lane);
                    win_advance(st, nx, dexp, SH, win);
                }
                __builtin_amdgcn_s_waitcnt(0);
                phase = 3;
                sq = 0;
                continue;
            }
            // phase 3: the step's product is done
            win_advance(st, nx, dexp, SH, win);
            sq = 0;
        }
    } else {
        // fixed windows of win bits from the top: T[k] = x~^k (T[0] = R mod p)
        const int T = 1 << win;
        const int NW = (32 * SH + win - 1) / win;  // digits of the exponent
        // One call site each for the product and the square keeps the loop's
        // code within the instruction cache.  Phases:
        //   0  MM(c_lo, R^2) = c_lo R mod p            (parked in T[1])
        //   1  MM(c_hi, R^3) = c_hi R^2 mod p; x~ = sum (below 4p), T[1] = x~
        //   2  T[e] = T[e-1] x~ for e = 2 .. T-1
        //   3  per digit below the top one: win squarings (while T[digit] is
        //      copied into LDS), then times T[digit]
        //   4  MM(., 1): leave Montgomery form
        int phase = 0, e = 2, digit = NW - 2, sq = 0;
        for (;;) {
            if (phase == 3) {
                if (sq < win) {
                    if (sq == 0) prefetch_row4<NL>(lds, tbl, digit_of(dexp, SH, digit, win), lane);
                    mont_sqr<NL, LB>(acc, acc, n, n0);
                    ++sq;
                    continue;
                }
                take_row4(b, lds, lane);
            }
            mont_mul<NL, LB>(acc, acc, b, n, n0);
            if (phase == 4) break;
            if (phase == 0) {
                store_row4(tbl, 1, lane, acc);
                load_row4(acc, tbl, 0, lane);
                load_limbs(b, hr + G.h_rrr);
                phase = 1;
                // table-building steps leave nothing in flight: the wait the
                // compiler puts where the digit loop joins them would otherwise
                // also wait for the digit prefetch
                __builtin_amdgcn_s_waitcnt(0);
                continue;
            }
            if (phase == 1) {
                load_row4(b, tbl, 1, lane);
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    const uint32_t v = acc[j] + b[j] + c;
                    acc[j] = v & Radix<LB>::MASK;
                    c = v >> LB;
                }
                store_row4(tbl, 1, lane, acc);
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // x~, the multiplier of phase 2
                phase = 2;
                __builtin_amdgcn_s_waitcnt(0);
            } else if (phase == 2) {
                store_row4(tbl, e, lane, acc);
                ++e;
                __builtin_amdgcn_s_waitcnt(0);
            } else {  // phase 3: the digit's multiply is done
                --digit;
                sq = 0;
            }
            if (phase == 2 && e == T) {
                // table complete: T[0] = R mod p (the Montgomery one), start from the top digit
                load_limbs(b, one_h);
                store_row4(tbl, 0, lane, b);
                load_row4(acc, tbl, digit_of(dexp, SH, NW - 1, win), lane);
                __builtin_amdgcn_s_waitcnt(0);
                phase = 3;
            }
            if (phase == 3 && digit < 0) {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                phase = 4;
            }
        }
    }
    canonicalize<NL, LB>(acc, n);
    uint32_t *dst = r.half + ((size_t)jt * NL) * kTile + lane;
#pragma unroll
    for (int j = 0; j < NL; ++j) dst[(size_t)j * kTile] = acc[j];
}

// ------------------------------------------------------------------ blinded halves, one pass
// Blinded decryption (Sec. 3.1): per prime, (c*)^d_p (c_R^d_p)^-1 = (c*)^d_p c_R^(p-1-d_p)
// mod p.  Both powers in one chain (interleaved sliding windows, Moller 2001): one
// squaring per exponent bit for both exponents, and a product by the odd power of c* or
// c_R wherever a window of d_p or of p-1-d_p ends; two odd-power tables.  Against two
// separate exponentiations this drops one of the two squaring chains.  c* comes from
// r.x32, c_R from r.fin32; the result goes to r.half like a CRT half.  A c_R divisible
// by the prime sets bit 1 of r.err.
template <int CB>
PMK_DEV void halves_joint_unit(const ClassRun r, uint32_t jt, uint32_t *tbl, uint32_t *lds) {
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S, SH = G.SH;
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const int win = r.win, TH = 1 << (win - 1);  // T1 = entries [0, TH), T2 = [TH, 2 TH)
    const int lane = threadIdx.x;
    const uint32_t tile = jt >> 1;
    const int h = jt & 1;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;  // wave-uniform
    const uint32_t *hr = kr + G.off_half[0] + h * G.h_size;
    uint32_t n[NL];
    load_uniform(n, hr + G.h_m);
    const uint32_t n0 = uni(hr[G.h_m0]);
    const uint32_t *d1 = hr + G.h_d, *d2 = hr + G.h_d2;
    const uint32_t *w1 = fresh_v(r.x32 + (size_t)tile * S * kTile + lane);
    const uint32_t *w2 = fresh_v(r.fin32 + (size_t)tile * S * kTile + lane);
    if (h == 0 && r.desc[(size_t)tile * kTile + lane].msg_len) {
        // both blocks must lie in Z_N: compare with N, most significant word first
        const uint32_t *n32 = kr + G.off_n32;
        int cmp1 = 0, cmp2 = 0;
#pragma unroll 1
        for (int k = S - 1; k >= 0 && (cmp1 == 0 || cmp2 == 0); --k) {
            const uint32_t y = n32[k], a = w1[(size_t)k * kTile], b = w2[(size_t)k * kTile];
            if (cmp1 == 0) cmp1 = (a > y) - (a < y);
            if (cmp2 == 0) cmp2 = (b > y) - (b < y);
        }
        if (cmp1 >= 0 || cmp2 >= 0) atomicOr(r.err, 1u);
    }
    uint32_t acc[NL], b[NL];
    // c*_hi parked in entry 0, c*_lo first
#pragma unroll
    for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w1, kTile, j + NL);
    store_row4(tbl, 0, lane, acc);
#pragma unroll
    for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w1, kTile, j);
    load_limbs(b, hr + G.h_rr);
    // Phases, for input k = 0 (c*, table base 0) then k = 1 (c_R, table base TH):
    //   0 MM(lo, R^2) parked in base+1; 1 MM(hi, R^3) + parked = x~ -> entry base;
    //   2 x~^2; 3 odd powers base+e; 4 (c_R only) MM(x~, 1) = c_R mod p for the
    //   divisibility check; then 5 the joint chain: squarings down to the next
    //   window end, products by the odd powers ending there; 6 MM(., 1).
    int phase = 0, k = 0, e = 1, sq = 0, nsq = 0, pos = 0;
    uint32_t pend = 0;  // bit 0: a product by T1 at this event, bit 1: by T2
    WinStep s1 = WinStep::make(0, 0u, false, -1), s2 = s1;
    ExpWords nx1{0u, 0u, 0u}, nx2{0u, 0u, 0u};
    for (;;) {
        if (phase == 5) {
            if (sq < nsq) {
                if (sq == 0 && pend) prefetch_row4<NL>(lds, tbl, (pend & 1u) ? s1.idx() : TH + s2.idx(), lane);
                mont_sqr<NL, LB>(acc, acc, n, n0);
                ++sq;
                continue;
            }
            if (!pend) {  // squarings below the last window done
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                phase = 6;
            } else if (sq == nsq) {  // the event's first product: its entry is in LDS
                take_row4(b, lds, lane);
                sq = nsq + 1;
            } else {  // windows of both exponents end here: the T2 product, from memory
                load_row4(b, tbl, TH + s2.idx(), lane);
                __builtin_amdgcn_s_waitcnt(0);
                sq = nsq + 2;
            }
        }
        mont_mul<NL, LB>(acc, acc, b, n, n0);
        if (phase == 6) break;
        const int base = k * TH;
        if (phase == 0) {
            store_row4(tbl, base + 1, lane, acc);
            load_row4(acc, tbl, base, lane);
            load_limbs(b, hr + G.h_rrr);
            phase = 1;
            __builtin_amdgcn_s_waitcnt(0);
            continue;
        }
        if (phase == 1) {
            load_row4(b, tbl, base + 1, lane);
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const uint32_t v = acc[j] + b[j] + c;
                acc[j] = v & MASK;
                c = v >> LB;
            }
            store_row4(tbl, base, lane, acc);
            if (k == 1) {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                phase = 4;
            } else {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // next: x~ x~
                phase = 2;
            }
            __builtin_amdgcn_s_waitcnt(0);
            continue;
        }
        if (phase == 4) {
            // acc = c_R mod p in [0, p]: zero or p means p divides c_R
            uint32_t z = 0, q = 0;
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                z |= acc[j];
                q |= acc[j] ^ n[j];
            }
            if ((z == 0 || q == 0) && r.desc[(size_t)tile * kTile + lane].msg_len) atomicOr(r.err, 2u);
            load_row4(acc, tbl, base, lane);
#pragma unroll
            for (int j = 0; j < NL; ++j) b[j] = acc[j];  // next: x~ x~
            phase = 2;
            __builtin_amdgcn_s_waitcnt(0);
            continue;
        }
        if (phase == 2) {
#pragma unroll
            for (int j = 0; j < NL; ++j) b[j] = acc[j];  // x~^2, the step between odd powers
            load_row4(acc, tbl, base, lane);
            phase = 3;
            e = 1;
            __builtin_amdgcn_s_waitcnt(0);
            continue;
        }
        if (phase == 3) {
            store_row4(tbl, base + e, lane, acc);
            ++e;
            __builtin_amdgcn_s_waitcnt(0);
            if (e < TH) continue;
            if (k == 0) {  // c_R next: its hi part parked in entry TH, lo first
                k = 1;
                // an opaque copy of the base: the limb addresses are formed here,
                // not hoisted out of the loop into registers
                const uint32_t *wc = fresh_v(w2);
#pragma unroll
                for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(wc, kTile, j + NL);
                store_row4(tbl, TH, lane, acc);
                wc = fresh_v(wc);
#pragma unroll
                for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(wc, kTile, j);
                load_limbs(b, hr + G.h_rr);
                phase = 0;
                __builtin_amdgcn_s_waitcnt(0);
                continue;
            }
            // tables complete: the chain starts from the Montgomery one above the
            // higher of the two top bits
            load_limbs(acc, hr + G.h_one);
            const int t1 = exp_top_bit(d1, SH), t2 = exp_top_bit(d2, SH);
            if (t1 >= 0) s1 = win_first(nx1, d1, SH, t1, win);
            if (t2 >= 0) s2 = win_first(nx2, d2, SH, t2, win);
            pos = (t1 > t2 ? t1 : t2) + 1;
            phase = 5;
        } else if (sq == nsq + 1 && pend == 3u) {
            continue;  // phase 5: the T1 product is done, the T2 product of the same event follows
        } else {  // phase 5: the event's products are done
            if (pend & 1u) win_advance(s1, nx1, d1, SH, win);
            if (pend & 2u) win_advance(s2, nx2, d2, SH, win);
        }
        // next event: the higher window end still pending (window [l, ...], l = next + 1)
        const int l1 = s1.mul() ? s1.next() + 1 : -1, l2 = s2.mul() ? s2.next() + 1 : -1;
        const int ev = l1 > l2 ? l1 : l2;
        pend = ev < 0 ? 0u : (l1 == ev ? 1u : 0u) | (l2 == ev ? 2u : 0u);
        nsq = pos - (ev < 0 ? 0 : ev);  // no window left: square down to bit 0, then MM(., 1)
        pos = ev < 0 ? 0 : ev;
        sq = 0;
    }
    canonicalize<NL, LB>(acc, n);
    uint32_t *dst = r.half + ((size_t)jt * NL) * kTile + lane;
#pragma unroll
    for (int j = 0; j < NL; ++j) dst[(size_t)j * kTile] = acc[j];
}

// ------------------------------------------------------------------ lane groups
// 3072- and 4096-bit classes: a number is spread over a group of L lanes, lane
// `pos` holding limbs [pos K, pos K + K).  The multiplier of every product is
// staged in LDS as one column per group (limb i of group g at lds[i * NG + g]),
// so one call site serves squarings (stage acc), table products (x~ stays
// staged) and digit products (stage T[digit]).

// stage this lane's K limbs of a number into its group's LDS column (the
// per-lane base goes through an opaque copy so the K addresses are formed at
// each use as base + immediate, not hoisted into registers for the whole kernel)
template <int K, bool Flat = false>
PMK_DEV void stage_limbs(uint32_t *col, int ng, int pos, const uint32_t (&x)[K]) {
    lds_word<Flat> *d = opaque_lds(lds_k<Flat>(col + pos * K * ng));
#pragma unroll
    for (int j = 0; j < K; ++j) d[j * ng] = x[j];
}
// the same from memory: limb pos*K + j at src[j * stride]
template <int K, bool Flat = false>
PMK_DEV void stage_mem(uint32_t *col, int ng, int pos, const uint32_t *src, size_t stride) {
    uint32_t v[K];
    src = fresh_v(src);
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = src[j * stride];
    lds_word<Flat> *d = opaque_lds(lds_k<Flat>(col + pos * K * ng));
#pragma unroll
    for (int j = 0; j < K; ++j) d[j * ng] = v[j];
}
// the constant 1
template <int K, bool Flat = false>
PMK_DEV void stage_one(uint32_t *col, int ng, int pos) {
    lds_word<Flat> *d = opaque_lds(lds_k<Flat>(col + pos * K * ng));
#pragma unroll
    for (int j = 0; j < K; ++j) d[j * ng] = (pos == 0 && j == 0) ? 1u : 0u;
}
// this lane's radix limbs [first, first + K) of the number whose 32-bit words
// are in the group's LDS column
template <int K, int LB, bool Flat = false>
PMK_DEV void limbs_from_words(uint32_t (&x)[K], const uint32_t *col, int ng, int nwords, int first) {
    const lds_word<Flat> *cl = opaque_lds(lds_k<Flat>(col));
    first = fresh_i(first);  // keep the K word indices and shifts out of the loop-invariant set
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int bit = LB * (first + j);
        const int k = bit >> 5, sh = bit & 31;
        const uint32_t lo = k < nwords ? cl[k * ng] : 0u;
        const uint32_t hi = k + 1 < nwords ? cl[(k + 1) * ng] : 0u;
        x[j] = (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) & Radix<LB>::MASK;
    }
}

// LDS words the lane-group units of a class need
template <int CB>
constexpr int lds_words_enc() {
    return (make_geom(CB).nlf > make_geom(CB).S ? make_geom(CB).nlf : make_geom(CB).S) * (64 / lanes_full(CB));
}
// LDS words of the CRT-halves units: one-lane classes hold one prefetched
// table entry per wavefront; lane groups of L lanes one multiplier column per
// group (of nla limbs, or of the S input words while they are staged)
template <int CB, int L>
constexpr int lds_words_lanes() {
    return (lane_limbs(make_geom(CB), L) > make_geom(CB).S ? lane_limbs(make_geom(CB), L) : make_geom(CB).S) *
           (64 / L);
}
template <int CB>
constexpr int lds_words_dec() {
    return lanes_half(CB) == 1 ? pad4(make_geom(CB).nlh) * kTile : lds_words_lanes<CB, lanes_half(CB)>();
}

// Unit u encrypts chunks [part NG, part NG + NG) of tile u / L (part = u % L):
// a tile of 64 chunks takes L wavefronts of NG = 64 / L groups.
template <int CB>
PMK_DEV void encrypt_lanes_unit(const ClassRun r, uint32_t u, uint32_t *tbl, uint32_t *lds) {
    constexpr Geom G = make_geom(CB);
    constexpr int L = lanes_full(CB), NLT = G.nlf, K = NLT / L, LB = G.lbf, S = G.S;
    constexpr int NG = 64 / L;  // groups (chunks) per wavefront
    const uint32_t tile = u / L;
    const int part = (int)(u % L);
    const int lane = threadIdx.x, pos = lane % L, grp = lane / L;
    const int c = part * NG + grp;  // chunk within the tile
    uint32_t *col = lds + grp;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;  // wave-uniform
    uint32_t n[K];
    load_limbs(n, fresh_v(kr + G.off_nf + pos * K));
    const uint32_t n0 = uni(kr[G.off_n0f]);
    const uint32_t e0 = uni(kr[G.off_e]), e1 = uni(kr[G.off_e + 1]);
    const int top = (int)uni(kr[G.off_ebits]) - 1;

    uint32_t acc[K];
    for (int k = pos; k < S; k += L) col[k * NG] = r.x32[((size_t)tile * S + k) * kTile + c];
    limbs_from_words<K, LB>(acc, col, NG, S, pos * K);
    stage_mem<K>(col, NG, pos, kr + G.off_rrf + pos * K, 1);

    // phase 0: to Montgomery, 1: square, 2: multiply by x~, 3: from Montgomery
    int phase = 0, bit = top - 1;
    for (;;) {
        mont_mul_lanes<NLT, LB, L>(acc, acc, col, NG, n, n0, pos);
        if (phase == 3) break;
        if (phase == 0) {
            store_entry(tbl, 1, lane, acc);  // x~
        } else if (phase == 1) {
            const uint32_t eb = bit >= 32 ? (e1 >> (bit - 32)) & 1u : (e0 >> bit) & 1u;
            if (eb) {
                phase = 2;
                stage_mem<K>(col, NG, pos, fresh(tbl) + K * kTile + lane, kTile);
                continue;
            }
        }
        // next bit, or leave
        if (phase != 0) --bit;
        if (phase == 0) bit = top - 1;
        if (bit >= 0) {
            phase = 1;
            stage_limbs(col, NG, pos, acc);
        } else {
            phase = 3;
            if (r.fin32) {
                // final factor v (blinded encryption): this lane's K limbs of v into the column
                const uint32_t *v = fresh_v(r.fin32 + (size_t)tile * S * kTile + c);
#pragma unroll 1
                for (int j = 0; j < K; ++j) col[(pos * K + j) * NG] = radix_limb_mem<S, LB>(v, kTile, pos * K + j);
            } else {
                stage_one<K>(col, NG, pos);
            }
        }
    }
    canonicalize_lanes<K, LB, L>(acc, n, pos);
    // radix limbs -> 32-bit words through the group's column
    stage_limbs(col, NG, pos, acc);
    for (int k = pos; k < S; k += L) {
        const int bit = 32 * k, j = bit / LB, sh = bit % LB;
        const uint64_t l0 = j < NLT ? col[j * NG] : 0u;
        const uint64_t l1 = j + 1 < NLT ? col[(j + 1) * NG] : 0u;
        const uint64_t l2 = j + 2 < NLT ? col[(j + 2) * NG] : 0u;
        r.y32[((size_t)tile * S + k) * kTile + c] = (uint32_t)((l0 >> sh) | (l1 << (LB - sh)) | (l2 << (2 * LB - sh)));
    }
}

// CRT halves with L lanes per number: the only form of the 6144/8192-bit
// classes (L = 4), and for the one-lane classes the form of a launch's last
// partial round or of a launch too small to fill the chip (L = 2 or 4, on
// numbers of nla limbs with the record's lane-group constants).  Unit u works
// on chunks [part 64/L, part 64/L + 64/L) of tile t modulo p (h = 0) or q
// (h = 1), with u = (2 t + h) L + part.  The exponent is wave-uniform; the
// window table holds each lane's K limbs per entry ([entry][limb][lane]).
template <int CB, int L = lanes_half(CB)>
PMK_DEV void halves_lanes_unit(const ClassRun r, uint32_t u, uint32_t *tbl, uint32_t *lds) {
    constexpr Geom G = make_geom(CB);
    constexpr int NLT = lane_limbs(G, L), K = NLT / L, LB = G.lbh, S = G.S, SH = G.SH;
    static_assert(K * L == NLT, "lane-group limbs must split evenly");
    constexpr bool F = CB == 8192;  // generic pointers into the multiplier column (measured faster here)
    constexpr int NG = 64 / L;  // groups (chunks) per wavefront
    const int win = r.win, TH = 1 << (win - 1);  // odd powers x~, x~^3, ..., x~^(2 TH - 1)
    const uint32_t jt = u / L, tile = jt >> 1;
    const int h = (int)(jt & 1), part = (int)(u % L);
    const int lane = threadIdx.x, pos = lane % L, grp = lane / L;
    const int c = part * NG + grp;  // chunk within the tile
    uint32_t *col = lds + grp;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;
    const uint32_t *hr = kr + G.off_half[0] + h * G.h_size;
    uint32_t n[K];
    load_limbs(n, fresh_v(hr + G.h_m + pos * K));
    const uint32_t n0 = uni(hr[G.h_m0]);
    const uint32_t *dexp = hr + G.h_d;

    uint32_t acc[K];
    for (int k = pos; k < S; k += L) col[k * NG] = r.x32[((size_t)tile * S + k) * kTile + c];
    if (h == 0 && pos == 0 && r.desc[(size_t)tile * kTile + c].msg_len) {
        // C must lie in Z_N
        const uint32_t *n32 = kr + G.off_n32;
        int cmp = 0;
        for (int k = S - 1; k >= 0 && cmp == 0; --k) {
            const uint32_t w = col[k * NG];
            cmp = (w > n32[k]) - (w < n32[k]);
        }
        if (cmp >= 0) atomicOr(r.err, 1u);
    }
    limbs_from_words<K, LB, F>(acc, col, NG, S, NLT + pos * K);  // c_hi
    store_entry(tbl, 0, lane, acc);
    limbs_from_words<K, LB, F>(acc, col, NG, S, pos * K);        // c_lo
    stage_mem<K, F>(col, NG, pos, hr + lane_rr(G, L) + pos * K, 1);

    // phases as in halves_unit: 0 c_lo R, 1 c_hi R^2 and x~ (entry 0), 2 x~^2,
    // 5 odd powers (entry e = x~^(2e+1)), 3 sliding-window steps (squarings,
    // then a table product), 4 leave Montgomery form
    int phase = 0, e = 1, sq = 0;
    WinStep st = WinStep::make(0, 0u, false, -1);
    ExpWords nx{0u, 0u, 0u};
    for (;;) {
        mont_mul_lanes<NLT, LB, L, F>(acc, acc, col, NG, n, n0, pos);
        if (phase == 4) break;
        if (phase == 0) {
            store_entry(tbl, 1, lane, acc);
            load_entry(acc, tbl, 0, lane);
            stage_mem<K, F>(col, NG, pos, hr + lane_rrr(G, L) + pos * K, 1);
            phase = 1;
            continue;
        }
        if (phase == 1) {
            // x~ = acc + entry 1: limb-wise, carries across the group's lanes
            uint32_t lo[K];
            load_entry(lo, tbl, 1, lane);
            uint32_t cy = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t v = acc[j] + lo[j] + cy;
                acc[j] = v & Radix<LB>::MASK;
                cy = v >> LB;
            }
#pragma unroll
            for (int s = 1; s < L; ++s) {
                uint32_t cin = grp_prev<L>(cy, pos);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const uint32_t v = acc[j] + cin;
                    acc[j] = v & Radix<LB>::MASK;
                    cin = v >> LB;
                }
                cy = cin;
            }
            store_entry(tbl, 0, lane, acc);
            stage_limbs<K, F>(col, NG, pos, acc);  // next: x~ x~
            phase = 2;
            continue;
        }
        if (phase == 2) {
            stage_limbs<K, F>(col, NG, pos, acc);  // x~^2, the step between odd powers
            load_entry(acc, tbl, 0, lane);
            phase = 5;
            continue;
        }
        if (phase == 5) {
            store_entry(tbl, e, lane, acc);
            if (++e < TH) continue;
            // table complete: the first window starts at the top set bit
            const int top = exp_top_bit(dexp, SH);
            if (top < 0) {
                load_limbs(acc, fresh_v(hr + lane_one(G, L) + pos * K));
                st = WinStep::make(0, 0u, false, -1);
            } else {
                st = win_first(nx, dexp, SH, top, win);
                load_entry(acc, tbl, st.idx(), lane);
                win_advance(st, nx, dexp, SH, win);
            }
            phase = 3;
            sq = 0;
        } else if (sq > st.nsq()) {  // phase 3: the step's product is done
            win_advance(st, nx, dexp, SH, win);
            sq = 0;
        }
        // phase 3: next squaring, the step's product, or the end
        if (sq < st.nsq()) {
            stage_limbs<K, F>(col, NG, pos, acc);
            ++sq;
        } else if (st.mul()) {
            stage_mem<K, F>(col, NG, pos, fresh(tbl) + (size_t)st.idx() * K * kTile + lane, kTile);
            sq = st.nsq() + 1;
        } else {
            stage_one<K, F>(col, NG, pos);
            phase = 4;
        }
    }
    canonicalize_lanes<K, LB, L>(acc, n, pos);
    // the result is below p: limbs from nlh up are zero and not stored (the
    // half buffer holds nlh limbs per number)
    uint32_t *dst = r.half + ((size_t)(2 * tile + h) * G.nlh + pos * K) * kTile + c;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (NLT == G.nlh || pos * K + j < G.nlh) dst[(size_t)j * kTile] = acc[j];
}

// Blinded decryption in one pass per prime with each CRT half spread over a
// group of L lanes: the chain of halves_joint_unit, with each product's
// multiplier staged in LDS as in halves_lanes_unit.  The lane-group classes
// (L = lanes_half) always run it; the one-lane classes run it with L = 2 or 4
// in nla limbs (R_A = 2^(lbh nla), the constants at h_rra, h_rrra, h_onea)
// for launches that leave SIMDs idle.
template <int CB, int L = lanes_half(CB)>
PMK_DEV void halves_lanes_joint_unit(const ClassRun r, uint32_t u, uint32_t *tbl, uint32_t *lds) {
    constexpr Geom G = make_geom(CB);
    constexpr int NLT = lane_limbs(G, L), K = NLT / L, LB = G.lbh, S = G.S, SH = G.SH;
    static_assert(K * L == NLT, "lane-group limbs must split evenly");
    constexpr int NG = 64 / L;  // groups (chunks) per wavefront
    const int win = r.win, TH = 1 << (win - 1);  // T1 = entries [0, TH), T2 = [TH, 2 TH)
    const uint32_t jt = u / L, tile = jt >> 1;
    const int h = (int)(jt & 1), part = (int)(u % L);
    const int lane = threadIdx.x, pos = lane % L, grp = lane / L;
    const int c = part * NG + grp;  // chunk within the tile
    uint32_t *col = lds + grp;
    const uint32_t *kr = r.keys + (size_t)uni(r.tile_key[tile]) * G.stride;
    const uint32_t *hr = kr + G.off_half[0] + h * G.h_size;
    uint32_t n[K];
    load_limbs(n, fresh_v(hr + G.h_m + pos * K));
    const uint32_t n0 = uni(hr[G.h_m0]);
    const uint32_t *d1 = hr + G.h_d, *d2 = hr + G.h_d2;
    const bool live = r.desc[(size_t)tile * kTile + c].msg_len != 0;
    uint32_t acc[K];
    // input x (c* or c_R): words staged in the group's LDS column, range check,
    // hi part parked in entry `base`, lo part in acc, R^2 staged as the multiplier
    auto take_input = [&](const uint32_t *x32, int base) {
        for (int k = pos; k < S; k += L) col[k * NG] = x32[((size_t)tile * S + k) * kTile + c];
        if (h == 0 && pos == 0 && live) {
            const uint32_t *n32 = kr + G.off_n32;
            int cmp = 0;
            for (int k = S - 1; k >= 0 && cmp == 0; --k) {
                const uint32_t w = col[k * NG];
                cmp = (w > n32[k]) - (w < n32[k]);
            }
            if (cmp >= 0) atomicOr(r.err, 1u);
        }
        limbs_from_words<K, LB>(acc, col, NG, S, NLT + pos * K);
        store_entry(tbl, base, lane, acc);
        limbs_from_words<K, LB>(acc, col, NG, S, pos * K);
        stage_mem<K>(col, NG, pos, hr + lane_rr(G, L) + pos * K, 1);
    };
    take_input(r.x32, 0);
    // phases as in halves_joint_unit: 0 lo R, 1 hi R^2 and x~ (entry base),
    // 4 (c_R) MM(x~, 1) for the divisibility check, 2 x~^2, 3 odd powers, 5 the
    // joint chain, 6 MM(., 1)
    int phase = 0, k = 0, e = 1, sq = 0, nsq = 0, at = 0;
    uint32_t pend = 0;
    WinStep s1 = WinStep::make(0, 0u, false, -1), s2 = s1;
    ExpWords nx1{0u, 0u, 0u}, nx2{0u, 0u, 0u};
    for (;;) {
        mont_mul_lanes<NLT, LB, L>(acc, acc, col, NG, n, n0, pos);
        if (phase == 6) break;
        const int base = k * TH;
        if (phase == 0) {
            store_entry(tbl, base + 1, lane, acc);
            load_entry(acc, tbl, base, lane);
            stage_mem<K>(col, NG, pos, hr + lane_rrr(G, L) + pos * K, 1);
            phase = 1;
            continue;
        }
        if (phase == 1) {
            // x~ = acc + entry base+1: limb-wise, carries across the group's lanes
            uint32_t lo[K];
            load_entry(lo, tbl, base + 1, lane);
            uint32_t cy = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t v = acc[j] + lo[j] + cy;
                acc[j] = v & Radix<LB>::MASK;
                cy = v >> LB;
            }
#pragma unroll
            for (int s = 1; s < L; ++s) {
                uint32_t cin = grp_prev<L>(cy, pos);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const uint32_t v = acc[j] + cin;
                    acc[j] = v & Radix<LB>::MASK;
                    cin = v >> LB;
                }
                cy = cin;
            }
            store_entry(tbl, base, lane, acc);
            if (k == 1) {
                stage_one<K>(col, NG, pos);
                phase = 4;
            } else {
                stage_limbs(col, NG, pos, acc);  // next: x~ x~
                phase = 2;
            }
            continue;
        }
        if (phase == 4) {
            // acc = c_R mod p in [0, p], over the group: zero or p means p divides c_R
            uint32_t z = 0, q = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                z |= acc[j];
                q |= acc[j] ^ n[j];
            }
#pragma unroll
            for (int off = 1; off < L; off <<= 1) {
                z |= (uint32_t)__shfl_xor((int)z, off, 64);
                q |= (uint32_t)__shfl_xor((int)q, off, 64);
            }
            if ((z == 0 || q == 0) && pos == 0 && live) atomicOr(r.err, 2u);
            load_entry(acc, tbl, base, lane);
            stage_limbs(col, NG, pos, acc);  // next: x~ x~
            phase = 2;
            continue;
        }
        if (phase == 2) {
            stage_limbs(col, NG, pos, acc);  // x~^2, the step between odd powers
            load_entry(acc, tbl, base, lane);
            phase = 3;
            e = 1;
            continue;
        }
        bool plan = false;
        if (phase == 3) {
            store_entry(tbl, base + e, lane, acc);
            if (++e < TH) continue;
            if (k == 0) {  // c_R next
                k = 1;
                take_input(r.fin32, TH);
                phase = 0;
                continue;
            }
            // tables complete: the chain starts from the Montgomery one above the
            // higher of the two top bits
            load_limbs(acc, fresh_v(hr + lane_one(G, L) + pos * K));
            const int t1 = exp_top_bit(d1, SH), t2 = exp_top_bit(d2, SH);
            if (t1 >= 0) s1 = win_first(nx1, d1, SH, t1, win);
            if (t2 >= 0) s2 = win_first(nx2, d2, SH, t2, win);
            at = (t1 > t2 ? t1 : t2) + 1;
            phase = 5;
            plan = true;
        } else if (sq > nsq) {  // phase 5: a product of the event is done
            if (sq == nsq + 1 && pend == 3u) {  // windows of both exponents end here: T2 next
                stage_mem<K>(col, NG, pos, fresh(tbl) + (size_t)(TH + s2.idx()) * K * kTile + lane, kTile);
                sq = nsq + 2;
                continue;
            }
            if (pend & 1u) win_advance(s1, nx1, d1, SH, win);
            if (pend & 2u) win_advance(s2, nx2, d2, SH, win);
            plan = true;
        }
        if (plan) {  // next event: the higher window end still pending (l = next + 1)
            const int l1 = s1.mul() ? s1.next() + 1 : -1, l2 = s2.mul() ? s2.next() + 1 : -1;
            const int ev = l1 > l2 ? l1 : l2;
            pend = ev < 0 ? 0u : (l1 == ev ? 1u : 0u) | (l2 == ev ? 2u : 0u);
            nsq = at - (ev < 0 ? 0 : ev);
            at = ev < 0 ? 0 : ev;
            sq = 0;
        }
        // phase 5: the next squaring, the event's first product, or the end
        if (sq < nsq) {
            stage_limbs(col, NG, pos, acc);
            ++sq;
        } else if (!pend) {
            stage_one<K>(col, NG, pos);
            phase = 6;
        } else {
            const uint32_t ent = (pend & 1u) ? s1.idx() : TH + s2.idx();
            stage_mem<K>(col, NG, pos, fresh(tbl) + (size_t)ent * K * kTile + lane, kTile);
            sq = nsq + 1;
        }
    }
    canonicalize_lanes<K, LB, L>(acc, n, pos);
    // below p: limbs from nlh up are zero and not stored (nlh limbs per number)
    uint32_t *dst = r.half + ((size_t)(2 * tile + h) * G.nlh + pos * K) * kTile + c;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (NLT == G.nlh || pos * K + j < G.nlh) dst[(size_t)j * kTile] = acc[j];
}

// ------------------------------------------------------------------ per-class kernels
// Persistent grids: block b owns table slot b and walks units b, b + grid, ...
template <int CB>
constexpr int kEncWaves = 2;
template <int CB>
constexpr int kDecWaves = (make_geom(CB).nlh > 40 || lanes_half(CB) > 1) ? 2 : 3;

template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kEncWaves<CB>))) void encrypt_kernel(
    ClassRun r, uint64_t slot_words) {
    code_align<code_id(kCodeEncrypt, CB, 0)>();
    uint32_t *tbl = r.table + (size_t)blockIdx.x * slot_words;
    if constexpr (lanes_full(CB) > 1) {
        __shared__ uint32_t lds[lds_words_enc<CB>()];
        const uint32_t units = r.ntiles * lanes_full(CB);
        for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) encrypt_lanes_unit<CB>(r, u, tbl, lds);
    } else {
        for (uint32_t u = blockIdx.x; u < r.ntiles; u += gridDim.x) encrypt_unit<CB>(r, u, tbl);
    }
}

// blinded decryption in one pass (every class: one lane per number up to 4096
// bits, lane groups above; the chain uses sliding windows whatever the class's
// plain decryption uses); two waves per SIMD: the second table's state does not
// fit the three-wave budget
template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void halves_joint_kernel(
    ClassRun r, uint64_t slot_words, uint32_t u_begin, uint32_t u_end) {
    code_align<code_id(kCodeJoint, CB, 0)>();
    uint32_t *tbl = r.table + (size_t)blockIdx.x * slot_words;
    __shared__ uint32_t lds[lds_words_dec<CB>()];
    for (uint32_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) {
        if constexpr (lanes_half(CB) > 1)
            halves_lanes_joint_unit<CB>(r, u, tbl, lds);
        else
            halves_joint_unit<CB>(r, u, tbl, lds);
    }
}

// blinded decryption of a one-lane class in lane groups of L lanes: lane-group
// units [u_begin, u_end) (u = job tile x L + part)
template <int CB, int L>
__global__ __launch_bounds__(64) void halves_lanes_joint_kernel(ClassRun r, uint64_t slot_words, uint32_t u_begin,
                                                                uint32_t u_end) {
    code_align<code_id(kCodeJointLanes, CB, L)>();
    uint32_t *tbl = r.table + (size_t)blockIdx.x * slot_words;
    __shared__ uint32_t lds[lds_words_lanes<CB, L>()];
    for (uint32_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) halves_lanes_joint_unit<CB, L>(r, u, tbl, lds);
}

template <int CB>
// units [u_begin, u_end) of the class's own form (job tiles 2 t + h for one
// lane per number, lane-group units for the 6144/8192-bit classes)
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kDecWaves<CB>))) void halves_kernel(
    ClassRun r, uint64_t slot_words, uint32_t u_begin, uint32_t u_end) {
    code_align<code_id(kCodeHalves, CB, 0)>();
    uint32_t *tbl = r.table + (size_t)blockIdx.x * slot_words;
    __shared__ uint32_t lds[lds_words_dec<CB>()];
    for (uint32_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) {
        if constexpr (lanes_half(CB) > 1)
            halves_lanes_unit<CB>(r, u, tbl, lds);
        else
            halves_unit<CB>(r, u, tbl, lds);
    }
}

// CRT halves of a one-lane class in lane groups of L lanes: lane-group units
// [u_begin, u_end) (u = job tile x L + part)
template <int CB, int L>
__global__ __launch_bounds__(64) void halves_lanes_kernel(ClassRun r, uint64_t slot_words, uint32_t u_begin,
                                                          uint32_t u_end) {
    code_align<code_id(kCodeLanes, CB, L)>();
    uint32_t *tbl = r.table + (size_t)blockIdx.x * slot_words;
    __shared__ uint32_t lds[lds_words_lanes<CB, L>()];
    for (uint32_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) halves_lanes_unit<CB, L>(r, u, tbl, lds);
}

// ------------------------------------------------------------------ Garner
// One lane per chunk slot (64 consecutive slots per block, keys per lane):
// h = MM(m_p + p - m_q, qinv R mod p) = qinv (m_p - m_q) mod p, canonical;
// m = m_q + h q by schoolbook columns.
template <int CB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(make_geom(CB).nlh > 40 ? 1 : 2))) void garner_kernel(
    const uint32_t *__restrict__ keys, const ChunkDesc *__restrict__ desc, uint32_t nslots,
    const uint32_t *__restrict__ half, uint32_t *__restrict__ y32) {
    code_align<code_id(kCodeGarner, CB, 0)>();
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S, CPT = chunks_per_tile(CB);
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const uint32_t slot0 = blockIdx.x * 64 + threadIdx.x;
    const uint32_t slot = slot0 < nslots ? slot0 : nslots - 1;
    const uint32_t tile = slot / CPT, c = slot % CPT;
    const uint32_t *kr = keys + (size_t)desc[slot].key * G.stride;
    const uint32_t *hp = kr + G.off_half[0];
    const uint32_t *hq = kr + G.off_half[1];
    const uint32_t *mp_src = half + ((size_t)(2 * tile) * NL) * CPT + c;
    const uint32_t *mq_src = half + ((size_t)(2 * tile + 1) * NL) * CPT + c;

    uint32_t p[NL], mq[NL], a[NL], b[NL];
    load_limbs(p, hp + G.h_m);
#pragma unroll
    for (int j = 0; j < NL; ++j) mq[j] = mq_src[(size_t)j * CPT];
    {
        // a = m_p + p - m_q, in (0, 2p): limb-wise with signed carries
        int32_t cy = 0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int32_t v = (int32_t)mp_src[(size_t)j * CPT] + (int32_t)p[j] - (int32_t)mq[j] + cy;
            a[j] = (uint32_t)v & MASK;
            cy = v >> LB;  // arithmetic shift: -1, 0 or 1
        }
    }
    load_limbs(b, kr + G.off_qinvr);
    mont_mul<NL, LB>(a, a, b, p, hp[G.h_m0]);
    canonicalize<NL, LB>(a, p);  // h

    uint32_t q[NL];
    load_limbs(q, hq + G.h_m);
    uint32_t m[2 * NL];
    uint64_t cy = 0;
#pragma unroll
    for (int k = 0; k < 2 * NL; ++k) {  // m = m_q + h q, column by column
        uint64_t acc = cy + (k < NL ? mq[k] : 0u);
#pragma unroll
        for (int i = (k - NL + 1 > 0 ? k - NL + 1 : 0); i <= (k < NL ? k : NL - 1); ++i)
            acc += (uint64_t)a[i] * q[k - i];
        m[k] = (uint32_t)acc & MASK;
        cy = acc >> LB;
    }
    if (slot0 < nslots) {
#pragma unroll
        for (int k = 0; k < S; ++k) y32[((size_t)tile * S + k) * CPT + c] = radix_word<2 * NL, LB>(m, k);
    }
}

// The CRT recombination of the 6144/8192-bit classes (CRT halves of 112/152
// limbs, one lane per chunk slot): the numbers do not fit a lane's registers,
// so each lane keeps them in LDS, [limb][lane] rows that 32 lanes read without
// bank conflicts (32 slots per block: a block never spans two tiles, so p, q
// and the constants are the block's, staged once).  Operand-scanning
// Montgomery product over a circular accumulator (no shifting: at step i
// logical limb j of t sits in row (i + j) mod (NL + 1)), then the schoolbook
// product h q column by column, written out word by word.
constexpr int kGarnerLdsSlots = 32;

template <int CB>
__global__ __launch_bounds__(kGarnerLdsSlots) void garner_lds_kernel(const uint32_t *__restrict__ keys,
                                                                     const ChunkDesc *__restrict__ desc,
                                                                     uint32_t nslots,
                                                                     const uint32_t *__restrict__ half,
                                                                     uint32_t *__restrict__ y32) {
    code_align<code_id(kCodeGarnerLds, CB, 0)>();
    constexpr Geom G = make_geom(CB);
    constexpr int NL = G.nlh, LB = G.lbh, S = G.S, CPT = chunks_per_tile(CB), B = kGarnerLdsSlots, M = NL + 1;
    constexpr uint32_t MASK = Radix<LB>::MASK;
    static_assert(CPT % B == 0, "a block must lie within one tile");
    static_assert((2.0 * NL + 1) * (double)(1ull << LB) * (double)(1ull << LB) < 18446744073709551615.0,
                  "column sums may overflow 64 bits");
    __shared__ uint64_t t[M][B];      // the product's accumulator (circular)
    __shared__ uint32_t a[NL][B];     // m_p + p - m_q, then h
    __shared__ uint32_t pn[NL], qinv[NL], qn[NL];
    const int lane = threadIdx.x;
    const uint32_t slot0 = blockIdx.x * B + lane;
    const uint32_t slot = slot0 < nslots ? slot0 : nslots - 1;
    const uint32_t tile = slot / CPT, c = slot % CPT;
    // the block's key (every slot of a tile, padding included, carries it)
    const uint32_t *kr = keys + (size_t)desc[(size_t)blockIdx.x * B].key * G.stride;
    const uint32_t *hp = kr + G.off_half[0];
    const uint32_t *hq = kr + G.off_half[1];
    for (int j = lane; j < NL; j += B) {
        pn[j] = hp[G.h_m + j];
        qinv[j] = kr[G.off_qinvr + j];
        qn[j] = hq[G.h_m + j];
    }
    const uint32_t n0 = hp[G.h_m0];
    __syncthreads();
    const uint32_t *mp_src = half + ((size_t)(2 * tile) * NL) * CPT + c;
    const uint32_t *mq_src = half + ((size_t)(2 * tile + 1) * NL) * CPT + c;
    {
        // a = m_p + p - m_q, in (0, 2p)
        int32_t cy = 0;
#pragma unroll 4
        for (int j = 0; j < NL; ++j) {
            const int32_t v = (int32_t)mp_src[(size_t)j * CPT] + (int32_t)pn[j] - (int32_t)mq_src[(size_t)j * CPT] + cy;
            a[j][lane] = (uint32_t)v & MASK;
            cy = v >> LB;
        }
    }
#pragma unroll 4
    for (int j = 0; j < M; ++j) t[j][lane] = 0;
    // t = a qinv R^-1 (mod p) by operand scanning: at step i, t += a qinv_i,
    // then + m_i p, then divide by 2^LB; logical limb j of t in row (i + j) mod M
#pragma unroll 1
    for (int i = 0; i < NL; ++i) {
        const uint64_t bi = qinv[i];
        int r = i;
#pragma unroll 4
        for (int j = 0; j < NL; ++j) {
            t[r][lane] += (uint64_t)a[j][lane] * bi;
            r = r + 1 == M ? 0 : r + 1;
        }
        const uint64_t t0 = t[i][lane];
        const uint64_t m = ((uint32_t)t0 * n0) & MASK;
        r = i;
#pragma unroll 4
        for (int j = 0; j < NL; ++j) {
            t[r][lane] += m * pn[j];
            r = r + 1 == M ? 0 : r + 1;
        }
        // the lowest limb is now a multiple of 2^LB: its carry moves up, its row
        // becomes the spare row (logical limb NL) of the next step
        const uint64_t carry = t[i][lane] >> LB;
        t[i][lane] = 0;
        const int r1 = i + 1 == M ? 0 : i + 1;
        t[r1][lane] += carry;
    }
    // settle the carries of the result (logical limb j in row (NL + j) mod M)
    {
        uint64_t cy = 0;
        int r = NL % M;
#pragma unroll 4
        for (int j = 0; j < NL; ++j) {
            const uint64_t v = t[r][lane] + cy;
            a[j][lane] = (uint32_t)v & MASK;
            cy = v >> LB;
            r = r + 1 == M ? 0 : r + 1;
        }
    }
    // a < 2p -> h = a mod p: keep a - p when it does not borrow
    {
        int32_t borrow = 0;
#pragma unroll 4
        for (int j = 0; j < NL; ++j) borrow = ((int32_t)a[j][lane] - (int32_t)pn[j] - borrow) < 0 ? 1 : 0;
        if (!borrow) {
            borrow = 0;
#pragma unroll 4
            for (int j = 0; j < NL; ++j) {
                const int32_t v = (int32_t)a[j][lane] - (int32_t)pn[j] - borrow;
                a[j][lane] = (uint32_t)v & MASK;
                borrow = v < 0 ? 1 : 0;
            }
        }
    }
    // m = m_q + h q, column by column, written out word by word as columns complete
    uint64_t cy = 0, wacc = 0;
    int wbits = 0, k32 = 0;
#pragma unroll 1
    for (int k = 0; k < 2 * NL && k32 < S; ++k) {
        uint64_t acc = cy + (k < NL ? mq_src[(size_t)k * CPT] : 0u);
        const int lo = k - NL + 1 > 0 ? k - NL + 1 : 0, hi = k < NL ? k : NL - 1;
#pragma unroll 4
        for (int i = lo; i <= hi; ++i) acc += (uint64_t)a[i][lane] * qn[k - i];
        wacc |= (uint64_t)((uint32_t)acc & MASK) << wbits;
        wbits += LB;
        cy = acc >> LB;
        while (wbits >= 32 && k32 < S) {
            if (slot0 < nslots) y32[((size_t)tile * S + k32) * CPT + c] = (uint32_t)wacc;
            wacc >>= 32;
            wbits -= 32;
            ++k32;
        }
    }
    for (; k32 < S; ++k32) {  // (not reached: 2 NL LB >= 32 S)
        if (slot0 < nslots) y32[((size_t)tile * S + k32) * CPT + c] = (uint32_t)wacc;
        wacc >>= 32;
    }
}

}  // namespace pmk
