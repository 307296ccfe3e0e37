// Multi-prime CRT keys (Sec. 2.1, the multi-prime variant of CRT-RSA: N is a
// product of b distinct primes and decryption runs b exponentiations of size
// bits/b): record layout shared by the host (key load) and the kernels.
// Supported: 3072-bit keys with 3 primes and 4096-bit keys with 4 primes, all
// primes of 1024 bits, held as 37 limbs of 28 bits (the geometry of the
// 2048-bit class's CRT halves).
#pragma once
#include "pmk_internal.hpp"

namespace pmk {

constexpr int kMpMaxParts = 4;
constexpr int kMpLB = 28;
constexpr int kMpNL = nl_for(1024, kMpLB);  // 37 limbs: R = 2^1036
constexpr int kMpSP = 32;                   // words of a prime and of its exponent
constexpr int kMpClasses = 2;               // [0] 3072 bits / 3 primes, [1] 4096 bits / 4 primes
constexpr int mp_bits(int k) { return k == 0 ? 3072 : 4096; }
constexpr int mp_parts(int k) { return k == 0 ? 3 : 4; }

// Offsets (words) of one multi-prime key record of class k.
struct MpGeom {
    int S;                       // words of N
    int parts;                   // primes
    int off_n32, off_kbytes;     // N as words (range check), key bytes
    int off_part[kMpMaxParts];   // part records
    // within a part record: p (radix), p0 = -p^-1 mod 2^LB, R^(2+k) mod p for
    // k < parts (radix; R^2 .. R^(parts+1)), R mod p, d mod (p-1) as words,
    // then (p_j^-1 mod p) R mod p for every earlier prime j (radix)
    int q_m, q_m0, q_rpow, q_one, q_d, q_cinv, q_size;
    int stride;
};

PMK_HD constexpr MpGeom make_mp_geom(int k) {
    MpGeom g{};
    g.S = mp_bits(k) / 32;
    g.parts = mp_parts(k);
    constexpr int pl = pad4(kMpNL);
    g.q_m = 0;
    g.q_m0 = pl;
    g.q_rpow = pl + 4;
    g.q_one = g.q_rpow + kMpMaxParts * pl;
    g.q_d = g.q_one + pl;
    g.q_cinv = g.q_d + kMpSP;
    g.q_size = g.q_cinv + (kMpMaxParts - 1) * pl;
    int o = 0;
    g.off_n32 = o;
    o += pad4(g.S);
    g.off_kbytes = o;
    o += 4;
    for (int i = 0; i < kMpMaxParts; ++i) {
        g.off_part[i] = o;
        o += g.q_size;
    }
    g.stride = pad4(o);
    return g;
}

// Launchers (kmp.hip); asynchronous on `stream`, return hipError_t as int.
// Buffers: x32/y32 [tile][word][chunk] (S words), parts [tile][part][limb][chunk].
int mp_launch_pack(int k, const uint8_t *src, const ChunkDesc *desc, const uint32_t *keys, const uint32_t *tile_key,
                   uint32_t ntiles, uint32_t *x32, void *stream);
int mp_launch_parts(int k, const uint32_t *keys, const uint32_t *tile_key, const ChunkDesc *desc, uint32_t ntiles,
                    const uint32_t *x32, uint32_t *parts, uint32_t *table, uint64_t slot_words, uint32_t grid,
                    int win, uint32_t *err, void *stream);
int mp_launch_garner(int k, const uint32_t *keys, const ChunkDesc *desc, uint32_t ntiles, uint32_t *parts,
                     uint32_t *y32, void *stream);
// plaintext chunks; a block not below N (checked against x32) or a plaintext
// wider than its chunk is written as zeros and sets bit 0 of *err
int mp_launch_unpack(int k, const uint32_t *y32, const ChunkDesc *desc, const uint32_t *keys,
                     const uint32_t *tile_key, uint32_t ntiles, const uint32_t *x32, uint8_t *dst, uint32_t *err,
                     void *stream);
uint64_t mp_slot_words(int win);
uint32_t mp_wave_slots(int num_cus);

}  // namespace pmk
