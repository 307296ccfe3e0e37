// Internal layout shared by the host side of the library and its kernels.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define PMK_HD __host__ __device__
#else
#define PMK_HD
#endif

namespace pmk {

// Modulus size classes the kernels are instantiated for (kMaxClass: the
// largest one built).  A key of `bits`
// bits runs in the smallest class with at least that many bits: Montgomery
// arithmetic only needs R > 4m, so a smaller modulus fits a larger class.
constexpr int kNumClasses = 9;
constexpr int kClassBits[kNumClasses] = {128, 256, 512, 1024, 2048, 3072, 4096, 6144, 8192};
constexpr int kMaxClass = 8;

PMK_HD constexpr int nl_for(int bits, int lb) { return (bits + 2 + lb - 1) / lb; }

// Radix of the full-size modulus: 28-bit limbs keep every column sum of a
// Montgomery product below 2^64 up to 3072 bits; 4096-bit moduli use 27 bits.
PMK_HD constexpr int lb_full(int bits) { return bits > 3072 ? 27 : 28; }
PMK_HD constexpr int lb_half(int bits) { return lb_full(bits / 2); }

// Lanes per bignum.  Full-size numbers: one lane up to 2048-bit moduli, a
// group of 4 lanes at 3072/4096 bits and of 8 lanes at 6144/8192 bits.  CRT
// halves: one lane up to 2048-bit primes (4096-bit keys), 4 lanes above.
PMK_HD constexpr int lanes_full(int bits) { return bits >= 6144 ? 8 : (bits >= 3072 ? 4 : 1); }
PMK_HD constexpr int lanes_half(int bits) { return bits >= 6144 ? 4 : 1; }
// chunks per tile: 64, one wavefront of one-lane numbers; with L lanes per
// number a tile's exponentiation takes L wavefronts of 64/L chunks each
PMK_HD constexpr int chunks_per_tile(int) { return 64; }
PMK_HD constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }
// grid of a persistent launch: one wave per unit, at most `slots` (the table
// slots) and at most `cap` when a cap is set
PMK_HD constexpr uint32_t persistent_grid(uint32_t units, uint32_t slots, uint32_t cap) {
    const uint32_t g = units < slots ? units : slots;
    return cap && cap < g ? cap : g;
}

// Default window width of the fixed-window exponentiation of the CRT halves
// (the autotuner may pick another one up to kMaxWin).
PMK_HD constexpr int window_for(int bits) { return bits <= 256 ? 3 : (bits <= 512 ? 4 : 5); }

// Offsets (uint32 words) of one key record of a class.
struct Geom {
    int bits, S, SH;
    int lbf, nlf, lbh, nlh;
    // CRT halves spread over a lane group (2 or 4 lanes per number): nla
    // limbs (a multiple of 4) and the constants of R_A = 2^(lbh nla); for the
    // classes whose halves always run in lane groups these are the nlh-limb ones
    int nla;
    int ew;  // words of the public exponent
    // full-modulus part
    int off_n32, off_nf, off_n0f, off_rrf, off_rrrf, off_onef, off_e, off_ebits, off_kbytes;
    // half records (p then q): m, m0, rr, rrr, one, d, and d2 = m - 1 - d (the
    // exponent of the Fermat inverse of c^d, for blinded decryption), then
    // one, rr, rrr of the lane-group form
    int off_half[2];
    int h_m, h_m0, h_rr, h_rrr, h_one, h_d, h_d2, h_onea, h_rra, h_rrra, h_size;
    int nla8, h_onea8, h_rra8, h_rrra8;  // the same for groups of 8 lanes (nla8 a multiple of 8)
    int off_qinvr;
    int stride;
};

PMK_HD constexpr int pad4(int x) { return (x + 3) & ~3; }

// Every radix-form field starts on a 16-byte boundary and is padded to a
// multiple of 4 limbs, so kernels read it with 128-bit loads.
PMK_HD constexpr Geom make_geom(int bits) {
    Geom g{};
    g.bits = bits;
    g.S = bits / 32;
    g.SH = bits / 64;
    g.lbf = lb_full(bits);
    g.nlf = round_up(nl_for(bits, g.lbf), lanes_full(bits));
    g.lbh = lb_half(bits);
    g.nlh = round_up(nl_for(bits / 2, g.lbh), lanes_half(bits));
    g.ew = 2;
    // lane-group limb counts: nla (a multiple of 4: groups of 2 and 4 lanes)
    // and nla8 (a multiple of 8: groups of 8); the half fields hold the larger,
    // zero-padded, since a lane group reads its K limbs of every field at pos K
    const int nla = lanes_half(bits) > 1 ? g.nlh : round_up(g.nlh, 4);
    const int nla8 = lanes_half(bits) > 1 ? g.nlh : (bits >= 2048 ? round_up(g.nlh, 8) : nla);
    const int pf = pad4(g.nlf), ph = pad4(nla8);
    int o = 0;
    g.off_nf = o; o += pf;
    g.off_rrf = o; o += pf;
    g.off_rrrf = o; o += pf;
    g.off_onef = o; o += pf;
    g.off_n32 = o; o += pad4(g.S);
    g.off_n0f = o; o += 1;
    g.off_e = o; o += g.ew;
    g.off_ebits = o; o += 1;
    g.off_kbytes = o; o += 4;
    // half record: m, rr, rrr, one (radix form), then m0, d
    g.h_m = 0;
    g.h_rr = ph;
    g.h_rrr = 2 * ph;
    g.h_one = 3 * ph;
    g.h_m0 = 4 * ph;
    g.h_d = 4 * ph + 4;
    g.h_d2 = g.h_d + pad4(g.SH);
    g.nla = nla;
    g.nla8 = nla8;
    if (lanes_half(bits) > 1) {  // lane groups already: the same constants
        g.h_onea = g.h_onea8 = g.h_one;
        g.h_rra = g.h_rra8 = g.h_rr;
        g.h_rrra = g.h_rrra8 = g.h_rrr;
        g.h_size = pad4(g.h_d2 + g.SH);
    } else {
        g.h_onea = pad4(g.h_d2 + g.SH);
        g.h_rra = g.h_onea + nla;
        g.h_rrra = g.h_rra + nla;
        g.h_size = g.h_rrra + nla;
        if (nla8 == nla) {
            g.h_onea8 = g.h_onea;
            g.h_rra8 = g.h_rra;
            g.h_rrra8 = g.h_rrra;
        } else {  // 4096 bits: 74 limbs, 76 for 2 and 4 lanes, 80 for 8
            g.h_onea8 = g.h_size;
            g.h_rra8 = g.h_onea8 + nla8;
            g.h_rrra8 = g.h_rra8 + nla8;
            g.h_size = g.h_rrra8 + nla8;
        }
    }
    g.off_half[0] = o; o += g.h_size;
    g.off_half[1] = o; o += g.h_size;
    g.off_qinvr = o; o += ph;
    g.stride = pad4(o);
    return g;
}

// Chunks are grouped into tiles of up to chunks_per_tile chunks that share one
// key, so a wavefront's modulus and exponent are wave-uniform (scalar
// registers, no divergence).  Slot = tile * chunks_per_tile + chunk; a padding
// slot has msg_len 0 and is computed but never written back.
struct ChunkDesc {
    uint64_t msg_off;  // first plaintext byte of the chunk
    uint64_t ct_off;   // first ciphertext byte of the chunk's block
    uint32_t key;      // record index inside the class key table
    uint32_t msg_len;  // plaintext bytes of this chunk (kb - 4, or the remainder); 0 = padding
};

constexpr int kTile = 64;  // bignums per wavefront

// Arguments of one class's launches inside a plan.
struct ClassRun {
    int cls;                   // index into kClassBits
    uint32_t count;            // chunks of this class
    uint32_t ntiles;           // key-uniform tiles of this class
    const uint32_t *keys;      // class key table (device), Geom::stride words per key
    const ChunkDesc *desc;     // ntiles * cpt slot descriptors (device)
    const uint32_t *tile_key;  // ntiles key records (device)
    uint32_t *x32;             // [tile][word < S][chunk < cpt]: packed input words
    uint32_t *y32;             // same shape: result words before unpacking
    uint32_t *half;            // [tile][p, q][limb < nlh][chunk < cpt]: CRT half results
    uint32_t *table;           // per resident wave: window table scratch
    uint32_t slots_enc;        // wave slots in `table` for the encryption kernel
    uint32_t slots_dec;        // wave slots in `table` for the CRT-halves kernel
    uint32_t *err;             // device error word: bit 0 block out of range, bit 1 blinding factor not invertible
    uint8_t *slot_err;         // optional, per descriptor slot: 1 where unpacking rejected the chunk
    uint32_t grid_cap;         // 0, or the most resident waves a persistent launch may use
    int win;                   // window width of the CRT-halves exponentiation (3..6)
    int fill_lanes;            // lanes per number of the CRT halves of a launch under one round
                               // (one-lane classes 1, 2 or 4; lane-group classes lanes_half or twice it)
    int tail_lanes;            // one-lane classes: the same for the partial round after full ones,
                               // run as a launch of its own; 0: that round stays in the launch
    // blinded PMKRSA (Sec. 3.1, Algorithm 1)
    const uint32_t *fin32;     // encryption: words of a factor v < N the result is multiplied by
                               // (x^e v mod N; tile layout of y32), nullptr = 1; blinded decryption:
                               // the packed c_R blocks
};

constexpr int kMaxWin = 6;
// default lanes per number of a one-lane class's CRT halves in a launch that
// fills at most half a round, and in a short last round after full ones
// (measured: 4 lanes cut a 1 MiB 2048-bit decryption by a fifth; a 2-lane
// last round of the 100 MiB one is about even)
// One-lane classes whose CRT halves also run in groups of 8 lanes (2048- to
// 4096-bit keys, the classes whose record holds the nla8-limb constants), for
// small launches.
PMK_HD constexpr bool eight_lanes(int bits) { return lanes_half(bits) == 1 && bits >= 2048; }

// Limb count and constants (offsets in a half record) of the lane-group form
// with L lanes per number: nla limbs for 2 and 4 lanes, nla8 for 8.
PMK_HD constexpr int lane_limbs(const Geom &g, int L) { return L == 8 ? g.nla8 : g.nla; }
PMK_HD constexpr int lane_one(const Geom &g, int L) { return L == 8 ? g.h_onea8 : g.h_onea; }
PMK_HD constexpr int lane_rr(const Geom &g, int L) { return L == 8 ? g.h_rra8 : g.h_rra; }
PMK_HD constexpr int lane_rrr(const Geom &g, int L) { return L == 8 ? g.h_rrra8 : g.h_rrra; }
// Lanes-per-number settings a class takes: a one-lane class 1, 2 or 4 for
// both forms, and 8 for small launches where eight_lanes; a lane-group class
// its own count L0, or 2 L0 for small launches, and L0 for the tail form.
PMK_HD constexpr bool lanes_valid(int bits, int fill, int tail) {
    return lanes_half(bits) == 1
               ? ((fill == 1 || fill == 2 || fill == 4 || (fill == 8 && eight_lanes(bits))) &&
                  (tail == 1 || tail == 2 || tail == 4))
               : ((fill == lanes_half(bits) || fill == 2 * lanes_half(bits)) && tail == lanes_half(bits));
}
PMK_HD constexpr int default_fill_lanes(int bits) {
    return lanes_half(bits) > 1 ? 2 * lanes_half(bits) : (eight_lanes(bits) ? 8 : (bits >= 1024 ? 4 : 1));
}
PMK_HD constexpr int default_tail_lanes(int bits) { return lanes_half(bits) > 1 ? lanes_half(bits) : 1; }

// One persistent launch over the exponentiation work of the 1024- to 4096-bit
// classes of a plan: units (tiles, or job tiles of CRT halves) are numbered
// class by class, largest modulus first, and handed out by an atomic counter.
// The encryption of the 4096- and 3072-bit classes (4 lanes per number) runs
// as one persistent kernel whose waves take work units from a device counter,
// 4096-bit units first.
constexpr int kWideClasses = 2;
constexpr int kClass3072 = 5, kClass4096 = 6;
// class of entry i of the wide batch: 4096 bits, then 3072 bits
constexpr int wide_class(int i) { return kClass4096 - i; }
constexpr bool is_wide_class(int c) { return c == kClass3072 || c == kClass4096; }
struct BatchArgs {
    ClassRun runs[kWideClasses];       // runs[i] is class wide_class(i)
    uint32_t start[kWideClasses + 1];  // first unit of runs[i]; start[2] = total
    uint32_t *counter;                 // next unit to hand out (reset before each launch)
    uint32_t *table;                   // per-block window-table slots
    uint64_t slot_words;               // words per slot
};

// Launchers (kernels.hip).  All asynchronous on `stream`; return hipError_t as int.
int launch_pack(const ClassRun &r, const uint8_t *src, int decrypt, void *stream);
int launch_encrypt(const ClassRun &r, void *stream);
int launch_decrypt_halves(const ClassRun &r, void *stream);
int launch_garner(const ClassRun &r, void *stream);
// blinded decryption in one pass per prime: half[h] = (c*)^d_h c_R^(p_h-1-d_h) mod p_h
// with c* at r.x32 and c_R at r.fin32; tables need 2 table_words_per_slot(cls, 1, win)
// words per slot
int launch_decrypt_joint(const ClassRun &r, void *stream);
// CRT halves of job tiles [jt_begin, jt_end) in lane groups of L lanes per
// number: a one-lane class (128..4096 bits) with L = 2 or 4, a lane-group class
// (6144/8192 bits) with twice its own L (klanes.hip)
int launch_halves_lanes(const ClassRun &r, int L, uint32_t jt_begin, uint32_t jt_end, void *stream);
// resident waves of that lane-group kernel on the current device (0: no such kernel)
uint32_t lanes_resident(int cls, int L);
// Blinded decryption (one pass per prime) of job tiles [jt_begin, jt_end) in
// lane groups of L lanes (a one-lane class: 2 or 4; a lane-group class: twice
// its own), and that kernel's resident waves (kjlanes.hip)
int launch_joint_lanes(const ClassRun &r, int L, uint32_t jt_begin, uint32_t jt_end, void *stream);
uint32_t joint_lanes_resident(int cls, int L);

// Lanes per number for the part of a one-lane class's CRT launch that leaves
// SIMDs idle (L lanes per number give L times the waves, each with a chain
// about L times shorter).  units: job tiles of the launch; resident: waves of its one-lane
// kernel that fit the chip (already capped by the table slots and grid cap);
// simds: SIMDs of the device; room(cls, L): resident waves of the lane-group
// kernel.  A launch under one round runs wholly in lane groups of r.fill_lanes
// lanes, or of the largest smaller power of two that still gives every
// lane-group wave a SIMD of its own; the partial round after full ones runs
// with r.tail_lanes, or the largest smaller power of two whose waves fit one
// round of the lane-group kernel (1: one lane per number, still as a launch of
// its own; r.tail_lanes 0: no launch of its own).  Returns L and sets
// *lane_units to the job tiles of that last part (0: one launch).
inline int lanes_for_launch(const ClassRun &r, uint32_t units, uint32_t resident, uint32_t simds,
                            uint32_t (*room_of)(int, int), uint32_t *lane_units) {
    *lane_units = 0;
    if (resident == 0) return 1;
    const uint32_t rem = units % resident;
    auto fit = [&](int max_l, uint64_t limit) {
        for (int l = max_l; l >= 2; l /= 2) {
            uint64_t room = room_of(r.cls, l);
            if (limit < room) room = limit;
            if ((uint64_t)r.slots_dec * l < room) room = (uint64_t)r.slots_dec * l;  // table room
            if (r.grid_cap && r.grid_cap < room) room = r.grid_cap;
            if ((uint64_t)rem * l <= room) return l;
        }
        return 1;
    };
    int L = 1;
    if (units < resident) {
        L = fit(r.fill_lanes, simds);
        if (L > 1) *lane_units = rem;
    } else if (rem && r.tail_lanes > 0) {
        // the partial round after full ones runs as a launch of its own: its
        // waves then spread over the SIMDs, where the full rounds' last waves
        // would share them
        L = fit(r.tail_lanes, UINT64_MAX);
        *lane_units = rem;
    }
    return L;
}

// The lane-group classes (6144/8192-bit keys, L0 = lanes_half lanes per
// number): a launch of jt job tiles runs with r.fill_lanes = 2 L0 lanes per
// number when every such wave has a SIMD of its own and fits one round of
// that kernel (room: its resident waves) and the table (two such slots per
// slot of the L0 form).
inline bool wide_fill(const ClassRun &r, uint32_t jt, int L0, uint32_t simds, uint32_t room) {
    if (r.fill_lanes != 2 * L0) return false;
    uint64_t lim = simds < room ? simds : room;
    if ((uint64_t)r.slots_dec * 2 < lim) lim = (uint64_t)r.slots_dec * 2;
    if (r.grid_cap && r.grid_cap < lim) lim = r.grid_cap;
    return (uint64_t)jt * (uint64_t)r.fill_lanes <= lim;
}
// compute units of the current device
int device_cus();
// mode: 0 ciphertext blocks, 1 plaintext chunks (range-checked), 2 whole plaintext
// blocks (range-checked); the checks read the packed input at r.x32 (and r.fin32)
int launch_unpack(const ClassRun &r, uint8_t *dst, int mode, void *stream);
// table words needed per wave slot for a class (decryption: at window width win)
uint64_t table_words_per_slot(int cls, int decrypt, int win);
// resident wave slots the persistent kernels of a class use
uint32_t wave_slots(int cls, int decrypt, int num_cus);
// work units (wavefronts' worth of bignums) of the exponentiation kernels
uint32_t exp_units(int cls, int decrypt, uint32_t ntiles);
// persistent batched exponentiation (kbatch.hip)
int launch_batch(const BatchArgs &a, uint32_t grid, void *stream);
int launch_counter_reset(uint32_t *counter, void *stream);
uint32_t batch_wave_slots(int num_cus);
// table words per wave slot of the wide batch kernel
uint64_t batch_slot_words();

// primality testing for key generation (kprime.hip); classes 3..6 (1024..4096-bit keys)
int prime_class_ok(int cls);
uint64_t mr_slot_words(int cls, int win);
uint32_t mr_wave_slots(int cls, int num_cus);
int launch_sieve_class(int cls, const uint32_t *cand, uint32_t count, uint32_t *flags, int device, void *stream);
int launch_mr_class(int cls, const uint32_t *cand, uint32_t count, const uint32_t *bases, int rounds, int win,
                    uint32_t *table, uint64_t slot_words, uint32_t grid, uint32_t *result, void *stream);

}  // namespace pmk
