// Host-side key validation and key-record construction.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pmk.h"
#include "mp_geom.hpp"
#include "pmk_internal.hpp"

namespace pmk {

// Smallest instantiated size class holding a `bits`-bit modulus, or -1.
int class_for_bits(uint32_t bits);

// Checks one key pair (field sizes, N odd with exactly `bits` bits,
// n0inv, rr, odd e >= 3, p > q, p q = N, q qinv = 1 mod p, dp < p, dq < q).
// On failure returns false and puts the reason into *msg.
bool check_key(const pmk_key &k, std::string *msg);

// Writes the Geom(kClassBits[cls]).stride-word record of a checked key.
void build_record(const pmk_key &k, int cls, uint32_t *rec);

// Multi-prime keys: checks (3072 bits with 3 or 4096 bits with 4 primes of
// exactly 1024 bits, product N, pairwise coprime, d_i < p_i) and the
// make_mp_geom(cls).stride-word record (cls 0: 3072 bits, 1: 4096 bits).
bool check_key_mp(const pmk_key_mp &k, std::string *msg);
void build_record_mp(const pmk_key_mp &k, int cls, uint32_t *rec);

}  // namespace pmk
