// Host-side key preparation: validation of one key pair and the per-class key
// record the kernels read (Montgomery constants for the full modulus and for
// each CRT prime).  Plain C++: runs once per key table load, never per chunk.
//
// Constants are derived by modular doubling (x -> 2x mod m), which needs no
// division: R mod m is 1 doubled log2(R) times, R^2 and R^3 follow by doubling
// on, and qinv R mod p is qinv doubled log2(R) times.
#include "keyprep.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>

namespace pmk {

namespace {

using Words = std::vector<uint32_t>;

int bitlen(const Words &x) {
    for (int i = (int)x.size() - 1; i >= 0; --i)
        if (x[i]) return 32 * i + (32 - __builtin_clz(x[i]));
    return 0;
}

int cmp(const Words &a, const Words &b) {
    const size_t n = std::max(a.size(), b.size());
    for (size_t i = n; i-- > 0;) {
        const uint32_t x = i < a.size() ? a[i] : 0u, y = i < b.size() ? b[i] : 0u;
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

// a -= b (a >= b, same length)
void sub_in(Words &a, const Words &b) {
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        int64_t v = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - borrow;
        borrow = v < 0;
        a[i] = (uint32_t)(v + (borrow ? (int64_t)1 << 32 : 0));
    }
}

// x = 2x mod m, for 0 <= x < m (x.size() == m.size())
void mod_double(Words &x, const Words &m) {
    uint32_t carry = 0;
    for (size_t i = 0; i < x.size(); ++i) {
        const uint32_t v = x[i];
        x[i] = (v << 1) | carry;
        carry = v >> 31;
    }
    if (carry || cmp(x, m) >= 0) sub_in(x, m);  // a carry out means 2x >= 2^32k > m
}

// x = x + y mod m, both below m
void mod_add(Words &x, const Words &y, const Words &m) {
    uint64_t c = 0;
    for (size_t i = 0; i < x.size(); ++i) {
        const uint64_t v = (uint64_t)x[i] + y[i] + c;
        x[i] = (uint32_t)v;
        c = v >> 32;
    }
    if (c || cmp(x, m) >= 0) sub_in(x, m);
}

Words mul(const Words &a, const Words &b) {
    Words r(a.size() + b.size(), 0);
    for (size_t i = 0; i < a.size(); ++i) {
        uint64_t c = 0;
        for (size_t j = 0; j < b.size(); ++j) {
            const uint64_t t = (uint64_t)a[i] * b[j] + r[i + j] + c;
            r[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        r[i + b.size()] = (uint32_t)c;
    }
    return r;
}

// a * b mod m by double-and-add over the bits of b (a, b < m)
Words mulmod(const Words &a, const Words &b, const Words &m) {
    Words r(m.size(), 0);
    for (int i = bitlen(b) - 1; i >= 0; --i) {
        mod_double(r, m);
        if ((b[i / 32] >> (i % 32)) & 1u) mod_add(r, a, m);
    }
    return r;
}

Words from(const uint32_t *p, int n, int len) {
    Words w(len, 0);
    for (int i = 0; i < n && i < len; ++i) w[i] = p[i];
    return w;
}

uint32_t inv32(uint32_t a) {  // a odd: a^-1 mod 2^32 by Newton iteration
    uint32_t x = a;            // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}

void to_radix(const Words &x, int lb, int nl, uint32_t *out) {
    const uint32_t mask = (1u << lb) - 1u;
    for (int j = 0; j < nl; ++j) {
        const int bit = lb * j, k = bit / 32, sh = bit % 32;
        const uint64_t lo = k < (int)x.size() ? x[k] : 0u;
        const uint64_t hi = (k + 1) < (int)x.size() ? x[k + 1] : 0u;
        out[j] = (uint32_t)(((hi << 32) | lo) >> sh) & mask;
    }
}

// fills R mod m, R^2 mod m, R^3 mod m (R = 2^(lb*nl)) in radix form
void mont_consts(const Words &m, int lb, int nl, uint32_t *one, uint32_t *rr, uint32_t *rrr) {
    Words x(m.size(), 0);
    x[0] = 1;
    uint32_t *outs[3] = {one, rr, rrr};
    for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < lb * nl; ++i) mod_double(x, m);
        if (outs[k]) to_radix(x, lb, nl, outs[k]);
    }
}

bool is_one(const Words &x) {
    if (x.empty() || x[0] != 1u) return false;
    for (size_t i = 1; i < x.size(); ++i)
        if (x[i]) return false;
    return true;
}

bool is_zero(const Words &x) {
    for (uint32_t v : x)
        if (v) return false;
    return true;
}

void halve(Words &x) {  // x >>= 1
    for (size_t i = 0; i < x.size(); ++i) x[i] = (x[i] >> 1) | (i + 1 < x.size() ? x[i + 1] << 31 : 0u);
}

// x = x / 2 mod m for odd m, 0 <= x < m: (x + m) / 2 when x is odd
void half_mod(Words &x, const Words &m) {
    if (!(x[0] & 1u)) {
        halve(x);
        return;
    }
    uint64_t c = 0;
    for (size_t i = 0; i < x.size(); ++i) {
        const uint64_t v = (uint64_t)x[i] + m[i] + c;
        x[i] = (uint32_t)v;
        c = v >> 32;
    }
    halve(x);
    x.back() |= (uint32_t)c << 31;
}

// x = x - y mod m, both below m
void mod_sub(Words &x, const Words &y, const Words &m) {
    if (cmp(x, y) >= 0) {
        sub_in(x, y);
        return;
    }
    Words d = y;
    sub_in(d, x);  // y - x, below m
    x = m;
    sub_in(x, d);
}

// a^-1 mod m for odd m and 0 < a < m by the binary extended Euclidean
// algorithm (invariants x1 a = u, x2 a = v mod m); false when gcd(a, m) > 1
bool mod_inverse(const Words &a, const Words &m, Words *out) {
    Words u = a, v = m, x1(m.size(), 0), x2(m.size(), 0);
    x1[0] = 1;
    while (!is_one(u) && !is_one(v)) {
        if (is_zero(u)) return false;  // gcd = v > 1
        while (!(u[0] & 1u)) {
            halve(u);
            half_mod(x1, m);
        }
        while (!(v[0] & 1u)) {
            halve(v);
            half_mod(x2, m);
        }
        if (cmp(u, v) >= 0) {
            sub_in(u, v);
            mod_sub(x1, x2, m);
        } else {
            sub_in(v, u);
            mod_sub(x2, x1, m);
        }
    }
    *out = is_one(u) ? x1 : x2;
    return true;
}

bool fail(std::string *msg, const char *what) {
    if (msg) *msg = what;
    return false;
}

}  // namespace

int class_for_bits(uint32_t bits) {
    for (int c = 0; c <= kMaxClass; ++c)
        if ((int)bits <= kClassBits[c]) return c;
    return -1;
}

bool check_key(const pmk_key &k, std::string *msg) {
    if (k.bits < 128 || k.bits > 8192 || k.bits % 64) return fail(msg, "bits must be a multiple of 64 in 128..8192");
    if (!k.n || !k.rr || !k.e || !k.p || !k.q || !k.dp || !k.dq || !k.qinv) return fail(msg, "null key field");
    const int S = k.bits / 32, SH = k.bits / 64;
    const Words n = from(k.n, S, S);
    if (!(n[0] & 1u)) return fail(msg, "modulus must be odd");
    if (bitlen(n) != (int)k.bits) return fail(msg, "modulus must have exactly `bits` bits");
    if ((uint32_t)(n[0] * k.n0inv) != 0xFFFFFFFFu) return fail(msg, "n0inv is not -N^-1 mod 2^32");
    {
        // R^2 mod N with R = 2^bits: 2^(bits-1) < N doubled bits+1 times
        Words x(S, 0);
        x[(k.bits - 1) / 32] = 1u << ((k.bits - 1) % 32);
        for (uint32_t i = 0; i < k.bits + 1; ++i) mod_double(x, n);
        if (cmp(x, from(k.rr, S, S)) != 0) return fail(msg, "rr is not R^2 mod N (R = 2^bits)");
    }
    if (k.e_limbs < 1 || k.e_limbs > 2) return fail(msg, "public exponent must have 1 or 2 limbs");
    const Words e = from(k.e, k.e_limbs, 2);
    if (!(e[0] & 1u) || bitlen(e) < 2) return fail(msg, "public exponent must be odd and at least 3");
    const Words p = from(k.p, SH, SH), q = from(k.q, SH, SH);
    if (!(p[0] & 1u) || !(q[0] & 1u)) return fail(msg, "primes must be odd");
    if (cmp(p, q) <= 0) return fail(msg, "p must be greater than q");
    if (cmp(mul(p, q), n) != 0) return fail(msg, "p * q != N");
    const Words qinv = from(k.qinv, SH, SH);
    if (cmp(qinv, p) >= 0) return fail(msg, "qinv must be below p");
    {
        Words qr = q;
        if (cmp(qr, p) >= 0) sub_in(qr, p);
        const Words one = mulmod(qinv, qr, p);
        Words unit(SH, 0);
        unit[0] = 1;
        if (cmp(one, unit) != 0) return fail(msg, "q * qinv != 1 mod p");
    }
    if (cmp(from(k.dp, SH, SH), p) >= 0 || cmp(from(k.dq, SH, SH), q) >= 0)
        return fail(msg, "dp / dq must be below p / q");
    return true;
}

void build_record(const pmk_key &k, int cls, uint32_t *rec) {
    const Geom g = make_geom(kClassBits[cls]);
    std::memset(rec, 0, sizeof(uint32_t) * g.stride);
    const int S = k.bits / 32, SH = k.bits / 64;
    const Words n = from(k.n, S, g.S);
    for (int i = 0; i < g.S; ++i) rec[g.off_n32 + i] = n[i];
    to_radix(n, g.lbf, g.nlf, rec + g.off_nf);
    rec[g.off_n0f] = (0u - inv32(n[0])) & ((1u << g.lbf) - 1u);
    mont_consts(n, g.lbf, g.nlf, rec + g.off_onef, rec + g.off_rrf, rec + g.off_rrrf);
    const Words e = from(k.e, k.e_limbs, 2);
    rec[g.off_e] = e[0];
    rec[g.off_e + 1] = e[1];
    rec[g.off_ebits] = (uint32_t)bitlen(e);
    rec[g.off_kbytes] = k.bits / 8;
    const uint32_t *primes[2] = {k.p, k.q}, *exps[2] = {k.dp, k.dq};
    for (int h = 0; h < 2; ++h) {
        uint32_t *hr = rec + g.off_half[h];
        const Words m = from(primes[h], SH, g.SH);
        to_radix(m, g.lbh, g.nlh, hr + g.h_m);
        hr[g.h_m0] = (0u - inv32(m[0])) & ((1u << g.lbh) - 1u);
        mont_consts(m, g.lbh, g.nlh, hr + g.h_one, hr + g.h_rr, hr + g.h_rrr);
        if (g.nla != g.nlh) mont_consts(m, g.lbh, g.nla, hr + g.h_onea, hr + g.h_rra, hr + g.h_rrra);
        if (g.nla8 != g.nla) mont_consts(m, g.lbh, g.nla8, hr + g.h_onea8, hr + g.h_rra8, hr + g.h_rrra8);
        const Words d = from(exps[h], SH, g.SH);
        for (int i = 0; i < g.SH; ++i) hr[g.h_d + i] = d[i];
        // d2 = m - 1 - d: (c^d)^-1 = c^d2 mod m for c not divisible by m (Fermat)
        Words d2 = m;
        d2[0] -= 1;  // m is odd, so no borrow
        sub_in(d2, d);
        for (int i = 0; i < g.SH; ++i) hr[g.h_d2 + i] = d2[i];
    }
    {
        const Words p = from(k.p, SH, g.SH);
        Words x = from(k.qinv, SH, g.SH);
        for (int i = 0; i < g.lbh * g.nlh; ++i) mod_double(x, p);
        to_radix(x, g.lbh, g.nlh, rec + g.off_qinvr);
    }
}

bool check_key_mp(const pmk_key_mp &k, std::string *msg) {
    if (k.bits != 3072 && k.bits != 4096) return fail(msg, "multi-prime keys must have 3072 or 4096 bits");
    if (k.nprimes != k.bits / 1024) return fail(msg, "nprimes must be bits / 1024 (primes of 1024 bits)");
    if (!k.n || !k.primes || !k.d) return fail(msg, "null key field");
    const int S = k.bits / 32, P = (int)k.nprimes;
    const Words n = from(k.n, S, S);
    if (!(n[0] & 1u)) return fail(msg, "modulus must be odd");
    if (bitlen(n) != (int)k.bits) return fail(msg, "modulus must have exactly `bits` bits");
    std::vector<Words> p(P);
    Words prod(1, 1u);
    for (int i = 0; i < P; ++i) {
        p[i] = from(k.primes + 32 * i, 32, 32);
        if (!(p[i][0] & 1u) || bitlen(p[i]) != 1024) return fail(msg, "every prime must be odd with exactly 1024 bits");
        if (cmp(from(k.d + 32 * i, 32, 32), p[i]) >= 0) return fail(msg, "d_i must be below p_i");
        prod = mul(prod, p[i]);
    }
    if (cmp(prod, n) != 0) return fail(msg, "the product of the primes is not N");
    for (int i = 1; i < P; ++i)
        for (int j = 0; j < i; ++j) {
            Words a = p[j], inv;
            if (cmp(a, p[i]) >= 0) sub_in(a, p[i]);  // p_j < 2 p_i
            if (!mod_inverse(a, p[i], &inv)) return fail(msg, "primes must be pairwise coprime");
            Words unit(32, 0);
            unit[0] = 1;
            if (cmp(mulmod(inv, a, p[i]), unit) != 0) return fail(msg, "prime inverse check failed");
        }
    return true;
}

void build_record_mp(const pmk_key_mp &k, int cls, uint32_t *rec) {
    const MpGeom g = make_mp_geom(cls);
    std::memset(rec, 0, sizeof(uint32_t) * g.stride);
    const Words n = from(k.n, g.S, g.S);
    for (int i = 0; i < g.S; ++i) rec[g.off_n32 + i] = n[i];
    rec[g.off_kbytes] = k.bits / 8;
    constexpr int PL = pad4(kMpNL), RB = kMpLB * kMpNL;  // R = 2^RB
    for (int i = 0; i < g.parts; ++i) {
        uint32_t *qr = rec + g.off_part[i];
        const Words m = from(k.primes + 32 * i, 32, 32);
        to_radix(m, kMpLB, kMpNL, qr + g.q_m);
        qr[g.q_m0] = (0u - inv32(m[0])) & ((1u << kMpLB) - 1u);
        Words x(32, 0);
        x[0] = 1;
        for (int r = 1; r <= g.parts + 1; ++r) {  // R^r mod p
            for (int b = 0; b < RB; ++b) mod_double(x, m);
            if (r == 1) to_radix(x, kMpLB, kMpNL, qr + g.q_one);
            else to_radix(x, kMpLB, kMpNL, qr + g.q_rpow + (r - 2) * PL);
        }
        for (int w = 0; w < 32; ++w) qr[g.q_d + w] = k.d[32 * i + w];
        for (int j = 0; j < i; ++j) {
            Words a = from(k.primes + 32 * j, 32, 32), inv;
            if (cmp(a, m) >= 0) sub_in(a, m);
            mod_inverse(a, m, &inv);  // checked by check_key_mp
            for (int b = 0; b < RB; ++b) mod_double(inv, m);
            to_radix(inv, kMpLB, kMpNL, qr + g.q_cinv + j * PL);
        }
    }
}

}  // namespace pmk
