/*
 * oracle.c -- plain, slow, CPU reference of the PMKRSA per-chunk arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test-suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark.  The product library
 * (the HIP path) never includes, links or calls it, and it shares no header,
 * helper, table or constant with that library.
 *
 * What it computes (paper: "A Variant RSA Acceleration with Parallelization",
 * arXiv 2111.11924):
 *   - chunking of a message into one integer per chunk, one key pair per chunk
 *     (Sec. 3.1, the plaintext vector reshaped so that each row uses its own
 *     key pair);
 *   - textbook RSA encryption c = m^e mod N (Sec. 1.1, step 2; Algorithm 1,
 *     Encryption procedure without blinding);
 *   - textbook RSA decryption m = c^d mod N (Sec. 1.1, step 3);
 *   - CRT-RSA decryption (Sec. 2.1, equation CRT-RSA);
 *   - the blinded PMKRSA forms c* = (r m)^e, c_R = r^e and
 *     m = (c*)^d (c_R^d)^-1 mod N (Sec. 3.1, Eqs. 3-10, Algorithm 1).
 *
 * How: little-endian base-2^32 limbs; schoolbook multiplication; remainders by
 * Knuth's Algorithm D (TAOCP vol. 2, Sec. 4.3.1); modular exponentiation
 * y = x^e mod N (the operation Algorithm 2 computes) written from that
 * definition as left-to-right square-and-multiply over the bits of e.  No
 * Montgomery arithmetic, no windows, no lane tricks.  Inputs longer than the
 * fixed limb capacity are refused with an error, never truncated.
 *
 * Readings of the paper taken here (each one listed in the design notes):
 *   - a chunk is the big-endian integer of (modulus bytes - 4) message bytes,
 *     the last chunk the big-endian integer of the remaining bytes; so every
 *     chunk lies in Z_N;
 *   - the CRT equations are read with exponents d_p, d_q (the printed text
 *     shows d) and m_1, m_2 read as m_p, m_q; the ciphertext is reduced mod p
 *     and mod q first; h is taken as the non-negative residue;
 *   - ciphertext blocks are (modulus bytes) big-endian bytes each.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 520 /* limbs: holds the product of two 8192-bit numbers, plus slack */

typedef struct {
    uint32_t v[OR_MAXL];
    int len; /* number of limbs in use; v[len-1] != 0 unless len == 0 (the value 0) */
} bn;

/* ---------- basic helpers ---------------------------------------------------------- */

static void bn_norm(bn *a) {
    while (a->len > 0 && a->v[a->len - 1] == 0) a->len--;
}

static void bn_zero(bn *a) { a->len = 0; }

static void bn_set_u32(bn *a, uint32_t x) {
    a->v[0] = x;
    a->len = 1;
    bn_norm(a);
}

static void bn_copy(bn *dst, const bn *src) {
    dst->len = src->len;
    memcpy(dst->v, src->v, sizeof(uint32_t) * (size_t)src->len);
}

/* returns -1 (and leaves a = 0) when the value needs more than OR_MAXL limbs */
static int bn_from_limbs(bn *a, const uint32_t *limbs, int n) {
    while (n > 0 && limbs[n - 1] == 0) n--;
    if (n > OR_MAXL) {
        bn_zero(a);
        return -1;
    }
    memcpy(a->v, limbs, sizeof(uint32_t) * (size_t)n);
    a->len = n;
    return 0;
}

/* writes exactly n limbs (zero-padded); returns -1 if the value does not fit */
static int bn_to_limbs(const bn *a, uint32_t *limbs, int n) {
    if (a->len > n) return -1;
    for (int i = 0; i < n; i++) limbs[i] = i < a->len ? a->v[i] : 0;
    return 0;
}

static int bn_cmp(const bn *a, const bn *b) {
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    for (int i = a->len - 1; i >= 0; i--)
        if (a->v[i] != b->v[i]) return a->v[i] < b->v[i] ? -1 : 1;
    return 0;
}

/* r = a + b */
static void bn_add(bn *r, const bn *a, const bn *b) {
    int n = a->len > b->len ? a->len : b->len;
    if (n + 1 > OR_MAXL) abort(); /* callers stay within capacity; overflowing it is a bug */
    uint64_t carry = 0;
    for (int i = 0; i < n; i++) {
        uint64_t s = carry;
        if (i < a->len) s += a->v[i];
        if (i < b->len) s += b->v[i];
        r->v[i] = (uint32_t)s;
        carry = s >> 32;
    }
    r->v[n] = (uint32_t)carry;
    r->len = n + 1;
    bn_norm(r);
}

/* r = a - b, requires a >= b */
static void bn_sub(bn *r, const bn *a, const bn *b) {
    int64_t borrow = 0;
    for (int i = 0; i < a->len; i++) {
        int64_t s = (int64_t)a->v[i] - borrow - (i < b->len ? (int64_t)b->v[i] : 0);
        borrow = 0;
        if (s < 0) {
            s += (int64_t)1 << 32;
            borrow = 1;
        }
        r->v[i] = (uint32_t)s;
    }
    r->len = a->len;
    bn_norm(r);
}

/* r = a * b, schoolbook; r must not alias a or b */
static void bn_mul(bn *r, const bn *a, const bn *b) {
    if (a->len == 0 || b->len == 0) {
        bn_zero(r);
        return;
    }
    int n = a->len + b->len;
    if (n > OR_MAXL) abort(); /* entry points bound their operands; overflowing is a bug */
    for (int i = 0; i < n; i++) r->v[i] = 0;
    for (int i = 0; i < a->len; i++) {
        uint64_t carry = 0;
        for (int j = 0; j < b->len; j++) {
            uint64_t t = (uint64_t)a->v[i] * b->v[j] + r->v[i + j] + carry;
            r->v[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        r->v[i + b->len] = (uint32_t)carry;
    }
    r->len = n;
    bn_norm(r);
}

static int clz32(uint32_t x) {
    int n = 0;
    if (x == 0) return 32;
    while (!(x & 0x80000000u)) {
        x <<= 1;
        n++;
    }
    return n;
}

/*
 * q = u / v, rem = u mod v (either output may be NULL).  Knuth, TAOCP vol. 2,
 * Sec. 4.3.1, Algorithm D: normalise so the divisor's top limb has its top bit
 * set, estimate each quotient limb from the top two limbs of the running
 * remainder, correct the estimate with the divisor's second limb, multiply and
 * subtract, add back on the rare over-estimate.  A one-limb divisor uses plain
 * short division.  Returns -1 on division by zero.
 */
static int bn_divmod(bn *q, bn *rem, const bn *u, const bn *v) {
    if (v->len == 0) return -1;
    if (bn_cmp(u, v) < 0) {
        if (rem && rem != u) bn_copy(rem, u);
        if (q) bn_zero(q);
        return 0;
    }
    int n = v->len, m = u->len - v->len;
    if (n == 1) {
        uint64_t r = 0;
        bn qq;
        for (int i = u->len - 1; i >= 0; i--) {
            uint64_t cur = (r << 32) | u->v[i];
            qq.v[i] = (uint32_t)(cur / v->v[0]);
            r = cur % v->v[0];
        }
        qq.len = u->len;
        bn_norm(&qq);
        if (q) bn_copy(q, &qq);
        if (rem) bn_set_u32(rem, (uint32_t)r);
        return 0;
    }
    /* D1: normalise */
    static const uint64_t B = (uint64_t)1 << 32;
    int s = clz32(v->v[n - 1]);
    uint32_t vn[OR_MAXL], un[OR_MAXL + 1];
    for (int i = n - 1; i > 0; i--)
        vn[i] = s ? (v->v[i] << s) | (v->v[i - 1] >> (32 - s)) : v->v[i];
    vn[0] = v->v[0] << s;
    un[m + n] = s ? u->v[m + n - 1] >> (32 - s) : 0;
    for (int i = m + n - 1; i > 0; i--)
        un[i] = s ? (u->v[i] << s) | (u->v[i - 1] >> (32 - s)) : u->v[i];
    un[0] = u->v[0] << s;

    bn qq;
    /* D2..D7: one quotient limb per step, most significant first */
    for (int j = m; j >= 0; j--) {
        /* D3: estimate qhat from the top two limbs, then refine with vn[n-2] */
        uint64_t top = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
        uint64_t qhat = top / vn[n - 1];
        uint64_t rhat = top % vn[n - 1];
        while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
            qhat--;
            rhat += vn[n - 1];
            if (rhat >= B) break;
        }
        /* D4: multiply and subtract qhat * vn from un[j .. j+n] */
        int64_t borrow = 0;
        uint64_t carry = 0;
        for (int i = 0; i < n; i++) {
            uint64_t p = qhat * vn[i] + carry;
            carry = p >> 32;
            int64_t t = (int64_t)un[i + j] - borrow - (int64_t)(p & 0xFFFFFFFFu);
            borrow = 0;
            if (t < 0) {
                t += (int64_t)B;
                borrow = 1;
            }
            un[i + j] = (uint32_t)t;
        }
        int64_t t = (int64_t)un[j + n] - borrow - (int64_t)carry;
        int negative = t < 0;
        un[j + n] = (uint32_t)(negative ? t + (int64_t)B : t);
        /* D5/D6: the estimate was one too large -- add the divisor back */
        if (negative) {
            qhat--;
            uint64_t c = 0;
            for (int i = 0; i < n; i++) {
                uint64_t s2 = (uint64_t)un[i + j] + vn[i] + c;
                un[i + j] = (uint32_t)s2;
                c = s2 >> 32;
            }
            un[j + n] = (uint32_t)((uint64_t)un[j + n] + c);
        }
        qq.v[j] = (uint32_t)qhat;
    }
    qq.len = m + 1;
    bn_norm(&qq);
    if (q) bn_copy(q, &qq);
    /* D8: unnormalise the remainder */
    if (rem) {
        for (int i = 0; i < n; i++)
            rem->v[i] = s ? (un[i] >> s) | (un[i + 1] << (32 - s)) : un[i];
        rem->len = n;
        bn_norm(rem);
    }
    return 0;
}

/* r = a mod m */
static void bn_mod(bn *r, const bn *a, const bn *m) { bn_divmod(NULL, r, a, m); }

/* r = a * b mod m (r may alias a or b) */
static void bn_mulmod(bn *r, const bn *a, const bn *b, const bn *m) {
    bn t;
    bn_mul(&t, a, b);
    bn_mod(r, &t, m);
}

static int bn_bit(const bn *a, int i) {
    int limb = i / 32;
    if (limb >= a->len) return 0;
    return (a->v[limb] >> (i % 32)) & 1;
}

static int bn_bitlen(const bn *a) {
    if (a->len == 0) return 0;
    return 32 * (a->len - 1) + (32 - clz32(a->v[a->len - 1]));
}

/*
 * y = x^e mod N, the operation of Algorithm 2 (binary exponentiation), written
 * from its definition: with e = sum_i e_i 2^i, scan the bits from the top one
 * down; before bit i is taken in, y = x^(e >> (i+1)) mod N, so squaring y and
 * multiplying by x where e_i = 1 gives x^(e >> i) mod N.  After bit 0,
 * y = x^e mod N.  e = 0 gives 1 mod N (the empty product); N must be non-zero,
 * and N = 1 gives 0.
 */
static void bn_modexp(bn *y, const bn *x_in, const bn *e, const bn *N) {
    bn one, x;
    bn_set_u32(&one, 1);
    bn_mod(y, &one, N);
    bn_mod(&x, x_in, N);
    for (int i = bn_bitlen(e) - 1; i >= 0; i--) {
        bn_mulmod(y, y, y, N);
        if (bn_bit(e, i)) bn_mulmod(y, y, &x, N);
    }
}

/* ---------- byte <-> integer -------------------------------------------------------- */

static void bn_from_be(bn *a, const uint8_t *bytes, size_t len) {
    int nl = (int)((len + 3) / 4);
    for (int i = 0; i < nl; i++) a->v[i] = 0;
    for (size_t k = 0; k < len; k++) {
        size_t pos = len - 1 - k; /* byte k from the end has weight 256^k */
        a->v[k / 4] |= (uint32_t)bytes[pos] << (8 * (k % 4));
    }
    a->len = nl;
    bn_norm(a);
}

/* writes exactly len bytes, big-endian, left-padded with zeros; -1 if too large */
static int bn_to_be(const bn *a, uint8_t *bytes, size_t len) {
    if ((size_t)bn_bitlen(a) > 8 * len) return -1;
    for (size_t k = 0; k < len; k++) {
        size_t limb = k / 4;
        uint32_t w = limb < (size_t)a->len ? a->v[limb] : 0;
        bytes[len - 1 - k] = (uint8_t)(w >> (8 * (k % 4)));
    }
    return 0;
}

/* ---------- keys and chunks ---------------------------------------------------------- */

/*
 * One RSA key pair (Sec. 1.1 step 1; Algorithm 1, Initialization).  Every field
 * is a little-endian base-2^32 limb array with its own length.
 */
typedef struct {
    int32_t bits; /* modulus length; modulus bytes kb = bits / 8 */
    const uint32_t *n;    int32_t n_len;
    const uint32_t *e;    int32_t e_len;
    const uint32_t *d;    int32_t d_len;
    const uint32_t *p;    int32_t p_len;
    const uint32_t *q;    int32_t q_len;
    const uint32_t *dp;   int32_t dp_len;
    const uint32_t *dq;   int32_t dq_len;
    const uint32_t *qinv; int32_t qinv_len;
} oracle_key;

/*
 * Chunk layout (Sec. 3.1: the message split into chunks m_1..m_k, chunk i under
 * its own key).  Chunk i carries kb_i - 4 message bytes, kb_i = bits/8 of its
 * key; the last chunk carries what remains.  Ciphertext block i has kb_i bytes.
 * Fills msg_off/msg_len/ct_off for each chunk and returns the ciphertext
 * length, or -1 when nchunks is not the exact number of chunks the message
 * needs or a key index is out of range.
 */
long long oracle_plan(const oracle_key *keys, int nkeys, const uint32_t *key_map,
                      long long nchunks, long long msg_len, long long *msg_off,
                      long long *chunk_len, long long *ct_off) {
    long long off = 0, ct = 0;
    if (msg_len == 0) return nchunks == 0 ? 0 : -1;
    for (long long i = 0; i < nchunks; i++) {
        if (key_map[i] >= (uint32_t)nkeys) return -1;
        long long cap = keys[key_map[i]].bits / 8 - 4;
        long long left = msg_len - off;
        if (left <= 0) return -1; /* more chunks than the message needs */
        long long len = left < cap ? left : cap;
        if (i == nchunks - 1 && left > cap) return -1; /* too few chunks */
        msg_off[i] = off;
        chunk_len[i] = len;
        ct_off[i] = ct;
        off += len;
        ct += keys[key_map[i]].bits / 8;
    }
    return ct;
}

static void key_part(bn *out, const uint32_t *limbs, int len) { bn_from_limbs(out, limbs, len); }

/* number of limbs of a limb array once its zero top limbs are dropped */
static int used_limbs(const uint32_t *limbs, int n) {
    while (n > 0 && limbs[n - 1] == 0) n--;
    return n;
}

/* every field of a key fits half the limb capacity, so that a product of two
 * residues (and every intermediate of the routines below) fits the capacity */
static int key_ok(const oracle_key *k) {
    const int half = OR_MAXL / 2;
    return used_limbs(k->n, k->n_len) <= half && used_limbs(k->e, k->e_len) <= half &&
           used_limbs(k->d, k->d_len) <= half && used_limbs(k->p, k->p_len) <= half &&
           used_limbs(k->q, k->q_len) <= half && used_limbs(k->dp, k->dp_len) <= half &&
           used_limbs(k->dq, k->dq_len) <= half && used_limbs(k->qinv, k->qinv_len) <= half &&
           k->bits > 0 && k->bits <= 32 * half;
}

static int keys_ok(const oracle_key *keys, int nkeys) {
    for (int i = 0; i < nkeys; i++)
        if (!key_ok(&keys[i])) return 0;
    return 1;
}

/* Sec. 1.1 step 2 / Algorithm 1 (Encryption without blinding): c = m^e mod N */
static void rsa_encrypt_int(bn *c, const bn *m, const oracle_key *k) {
    bn N, e;
    key_part(&N, k->n, k->n_len);
    key_part(&e, k->e, k->e_len);
    bn_modexp(c, m, &e, &N);
}

/* Sec. 1.1 step 3: m = c^d mod N (no CRT) */
static void rsa_decrypt_plain_int(bn *m, const bn *c, const oracle_key *k) {
    bn N, d;
    key_part(&N, k->n, k->n_len);
    key_part(&d, k->d, k->d_len);
    bn_modexp(m, c, &d, &N);
}

/*
 * Sec. 2.1, equation CRT-RSA: m_p = c^{d_p} mod p, m_q = c^{d_q} mod q,
 * h = q^{-1} (m_p - m_q) mod p, m = m_q + h q.  c is reduced mod p and mod q
 * before exponentiating; (m_p - m_q) is brought into [0, p) before the product.
 */
static void rsa_decrypt_crt_int(bn *m, const bn *c, const oracle_key *k) {
    bn p, q, dp, dq, qinv, cp, cq, mp, mq, mq_modp, diff, h, hq;
    key_part(&p, k->p, k->p_len);
    key_part(&q, k->q, k->q_len);
    key_part(&dp, k->dp, k->dp_len);
    key_part(&dq, k->dq, k->dq_len);
    key_part(&qinv, k->qinv, k->qinv_len);
    bn_mod(&cp, c, &p);
    bn_mod(&cq, c, &q);
    bn_modexp(&mp, &cp, &dp, &p);
    bn_modexp(&mq, &cq, &dq, &q);
    bn_mod(&mq_modp, &mq, &p);
    if (bn_cmp(&mp, &mq_modp) >= 0) {
        bn_sub(&diff, &mp, &mq_modp);
    } else {
        bn t;
        bn_add(&t, &mp, &p);
        bn_sub(&diff, &t, &mq_modp);
    }
    bn_mulmod(&h, &qinv, &diff, &p);
    bn_mul(&hq, &h, &q);
    bn_add(m, &mq, &hq);
}

/* ---------- exported primitives (for pinning the oracle against Python integers) ---- */

/* r (rn limbs) = a * b; returns -1 if rn is too small, -2 if the product exceeds the capacity */
int oracle_mul(const uint32_t *a, int an, const uint32_t *b, int bn_, uint32_t *r, int rn) {
    bn A, Bv, R;
    if (bn_from_limbs(&A, a, an) != 0 || bn_from_limbs(&Bv, b, bn_) != 0) return -2;
    if (A.len + Bv.len > OR_MAXL) return -2;
    bn_mul(&R, &A, &Bv);
    return bn_to_limbs(&R, r, rn);
}

/* q (qn limbs) = u / v, r (rn limbs) = u mod v; -1 for v = 0 or short outputs, -2 for an
 * operand beyond the capacity */
int oracle_divmod(const uint32_t *u, int un, const uint32_t *v, int vn, uint32_t *q, int qn,
                  uint32_t *r, int rn) {
    bn U, V, Q, R;
    if (bn_from_limbs(&U, u, un) != 0 || bn_from_limbs(&V, v, vn) != 0) return -2;
    if (bn_divmod(&Q, &R, &U, &V) != 0) return -1;
    if (bn_to_limbs(&Q, q, qn) != 0) return -1;
    return bn_to_limbs(&R, r, rn);
}

/* y (yn limbs) = x^e mod m (the operation of Algorithm 2); -1 for m = 0 or a short output,
 * -2 for operands beyond the capacity (m may have at most half of it) */
int oracle_modexp(const uint32_t *x, int xn, const uint32_t *e, int en, const uint32_t *m, int mn,
                  uint32_t *y, int yn) {
    bn X, E, M, Y;
    if (bn_from_limbs(&X, x, xn) != 0 || bn_from_limbs(&E, e, en) != 0 || bn_from_limbs(&M, m, mn) != 0)
        return -2;
    if (M.len > OR_MAXL / 2) return -2;
    if (M.len == 0) return -1;
    bn_modexp(&Y, &X, &E, &M);
    return bn_to_limbs(&Y, y, yn);
}

/* ---------- whole-message operations ------------------------------------------------- */

/*
 * Encrypt a message chunk by chunk (Algorithm 1, Encryption; the loop over
 * chunks is the one the paper marks as parallel).  ct must hold the ciphertext
 * length returned by oracle_plan.  Returns 0, or -1 on a bad plan or a key
 * beyond the capacity.
 */
int oracle_encrypt(const oracle_key *keys, int nkeys, const uint8_t *msg, long long msg_len,
                   const uint32_t *key_map, long long nchunks, uint8_t *ct) {
    long long *off = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long *len = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long *cto = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long total = keys_ok(keys, nkeys) ? oracle_plan(keys, nkeys, key_map, nchunks, msg_len, off, len, cto) : -1;
    int status = total < 0 ? -1 : 0;
    if (status == 0) {
#pragma omp parallel for schedule(dynamic, 4)
        for (long long i = 0; i < nchunks; i++) {
            const oracle_key *k = &keys[key_map[i]];
            bn m, c;
            bn_from_be(&m, msg + off[i], (size_t)len[i]);
            rsa_encrypt_int(&c, &m, k);
            bn_to_be(&c, ct + cto[i], (size_t)(k->bits / 8));
        }
    }
    free(off);
    free(len);
    free(cto);
    return status;
}

/*
 * Decrypt a ciphertext made by oracle_encrypt back into msg_len message bytes.
 * use_crt = 1 takes the CRT route, 0 the plain c^d route.  Returns 0; -1 on a
 * bad plan; -3 when some ciphertext block is not below its modulus (that
 * chunk's output bytes are then left as zeros).
 */
int oracle_decrypt(const oracle_key *keys, int nkeys, const uint8_t *ct, long long msg_len,
                   const uint32_t *key_map, long long nchunks, uint8_t *msg, int use_crt) {
    long long *off = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long *len = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long *cto = malloc(sizeof(long long) * (size_t)(nchunks + 1));
    long long total = keys_ok(keys, nkeys) ? oracle_plan(keys, nkeys, key_map, nchunks, msg_len, off, len, cto) : -1;
    int status = total < 0 ? -1 : 0;
    int range_err = 0;
    if (status == 0) {
#pragma omp parallel for schedule(dynamic, 4) reduction(| : range_err)
        for (long long i = 0; i < nchunks; i++) {
            const oracle_key *k = &keys[key_map[i]];
            bn c, m, N;
            bn_from_be(&c, ct + cto[i], (size_t)(k->bits / 8));
            key_part(&N, k->n, k->n_len);
            if (bn_cmp(&c, &N) >= 0) {
                memset(msg + off[i], 0, (size_t)len[i]);
                range_err |= 1;
                continue;
            }
            if (use_crt)
                rsa_decrypt_crt_int(&m, &c, k);
            else
                rsa_decrypt_plain_int(&m, &c, k);
            if (bn_to_be(&m, msg + off[i], (size_t)len[i]) != 0) {
                /* a plaintext wider than its chunk: not a ciphertext of this scheme */
                memset(msg + off[i], 0, (size_t)len[i]);
                range_err |= 1;
            }
        }
    }
    free(off);
    free(len);
    free(cto);
    if (status == 0 && range_err) status = -3;
    return status;
}

/*
 * Single-chunk forms on limb arrays, for tests that work on integers directly.
 * mode 0: c = m^e mod N; 1: m = c^d mod N; 2: CRT decryption.
 * out receives out_len limbs.  -2: a key field or x beyond the capacity.
 */
int oracle_rsa_int(const oracle_key *k, int mode, const uint32_t *x, int xn, uint32_t *out,
                   int out_len) {
    bn X, Y;
    if (!key_ok(k) || bn_from_limbs(&X, x, xn) != 0) return -2;
    if (mode == 0)
        rsa_encrypt_int(&Y, &X, k);
    else if (mode == 1)
        rsa_decrypt_plain_int(&Y, &X, k);
    else if (mode == 2)
        rsa_decrypt_crt_int(&Y, &X, k);
    else
        return -1;
    return bn_to_limbs(&Y, out, out_len);
}

/*
 * PMKRSA blinding (Sec. 3.1, Eqs. 3-10; Algorithm 1).  Per chunk, with r drawn
 * by the caller from [1, N) and coprime to N:
 *   encryption:  c* = (r m)^e mod N  (= m^e r^e mod N),   c_R = r^e mod N;
 *   decryption:  r' = c_R^d mod N,   m'* = (c*)^d mod N,   m = m'* r'^-1 mod N.
 * The inverse r'^-1 is found by the extended Euclidean algorithm on integers.
 * mode 0 (encrypt): x = m, aux = r  ->  out = c*, out2 = c_R.
 * mode 1 (decrypt): x = c*, aux = c_R -> out = m, out2 = r'.
 * Returns -2 when r' is not invertible mod N, -3 for a key field or an input
 * beyond the capacity.
 */
static int bn_modinv(bn *inv, const bn *a, const bn *N);

int oracle_blind_int(const oracle_key *k, int mode, const uint32_t *x, int xn, const uint32_t *aux,
                     int auxn, uint32_t *out, uint32_t *out2, int out_len) {
    bn X, A, N, e, d, t, y, y2;
    if (!key_ok(k) || bn_from_limbs(&X, x, xn) != 0 || bn_from_limbs(&A, aux, auxn) != 0) return -3;
    key_part(&N, k->n, k->n_len);
    key_part(&e, k->e, k->e_len);
    key_part(&d, k->d, k->d_len);
    if (N.len == 0) return -1;
    if (mode == 0) {
        bn ra, rx; /* r m mod N from the reduced factors */
        bn_mod(&ra, &A, &N);
        bn_mod(&rx, &X, &N);
        bn_mulmod(&t, &ra, &rx, &N);
        bn_modexp(&y, &t, &e, &N);
        bn_modexp(&y2, &A, &e, &N);
    } else if (mode == 1) {
        bn rinv, ms;
        bn_modexp(&y2, &A, &d, &N);
        bn_modexp(&ms, &X, &d, &N);
        if (bn_modinv(&rinv, &y2, &N) != 0) return -2;
        bn_mulmod(&y, &ms, &rinv, &N);
    } else {
        return -1;
    }
    if (bn_to_limbs(&y, out, out_len) != 0) return -1;
    return bn_to_limbs(&y2, out2, out_len);
}

/*
 * inv = a^-1 mod N by the extended Euclidean algorithm, tracking the Bezout
 * coefficient of a modulo N so that every quantity stays non-negative.
 * Returns -1 when gcd(a, N) != 1.
 */
static int bn_modinv(bn *inv, const bn *a, const bn *N) {
    bn r0, r1, s0, s1, qq, rr, tmp, prod;
    bn_copy(&r0, N);
    bn_mod(&r1, a, N);
    bn_zero(&s0);       /* coefficient of a in r0, mod N */
    bn_set_u32(&s1, 1); /* coefficient of a in r1, mod N */
    while (r1.len != 0) {
        bn_divmod(&qq, &rr, &r0, &r1);
        /* s_new = s0 - qq*s1 mod N */
        bn_mulmod(&prod, &qq, &s1, N);
        if (bn_cmp(&s0, &prod) >= 0) {
            bn_sub(&tmp, &s0, &prod);
        } else {
            bn t2;
            bn_add(&t2, &s0, N);
            bn_sub(&tmp, &t2, &prod);
        }
        bn_copy(&r0, &r1);
        bn_copy(&r1, &rr);
        bn_copy(&s0, &s1);
        bn_copy(&s1, &tmp);
    }
    bn one;
    bn_set_u32(&one, 1);
    if (bn_cmp(&r0, &one) != 0) return -1;
    bn_copy(inv, &s0);
    return 0;
}

/* number of OpenMP threads a parallel region uses (1 without OpenMP) */
#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n); }
#else
int oracle_threads(void) { return 1; }
void oracle_set_threads(int n) { (void)n; }
#endif
