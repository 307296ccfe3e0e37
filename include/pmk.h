/*
 * pmk.h -- C ABI of the PMKRSA batched modular-exponentiation library (MI355X, gfx950).
 *
 * The library runs the data-parallel part of the parallelised multi-key RSA
 * scheme of "A Variant RSA Acceleration with Parallelization" (arXiv
 * 2111.11924): a message is split into chunks, chunk i is encrypted under its
 * own key pair (Sec. 3.1 and Algorithm 1), with c = m^e mod N (Sec. 1.1, step 2)
 * and decrypted with the private exponent through the Chinese Remainder
 * Theorem (Sec. 2.1, equation CRT-RSA).  Modular exponentiation and Montgomery
 * multiplication follow Sec. 3.2 (Algorithms 2 and 3); all of it runs in HIP
 * kernels on the GPU.
 *
 * Conventions
 *   - Big integers are little-endian arrays of uint32_t limbs.
 *   - Plaintext chunk i holds kb_i - 4 message bytes, kb_i = bits/8 of its key;
 *     the last chunk holds the remaining 1..kb_i-4 bytes.  A chunk is read as a
 *     big-endian integer, so every chunk is below its modulus.
 *   - Ciphertext block i is kb_i bytes, big-endian; blocks are concatenated in
 *     chunk order.  The ciphertext length is the sum of kb_i.
 *   - Functions return PMK_OK (0) or a negative status; on a validation error
 *     no output buffer is touched.  pmk_last_error() gives a message.
 *   - "Device pointer" means memory of the context's GPU (hipMalloc, or a torch
 *     CUDA tensor); "stream" is a hipStream_t passed as void* (NULL = the
 *     default stream).  Work on a stream is asynchronous: a zero return covers
 *     host-side validation and launch; errors the GPU detects (a ciphertext
 *     block out of range) are reported by pmk_plan_check().
 *   - One context per host thread; a context is not thread-safe.
 */
#ifndef PMK_H
#define PMK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PMK_OK = 0,
    PMK_EINVAL = -1,      /* bad argument or inconsistent key material */
    PMK_EKEY = -2,        /* a chunk names a key index >= number of loaded keys */
    PMK_ERANGE = -3,      /* a ciphertext block is not below its modulus (C must lie in Z_N, Sec. 1.1),
                             or decrypts to a plaintext wider than its chunk */
    PMK_ESIZE = -4,       /* chunk count / buffer sizes do not match the message */
    PMK_ENOMEM = -5,      /* device or host allocation failed */
    PMK_EDEVICE = -6,     /* HIP runtime error */
    PMK_EBUSY = -7,       /* keys replaced while plans made from them still exist */
    PMK_EUNSUPPORTED = -8, /* modulus size or exponent the library has no kernel for */
    PMK_EBLIND = -9        /* a blinding ciphertext block c_R is not invertible modulo N */
};

typedef struct pmk_ctx pmk_ctx;
typedef struct pmk_plan pmk_plan;

/*
 * One key pair (Sec. 1.1 step 1; Algorithm 1, Initialization: N = p q, public
 * exponent e, private exponent split for CRT decryption into
 * dp = d mod (p-1), dq = d mod (q-1) and qinv = q^-1 mod p, Sec. 2.1).
 *   bits    modulus length: a multiple of 64, 128..8192; N must have exactly
 *           this many bits.
 *   n       bits/32 limbs.
 *   n0inv   -N^-1 mod 2^32 (Montgomery constant of Algorithm 3 for r = 2^32).
 *   rr      bits/32 limbs: R^2 mod N with R = 2^bits.
 *   e       e_limbs limbs (1 or 2): the public exponent, odd, >= 3, < 2^64.
 *   p, q    bits/64 limbs each, p > q, p q = N.
 *   dp, dq  bits/64 limbs each.
 *   qinv    bits/64 limbs: q^-1 mod p.
 * n0inv, rr and p q = N, q qinv = 1 mod p are checked at load time.
 * The caller keeps ownership of every array; the library copies them.
 */
typedef struct {
    uint32_t bits;
    const uint32_t *n;
    uint32_t n0inv;
    const uint32_t *rr;
    const uint32_t *e;
    uint32_t e_limbs;
    const uint32_t *p;
    const uint32_t *q;
    const uint32_t *dp;
    const uint32_t *dq;
    const uint32_t *qinv;
} pmk_key;

/* Create a context on HIP device `device`.  *out receives the handle. */
int pmk_create(int device, pmk_ctx **out);

/* Free the context, its device key table and every plan still attached to it. */
void pmk_destroy(pmk_ctx *ctx);

/* Message of the last error on this context (never NULL; "" when none). */
const char *pmk_last_error(const pmk_ctx *ctx);

/*
 * Load (replace) the device key table: the key vectors E, D, N of Sec. 3.1
 * (one key pair per row of the chunk matrix).  Validates every key, derives the
 * per-prime Montgomery constants used by the kernels, and uploads the table.
 * Synchronous.  PMK_EINVAL names the first bad key in pmk_last_error();
 * PMK_EBUSY if plans made from the previous table are still alive.
 */
int pmk_keys_load(pmk_ctx *ctx, const pmk_key *keys, uint32_t nkeys);

/*
 * Host-only check of one key pair, the same checks pmk_keys_load makes (no GPU
 * needed).  Returns PMK_OK, PMK_EINVAL (reason written to msg[0..msg_cap),
 * msg may be NULL) or PMK_EUNSUPPORTED (no kernel for the modulus size).
 */
int pmk_key_check(const pmk_key *key, char *msg, size_t msg_cap);

/*
 * Host-only form of the chunk planning (no GPU needed): given the modulus bits
 * of nkeys keys, check key_map[0..nchunks) against a msg_len-byte message as
 * pmk_plan_create does (PMK_EKEY, PMK_ESIZE; PMK_EINVAL for bad key sizes) and
 * return the ciphertext length in *ct_len (may be NULL).
 */
int pmk_plan_validate(const uint32_t *key_bits, uint32_t nkeys, const uint32_t *key_map,
                      uint64_t nchunks, uint64_t msg_len, uint64_t *ct_len);

/* Number of keys loaded and the modulus bits of key `index` (0 if out of range). */
uint32_t pmk_key_count(const pmk_ctx *ctx);
uint32_t pmk_key_bits(const pmk_ctx *ctx, uint32_t index);

/*
 * Plan the chunking of a msg_len-byte message over the chunk-to-key map
 * key_map[0..nchunks) (HOST memory; chunk i uses key key_map[i]; Sec. 3.1).
 * Checks every key index (PMK_EKEY) and that nchunks is exactly the number of
 * chunks the message needs (PMK_ESIZE); msg_len = 0 requires nchunks = 0.
 * Sorts chunks by modulus size, computes chunk offsets, uploads them and
 * allocates the device scratch the kernels need.  *ct_len (may be NULL)
 * receives the ciphertext length.  The plan stays valid until destroyed or
 * until its context is destroyed.
 */
int pmk_plan_create(pmk_ctx *ctx, const uint32_t *key_map, uint64_t nchunks, uint64_t msg_len,
                    pmk_plan **out, uint64_t *ct_len);
void pmk_plan_destroy(pmk_plan *plan);

/* Sizes recorded in a plan. */
int pmk_plan_info(const pmk_plan *plan, uint64_t *msg_len, uint64_t *nchunks, uint64_t *ct_len);

/*
 * Encrypt (Algorithm 1, Encryption, without the blinding factor): for every
 * chunk c_i = m_i^e mod N_key(i).  d_msg: plan msg_len bytes (device);
 * d_ct: plan ct_len bytes (device).  Asynchronous on `stream`.
 */
int pmk_encrypt_plan(pmk_plan *plan, const uint8_t *d_msg, uint8_t *d_ct, void *stream);

/*
 * Decrypt by CRT (Sec. 2.1): m_p = c^dp mod p, m_q = c^dq mod q,
 * h = qinv (m_p - m_q) mod p, m = m_q + h q; writes msg_len bytes.  d_ct: plan
 * ct_len bytes (device); d_msg: plan msg_len bytes (device).  A block that is
 * not below its modulus (a ciphertext lies in Z_N, Sec. 1.1), or whose
 * plaintext does not fit its chunk's length (no encryption of a chunk of that
 * length produces it), sets the plan's device error flag (PMK_ERANGE from
 * pmk_plan_check) and that chunk's output bytes are written as zeros.
 */
int pmk_decrypt_plan(pmk_plan *plan, const uint8_t *d_ct, uint8_t *d_msg, void *stream);

/*
 * Output form of the plan's decryptions (pmk_decrypt_plan, the blinded and the
 * batched forms):
 *   PMK_DEC_CHUNKS  (default) msg_len bytes, chunk i as its own length, with
 *                   the range rules above;
 *   PMK_DEC_BLOCKS  every decrypted block in full, m_i = c_i^d mod N as kb_i
 *                   big-endian bytes laid out like the ciphertext (the output
 *                   buffer holds ct_len bytes): the private-key operation of
 *                   Sec. 1.1 step 3 on any block of Z_N, without the chunk
 *                   length check; a block not below N still sets PMK_ERANGE
 *                   and is written as zeros.
 * Host only; a change drops the plan's captured graphs (after waiting for the
 * device).  PMK_EINVAL for another value.
 */
enum { PMK_DEC_CHUNKS = 0, PMK_DEC_BLOCKS = 1 };
int pmk_plan_set_decrypt_output(pmk_plan *plan, int form);

/*
 * Blinded PMKRSA (Sec. 3.1, Eqs. 3-10, Algorithm 1 with its blinding factor R).
 * Encryption takes one blinding factor r_i per chunk in d_r -- laid out like
 * ciphertext blocks: kb_i bytes big-endian per chunk, ct_len bytes in all, each
 * 1 <= r_i < N with gcd(r_i, N) = 1 (the caller draws them) -- and writes
 * c*_i = (r_i m_i)^e mod N to d_ct_star and c_R,i = r_i^e mod N to d_ct_r (ct_len
 * bytes each, same block layout).  Decryption computes
 * m_i = (c*_i)^d (c_R,i^d)^-1 mod N, i.e. r'_i = c_R,i^d = r_i is divided out,
 * through CRT: per prime, (c*)^(d_p) times c_R^(p-1-d_p) (Fermat's inverse;
 * both powers in one squaring chain), then Garner.  A c* or c_R block not
 * below N, or a plaintext wider than its chunk, sets PMK_ERANGE and zeroes
 * that chunk's output (as pmk_decrypt_plan); a c_R divisible by p or q sets
 * PMK_EBLIND (both from pmk_plan_check).  Asynchronous on `stream`; every
 * buffer device memory, 4-byte aligned.
 */
int pmk_encrypt_blinded_plan(pmk_plan *plan, const uint8_t *d_msg, const uint8_t *d_r, uint8_t *d_ct_star,
                             uint8_t *d_ct_r, void *stream);
int pmk_decrypt_blinded_plan(pmk_plan *plan, const uint8_t *d_ct_star, const uint8_t *d_ct_r, uint8_t *d_msg,
                             void *stream);

/*
 * Batched form (the parallel loops of Algorithm 1, all size classes at once):
 * after packing, the exponentiation kernels of the plan's size classes run
 * side by side on `stream` and internal side streams (default priority),
 * forked and joined with events, so classes too small to fill the GPU share
 * it.  Encryption of the 3072- and 4096-bit classes is ONE persistent
 * work-queue launch whose waves take units (a quarter tile each) from a
 * device counter, 4096-bit units first; every other exponentiation is its
 * class's persistent kernel; for the CRT halves the two classes with the most
 * work get streams of their own and the others follow one another on a third.  The whole sequence (packing, exponentiation, CRT recombination,
 * unpacking) is captured once into a HIP graph per (input, output) buffer pair
 * and replayed on `stream`; a new buffer pair or window setting recaptures it.
 * Results are byte-identical to pmk_encrypt_plan / pmk_decrypt_plan.  With
 * profiling on (pmk_plan_profile) the sequence runs uncaptured so that each
 * launch can be timed (concurrent launches then overlap in the sums).  Same
 * buffer rules and errors as the plan forms; a plan's batch calls must not
 * overlap each other on different streams (they share its scratch).
 */
int pmk_encrypt_batch(pmk_plan *plan, const uint8_t *d_msg, uint8_t *d_ct, void *stream);
int pmk_decrypt_batch(pmk_plan *plan, const uint8_t *d_ct, uint8_t *d_msg, void *stream);

/*
 * Tuning: the window width of the fixed-window CRT exponentiation (2..6) of
 * the size class holding `bits`-bit moduli.  Changing it never changes
 * results, only speed; plans already made pick it up (graphs are recaptured).
 * pmk_get_window returns the width or a negative status.
 */
int pmk_set_window(pmk_ctx *ctx, uint32_t bits, int win);
int pmk_get_window(const pmk_ctx *ctx, uint32_t bits);

/*
 * Tuning: lanes per number of the CRT exponentiations (the parallel loops of
 * Algorithm 1 over the chunks; plain and blinded decryption alike) of the size
 * class holding `bits`-bit moduli,
 * where a launch would leave SIMDs idle (L lanes per number shorten each
 * wave's chain about L times, for more instructions).  A class whose CRT halves run one lane per
 * number (128- to 4096-bit keys) runs
 *   - a launch under one round of resident waves with `fill_lanes` lanes per
 *     number, or the largest smaller power of two for which every lane-group
 *     wave still has a SIMD of its own (units of 64 numbers modulo one prime
 *     times L at most 4 per compute unit), else one lane, and
 *   - the partial round after full ones as a launch of its own (its waves
 *     then spread over the SIMDs) with `tail_lanes` lanes per number, or the
 *     largest smaller power of two whose waves fit one round,
 * each 1, 2 or 4: L lanes per number give L times the waves, each with a
 * shorter chain per Montgomery product, for about twice the instructions per
 * number.  The 6144/8192-bit classes run 4 lanes per number; their
 * `fill_lanes` may be 8 (a launch whose 8-lane waves each get a SIMD of their
 * own then runs with 8) and their `tail_lanes` must be 4; the one-lane classes
 * take 1, 2 or 4, and `fill_lanes` 8 at 2048, 3072 and 4096 bits (PMK_EUNSUPPORTED
 * for other supported counts, PMK_EINVAL for counts other than 1, 2, 4, 8).  Results never change; graphs are
 * recaptured; PMK_EBUSY while a server runs.  pmk_get_lanes fills the current
 * values.
 */
int pmk_set_lanes(pmk_ctx *ctx, uint32_t bits, int fill_lanes, int tail_lanes);
int pmk_get_lanes(const pmk_ctx *ctx, uint32_t bits, int *fill_lanes, int *tail_lanes);

/*
 * Upper bound on the resident waves (workgroups) of every persistent
 * exponentiation launch of the context (the CRT halves, encryption, the
 * batched work queue, multi-prime parts and primality tests); 0 (the default)
 * leaves each launch at its kernel's occupancy on this device.  Each wave
 * then walks more work units (the parallel loops of Algorithm 1 over fewer
 * workers): a control for sharing the GPU with other work and for tuning;
 * results never change.  Graphs are recaptured.  PMK_EBUSY while a server
 * runs.
 */
int pmk_set_grid_limit(pmk_ctx *ctx, uint32_t waves);

/*
 * Autotuner for the launch configuration (L lanes per number, w window bits):
 * for every size class that has keys in the loaded table, time the CRT
 * decryption of full-size chunks (zero blocks: the exponentiation costs the
 * same for any input) under the first key of that class -- four rounds of
 * resident waves at three window widths ({4,5,6} for 1024-bit classes and up,
 * {3,4,5} below), keeping the fastest (pmk_set_window); then, for the classes
 * with one lane per number, a launch of a quarter of the compute units' worth
 * of job tiles and one of one and a third rounds at 1, 2 and 4 lanes per
 * number (fill also 8 at 2048-4096 bits), keeping the fastest fill and
 * tail forms, and for the 6144/8192-bit classes the first of these at 4 and 8
 * lanes (pmk_set_lanes); a form with more lanes is kept only if it wins by
 * 1 %.  cache_path (may be NULL): a
 * text file -- a signature line (GPU architecture, compute units, HIP runtime
 * version), then "<class bits> <window> <fill lanes> <tail lanes> <ms>"
 * lines.  When it exists and its signature matches this device, its windows
 * and lanes are applied without measuring, unless flags has
 * PMK_AUTOTUNE_FORCE; otherwise the measured choice is written there.  Synchronous; allocates (and frees) its own device buffers; needs a
 * loaded key table (PMK_EINVAL otherwise).
 */
enum { PMK_AUTOTUNE_FORCE = 1 };
int pmk_autotune(pmk_ctx *ctx, const char *cache_path, int flags);

/*
 * Wait for `stream`, then return and clear the plan's device-detected error
 * (PMK_OK, PMK_ERANGE or PMK_EBLIND; PMK_EBLIND when both were seen, since a
 * non-invertible blinding block also leaves its chunk's plaintext out of range).
 */
int pmk_plan_check(pmk_plan *plan, void *stream);

/*
 * Kernel timing (profiling aid).  pmk_plan_profile(plan, 1) waits for the
 * device, forgets earlier timings and from then on brackets every kernel the
 * plan launches with HIP events recorded on the launch stream;
 * pmk_plan_profile(plan, 0) stops.  pmk_plan_kernel_time sums, over the
 * recorded launches of one kernel kind, the event-measured durations in
 * milliseconds (waiting for them to complete) and their count.
 */
enum {
    PMK_KERNEL_PACK = 0,       /* bytes -> limbs */
    PMK_KERNEL_ENCRYPT = 1,    /* c = m^e mod N */
    PMK_KERNEL_CRT_HALVES = 2, /* m_p = c^dp mod p, m_q = c^dq mod q */
    PMK_KERNEL_GARNER = 3,     /* CRT recombination */
    PMK_KERNEL_UNPACK = 4,     /* limbs -> bytes */
    PMK_KERNEL_BATCH = 5,      /* persistent work-queue encryption (3072/4096-bit classes) */
    PMK_KERNEL_KINDS = 6
};
int pmk_plan_profile(pmk_plan *plan, int enable);
int pmk_plan_kernel_time(pmk_plan *plan, int kind, double *ms_total, uint64_t *launches);

/*
 * One-shot forms: plan, run, check and free in one call; synchronous on
 * `stream`.  key_map is host memory; d_msg / d_ct are device memory.
 * ct_cap / msg_len are checked against the plan (PMK_ESIZE).
 */
int pmk_encrypt(pmk_ctx *ctx, const uint8_t *d_msg, uint64_t msg_len, const uint32_t *key_map,
                uint64_t nchunks, uint8_t *d_ct, uint64_t ct_cap, void *stream);
int pmk_decrypt(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map,
                uint64_t nchunks, uint8_t *d_msg, uint64_t msg_len, void *stream);

/*
 * Host-buffer forms (the paper's transfer / compute / merge pipeline of its
 * CPU+GPU implementation, Sec. 3.3): msg and ct are HOST memory (pinned --
 * hipHostMalloc, or a torch tensor with pin_memory -- for asynchronous copies;
 * pageable memory works, with copies the runtime stages itself).  The plan's
 * chunk range is cut into `slices` runs of chunks of about equal bytes; slice
 * s is copied to the device, encrypted or decrypted, and copied back on three
 * streams, so the copies of one slice overlap the computation of the others.
 * slices = 0 picks, for encryption, up to four slices of at least 65,536
 * chunks each; for decryption, slices that each end on a whole round of CRT
 * work (1, 2, 4, ... rounds of resident waves) where the key map allows it (a
 * plan of one size class up to 4096 bits whose slices give every key only full
 * tiles, as a round-robin map does), else one slice -- so slicing adds no
 * partial round.  Sizes as pmk_encrypt_plan / pmk_decrypt_plan (the
 * decryption output form of the plan applies).  Synchronous: returns once the
 * output is in host memory, with the device-detected status (PMK_ERANGE as
 * pmk_plan_check).  The first call of a direction with a slicing plans its
 * slices (kept per direction) and the first call allocates device copies of
 * the whole input and output (kept with the plan); calls on one plan must not
 * overlap.
 */
int pmk_encrypt_host(pmk_plan *plan, const uint8_t *msg, uint8_t *ct, uint32_t slices);
int pmk_decrypt_host(pmk_plan *plan, const uint8_t *ct, uint8_t *msg, uint32_t slices);

/*
 * For callers that cannot allocate while they run (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pmk_decrypt
 * with the same arguments, results and errors, but calling no hipMalloc,
 * hipFree or other allocating routine.  Every device buffer its kernels use
 * (chunk descriptors, packed words, CRT half results, window tables, the
 * error word) lives in one fixed device array of 64 MiB that the library
 * holds on each GPU it runs on until the process ends; the host-side planning
 * uses buffers made at pmk_create / pmk_keys_load.  Limits: at most 65,536
 * chunks, and the chunk data plus at least one window table per size class
 * must fit the 64 MiB (PMK_ESIZE, before anything is launched, otherwise);
 * fewer table slots than pmk_decrypt's may run the exponentiation in more
 * rounds.  d_ct / d_msg are device memory, key_map host memory.  Synchronous
 * on `stream`.  Every call on one GPU, from any context or thread, shares that
 * GPU's array and keeps nothing from the previous call: calls that overlap on
 * one GPU race.
 */
int pmk_decrypt_noalloc(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map,
                        uint64_t nchunks, uint8_t *d_msg, uint64_t msg_len, void *stream);

/*
 * Multi-prime keys (Sec. 2.1, the multi-prime variant: N is the product of b
 * distinct primes of bits/b bits, and decryption runs b exponentiations modulo
 * the primes, on numbers of bits/b bits, then one recombination; against two
 * CRT halves of bits/2 bits that is b^2/4 times less work).  Supported: b = 3 with 3072-bit N and b = 4 with
 * 4096-bit N, every prime of exactly 1024 bits.
 *   bits     3072 or 4096.
 *   nprimes  bits / 1024.
 *   n        bits/32 limbs.
 *   primes   nprimes x 32 limbs: p_0, p_1, ... one after another.
 *   d        nprimes x 32 limbs: d_i = d mod (p_i - 1), below p_i.
 * Checked at load time: N odd with exactly `bits` bits, every prime odd with
 * 1024 bits, product of the primes = N, primes pairwise coprime, d_i < p_i.
 * The caller keeps ownership of the arrays; the library copies them.
 */
typedef struct {
    uint32_t bits;
    uint32_t nprimes;
    const uint32_t *n;
    const uint32_t *primes;
    const uint32_t *d;
} pmk_key_mp;

/* Host-only check of one multi-prime key: PMK_OK or PMK_EINVAL (reason in
 * msg[0..msg_cap), msg may be NULL). */
int pmk_mp_key_check(const pmk_key_mp *key, char *msg, size_t msg_cap);

/*
 * Load (replace) the context's multi-prime key table, separate from the
 * two-prime table of pmk_keys_load (key indices of pmk_mp_decrypt name rows of
 * this table).  Derives the per-prime Montgomery constants and the inverses
 * p_j^-1 mod p_i of the recombination.  Synchronous; PMK_EINVAL names the
 * first bad key.
 */
int pmk_mp_keys_load(pmk_ctx *ctx, const pmk_key_mp *keys, uint32_t nkeys);
uint32_t pmk_mp_key_count(const pmk_ctx *ctx);

/*
 * Decrypt a ciphertext made under multi-prime keys: the chunk layout of
 * pmk_plan_create (chunk i of key key_map[i] carries up to bits/8 - 4
 * plaintext bytes in one bits/8-byte block; key_map is host memory), every
 * block m = C^d mod N by one exponentiation per prime, m_i = C^(d_i) mod p_i,
 * and Garner's mixed-radix recombination
 * m = v_0 + p_0 (v_1 + p_1 (v_2 + ...)).  d_ct (ct_len bytes) and d_msg
 * (msg_len bytes) are device memory, 4-byte aligned.  Synchronous on
 * `stream`; its device scratch is a context-held arena, grown when a call
 * needs more and freed by pmk_destroy (calls on one context must not overlap).
 * PMK_EKEY / PMK_ESIZE as
 * pmk_plan_create, PMK_ERANGE when a block is not below its modulus or its
 * plaintext is wider than its chunk (that chunk's bytes are then zeros, as in
 * pmk_decrypt_plan).
 */
int pmk_mp_decrypt(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map,
                   uint64_t nchunks, uint8_t *d_msg, uint64_t msg_len, void *stream);

/*
 * Batched primality testing for key generation: the primes p, q of every key
 * pair of Algorithm 1's initialisation (Sec. 1.1 step 1; Sec. 3.1), tested on
 * the GPU, one lane per candidate.  `bits` is the key size the primes are for:
 * 1024, 2048, 3072 or 4096 (candidates of up to bits/2 bits; PMK_EUNSUPPORTED
 * otherwise).  Candidate i is the bits/64 little-endian 32-bit words at
 * d_cand[i * bits/64], odd and above 3 (above 4096 for the sieve).  Device
 * buffers; asynchronous on `stream`.
 *   pmk_sieve: d_flags[i] = 1 if no odd prime below 4096 divides candidate i, else 0.
 *   pmk_miller_rabin: d_result[i] = 1 if candidate i passes Miller-Rabin for
 *     every one of its `rounds` bases (1..256), base r at
 *     d_bases[(i * rounds + r) * bits/64] with 1 < base < m - 1 (the caller draws
 *     them); 0 if some base shows it composite.  Uses the context's window width
 *     for the `bits` class; keeps a table scratch on the context.
 */
int pmk_sieve(pmk_ctx *ctx, uint32_t bits, const uint32_t *d_cand, uint32_t count, uint32_t *d_flags, void *stream);
int pmk_miller_rabin(pmk_ctx *ctx, uint32_t bits, const uint32_t *d_cand, uint32_t count, const uint32_t *d_bases,
                     uint32_t rounds, uint32_t *d_result, void *stream);

/*
 * Request server (continuous batching).  A scheduler thread on the context
 * serves encryption and CRT-decryption requests of any size against the
 * loaded key table: the chunks of every admitted request join batching rounds
 * (chunks under one key share tiles across requests; each in-flight request
 * gets a fair share of a round, so small requests are not stuck behind large
 * ones), in the spirit of the paper's parallel chunk loops and transfer /
 * compute pipeline (Sec. 3.1, Algorithm 1; Sec. 3.3).  Requests are admitted in
 * arrival order while the device staging slab has room for their input and
 * output; their host buffers are copied in at admission and out at
 * completion.  Results are byte-identical to pmk_encrypt_plan /
 * pmk_decrypt_plan on the same input.
 *
 * pmk_server_start: staging_bytes (0: 512 MiB) is the admission budget of
 *   device memory for inputs and outputs in flight (with a pinned host mirror
 *   of the same size, through which the copies run asynchronously beside the
 *   rounds); round_chunks (0: two
 *   chip-filling rounds of 2048-bit CRT halves) bounds the chunks of one
 *   round; pipeline_depth as in the struct.  The key table and window widths may not change while the server
 *   runs (PMK_EBUSY).  PMK_EBUSY if a server already runs.
 * pmk_submit (thread-safe): validates like pmk_plan_create (PMK_EKEY,
 *   PMK_ESIZE, PMK_EINVAL; PMK_ESIZE also when out_cap is too small or the
 *   request could never fit the staging slab), copies key_map, and returns a
 *   ticket.  `in` and `out` are HOST memory that must stay valid until the
 *   ticket is reported done: encryption reads msg_len bytes and writes the
 *   ciphertext; decryption reads the ciphertext (its length follows from the
 *   key map) and writes msg_len bytes.
 * pmk_poll (thread-safe, non-blocking) / pmk_wait (thread-safe, blocking):
 *   fill *info; once a ticket has been reported done it is forgotten (a later
 *   call returns PMK_EINVAL).  info->status is the request's result (PMK_OK,
 *   PMK_ERANGE for a ciphertext block not below its modulus -- that request's
 *   output is then unspecified -- or PMK_EDEVICE).  Times are CLOCK_MONOTONIC
 *   nanoseconds.
 * pmk_server_stop: finishes every submitted request, then stops the thread.
 *   pmk_destroy stops a running server the same way.
 */
typedef struct {
    uint64_t staging_bytes;
    uint64_t round_chunks;
    uint32_t pipeline_depth; /* rounds in flight: 0 or 1 = one at a time (lower latency),
                                2 = the next round is built and queued while one runs */
} pmk_server_cfg;

enum { PMK_OP_ENCRYPT = 0, PMK_OP_DECRYPT = 1 };
enum { PMK_REQ_QUEUED = 0, PMK_REQ_ADMITTED = 1, PMK_REQ_DONE = 2 };

typedef struct {
    int op;                  /* PMK_OP_ENCRYPT or PMK_OP_DECRYPT */
    const uint8_t *in;       /* host input */
    uint8_t *out;            /* host output */
    uint64_t out_cap;        /* bytes available at out */
    uint64_t msg_len;        /* plaintext bytes */
    const uint32_t *key_map; /* host, nchunks key indices (copied at submit) */
    uint64_t nchunks;
} pmk_request;

typedef struct {
    int state;   /* PMK_REQ_* */
    int status;  /* valid when state == PMK_REQ_DONE */
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;
} pmk_ticket_info;

typedef struct {
    uint64_t requests_submitted, requests_done;
    uint64_t rounds, chunks;  /* batching rounds run and chunks they processed */
    uint64_t busy_ns;         /* time the scheduler spent in rounds */
    uint64_t queued;          /* requests waiting for admission now */
} pmk_server_stats;

int pmk_server_start(pmk_ctx *ctx, const pmk_server_cfg *cfg);
int pmk_submit(pmk_ctx *ctx, const pmk_request *req, uint64_t *ticket);
int pmk_poll(pmk_ctx *ctx, uint64_t ticket, pmk_ticket_info *info);
int pmk_wait(pmk_ctx *ctx, uint64_t ticket, pmk_ticket_info *info);
int pmk_server_stats_get(pmk_ctx *ctx, pmk_server_stats *out);
int pmk_server_stop(pmk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PMK_H */
