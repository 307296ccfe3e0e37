// Multi-prime CRT decryption (Sec. 2.1, the multi-prime variant of CRT-RSA):
// N = p_0 p_1 ... p_(b-1), m_i = c^(d_i) mod p_i with d_i = d mod (p_i - 1),
// then Garner's mixed-radix recombination m = v_0 + p_0 (v_1 + p_1 (v_2 + ...)).
//   mp_part_kernel    one lane per chunk, one job per (tile, prime): c mod p_i
//                     and into Montgomery form at once, as the sum of
//                     MM(c_k, R^(k+2)) over the b radix pieces c_k of c (so
//                     x~ = c R mod p_i), then the sliding-window exponentiation;
//   mp_garner_kernel  v_i = (...((m_i - v_0) p_0^-1 - v_1) p_1^-1 ... - v_(i-1)) p_(i-1)^-1
//                     mod p_i, then Horner's rule over the v_i.
#include "kernels_impl.hpp"
#include "mp_geom.hpp"

namespace pmk {

template <int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void mp_part_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ tile_key, const ChunkDesc *__restrict__ desc,
    uint32_t ntiles, const uint32_t *__restrict__ x32, uint32_t *__restrict__ parts, uint32_t *table,
    uint64_t slot_words, int win, uint32_t *err) {
    code_align<code_id(kCodeMpPart, K, 0)>();
    constexpr MpGeom G = make_mp_geom(K);
    constexpr int NL = kMpNL, LB = kMpLB, S = G.S, P = G.parts, SP = kMpSP, PL = pad4(kMpNL);
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const int lane = threadIdx.x;
    uint32_t *tbl = table + (size_t)blockIdx.x * slot_words;
    const uint32_t units = ntiles * P;
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
        const uint32_t tile = u / P;
        const int part = (int)(u % P);
        const uint32_t *kr = keys + (size_t)uni(tile_key[tile]) * G.stride;  // wave-uniform
        const uint32_t *qr = kr + G.off_part[part];
        uint32_t n[NL];
        load_uniform(n, qr + G.q_m);
        const uint32_t n0 = uni(qr[G.q_m0]);
        const uint32_t *dexp = qr + G.q_d;
        const uint32_t *w = fresh_v(x32 + (size_t)tile * S * kTile + lane);
        if (part == 0 && desc[(size_t)tile * kTile + lane].msg_len) {
            // C must lie in Z_N: compare with N, most significant word first
            const uint32_t *n32 = kr + G.off_n32;
            int cmp = 0;
#pragma unroll 1
            for (int k = S - 1; k >= 0 && cmp == 0; --k) {
                const uint32_t x = w[(size_t)k * kTile], y = n32[k];
                cmp = (x > y) - (x < y);
            }
            if (cmp >= 0) atomicOr(err, 1u);
        }
        uint32_t acc[NL], b[NL];
        // pieces: c = sum_k c_k R^k; MM(c_k, R^(k+2)) = c_k R^(k+1) mod p, summed
        // (below 2 P p, inside R) into x~ = c R mod p.  Phases: 0 pieces (running
        // sum parked in entry 1), 1 x~^2, 5 odd powers: entry e = x~^(2e+1),
        // 2 sliding-window steps (squarings, then times an odd power), 3 MM(., 1)
#pragma unroll
        for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w, kTile, j);
        load_limbs(b, qr + G.q_rpow);
        const int TH = 1 << (win - 1);
        int phase = 0, piece = 0, e = 1, sq = 0;
        WinStep st = WinStep::make(0, 0u, false, -1);
        ExpWords nx{0u, 0u, 0u};
        for (;;) {
            if (phase == 2) {
                if (sq < st.nsq()) {
                    mont_sqr<NL, LB>(acc, acc, n, n0);
                    ++sq;
                    continue;
                }
                if (st.mul()) {
                    load_entry(b, tbl, st.idx(), lane);
                } else {
#pragma unroll
                    for (int j = 0; j < NL; ++j) b[j] = j == 0 ? 1u : 0u;
                    phase = 3;
                }
            }
            mont_mul<NL, LB>(acc, acc, b, n, n0);
            if (phase == 3) break;
            if (phase == 0) {
                if (piece > 0) {
                    load_entry(b, tbl, 1, lane);
                    uint32_t c = 0;
#pragma unroll
                    for (int j = 0; j < NL; ++j) {
                        const uint32_t v = acc[j] + b[j] + c;
                        acc[j] = v & MASK;
                        c = v >> LB;
                    }
                }
                if (++piece < P) {
                    store_entry(tbl, 1, lane, acc);
#pragma unroll
                    for (int j = 0; j < NL; ++j) acc[j] = radix_limb_mem<S, LB>(w, kTile, piece * NL + j);
                    load_limbs(b, qr + G.q_rpow + piece * PL);
                    continue;
                }
                store_entry(tbl, 0, lane, acc);  // x~
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];
                phase = 1;
                continue;
            }
            if (phase == 1) {
#pragma unroll
                for (int j = 0; j < NL; ++j) b[j] = acc[j];  // x~^2, the step between odd powers
                load_entry(acc, tbl, 0, lane);
                phase = 5;
                continue;
            }
            if (phase == 5) {
                store_entry(tbl, e, lane, acc);
                if (++e < TH) continue;
                const int top = exp_top_bit(dexp, SP);
                if (top < 0) {
                    load_limbs(acc, qr + G.q_one);
                    st = WinStep::make(0, 0u, false, -1);
                } else {
                    st = win_first(nx, dexp, SP, top, win);
                    load_entry(acc, tbl, st.idx(), lane);
                    win_advance(st, nx, dexp, SP, win);
                }
                phase = 2;
                sq = 0;
                continue;
            }
            // phase 2: the step's product is done
            win_advance(st, nx, dexp, SP, win);
            sq = 0;
        }
        canonicalize<NL, LB>(acc, n);
        uint32_t *dst = parts + ((size_t)(tile * P + part) * NL) * kTile + lane;
#pragma unroll
        for (int j = 0; j < NL; ++j) dst[(size_t)j * kTile] = acc[j];
    }
}

// One lane per chunk slot (block = tile): Garner's coefficients v_i written
// over the part results, then Horner's rule into the S result words.
template <int K>
__global__ __launch_bounds__(64) void mp_garner_kernel(const uint32_t *__restrict__ keys,
                                                       const ChunkDesc *__restrict__ desc, uint32_t ntiles,
                                                       uint32_t *__restrict__ parts, uint32_t *__restrict__ y32) {
    code_align<code_id(kCodeMpGarner, K, 0)>();
    constexpr MpGeom G = make_mp_geom(K);
    constexpr int NL = kMpNL, LB = kMpLB, S = G.S, P = G.parts, PL = pad4(kMpNL);
    constexpr uint32_t MASK = Radix<LB>::MASK;
    const uint32_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    if (tile >= ntiles) return;
    const uint32_t *kr = keys + (size_t)desc[(size_t)tile * kTile + lane].key * G.stride;
    auto part_at = [&](int i) { return parts + ((size_t)(tile * P + i) * NL) * kTile + lane; };
    for (int i = 1; i < P; ++i) {
        const uint32_t *qr = kr + G.off_part[i];
        uint32_t p[NL], t[NL], a[NL];
        load_limbs(p, qr + G.q_m);
        const uint32_t p0 = qr[G.q_m0];
        const uint32_t *mi = part_at(i);
#pragma unroll
        for (int j = 0; j < NL; ++j) t[j] = mi[(size_t)j * kTile];
        for (int jv = 0; jv < i; ++jv) {
            // a = t + 2 p - v_jv in (0, 4p) (v_jv < p_jv < 2 p for primes of one size)
            const uint32_t *vj = part_at(jv);
            int32_t cy = 0;
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const int32_t v = (int32_t)t[j] + 2 * (int32_t)p[j] - (int32_t)vj[(size_t)j * kTile] + cy;
                a[j] = (uint32_t)v & MASK;
                cy = v >> LB;  // arithmetic shift
            }
            load_limbs(t, qr + G.q_cinv + jv * PL);  // (p_jv^-1 mod p) R mod p
            mont_mul<NL, LB>(t, a, t, p, p0);         // (t - v_jv) p_jv^-1 mod p, below 2p
        }
        canonicalize<NL, LB>(t, p);
        uint32_t *vi = part_at(i);
#pragma unroll
        for (int j = 0; j < NL; ++j) vi[(size_t)j * kTile] = t[j];
    }
    // Horner: x = v_(P-1); x = x p_i + v_i for i = P-2 .. 0 (limbs of LB bits)
    uint32_t x[P * NL], y[P * NL];
    int xl = NL;
    {
        const uint32_t *v = part_at(P - 1);
#pragma unroll 1
        for (int j = 0; j < NL; ++j) x[j] = v[(size_t)j * kTile];
    }
#pragma unroll 1
    for (int i = P - 2; i >= 0; --i) {
        const uint32_t *pm = kr + G.off_part[i] + G.q_m;
        const uint32_t *v = part_at(i);
        uint64_t cy = 0;
        const int yl = xl + NL;
#pragma unroll 1
        for (int k = 0; k < yl; ++k) {
            uint64_t acc = cy + (k < NL ? v[(size_t)k * kTile] : 0u);
            const int lo = k - NL + 1 > 0 ? k - NL + 1 : 0, hi = k < xl ? k : xl - 1;
#pragma unroll 1
            for (int a = lo; a <= hi; ++a) acc += (uint64_t)x[a] * pm[k - a];
            y[k] = (uint32_t)acc & MASK;
            cy = acc >> LB;
        }
#pragma unroll 1
        for (int k = 0; k < yl; ++k) x[k] = y[k];
        xl = yl;
    }
    // limbs -> S little-endian words
    const bool live = desc[(size_t)tile * kTile + lane].msg_len != 0;
#pragma unroll 1
    for (int k = 0; k < S; ++k) {
        const int bit = 32 * k, j = bit / LB, sh = bit % LB;
        const uint64_t l0 = j < xl ? x[j] : 0u;
        const uint64_t l1 = j + 1 < xl ? x[j + 1] : 0u;
        const uint64_t l2 = j + 2 < xl ? x[j + 2] : 0u;
        const uint32_t word = (uint32_t)((l0 >> sh) | (l1 << (LB - sh)) | (l2 << (2 * LB - sh)));
        if (live) y32[((size_t)tile * S + k) * kTile + lane] = word;
    }
}

namespace {

template <int K>
int launch_pack_k(const uint8_t *src, const ChunkDesc *desc, const uint32_t *keys, const uint32_t *tile_key,
                  uint32_t ntiles, uint32_t *x32, hipStream_t s) {
    constexpr MpGeom G = make_mp_geom(K);
    hipLaunchKernelGGL((pack_kernel<G.S, kTile>), dim3(ntiles), dim3(256), 0, s, src, desc, keys, tile_key, G.stride,
                       G.off_kbytes, x32, 1);
    return (int)hipGetLastError();
}

// plaintext chunks, range-checked against the packed ciphertext x32 (as the
// two-prime decryption)
template <int K>
int launch_unpack_k(const uint32_t *y32, const ChunkDesc *desc, const uint32_t *keys, const uint32_t *tile_key,
                    uint32_t ntiles, const uint32_t *x32, uint8_t *dst, uint32_t *err, hipStream_t s) {
    constexpr MpGeom G = make_mp_geom(K);
    hipLaunchKernelGGL((unpack_kernel<G.S, kTile>), dim3(ntiles), dim3(256), 0, s, y32, desc, keys, tile_key,
                       G.stride, G.off_kbytes, G.off_n32, dst, (int)kOutChunks, x32, nullptr, err, nullptr);
    return (int)hipGetLastError();
}

}  // namespace

int mp_launch_pack(int k, const uint8_t *src, const ChunkDesc *desc, const uint32_t *keys, const uint32_t *tile_key,
                   uint32_t ntiles, uint32_t *x32, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    return k == 0 ? launch_pack_k<0>(src, desc, keys, tile_key, ntiles, x32, s)
                  : launch_pack_k<1>(src, desc, keys, tile_key, ntiles, x32, s);
}

int mp_launch_unpack(int k, const uint32_t *y32, const ChunkDesc *desc, const uint32_t *keys,
                     const uint32_t *tile_key, uint32_t ntiles, const uint32_t *x32, uint8_t *dst, uint32_t *err,
                     void *stream) {
    hipStream_t s = (hipStream_t)stream;
    return k == 0 ? launch_unpack_k<0>(y32, desc, keys, tile_key, ntiles, x32, dst, err, s)
                  : launch_unpack_k<1>(y32, desc, keys, tile_key, ntiles, x32, dst, err, s);
}

int mp_launch_parts(int k, const uint32_t *keys, const uint32_t *tile_key, const ChunkDesc *desc, uint32_t ntiles,
                    const uint32_t *x32, uint32_t *parts, uint32_t *table, uint64_t slot_words, uint32_t grid,
                    int win, uint32_t *err, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (k == 0)
        hipLaunchKernelGGL(mp_part_kernel<0>, dim3(grid), dim3(64), 0, s, keys, tile_key, desc, ntiles, x32, parts,
                           table, slot_words, win, err);
    else
        hipLaunchKernelGGL(mp_part_kernel<1>, dim3(grid), dim3(64), 0, s, keys, tile_key, desc, ntiles, x32, parts,
                           table, slot_words, win, err);
    return (int)hipGetLastError();
}

int mp_launch_garner(int k, const uint32_t *keys, const ChunkDesc *desc, uint32_t ntiles, uint32_t *parts,
                     uint32_t *y32, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (k == 0)
        hipLaunchKernelGGL(mp_garner_kernel<0>, dim3(ntiles), dim3(64), 0, s, keys, desc, ntiles, parts, y32);
    else
        hipLaunchKernelGGL(mp_garner_kernel<1>, dim3(ntiles), dim3(64), 0, s, keys, desc, ntiles, parts, y32);
    return (int)hipGetLastError();
}

uint64_t mp_slot_words(int win) { return (uint64_t)(1u << (win - 1)) * kMpNL * kTile; }

uint32_t mp_wave_slots(int num_cus) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)mp_part_kernel<1>, 64, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return (uint32_t)nb * (uint32_t)num_cus;
}

}  // namespace pmk
