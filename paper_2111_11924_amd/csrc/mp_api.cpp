// C ABI of the multi-prime decryption (declared in include/pmk.h): key table
// load and the one-shot decryption, pack -> one exponentiation per prime ->
// Garner -> unpack, in a device arena the context keeps between calls.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>
#include <vector>

#include "../../include/pmk.h"
#include "keyprep.hpp"
#include "mp_geom.hpp"
#include "pmk_state.hpp"

using namespace pmk;

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

extern "C" {

int pmk_mp_key_check(const pmk_key_mp *key, char *msg, size_t msg_cap) {
    if (!key) return PMK_EINVAL;
    std::string why;
    if (!check_key_mp(*key, &why)) {
        if (msg && msg_cap) snprintf(msg, msg_cap, "%s", why.c_str());
        return PMK_EINVAL;
    }
    if (msg && msg_cap) msg[0] = 0;
    return PMK_OK;
}

int pmk_mp_keys_load(pmk_ctx *ctx, const pmk_key_mp *keys, uint32_t nkeys) {
    if (!ctx) return PMK_EINVAL;
    if (nkeys && !keys) return set_err(ctx, PMK_EINVAL, "keys is NULL");
    std::vector<KeySlot> slots(nkeys);
    uint32_t counts[kMpClasses] = {};
    for (uint32_t i = 0; i < nkeys; ++i) {
        char why[256];
        const int rc = pmk_mp_key_check(&keys[i], why, sizeof why);
        if (rc != PMK_OK) return set_err(ctx, rc, "key %u: %s", i, why);
        const int c = keys[i].bits == 3072 ? 0 : 1;
        slots[i] = {c, counts[c]++, keys[i].bits, std::vector<uint32_t>(keys[i].n, keys[i].n + keys[i].bits / 32)};
    }
    std::vector<std::vector<uint32_t>> host(kMpClasses);
    for (int c = 0; c < kMpClasses; ++c)
        if (counts[c]) host[c].assign((size_t)counts[c] * make_mp_geom(c).stride, 0u);
    for (uint32_t i = 0; i < nkeys; ++i) {
        const int c = slots[i].cls;
        build_record_mp(keys[i], c, host[c].data() + (size_t)slots[i].slot * make_mp_geom(c).stride);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    uint32_t *fresh[kMpClasses] = {};
    for (int c = 0; c < kMpClasses; ++c) {
        if (!counts[c]) continue;
        const size_t bytes = host[c].size() * sizeof(uint32_t);
        hipError_t e = hipMalloc(&fresh[c], bytes);
        if (e == hipSuccess) e = hipMemcpy(fresh[c], host[c].data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            for (auto &p : fresh)
                if (p) (void)hipFree(p);
            return hip_err(ctx, e, "multi-prime key table upload");
        }
    }
    for (int c = 0; c < kMpClasses; ++c) {
        if (ctx->d_mp_keys[c]) (void)hipFree(ctx->d_mp_keys[c]);
        ctx->d_mp_keys[c] = fresh[c];
    }
    ctx->mp_keys.swap(slots);
    ctx->err.clear();
    return PMK_OK;
}

uint32_t pmk_mp_key_count(const pmk_ctx *ctx) { return ctx ? (uint32_t)ctx->mp_keys.size() : 0u; }

int pmk_mp_decrypt(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map, uint64_t nchunks,
                   uint8_t *d_msg, uint64_t msg_len, void *stream) {
    if (!ctx) return PMK_EINVAL;
    std::vector<uint32_t> bits(ctx->mp_keys.size());
    for (size_t i = 0; i < bits.size(); ++i) bits[i] = ctx->mp_keys[i].bits;
    std::vector<std::vector<ChunkDesc>> per_key(bits.size());
    std::string why;
    uint64_t need = 0;
    const int rc = walk_chunks(bits.data(), (uint32_t)bits.size(), key_map, nchunks, msg_len, &need, &why,
                               [&](uint64_t, uint32_t k, uint64_t off, uint64_t len, uint64_t ct) {
                                   per_key[k].push_back(ChunkDesc{off, ct, ctx->mp_keys[k].slot, (uint32_t)len});
                               });
    if (rc != PMK_OK) return set_err(ctx, rc, "%s", why.c_str());
    if (ct_len != need)
        return set_err(ctx, PMK_ESIZE, "ciphertext has %llu bytes, the chunks need %llu", (unsigned long long)ct_len,
                       (unsigned long long)need);
    if (msg_len == 0) return PMK_OK;
    if (!d_ct || !d_msg || ((uintptr_t)d_ct & 3u) || ((uintptr_t)d_msg & 3u))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    // key-uniform tiles of 64 chunks per class; padding slots keep the tile's key
    std::vector<ChunkDesc> per[kMpClasses];
    std::vector<uint32_t> tkeys[kMpClasses];
    for (size_t k = 0; k < per_key.size(); ++k) {
        const auto &list = per_key[k];
        const int c = ctx->mp_keys[k].cls;
        for (size_t i = 0; i < list.size(); i += kTile) {
            tkeys[c].push_back(ctx->mp_keys[k].slot);
            for (size_t l = 0; l < (size_t)kTile; ++l)
                per[c].push_back(i + l < list.size() ? list[i + l] : ChunkDesc{0, 0, ctx->mp_keys[k].slot, 0});
        }
    }
    for (int c = 0; c < kMpClasses; ++c)
        if (tkeys[c].size() > 0x3FFFFFFull) return set_err(ctx, PMK_ESIZE, "too many chunks in one size class");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    const int win = window_for(1024);
    // one context-held device arena, grown when a call needs more (the call is
    // synchronous, so nothing still uses the old one): error flag, then per class
    // descriptors, tile keys, packed input, packed output, prime results, tables
    struct Part {
        uint64_t desc, tk, x32, y32, parts, table;
        uint32_t grid;
    } at[kMpClasses] = {};
    uint64_t total = kAlign;  // the error flag
    for (int c = 0; c < kMpClasses; ++c) {
        const uint64_t ntiles = tkeys[c].size();
        if (!ntiles) continue;
        const MpGeom g = make_mp_geom(c);
        const uint32_t units = (uint32_t)(ntiles * g.parts);
        Part &a = at[c];
        a.grid = std::max<uint32_t>(1, persistent_grid(units, mp_wave_slots(ctx->num_cus), ctx->grid_limit));
        a.desc = total;
        total += align_up(per[c].size() * sizeof(ChunkDesc));
        a.tk = total;
        total += align_up(ntiles * sizeof(uint32_t));
        a.x32 = total;
        total += align_up(ntiles * g.S * kTile * sizeof(uint32_t));
        a.y32 = total;
        total += align_up(ntiles * g.S * kTile * sizeof(uint32_t));
        a.parts = total;
        total += align_up(ntiles * g.parts * kMpNL * kTile * sizeof(uint32_t));
        a.table = total;
        total += align_up((uint64_t)a.grid * mp_slot_words(win) * sizeof(uint32_t));
    }
    hipError_t e = hipSuccess;
    if (total > ctx->mp_scratch_bytes) {
        if (ctx->mp_scratch) (void)hipFree(ctx->mp_scratch);
        ctx->mp_scratch = nullptr;
        ctx->mp_scratch_bytes = 0;
        e = hipMalloc(&ctx->mp_scratch, total);
        if (e != hipSuccess) {
            ctx->mp_scratch = nullptr;
            return hip_err(ctx, e, "multi-prime scratch allocation");
        }
        ctx->mp_scratch_bytes = total;
    }
    uint8_t *base = (uint8_t *)ctx->mp_scratch;
    uint32_t *d_err = (uint32_t *)base;
    e = hipMemsetAsync(d_err, 0, sizeof(uint32_t), s);
    for (int c = 0; c < kMpClasses && e == hipSuccess; ++c) {
        const uint64_t ntiles = tkeys[c].size();
        if (!ntiles) continue;
        const Part &a = at[c];
        ChunkDesc *desc = (ChunkDesc *)(base + a.desc);
        uint32_t *tk = (uint32_t *)(base + a.tk), *x32 = (uint32_t *)(base + a.x32), *y32 = (uint32_t *)(base + a.y32);
        uint32_t *parts = (uint32_t *)(base + a.parts), *table = (uint32_t *)(base + a.table);
        e = hipMemcpyAsync(desc, per[c].data(), per[c].size() * sizeof(ChunkDesc), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(tk, tkeys[c].data(), ntiles * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) break;
        const uint32_t *keys = ctx->d_mp_keys[c];
        int le = mp_launch_pack(c, d_ct, desc, keys, tk, (uint32_t)ntiles, x32, s);
        if (!le)
            le = mp_launch_parts(c, keys, tk, desc, (uint32_t)ntiles, x32, parts, table, mp_slot_words(win), a.grid,
                                 win, d_err, s);
        if (!le) le = mp_launch_garner(c, keys, desc, (uint32_t)ntiles, parts, y32, s);
        if (!le) le = mp_launch_unpack(c, y32, desc, keys, tk, (uint32_t)ntiles, x32, d_msg, d_err, s);
        if (le) e = (hipError_t)le;
    }
    // the host vectors per[c] / tkeys[c] must outlive the asynchronous copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    uint32_t flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, d_err, sizeof flag, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return hip_err(ctx, e, "multi-prime decryption");
    }
    if (flag & 1u)
        return set_err(ctx, PMK_ERANGE, "a ciphertext block is not below its modulus or decrypts wider than its chunk");
    ctx->err.clear();
    return PMK_OK;
}

}  // extern "C"
