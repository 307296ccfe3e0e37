// C ABI of the library: context, key table, plans, and the encrypt / decrypt
// entry points (declared in include/pmk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/pmk.h"
#include "keyprep.hpp"
#include "pmk_internal.hpp"
#include "pmk_state.hpp"

using namespace pmk;

namespace pmk {

int set_err(pmk_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int hip_err(pmk_ctx *ctx, hipError_t e, const char *where) {
    return set_err(ctx, e == hipErrorOutOfMemory ? PMK_ENOMEM : PMK_EDEVICE, "%s: %s", where,
                   hipGetErrorString(e));
}


void drop_timings(pmk_plan *pl) {
    for (auto &t : pl->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    pl->timed.clear();
}

void drop_graphs(pmk_plan *pl) {
    for (auto &g : pl->graph) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = CapturedGraph{};
    }
}

void free_plan_memory(pmk_plan *pl) {
    drop_timings(pl);
    drop_graphs(pl);
    for (auto &h : pl->hp) {
        for (pmk_plan *s : h.sub) pmk_plan_destroy(s);
        for (hipEvent_t ev : h.ev) (void)hipEventDestroy(ev);
        h = pmk_plan::HostSlices{};
    }
    for (int i = 0; i < pmk_plan::kPipe; ++i) {
        if (pl->hp_stream[i]) (void)hipStreamDestroy(pl->hp_stream[i]);
        pl->hp_stream[i] = nullptr;
    }
    if (pl->capture_stream) (void)hipStreamDestroy(pl->capture_stream);
    for (int i = 0; i < pmk_plan::kSide; ++i) {
        if (pl->side_stream[i]) (void)hipStreamDestroy(pl->side_stream[i]);
        if (pl->join_event[i]) (void)hipEventDestroy(pl->join_event[i]);
        pl->side_stream[i] = nullptr;
        pl->join_event[i] = nullptr;
    }
    if (pl->fork_event) (void)hipEventDestroy(pl->fork_event);
    pl->capture_stream = nullptr;
    pl->fork_event = nullptr;
    for (void *p : pl->allocs) (void)hipFree(p);
    pl->allocs.clear();
}

// Grows a per-wave table buffer to at least `need` words.  Tables are sized
// for the window widths in force; a wider window set later reallocates them
// here, before any launch that would index past the old size.
hipError_t regrow(pmk_plan *pl, uint32_t **p, uint64_t &cap, uint64_t need) {
    if (need <= cap) return hipSuccess;
    if (*p) {
        (void)hipDeviceSynchronize();  // launches already queued may still read it
        for (size_t i = 0; i < pl->allocs.size(); ++i)
            if (pl->allocs[i] == (void *)*p) {
                pl->allocs.erase(pl->allocs.begin() + i);
                break;
            }
        (void)hipFree(*p);
        *p = nullptr;
        cap = 0;
    }
    drop_graphs(pl);
    hipError_t e = dev_alloc(pl, p, need * sizeof(uint32_t));
    if (e == hipSuccess) cap = need;
    return e;
}

// Window tables of every class of the plan, sized for the context's windows.
hipError_t ensure_tables(pmk_plan *pl) {
    for (int c = 0; c < kNumClasses; ++c) {
        ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        r.win = pl->ctx->win[c];
        r.grid_cap = pl->ctx->grid_limit;
        r.fill_lanes = pl->ctx->fill_lanes[c];
        r.tail_lanes = pl->ctx->tail_lanes[c];
        const uint64_t need = std::max(r.slots_enc * table_words_per_slot(c, 0, 0),
                                       r.slots_dec * table_words_per_slot(c, 1, r.win));
        const hipError_t e = regrow(pl, &r.table, pl->table_cap[c], need);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}



}  // namespace pmk

extern "C" {

int pmk_create(int device, pmk_ctx **out) {
    if (!out) return PMK_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PMK_EDEVICE;
    pmk_ctx *ctx = new (std::nothrow) pmk_ctx();
    if (!ctx) return PMK_ENOMEM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return PMK_EDEVICE;
    }
    ctx->num_cus = prop.multiProcessorCount;
    ctx->device_name = prop.gcnArchName;
    for (int c = 0; c < kNumClasses; ++c) {
        ctx->win[c] = window_for(kClassBits[c] / 2);
        ctx->fill_lanes[c] = default_fill_lanes(kClassBits[c]);
        ctx->tail_lanes[c] = default_tail_lanes(kClassBits[c]);
    }
    ctx->err.reserve(600);  // messages (below 512 bytes) are then stored without allocating
    // the allocation-free entry point reports it if its scratch is unavailable
    (void)noalloc_setup(ctx);
    *out = ctx;
    return PMK_OK;
}

void pmk_destroy(pmk_ctx *ctx) {
    if (!ctx) return;
    server_shutdown(ctx);
    (void)hipSetDevice(ctx->device);
    while (!ctx->plans.empty()) pmk_plan_destroy(*ctx->plans.begin());
    for (auto &p : ctx->d_keys)
        if (p) (void)hipFree(p);
    if (ctx->mr_table) (void)hipFree(ctx->mr_table);
    for (auto &p : ctx->d_mp_keys)
        if (p) (void)hipFree(p);
    if (ctx->mp_scratch) (void)hipFree(ctx->mp_scratch);
    if (ctx->na_host) (void)hipHostFree(ctx->na_host);
    delete ctx;
}

const char *pmk_last_error(const pmk_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int pmk_key_check(const pmk_key *key, char *msg, size_t msg_cap) {
    if (!key) return PMK_EINVAL;
    std::string why;
    if (!check_key(*key, &why)) {
        if (msg && msg_cap) snprintf(msg, msg_cap, "%s", why.c_str());
        return PMK_EINVAL;
    }
    if (class_for_bits(key->bits) < 0) {
        if (msg && msg_cap) snprintf(msg, msg_cap, "no kernel for %u-bit moduli", key->bits);
        return PMK_EUNSUPPORTED;
    }
    if (msg && msg_cap) msg[0] = 0;
    return PMK_OK;
}

int pmk_keys_load(pmk_ctx *ctx, const pmk_key *keys, uint32_t nkeys) {
    if (!ctx) return PMK_EINVAL;
    if (ctx->live_plans) return set_err(ctx, PMK_EBUSY, "%d plan(s) still use the current key table", ctx->live_plans);
    if (nkeys && !keys) return set_err(ctx, PMK_EINVAL, "keys is NULL");
    std::vector<KeySlot> slots(nkeys);
    uint32_t counts[kNumClasses] = {};
    for (uint32_t i = 0; i < nkeys; ++i) {
        char why[256];
        const int rc = pmk_key_check(&keys[i], why, sizeof why);
        if (rc != PMK_OK) return set_err(ctx, rc, "key %u: %s", i, why);
        const int c = class_for_bits(keys[i].bits);
        slots[i] = {c, counts[c]++, keys[i].bits, std::vector<uint32_t>(keys[i].n, keys[i].n + keys[i].bits / 32)};
    }
    std::vector<std::vector<uint32_t>> host(kNumClasses);
    for (int c = 0; c < kNumClasses; ++c)
        if (counts[c]) host[c].assign((size_t)counts[c] * make_geom(kClassBits[c]).stride, 0u);
    for (uint32_t i = 0; i < nkeys; ++i) {
        const int c = slots[i].cls;
        build_record(keys[i], c, host[c].data() + (size_t)slots[i].slot * make_geom(kClassBits[c]).stride);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    uint32_t *fresh[kNumClasses] = {};
    for (int c = 0; c < kNumClasses; ++c) {
        if (!counts[c]) continue;
        const size_t bytes = host[c].size() * sizeof(uint32_t);
        hipError_t e = hipMalloc(&fresh[c], bytes);
        if (e == hipSuccess) e = hipMemcpy(fresh[c], host[c].data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            for (auto &p : fresh)
                if (p) (void)hipFree(p);
            return hip_err(ctx, e, "key table upload");
        }
    }
    for (int c = 0; c < kNumClasses; ++c) {
        if (ctx->d_keys[c]) (void)hipFree(ctx->d_keys[c]);
        ctx->d_keys[c] = fresh[c];
        ctx->class_count[c] = counts[c];
    }
    ctx->keys.swap(slots);
    ctx->err.clear();
    if (noalloc_keys(ctx) != PMK_OK) return set_err(ctx, PMK_ENOMEM, "host planning buffers");
    return PMK_OK;
}

uint32_t pmk_key_count(const pmk_ctx *ctx) { return ctx ? (uint32_t)ctx->keys.size() : 0u; }

uint32_t pmk_key_bits(const pmk_ctx *ctx, uint32_t index) {
    return ctx && index < ctx->keys.size() ? ctx->keys[index].bits : 0u;
}

int pmk_plan_validate(const uint32_t *key_bits, uint32_t nkeys, const uint32_t *key_map, uint64_t nchunks,
                      uint64_t msg_len, uint64_t *ct_len) {
    if (nkeys && !key_bits) return PMK_EINVAL;
    for (uint32_t i = 0; i < nkeys; ++i)
        if (key_bits[i] < 128 || key_bits[i] > 8192 || key_bits[i] % 64) return PMK_EINVAL;
    return walk_chunks(key_bits, nkeys, key_map, nchunks, msg_len, ct_len, nullptr,
                       [](uint64_t, uint32_t, uint64_t, uint64_t, uint64_t) {});
}

int pmk_plan_create(pmk_ctx *ctx, const uint32_t *key_map, uint64_t nchunks, uint64_t msg_len,
                    pmk_plan **out, uint64_t *ct_len) {
    if (!ctx || !out) return PMK_EINVAL;
    *out = nullptr;
    std::vector<uint32_t> bits(ctx->keys.size());
    for (size_t i = 0; i < bits.size(); ++i) bits[i] = ctx->keys[i].bits;
    // chunks of each key, in message order
    std::vector<std::vector<ChunkDesc>> per_key(ctx->keys.size());
    std::string why;
    uint64_t total = 0;
    const int rc = walk_chunks(bits.data(), (uint32_t)bits.size(), key_map, nchunks, msg_len, &total, &why,
                               [&](uint64_t, uint32_t k, uint64_t off, uint64_t len, uint64_t ct) {
                                   per_key[k].push_back(ChunkDesc{off, ct, ctx->keys[k].slot, (uint32_t)len});
                               });
    if (rc != PMK_OK) return set_err(ctx, rc, "%s", why.c_str());
    // key-uniform tiles of up to 64 chunks, per size class; padding slots keep
    // the tile's key and have msg_len 0
    std::vector<std::vector<ChunkDesc>> per(kNumClasses);
    std::vector<std::vector<uint32_t>> tkeys(kNumClasses);
    uint32_t counts[kNumClasses] = {};
    for (size_t k = 0; k < per_key.size(); ++k) {
        const auto &list = per_key[k];
        const int c = ctx->keys[k].cls;
        const size_t cpt = (size_t)chunks_per_tile(kClassBits[c]);
        counts[c] += (uint32_t)list.size();
        for (size_t i = 0; i < list.size(); i += cpt) {
            tkeys[c].push_back(ctx->keys[k].slot);
            for (size_t l = 0; l < cpt; ++l)
                per[c].push_back(i + l < list.size() ? list[i + l] : ChunkDesc{0, 0, ctx->keys[k].slot, 0});
        }
    }
    for (int c = 0; c < kNumClasses; ++c)
        if (tkeys[c].size() > 0x3FFFFFFull) return set_err(ctx, PMK_ESIZE, "too many chunks in one size class");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");

    pmk_plan *pl = new (std::nothrow) pmk_plan();
    if (!pl) return set_err(ctx, PMK_ENOMEM, "plan allocation");
    pl->ctx = ctx;
    pl->msg_len = msg_len;
    pl->nchunks = nchunks;
    pl->ct_len = total;
    if (nchunks) pl->key_map.assign(key_map, key_map + nchunks);
    hipError_t e = dev_alloc(pl, &pl->d_err, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(pl->d_err, 0, sizeof(uint32_t));
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
        ClassRun &r = pl->runs[c];
        r.cls = c;
        r.count = counts[c];
        r.ntiles = (uint32_t)tkeys[c].size();
        r.err = pl->d_err;
        r.win = ctx->win[c];
        if (!r.ntiles) continue;
        const Geom g = make_geom(kClassBits[c]);
        const uint64_t tiles = r.ntiles, cpt = (uint64_t)chunks_per_tile(kClassBits[c]);
        r.keys = ctx->d_keys[c];
        r.slots_enc = std::max<uint32_t>(1, std::min<uint64_t>(wave_slots(c, 0, ctx->num_cus), exp_units(c, 0, r.ntiles)));
        r.slots_dec = std::max<uint32_t>(1, std::min<uint64_t>(wave_slots(c, 1, ctx->num_cus), exp_units(c, 1, r.ntiles)));
        ChunkDesc *d = nullptr;
        uint32_t *tk = nullptr;
        e = dev_alloc(pl, &d, per[c].size() * sizeof(ChunkDesc));
        if (e == hipSuccess)
            e = hipMemcpy(d, per[c].data(), per[c].size() * sizeof(ChunkDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = dev_alloc(pl, &tk, tkeys[c].size() * sizeof(uint32_t));
        if (e == hipSuccess)
            e = hipMemcpy(tk, tkeys[c].data(), tkeys[c].size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        r.desc = d;
        r.tile_key = tk;
        if (e == hipSuccess) e = dev_alloc(pl, &r.x32, tiles * g.S * cpt * sizeof(uint32_t));
        if (e == hipSuccess) e = dev_alloc(pl, &r.y32, tiles * g.S * cpt * sizeof(uint32_t));
        if (e == hipSuccess) e = dev_alloc(pl, &r.half, tiles * 2 * g.nlh * cpt * sizeof(uint32_t));
    }
    if (e == hipSuccess) e = ensure_tables(pl);
    if (e != hipSuccess) {
        free_plan_memory(pl);
        delete pl;
        return hip_err(ctx, e, "plan allocation");
    }
    ctx->live_plans++;
    ctx->plans.insert(pl);
    if (ct_len) *ct_len = total;
    *out = pl;
    return PMK_OK;
}

void pmk_plan_destroy(pmk_plan *pl) {
    if (!pl) return;
    (void)hipSetDevice(pl->ctx->device);
    (void)hipDeviceSynchronize();
    free_plan_memory(pl);
    pl->ctx->live_plans--;
    pl->ctx->plans.erase(pl);
    delete pl;
}

int pmk_plan_info(const pmk_plan *pl, uint64_t *msg_len, uint64_t *nchunks, uint64_t *ct_len) {
    if (!pl) return PMK_EINVAL;
    if (msg_len) *msg_len = pl->msg_len;
    if (nchunks) *nchunks = pl->nchunks;
    if (ct_len) *ct_len = pl->ct_len;
    return PMK_OK;
}

static int aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

int pmk_encrypt_plan(pmk_plan *pl, const uint8_t *d_msg, uint8_t *d_ct, void *stream) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!d_msg || !d_ct || !aligned4(d_msg) || !aligned4(d_ct))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    if (const hipError_t te = ensure_tables(pl)) return hip_err(ctx, te, "window table allocation");
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        int e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, d_msg, 0, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_ENCRYPT, stream, [&] { return launch_encrypt(r, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, d_ct, 0, stream); });
        if (e) return hip_err(ctx, (hipError_t)e, "encrypt launch");
    }
    return PMK_OK;
}

int pmk_decrypt_plan(pmk_plan *pl, const uint8_t *d_ct, uint8_t *d_msg, void *stream) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!d_msg || !d_ct || !aligned4(d_msg) || !aligned4(d_ct))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    if (const hipError_t te = ensure_tables(pl)) return hip_err(ctx, te, "window table allocation");
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        int e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, d_ct, 1, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_CRT_HALVES, stream, [&] { return launch_decrypt_halves(r, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_GARNER, stream, [&] { return launch_garner(r, stream); });
        if (!e)
            e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, d_msg, pl->dec_mode, stream); });
        if (e) return hip_err(ctx, (hipError_t)e, "decrypt launch");
    }
    return PMK_OK;
}

static int blind_prepare(pmk_plan *pl) {
    if (pl->blind_ready) return PMK_OK;
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        const Geom g = make_geom(kClassBits[c]);
        const uint64_t tiles = r.ntiles, cpt = (uint64_t)chunks_per_tile(kClassBits[c]);
        const hipError_t e = dev_alloc(pl, &pl->x32b[c], tiles * g.S * cpt * sizeof(uint32_t));
        if (e != hipSuccess) return hip_err(pl->ctx, e, "blinding buffers");
    }
    pl->blind_ready = true;
    return PMK_OK;
}

int pmk_encrypt_blinded_plan(pmk_plan *pl, const uint8_t *d_msg, const uint8_t *d_r, uint8_t *d_ct_star,
                             uint8_t *d_ct_r, void *stream) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!d_msg || !d_r || !d_ct_star || !d_ct_r || !aligned4(d_msg) || !aligned4(d_r) || !aligned4(d_ct_star) ||
        !aligned4(d_ct_r))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    if (const hipError_t te = ensure_tables(pl)) return hip_err(ctx, te, "window table allocation");
    int rc = blind_prepare(pl);
    if (rc != PMK_OK) return rc;
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        ClassRun rb = r;  // c_R = r^e, from the blinding blocks (packed like ciphertext blocks)
        rb.x32 = pl->x32b[c];
        ClassRun star = r;  // c* = m^e c_R = (m r)^e: the last product takes c_R instead of 1
        star.fin32 = r.y32;
        int e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(rb, d_r, 1, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_ENCRYPT, stream, [&] { return launch_encrypt(rb, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, d_ct_r, 0, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, d_msg, 0, stream); });
        // each unit reads its tile's c_R words before writing that tile's result over them
        if (!e) e = timed_launch(pl, PMK_KERNEL_ENCRYPT, stream, [&] { return launch_encrypt(star, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, d_ct_star, 0, stream); });
        if (e) return hip_err(ctx, (hipError_t)e, "blinded encrypt launch");
    }
    return PMK_OK;
}

int pmk_decrypt_blinded_plan(pmk_plan *pl, const uint8_t *d_ct_star, const uint8_t *d_ct_r, uint8_t *d_msg,
                             void *stream) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!d_msg || !d_ct_star || !d_ct_r || !aligned4(d_msg) || !aligned4(d_ct_star) || !aligned4(d_ct_r))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    if (const hipError_t te = ensure_tables(pl)) return hip_err(ctx, te, "window table allocation");
    int rc = blind_prepare(pl);
    if (rc != PMK_OK) return rc;
    for (int c = 0; c < kNumClasses; ++c) {
        ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        // the one-pass form keeps two odd-power tables per slot
        const hipError_t te = regrow(pl, &r.table, pl->table_cap[c], 2 * r.slots_dec * table_words_per_slot(c, 1, r.win));
        if (te != hipSuccess) return hip_err(ctx, te, "window table allocation");
    }
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        // (c*)^d_p c_R^(p-1-d_p) in one chain per prime; c* packed at x32, c_R at x32b
        ClassRun rj = r;
        rj.fin32 = pl->x32b[c];
        ClassRun rr = r;
        rr.x32 = pl->x32b[c];
        int e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, d_ct_star, 1, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(rr, d_ct_r, 1, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_CRT_HALVES, stream, [&] { return launch_decrypt_joint(rj, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_GARNER, stream, [&] { return launch_garner(r, stream); });
        // both blocks are range-checked while unpacking
        if (!e)
            e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(rj, d_msg, pl->dec_mode, stream); });
        if (e) return hip_err(ctx, (hipError_t)e, "blinded decrypt launch");
    }
    return PMK_OK;
}

int pmk_plan_set_decrypt_output(pmk_plan *pl, int form) {
    if (!pl) return PMK_EINVAL;
    if (form != PMK_DEC_CHUNKS && form != PMK_DEC_BLOCKS)
        return set_err(pl->ctx, PMK_EINVAL, "decryption output form must be PMK_DEC_CHUNKS or PMK_DEC_BLOCKS");
    const int mode = form == PMK_DEC_BLOCKS ? 2 : 1;
    if (mode != pl->dec_mode) {
        (void)hipSetDevice(pl->ctx->device);
        (void)hipDeviceSynchronize();  // a replay in flight still uses its graph
        drop_graphs(pl);               // captured sequences hold the old unpack form
        pl->dec_mode = mode;
    }
    return PMK_OK;
}

int pmk_plan_profile(pmk_plan *pl, int enable) {
    if (!pl) return PMK_EINVAL;
    (void)hipSetDevice(pl->ctx->device);
    (void)hipDeviceSynchronize();
    drop_timings(pl);
    pl->profile = enable != 0;
    return PMK_OK;
}

int pmk_plan_kernel_time(pmk_plan *pl, int kind, double *ms_total, uint64_t *launches) {
    if (!pl || kind < 0 || kind >= PMK_KERNEL_KINDS) return PMK_EINVAL;
    double total = 0;
    uint64_t n = 0;
    for (auto &t : pl->timed) {
        if (t.kind != kind) continue;
        float ms = 0;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) return hip_err(pl->ctx, e, "kernel timing");
        total += ms;
        ++n;
    }
    if (ms_total) *ms_total = total;
    if (launches) *launches = n;
    return PMK_OK;
}

}  // extern "C"

namespace pmk {

// Launches of one pass of the batched path.  Packing runs on `stream`; then
// the exponentiation kernels of the size classes run side by side on `stream`
// and the plan's side streams (forked and joined with events), so that
// classes too small to fill the chip share it:
//   encryption: the 4096- and 3072-bit classes as one persistent work-queue
//     launch on a side stream, the one-lane classes on `stream`, largest first;
//   decryption: each class's CRT-halves kernel, classes ordered by their work:
//     the two largest on streams of their own, the others in that order on a
//     third.
// Garner recombination and unpacking follow on `stream`.
int batch_sequence(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, void *stream) {
    pmk_ctx *ctx = pl->ctx;
    BatchArgs a{};
    uint32_t total = 0;
    for (int i = 0; i < kWideClasses; ++i) {
        const int c = wide_class(i);
        a.runs[i] = pl->runs[c];
        a.runs[i].win = ctx->win[c];
        a.start[i] = total;
        total += pl->runs[c].ntiles ? exp_units(c, 0, pl->runs[c].ntiles) : 0u;
    }
    a.start[kWideClasses] = total;
    a.counter = pl->d_counter;
    a.table = pl->batch_table;
    a.slot_words = batch_slot_words();
    int e = 0;
    if (!decrypt && total) e = launch_counter_reset(pl->d_counter, stream);
    // launches of the exponentiation stage: (class, stream index)
    int order[kNumClasses], nl = 0;
    for (int c = kNumClasses - 1; c >= 0 && !e; --c) {
        ClassRun r = pl->runs[c];
        if (!r.ntiles) continue;
        e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, in, decrypt, stream); });
        if (decrypt || !is_wide_class(c)) order[nl++] = c;
    }
    if (decrypt) {  // classes by canonical work, largest first
        auto work = [&](int c) {
            const double s = kClassBits[c] / 64.0;
            return (double)pl->runs[c].ntiles * kClassBits[c] * (2 * s * s + s);
        };
        std::sort(order, order + nl, [&](int x, int y) { return work(x) > work(y); });
    }
    // decryption: the two largest classes on streams of their own, the rest one
    // after another on a third (measured on the mixed 25 MiB workload: 60.7
    // against 61.8 ms with every class on a stream of its own, 65.0 ms with the
    // largest class alone beside all others)
    const int lanes = decrypt ? std::min(nl, 3) : (total && nl ? 2 : 1);
    if (!e && lanes > 1) {
        e = hipEventRecord(pl->fork_event, (hipStream_t)stream);
        for (int i = 0; i < lanes - 1 && !e; ++i) e = hipStreamWaitEvent(pl->side_stream[i], pl->fork_event, 0);
    }
    auto stream_of = [&](int lane) { return lane == 0 ? stream : (void *)pl->side_stream[lane - 1]; };
    if (!e && !decrypt && total) {
        void *s = stream_of(lanes - 1);
        const uint32_t grid = persistent_grid(total, pl->batch_slots, ctx->grid_limit);
        e = timed_launch(pl, PMK_KERNEL_BATCH, s, [&] { return launch_batch(a, grid, s); });
    }
    for (int i = 0; i < nl && !e; ++i) {
        ClassRun r = pl->runs[order[i]];
        r.win = ctx->win[order[i]];
        if (decrypt && nl > 1) {
            // classes side by side fill the chip together: no class's launch is
            // short of work on its own, so every number keeps one lane
            // (measured: lane groups here cost 47 % on the mixed 25 MiB workload)
            // and a class's last partial round stays in its launch, where its
            // waves start as soon as waves of that launch finish
            r.fill_lanes = lanes_half(kClassBits[order[i]]);
            r.tail_lanes = lanes_half(kClassBits[order[i]]) > 1 ? r.fill_lanes : 0;
        }
        void *s = decrypt ? stream_of(i < lanes ? i : lanes - 1) : stream;
        e = timed_launch(pl, decrypt ? PMK_KERNEL_CRT_HALVES : PMK_KERNEL_ENCRYPT, s, [&] {
            return decrypt ? launch_decrypt_halves(r, s) : launch_encrypt(r, s);
        });
    }
    for (int i = 0; i < lanes - 1 && !e; ++i) {
        e = hipEventRecord(pl->join_event[i], pl->side_stream[i]);
        if (!e) e = hipStreamWaitEvent((hipStream_t)stream, pl->join_event[i], 0);
    }
    for (int c = kNumClasses - 1; c >= 0 && !e; --c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        if (decrypt) e = timed_launch(pl, PMK_KERNEL_GARNER, stream, [&] { return launch_garner(r, stream); });
        if (!e) {
            const int mode = decrypt ? pl->dec_mode : 0;
            e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, out, mode, stream); });
        }
    }
    return e;
}

int batch_prepare(pmk_plan *pl) {
    if (pl->d_counter) return PMK_OK;
    pmk_ctx *ctx = pl->ctx;
    uint32_t units = 0;
    for (int i = 0; i < kWideClasses; ++i) {
        const int c = wide_class(i);
        units += pl->runs[c].ntiles ? exp_units(c, 0, pl->runs[c].ntiles) : 0u;
    }
    pl->batch_slots = std::max<uint32_t>(1, std::min(batch_wave_slots(ctx->num_cus), units));
    uint32_t *counter = nullptr;
    hipError_t e = dev_alloc(pl, &counter, sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking);
    for (int i = 0; i < pmk_plan::kSide && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&pl->side_stream[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join_event[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork_event, hipEventDisableTiming);
    if (e != hipSuccess) return hip_err(ctx, e, "batch scratch allocation");
    pl->d_counter = counter;
    return PMK_OK;
}

// The wide batch kernel's table (encryption keeps two numbers per wave).
hipError_t ensure_batch_table(pmk_plan *pl) {
    bool any = false;
    for (int i = 0; i < kWideClasses; ++i) any = any || pl->runs[wide_class(i)].ntiles;
    const uint64_t need = any ? (uint64_t)pl->batch_slots * batch_slot_words() : 0;
    return regrow(pl, &pl->batch_table, pl->batch_cap, need);
}

int batch_run(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, void *stream) {
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!in || !out || ((uintptr_t)in & 3u) || ((uintptr_t)out & 3u))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    int rc = batch_prepare(pl);
    if (rc != PMK_OK) return rc;
    hipError_t te = ensure_tables(pl);
    if (te == hipSuccess) te = ensure_batch_table(pl);
    if (te != hipSuccess) return hip_err(ctx, te, "window table allocation");
    if (pl->profile) {
        // kernel timing needs events around each launch: run the sequence uncaptured
        const int e = batch_sequence(pl, decrypt, in, out, stream);
        return e ? hip_err(ctx, (hipError_t)e, "batch launch") : PMK_OK;
    }
    CapturedGraph &g = pl->graph[decrypt];
    if (!g.exec || g.in != in || g.out != out || g.epoch != ctx->epoch) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = CapturedGraph{};
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_err(ctx, e, "graph capture");
        const int le = batch_sequence(pl, decrypt, in, out, pl->capture_stream);
        e = hipStreamEndCapture(pl->capture_stream, &graph);
        if (le || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_err(ctx, le ? (hipError_t)le : e, "batch launch (capture)");
        }
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g = CapturedGraph{};
            return hip_err(ctx, e, "graph instantiate");
        }
        g.in = in;
        g.out = out;
        g.epoch = ctx->epoch;
    }
    const hipError_t e = hipGraphLaunch(g.exec, (hipStream_t)stream);
    return e == hipSuccess ? PMK_OK : hip_err(ctx, e, "graph launch");
}

}  // namespace pmk

extern "C" {

int pmk_encrypt_batch(pmk_plan *pl, const uint8_t *d_msg, uint8_t *d_ct, void *stream) {
    if (!pl) return PMK_EINVAL;
    return batch_run(pl, 0, d_msg, d_ct, stream);
}

int pmk_decrypt_batch(pmk_plan *pl, const uint8_t *d_ct, uint8_t *d_msg, void *stream) {
    if (!pl) return PMK_EINVAL;
    return batch_run(pl, 1, d_ct, d_msg, stream);
}

int pmk_set_window(pmk_ctx *ctx, uint32_t bits, int win) {
    if (!ctx) return PMK_EINVAL;
    const int c = class_for_bits(bits);
    if (c < 0) return set_err(ctx, PMK_EUNSUPPORTED, "no size class for %u bits", bits);
    if (win < 2 || win > kMaxWin) return set_err(ctx, PMK_EINVAL, "window width must be 2..%d", kMaxWin);
    if (ctx->server) return set_err(ctx, PMK_EBUSY, "window widths are fixed while a server runs");
    if (ctx->win[c] != win) {
        ctx->win[c] = win;
        ctx->epoch++;
        for (pmk_plan *pl : ctx->plans) pl->runs[c].win = win;
    }
    return PMK_OK;
}

int pmk_get_window(const pmk_ctx *ctx, uint32_t bits) {
    if (!ctx) return PMK_EINVAL;
    const int c = class_for_bits(bits);
    return c < 0 ? PMK_EUNSUPPORTED : ctx->win[c];
}

int pmk_set_lanes(pmk_ctx *ctx, uint32_t bits, int fill_lanes, int tail_lanes) {
    if (!ctx) return PMK_EINVAL;
    const int c = class_for_bits(bits);
    if (c < 0) return set_err(ctx, PMK_EUNSUPPORTED, "no size class for %u bits", bits);
    auto ok = [](int l) { return l == 1 || l == 2 || l == 4 || l == 8; };
    if (!ok(fill_lanes) || !ok(tail_lanes)) return set_err(ctx, PMK_EINVAL, "lanes per number must be 1, 2, 4 or 8");
    if (!lanes_valid(kClassBits[c], fill_lanes, tail_lanes)) {
        const int fixed = lanes_half(kClassBits[c]);
        if (fixed == 1)
            return set_err(ctx, PMK_EUNSUPPORTED,
                           "the %d-bit class takes 1, 2 or 4 lanes per number (fill 8 at 2048-4096 bits)",
                           kClassBits[c]);
        return set_err(ctx, PMK_EUNSUPPORTED,
                       "the %d-bit class runs its CRT halves in groups of %d lanes (small launches %d or %d)",
                       kClassBits[c], fixed, fixed, 2 * fixed);
    }
    if (ctx->server) return set_err(ctx, PMK_EBUSY, "lane settings are fixed while a server runs");
    if (ctx->fill_lanes[c] != fill_lanes || ctx->tail_lanes[c] != tail_lanes) {
        ctx->fill_lanes[c] = fill_lanes;
        ctx->tail_lanes[c] = tail_lanes;
        ctx->epoch++;
    }
    return PMK_OK;
}

int pmk_get_lanes(const pmk_ctx *ctx, uint32_t bits, int *fill_lanes, int *tail_lanes) {
    if (!ctx) return PMK_EINVAL;
    const int c = class_for_bits(bits);
    if (c < 0) return PMK_EUNSUPPORTED;
    if (fill_lanes) *fill_lanes = ctx->fill_lanes[c];
    if (tail_lanes) *tail_lanes = ctx->tail_lanes[c];
    return PMK_OK;
}

int pmk_set_grid_limit(pmk_ctx *ctx, uint32_t waves) {
    if (!ctx) return PMK_EINVAL;
    if (ctx->server) return set_err(ctx, PMK_EBUSY, "the grid limit is fixed while a server runs");
    if (ctx->grid_limit != waves) {
        ctx->grid_limit = waves;
        ctx->epoch++;  // captured graphs hold the old grids
    }
    return PMK_OK;
}

}  // extern "C"

namespace {

// identity of the device and runtime an autotuning result belongs to
std::string tune_signature(const pmk_ctx *ctx) {
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    char buf[256];
    std::snprintf(buf, sizeof buf, "pmk-autotune 2 %s cus=%d hip=%d", ctx->device_name.c_str(), ctx->num_cus, rt);
    return buf;
}

// Applies a cache file written for this device; false if absent or foreign.
bool tune_load(pmk_ctx *ctx, const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool ok = std::fgets(line, sizeof line, f) != nullptr;
    if (ok) {
        line[strcspn(line, "\r\n")] = 0;
        ok = tune_signature(ctx) == line;
    }
    int got[kNumClasses], fill[kNumClasses], tail[kNumClasses];
    for (int c = 0; c < kNumClasses; ++c) {
        got[c] = ctx->win[c];
        fill[c] = ctx->fill_lanes[c];
        tail[c] = ctx->tail_lanes[c];
    }
    unsigned bits = 0;
    int win = 0, fl = 0, tl = 0;
    while (ok && std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%u %d %d %d", &bits, &win, &fl, &tl) != 4) continue;
        const int c = class_for_bits(bits);
        if (c < 0 || kClassBits[c] != (int)bits || win < 2 || win > kMaxWin || !lanes_valid(kClassBits[c], fl, tl)) {
            ok = false;
            break;
        }
        got[c] = win;
        fill[c] = fl;
        tail[c] = tl;
    }
    std::fclose(f);
    if (!ok) return false;
    for (int c = 0; c < kNumClasses; ++c) {
        (void)pmk_set_window(ctx, (uint32_t)kClassBits[c], got[c]);
        (void)pmk_set_lanes(ctx, (uint32_t)kClassBits[c], fill[c], tail[c]);
    }
    return true;
}

// Best-of-`reps` time of the CRT decryption of `tiles` full tiles under key k0
// (zero blocks: the exponentiation costs the same for any input), or PMK error.
int tune_time(pmk_plan *pl, const uint8_t *ct, uint8_t *out, hipStream_t st, int reps, float *best);
int tune_batch(pmk_ctx *ctx, uint32_t k0, uint64_t tiles, hipStream_t st, int reps, float *best) {
    const uint64_t nch = tiles * (uint64_t)kTile;
    const uint64_t kb = ctx->keys[k0].bits / 8;
    std::vector<uint32_t> km(nch, k0);
    pmk_plan *pl = nullptr;
    uint64_t ct_len = 0;
    int rc = pmk_plan_create(ctx, km.data(), nch, nch * (kb - 4), &pl, &ct_len);
    if (rc != PMK_OK) return rc;
    uint8_t *ct = nullptr, *out = nullptr;
    hipError_t e = hipMalloc(&ct, ct_len);
    if (e == hipSuccess) e = hipMalloc(&out, nch * (kb - 4));
    if (e == hipSuccess) e = hipMemset(ct, 0, ct_len);
    rc = e == hipSuccess ? tune_time(pl, ct, out, st, reps, best) : hip_err(ctx, e, "autotune buffers");
    if (ct) (void)hipFree(ct);
    if (out) (void)hipFree(out);
    pmk_plan_destroy(pl);
    return rc;
}

// Time of one CRT decryption of `pl` (device-resident buffers), best of `reps`.
int tune_time(pmk_plan *pl, const uint8_t *ct, uint8_t *out, hipStream_t st, int reps, float *best) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int rc = e == hipSuccess ? pmk_decrypt_plan(pl, ct, out, st) : PMK_EDEVICE;  // warm-up, sizes tables
    *best = 1e30f;
    for (int i = 0; i < reps && rc == PMK_OK; ++i) {
        (void)hipEventRecord(a, st);
        rc = pmk_decrypt_plan(pl, ct, out, st);
        (void)hipEventRecord(b, st);
        float ms = 0.f;
        if (rc == PMK_OK && hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess)
            *best = std::min(*best, ms);
        else if (rc == PMK_OK)
            rc = PMK_EDEVICE;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return rc;
}

}  // namespace

extern "C" {

int pmk_autotune(pmk_ctx *ctx, const char *cache_path, int flags) {
    if (!ctx) return PMK_EINVAL;
    if (ctx->keys.empty()) return set_err(ctx, PMK_EINVAL, "autotuning needs a loaded key table");
    if (ctx->server) return set_err(ctx, PMK_EBUSY, "autotuning is not possible while a server runs");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    if (cache_path && !(flags & PMK_AUTOTUNE_FORCE) && tune_load(ctx, cache_path)) return PMK_OK;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return set_err(ctx, PMK_EDEVICE, "stream creation failed");
    std::string report = tune_signature(ctx) + "\n";
    int rc = PMK_OK;
    for (int c = 0; c < kNumClasses && rc == PMK_OK; ++c) {
        uint32_t k0 = UINT32_MAX;
        for (uint32_t k = 0; k < ctx->keys.size(); ++k)
            if (ctx->keys[k].cls == c) {
                k0 = k;
                break;
            }
        if (k0 == UINT32_MAX) continue;
        const int cb = kClassBits[c];
        const uint32_t per_tile = exp_units(c, 1, 1);
        // four chip-filling rounds of work units (steady state, not one wave of launches)
        const uint64_t tiles = std::max<uint32_t>(1, 4 * wave_slots(c, 1, ctx->num_cus) / per_tile);
        const uint64_t nch = tiles * (uint64_t)chunks_per_tile(cb);
        const uint64_t kb = ctx->keys[k0].bits / 8;
        std::vector<uint32_t> km(nch, k0);
        pmk_plan *pl = nullptr;
        uint64_t ct_len = 0;
        rc = pmk_plan_create(ctx, km.data(), nch, nch * (kb - 4), &pl, &ct_len);
        if (rc != PMK_OK) break;
        uint8_t *ct = nullptr, *out = nullptr;
        hipError_t e = hipMalloc(&ct, ct_len);
        if (e == hipSuccess) e = hipMalloc(&out, nch * (kb - 4));
        if (e == hipSuccess) e = hipMemset(ct, 0, ct_len);  // zero blocks: valid input, data-independent timing
        if (e != hipSuccess) rc = hip_err(ctx, e, "autotune buffers");
        const int w0 = window_for(cb / 2) > 4 ? 4 : 3;
        int best_w = ctx->win[c];
        float best_ms = 1e30f;
        char line[128];
        for (int w = w0; w < w0 + 3 && w <= kMaxWin && rc == PMK_OK; ++w) {
            (void)pmk_set_window(ctx, (uint32_t)cb, w);
            float ms = 0.f;
            rc = tune_time(pl, ct, out, st, 3, &ms);
            // a wider window must win by 1% to be taken: its table costs memory
            if (rc == PMK_OK && ms < 0.99f * best_ms) {
                best_ms = ms;
                best_w = w;
            }
        }
        (void)pmk_set_window(ctx, (uint32_t)cb, best_w);
        if (ct) (void)hipFree(ct);
        if (out) (void)hipFree(out);
        pmk_plan_destroy(pl);
        // lanes per number where a launch leaves the chip idle: one-lane
        // classes: one unit per two compute units (fill), then one and a third
        // rounds of resident waves (the last third is the tail); lane-group
        // classes: the fill form only (their own or twice as many lanes); a
        // wider form must win by 1 %
        int best_fill = ctx->fill_lanes[c], best_tail = ctx->tail_lanes[c];
        if (rc == PMK_OK && lanes_half(cb) > 1) {
            const int L0 = lanes_half(cb);
            const uint64_t size = std::max<uint64_t>(1, (uint64_t)ctx->num_cus / 4);
            float lbest = 1e30f;
            for (int L : {L0, 2 * L0}) {
                (void)pmk_set_lanes(ctx, (uint32_t)cb, L, L0);
                float ms = 0.f;
                rc = tune_batch(ctx, k0, size, st, 3, &ms);
                if (rc != PMK_OK) break;
                if (ms < (L == L0 ? 1.0f : 0.99f) * lbest) {
                    lbest = ms;
                    best_fill = L;
                }
            }
            (void)pmk_set_lanes(ctx, (uint32_t)cb, best_fill, L0);
        }
        if (rc == PMK_OK && lanes_half(cb) == 1) {
            const uint64_t resident = wave_slots(c, 1, ctx->num_cus);  // one-lane waves, 2 per tile
            const uint64_t sizes[2] = {std::max<uint64_t>(1, (uint64_t)ctx->num_cus / 4),
                                       std::max<uint64_t>(1, resident * 2 / 3)};
            for (int which = 0; which < 2 && rc == PMK_OK; ++which) {
                float lbest = 1e30f;
                int lpick = 1;
                for (int L : {1, 2, 4, 8}) {
                    if (L == 8 && (which == 1 || !eight_lanes(cb))) continue;  // fill only, where supported
                    (void)pmk_set_lanes(ctx, (uint32_t)cb, which == 0 ? L : best_fill, which == 0 ? best_tail : L);
                    float ms = 0.f;
                    rc = tune_batch(ctx, k0, sizes[which], st, 3, &ms);
                    if (rc != PMK_OK) break;
                    if (ms < (L == 1 ? 1.0f : 0.99f) * lbest) {
                        lbest = ms;
                        lpick = L;
                    }
                }
                (which == 0 ? best_fill : best_tail) = lpick;
            }
            (void)pmk_set_lanes(ctx, (uint32_t)cb, best_fill, best_tail);
        }
        if (rc == PMK_OK) {
            std::snprintf(line, sizeof line, "%d %d %d %d %.4f\n", cb, best_w, best_fill, best_tail, best_ms);
            report += line;
        }
    }
    (void)hipStreamDestroy(st);
    if (rc != PMK_OK) return rc;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (!f) return set_err(ctx, PMK_EINVAL, "cannot write autotune cache %s", cache_path);
        std::fputs(report.c_str(), f);
        std::fclose(f);
    }
    return PMK_OK;
}

static int prime_args(pmk_ctx *ctx, uint32_t bits, const void *cand, uint32_t count, const void *out, int *cls) {
    if (!ctx) return PMK_EINVAL;
    const int c = class_for_bits(bits);
    if (c < 0 || kClassBits[c] != (int)bits || !prime_class_ok(c))
        return set_err(ctx, PMK_EUNSUPPORTED, "primality tests take candidates for 1024-, 2048-, 3072- or 4096-bit keys");
    if (count && (!cand || !out)) return set_err(ctx, PMK_EINVAL, "NULL buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    *cls = c;
    return PMK_OK;
}

int pmk_sieve(pmk_ctx *ctx, uint32_t bits, const uint32_t *d_cand, uint32_t count, uint32_t *d_flags, void *stream) {
    int c = 0;
    const int rc = prime_args(ctx, bits, d_cand, count, d_flags, &c);
    if (rc != PMK_OK || count == 0) return rc;
    const int e = launch_sieve_class(c, d_cand, count, d_flags, ctx->device, stream);
    return e ? hip_err(ctx, (hipError_t)e, "sieve launch") : PMK_OK;
}

int pmk_miller_rabin(pmk_ctx *ctx, uint32_t bits, const uint32_t *d_cand, uint32_t count, const uint32_t *d_bases,
                     uint32_t rounds, uint32_t *d_result, void *stream) {
    int c = 0;
    int rc = prime_args(ctx, bits, d_cand, count, d_result, &c);
    if (rc != PMK_OK || count == 0) return rc;
    if (!d_bases || rounds == 0 || rounds > 256) return set_err(ctx, PMK_EINVAL, "need 1..256 bases per candidate");
    const int win = ctx->win[c];
    const uint32_t units = (count + kTile - 1) / kTile;
    const uint32_t grid = std::max<uint32_t>(1, persistent_grid(units, mr_wave_slots(c, ctx->num_cus), ctx->grid_limit));
    const uint64_t slot = mr_slot_words(c, win);
    const uint64_t need = (uint64_t)grid * slot;
    if (need > ctx->mr_cap) {
        (void)hipDeviceSynchronize();  // earlier tests may still use the old table
        if (ctx->mr_table) (void)hipFree(ctx->mr_table);
        ctx->mr_table = nullptr;
        ctx->mr_cap = 0;
        void *v = nullptr;
        const hipError_t e = hipMalloc(&v, need * sizeof(uint32_t));
        if (e != hipSuccess) return hip_err(ctx, e, "primality test tables");
        ctx->mr_table = (uint32_t *)v;
        ctx->mr_cap = need;
    }
    const int e = launch_mr_class(c, d_cand, count, d_bases, (int)rounds, win, ctx->mr_table, slot, grid, d_result,
                                  stream);
    return e ? hip_err(ctx, (hipError_t)e, "Miller-Rabin launch") : PMK_OK;
}

int pmk_plan_check(pmk_plan *pl, void *stream) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_err(ctx, e, "stream synchronize");
    uint32_t flag = 0;
    e = hipMemcpy(&flag, pl->d_err, sizeof flag, hipMemcpyDeviceToHost);
    if (e == hipSuccess && flag) {
        const uint32_t zero = 0;
        e = hipMemcpy(pl->d_err, &zero, sizeof zero, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_err(ctx, e, "error flag read");
    // a non-invertible blinding block also leaves its chunk's plaintext out of
    // range: the more specific status wins
    if (flag & 2u) return set_err(ctx, PMK_EBLIND, "a blinding block is not invertible modulo N");
    if (flag & 1u)
        return set_err(ctx, PMK_ERANGE, "a ciphertext block is not below its modulus or decrypts wider than its chunk");
    return PMK_OK;
}

int pmk_encrypt(pmk_ctx *ctx, const uint8_t *d_msg, uint64_t msg_len, const uint32_t *key_map, uint64_t nchunks,
                uint8_t *d_ct, uint64_t ct_cap, void *stream) {
    pmk_plan *pl = nullptr;
    uint64_t ct_len = 0;
    int rc = pmk_plan_create(ctx, key_map, nchunks, msg_len, &pl, &ct_len);
    if (rc != PMK_OK) return rc;
    if (ct_cap < ct_len) rc = set_err(ctx, PMK_ESIZE, "ciphertext buffer holds %llu bytes, needs %llu",
                                      (unsigned long long)ct_cap, (unsigned long long)ct_len);
    if (rc == PMK_OK) rc = pmk_encrypt_plan(pl, d_msg, d_ct, stream);
    if (rc == PMK_OK) rc = pmk_plan_check(pl, stream);
    pmk_plan_destroy(pl);
    return rc;
}

int pmk_decrypt(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map, uint64_t nchunks,
                uint8_t *d_msg, uint64_t msg_len, void *stream) {
    pmk_plan *pl = nullptr;
    uint64_t need = 0;
    int rc = pmk_plan_create(ctx, key_map, nchunks, msg_len, &pl, &need);
    if (rc != PMK_OK) return rc;
    if (ct_len != need) rc = set_err(ctx, PMK_ESIZE, "ciphertext has %llu bytes, the plan needs %llu",
                                     (unsigned long long)ct_len, (unsigned long long)need);
    if (rc == PMK_OK) rc = pmk_decrypt_plan(pl, d_ct, d_msg, stream);
    if (rc == PMK_OK) rc = pmk_plan_check(pl, stream);
    pmk_plan_destroy(pl);
    return rc;
}


}  // extern "C"

namespace {

// Slices of a plan's chunk range for the host-buffer forms: `n` contiguous
// runs of chunks of about equal message bytes, each planned on its own (its
// offsets relative to the slice), device copies of the whole input and output,
// and the pipeline's streams and events.
// Cuts of a decryption into slices that each end on a whole round of CRT
// work: a plan of one one-lane class whose slices [0, c_1), [c_1, c_2), ...
// give every key only full tiles and 1, 2, 4, ... rounds of job tiles (one
// job tile per resident wave) -- so slicing adds no partial round, and the
// copies of one slice overlap the kernels of its neighbours.  Empty when the
// key map has no such cuts (then one slice).
std::vector<uint64_t> round_cuts(const pmk_plan *pl) {
    const pmk_ctx *ctx = pl->ctx;
    std::vector<uint64_t> cuts;
    if (pl->nchunks == 0) return cuts;
    const int c = ctx->keys[pl->key_map[0]].cls;
    if (lanes_half(kClassBits[c]) != 1) return cuts;
    for (uint64_t i = 0; i < pl->nchunks; ++i)
        if (ctx->keys[pl->key_map[i]].cls != c) return cuts;
    const uint64_t tiles_per_round = std::max<uint32_t>(1, wave_slots(c, 1, ctx->num_cus) / 2);
    std::vector<uint32_t> cnt(ctx->keys.size(), 0);
    uint64_t tiles = 0, ragged = 0, want = tiles_per_round;
    for (uint64_t i = 0; i < pl->nchunks; ++i) {
        uint32_t &n = cnt[pl->key_map[i]];
        if (n % kTile == 0) {
            ++tiles;
            ++ragged;
        }
        if (++n % kTile == 0) --ragged;
        if (ragged == 0 && tiles == want && i + 1 < pl->nchunks) {
            cuts.push_back(i + 1);
            want = 2 * want + tiles_per_round;  // next slice twice as long
        } else if (tiles > want) {
            want = (tiles / tiles_per_round + 1) * tiles_per_round;  // no cut there: the next round end
        }
    }
    return cuts;
}

// Host pipeline of a plan: its chunks cut into slices -- n slices of about
// equal message bytes, or (n = 0) the round cuts of a decryption -- each
// planned on its own (offsets relative to the slice), per direction; device
// copies of the whole input and output, and the pipeline's streams.
int host_prepare(pmk_plan *pl, int decrypt, uint32_t n) {
    pmk_ctx *ctx = pl->ctx;
    if (!pl->hp_in) {
        hipError_t e = dev_alloc(pl, &pl->hp_in, pl->ct_len);  // ct_len >= msg_len
        if (e == hipSuccess) e = dev_alloc(pl, &pl->hp_out, pl->ct_len);
        for (int i = 0; i < pmk_plan::kPipe && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&pl->hp_stream[i], hipStreamNonBlocking);
        if (e != hipSuccess) return hip_err(ctx, e, "host pipeline setup");
    }
    pmk_plan::HostSlices &h = pl->hp[decrypt ? 1 : 0];
    const uint32_t key = n ? n : UINT32_MAX;  // n of the round cuts
    if (h.n == key) return PMK_OK;
    (void)hipDeviceSynchronize();
    for (pmk_plan *s : h.sub) pmk_plan_destroy(s);
    for (hipEvent_t ev : h.ev) (void)hipEventDestroy(ev);
    h = pmk_plan::HostSlices{};
    h.chunk.assign(1, 0);
    h.msg.assign(1, 0);
    h.ct.assign(1, 0);
    const std::vector<uint64_t> cuts = n ? std::vector<uint64_t>() : round_cuts(pl);
    size_t next_cut = 0;
    uint64_t off = 0, ct = 0;
    for (uint64_t i = 0; i < pl->nchunks; ++i) {
        const uint32_t kb = ctx->keys[pl->key_map[i]].bits / 8;
        off += std::min<uint64_t>(kb - 4, pl->msg_len - off);
        ct += kb;
        bool cut = false;
        if (n) {
            const uint64_t s = h.chunk.size();  // next cut: s / n of the message
            cut = s < n && off * n >= s * pl->msg_len;
        } else {
            cut = next_cut < cuts.size() && cuts[next_cut] == i + 1;
            if (cut) ++next_cut;
        }
        if (cut) {
            h.chunk.push_back(i + 1);
            h.msg.push_back(off);
            h.ct.push_back(ct);
        }
    }
    if (h.chunk.back() != pl->nchunks) {
        h.chunk.push_back(pl->nchunks);
        h.msg.push_back(off);
        h.ct.push_back(ct);
    }
    const size_t ns = h.chunk.size() - 1;
    for (size_t s = 0; s < ns; ++s) {
        pmk_plan *sub = nullptr;
        const int rc = pmk_plan_create(ctx, pl->key_map.data() + h.chunk[s], h.chunk[s + 1] - h.chunk[s],
                                       h.msg[s + 1] - h.msg[s], &sub, nullptr);
        if (rc != PMK_OK) return rc;
        h.sub.push_back(sub);
        for (int k = 0; k < 2; ++k) {
            hipEvent_t ev = nullptr;
            const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_err(ctx, e, "host pipeline events");
            h.ev.push_back(ev);
        }
    }
    h.n = key;
    return PMK_OK;
}

// The paper's transfer / compute pipeline over host buffers: slice s is copied
// to the device, computed, and copied back, on three streams, so copies of one
// slice overlap the computation of another.
int host_run(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, uint32_t slices) {
    if (!pl) return PMK_EINVAL;
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!in || !out) return set_err(ctx, PMK_EINVAL, "NULL buffer");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    // default: decryption cut at whole rounds of CRT work (round_cuts; one
    // slice when the key map has no such cuts), encryption in up to four
    // slices of equal bytes, each large enough to fill the chip
    uint32_t n = slices ? slices : (decrypt ? 0u : (uint32_t)std::min<uint64_t>(4, std::max<uint64_t>(1, pl->nchunks / 65536)));
    n = (uint32_t)std::min<uint64_t>(n, pl->nchunks);
    int rc = host_prepare(pl, decrypt, n);
    if (rc != PMK_OK) return rc;
    pmk_plan::HostSlices &h = pl->hp[decrypt ? 1 : 0];
    const bool blocks = decrypt && pl->dec_mode == 2;
    const std::vector<uint64_t> &in_off = decrypt ? h.ct : h.msg;
    const std::vector<uint64_t> &out_off = (decrypt && !blocks) ? h.msg : h.ct;
    hipStream_t cin = pl->hp_stream[0], comp = pl->hp_stream[1], cout = pl->hp_stream[2];
    hipError_t e = hipSuccess;
    for (size_t s = 0; s < h.sub.size() && rc == PMK_OK && e == hipSuccess; ++s) {
        pmk_plan *sub = h.sub[s];
        sub->dec_mode = pl->dec_mode;
        const uint64_t ib = in_off[s], il = in_off[s + 1] - ib, ob = out_off[s], ol = out_off[s + 1] - ob;
        e = hipMemcpyAsync(pl->hp_in + ib, in + ib, il, hipMemcpyHostToDevice, cin);
        if (e == hipSuccess) e = hipEventRecord(h.ev[2 * s], cin);
        if (e == hipSuccess) e = hipStreamWaitEvent(comp, h.ev[2 * s], 0);
        if (e != hipSuccess) break;
        rc = decrypt ? pmk_decrypt_plan(sub, pl->hp_in + ib, pl->hp_out + ob, comp)
                     : pmk_encrypt_plan(sub, pl->hp_in + ib, pl->hp_out + ob, comp);
        if (rc != PMK_OK) break;
        e = hipEventRecord(h.ev[2 * s + 1], comp);
        if (e == hipSuccess) e = hipStreamWaitEvent(cout, h.ev[2 * s + 1], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(out + ob, pl->hp_out + ob, ol, hipMemcpyDeviceToHost, cout);
    }
    const hipError_t e1 = hipStreamSynchronize(cin), e2 = hipStreamSynchronize(comp), e3 = hipStreamSynchronize(cout);
    if (rc != PMK_OK) return rc;
    if (e == hipSuccess) e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
    if (e != hipSuccess) return hip_err(ctx, e, "host pipeline");
    // device-detected errors of every slice (PMK_EBLIND cannot occur here)
    for (pmk_plan *sub : h.sub) {
        const int c = pmk_plan_check(sub, comp);
        if (c != PMK_OK) rc = rc == PMK_OK ? c : rc;
    }
    return rc;
}

}  // namespace

extern "C" {

int pmk_encrypt_host(pmk_plan *plan, const uint8_t *msg, uint8_t *ct, uint32_t slices) {
    return host_run(plan, 0, msg, ct, slices);
}

int pmk_decrypt_host(pmk_plan *plan, const uint8_t *ct, uint8_t *msg, uint32_t slices) {
    return host_run(plan, 1, ct, msg, slices);
}

}  // extern "C"
