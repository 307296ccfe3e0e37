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

using namespace pmk;

struct KeySlot {
    int cls;
    uint32_t slot;  // record index within the class table
    uint32_t bits;
};

struct pmk_ctx {
    int device = 0;
    int num_cus = 0;
    std::string err;
    std::vector<KeySlot> keys;
    uint32_t *d_keys[kNumClasses] = {};
    uint32_t class_count[kNumClasses] = {};
    int live_plans = 0;
    std::set<pmk_plan *> plans;
    int win[kNumClasses] = {};  // CRT-halves window width per class
    uint32_t epoch = 0;         // bumped when a tuning choice changes (captured graphs go stale)
    std::string device_name;
};

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

// a captured launch sequence and the buffers / tuning it was captured for
struct CapturedGraph {
    hipGraphExec_t exec = nullptr;
    const void *in = nullptr;
    void *out = nullptr;
    uint32_t epoch = 0;
};

struct pmk_plan {
    pmk_ctx *ctx = nullptr;
    uint64_t msg_len = 0, nchunks = 0, ct_len = 0;
    ClassRun runs[kNumClasses] = {};
    std::vector<void *> allocs;
    uint32_t *d_err = nullptr;
    bool profile = false;
    std::vector<TimedLaunch> timed;
    // batched persistent path (allocated on first use)
    uint32_t *d_counter = nullptr;     // work counter of the wide batch kernel
    uint32_t *batch_table = nullptr;   // its window-table slots
    uint32_t batch_slots[2] = {};      // its resident waves, [encrypt, decrypt]
    uint64_t batch_slot_words = 0;
    CapturedGraph graph[2];                         // [0] encrypt, [1] decrypt
    hipStream_t capture_stream = nullptr, side_stream = nullptr;
    hipEvent_t fork_event = nullptr, join_event = nullptr;
};

namespace {

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

template <typename T>
hipError_t dev_alloc(pmk_plan *pl, T **p, size_t bytes) {
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 4);
    if (e == hipSuccess) pl->allocs.push_back(v);
    *p = (T *)v;
    return e;
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
    if (pl->capture_stream) (void)hipStreamDestroy(pl->capture_stream);
    if (pl->side_stream) (void)hipStreamDestroy(pl->side_stream);
    if (pl->fork_event) (void)hipEventDestroy(pl->fork_event);
    if (pl->join_event) (void)hipEventDestroy(pl->join_event);
    pl->capture_stream = pl->side_stream = nullptr;
    pl->fork_event = pl->join_event = nullptr;
    for (void *p : pl->allocs) (void)hipFree(p);
    pl->allocs.clear();
}

// Runs one launcher; with profiling on, brackets it with events on `stream`.
template <typename F>
int timed_launch(pmk_plan *pl, int kind, void *stream, F launch) {
    if (!pl->profile) return launch();
    TimedLaunch t{kind, nullptr, nullptr};
    if (hipEventCreate(&t.start) != hipSuccess) return (int)hipErrorOutOfMemory;
    if (hipEventCreate(&t.stop) != hipSuccess) {
        (void)hipEventDestroy(t.start);
        return (int)hipErrorOutOfMemory;
    }
    (void)hipEventRecord(t.start, (hipStream_t)stream);
    const int e = launch();
    (void)hipEventRecord(t.stop, (hipStream_t)stream);
    pl->timed.push_back(t);
    return e;
}

// Host-side chunk planning shared by pmk_plan_create and pmk_plan_validate.
// Calls visit(i, key, msg_off, len, ct_off) per chunk; returns status.
template <typename Visit>
int walk_chunks(const uint32_t *key_bits, uint32_t nkeys, const uint32_t *key_map, uint64_t nchunks,
                uint64_t msg_len, uint64_t *ct_len, std::string *why, Visit visit) {
    if (msg_len == 0) {
        if (nchunks != 0) {
            if (why) *why = "empty message needs zero chunks";
            return PMK_ESIZE;
        }
        if (ct_len) *ct_len = 0;
        return PMK_OK;
    }
    if (!key_map) {
        if (why) *why = "key_map is NULL";
        return PMK_EINVAL;
    }
    uint64_t off = 0, ct = 0;
    for (uint64_t i = 0; i < nchunks; ++i) {
        const uint32_t k = key_map[i];
        if (k >= nkeys) {
            if (why) *why = "chunk " + std::to_string(i) + " names key " + std::to_string(k);
            return PMK_EKEY;
        }
        const uint64_t cap = key_bits[k] / 8 - 4;
        if (off >= msg_len) {
            if (why) *why = "more chunks than the message needs";
            return PMK_ESIZE;
        }
        const uint64_t len = std::min<uint64_t>(cap, msg_len - off);
        if (i + 1 == nchunks && off + len != msg_len) {
            if (why) *why = "fewer chunks than the message needs";
            return PMK_ESIZE;
        }
        visit(i, k, off, len, ct);
        off += len;
        ct += key_bits[k] / 8;
    }
    if (nchunks == 0) {
        if (why) *why = "non-empty message needs chunks";
        return PMK_ESIZE;
    }
    if (ct_len) *ct_len = ct;
    return PMK_OK;
}

}  // namespace

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
    for (int c = 0; c < kNumClasses; ++c) ctx->win[c] = window_for(kClassBits[c] / 2);
    *out = ctx;
    return PMK_OK;
}

void pmk_destroy(pmk_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    while (!ctx->plans.empty()) pmk_plan_destroy(*ctx->plans.begin());
    for (auto &p : ctx->d_keys)
        if (p) (void)hipFree(p);
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
        slots[i] = {c, counts[c]++, keys[i].bits};
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
        if (key_bits[i] < 128 || key_bits[i] > 4096 || key_bits[i] % 64) return PMK_EINVAL;
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
        const uint64_t tbl_words = std::max(r.slots_enc * table_words_per_slot(c, 0),
                                            r.slots_dec * table_words_per_slot(c, 1));
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
        if (e == hipSuccess) e = dev_alloc(pl, &r.table, tbl_words * sizeof(uint32_t));
    }
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
    for (int c = 0; c < kNumClasses; ++c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        int e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, d_ct, 1, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_CRT_HALVES, stream, [&] { return launch_decrypt_halves(r, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_GARNER, stream, [&] { return launch_garner(r, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, d_msg, 1, stream); });
        if (e) return hip_err(ctx, (hipError_t)e, "decrypt launch");
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

namespace {

// Launches of one pass of the batched path.  Packing runs on `stream`; then
// the multi-lane classes (4096, 3072 bits) run as one persistent work-queue
// launch on the plan's side stream while the one-lane classes (2048 bits down)
// run their own kernels, largest first, on `stream` (forked and joined with
// events, so the two can share the chip); Garner recombination and unpacking
// follow on `stream`.
int batch_sequence(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, void *stream) {
    pmk_ctx *ctx = pl->ctx;
    BatchArgs a{};
    uint32_t total = 0;
    for (int i = 0; i < kWideClasses; ++i) {
        const int c = wide_class(i);
        a.runs[i] = pl->runs[c];
        a.runs[i].win = ctx->win[c];
        a.start[i] = total;
        total += pl->runs[c].ntiles ? exp_units(c, decrypt, pl->runs[c].ntiles) : 0u;
    }
    a.start[kWideClasses] = total;
    a.counter = pl->d_counter;
    a.table = pl->batch_table;
    a.slot_words = pl->batch_slot_words;
    int e = total ? launch_counter_reset(pl->d_counter, stream) : 0;
    bool narrow = false;
    for (int c = kNumClasses - 1; c >= 0 && !e; --c) {
        ClassRun r = pl->runs[c];
        if (!r.ntiles) continue;
        narrow = narrow || c < kWideFirst;
        e = timed_launch(pl, PMK_KERNEL_PACK, stream, [&] { return launch_pack(r, in, decrypt, stream); });
    }
    const bool fork = !e && total && narrow;
    if (fork) {
        e = hipEventRecord(pl->fork_event, (hipStream_t)stream);
        if (!e) e = hipStreamWaitEvent(pl->side_stream, pl->fork_event, 0);
    }
    if (!e && total) {
        void *s = fork ? (void *)pl->side_stream : stream;
        const uint32_t grid = std::min(total, pl->batch_slots[decrypt]);
        e = timed_launch(pl, PMK_KERNEL_BATCH, s, [&] { return launch_batch(a, decrypt, grid, s); });
    }
    for (int c = kWideFirst - 1; c >= 0 && !e; --c) {
        ClassRun r = pl->runs[c];
        if (!r.ntiles) continue;
        r.win = ctx->win[c];
        e = timed_launch(pl, decrypt ? PMK_KERNEL_CRT_HALVES : PMK_KERNEL_ENCRYPT, stream, [&] {
            return decrypt ? launch_decrypt_halves(r, stream) : launch_encrypt(r, stream);
        });
    }
    if (fork && !e) {
        e = hipEventRecord(pl->join_event, pl->side_stream);
        if (!e) e = hipStreamWaitEvent((hipStream_t)stream, pl->join_event, 0);
    }
    for (int c = kNumClasses - 1; c >= 0 && !e; --c) {
        const ClassRun &r = pl->runs[c];
        if (!r.ntiles) continue;
        if (decrypt) e = timed_launch(pl, PMK_KERNEL_GARNER, stream, [&] { return launch_garner(r, stream); });
        if (!e) e = timed_launch(pl, PMK_KERNEL_UNPACK, stream, [&] { return launch_unpack(r, out, decrypt, stream); });
    }
    return e;
}

int batch_prepare(pmk_plan *pl) {
    if (pl->d_counter) return PMK_OK;
    pmk_ctx *ctx = pl->ctx;
    uint32_t units[2] = {0, 0};
    for (int i = 0; i < kWideClasses; ++i) {
        const int c = wide_class(i);
        for (int d = 0; d < 2; ++d) units[d] += pl->runs[c].ntiles ? exp_units(c, d, pl->runs[c].ntiles) : 0u;
    }
    uint64_t slots = 0;
    for (int d = 0; d < 2; ++d) {
        pl->batch_slots[d] = std::max<uint32_t>(1, std::min(batch_wave_slots(d, ctx->num_cus), units[d]));
        if (units[d]) slots = std::max<uint64_t>(slots, pl->batch_slots[d]);
    }
    pl->batch_slot_words = std::max(batch_slot_words(0), batch_slot_words(1));
    uint32_t *counter = nullptr;
    hipError_t e = dev_alloc(pl, &counter, sizeof(uint32_t));
    if (e == hipSuccess && slots) e = dev_alloc(pl, &pl->batch_table, slots * pl->batch_slot_words * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->side_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork_event, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join_event, hipEventDisableTiming);
    if (e != hipSuccess) return hip_err(ctx, e, "batch scratch allocation");
    pl->d_counter = counter;
    return PMK_OK;
}

int batch_run(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, void *stream) {
    pmk_ctx *ctx = pl->ctx;
    if (pl->msg_len == 0) return PMK_OK;
    if (!in || !out || ((uintptr_t)in & 3u) || ((uintptr_t)out & 3u))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    int rc = batch_prepare(pl);
    if (rc != PMK_OK) return rc;
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

}  // namespace

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
    if (flag) return set_err(ctx, PMK_ERANGE, "a ciphertext block is not below its modulus");
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
