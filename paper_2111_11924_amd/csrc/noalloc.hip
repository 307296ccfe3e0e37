// CRT decryption without any allocation (pmk_decrypt_noalloc): the one-shot
// pmk_decrypt with every device buffer its kernels need -- chunk descriptors,
// packed input and output words, CRT half results, window tables, the error
// word -- placed in one fixed device array per GPU, and its host-side
// planning done in buffers the context sized at pmk_create / pmk_keys_load.
// For callers that cannot allocate while they run.
//
// The array's name is a host-side stand-in in host code: its device address
// is taken once per device with hipGetSymbolAddress (at pmk_create, with that
// device current) and only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "pmk_state.hpp"

namespace pmk {
namespace {

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (null: not yet taken)

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

int noalloc_setup(pmk_ctx *ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return PMK_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[ctx->device]) {
        void *p = nullptr;
        // the caller (pmk_create) made ctx->device current
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return PMK_EDEVICE;
        g_ptr[ctx->device] = p;
    }
    ctx->na_scratch = (uint8_t *)g_ptr[ctx->device];
    return PMK_OK;
}

// Host planning buffers for the key table just loaded: per-key counters and a
// pinned mirror of the descriptor region (at most kNoAllocMaxChunks chunks,
// each key's last tile padded).
int noalloc_keys(pmk_ctx *ctx) {
    const size_t nk = ctx->keys.size();
    ctx->na_bits.resize(nk);
    for (size_t i = 0; i < nk; ++i) ctx->na_bits[i] = ctx->keys[i].bits;
    ctx->na_count.assign(nk, 0);
    ctx->na_tile.assign(nk, 0);
    // padded slots over all classes <= chunks + 63 per key; per class two
    // aligned arrays (descriptors, one tile key per 64 slots) after the error word
    const uint64_t slots = kNoAllocMaxChunks + (uint64_t)(kTile - 1) * nk;
    const uint64_t need = kAlign + slots * (sizeof(ChunkDesc) + sizeof(uint32_t)) + 2 * kAlign * kNumClasses;
    if (need > ctx->na_host_bytes) {
        if (ctx->na_host) (void)hipHostFree(ctx->na_host);
        ctx->na_host = nullptr;
        ctx->na_host_bytes = 0;
        void *p = nullptr;
        const hipError_t e = hipHostMalloc(&p, need, hipHostMallocDefault);
        if (e != hipSuccess) return PMK_ENOMEM;
        ctx->na_host = (uint8_t *)p;
        ctx->na_host_bytes = need;
    }
    return PMK_OK;
}

}  // namespace pmk

using namespace pmk;

extern "C" {

int pmk_decrypt_noalloc(pmk_ctx *ctx, const uint8_t *d_ct, uint64_t ct_len, const uint32_t *key_map,
                        uint64_t nchunks, uint8_t *d_msg, uint64_t msg_len, void *stream) {
    if (!ctx) return PMK_EINVAL;
    if (!ctx->na_scratch) return set_err(ctx, PMK_EDEVICE, "the static scratch of this device is not available");
    if (nchunks > kNoAllocMaxChunks)
        return set_err(ctx, PMK_ESIZE, "%llu chunks: the allocation-free decryption takes at most %llu",
                       (unsigned long long)nchunks, (unsigned long long)kNoAllocMaxChunks);
    const uint32_t nk = (uint32_t)ctx->keys.size();
    if (ctx->na_bits.size() != nk) return set_err(ctx, PMK_EINVAL, "no key table loaded");
    // pass 1: validate, count chunks per key
    std::fill(ctx->na_count.begin(), ctx->na_count.end(), 0u);
    uint64_t need_ct = 0;
    int rc = walk_chunks(ctx->na_bits.data(), nk, key_map, nchunks, msg_len, &need_ct, nullptr,
                         [&](uint64_t, uint32_t k, uint64_t, uint64_t, uint64_t) { ctx->na_count[k]++; });
    if (rc != PMK_OK) return set_err(ctx, rc, "chunk plan does not match the message or the key table");
    if (ct_len != need_ct)
        return set_err(ctx, PMK_ESIZE, "ciphertext has %llu bytes, the chunks need %llu", (unsigned long long)ct_len,
                       (unsigned long long)need_ct);
    if (msg_len == 0) return PMK_OK;
    if (!d_ct || !d_msg || ((uintptr_t)d_ct & 3u) || ((uintptr_t)d_msg & 3u))
        return set_err(ctx, PMK_EINVAL, "buffers must be non-NULL and 4-byte aligned");
    // tiles per class, first tile of each key within its class
    uint32_t tiles[kNumClasses] = {};
    for (uint32_t k = 0; k < nk; ++k) {
        const int c = ctx->keys[k].cls;
        ctx->na_tile[k] = tiles[c];
        tiles[c] += (ctx->na_count[k] + kTile - 1) / kTile;
    }
    // scratch layout: error word; per class descriptors and tile keys (this
    // prefix mirrors the pinned host buffer); per class packed words, results,
    // CRT halves; per class window tables
    uint64_t off_desc[kNumClasses] = {}, off_tk[kNumClasses] = {}, off_x[kNumClasses] = {}, off_y[kNumClasses] = {},
             off_h[kNumClasses] = {}, off_t[kNumClasses] = {};
    uint64_t o = kAlign;  // [0, 4): the error word
    int present = 0;
    for (int c = 0; c < kNumClasses; ++c) {
        if (!tiles[c]) continue;
        ++present;
        off_desc[c] = o;
        o += align_up((uint64_t)tiles[c] * kTile * sizeof(ChunkDesc));
        off_tk[c] = o;
        o += align_up((uint64_t)tiles[c] * sizeof(uint32_t));
    }
    const uint64_t prefix = o;
    for (int c = 0; c < kNumClasses; ++c) {
        if (!tiles[c]) continue;
        const Geom g = make_geom(kClassBits[c]);
        off_x[c] = o;
        o += align_up((uint64_t)tiles[c] * g.S * kTile * 4);
        off_y[c] = o;
        o += align_up((uint64_t)tiles[c] * g.S * kTile * 4);
        off_h[c] = o;
        o += align_up((uint64_t)tiles[c] * 2 * g.nlh * kTile * 4);
    }
    if (prefix > ctx->na_host_bytes || o >= kNoAllocScratchBytes)
        return set_err(ctx, PMK_ESIZE, "the chunks need %llu bytes of scratch, the static scratch holds %llu",
                       (unsigned long long)o, (unsigned long long)kNoAllocScratchBytes);
    // window tables: what is left, shared evenly by the classes present; each
    // class gets at most its occupancy and its unit count in wave slots
    const uint64_t share = (kNoAllocScratchBytes - o) / (uint64_t)present;
    uint32_t slots[kNumClasses] = {};
    for (int c = 0; c < kNumClasses; ++c) {
        if (!tiles[c]) continue;
        const uint64_t slot_bytes = table_words_per_slot(c, 1, ctx->win[c]) * 4;
        const uint64_t fit = share / slot_bytes;
        slots[c] = (uint32_t)std::min<uint64_t>({fit, wave_slots(c, 1, ctx->num_cus), exp_units(c, 1, tiles[c])});
        if (!slots[c])
            return set_err(ctx, PMK_ESIZE, "no room left in the static scratch for a %d-bit window table",
                           kClassBits[c]);
        off_t[c] = o;
        o += align_up((uint64_t)slots[c] * slot_bytes);
    }
    if (o > kNoAllocScratchBytes)  // (table slots are whole multiples of 256 bytes: not reached)
        return set_err(ctx, PMK_ESIZE, "the window tables do not fit the static scratch");
    // pass 2: descriptors into the pinned mirror, grouped per key into tiles
    uint8_t *h = ctx->na_host;
    std::fill(ctx->na_count.begin(), ctx->na_count.end(), 0u);  // now: chunks placed per key
    (void)walk_chunks(ctx->na_bits.data(), nk, key_map, nchunks, msg_len, nullptr, nullptr,
                      [&](uint64_t, uint32_t k, uint64_t off, uint64_t len, uint64_t ct) {
                          const KeySlot &ks = ctx->keys[k];
                          ChunkDesc *d = (ChunkDesc *)(h + off_desc[ks.cls]);
                          d[(uint64_t)ctx->na_tile[k] * kTile + ctx->na_count[k]++] =
                              ChunkDesc{off, ct, ks.slot, (uint32_t)len};
                      });
    for (uint32_t k = 0; k < nk; ++k) {
        const uint32_t n = ctx->na_count[k];
        if (!n) continue;
        const KeySlot &ks = ctx->keys[k];
        ChunkDesc *d = (ChunkDesc *)(h + off_desc[ks.cls]) + (uint64_t)ctx->na_tile[k] * kTile;
        uint32_t *tk = (uint32_t *)(h + off_tk[ks.cls]) + ctx->na_tile[k];
        const uint32_t nt = (n + kTile - 1) / kTile;
        for (uint32_t t = 0; t < nt; ++t) tk[t] = ks.slot;
        for (uint32_t i = n; i < nt * kTile; ++i) d[i] = ChunkDesc{0, 0, ks.slot, 0};  // padding slots
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    uint8_t *base = ctx->na_scratch;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *d_err = (uint32_t *)base;
    // the descriptor prefix (after the error word) in one copy; the error word
    // cleared by a kernel
    hipError_t e = hipMemcpyAsync(base + kAlign, h + kAlign, prefix - kAlign, hipMemcpyHostToDevice, s);
    int le = e == hipSuccess ? launch_counter_reset(d_err, s) : 0;
    for (int c = 0; c < kNumClasses && e == hipSuccess && !le; ++c) {
        if (!tiles[c]) continue;
        ClassRun r{};
        r.cls = c;
        r.ntiles = tiles[c];
        r.keys = ctx->d_keys[c];
        r.desc = (const ChunkDesc *)(base + off_desc[c]);
        r.tile_key = (const uint32_t *)(base + off_tk[c]);
        r.x32 = (uint32_t *)(base + off_x[c]);
        r.y32 = (uint32_t *)(base + off_y[c]);
        r.half = (uint32_t *)(base + off_h[c]);
        r.table = (uint32_t *)(base + off_t[c]);
        r.slots_dec = slots[c];
        r.slots_enc = 0;
        r.err = d_err;
        r.grid_cap = ctx->grid_limit;
        r.win = ctx->win[c];
        r.fill_lanes = ctx->fill_lanes[c];
        r.tail_lanes = ctx->tail_lanes[c];
        le = launch_pack(r, d_ct, 1, s);
        if (!le) le = launch_decrypt_halves(r, s);
        if (!le) le = launch_garner(r, s);
        if (!le) le = launch_unpack(r, d_msg, 1, s);
    }
    if (e == hipSuccess && le) e = (hipError_t)le;
    uint32_t *h_flag = (uint32_t *)h;  // the mirror's first word stands for the error word
    if (e == hipSuccess) e = hipMemcpyAsync(h_flag, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    // the pinned mirror is reused by the next call: wait for every copy
    const hipError_t se = hipStreamSynchronize(s);
    if (e == hipSuccess) e = se;
    if (e != hipSuccess) return hip_err(ctx, e, "allocation-free decryption");
    if (*h_flag & 1u)
        return set_err(ctx, PMK_ERANGE, "a ciphertext block is not below its modulus or decrypts wider than its chunk");
    return PMK_OK;
}

}  // extern "C"
