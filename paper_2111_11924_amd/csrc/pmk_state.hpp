// Host-side state of the library (context and plan) and the helpers the
// API and the request server share.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <set>
#include <string>
#include <vector>

#include "../../include/pmk.h"
#include "pmk_internal.hpp"

namespace pmk {
struct Server;
// pmk_decrypt_noalloc: size of the fixed device array holding all its scratch
// (one per GPU, for the life of the process), and its chunk limit
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
constexpr uint64_t kNoAllocMaxChunks = 65536;
}
using pmk::ClassRun;
using pmk::kNumClasses;
using pmk::kWideClasses;

struct KeySlot {
    int cls;
    uint32_t slot;  // record index within the class table
    uint32_t bits;
    std::vector<uint32_t> n;  // modulus, little-endian limbs (host copy)
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
    // lanes per number of the CRT halves where a launch leaves the chip idle:
    // a launch of at most half a round, and a short last round (1: off)
    int fill_lanes[kNumClasses] = {}, tail_lanes[kNumClasses] = {};
    uint32_t epoch = 0;         // bumped when a tuning choice changes (captured graphs go stale)
    uint32_t grid_limit = 0;    // pmk_set_grid_limit: most resident waves per persistent launch (0: none)
    std::string device_name;
    pmk::Server *server = nullptr;  // request server (pmk_server_start), if running
    uint32_t *mr_table = nullptr;   // window tables of the primality tests
    uint64_t mr_cap = 0;            // words at mr_table
    // multi-prime key table (pmk_mp_keys_load): records per class (3072 / 4096 bits)
    std::vector<KeySlot> mp_keys;
    uint32_t *d_mp_keys[2] = {};
    void *mp_scratch = nullptr;  // device arena of pmk_mp_decrypt (grown on demand)
    uint64_t mp_scratch_bytes = 0;
    // pmk_decrypt_noalloc: the device address of this GPU's static scratch
    // (taken at pmk_create) and host planning buffers sized at pmk_keys_load
    uint8_t *na_scratch = nullptr;
    std::vector<uint32_t> na_bits, na_count, na_tile;  // per key: modulus bits, chunks, first tile
    uint8_t *na_host = nullptr;  // pinned mirror of the scratch's descriptor region
    uint64_t na_host_bytes = 0;
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
    uint64_t batch_cap = 0;            // words allocated at batch_table
    uint64_t table_cap[kNumClasses] = {};  // words allocated at runs[c].table
    uint32_t batch_slots = 0;          // its resident waves
    CapturedGraph graph[2];                         // [0] encrypt, [1] decrypt
    static constexpr int kSide = 3;  // side streams of the batched sequence
    hipStream_t capture_stream = nullptr, side_stream[kSide] = {};
    hipEvent_t fork_event = nullptr, join_event[kSide] = {};
    // blinded PMKRSA: tiles of the c_R blocks (allocated on first use)
    uint32_t *x32b[kNumClasses] = {};
    bool blind_ready = false;
    int dec_mode = 1;  // unpack mode of decryptions: 1 plaintext chunks, 2 whole blocks
    // host-buffer forms (pmk_encrypt_host / pmk_decrypt_host), made on first use
    std::vector<uint32_t> key_map;      // the chunk-to-key map the plan was made from
    uint8_t *hp_in = nullptr, *hp_out = nullptr;  // device copies of the whole input / output
    // the slices of one direction (kept apart, so alternating encryption and
    // decryption does not re-plan)
    struct HostSlices {
        std::vector<pmk_plan *> sub;         // one plan per slice of the chunk range
        uint32_t n = 0;                      // slicing they were made for (0: none yet)
        std::vector<uint64_t> chunk, msg, ct;  // slice boundaries: chunk, message and ciphertext offsets
        std::vector<hipEvent_t> ev;          // per slice: input copied, slice computed
    };
    HostSlices hp[2];                   // [0] encryption, [1] decryption
    static constexpr int kPipe = 3;     // streams: host-to-device copies, compute, device-to-host copies
    hipStream_t hp_stream[kPipe] = {};
};

namespace pmk {

// Records a message on the context and returns `code`.
int set_err(pmk_ctx *ctx, int code, const char *fmt, ...);
// Maps a HIP error to a status (PMK_ENOMEM or PMK_EDEVICE) with a message.
int hip_err(pmk_ctx *ctx, hipError_t e, const char *where);

template <typename T>
hipError_t dev_alloc(pmk_plan *pl, T **p, size_t bytes) {
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, bytes ? bytes : 4);
    if (e == hipSuccess) pl->allocs.push_back(v);
    *p = (T *)v;
    return e;
}

void drop_timings(pmk_plan *pl);
void drop_graphs(pmk_plan *pl);
void free_plan_memory(pmk_plan *pl);
// Grows a plan-owned device buffer to at least `need` words (device-synchronous
// when it reallocates; captured graphs are dropped).
hipError_t regrow(pmk_plan *pl, uint32_t **p, uint64_t &cap, uint64_t need);
// Window tables of every class of the plan, sized for the context's windows.
hipError_t ensure_tables(pmk_plan *pl);
// Scratch of the batched path (counter, streams, events) and its table.
int batch_prepare(pmk_plan *pl);
hipError_t ensure_batch_table(pmk_plan *pl);
// One uncaptured pass of the batched launch sequence; returns a hipError_t.
int batch_sequence(pmk_plan *pl, int decrypt, const uint8_t *in, uint8_t *out, void *stream);
// Stops and frees the request server of a context (server.cpp).
void server_shutdown(pmk_ctx *ctx);
// pmk_decrypt_noalloc set-up (noalloc.hip): the device address of the static
// scratch on ctx->device (current), once per device; and the host planning
// buffers for the loaded key table.  Return a status.
int noalloc_setup(pmk_ctx *ctx);
int noalloc_keys(pmk_ctx *ctx);

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

}  // namespace pmk
