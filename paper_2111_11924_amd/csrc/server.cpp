// Request server: a scheduler thread that serves encryption and CRT-decryption
// requests of any size against the context's device-resident key table, with
// continuous tile-level batching.  The paper runs its chunk loops in parallel
// and streams data through a transfer/compute pipeline (Sec. 3.1, Algorithm 1,
// and the implementation steps of Sec. 3.3); here each request's chunks join
// batching rounds as soon as the request is admitted, and a round mixes the
// chunks of every in-flight request (chunks under one key share tiles).
//
// Loop of the scheduler thread:
//   1. Build a round: each in-flight request contributes up to a fair share of
//      the round's chunk budget (so small requests finish within a round or two
//      while large ones continue over several); chunks are grouped per key into
//      tiles and the descriptors uploaded.
//   2. Launch the round (the batched launch sequence: encryption and
//      decryption passes) on the compute stream.
//   3. Admit queued requests in arrival order as long as the staging slab has
//      room for their input and output: the input goes into a pinned host
//      mirror of the slab and from there to the device on the copy stream,
//      asynchronously; the next round's launch waits for those copies on the
//      device, not on the host.
//   4. Deliver what earlier rounds finished (their device-to-host copies ran
//      on the copy stream beside the current round): results into the
//      requests' host buffers, staging released.
//   5. Wait for the round; queue the device-to-host copies of the requests it
//      completed; release their input staging.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "pmk_state.hpp"

namespace pmk {
namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t kAlign = 256;

// First-fit allocator over the device staging slab (offsets only).
class Slab {
public:
    void reset(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t n, uint64_t *off) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const uint64_t rest = it->second - n, start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
};

struct Chunk {
    uint64_t msg_off, ct_off;  // within the request's message / ciphertext
    uint32_t key;              // key index
    uint32_t len;              // plaintext bytes
};

struct Request {
    uint64_t ticket = 0;
    int op = 0;
    const uint8_t *in = nullptr;
    uint8_t *out = nullptr;
    uint64_t msg_len = 0, ct_len = 0, in_len = 0, out_len = 0;
    std::vector<Chunk> chunks;
    uint64_t next = 0;         // chunks handed to rounds
    uint64_t done_chunks = 0;  // chunks whose rounds have finished
    uint64_t in_off = 0, out_off = 0;
    int state = PMK_REQ_QUEUED, status = PMK_OK;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
};

// Device storage of one direction's rounds: a plan whose per-class buffers
// grow to the largest round seen and are refilled every round.
struct RoundPlan {
    pmk_plan pl;
    uint64_t cap_tiles[kNumClasses] = {};
    ChunkDesc *desc[kNumClasses] = {};
    uint32_t *tkey[kNumClasses] = {};
    uint8_t *slot_err[kNumClasses] = {};  // decryption: chunks rejected by unpacking, per slot
    std::vector<ChunkDesc> h_desc[kNumClasses];
    std::vector<uint32_t> h_tkey[kNumClasses];
    std::vector<Request *> h_req[kNumClasses];  // request of each descriptor slot (nullptr: padding)
};

// Per-round bookkeeping: which chunks of which request went into the round.
struct Taken {
    Request *req;
    uint64_t first, count;
};

// A launched round: its slot (device buffers), chunks per direction, completion event.
struct Round {
    int slot;
    std::vector<Taken> taken[2];
    uint64_t t0;
};

}  // namespace

struct Server {
    pmk_ctx *ctx = nullptr;
    pmk_server_cfg cfg{};
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;                    // submitted, not admitted
    std::vector<Request *> inflight;                // admitted, not finished (admission order)
    std::unordered_map<uint64_t, Request *> tickets;
    bool stopping = false;
    int fatal = PMK_OK;
    uint64_t next_ticket = 1;
    // device side (scheduler thread only)
    uint8_t *d_slab = nullptr;
    uint8_t *h_slab = nullptr;  // pinned host mirror of d_slab (same offsets)
    Slab slab;
    hipStream_t stream = nullptr, copy_stream = nullptr;
    hipEvent_t in_copied = nullptr;  // the latest admission copies
    bool in_pending = false;         // admitted input the next round's launch must wait for
    // completed requests whose results are on their way to h_slab
    struct Delivery {
        std::vector<Request *> reqs;
        hipEvent_t ev;
    };
    std::deque<Delivery> deliveries;
    std::vector<hipEvent_t> spare_events;
    // two round slots: with pipeline depth 2 the host builds and queues round
    // k+1 while round k runs
    RoundPlan rp[2][2];  // [slot][encrypt, decrypt]
    hipEvent_t round_done[2] = {};
    std::deque<Round> flight;
    pmk_server_stats stats{};
};

namespace {

hipError_t grow_buffer(pmk_plan *pl, void **p, uint64_t &cap_bytes, uint64_t need) {
    if (need <= cap_bytes && *p) return hipSuccess;
    if (*p) {
        for (size_t i = 0; i < pl->allocs.size(); ++i)
            if (pl->allocs[i] == *p) {
                pl->allocs.erase(pl->allocs.begin() + i);
                break;
            }
        (void)hipFree(*p);
        *p = nullptr;
    }
    cap_bytes = 0;
    hipError_t e = dev_alloc(pl, p, need);
    if (e == hipSuccess) cap_bytes = need;
    return e;
}

// Size class storage for `tiles` tiles (grows by half again when short).
hipError_t ensure_class(Server *sv, RoundPlan &R, int c, uint64_t tiles) {
    if (tiles <= R.cap_tiles[c]) return hipSuccess;
    const uint64_t t = std::max<uint64_t>(tiles + tiles / 2, 16);
    const Geom g = make_geom(kClassBits[c]);
    const uint64_t cpt = (uint64_t)chunks_per_tile(kClassBits[c]);
    ClassRun &r = R.pl.runs[c];
    uint64_t cap = 0;
    (void)hipStreamSynchronize(sv->stream);
    hipError_t e = grow_buffer(&R.pl, (void **)&R.desc[c], cap, t * cpt * sizeof(ChunkDesc));
    cap = 0;
    if (e == hipSuccess) e = grow_buffer(&R.pl, (void **)&R.tkey[c], cap, t * sizeof(uint32_t));
    cap = 0;
    if (e == hipSuccess) e = grow_buffer(&R.pl, (void **)&r.x32, cap, t * g.S * cpt * sizeof(uint32_t));
    cap = 0;
    if (e == hipSuccess) e = grow_buffer(&R.pl, (void **)&r.y32, cap, t * g.S * cpt * sizeof(uint32_t));
    cap = 0;
    if (e == hipSuccess) e = grow_buffer(&R.pl, (void **)&r.half, cap, t * 2 * g.nlh * cpt * sizeof(uint32_t));
    cap = 0;
    if (e == hipSuccess) e = grow_buffer(&R.pl, (void **)&R.slot_err[c], cap, t * cpt);
    if (e == hipSuccess) R.cap_tiles[c] = t;
    r.desc = R.desc[c];
    r.tile_key = R.tkey[c];
    return e;
}

// Fills R with the chunks of `taken` (one direction) and launches the round.
// Returns a hipError_t.
int launch_round(Server *sv, RoundPlan &R, int decrypt, const std::vector<Taken> &taken) {
    pmk_ctx *ctx = sv->ctx;
    // chunks grouped per key, in request order (with the request of each)
    std::unordered_map<uint32_t, std::vector<std::pair<ChunkDesc, Request *>>> per_key;
    std::vector<uint32_t> key_order;
    for (const Taken &t : taken) {
        Request *q = t.req;
        for (uint64_t i = t.first; i < t.first + t.count; ++i) {
            const Chunk &ch = q->chunks[i];
            ChunkDesc d;
            d.key = ctx->keys[ch.key].slot;
            d.msg_len = ch.len;
            // the kernels address one base (the slab): input and output regions
            d.msg_off = (decrypt ? q->out_off : q->in_off) + ch.msg_off;
            d.ct_off = (decrypt ? q->in_off : q->out_off) + ch.ct_off;
            auto it = per_key.find(ch.key);
            if (it == per_key.end()) {
                key_order.push_back(ch.key);
                it = per_key.emplace(ch.key, std::vector<std::pair<ChunkDesc, Request *>>()).first;
            }
            it->second.emplace_back(d, q);
        }
    }
    for (int c = 0; c < kNumClasses; ++c) {
        R.h_desc[c].clear();
        R.h_tkey[c].clear();
        R.h_req[c].clear();
        R.pl.runs[c].ntiles = 0;
        R.pl.runs[c].count = 0;
    }
    for (uint32_t k : key_order) {
        const int c = ctx->keys[k].cls;
        const uint32_t slot = ctx->keys[k].slot;
        const size_t cpt = (size_t)chunks_per_tile(kClassBits[c]);
        const auto &list = per_key[k];
        R.pl.runs[c].count += (uint32_t)list.size();
        for (size_t i = 0; i < list.size(); i += cpt) {
            R.h_tkey[c].push_back(slot);
            for (size_t l = 0; l < cpt; ++l) {
                const bool real = i + l < list.size();
                R.h_desc[c].push_back(real ? list[i + l].first : ChunkDesc{0, 0, slot, 0});
                R.h_req[c].push_back(real ? list[i + l].second : nullptr);
            }
        }
    }
    uint32_t units = 0;  // work units of the wide encryption kernel
    for (int c = 0; c < kNumClasses; ++c) {
        ClassRun &r = R.pl.runs[c];
        const uint64_t tiles = R.h_tkey[c].size();
        if (!tiles) continue;
        hipError_t e = ensure_class(sv, R, c, tiles);
        if (e != hipSuccess) return (int)e;
        r.ntiles = (uint32_t)tiles;
        r.keys = ctx->d_keys[c];
        r.err = R.pl.d_err;
        r.slot_err = decrypt ? R.slot_err[c] : nullptr;
        if (decrypt) {
            e = hipMemsetAsync(R.slot_err[c], 0, R.h_desc[c].size(), sv->stream);
            if (e != hipSuccess) return (int)e;
        }
        r.slots_enc = std::max<uint32_t>(1, std::min<uint64_t>(wave_slots(c, 0, ctx->num_cus), exp_units(c, 0, r.ntiles)));
        r.slots_dec = std::max<uint32_t>(1, std::min<uint64_t>(wave_slots(c, 1, ctx->num_cus), exp_units(c, 1, r.ntiles)));
        if (is_wide_class(c)) units += exp_units(c, 0, r.ntiles);
        e = hipMemcpyAsync(R.desc[c], R.h_desc[c].data(), R.h_desc[c].size() * sizeof(ChunkDesc),
                           hipMemcpyHostToDevice, sv->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(R.tkey[c], R.h_tkey[c].data(), tiles * sizeof(uint32_t), hipMemcpyHostToDevice,
                               sv->stream);
        if (e != hipSuccess) return (int)e;
    }
    if (sv->in_pending) {  // admitted input still on its way to the device
        const hipError_t we = hipStreamWaitEvent(sv->stream, sv->in_copied, 0);
        if (we != hipSuccess) return (int)we;
        sv->in_pending = false;
    }
    int rc = batch_prepare(&R.pl);
    if (rc != PMK_OK) return (int)hipErrorOutOfMemory;
    R.pl.batch_slots = std::max<uint32_t>(1, std::min(batch_wave_slots(ctx->num_cus), units));
    hipError_t e = ensure_tables(&R.pl);
    if (e == hipSuccess) e = ensure_batch_table(&R.pl);
    if (e != hipSuccess) return (int)e;
    return batch_sequence(&R.pl, decrypt, sv->d_slab, sv->d_slab, sv->stream);
}

// After a round whose device flag is set: the requests of the decryption
// chunks that unpacking rejected (block out of range) get PMK_ERANGE.
hipError_t name_rejected(RoundPlan &R) {
    std::vector<uint8_t> h;
    for (int c = 0; c < kNumClasses; ++c) {
        const size_t n = R.h_req[c].size();
        if (!n || !R.pl.runs[c].ntiles) continue;
        h.resize(n);
        const hipError_t e = hipMemcpy(h.data(), R.slot_err[c], n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        for (size_t i = 0; i < n; ++i)
            if (h[i] && R.h_req[c][i]) R.h_req[c][i]->status = PMK_ERANGE;
    }
    return hipSuccess;
}

void finish(Server *sv, Request *q, int status) {
    std::lock_guard<std::mutex> lk(sv->mu);
    q->status = status;
    q->state = PMK_REQ_DONE;
    q->t_done = now_ns();
    sv->stats.requests_done++;
    sv->cv_done.notify_all();
}

// Admission: queued requests, in arrival order, while the slab has room.
void admit(Server *sv) {
    for (;;) {
        Request *q = nullptr;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->queue.empty()) return;
            q = sv->queue.front();
        }
        uint64_t in_off = 0, out_off = 0;
        if (!sv->slab.alloc(std::max<uint64_t>(q->in_len, 4), &in_off)) return;
        if (!sv->slab.alloc(std::max<uint64_t>(q->out_len, 4), &out_off)) {
            sv->slab.release(in_off, std::max<uint64_t>(q->in_len, 4));
            return;
        }
        q->in_off = in_off;
        q->out_off = out_off;
        hipError_t e = hipSuccess;
        if (q->in_len) {
            // the region's previous users are done with it (released only after
            // their copies completed)
            std::memcpy(sv->h_slab + in_off, q->in, q->in_len);
            e = hipMemcpyAsync(sv->d_slab + in_off, sv->h_slab + in_off, q->in_len, hipMemcpyHostToDevice,
                               sv->copy_stream);
            if (e == hipSuccess) e = hipEventRecord(sv->in_copied, sv->copy_stream);
            if (e == hipSuccess) sv->in_pending = true;
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->queue.pop_front();
            q->t_admit = now_ns();
            q->state = PMK_REQ_ADMITTED;
        }
        if (e != hipSuccess) {
            sv->slab.release(in_off, std::max<uint64_t>(q->in_len, 4));
            sv->slab.release(out_off, std::max<uint64_t>(q->out_len, 4));
            finish(sv, q, PMK_EDEVICE);
            continue;
        }
        if (q->chunks.empty()) {  // empty message: nothing to compute
            sv->slab.release(in_off, std::max<uint64_t>(q->in_len, 4));
            sv->slab.release(out_off, std::max<uint64_t>(q->out_len, 4));
            finish(sv, q, PMK_OK);
            continue;
        }
        sv->inflight.push_back(q);
    }
}

// Picks the chunks of the next round: a fair share of the budget per
// in-flight request, then what is left in admission order.
void pick_round(Server *sv, std::vector<Taken> out[2]) {
    out[0].clear();
    out[1].clear();
    const uint64_t budget = sv->cfg.round_chunks;
    const size_t n = sv->inflight.size();
    size_t open = 0;  // requests with chunks not yet handed to a round
    for (const Request *q : sv->inflight) open += q->next < q->chunks.size();
    if (!open) return;
    const uint64_t share = std::max<uint64_t>(64, budget / open);
    std::vector<uint64_t> take(n, 0);
    uint64_t used = 0;
    for (size_t i = 0; i < n && used < budget; ++i) {
        const Request *q = sv->inflight[i];
        take[i] = std::min<uint64_t>({share, q->chunks.size() - q->next, budget - used});
        used += take[i];
    }
    for (size_t i = 0; i < n && used < budget; ++i) {
        const Request *q = sv->inflight[i];
        const uint64_t more = std::min<uint64_t>(q->chunks.size() - q->next - take[i], budget - used);
        take[i] += more;
        used += more;
    }
    for (size_t i = 0; i < n; ++i) {
        Request *q = sv->inflight[i];
        if (!take[i]) continue;
        out[q->op == PMK_OP_DECRYPT ? 1 : 0].push_back(Taken{q, q->next, take[i]});
        q->next += take[i];
    }
}

void fail_all(Server *sv, int status) {
    for (Request *q : sv->inflight) finish(sv, q, status);
    sv->inflight.clear();
    for (auto &d : sv->deliveries) {
        for (Request *q : d.reqs) finish(sv, q, status);
        if (d.ev) sv->spare_events.push_back(d.ev);
    }
    sv->deliveries.clear();
    sv->flight.clear();
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->fatal = status;
}

// Waits for the oldest launched round and completes what it finished.
// Returns a hipError_t.
int complete_round(Server *sv) {
    Round r = std::move(sv->flight.front());
    sv->flight.pop_front();
    int e = (int)hipEventSynchronize(sv->round_done[r.slot]);
    // device range flag of the decryption part
    uint32_t flag = 0;
    if (!e && !r.taken[1].empty()) {
        e = (int)hipMemcpy(&flag, sv->rp[r.slot][1].pl.d_err, sizeof flag, hipMemcpyDeviceToHost);
        if (!e && flag) e = (int)hipMemset(sv->rp[r.slot][1].pl.d_err, 0, sizeof flag);
        if (!e && flag) e = (int)name_rejected(sv->rp[r.slot][1]);
    }
    if (e) return e;
    uint64_t chunks = 0;
    for (int d = 0; d < 2; ++d)
        for (const Taken &t : r.taken[d]) {
            chunks += t.count;
            t.req->done_chunks += t.count;
        }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stats.rounds++;
        sv->stats.chunks += chunks;
        sv->stats.busy_ns += now_ns() - r.t0;
    }
    // completed requests: results queued for the host (copy stream), input
    // staging released; the output staging goes with the delivery
    std::vector<Request *> still;
    Server::Delivery d{{}, nullptr};
    for (Request *q : sv->inflight) {
        if (q->done_chunks < q->chunks.size()) {
            still.push_back(q);
            continue;
        }
        if (!e && q->out_len)
            e = (int)hipMemcpyAsync(sv->h_slab + q->out_off, sv->d_slab + q->out_off, q->out_len,
                                    hipMemcpyDeviceToHost, sv->copy_stream);
        sv->slab.release(q->in_off, std::max<uint64_t>(q->in_len, 4));
        d.reqs.push_back(q);
    }
    sv->inflight.swap(still);
    if (!d.reqs.empty()) {
        if (!sv->spare_events.empty()) {
            d.ev = sv->spare_events.back();
            sv->spare_events.pop_back();
        } else if (!e) {
            e = (int)hipEventCreateWithFlags(&d.ev, hipEventDisableTiming);
        }
        if (!e) e = (int)hipEventRecord(d.ev, sv->copy_stream);
        sv->deliveries.push_back(std::move(d));
    }
    return e;
}

// Results of completed requests into their host buffers: each delivery waits
// for its device-to-host copies, then copies out of the pinned mirror.
// Returns whether anything was delivered.
bool deliver(Server *sv) {
    const bool any = !sv->deliveries.empty();
    while (!sv->deliveries.empty()) {
        Server::Delivery d = std::move(sv->deliveries.front());
        sv->deliveries.pop_front();
        const hipError_t e = d.ev ? hipEventSynchronize(d.ev) : hipErrorInvalidValue;
        for (Request *q : d.reqs) {
            if (e == hipSuccess && q->out_len) std::memcpy(q->out, sv->h_slab + q->out_off, q->out_len);
            sv->slab.release(q->out_off, std::max<uint64_t>(q->out_len, 4));
            finish(sv, q, e != hipSuccess ? PMK_EDEVICE : q->status);
        }
        if (d.ev) sv->spare_events.push_back(d.ev);
    }
    return any;
}

void run(Server *sv) {
    pmk_ctx *ctx = sv->ctx;
    (void)hipSetDevice(ctx->device);
    std::vector<Taken> round[2];
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] {
                return sv->stopping || !sv->queue.empty() || !sv->inflight.empty() || !sv->flight.empty() ||
                       !sv->deliveries.empty();
            });
            if (sv->stopping && sv->queue.empty() && sv->inflight.empty() && sv->flight.empty() &&
                sv->deliveries.empty())
                break;
        }
        admit(sv);
        bool launched = false;
        const size_t depth = sv->cfg.pipeline_depth >= 2 ? 2 : 1;
        if (sv->flight.size() < depth) {
            pick_round(sv, round);
            if (!round[0].empty() || !round[1].empty()) {
                const int slot = sv->flight.empty() ? 0 : 1 - sv->flight.front().slot;
                Round r{slot, {}, now_ns()};
                int e = 0;
                for (int d = 0; d < 2 && !e; ++d)
                    if (!round[d].empty()) e = launch_round(sv, sv->rp[slot][d], d, round[d]);
                if (!e) e = (int)hipEventRecord(sv->round_done[slot], sv->stream);
                if (e) {
                    fail_all(sv, PMK_EDEVICE);
                    continue;
                }
                r.taken[0].swap(round[0]);
                r.taken[1].swap(round[1]);
                sv->flight.push_back(std::move(r));
                launched = true;
            }
        }
        // results of earlier rounds while the new one runs (their staging frees up)
        const bool delivered = deliver(sv);
        if (sv->flight.empty()) {
            // nothing runs and nothing can be picked: a queued request larger
            // than the whole free slab can never be admitted (after what was
            // just delivered has released its staging)
            if (sv->inflight.empty() && !delivered) {
                std::unique_lock<std::mutex> lk(sv->mu);
                if (!sv->queue.empty()) {
                    Request *q = sv->queue.front();
                    sv->queue.pop_front();
                    lk.unlock();
                    finish(sv, q, PMK_ESIZE);
                }
            }
            continue;
        }
        if (launched && sv->flight.size() < depth) continue;  // queue a second round first if there is work
        if (complete_round(sv)) fail_all(sv, PMK_EDEVICE);
    }
}

void free_server(Server *sv) {
    for (auto &slot : sv->rp)
        for (auto &R : slot) free_plan_memory(&R.pl);
    for (auto &ev : sv->round_done)
        if (ev) (void)hipEventDestroy(ev);
    if (sv->d_slab) (void)hipFree(sv->d_slab);
    if (sv->h_slab) (void)hipHostFree(sv->h_slab);
    if (sv->in_copied) (void)hipEventDestroy(sv->in_copied);
    for (auto &d : sv->deliveries)
        if (d.ev) (void)hipEventDestroy(d.ev);
    for (hipEvent_t ev : sv->spare_events) (void)hipEventDestroy(ev);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    if (sv->copy_stream) (void)hipStreamDestroy(sv->copy_stream);
    for (auto &kv : sv->tickets) delete kv.second;
    delete sv;
}

}  // namespace

void server_shutdown(pmk_ctx *ctx) {
    Server *sv = ctx ? ctx->server : nullptr;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    if (sv->th.joinable()) sv->th.join();
    ctx->server = nullptr;
    ctx->live_plans--;
    free_server(sv);
}

}  // namespace pmk

using namespace pmk;

extern "C" {

int pmk_server_start(pmk_ctx *ctx, const pmk_server_cfg *cfg) {
    if (!ctx) return PMK_EINVAL;
    if (ctx->server) return set_err(ctx, PMK_EBUSY, "a server is already running on this context");
    if (ctx->keys.empty()) return set_err(ctx, PMK_EINVAL, "the server needs a loaded key table");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, PMK_EDEVICE, "hipSetDevice failed");
    Server *sv = new (std::nothrow) Server();
    if (!sv) return set_err(ctx, PMK_ENOMEM, "server allocation");
    sv->ctx = ctx;
    if (cfg) sv->cfg = *cfg;
    if (!sv->cfg.staging_bytes) sv->cfg.staging_bytes = (uint64_t)512 << 20;
    if (!sv->cfg.round_chunks) {
        // about two chip-filling rounds of 2048-bit CRT halves
        sv->cfg.round_chunks = (uint64_t)wave_slots(4, 1, ctx->num_cus) * kTile;
    }
    hipError_t e = hipMalloc(&sv->d_slab, sv->cfg.staging_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->h_slab, sv->cfg.staging_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->in_copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->copy_stream, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&sv->round_done[i], hipEventDisableTiming);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        pmk_plan &pl = sv->rp[k / 2][k % 2].pl;
        pl.ctx = ctx;
        for (int c = 0; c < kNumClasses; ++c) {
            pl.runs[c].cls = c;
            pl.runs[c].win = ctx->win[c];
        }
        e = dev_alloc(&pl, &pl.d_err, sizeof(uint32_t));
        if (e == hipSuccess) e = hipMemset(pl.d_err, 0, sizeof(uint32_t));
    }
    if (e != hipSuccess) {
        free_server(sv);
        return hip_err(ctx, e, "server setup");
    }
    sv->slab.reset(sv->cfg.staging_bytes);
    ctx->server = sv;
    ctx->live_plans++;  // the key table may not change under the server
    try {
        sv->th = std::thread(run, sv);
    } catch (...) {
        ctx->server = nullptr;
        ctx->live_plans--;
        free_server(sv);
        return set_err(ctx, PMK_ENOMEM, "server thread");
    }
    return PMK_OK;
}

int pmk_server_stop(pmk_ctx *ctx) {
    if (!ctx) return PMK_EINVAL;
    if (!ctx->server) return set_err(ctx, PMK_EINVAL, "no server running");
    server_shutdown(ctx);
    return PMK_OK;
}

int pmk_submit(pmk_ctx *ctx, const pmk_request *req, uint64_t *ticket) {
    if (!ctx || !req || !ticket) return PMK_EINVAL;
    Server *sv = ctx->server;
    if (!sv) return PMK_EINVAL;
    if (req->op != PMK_OP_ENCRYPT && req->op != PMK_OP_DECRYPT) return PMK_EINVAL;
    Request *q = new (std::nothrow) Request();
    if (!q) return PMK_ENOMEM;
    q->op = req->op;
    q->in = req->in;
    q->out = req->out;
    q->msg_len = req->msg_len;
    std::vector<uint32_t> bits(ctx->keys.size());
    for (size_t i = 0; i < bits.size(); ++i) bits[i] = ctx->keys[i].bits;
    uint64_t ct_len = 0;
    const int rc = walk_chunks(bits.data(), (uint32_t)bits.size(), req->key_map, req->nchunks, req->msg_len, &ct_len,
                               nullptr, [&](uint64_t, uint32_t k, uint64_t off, uint64_t len, uint64_t ct) {
                                   q->chunks.push_back(Chunk{off, ct, k, (uint32_t)len});
                               });
    q->ct_len = ct_len;
    q->in_len = q->op == PMK_OP_ENCRYPT ? q->msg_len : q->ct_len;
    q->out_len = q->op == PMK_OP_ENCRYPT ? q->ct_len : q->msg_len;
    int bad = rc;
    if (!bad && q->in_len && (!q->in || !q->out)) bad = PMK_EINVAL;
    if (!bad && req->out_cap < q->out_len) bad = PMK_ESIZE;
    const uint64_t need = (q->in_len + kAlign) / kAlign * kAlign + (q->out_len + kAlign) / kAlign * kAlign;
    if (!bad && need > sv->cfg.staging_bytes) bad = PMK_ESIZE;  // could never be admitted
    if (bad) {
        delete q;
        return bad;
    }
    q->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->fatal || sv->stopping) {
            const int f = sv->fatal ? sv->fatal : PMK_EINVAL;
            delete q;
            return f;
        }
        q->ticket = sv->next_ticket++;
        sv->tickets[q->ticket] = q;
        sv->queue.push_back(q);
        sv->stats.requests_submitted++;
    }
    sv->cv_work.notify_one();
    *ticket = q->ticket;
    return PMK_OK;
}

static int report(Server *sv, uint64_t ticket, pmk_ticket_info *info, bool wait) {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return PMK_EINVAL;
    Request *q = it->second;
    if (wait) sv->cv_done.wait(lk, [&] { return q->state == PMK_REQ_DONE; });
    if (info) {
        info->state = q->state;
        info->status = q->status;
        info->t_submit_ns = q->t_submit;
        info->t_admit_ns = q->t_admit;
        info->t_done_ns = q->t_done;
    }
    if (q->state == PMK_REQ_DONE) {
        sv->tickets.erase(it);
        delete q;
    }
    return PMK_OK;
}

int pmk_poll(pmk_ctx *ctx, uint64_t ticket, pmk_ticket_info *info) {
    if (!ctx || !ctx->server) return PMK_EINVAL;
    return report(ctx->server, ticket, info, false);
}

int pmk_wait(pmk_ctx *ctx, uint64_t ticket, pmk_ticket_info *info) {
    if (!ctx || !ctx->server) return PMK_EINVAL;
    return report(ctx->server, ticket, info, true);
}

int pmk_server_stats_get(pmk_ctx *ctx, pmk_server_stats *out) {
    if (!ctx || !ctx->server || !out) return PMK_EINVAL;
    Server *sv = ctx->server;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->queued = sv->queue.size();
    return PMK_OK;
}

}  // extern "C"
