// Continuous-batching server over a reference set resident in HBM.
//
// A request is a batch of query sequences (host ASCII) with a candidate list
// of (query, reference) pairs.  It is admitted only when a slot (a HIP stream
// with its own alignment workspace) is free and its in-flight device state
// fits in what is left of the HBM budget; otherwise submit returns SW_EAGAIN
// and the caller retries when an earlier request completes.  Admitted
// requests run concurrently on their slots' streams: each one is copied in,
// packed and aligned by one persistent launch against the resident set, and
// its results are copied back; the persistent grids of different requests
// share the compute units as their blocks drain.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "sw_internal.h"

using namespace swk;

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit sub-allocator over one device arena; the arena size is the HBM
// budget for in-flight request state.
class Arena {
public:
    bool init(size_t bytes)
    {
        size_ = bytes;
        if (bytes == 0) return true;
        if (hipMalloc(&base_, bytes) != hipSuccess) return false;
        free_[0] = bytes;
        return true;
    }
    void release()
    {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    // returns offset or SIZE_MAX
    size_t alloc(size_t bytes)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void free(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    char* ptr(size_t off) const { return reinterpret_cast<char*>(base_) + off; }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    void* base_ = nullptr;
    size_t size_ = 0;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t ticket = 0;
    int slot = -1;
    size_t dev_off = 0, dev_bytes = 0;
    int64_t n_cand = 0;
    sw_result* out_host = nullptr;
    sw_result* staged = nullptr;  // pinned, inside the slot's staging buffer
    hipEvent_t done = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    char* pinned = nullptr;  // staging for inputs and results
    size_t pinned_bytes = 0;
};

}  // namespace

struct sw_server {
    int device = 0;
    const void* refs_packed = nullptr;
    const int64_t* ref_offsets = nullptr;
    int64_t n_refs = 0;
    sw_scoring scoring{};
    Arena arena;
    std::vector<Slot> slots;
    std::map<uint64_t, Request> inflight;
    uint64_t next_ticket = 1;
    bool shutting_down = false;
    std::mutex mu;
};

namespace {

// Device bytes a request needs: ASCII, packed queries, offsets, pairs, results.
size_t request_bytes(int64_t n_res, int64_t n_q, int64_t n_cand)
{
    return align_up((size_t)n_res) + align_up(sw_packed_bytes(n_res)) + align_up(8 * (size_t)(n_q + 1)) +
           align_up(8 * (size_t)n_cand) + align_up(sizeof(sw_result) * (size_t)n_cand);
}

// Completion of one request: results to the caller, memory and slot freed.
int retire(sw_server* s, Request& r)
{
    hipError_t e = hipEventSynchronize(r.done);
    if (e != hipSuccess) return SW_EDEVICE;
    std::memcpy(r.out_host, r.staged, sizeof(sw_result) * (size_t)r.n_cand);
    (void)hipEventDestroy(r.done);
    s->arena.free(r.dev_off, r.dev_bytes);
    s->slots[r.slot].busy = false;
    return SW_OK;
}

}  // namespace

extern "C" {

SW_API int sw_server_create(const void* refs_packed_dev, const int64_t* ref_offsets_dev, int64_t n_refs,
                            const sw_scoring* scoring, size_t hbm_budget_bytes, int max_slots,
                            sw_server** server)
{
    if (!server || !refs_packed_dev || !ref_offsets_dev || n_refs < 0 || !scoring || max_slots < 1 ||
        max_slots > 64)
        return SW_EINVAL;
    if (scoring->matrix_id != 0 || scoring->gap_open < 1 || scoring->gap_open > (1 << 20) ||
        scoring->gap_extend < 0 || scoring->gap_extend > scoring->gap_open)
        return SW_EINVAL;
    sw_server* s = new sw_server();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return SW_EDEVICE;
    }
    s->refs_packed = refs_packed_dev;
    s->ref_offsets = ref_offsets_dev;
    s->n_refs = n_refs;
    s->scoring = *scoring;
    if (!s->arena.init(hbm_budget_bytes)) {
        delete s;
        return SW_ENOMEM;
    }
    s->slots.resize(max_slots);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            s->arena.release();
            delete s;
            return SW_EDEVICE;
        }
    }
    *server = s;
    return SW_OK;
}

SW_API int sw_server_submit(sw_server* s, const char* q_ascii, const int64_t* q_offsets, int64_t n_q,
                            const int32_t* cand, int64_t n_cand, sw_result* out_host, uint64_t* ticket)
{
    if (!s || !q_offsets || n_q < 0 || n_cand < 0 || !ticket || (n_cand > 0 && (!cand || !out_host)))
        return SW_EINVAL;
    const int64_t n_res = n_q > 0 ? q_offsets[n_q] : 0;
    if (n_res < 0 || (n_res > 0 && !q_ascii)) return SW_EINVAL;
    for (int64_t k = 0; k < n_q; ++k)
        if (q_offsets[k + 1] < q_offsets[k] || q_offsets[k] < 0) return SW_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->shutting_down) return SW_ECANCELED;
    const size_t need = request_bytes(n_res, n_q, n_cand);
    if (need > s->arena.size()) return SW_ENOMEM;  // can never be admitted
    int slot = -1;
    for (int k = 0; k < (int)s->slots.size(); ++k)
        if (!s->slots[k].busy) {
            slot = k;
            break;
        }
    if (slot < 0) return SW_EAGAIN;
    const size_t off = s->arena.alloc(need);
    if (off == SIZE_MAX) return SW_EAGAIN;
    Slot& sl = s->slots[slot];
    if (hipSetDevice(s->device) != hipSuccess) {
        s->arena.free(off, need);
        return SW_EDEVICE;
    }
    // pinned staging: inputs then results
    const size_t in_bytes = align_up((size_t)n_res) + align_up(8 * (size_t)(n_q + 1)) + align_up(8 * (size_t)n_cand);
    const size_t stage = in_bytes + align_up(sizeof(sw_result) * (size_t)n_cand);
    if (stage > sl.pinned_bytes) {
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        sl.pinned_bytes = 0;
        if (hipHostMalloc((void**)&sl.pinned, std::max<size_t>(stage, 1 << 20)) != hipSuccess) {
            s->arena.free(off, need);
            return SW_ENOMEM;
        }
        sl.pinned_bytes = std::max<size_t>(stage, 1 << 20);
    }
    char* p = sl.pinned;
    char* h_ascii = p;
    int64_t* h_offs = reinterpret_cast<int64_t*>(p + align_up((size_t)n_res));
    int32_t* h_pairs = reinterpret_cast<int32_t*>(p + align_up((size_t)n_res) + align_up(8 * (size_t)(n_q + 1)));
    sw_result* h_out = reinterpret_cast<sw_result*>(p + in_bytes);
    if (n_res) std::memcpy(h_ascii, q_ascii, (size_t)n_res);
    std::memcpy(h_offs, q_offsets, 8 * (size_t)(n_q + 1));
    if (n_cand) std::memcpy(h_pairs, cand, 8 * (size_t)n_cand);

    char* d = s->arena.ptr(off);
    char* d_ascii = d;
    char* d_packed = d_ascii + align_up((size_t)n_res);
    int64_t* d_offs = reinterpret_cast<int64_t*>(d_packed + align_up(sw_packed_bytes(n_res)));
    int32_t* d_pairs = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_offs) + align_up(8 * (size_t)(n_q + 1)));
    sw_result* d_out = reinterpret_cast<sw_result*>(reinterpret_cast<char*>(d_pairs) + align_up(8 * (size_t)n_cand));

    hipStream_t st = sl.stream;
    int rc = SW_OK;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(st);
        s->arena.free(off, need);
        return code;
    };
    if (n_res && hipMemcpyAsync(d_ascii, h_ascii, (size_t)n_res, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(SW_EDEVICE);
    if (hipMemcpyAsync(d_offs, h_offs, 8 * (size_t)(n_q + 1), hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(SW_EDEVICE);
    if (n_cand && hipMemcpyAsync(d_pairs, h_pairs, 8 * (size_t)n_cand, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(SW_EDEVICE);
    if ((rc = sw_pack(d_ascii, n_res, d_packed, sw_packed_bytes(n_res), st)) != SW_OK) return fail(rc);
    if (n_cand) {
        rc = sw_align_sets(d_packed, d_offs, n_q, s->refs_packed, s->ref_offsets, s->n_refs, d_pairs, n_cand,
                           &s->scoring, d_out, st, SW_NO_GRAPH);
        if (rc != SW_OK) return fail(rc);
        if (hipMemcpyAsync(h_out, d_out, sizeof(sw_result) * (size_t)n_cand, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return fail(SW_EDEVICE);
    }
    Request r;
    r.ticket = s->next_ticket++;
    r.slot = slot;
    r.dev_off = off;
    r.dev_bytes = need;
    r.n_cand = n_cand;
    r.out_host = out_host;
    r.staged = h_out;
    if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(r.done, st) != hipSuccess)
        return fail(SW_EDEVICE);
    sl.busy = true;
    s->inflight[r.ticket] = r;
    *ticket = r.ticket;
    return SW_OK;
}

SW_API int sw_server_poll(sw_server* s, uint64_t ticket)
{
    if (!s) return SW_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->inflight.find(ticket);
    if (it == s->inflight.end()) return SW_EINVAL;
    hipError_t e = hipEventQuery(it->second.done);
    if (e == hipErrorNotReady) return SW_EAGAIN;
    if (e != hipSuccess) return SW_EDEVICE;
    int rc = retire(s, it->second);
    s->inflight.erase(it);
    return rc;
}

SW_API int sw_server_wait(sw_server* s, uint64_t ticket, int64_t timeout_us)
{
    if (!s) return SW_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        int rc = sw_server_poll(s, ticket);
        if (rc != SW_EAGAIN) return rc;
        if (timeout_us >= 0) {
            const auto us = std::chrono::duration_cast<std::chrono::microseconds>(
                                std::chrono::steady_clock::now() - t0).count();
            if (us >= timeout_us) return SW_ETIMEOUT;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

SW_API int sw_server_stats(sw_server* s, int64_t* inflight, int64_t* bytes_in_use, int64_t* budget)
{
    if (!s) return SW_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (inflight) *inflight = (int64_t)s->inflight.size();
    if (bytes_in_use) *bytes_in_use = (int64_t)s->arena.used();
    if (budget) *budget = (int64_t)s->arena.size();
    return SW_OK;
}

SW_API size_t sw_server_request_bytes(int64_t n_residues, int64_t n_q, int64_t n_cand)
{
    if (n_residues < 0 || n_q < 0 || n_cand < 0) return 0;
    return request_bytes(n_residues, n_q, n_cand);
}

SW_API int sw_server_destroy(sw_server* s)
{
    if (!s) return SW_EINVAL;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->shutting_down = true;
        for (auto& kv : s->inflight) {
            (void)hipEventSynchronize(kv.second.done);
            (void)hipEventDestroy(kv.second.done);
        }
        s->inflight.clear();
        for (auto& sl : s->slots) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
            if (sl.pinned) (void)hipHostFree(sl.pinned);
        }
        s->arena.release();
    }
    delete s;
    return SW_OK;
}

}  // extern "C"
