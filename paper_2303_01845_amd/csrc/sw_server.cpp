// Continuous-batching server over a reference set resident in HBM.
//
// A request is a batch of query sequences (host ASCII) with a candidate list
// of (query, reference) pairs.  It is admitted when its device state fits in
// what is left of the HBM budget (otherwise submit returns SW_EAGAIN and the
// caller retries after a completion); admitted requests queue in arrival
// order.  Whenever a slot (a HIP stream with its own alignment workspace) is
// free, every queued request is merged into one launch on it: the queries
// are concatenated, copied in, packed and aligned against the resident set by
// one persistent launch, and the results are copied back and handed to each
// request.  Under load the launches grow, so the device stays busy; at low
// load a request starts as soon as it arrives.  Launches on different slots
// run concurrently.  Completions are found and new launches started inside
// submit, poll, wait and stats.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
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
    int64_t n_q = 0, n_res = 0, n_cand = 0;
    size_t reserved = 0;  // budget bytes held from admission to completion
    std::vector<char> ascii;
    std::vector<int64_t> offs;
    std::vector<int32_t> cand;
    sw_result* out_host = nullptr;
    bool done = false;
    int status = SW_OK;
};

// One launch: the requests merged into it, their device region and the
// pinned results.
struct Batch {
    std::vector<uint64_t> tickets;
    std::vector<int64_t> first;  // first result of each request
    size_t dev_off = 0, dev_bytes = 0;
    sw_result* staged = nullptr;
    hipEvent_t done = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    Batch batch;
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
    size_t reserved = 0;  // budget held by admitted, unfinished requests
    std::vector<Slot> slots;
    std::map<uint64_t, Request> requests;  // admitted and not yet retired by poll
    std::deque<uint64_t> pending;          // admitted, waiting for a slot
    uint64_t next_ticket = 1;
    bool shutting_down = false;
    std::mutex mu;
};

namespace {

constexpr int64_t kMaxBatchPairs = (int64_t)1 << 24;

// Device bytes a request needs: ASCII, packed queries, offsets, pairs, results.
size_t request_bytes(int64_t n_res, int64_t n_q, int64_t n_cand)
{
    return align_up((size_t)n_res) + align_up(sw_packed_bytes(n_res)) + align_up(8 * (size_t)(n_q + 1)) +
           align_up(8 * (size_t)n_cand) + align_up(sizeof(sw_result) * (size_t)n_cand);
}

// A finished launch: results to the callers, budget and slot freed.
void complete(sw_server* s, Slot& sl, int status)
{
    Batch& b = sl.batch;
    for (size_t k = 0; k < b.tickets.size(); ++k) {
        Request& r = s->requests[b.tickets[k]];
        if (status == SW_OK && r.n_cand)
            std::memcpy(r.out_host, b.staged + b.first[k], sizeof(sw_result) * (size_t)r.n_cand);
        r.status = status;
        r.done = true;
        s->reserved -= r.reserved;
        std::vector<char>().swap(r.ascii);
        std::vector<int64_t>().swap(r.offs);
        std::vector<int32_t>().swap(r.cand);
    }
    if (b.done) (void)hipEventDestroy(b.done);
    s->arena.free(b.dev_off, b.dev_bytes);
    b = Batch();
    sl.busy = false;
}

// Merge requests from the head of the queue into one launch on a free slot:
// the queries are concatenated (query indexes of the candidates shifted
// accordingly), copied in, packed and aligned against the resident set in
// one call, and the results copied back.  Returns false when nothing could
// be launched (no request waiting, or no arena space until a launch ends).
bool launch(sw_server* s, Slot& sl)
{
    int64_t n_res = 0, n_q = 0, n_cand = 0;
    size_t take = 0;
    while (take < s->pending.size()) {
        const Request& r = s->requests[s->pending[take]];
        if (take > 0 && n_cand + r.n_cand > kMaxBatchPairs) break;
        n_res += r.n_res;
        n_q += r.n_q;
        n_cand += r.n_cand;
        ++take;
    }
    if (take == 0) return false;
    const size_t need = request_bytes(n_res, n_q, n_cand);
    const size_t off = s->arena.alloc(need);
    if (off == SIZE_MAX) return false;

    const size_t in_bytes = align_up((size_t)n_res) + align_up(8 * (size_t)(n_q + 1)) + align_up(8 * (size_t)n_cand);
    const size_t stage = in_bytes + align_up(sizeof(sw_result) * (size_t)n_cand);
    Batch b;
    b.dev_off = off;
    b.dev_bytes = need;
    int status = SW_OK;
    if (stage > sl.pinned_bytes) {
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        sl.pinned_bytes = 0;
        const size_t bytes = std::max<size_t>(stage + stage / 4, 1 << 20);
        if (hipHostMalloc((void**)&sl.pinned, bytes) != hipSuccess) status = SW_ENOMEM;
        else sl.pinned_bytes = bytes;
    }
    // gather the requests into the staging buffer
    char* h_ascii = sl.pinned;
    int64_t* h_offs = reinterpret_cast<int64_t*>(sl.pinned + align_up((size_t)n_res));
    int32_t* h_pairs = reinterpret_cast<int32_t*>(sl.pinned + align_up((size_t)n_res) + align_up(8 * (size_t)(n_q + 1)));
    b.staged = reinterpret_cast<sw_result*>(sl.pinned + in_bytes);
    int64_t res0 = 0, q0 = 0, c0 = 0;
    for (size_t k = 0; k < take; ++k) {
        const uint64_t t = s->pending.front();
        s->pending.pop_front();
        Request& r = s->requests[t];
        b.tickets.push_back(t);
        b.first.push_back(c0);
        if (status != SW_OK) continue;
        if (r.n_res) std::memcpy(h_ascii + res0, r.ascii.data(), (size_t)r.n_res);
        for (int64_t i = 0; i < r.n_q; ++i) h_offs[q0 + i] = res0 + r.offs[i];
        for (int64_t i = 0; i < r.n_cand; ++i) {
            h_pairs[2 * (c0 + i)] = (int32_t)(q0 + r.cand[2 * i]);
            h_pairs[2 * (c0 + i) + 1] = r.cand[2 * i + 1];
        }
        res0 += r.n_res;
        q0 += r.n_q;
        c0 += r.n_cand;
    }
    if (status == SW_OK) h_offs[n_q] = n_res;

    char* d = s->arena.ptr(off);
    char* d_ascii = d;
    char* d_packed = d_ascii + align_up((size_t)n_res);
    int64_t* d_offs = reinterpret_cast<int64_t*>(d_packed + align_up(sw_packed_bytes(n_res)));
    int32_t* d_pairs = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_offs) + align_up(8 * (size_t)(n_q + 1)));
    sw_result* d_out = reinterpret_cast<sw_result*>(reinterpret_cast<char*>(d_pairs) + align_up(8 * (size_t)n_cand));
    hipStream_t st = sl.stream;
    if (status == SW_OK && hipSetDevice(s->device) != hipSuccess) status = SW_EDEVICE;
    if (status == SW_OK && n_res && hipMemcpyAsync(d_ascii, h_ascii, (size_t)n_res, hipMemcpyHostToDevice, st) != hipSuccess)
        status = SW_EDEVICE;
    if (status == SW_OK && hipMemcpyAsync(d_offs, h_offs, 8 * (size_t)(n_q + 1), hipMemcpyHostToDevice, st) != hipSuccess)
        status = SW_EDEVICE;
    if (status == SW_OK && n_cand && hipMemcpyAsync(d_pairs, h_pairs, 8 * (size_t)n_cand, hipMemcpyHostToDevice, st) != hipSuccess)
        status = SW_EDEVICE;
    if (status == SW_OK) status = sw_pack(d_ascii, n_res, d_packed, sw_packed_bytes(n_res), st);
    if (status == SW_OK && n_cand)
        status = sw_align_sets(d_packed, d_offs, n_q, s->refs_packed, s->ref_offsets, s->n_refs, d_pairs, n_cand,
                               &s->scoring, d_out, st, SW_NO_GRAPH);
    if (status == SW_OK && n_cand &&
        hipMemcpyAsync(b.staged, d_out, sizeof(sw_result) * (size_t)n_cand, hipMemcpyDeviceToHost, st) != hipSuccess)
        status = SW_EDEVICE;
    if (status == SW_OK && (hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
                            hipEventRecord(b.done, st) != hipSuccess))
        status = SW_EDEVICE;
    sl.batch = std::move(b);
    sl.busy = true;
    if (status != SW_OK) {
        (void)hipStreamSynchronize(st);
        complete(s, sl, status);
    }
    return true;
}

// Retire finished launches and start new ones while slots and requests allow.
void pump(sw_server* s)
{
    for (auto& sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t e = hipEventQuery(sl.batch.done);
        if (e == hipErrorNotReady) continue;
        complete(s, sl, e == hipSuccess ? SW_OK : SW_EDEVICE);
    }
    for (auto& sl : s->slots) {
        if (s->pending.empty()) break;
        if (!sl.busy && !launch(s, sl)) break;
    }
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
    if (n_cand > kMaxBatchPairs) return SW_ERANGE;
    const int64_t n_res = n_q > 0 ? q_offsets[n_q] : 0;
    if (n_res < 0 || (n_res > 0 && !q_ascii) || q_offsets[0] != 0) return SW_EINVAL;
    for (int64_t k = 0; k < n_q; ++k)
        if (q_offsets[k + 1] < q_offsets[k]) return SW_EINVAL;
    for (int64_t k = 0; k < n_cand; ++k)
        if (cand[2 * k] < 0 || cand[2 * k] >= n_q) return SW_ERANGE;
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->shutting_down) return SW_ECANCELED;
    const size_t need = request_bytes(n_res, n_q, n_cand);
    if (need > s->arena.size()) return SW_ENOMEM;  // can never be admitted
    pump(s);
    if (s->reserved + need > s->arena.size()) return SW_EAGAIN;
    Request r;
    r.n_q = n_q;
    r.n_res = n_res;
    r.n_cand = n_cand;
    r.reserved = need;
    r.out_host = out_host;
    r.ascii.assign(q_ascii, q_ascii + n_res);
    r.offs.assign(q_offsets, q_offsets + n_q + 1);
    r.cand.assign(cand, cand + 2 * n_cand);
    const uint64_t t = s->next_ticket++;
    s->requests.emplace(t, std::move(r));
    s->reserved += need;
    s->pending.push_back(t);
    pump(s);
    *ticket = t;
    return SW_OK;
}

SW_API int sw_server_poll(sw_server* s, uint64_t ticket)
{
    if (!s) return SW_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return SW_EINVAL;
    if (!it->second.done) pump(s);
    if (!it->second.done) return SW_EAGAIN;
    const int rc = it->second.status;
    s->requests.erase(it);
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
    pump(s);
    int64_t n = 0;
    for (const auto& kv : s->requests) n += kv.second.done ? 0 : 1;
    if (inflight) *inflight = n;
    if (bytes_in_use) *bytes_in_use = (int64_t)s->reserved;
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
        for (auto& sl : s->slots) {
            if (sl.busy) {
                (void)hipEventSynchronize(sl.batch.done);
                complete(s, sl, SW_ECANCELED);
            }
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
            if (sl.pinned) (void)hipHostFree(sl.pinned);
        }
        s->requests.clear();
        s->pending.clear();
        s->arena.release();
    }
    delete s;
    return SW_OK;
}

}  // extern "C"
