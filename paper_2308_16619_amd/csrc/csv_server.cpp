// Serving loop: brick requests arrive as a renderer issues them (Sec. 4: a
// frame's raymarcher requests missing (brick, LOD) pairs, the GPU decodes
// them into a cache, the next frame uses them; Sec. 4.1: the cache).  Here a
// worker thread takes requests continuously:
//   - a hit in the decoded-brick cache (HBM) completes at once;
//   - a request for a brick that is being decoded joins that decode;
//   - a miss is admitted while the decoded bytes in flight stay within the
//     budget and the cache can give it a slot (LRU eviction within its LOD
//     class; when nothing of that class can be evicted and the cache is
//     full, the cache is rebuilt, as the paper's cache does on
//     fragmentation), then joins the batch being formed;
//   - a batch is launched as soon as a device stream is free, so batches
//     formed while others run overlap on the GPU (continuous batching).
// Completion time is when the worker sees the batch's event complete.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/csv.h"

namespace {

constexpr int kClasses = 6;  // LOD 0..5: (32 >> t)^3 uint32
constexpr uint64_t kPage = 32 * 32 * 32 * 4;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}
uint64_t class_bytes(int t) {
    const uint64_t g = 32u >> t;
    return g * g * g * 4;
}

enum State : uint8_t { kFree = 0, kDecoding = 1, kValid = 2 };

struct Entry {
    uint32_t brick = 0;
    uint8_t lod = 0;
    State state = kFree;
    bool in_lru = false;
    uint8_t ref = 0;                 // hit since it last passed the eviction scan (second chance)
    uint32_t pins = 0;               // completions not yet released by the next poll
    uint64_t slot = 0;               // byte offset in the cache
    int32_t prev = -1, next = -1;    // LRU neighbours within the LOD class (prev: more recent)
    int32_t waiters = -1;            // first request waiting for this decode (chained by req_next)
};

// intrusive LRU list of one LOD class: head most recent
struct Lru {
    int32_t head = -1, tail = -1;
};

struct Pending {
    csv_request r;
    uint32_t idx;  // request slot
};

struct Batch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // a batch's requests, u64 offsets[n], u32 ids[n], i32 status[n], u8 lods[n],
    // in pinned host memory that the decode kernels read (and, for failed
    // requests, write) directly (d_buf: its device address)
    uint8_t *h_buf = nullptr;
    uint8_t *d_buf = nullptr;
    std::vector<uint32_t> entries;  // entry ids decoded by this batch
    uint64_t bytes = 0;
    bool busy = false;
    int launch_rc = CSV_OK;         // the launch itself failed: every entry fails with it
    // full-LOD bricks whose level-0 detail is in host memory: staged before the decode
    std::vector<uint32_t> stage_ids;
    bool staged = false;
};

}  // namespace

struct csv_server {
    csv_pool *pool = nullptr;
    csv_server_opts opts{};
    int device = 0;
    uint32_t n_bricks = 0;
    uint8_t *d_cache = nullptr;
    // cache allocator: pages carved per LOD class, free stacks, per-class LRU
    uint64_t top = 0;
    std::vector<uint64_t> free_slots[kClasses];
    Lru lru[kClasses];
    std::vector<Entry> entries;
    std::vector<uint32_t> free_entries;
    std::vector<int32_t> index;  // brick * 6 + lod -> entry id or -1
    // requests
    std::mutex in_mu;
    std::vector<csv_request> inbox;
    std::vector<uint8_t> vis_in;     // visibility table handed in (under in_mu)
    int vis_new = 0;                 // 1: vis_in is a new table, 2: clear the table
    std::vector<uint8_t> visible;    // the worker's table (empty: every brick visible)
    std::deque<Pending> pending;
    std::vector<csv_request> reqs;   // request table (worker)
    std::vector<int32_t> req_next;   // next waiter of the same decode
    std::vector<uint32_t> free_reqs;
    std::mutex out_mu;
    std::vector<csv_completion> outbox;
    std::vector<int32_t> outbox_entry;  // cache entry each completion points into (-1: none)
    size_t outbox_head = 0;             // completions before it have been handed out
    std::vector<uint32_t> delivered;    // entries of the completions handed out by the last poll
    std::vector<uint32_t> to_unpin;     // entries whose completions the client has released
    // batches
    std::vector<Batch> batches;
    Batch *forming = nullptr;
    uint64_t inflight = 0;
    // worker-local completions and statistics, published once per loop
    std::vector<csv_completion> c_local;
    std::vector<int32_t> e_local;
    std::vector<float> l_all, l_miss;
    uint64_t d_req = 0, d_hit = 0, d_miss = 0, d_join = 0, d_busy = 0, d_launch = 0, d_skip = 0;
    // stats
    std::mutex st_mu;
    std::deque<float> lat_all, lat_miss;  // a deque grows without copying what it holds
    uint64_t n_req = 0, n_hit = 0, n_miss = 0, n_join = 0, n_batches = 0, n_evict = 0, n_rebuild = 0,
             decoded_bytes = 0, n_launch_err = 0, busy_ns = 0, launch_ns = 0, n_skip = 0, n_failed = 0;
    uint64_t stall[4] = {0, 0, 0, 0};  // admission stopped: no free batch, in-flight budget, no slot, staging
    // detail separation (Sec. 4.2): bytes of the staging buffer promised to
    // admitted full-LOD misses since the last release, launched batches that
    // staged detail and have not retired
    bool split = false;
    uint64_t stage_cap = 0, stage_planned = 0, n_staged_bytes = 0, n_releases = 0;
    uint32_t staged_inflight = 0;

    std::atomic<uint64_t> submitted{0}, completed{0};
    std::atomic<bool> stop{false};
    std::thread worker;
    int error = CSV_OK;
};

namespace {

void complete(csv_server *s, uint32_t ridx, Entry *e, int status, bool hit, uint64_t t, bool skipped = false) {
    const csv_request &r = s->reqs[ridx];
    csv_completion c{};
    c.tag = r.tag;
    c.brick_id = r.brick_id;
    c.lod = r.lod;
    c.status = status;
    c.hit = hit ? 1u : 0u;
    c.skipped = skipped ? 1u : 0u;
    c.t_arrival_ns = r.t_arrival_ns;
    c.t_done_ns = t;
    int32_t eid = -1;
    if (e && status == CSV_OK) {
        c.data = reinterpret_cast<const uint32_t *>(s->d_cache + e->slot);
        c.elems = (uint32_t)(class_bytes(e->lod) / 4);
        e->pins++;  // until the client releases it
        eid = (int32_t)(e - s->entries.data());
    }
    const float us = (float)((double)(t - r.t_arrival_ns) * 1e-3);
    if (!skipped) {
        s->l_all.push_back(us);
        if (!hit) s->l_miss.push_back(us);
    }
    s->c_local.push_back(c);
    s->e_local.push_back(eid);
    s->free_reqs.push_back(ridx);
}

// hand this loop's statistics, then its completions, to the client side
// (a completion the client sees is already counted)
void publish(csv_server *s) {
    if (!s->l_all.empty() || s->d_req || s->d_hit || s->d_miss || s->d_join || s->d_busy || s->d_skip) {
        std::lock_guard<std::mutex> lk(s->st_mu);
        s->busy_ns += s->d_busy;
        s->launch_ns += s->d_launch;
        s->d_busy = s->d_launch = 0;
        s->lat_all.insert(s->lat_all.end(), s->l_all.begin(), s->l_all.end());
        s->lat_miss.insert(s->lat_miss.end(), s->l_miss.begin(), s->l_miss.end());
        s->n_req += s->d_req;
        s->n_hit += s->d_hit;
        s->n_miss += s->d_miss;
        s->n_join += s->d_join;
        s->n_skip += s->d_skip;
        s->l_all.clear();
        s->l_miss.clear();
        s->d_req = s->d_hit = s->d_miss = s->d_join = s->d_skip = 0;
    }
    if (!s->c_local.empty()) {
        const size_t k = s->c_local.size();
        s->completed.fetch_add(k, std::memory_order_relaxed);
        std::lock_guard<std::mutex> lk(s->out_mu);
        s->outbox.insert(s->outbox.end(), s->c_local.begin(), s->c_local.end());
        s->outbox_entry.insert(s->outbox_entry.end(), s->e_local.begin(), s->e_local.end());
        s->c_local.clear();
        s->e_local.clear();
    }
}

void lru_unlink(csv_server *s, uint32_t id) {
    Entry &e = s->entries[id];
    Lru &L = s->lru[e.lod];
    if (e.prev >= 0) s->entries[e.prev].next = e.next;
    else L.head = e.next;
    if (e.next >= 0) s->entries[e.next].prev = e.prev;
    else L.tail = e.prev;
    e.prev = e.next = -1;
    e.in_lru = false;
}

void lru_touch(csv_server *s, uint32_t id) {
    Entry &e = s->entries[id];
    Lru &L = s->lru[e.lod];
    if (e.in_lru) {
        if (L.head == (int32_t)id) return;
        lru_unlink(s, id);
    }
    e.prev = -1;
    e.next = L.head;
    if (L.head >= 0) s->entries[L.head].prev = (int32_t)id;
    L.head = (int32_t)id;
    if (L.tail < 0) L.tail = (int32_t)id;
    e.in_lru = true;
}

void drop_entry(csv_server *s, uint32_t id) {
    if (s->entries[id].in_lru) lru_unlink(s, id);
    Entry &e = s->entries[id];
    s->index[(size_t)e.brick * kClasses + e.lod] = -1;
    e.state = kFree;
    e.waiters = -1;
    s->free_entries.push_back(id);
}

// the least recently used unpinned valid entry of class t, or -1.  An entry
// hit since the scan last passed it gets a second chance (its flag is
// cleared and the scan moves on; a hit itself only sets the flag, which
// keeps hits cheap).  The scan is bounded; past the bound the first
// unpinned entry it saw is taken.
int32_t evictable(csv_server *s, int t) {
    int32_t id = s->lru[t].tail, first = -1;
    for (int budget = 32; id >= 0 && budget > 0; budget--) {
        Entry &e = s->entries[id];
        if (e.pins == 0 && e.state == kValid) {
            if (!e.ref) return id;
            e.ref = 0;
            if (first < 0) first = id;
        }
        id = e.prev;
    }
    return first;
}

// a cache slot for LOD class t, or false
bool alloc_slot(csv_server *s, int t, uint64_t *slot) {
    auto &fs = s->free_slots[t];
    if (!fs.empty()) {
        *slot = fs.back();
        fs.pop_back();
        return true;
    }
    if (s->top + kPage <= s->opts.cache_bytes) {
        const uint64_t sz = class_bytes(t);
        for (uint64_t o = kPage; o >= 2 * sz; o -= sz) fs.push_back(s->top + o - sz);
        *slot = s->top;
        s->top += kPage;
        return true;
    }
    // evict the least recently used unpinned entry of the same class
    int32_t id = evictable(s, t);
    if (id >= 0) {
        *slot = s->entries[id].slot;
        drop_entry(s, (uint32_t)id);
        s->n_evict++;
        return true;
    }
    // a smaller class takes over the page of the least recently used unpinned
    // full-LOD entry (one page each), so that classes follow the request mix
    if (t > 0 && (id = evictable(s, 0)) >= 0) {
        const uint64_t page = s->entries[id].slot, sz = class_bytes(t);
        drop_entry(s, (uint32_t)id);
        s->n_evict++;
        for (uint64_t o = kPage; o >= 2 * sz; o -= sz) fs.push_back(page + o - sz);
        *slot = page;
        return true;
    }
    return false;
}

// drop every valid unpinned entry and start the allocator afresh; only when
// nothing is in flight or pinned
bool rebuild(csv_server *s) {
    if (s->inflight || (s->forming && !s->forming->entries.empty())) return false;
    for (uint32_t id = 0; id < s->entries.size(); id++)
        if (s->entries[id].state != kFree && s->entries[id].pins) return false;
    for (uint32_t id = 0; id < s->entries.size(); id++)
        if (s->entries[id].state == kValid) drop_entry(s, id);
    for (auto &f : s->free_slots) f.clear();
    for (auto &L : s->lru) L = Lru{};
    s->top = 0;
    s->n_rebuild++;
    return true;
}

Batch *free_batch(csv_server *s) {
    for (auto &b : s->batches)
        if (!b.busy && &b != s->forming) return &b;
    return nullptr;
}

void launch_batch(csv_server *s, Batch *b) {
    const uint64_t t0 = now_ns();
    const uint32_t n = (uint32_t)b->entries.size();
    uint64_t *h_off = reinterpret_cast<uint64_t *>(b->h_buf);
    uint32_t *h_ids = reinterpret_cast<uint32_t *>(h_off + n);
    int32_t *h_status = reinterpret_cast<int32_t *>(h_ids + n);
    uint8_t *h_lods = reinterpret_cast<uint8_t *>(h_status + n);
    for (uint32_t i = 0; i < n; i++) {
        const Entry &e = s->entries[b->entries[i]];
        h_ids[i] = e.brick;
        h_lods[i] = e.lod;
        h_off[i] = e.slot / 4;
        h_status[i] = CSV_OK;
    }
    const uint64_t *d_off = reinterpret_cast<const uint64_t *>(b->d_buf);
    const uint32_t *d_ids = reinterpret_cast<const uint32_t *>(d_off + n);
    int32_t *d_status = reinterpret_cast<int32_t *>(const_cast<uint32_t *>(d_ids + n));
    const uint8_t *d_lods = reinterpret_cast<const uint8_t *>(d_status + n);
    int rc = CSV_OK;
    if (!b->stage_ids.empty()) {
        // the level-0 detail of the batch's full-LOD bricks, on the batch's stream
        uint32_t done = 0;
        rc = csv_pool_stage_detail(s->pool, b->stage_ids.data(), (uint32_t)b->stage_ids.size(), b->stream, &done);
        if (!rc && done != b->stage_ids.size()) rc = CSV_ENOMEM;
        b->staged = true;
        s->staged_inflight++;
    }
    if (!rc)
        rc = csv_decode_bricks_status(s->pool, d_ids, d_lods, 0, d_off, n, reinterpret_cast<uint32_t *>(s->d_cache),
                                      b->stream, d_status);
    if (hipEventRecord(b->done, b->stream) != hipSuccess && !rc) rc = CSV_EHIP;
    b->launch_rc = rc;
    if (rc) {
        s->n_launch_err++;
        s->error = rc;
    }
    b->busy = true;
    s->n_batches++;
    s->d_launch += now_ns() - t0;
}

void retire(csv_server *s, Batch &b, uint64_t t) {
    const uint32_t n = (uint32_t)b.entries.size();
    const int32_t *h_status = reinterpret_cast<const int32_t *>(b.h_buf + 12ull * n);
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t id = b.entries[i];
        Entry &e = s->entries[id];
        // the kernels wrote the code of each failed request into the batch's status array
        const int code = b.launch_rc ? b.launch_rc : h_status[i];
        int32_t w = e.waiters;
        e.waiters = -1;
        if (code != CSV_OK) {  // not cached: the slot goes back to its class, waiters get the code
            s->free_slots[e.lod].push_back(e.slot);
            drop_entry(s, id);
            s->n_failed++;
            s->error = code;
            while (w >= 0) {
                const int32_t nx = s->req_next[(size_t)w];
                complete(s, (uint32_t)w, nullptr, code, false, t);
                w = nx;
            }
            continue;
        }
        e.state = kValid;
        lru_touch(s, id);
        while (w >= 0) {
            const int32_t nx = s->req_next[(size_t)w];
            complete(s, (uint32_t)w, &s->entries[id], CSV_OK, false, t);
            w = nx;
        }
    }
    b.launch_rc = CSV_OK;
    s->decoded_bytes += b.bytes;
    s->inflight -= b.bytes;
    b.entries.clear();
    b.bytes = 0;
    b.busy = false;
    if (b.staged) {
        s->staged_inflight--;
        b.staged = false;
    }
    b.stage_ids.clear();
}

// the staged detail is dropped once no launched batch reads it and the
// batch being formed has promised none of it
void release_detail(csv_server *s) {
    if (!s->split || s->stage_planned == 0 || s->staged_inflight != 0) return;
    if (s->forming && !s->forming->stage_ids.empty()) return;
    if (csv_pool_release_detail(s->pool, s->batches[0].stream) != CSV_OK) {
        s->n_launch_err++;
        s->error = CSV_EHIP;
    }
    s->stage_planned = 0;
    s->n_releases++;
}

// one request: true if handled (completed, joined or admitted), false if it
// must wait; t_now: the time of this admission round (hits complete at it)
bool admit(csv_server *s, const Pending &p, uint64_t t_now) {
    const csv_request &r = p.r;
    if (r.brick_id >= s->n_bricks || r.lod > 5) {
        complete(s, p.idx, nullptr, CSV_ERANGE, false, t_now);
        return true;
    }
    if (!s->visible.empty() && !s->visible[r.brick_id]) {  // empty space: nothing to decode
        complete(s, p.idx, nullptr, CSV_OK, false, t_now, true);
        s->d_skip++;
        return true;
    }
    const size_t key = (size_t)r.brick_id * kClasses + r.lod;
    int32_t id = s->index[key];
    if (id >= 0) {
        Entry &e = s->entries[id];
        if (e.state == kValid) {
            e.ref = 1;
            complete(s, p.idx, &s->entries[(size_t)id], CSV_OK, true, t_now);
            s->d_hit++;
        } else {
            s->req_next[p.idx] = e.waiters;
            e.waiters = (int32_t)p.idx;
            s->d_join++;
        }
        return true;
    }
    const uint64_t bytes = class_bytes(r.lod);
    // a full-LOD miss on a brick with its detail in host memory takes its
    // share of the staging buffer until the next release
    uint32_t det = 0;
    if (s->split && r.lod == 0 && csv_pool_detail_bytes(s->pool, r.brick_id, &det, nullptr) == CSV_OK && det) {
        if (det > s->stage_cap) {  // can never be staged
            complete(s, p.idx, nullptr, CSV_EDETAIL, false, t_now);
            return true;
        }
        if (s->stage_planned + det > s->stage_cap) {
            s->stall[3]++;
            return false;
        }
    }
    // decodes in flight hold cache slots: keep them within a quarter of the cache
    const uint64_t budget = std::min(s->opts.inflight_bytes, s->opts.cache_bytes / 4);
    if (s->inflight + bytes > budget && s->inflight > 0) {
        s->stall[1]++;
        return false;
    }
    if (!s->forming) s->forming = free_batch(s);
    if (!s->forming) {
        s->stall[0]++;
        return false;
    }
    uint64_t slot;
    if (!alloc_slot(s, r.lod, &slot)) {
        if (!rebuild(s) || !alloc_slot(s, r.lod, &slot)) {
            s->stall[2]++;
            return false;
        }
    }
    uint32_t nid;
    if (!s->free_entries.empty()) {
        nid = s->free_entries.back();
        s->free_entries.pop_back();
    } else {
        nid = (uint32_t)s->entries.size();
        s->entries.emplace_back();
    }
    Entry &e = s->entries[nid];
    e.brick = r.brick_id;
    e.lod = r.lod;
    e.state = kDecoding;
    e.pins = 0;
    e.slot = slot;
    e.in_lru = false;
    e.ref = 0;
    e.prev = e.next = -1;
    e.waiters = (int32_t)p.idx;
    s->req_next[p.idx] = -1;
    s->index[key] = (int32_t)nid;
    s->forming->entries.push_back(nid);
    s->forming->bytes += bytes;
    if (det) {
        s->forming->stage_ids.push_back(r.brick_id);
        s->stage_planned += det;
        s->n_staged_bytes += det;
    }
    s->inflight += bytes;
    s->d_miss++;
    if (s->forming->entries.size() >= s->opts.max_batch) {
        launch_batch(s, s->forming);
        s->forming = nullptr;
    }
    return true;
}

void worker_main(csv_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<csv_request> take;
    uint32_t idle = 0;
    while (!s->stop.load(std::memory_order_acquire)) {
        bool work = false;
        const uint64_t t_loop = now_ns();
        {
            std::lock_guard<std::mutex> lk(s->in_mu);
            take.swap(s->inbox);
            if (s->vis_new == 1) s->visible.swap(s->vis_in);
            if (s->vis_new == 2) s->visible.clear();
            s->vis_new = 0;
        }
        for (const csv_request &r : take) {
            uint32_t idx;
            if (!s->free_reqs.empty()) {
                idx = s->free_reqs.back();
                s->free_reqs.pop_back();
                s->reqs[idx] = r;
            } else {
                idx = (uint32_t)s->reqs.size();
                s->reqs.push_back(r);
                s->req_next.push_back(-1);
            }
            s->pending.push_back(Pending{r, idx});
        }
        s->d_req += take.size();
        work |= !take.empty();
        take.clear();
        // completed batches
        for (auto &b : s->batches) {
            if (b.busy && hipEventQuery(b.done) == hipSuccess) {
                retire(s, b, now_ns());
                work = true;
            }
        }
        release_detail(s);
        // entries pinned by completions the client has released
        {
            std::vector<uint32_t> rel;
            {
                std::lock_guard<std::mutex> lk(s->out_mu);
                rel.swap(s->to_unpin);
            }
            for (uint32_t id : rel)
                if (s->entries[id].pins) s->entries[id].pins--;
        }
        // admission, in arrival order
        const uint64_t t_now = now_ns();
        while (!s->pending.empty()) {
            if (!admit(s, s->pending.front(), t_now)) break;
            s->pending.pop_front();
            work = true;
        }
        // continuous batching: launch what has formed as soon as a stream is free
        if (s->forming && !s->forming->entries.empty()) {
            launch_batch(s, s->forming);
            s->forming = nullptr;
            work = true;
        }
        if (work) s->d_busy += now_ns() - t_loop;
        publish(s);
        if (work) {
            idle = 0;
        } else if (++idle > 2000) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else {
            std::this_thread::yield();
        }
    }
}

double pct(const std::deque<float> &d, double q) {
    std::vector<float> v(d.begin(), d.end());
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (long)k, v.end());
    return v[k];
}

}  // namespace

extern "C" {

uint64_t csv_now_ns(void) { return now_ns(); }

void csv_server_opts_default(csv_server_opts *o) {
    if (!o) return;
    o->cache_bytes = 1ull << 30;
    o->inflight_bytes = 256ull << 20;
    o->max_batch = 4096;
    o->streams = 4;
}

int csv_server_create(csv_pool *pool, const csv_server_opts *o, csv_server **out) {
    if (!pool || !out) return CSV_EINVAL;
    csv_server_opts opts;
    csv_server_opts_default(&opts);
    if (o) opts = *o;
    if (opts.cache_bytes < kPage || opts.max_batch < 1 || opts.streams < 1 || opts.streams > 16 ||
        opts.inflight_bytes < kPage)
        return CSV_EINVAL;
    csv_pool_info info;
    int rc = csv_pool_info_get(pool, &info);
    if (rc) return rc;
    if (info.n_bricks == 0 || info.brick_log2 != 5) return CSV_EINVAL;  // the cache holds 32^3 blocks
    csv_server *s = new (std::nothrow) csv_server;
    if (!s) return CSV_ENOMEM;
    s->pool = pool;
    s->opts = opts;
    s->opts.cache_bytes = opts.cache_bytes / kPage * kPage;
    s->device = info.device;
    s->n_bricks = info.n_bricks;
    s->split = info.host_bytes != 0;
    if (s->split && csv_pool_detail_bytes(pool, 0, nullptr, &s->stage_cap) != CSV_OK) {
        delete s;
        return CSV_EINVAL;
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    rc = CSV_OK;
    try {
        s->index.assign((size_t)info.n_bricks * kClasses, -1);
    } catch (const std::bad_alloc &) {
        rc = CSV_ENOMEM;
    }
    if (!rc && hipMalloc(reinterpret_cast<void **>(&s->d_cache), s->opts.cache_bytes) != hipSuccess) rc = CSV_ENOMEM;
    s->batches.resize(opts.streams + 1);  // one more than streams: a batch can form while all run
    for (auto &b : s->batches) {
        if (rc) break;
        const size_t n = opts.max_batch;
        if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&b.h_buf), 17 * n + 16, hipHostMallocMapped | hipHostMallocCoherent) !=
                hipSuccess ||
            hipHostGetDevicePointer(reinterpret_cast<void **>(&b.d_buf), b.h_buf, 0) != hipSuccess)
            rc = CSV_ENOMEM;
    }
    (void)hipSetDevice(prev);
    if (rc) {
        csv_server_destroy(s);
        return rc;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CSV_OK;
}

int csv_server_submit(csv_server *s, const csv_request *r, uint32_t n) {
    if (!s || (n && !r)) return CSV_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->in_mu);
        s->inbox.insert(s->inbox.end(), r, r + n);
    }
    s->submitted.fetch_add(n, std::memory_order_relaxed);
    return CSV_OK;
}

int csv_server_poll(csv_server *s, csv_completion *c, uint32_t cap, uint32_t *got) {
    if (!s || !got || (cap && !c)) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(s->out_mu);
    // the completions handed out by the previous poll are released now
    s->to_unpin.insert(s->to_unpin.end(), s->delivered.begin(), s->delivered.end());
    s->delivered.clear();
    const size_t h = s->outbox_head;
    const uint32_t k = (uint32_t)std::min<size_t>(cap, s->outbox.size() - h);
    std::copy(s->outbox.begin() + (long)h, s->outbox.begin() + (long)(h + k), c);
    for (uint32_t i = 0; i < k; i++)
        if (s->outbox_entry[h + i] >= 0) s->delivered.push_back((uint32_t)s->outbox_entry[h + i]);
    s->outbox_head = h + k;
    if (s->outbox_head == s->outbox.size()) {
        s->outbox.clear();
        s->outbox_entry.clear();
        s->outbox_head = 0;
    } else if (s->outbox_head > 65536 && 2 * s->outbox_head > s->outbox.size()) {  // compact now and then
        s->outbox.erase(s->outbox.begin(), s->outbox.begin() + (long)s->outbox_head);
        s->outbox_entry.erase(s->outbox_entry.begin(), s->outbox_entry.begin() + (long)s->outbox_head);
        s->outbox_head = 0;
    }
    *got = k;
    return CSV_OK;
}

int csv_server_stats(csv_server *s, csv_stats *st) {
    if (!s || !st) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(s->st_mu);
    std::memset(st, 0, sizeof(*st));
    st->requests = s->n_req;
    st->hits = s->n_hit;
    st->misses = s->n_miss;
    st->joined = s->n_join;
    st->completed = s->completed.load();
    st->batches = s->n_batches;
    st->evictions = s->n_evict;
    st->rebuilds = s->n_rebuild;
    st->decoded_bytes = s->decoded_bytes;
    st->cache_bytes_used = s->top;
    st->p50_us = pct(s->lat_all, 0.50);
    st->p99_us = pct(s->lat_all, 0.99);
    st->p50_miss_us = pct(s->lat_miss, 0.50);
    st->p99_miss_us = pct(s->lat_miss, 0.99);
    st->max_us = s->lat_all.empty() ? 0.0 : *std::max_element(s->lat_all.begin(), s->lat_all.end());
    st->error = s->error;
    st->worker_busy_ns = s->busy_ns;
    st->worker_launch_ns = s->launch_ns;
    st->stall_batch = s->stall[0];
    st->stall_inflight = s->stall[1];
    st->stall_slot = s->stall[2];
    st->skipped = s->n_skip;
    st->stall_staging = s->stall[3];
    st->detail_staged_bytes = s->n_staged_bytes;
    st->detail_releases = s->n_releases;
    st->failed = s->n_failed;
    return CSV_OK;
}

int csv_server_reset_stats(csv_server *s) {
    if (!s) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(s->st_mu);
    s->lat_all.clear();
    s->lat_miss.clear();
    s->n_req = s->n_hit = s->n_miss = s->n_join = s->n_batches = s->n_evict = s->n_rebuild = 0;
    s->decoded_bytes = 0;
    s->busy_ns = s->launch_ns = 0;
    s->stall[0] = s->stall[1] = s->stall[2] = s->stall[3] = 0;
    s->n_staged_bytes = s->n_releases = 0;
    s->n_skip = 0;
    s->n_failed = 0;
    return CSV_OK;
}

int csv_server_set_visible(csv_server *s, const uint8_t *visible, uint32_t n_bricks) {
    if (!s || (visible && n_bricks != s->n_bricks)) return CSV_EINVAL;
    std::vector<uint8_t> v;
    if (visible) {
        try {
            v.assign(visible, visible + n_bricks);
        } catch (...) {
            return CSV_ENOMEM;
        }
    }
    std::lock_guard<std::mutex> lk(s->in_mu);
    s->vis_in.swap(v);
    s->vis_new = visible ? 1 : 2;
    return CSV_OK;
}

void csv_server_destroy(csv_server *s) {
    if (!s) return;
    s->stop.store(true, std::memory_order_release);
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto &b : s->batches) {
        if (b.stream) (void)hipStreamSynchronize(b.stream);
        if (b.done) (void)hipEventDestroy(b.done);
        if (b.stream) (void)hipStreamDestroy(b.stream);
        (void)hipHostFree(b.h_buf);
    }
    (void)hipFree(s->d_cache);
    (void)hipSetDevice(prev);
    delete s;
}

const uint32_t *csv_server_cache_data(const csv_server *s) {
    return s ? reinterpret_cast<const uint32_t *>(s->d_cache) : nullptr;
}

int csv_server_read(csv_server *s, const csv_completion *c, uint32_t *host_dst) {
    if (!s || !c || !host_dst || !c->data) return CSV_EINVAL;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    const hipError_t e = hipMemcpy(host_dst, c->data, 4ull * c->elems, hipMemcpyDeviceToHost);
    (void)hipSetDevice(prev);
    return e == hipSuccess ? CSV_OK : CSV_EHIP;
}

/*
 * Replay a request trace in real time from the calling thread: request i
 * is submitted once csv_now_ns() reaches start + reqs[i].t_arrival_ns (its
 * arrival time is then set to that absolute time), completions are drained
 * as they come (and copied to `done` when not NULL), until all n requests
 * completed or timeout_ns passed since the last request arrived.
 */
int csv_server_run_trace(csv_server *s, const csv_request *reqs, uint32_t n, csv_completion *done,
                         uint64_t timeout_ns, uint32_t *n_done) {
    if (!s || (n && !reqs)) return CSV_EINVAL;
    std::vector<csv_request> batch;
    // modest polls: a poll's completions pin their cache entries until the next poll
    std::vector<csv_completion> buf(4096);
    const uint64_t t0 = now_ns();
    uint32_t next = 0, got_total = 0;
    uint64_t last_arrival = t0;
    while (got_total < n) {
        const uint64_t t = now_ns();
        batch.clear();
        while (next < n && t0 + reqs[next].t_arrival_ns <= t) {
            csv_request r = reqs[next++];
            r.t_arrival_ns += t0;
            last_arrival = r.t_arrival_ns;
            batch.push_back(r);
        }
        if (!batch.empty()) csv_server_submit(s, batch.data(), (uint32_t)batch.size());
        uint32_t got = 0;
        csv_server_poll(s, buf.data(), (uint32_t)buf.size(), &got);
        if (done && got) std::copy(buf.begin(), buf.begin() + got, done + got_total);
        got_total += got;
        if (next == n && t - last_arrival > timeout_ns) break;
        if (!got && batch.empty()) std::this_thread::yield();
    }
    uint32_t got = 0;
    csv_server_poll(s, buf.data(), 0, &got);  // release the last completions
    if (n_done) *n_done = got_total;
    return got_total == n ? CSV_OK : CSV_EBUSY;
}

}  // extern "C"
