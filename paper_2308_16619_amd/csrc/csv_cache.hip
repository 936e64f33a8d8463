// Frame cache of decoded bricks, resident on the GPU (Sec. 4.1, after
// Shading Atlas Streaming): the cache memory is a pool of base elements of
// 2^3 voxels; a brick at LOD t < N occupies a block of 8^(N-1-t) contiguous
// base elements.  One stack of free blocks per block size, a shared top
// pointer advanced atomically when a stack runs empty, and a rebuild that
// clears everything when the top reaches the end.  A frame's requests
// decide what stays: entries not requested (or invisible) in the frame are
// evicted and their blocks pushed on their stacks; new entries take blocks
// from the stacks first.  The coarsest LOD is the palette's first entry and
// is never stored.
//
// One frame = mark (dedupe, hits, misses per block size), evict (a scan of
// all (brick, LOD) keys), assign (one workgroup: stacks, top, rebuild),
// then the decode of the assigned bricks into their blocks, and the
// requests' slots.  With statistics requested, the host reads the frame
// state (how many bricks to decode, counts) between assign and decode;
// without, the decode reads the number of bricks from device memory
// (csv_decode_bricks_devcount) and nothing waits for the device.
//
// Detail streaming (Sec. 4.2), for pools that keep level-0 detail in host
// memory: a full-LOD request for a brick whose detail is not on the device
// and whose full LOD is not cached is served at LOD 1 (the finest level in
// HBM) and the brick goes on the frame's list of wanted detail.  Both
// options of the paper hide the resulting lag: the next frame uploads the
// wanted detail first, then the detail of the bricks the caller predicted
// (bricks close to the camera) that are not cached at full LOD, through
// the pool's staging buffer, so that predicted bricks are decoded at full
// LOD in the frame that first requests them.  The lists reach the host
// after the frame's work, in stream order; the next frame reads them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "csv.h"

namespace {

constexpr uint32_t kLods = 5;  // cached LODs 0..4 (LOD 5 is palette[0])
constexpr uint64_t kNone64 = ~0ull;

// base elements of a block for LOD t (2^3 voxels each)
__host__ __device__ constexpr uint32_t block_elems(uint32_t t) { return 1u << (3 * (4 - t)); }

struct FrameState {
    uint32_t frame;
    uint32_t n_miss[kLods];   // this frame's new keys per LOD
    uint32_t n_uniq[kLods];   // this frame's distinct visible keys per LOD
    uint32_t stack_top[kLods];
    uint64_t top;             // base elements handed out
    uint32_t n_dec, evicted, rebuilt, error;
    uint32_t n_want;          // bricks served at LOD 1 for want of level-0 detail
};

struct CacheDev {
    uint32_t n_bricks, n_req;
    uint64_t cap_elems;
    uint64_t *index;      // per key = brick * 5 + t: first base element, kNone64 if not cached
    uint32_t *stamp;      // per key: last frame that requested it (visible)
    uint64_t *stacks;     // kLods stacks of n_bricks free blocks (first base element)
    uint32_t *miss;       // kLods lists of n_req keys
    uint32_t *uniq;       // kLods lists of n_req keys
    uint32_t *dec_ids;    // decode list: brick ids, LODs, element offsets
    uint8_t *dec_lods;
    uint64_t *dec_off;
    FrameState *st;
    // detail streaming (nullptr for pools without detail in host memory)
    const uint8_t *det;   // per brick: bit 0 level-0 detail in host memory, bit 1 staged by this cache
    uint32_t *want;       // n_req bricks whose full-LOD request was served at LOD 1
    uint32_t *pred;       // n_req predicted bricks that need their detail uploaded (~0u: not)
};

constexpr uint8_t kSplit = 1, kStaged = 2;

// a full-LOD request of a brick whose detail is in host memory and not
// staged, when its full LOD is not cached
__device__ __forceinline__ bool wants_detail(const CacheDev &c, uint32_t id) {
    const uint8_t m = c.det[id];
    return (m & kSplit) && !(m & kStaged) && c.index[id * kLods] == kNone64;
}

__global__ void begin_kernel(CacheDev c) {
    if (threadIdx.x == 0) {
        c.st->frame++;
        c.st->n_dec = c.st->evicted = c.st->rebuilt = c.st->error = c.st->n_want = 0;
    }
    if (threadIdx.x < kLods) {
        c.st->n_miss[threadIdx.x] = 0;
        c.st->n_uniq[threadIdx.x] = 0;
    }
}

// request r: a visible, cacheable key is stamped with the frame; its first
// request this frame lists it (and, if not cached, as a miss).  A full-LOD
// request that wants detail takes the LOD-1 key; its brick is listed once
// (the full-LOD key's stamp, which eviction ignores as that key is not
// cached, marks it listed).
__global__ void mark_kernel(CacheDev c, const uint32_t *ids, const uint8_t *lods, const uint8_t *vis, uint32_t n) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = ids[r];
    uint32_t t = lods[r];
    if (id >= c.n_bricks || t >= kLods || (vis && !vis[r])) return;
    const uint32_t frame = c.st->frame;
    if (t == 0 && c.det && wants_detail(c, id)) {
        if (atomicExch(&c.stamp[id * kLods], frame) != frame) c.want[atomicAdd(&c.st->n_want, 1u)] = id;
        t = 1;
    }
    const uint32_t key = id * kLods + t;
    if (atomicExch(&c.stamp[key], frame) == frame) return;
    c.uniq[t * c.n_req + atomicAdd(&c.st->n_uniq[t], 1u)] = key;
    if (c.index[key] == kNone64) c.miss[t * c.n_req + atomicAdd(&c.st->n_miss[t], 1u)] = key;
}

// cached keys not requested this frame give their blocks back
__global__ void evict_kernel(CacheDev c) {
    const uint32_t nk = c.n_bricks * kLods, frame = c.st->frame;
    for (uint32_t key = blockIdx.x * blockDim.x + threadIdx.x; key < nk; key += gridDim.x * blockDim.x) {
        const uint64_t e = c.index[key];
        if (e == kNone64 || c.stamp[key] == frame) continue;
        const uint32_t t = key % kLods;
        const uint32_t p = atomicAdd(&c.st->stack_top[t], 1u);
        c.stacks[(size_t)t * c.n_bricks + p] = e;
        c.index[key] = kNone64;
        atomicAdd(&c.st->evicted, 1u);
    }
}

// one workgroup: blocks for the misses (stacks first, then the top), or a
// rebuild that gives every distinct key of the frame a block from an empty
// cache; the decode list
__global__ __launch_bounds__(1024) void assign_kernel(CacheDev c) {
    __shared__ uint32_t s_rebuild;
    const uint32_t tid = threadIdx.x;
    FrameState *st = c.st;
    if (tid == 0) {
        uint64_t need = 0;
        for (uint32_t t = 0; t < kLods; t++) {
            const uint32_t m = st->n_miss[t], avail = st->stack_top[t];
            if (m > avail) need += (uint64_t)(m - avail) * block_elems(t);
        }
        s_rebuild = st->top + need > c.cap_elems ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t *list = s_rebuild ? c.uniq : c.miss;
    if (s_rebuild) {
        // clear: every key uncached, stacks empty, top at the start
        const uint32_t nk = c.n_bricks * kLods;
        for (uint32_t key = tid; key < nk; key += blockDim.x) c.index[key] = kNone64;
        if (tid < kLods) st->stack_top[tid] = 0;
        if (tid == 0) {
            st->top = 0;
            st->rebuilt = 1;
            uint64_t need = 0;
            for (uint32_t t = 0; t < kLods; t++) need += (uint64_t)st->n_uniq[t] * block_elems(t);
            if (need > c.cap_elems) st->error = 1;  // the frame alone does not fit
        }
        __syncthreads();
        if (st->error) return;
    }
    uint32_t dec_base = 0;
    uint64_t top = st->top;
    for (uint32_t t = 0; t < kLods; t++) {
        const uint32_t m = s_rebuild ? st->n_uniq[t] : st->n_miss[t];
        const uint32_t avail = st->stack_top[t], take = min(m, avail);
        const uint32_t be = block_elems(t);
        for (uint32_t r = tid; r < m; r += blockDim.x) {
            const uint32_t key = list[t * c.n_req + r];
            const uint64_t e = r < take ? c.stacks[(size_t)t * c.n_bricks + (avail - 1 - r)]
                                        : top + (uint64_t)(r - take) * be;
            c.index[key] = e;
            c.dec_ids[dec_base + r] = key / kLods;
            c.dec_lods[dec_base + r] = (uint8_t)t;
            c.dec_off[dec_base + r] = e * 8;  // uint32 labels
        }
        top += (uint64_t)(m - take) * be;
        dec_base += m;
        __syncthreads();  // the stack entries taken are read before the top moves
        if (tid == 0) st->stack_top[t] = avail - take;
    }
    if (tid == 0) {
        st->top = top;
        st->n_dec = dec_base;
    }
}

// per request: element offset of its block in the cache, or ~0; with
// `served`, the LOD of that block (0xFF for none): a full-LOD request of a
// brick with detail in host memory whose full LOD is not cached was served
// at LOD 1
__global__ void slots_kernel(CacheDev c, const uint32_t *ids, const uint8_t *lods, const uint8_t *vis, uint32_t n,
                             uint64_t *slots, uint8_t *served) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = ids[r];
    uint32_t t = lods[r];
    uint64_t s = kNone64;
    if (id < c.n_bricks && t < kLods && (!vis || vis[r])) {
        if (t == 0 && c.det && (c.det[id] & kSplit) && c.index[id * kLods] == kNone64) t = 1;
        const uint64_t e = c.index[id * kLods + t];
        if (e != kNone64) s = e * 8;
    }
    slots[r] = s;
    if (served) served[r] = s == kNone64 ? (uint8_t)0xFF : (uint8_t)t;
}

// predicted bricks: pred[r] = the id if its detail is in host memory and
// its full LOD is not cached (after this frame's assignment), else ~0u;
// the caller's order is kept
__global__ void predict_kernel(CacheDev c, const uint32_t *ids, uint32_t n) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = ids[r];
    const bool need = id < c.n_bricks && (c.det[id] & kSplit) && c.index[id * kLods] == kNone64;
    c.pred[r] = need ? id : ~0u;
}

__global__ void fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct csv_frame_cache {
    csv_pool *pool = nullptr;
    int device = 0;
    uint32_t n_bricks = 0, max_req = 0;
    uint64_t cap_elems = 0;
    uint32_t *data = nullptr;  // the cache: cap_elems * 8 uint32 labels
    CacheDev d{};
    uint8_t *vis = nullptr;    // per request: visibility mask
    FrameState *h_st = nullptr;  // pinned copy of the frame state
    uint32_t last_n = 0;         // requests of the last frame
    // detail streaming (pools with level-0 detail in host memory)
    bool detail = false;
    uint8_t *d_det = nullptr;         // CacheDev::det
    uint8_t *h_det = nullptr;         // its pinned host image
    std::vector<uint32_t> det_gran;   // per brick: staging bytes of its detail (0: none in host memory)
    std::vector<uint32_t> staged;     // bricks this cache staged since the last release
    uint64_t stage_used = 0;          // staging bytes of those bricks
    uint8_t *h_lists = nullptr;       // pinned: frame state, wanted bricks, predictions of the last frame
    uint32_t list_n = 0, list_np = 0; // the last frame's requests and predictions
    bool lists_pending = false;
    hipEvent_t lists_ev = nullptr;    // the copy of the lists (and everything before it on the stream)
};

extern "C" {

int csv_frame_cache_create(csv_pool *pool, uint64_t cache_bytes, uint32_t max_requests, csv_frame_cache **out) {
    if (!pool || !out || max_requests == 0 || cache_bytes < 32) return CSV_EINVAL;
    *out = nullptr;
    csv_pool_info info;
    int rc = csv_pool_info_get(pool, &info);
    if (rc) return rc;
    if (info.n_bricks == 0 || info.brick_log2 != 5 || (uint64_t)info.n_bricks * kLods >= (1ull << 32))
        return CSV_EINVAL;  // blocks of 32^3 bricks
    csv_frame_cache *c = new (std::nothrow) csv_frame_cache;
    if (!c) return CSV_ENOMEM;
    c->pool = pool;
    c->device = info.device;
    c->n_bricks = info.n_bricks;
    c->max_req = max_requests;
    c->cap_elems = cache_bytes / 32;
    DeviceGuard g(c->device);
    const uint64_t nk = (uint64_t)info.n_bricks * kLods, nr = max_requests;
    CacheDev &d = c->d;
    d.n_bricks = info.n_bricks;
    d.n_req = max_requests;
    d.cap_elems = c->cap_elems;
    bool ok = hipMalloc(reinterpret_cast<void **>(&c->data), c->cap_elems * 32) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.index), 8 * nk) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.stamp), 4 * nk) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.stacks), 8ull * kLods * info.n_bricks) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.miss), 4 * kLods * nr) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.uniq), 4 * kLods * nr) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.dec_ids), 4 * nr) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.dec_lods), nr) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.dec_off), 8 * nr) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&d.st), sizeof(FrameState)) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&c->vis), nr) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void **>(&c->h_st), sizeof(FrameState), hipHostMallocDefault) ==
                  hipSuccess;
    if (ok && info.host_bytes) {
        // a pool with level-0 detail in host memory: which bricks, and how
        // much staging each takes
        c->detail = true;
        c->det_gran.assign(info.n_bricks, 0u);
        ok = hipHostMalloc(reinterpret_cast<void **>(&c->h_det), info.n_bricks, hipHostMallocDefault) == hipSuccess;
        for (uint32_t id = 0; ok && id < info.n_bricks; id++) {
            uint32_t b = 0;
            if (csv_pool_detail_bytes(pool, id, &b, nullptr) != CSV_OK) ok = false;
            c->det_gran[id] = b;
            c->h_det[id] = b ? kSplit : 0;
        }
        ok = ok && hipMalloc(reinterpret_cast<void **>(&c->d_det), info.n_bricks) == hipSuccess &&
             hipMalloc(reinterpret_cast<void **>(&d.want), 4 * nr) == hipSuccess &&
             hipMalloc(reinterpret_cast<void **>(&d.pred), 4 * nr) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void **>(&c->h_lists), sizeof(FrameState) + 8 * nr,
                           hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&c->lists_ev, hipEventDisableTiming) == hipSuccess &&
             hipMemcpy(c->d_det, c->h_det, info.n_bricks, hipMemcpyHostToDevice) == hipSuccess;
        d.det = c->d_det;
    }
    if (ok) {
        hipLaunchKernelGGL(fill_u64, dim3(256), dim3(256), 0, nullptr, d.index, nk, kNone64);
        hipLaunchKernelGGL(fill_u32, dim3(256), dim3(256), 0, nullptr, d.stamp, nk, 0u);
        ok = hipMemset(d.st, 0, sizeof(FrameState)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        csv_frame_cache_destroy(c);
        return CSV_ENOMEM;
    }
    *out = c;
    return CSV_OK;
}

static void fill_stats(const csv_frame_cache *c, const FrameState &st, csv_frame_stats *stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->frame = st.frame;
    stats->requests = c->last_n;
    for (uint32_t t = 0; t < kLods; t++) {
        stats->distinct += st.n_uniq[t];
        stats->new_entries += st.n_miss[t];
    }
    stats->decoded = st.error ? 0 : st.n_dec;
    stats->hits = st.error ? 0 : stats->distinct - st.n_dec;
    stats->evicted = st.evicted;
    stats->rebuilt = st.rebuilt;
    stats->used_bytes = st.top * 32;
    stats->capacity_bytes = c->cap_elems * 32;
}

// Detail for this frame (frames of caches over pools with level-0 detail in
// host memory): the last frame's wanted bricks (by id), then its predicted
// bricks that still need detail (in the caller's order), staged behind the
// detail already on the device when they fit, else after dropping it.
static int stage_frame_detail(csv_frame_cache *c, hipStream_t s, csv_frame_detail_stats *ds) {
    constexpr uint8_t kListed = 4;
    // the last frame's copies (lists, and the detail flags from the pinned
    // image) are done
    if (hipEventSynchronize(c->lists_ev) != hipSuccess) return CSV_EHIP;
    std::vector<uint32_t> list;  // each brick once: wanted (by id), then predicted
    uint32_t n_want = 0, n_pred = 0;
    if (c->lists_pending) {
        c->lists_pending = false;
        FrameState st;
        std::memcpy(&st, c->h_lists, sizeof(st));
        const uint32_t *want = reinterpret_cast<const uint32_t *>(c->h_lists + sizeof(FrameState));
        const uint32_t *pred = want + c->max_req;
        n_want = std::min(st.n_want, c->list_n);
        std::vector<uint32_t> w(want, want + n_want);
        std::sort(w.begin(), w.end());
        for (uint32_t r = 0; r < c->list_np; r++) n_pred += pred[r] < c->n_bricks ? 1u : 0u;
        auto add = [&](uint32_t id) {
            if (id >= c->n_bricks || (c->h_det[id] & kListed)) return;
            c->h_det[id] |= kListed;
            list.push_back(id);
        };
        for (uint32_t id : w) add(id);
        for (uint32_t r = 0; r < c->list_np; r++) add(pred[r]);
        for (uint32_t id : list) c->h_det[id] &= (uint8_t)~kListed;
    }
    uint64_t cap = 0;
    int rc = csv_pool_detail_bytes(c->pool, 0, nullptr, &cap);
    if (rc) return rc;
    // listed bricks whose detail is not staged
    std::vector<uint32_t> fresh;
    auto fresh_of = [&]() {
        uint64_t need = 0;
        fresh.clear();
        for (uint32_t id : list)
            if (!(c->h_det[id] & kStaged)) {
                fresh.push_back(id);
                need += c->det_gran[id];
            }
        return need;
    };
    const uint64_t need = fresh_of();
    bool changed = false, released = false;
    if (!c->staged.empty() && c->stage_used + need > cap) {
        rc = csv_pool_release_detail(c->pool, s);
        if (rc) return rc;
        for (uint32_t id : c->staged) c->h_det[id] &= (uint8_t)~kStaged;
        c->staged.clear();
        c->stage_used = 0;
        released = changed = true;
        fresh_of();
    }
    uint32_t done = 0;
    uint64_t up = 0;
    if (!fresh.empty()) {
        rc = csv_pool_stage_detail(c->pool, fresh.data(), (uint32_t)fresh.size(), s, &done);
        if (rc) return rc;
        for (uint32_t k = 0; k < done; k++) {
            const uint32_t id = fresh[k];
            if (!c->det_gran[id]) continue;
            c->h_det[id] |= kStaged;
            c->staged.push_back(id);
            c->stage_used += c->det_gran[id];
            up += c->det_gran[id];
        }
        changed = changed || done > 0;
    }
    if (changed && (hipMemcpyAsync(c->d_det, c->h_det, c->n_bricks, hipMemcpyHostToDevice, s) != hipSuccess ||
                    hipEventRecord(c->lists_ev, s) != hipSuccess))
        return CSV_EHIP;
    if (ds) {
        ds->wanted = n_want;
        ds->predicted = n_pred;
        for (uint32_t id : list) ds->staged += (c->h_det[id] & kStaged) ? 1u : 0u;
        ds->released = released ? 1u : 0u;
        ds->uploaded_bytes = up;
        ds->resident_bytes = c->stage_used;
    }
    return CSV_OK;
}

static int frame_impl(csv_frame_cache *c, const uint32_t *ids, const uint8_t *lods, uint32_t n,
                      const uint32_t *visible_bits, uint32_t n_label_bits, const uint32_t *pred, uint32_t n_pred,
                      uint64_t *slots, uint8_t *served, hipStream_t s, csv_frame_stats *stats,
                      csv_frame_detail_stats *dstats) {
    DeviceGuard g(c->device);
    const CacheDev &d = c->d;
    if (c->detail) {
        const int rc = stage_frame_detail(c, s, dstats);
        if (rc) return rc;
    }
    const bool test = visible_bits != nullptr || n_label_bits != 0;
    if (test && n) {
        const int rc = csv_bricks_visible(c->pool, ids, n, visible_bits, n_label_bits, c->vis, s);
        if (rc) return rc;
    }
    const uint8_t *vis = test ? c->vis : nullptr;
    const uint32_t gr = std::max(1u, (n + 255) / 256);
    hipLaunchKernelGGL(begin_kernel, dim3(1), dim3(64), 0, s, d);
    if (n) hipLaunchKernelGGL(mark_kernel, dim3(gr), dim3(256), 0, s, d, ids, lods, vis, n);
    const uint64_t nk = (uint64_t)c->n_bricks * kLods;
    hipLaunchKernelGGL(evict_kernel, dim3((uint32_t)std::min<uint64_t>((nk + 255) / 256, 4096)), dim3(256), 0, s, d);
    hipLaunchKernelGGL(assign_kernel, dim3(1), dim3(1024), 0, s, d);
    if (hipGetLastError() != hipSuccess) return CSV_EHIP;
    c->last_n = n;
    int rc = CSV_OK;
    FrameState st{};
    if (!stats) {
        // no round trip to the host: the decode reads the number of bricks
        // from the frame state (0 when the frame does not fit)
        if (n) rc = csv_decode_bricks_devcount(c->pool, d.dec_ids, d.dec_lods, 0, d.dec_off, n, &d.st->n_dec,
                                               c->data, s);
    } else {
        if (hipMemcpyAsync(c->h_st, d.st, sizeof(FrameState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return CSV_EHIP;
        st = *c->h_st;
        if (!st.error && st.n_dec)
            rc = csv_decode_bricks(c->pool, d.dec_ids, d.dec_lods, 0, d.dec_off, st.n_dec, c->data, s);
    }
    if (n) hipLaunchKernelGGL(slots_kernel, dim3(gr), dim3(256), 0, s, d, ids, lods, vis, n, slots, served);
    if (c->detail) {
        // the lists for the next frame: this frame's state (its count of
        // wanted bricks), the wanted bricks, the predictions still in need
        const uint32_t np = pred ? n_pred : 0;
        if (np) hipLaunchKernelGGL(predict_kernel, dim3((np + 255) / 256), dim3(256), 0, s, d, pred, np);
        uint8_t *hw = c->h_lists + sizeof(FrameState);
        if (hipMemcpyAsync(c->h_lists, d.st, sizeof(FrameState), hipMemcpyDeviceToHost, s) != hipSuccess ||
            (n && hipMemcpyAsync(hw, d.want, 4ull * n, hipMemcpyDeviceToHost, s) != hipSuccess) ||
            (np && hipMemcpyAsync(hw + 4ull * c->max_req, d.pred, 4ull * np, hipMemcpyDeviceToHost, s) !=
                       hipSuccess) ||
            hipEventRecord(c->lists_ev, s) != hipSuccess)
            return CSV_EHIP;
        c->list_n = n;
        c->list_np = np;
        c->lists_pending = true;
        if (dstats) dstats->fallbacks = st.n_want;
    }
    if (hipGetLastError() != hipSuccess && !rc) rc = CSV_EHIP;
    if (stats) {
        fill_stats(c, st, stats);
        if (!rc && st.error) rc = CSV_ENOMEM;
    }
    return rc;
}

int csv_frame_cache_frame(csv_frame_cache *c, const uint32_t *ids, const uint8_t *lods, uint32_t n,
                          const uint32_t *visible_bits, uint32_t n_label_bits, uint64_t *slots, void *stream,
                          csv_frame_stats *stats) {
    if (!c || c->detail || n > c->max_req || (n && (!ids || !lods || !slots))) return CSV_EINVAL;
    return frame_impl(c, ids, lods, n, visible_bits, n_label_bits, nullptr, 0, slots, nullptr,
                      reinterpret_cast<hipStream_t>(stream), stats, nullptr);
}

int csv_frame_cache_frame_detail(csv_frame_cache *c, const uint32_t *ids, const uint8_t *lods, uint32_t n,
                                 const uint32_t *visible_bits, uint32_t n_label_bits, const uint32_t *predict_ids,
                                 uint32_t n_predict, uint64_t *slots, uint8_t *served_lods, void *stream,
                                 csv_frame_stats *stats, csv_frame_detail_stats *detail_stats) {
    if (!c || n > c->max_req || n_predict > c->max_req || (n && (!ids || !lods || !slots)) ||
        (n_predict && !predict_ids) || (detail_stats && !stats))
        return CSV_EINVAL;
    if (detail_stats) std::memset(detail_stats, 0, sizeof(*detail_stats));
    return frame_impl(c, ids, lods, n, visible_bits, n_label_bits, predict_ids, n_predict, slots, served_lods,
                      reinterpret_cast<hipStream_t>(stream), stats, detail_stats);
}

int csv_frame_cache_last_stats(csv_frame_cache *c, csv_frame_stats *stats) {
    if (!c || !stats) return CSV_EINVAL;
    DeviceGuard g(c->device);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(c->h_st, c->d.st, sizeof(FrameState), hipMemcpyDeviceToHost) != hipSuccess)
        return CSV_EHIP;
    const FrameState st = *c->h_st;
    fill_stats(c, st, stats);
    return st.error ? CSV_ENOMEM : CSV_OK;
}

uint32_t *csv_frame_cache_data(csv_frame_cache *c) { return c ? c->data : nullptr; }

int csv_frame_cache_read(csv_frame_cache *c, uint64_t elem_offset, uint64_t n, uint32_t *host_dst) {
    if (!c || (n && !host_dst) || elem_offset > c->cap_elems * 8 || n > c->cap_elems * 8 - elem_offset)
        return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    DeviceGuard g(c->device);
    if (hipDeviceSynchronize() != hipSuccess) return CSV_EHIP;
    return hipMemcpy(host_dst, c->data + elem_offset, 4 * n, hipMemcpyDeviceToHost) == hipSuccess ? CSV_OK : CSV_EHIP;
}

void csv_frame_cache_destroy(csv_frame_cache *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->data);
    (void)hipFree(c->d.index);
    (void)hipFree(c->d.stamp);
    (void)hipFree(c->d.stacks);
    (void)hipFree(c->d.miss);
    (void)hipFree(c->d.uniq);
    (void)hipFree(c->d.dec_ids);
    (void)hipFree(c->d.dec_lods);
    (void)hipFree(c->d.dec_off);
    (void)hipFree(c->d.st);
    (void)hipFree(c->vis);
    if (c->h_st) (void)hipHostFree(c->h_st);
    if (c->h_det) (void)hipHostFree(c->h_det);
    (void)hipFree(c->d_det);
    (void)hipFree(c->d.want);
    (void)hipFree(c->d.pred);
    if (c->h_lists) (void)hipHostFree(c->h_lists);
    if (c->lists_ev) (void)hipEventDestroy(c->lists_ev);
    delete c;
}

}  // extern "C"
