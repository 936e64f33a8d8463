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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

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
};

__global__ void begin_kernel(CacheDev c) {
    if (threadIdx.x == 0) {
        c.st->frame++;
        c.st->n_dec = c.st->evicted = c.st->rebuilt = c.st->error = 0;
    }
    if (threadIdx.x < kLods) {
        c.st->n_miss[threadIdx.x] = 0;
        c.st->n_uniq[threadIdx.x] = 0;
    }
}

// request r: a visible, cacheable key is stamped with the frame; its first
// request this frame lists it (and, if not cached, as a miss)
__global__ void mark_kernel(CacheDev c, const uint32_t *ids, const uint8_t *lods, const uint8_t *vis, uint32_t n) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = ids[r], t = lods[r];
    if (id >= c.n_bricks || t >= kLods || (vis && !vis[r])) return;
    const uint32_t key = id * kLods + t, frame = c.st->frame;
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

// per request: element offset of its block in the cache, or ~0
__global__ void slots_kernel(CacheDev c, const uint32_t *ids, const uint8_t *lods, const uint8_t *vis, uint32_t n,
                             uint64_t *slots) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = ids[r], t = lods[r];
    uint64_t s = kNone64;
    if (id < c.n_bricks && t < kLods && (!vis || vis[r])) {
        const uint64_t e = c.index[id * kLods + t];
        if (e != kNone64) s = e * 8;
    }
    slots[r] = s;
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

int csv_frame_cache_frame(csv_frame_cache *c, const uint32_t *ids, const uint8_t *lods, uint32_t n,
                          const uint32_t *visible_bits, uint32_t n_label_bits, uint64_t *slots, void *stream,
                          csv_frame_stats *stats) {
    if (!c || n > c->max_req || (n && (!ids || !lods || !slots))) return CSV_EINVAL;
    DeviceGuard g(c->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const CacheDev &d = c->d;
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
    if (!stats) {
        // no round trip to the host: the decode reads the number of bricks
        // from the frame state (0 when the frame does not fit)
        int rc = CSV_OK;
        if (n) rc = csv_decode_bricks_devcount(c->pool, d.dec_ids, d.dec_lods, 0, d.dec_off, n, &d.st->n_dec,
                                               c->data, s);
        if (n) hipLaunchKernelGGL(slots_kernel, dim3(gr), dim3(256), 0, s, d, ids, lods, vis, n, slots);
        if (hipGetLastError() != hipSuccess && !rc) rc = CSV_EHIP;
        return rc;
    }
    if (hipMemcpyAsync(c->h_st, d.st, sizeof(FrameState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return CSV_EHIP;
    const FrameState st = *c->h_st;
    int rc = CSV_OK;
    if (!st.error && st.n_dec)
        rc = csv_decode_bricks(c->pool, d.dec_ids, d.dec_lods, 0, d.dec_off, st.n_dec, c->data, s);
    if (n) hipLaunchKernelGGL(slots_kernel, dim3(gr), dim3(256), 0, s, d, ids, lods, vis, n, slots);
    if (hipGetLastError() != hipSuccess && !rc) rc = CSV_EHIP;
    fill_stats(c, st, stats);
    if (!rc && st.error) rc = CSV_ENOMEM;
    return rc;
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
    delete c;
}

}  // extern "C"
