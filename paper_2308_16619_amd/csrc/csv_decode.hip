// GPU brick decoder for gfx950 and the device pool that feeds it.
//
// A decode of n requests (brick, level of detail t; Sec. 3.4, Alg. 1) is
// two persistent launches that take requests from device work counters:
//
// A. entropy decode (Sec. 3.3).  One wavefront per brick, many per CU (the
//    only LDS is the decode tables and a 2 KB word ring per wave, so the
//    serial rANS chains of many bricks hide each other's latency).  The W
//    interleaved states run in lockstep, one per lane; a renormalising lane
//    takes its 16-bit word at the stream cursor plus the number of lower
//    lanes that renormalise too (wave ballot + mbcnt).  Eight lanes' 4-bit
//    symbols are OR-ed into one dword with DPP row shifts and stored to a
//    per-request nibble buffer in global memory (it stays in L2 / MALL).
//
// B. operation replay and output (Sec. 3.2, Alg. 1).  One 4-wave workgroup
//    per brick, several per CU, level by level in Morton order as palette
//    indices in LDS (u8 when the palette has at most 253 entries):
//      - one lane per expanded parent, in stream order; SWAR on its 8
//        (op, stop) nibbles counts P_a, P_delta and expanded children; wave
//        prefix sums plus the totals of the lower waves give every child its
//        palette position, delta slot and the next level's expanded list;
//      - a neighbour reference to a later node reads the parent level; one to
//        an earlier node of the same level always lands on a child with one
//        more coordinate bit set, so three passes of decreasing child
//        popcount resolve every chain;
//      - leaf values are kept only for the expanded L_1 nodes, found by a
//        popcount rank over the expansion bitmask;
//      - the level-t block goes through the palette to HBM as dense rows of
//        16-byte stores (a wave's store covers eight whole 128-byte rows).
//    Bricks whose arrays do not fit the LDS arena use the same code with
//    u16 indices and an arena in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/csv.h"
#include "csv_format.hpp"

namespace {

constexpr int kLog2 = 5;                 // 32^3 bricks
constexpr int kLutMaxBits = 11;          // largest supported table precision
constexpr uint32_t kMaxSym = 2 * 37448;  // every node an operation plus a delta nibble
constexpr uint32_t kLdsBytes = 160 * 1024;
constexpr uint32_t kLutLdsCap = 24 * 1024;  // decode tables kept in LDS when they fit
constexpr uint32_t kPalFast = 253;       // u8 path: palette indices 0..252, 253..255 mark open references
constexpr uint32_t kRingWords = 1024;    // per-wave word ring of the entropy decoder
#ifndef CSV_WAVES_B
#define CSV_WAVES_B 4
#endif
constexpr int kWavesB = CSV_WAVES_B;     // waves of a replay workgroup
constexpr uint32_t kThreadsB = 64 * kWavesB;
#ifndef CSV_REPLAY_ATTR
#define CSV_REPLAY_ATTR
#endif

// level m (1..4) offsets (entries) inside the Morton-ordered level arrays
__device__ constexpr uint32_t kLvOff[5] = {0, 0, 4096, 4608, 4672};
// expanded-node bit arrays (bytes, one per parent) for levels 1..4
__device__ constexpr uint32_t kBmOff[5] = {0, 0, 512, 576, 584};
// lists of expanded nodes (u16 entries) for levels 2..4; level 1 has its own
__device__ constexpr uint32_t kLstOff[5] = {0, 0, 72, 8, 0};

struct DecodeArgs {
    const uint64_t *rec_ptr;
    const uint32_t *rec_size;
    const uint16_t *rec_vol;
    const uint32_t *luts;     // all volumes' decode tables, back to back
    const uint32_t *lut_off;  // per volume: first entry of its two tables
    const uint32_t *vol_bits; // per volume: table precision
    uint32_t n_bricks;
    const uint32_t *ids;
    const uint8_t *lods;
    uint32_t lod_scalar;
    const uint64_t *out_off;
    uint32_t *out;
    uint32_t n;
    int *err;  // [0] first error code, [1] brick id (or request index)
};

// per-request status written by the entropy decoder for the replay
enum : uint8_t { kStOk = 0, kStFail = 1, kStNone = 2 };

struct LaunchA {
    uint32_t lut_lds_words;  // decode-table words in LDS (0: tables read from global memory)
    uint32_t *queue;         // work counter (nullptr: static round robin)
    const uint32_t *order;   // processing order of requests (nullptr: identity)
    uint32_t *nib;           // slot_dw dwords of packed nibbles per request
    uint32_t slot_dw;
    uint8_t *status;
    uint32_t base;           // first request index
};

struct LaunchB {
    uint32_t arena_bytes;    // LDS arena per workgroup
    uint32_t *queue;
    const uint32_t *order;
    const uint32_t *nib;
    uint32_t slot_dw;
    const uint8_t *status;
    uint8_t *scratch;        // global arena per workgroup for bricks that do not fit LDS
    uint32_t slot_bytes;
    uint32_t base;
};

// ---------------------------------------------------------------------------
// wave primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// inclusive prefix sum over the 64 lanes (DPP row shifts, then row broadcasts)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}
// OR of lanes [L - (2^kLevels - 1) .. L] within a 16-lane row
template <int kLevels>
__device__ __forceinline__ uint32_t row_or(uint32_t v) {
    if (kLevels >= 1) v |= __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);
    if (kLevels >= 2) v |= __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);
    if (kLevels >= 3) v |= __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);
    return v;
}

// order a wave's own LDS operations
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void report(int *err, int code, uint32_t who) {
    if (atomicCAS(err, 0, code) == 0) atomicExch(err + 1, (int)who);
}

// Per-brick phase clocks, only in builds with CSV_PHASE_TIMING: entry i of
// a request's 16 holds the shader clock at the end of phase i.
#ifdef CSV_PHASE_TIMING
__device__ uint64_t *g_phase = nullptr;
__device__ __forceinline__ void phase_mark(uint32_t rq, int i) {
    if (g_phase && __lane_id() == 0 && (i < 2 || threadIdx.x == 0)) g_phase[16 * (size_t)rq + i] = __builtin_amdgcn_s_memtime();
}
#else
__device__ __forceinline__ void phase_mark(uint32_t, int) {}
#endif

// ---------------------------------------------------------------------------
// bit helpers
// ---------------------------------------------------------------------------
// nibble k of z is zero -> bit 4k of the result
__device__ __forceinline__ uint32_t zero_nibbles(uint32_t z) { return ~(z | (z >> 1) | (z >> 2) | (z >> 3)) & 0x11111111u; }
// bits 0,4,..,28 -> bits 0..7
__device__ __forceinline__ uint32_t compact_nibble_bits(uint32_t m) {
    m = (m | (m >> 3)) & 0x03030303u;
    m = (m | (m >> 6)) & 0x000F000Fu;
    return (m | (m >> 12)) & 0xFFu;
}
// 4-bit coordinate -> Morton bit positions 0,3,6,9
__device__ __forceinline__ uint32_t spread4(uint32_t v) {
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4) | ((v & 8u) << 6);
}
// Morton mask of axis a for a grid of `bits` coordinate bits
__device__ __forceinline__ uint32_t axis_mask(int a, uint32_t bits) { return (0x49249249u & ((1u << (3 * bits)) - 1u)) << a; }
__device__ __forceinline__ uint32_t morton_inc(uint32_t m, uint32_t mask) { return (((m | ~mask) + 1u) & mask) | (m & ~mask); }
__device__ __forceinline__ uint32_t morton_dec(uint32_t m, uint32_t mask) { return (((m & mask) - 1u) & mask) | (m & ~mask); }

// 8 nibbles starting at nibble position p of a packed nibble array
__device__ __forceinline__ uint32_t nib8(const uint32_t *nib, uint32_t p) {
    const uint32_t lo = nib[p >> 3], hi = nib[(p >> 3) + 1];
    return __builtin_amdgcn_alignbit(hi, lo, 4 * (p & 7));
}
__device__ __forceinline__ uint32_t nib1(const uint32_t *nib, uint32_t p) { return (nib[p >> 3] >> (4 * (p & 7))) & 15u; }

// 8 palette indices as one vector
template <class IdxT> struct Vec8;
template <> struct Vec8<uint8_t> {
    using T = uint2;
    static __device__ __forceinline__ uint32_t get(const T &v, int k) { return ((k < 4 ? v.x : v.y) >> (8 * (k & 3))) & 0xFFu; }
    static __device__ __forceinline__ void set(T &v, int k, uint32_t x) {
        uint32_t &w = k < 4 ? v.x : v.y;
        w = (w & ~(0xFFu << (8 * (k & 3)))) | (x << (8 * (k & 3)));
    }
    static __device__ __forceinline__ T splat(uint32_t x) { x *= 0x01010101u; return make_uint2(x, x); }
};
template <> struct Vec8<uint16_t> {
    using T = uint4;
    static __device__ __forceinline__ uint32_t get(const T &v, int k) {
        const uint32_t w = k < 2 ? v.x : (k < 4 ? v.y : (k < 6 ? v.z : v.w));
        return (w >> (16 * (k & 1))) & 0xFFFFu;
    }
    static __device__ __forceinline__ void set(T &v, int k, uint32_t x) {
        uint32_t &w = k < 2 ? v.x : (k < 4 ? v.y : (k < 6 ? v.z : v.w));
        w = (w & ~(0xFFFFu << (16 * (k & 1)))) | (x << (16 * (k & 1)));
    }
    static __device__ __forceinline__ T splat(uint32_t x) { x *= 0x00010001u; return make_uint4(x, x, x, x); }
};

__host__ __device__ inline uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }

// Pointers into global memory.  Going through the global address space lets
// the compiler emit global (not flat) loads: a flat load also waits for LDS
// traffic, and on gfx9 any vector-memory wait also waits for earlier stores.
template <class T>
__device__ __forceinline__ T *glob(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)p;
}
__device__ __forceinline__ const uint32_t *rec_at(uint64_t a) {
    return (const uint32_t *)(const __attribute__((address_space(1))) uint32_t *)a;
}

// ---------------------------------------------------------------------------
// record header
// ---------------------------------------------------------------------------
struct Hdr {
    const uint32_t *rec;
    uint32_t P, W, nw, t, vol, rq, id;
    // cumulative symbol counts (scalars: a run-time level never indexes a private array)
    uint32_t c0, c1, c2, c3, c4;
    __device__ __forceinline__ uint32_t c(uint32_t m) const {
        return m == 0 ? c0 : (m == 1 ? c1 : (m == 2 ? c2 : (m == 3 ? c3 : c4)));
    }
};

enum ReqKind { kReqBadLod, kReqBadId, kReqCorrupt, kReqFill, kReqDecode };

// read and check request rq; for kReqFill, fill is the value of every output label
__device__ __forceinline__ ReqKind load_request(const DecodeArgs &a, uint32_t rq, Hdr &h, uint32_t *&dst,
                                                uint32_t &count, uint32_t &fill) {
    h.rq = rq;
    h.id = uniform(a.ids[rq]);
    h.t = uniform(a.lods ? (uint32_t)a.lods[rq] : a.lod_scalar);
    dst = nullptr;
    count = 0;
    fill = 0;
    if (h.t > (uint32_t)kLog2) return kReqBadLod;
    const uint32_t G = 32u >> h.t;
    count = G * G * G;
    dst = a.out + (a.out_off ? a.out_off[rq] : (uint64_t)rq * count);
    if (h.id >= a.n_bricks) return kReqBadId;
    h.rec = rec_at(a.rec_ptr[h.id]);
    const uint32_t size = a.rec_size[h.id];
    h.vol = a.rec_vol[h.id];
    h.P = h.rec[0];
    h.W = h.rec[1];
    h.nw = h.rec[2];
    h.c0 = h.rec[3];
    h.c1 = h.rec[4];
    h.c2 = h.rec[5];
    h.c3 = h.rec[6];
    h.c4 = h.rec[7];
    const uint32_t hdr = csv::record_header_words(kLog2);
    bool ok = h.P >= 1 && h.W <= 64 && (h.W & (h.W - 1)) == 0 && ((h.c0 > 0) == (h.W > 0)) && h.c0 <= kMaxSym &&
              (uint64_t)4 * (hdr + h.P + h.W) + 2ull * h.nw <= size;
    ok = ok && h.c0 >= h.c1 && h.c1 >= h.c2 && h.c2 >= h.c3 && h.c3 >= h.c4;
    if (ok) ok = (h.c0 == 0) ? (h.P == 1) : (h.P >= 2);
    if (!ok) return kReqCorrupt;
    if (h.t == (uint32_t)kLog2 || h.c0 == 0) {  // coarsest level or uniform brick: palette[0]
        fill = h.rec[hdr];
        return kReqFill;
    }
    return kReqDecode;
}

// ===========================================================================
// A. entropy decode
// ===========================================================================
// kLutLds: the decode tables of every volume are copied to LDS (else read
// from global memory)
template <int WPG, bool kLutLds>
__global__ __launch_bounds__(WPG * 64) void rans_kernel(DecodeArgs a, LaunchA l) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *slut = reinterpret_cast<uint32_t *>(smem);
    if (kLutLds)
        for (uint32_t e = threadIdx.x; e < l.lut_lds_words; e += blockDim.x) slut[e] = a.luts[e];
    __syncthreads();
    const uint32_t L = lane(), wave = threadIdx.x >> 6;
    uint32_t *ring32 = reinterpret_cast<uint32_t *>(smem + align16(4 * l.lut_lds_words) + wave * kRingWords * 2);
    const uint16_t *ring = reinterpret_cast<const uint16_t *>(ring32);
    const uint32_t wid = blockIdx.x * WPG + wave;
    const uint32_t hdr = csv::record_header_words(kLog2);
    for (uint32_t k = 0;; k++) {
        uint32_t req;
        if (l.queue) {
            uint32_t v = 0;
            if (L == 0) v = atomicAdd(l.queue, 1u);
            req = uniform(v) + l.base;
        } else {
            req = l.base + wid + k * gridDim.x * WPG;
        }
        if (req >= a.n) break;
        const uint32_t rq = l.order ? l.order[req] : req;
        phase_mark(rq, 0);
        Hdr h;
        uint32_t *dst, count, fill;
        const ReqKind kind = load_request(a, rq, h, dst, count, fill);
        uint8_t st = kStOk;
        if (kind == kReqBadLod) {
            if (L == 0) report(a.err, CSV_ERANGE, rq);
            st = kStNone;
        } else if (kind == kReqBadId) {
            if (L == 0) report(a.err, CSV_ERANGE, rq);
            st = kStFail;
        } else if (kind == kReqCorrupt) {
            if (L == 0) report(a.err, CSV_ECORRUPT, h.id);
            st = kStFail;
        } else if (kind == kReqDecode) {
            const uint32_t n = h.c(h.t);
            uint32_t *out = glob(l.nib) + (size_t)rq * l.slot_dw;
            if (n + 16 > 8 * l.slot_dw) {  // the buffers are sized for the pool's largest brick
                if (L == 0) report(a.err, CSV_EINVAL, h.id);
                st = kStFail;
            } else {
                const uint32_t sbits = a.vol_bits[h.vol], lutn = 1u << sbits, mask = lutn - 1u;
                const uint32_t *lut = (kLutLds ? (const uint32_t *)slut : glob(a.luts)) + a.lut_off[h.vol];
                const uint32_t W = h.W, lw = 31u - (uint32_t)__builtin_clz(W), leaf = h.c1;
                const uint32_t *wg = h.rec + hdr + h.P + W;
                const uint32_t ndw = (h.nw + 1) / 2;  // word dwords in the record (the last one padded)
                uint32_t x = L < W ? h.rec[hdr + h.P + L] : 0u;
                // the ring holds words [ring_lo, ring_lo + 1024); pf holds the next 512
                uint32_t ring_lo = 0;
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const uint32_t d = L + 64 * q;
                    ring32[d] = d < ndw ? wg[d] : 0u;
                }
                uint32_t pf[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const uint32_t d = 512 + L + 64 * q;
                    pf[q] = d < ndw ? wg[d] : 0u;
                }
                wsync();
                uint32_t cursor = 0, acc = 0;
                bool bad = false;
                const uint32_t steps = (n + W - 1) >> lw;
                uint32_t s = 0;
                if (W == 64) {
                    // steps with all 64 lanes busy: no per-lane conditions; every
                    // lane reads a ring word and keeps it if it renormalises
                    for (const uint32_t full = n >> 6; s < full; s++) {
                        const uint32_t i = (s << 6) + L;
                        const uint32_t e = lut[(i >= leaf ? lutn : 0u) + (x & mask)];
                        const uint32_t sym = e & 15u;
                        x = (e >> 16) * (x >> sbits) + ((e >> 4) & 0xFFFu);
                        const bool need = x < csv::kRansLower;
                        const uint64_t bal = __ballot(need);
                        const uint32_t wd = ring[(cursor + mbcnt(bal)) & (kRingWords - 1)];
                        x = need ? ((x << 16) | wd) : x;
                        cursor += (uint32_t)__popcll(bal);
                        const uint32_t g = row_or<3>(sym << (4 * (L & 7u)));
                        if ((L & 7u) == 7u) out[(i - 7) >> 3] = g;
                        if (cursor >= ring_lo + 512) {  // the oldest half is consumed: refill it
                            const uint32_t hh = (ring_lo >> 9) & 1u;
                            wsync();
#pragma unroll
                            for (int q = 0; q < 4; q++) ring32[hh * 256 + L + 64 * q] = pf[q];
                            ring_lo += 512;
                            const uint32_t d0 = (ring_lo + 1024) >> 1;
#pragma unroll
                            for (int q = 0; q < 4; q++) {
                                const uint32_t d = d0 + L + 64 * q;
                                pf[q] = d < ndw ? wg[d] : 0u;
                            }
                            wsync();
                        }
                    }
                    // words past the end of the stream came from stale ring entries
                    bad = cursor > h.nw;
                    if (bad) s = steps;
                }
                for (; s < steps; s++) {
                    const uint32_t i = (s << lw) + L;
                    const bool act = L < W && i < n;
                    uint32_t sym = 0;
                    bool need = false;
                    if (act) {
                        const uint32_t e = lut[(i >= leaf ? lutn : 0u) + (x & mask)];
                        sym = e & 15u;
                        x = (e >> 16) * (x >> sbits) + ((e >> 4) & 0xFFFu);
                        need = x < csv::kRansLower;
                    }
                    const uint64_t bal = __ballot(need);
                    const uint32_t cnt = (uint32_t)__popcll(bal);
                    if (cursor + cnt > h.nw) {
                        bad = true;
                        break;
                    }
                    if (need) x = (x << 16) | (uint32_t)ring[(cursor + mbcnt(bal)) & (kRingWords - 1)];
                    cursor += cnt;
                    // 8 consecutive symbols -> one dword of the nibble buffer
                    const uint32_t v = sym << (4 * (i & 7));
                    if (W >= 8) {
                        const uint32_t g = row_or<3>(v);
                        if ((L & 7) == 7 && L < W && i - 7 < n) out[(i - 7) >> 3] = g;
                    } else {
                        const uint32_t g = W == 4 ? row_or<2>(v) : (W == 2 ? row_or<1>(v) : v);
                        acc |= g;
                        const bool full = (((s + 1) << lw) & 7) == 0;
                        if (L == W - 1 && (full || s + 1 == steps)) out[(s << lw) >> 3] = acc;
                        if (full) acc = 0;
                    }
                    if (cursor >= ring_lo + 512) {  // the oldest half is consumed: refill it
                        const uint32_t hh = (ring_lo >> 9) & 1u;
                        wsync();
#pragma unroll
                        for (int q = 0; q < 4; q++) ring32[hh * 256 + L + 64 * q] = pf[q];
                        ring_lo += 512;
                        const uint32_t d0 = (ring_lo + 1024) >> 1;
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const uint32_t d = d0 + L + 64 * q;
                            pf[q] = d < ndw ? wg[d] : 0u;
                        }
                        wsync();
                    }
                }
                // a complete decode ends in the encoder's initial states with every word read
                if (!bad && h.t == 0) bad = (__ballot(L < W && x != csv::kRansLower) != 0) || cursor != h.nw;
                if (bad) {
                    if (L == 0) report(a.err, CSV_ECORRUPT, h.id);
                    st = kStFail;
                }
            }
        }
        if (L == 0) l.status[rq] = st;
        phase_mark(rq, 1);
    }
}

// ===========================================================================
// B. operation replay and output
// ===========================================================================
struct SmallB {
    uint32_t req;
    int err;
    uint32_t wt[kWavesB][3];  // per-wave totals of P_a, P_delta, expanded children
};

struct LayoutB {
    uint32_t pal, nib, nib_dw, lv, bm, bpre, lst, list1, l0x, total;
};
// stage: the P palette entries and nib_dw dwords of packed nibbles are
// copied to the arena; S0 leaf-segment symbols (0 unless decoding to LOD 0);
// idx bytes per palette index
__host__ __device__ inline LayoutB make_layout_b(bool stage, uint32_t P, uint32_t S0, uint32_t idx, uint32_t nib_dw) {
    LayoutB L;
    uint32_t o = 0;
    const uint32_t e1 = S0 / 8 < 4096 ? S0 / 8 : 4096;
    L.pal = o; o += stage ? align16(4 * P) : 0;
    L.nib = o; o += stage ? align16(4 * nib_dw) : 0;
    L.nib_dw = stage ? nib_dw : 0;
    L.lv = o; o += align16(4680 * idx);
    L.bm = o; o += 592;
    L.bpre = o; o += 160;
    L.lst = o; o += align16(2 * (8 + 64 + 512));
    L.list1 = o; o += align16(2 * e1);
    L.l0x = o; o += align16(8 * e1 * idx);
    L.total = o;
    return L;
}

// children of one expanded parent from its 8 (op, stop) nibbles w: pv parent
// index; nb[a] the parent-level neighbour at +1 along axis a (valid if bit a
// of nbok); lowok bit a: the parent is not on the low face of axis a; ipb
// palette position before the first child; pam8/pdm8 children with P_a /
// P_delta; their deltas from nibble db of dnib on.
template <class IdxT>
__device__ __forceinline__ typename Vec8<IdxT>::T replay_children(uint32_t w, uint32_t pv, const uint32_t nb[3],
                                                                  uint32_t nbok, uint32_t lowok, uint32_t ipb,
                                                                  uint32_t pam8, uint32_t pdm8, const uint32_t *dnib,
                                                                  uint32_t db, uint32_t P, bool leaf, bool &bad) {
    using V = Vec8<IdxT>;
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    typename V::T out = V::splat(0);
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t nbl = (w >> (4 * k)) & 15u, op = nbl & 7u;
        const uint32_t below = (1u << k) - 1u;
        const uint32_t ipk = ipb + __builtin_popcount(pam8 & below);
        uint32_t v = pv;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (op == (uint32_t)(1 + a)) {
                if ((k >> a) & 1) {
                    v = nb[a];
                    bad |= !((nbok >> a) & 1u);
                } else {
                    v = kMark + (uint32_t)a;  // same-level neighbour at -1, resolved later
                    bad |= !((lowok >> a) & 1u);
                }
            }
        }
        if (op == csv::kP0) v = ipk;
        if (op == csv::kPa) {
            v = ipk + 1;
            bad |= ipk + 1 >= P;
        }
        if (op == csv::kPd) {
            const uint32_t d = nib1(dnib, db + __builtin_popcount(pdm8 & below));
            bad |= ipk < d + 1;
            v = ipk - 1 - d;
        }
        bad |= op == 7u;
        bad |= leaf && nbl >= 8u;
        V::set(out, k, v & (sizeof(IdxT) == 1 ? 0xFFu : 0xFFFFu));
    }
    return out;
}

// palette lookup; indices are checked while decoding, the clamp only keeps a
// malformed record from reading past a palette held in global memory
template <bool kG>
__device__ __forceinline__ uint32_t pal_at(const uint32_t *pal, uint32_t i, uint32_t P) {
    if constexpr (kG) return pal[i < P ? i : P - 1];
    return pal[i];
}

// four labels to dst (16-byte aligned when al16; outputs of mixed levels of
// detail need not be)
__device__ __forceinline__ void store4(uint32_t *dst, const uint4 &o, bool al16) {
    if (al16) {
        *reinterpret_cast<uint4 *>(dst) = o;
    } else {
        dst[0] = o.x;
        dst[1] = o.y;
        dst[2] = o.z;
        dst[3] = o.w;
    }
}

__device__ __forceinline__ void wg_fill(uint32_t *dst, uint32_t count, uint32_t v) {
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0 && (count & 3) == 0) {
        const uint4 q = make_uint4(v, v, v, v);
        for (uint32_t e = 4 * threadIdx.x; e < count; e += 4 * kThreadsB) *reinterpret_cast<uint4 *>(dst + e) = q;
    } else {
        for (uint32_t e = threadIdx.x; e < count; e += kThreadsB) dst[e] = v;
    }
}

// counts of one expanded parent's 8 nibbles: P_a | P_delta << 10 | (stop 0) << 20
__device__ __forceinline__ void nibble_counts(uint32_t w, bool act, uint32_t &pam, uint32_t &pdm, uint32_t &exm,
                                              uint32_t &cnt) {
    const uint32_t y = w & 0x77777777u;
    pam = act ? zero_nibbles(y ^ 0x66666666u) : 0u;
    pdm = act ? zero_nibbles(y ^ 0x55555555u) : 0u;
    exm = act ? (~w >> 3) & 0x11111111u : 0u;
    cnt = __builtin_popcount(pam) | (__builtin_popcount(pdm) << 10) | (__builtin_popcount(exm) << 20);
}

// the replay of one brick by one workgroup; false on a malformed stream
template <class IdxT, bool kG>
__device__ __forceinline__ bool replay_brick(const Hdr &h, const uint32_t *gnib, uint8_t *ar, const LayoutB &lay,
                                             SmallB *sm, uint32_t *dst) {
    using V = Vec8<IdxT>;
    using VT = typename V::T;
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    const uint32_t tid = threadIdx.x, L = lane(), w = tid >> 6;
    const uint32_t t = h.t, P = h.P;
    const uint32_t hdr = csv::record_header_words(kLog2);
    const uint32_t *pal = kG ? h.rec + hdr : reinterpret_cast<const uint32_t *>(ar + lay.pal);
    IdxT *lv = reinterpret_cast<IdxT *>(ar + lay.lv);
    uint8_t *bm = ar + lay.bm;
    uint16_t *bpre = reinterpret_cast<uint16_t *>(ar + lay.bpre);
    uint16_t *lst = reinterpret_cast<uint16_t *>(ar + lay.lst);
    uint16_t *list1 = reinterpret_cast<uint16_t *>(ar + lay.list1);
    const uint32_t tl = t > 1 ? t : 1u;  // finest upper level replayed
    const uint32_t S0 = t == 0 ? h.c0 - h.c1 : 0u;
    const uint32_t e1cap = S0 / 8 < 4096 ? S0 / 8 : 4096u;
    const uint32_t *nib = gnib;
    if (!kG) {  // stage the palette and the brick's nibbles (16-byte aligned at both ends)
        for (uint32_t e = tid; e < P; e += kThreadsB) reinterpret_cast<uint32_t *>(ar + lay.pal)[e] = h.rec[hdr + e];
        uint4 *ln = reinterpret_cast<uint4 *>(ar + lay.nib);
        const uint4 *src = reinterpret_cast<const uint4 *>(gnib);
        for (uint32_t e = tid; e < (lay.nib_dw + 3) / 4; e += kThreadsB) ln[e] = src[e];
        nib = reinterpret_cast<const uint32_t *>(ar + lay.nib);
    }
    if (tid == 0) sm->err = 0;
    __syncthreads();
    phase_mark(h.rq, 8);

    uint32_t E = 1;    // expanded parents of the level being built (the root)
    uint32_t ipl = 0;  // P_a operations so far
    for (int m = kLog2 - 1; m >= (int)tl; m--) {
        const uint32_t Bp = (uint32_t)(kLog2 - 1 - m);  // parent grid bits
        const uint32_t np = 1u << (3 * Bp);
        IdxT *cur = lv + kLvOff[m];
        const IdxT *up = (m + 1 <= 4) ? lv + kLvOff[m + 1] : nullptr;
        uint8_t *cbm = bm + kBmOff[m];
        const uint8_t *pbm = (m + 1 <= 4) ? bm + kBmOff[m + 1] : nullptr;
        const uint16_t *plist = (m + 1 <= 4) ? lst + kLstOff[m + 1] : nullptr;
        const bool want_list = (m >= 2) || t == 0;
        uint16_t *clist = (m >= 2) ? lst + kLstOff[m] : list1;
        const uint32_t list_cap = (m >= 2) ? (1u << (3 * (kLog2 - m))) : e1cap;
        // children of parents that are not expanded inherit the parent's index
        for (uint32_t q = tid; q < np; q += kThreadsB) {
            const bool ex = pbm ? ((pbm[q >> 3] >> (q & 7)) & 1u) : true;
            cbm[q] = 0;
            if (!ex) *reinterpret_cast<VT *>(cur + 8 * q) = V::splat(up ? (uint32_t)up[q] : 0u);
        }
        const uint32_t seg = (m == kLog2 - 1) ? 0u : h.c((uint32_t)m + 1), seg_end = h.c((uint32_t)m);
        if ((uint64_t)seg + 8ull * E > seg_end) return false;
        const uint32_t D = seg_end - seg - 8 * E, ops0 = seg + D;  // deltas precede the operations
        const uint32_t nch = (E + 63) / 64, cpw = (nch + kWavesB - 1) / kWavesB;
        const uint32_t cb = min(w * cpw, nch), ce = min(cb + cpw, nch);  // this wave's chunks
        // pass 1: this wave's totals
        uint32_t tpa = 0, tpd = 0, tex = 0;
        for (uint32_t c = cb; c < ce; c++) {
            const uint32_t r = 64 * c + L;
            const bool act = r < E;
            const uint32_t wd = act ? nib8(nib, ops0 + 8 * r) : 0u;
            uint32_t pam, pdm, exm, cnt;
            nibble_counts(wd, act, pam, pdm, exm, cnt);
            const uint32_t tot = uniform(__builtin_amdgcn_readlane(wave_incl_scan(cnt), 63));
            tpa += tot & 1023u;
            tpd += (tot >> 10) & 1023u;
            tex += tot >> 20;
        }
        if (L == 0) {
            sm->wt[w][0] = tpa;
            sm->wt[w][1] = tpd;
            sm->wt[w][2] = tex;
        }
        __syncthreads();
        uint32_t bpa = 0, bpd = 0, bex = 0, PAtot = 0, PDtot = 0, EXtot = 0;
#pragma unroll
        for (int v = 0; v < kWavesB; v++) {
            const uint32_t a0 = sm->wt[v][0], a1 = sm->wt[v][1], a2 = sm->wt[v][2];
            if ((uint32_t)v < w) {
                bpa += a0;
                bpd += a1;
                bex += a2;
            }
            PAtot += a0;
            PDtot += a1;
            EXtot += a2;
        }
        if (PDtot != D || (want_list && EXtot > list_cap)) return false;
        // pass 2: children
        bool bad = false;
        const uint32_t pmask0 = axis_mask(0, Bp), pmask1 = axis_mask(1, Bp), pmask2 = axis_mask(2, Bp);
        for (uint32_t c = cb; c < ce; c++) {
            const uint32_t r = 64 * c + L;
            const bool act = r < E;
            const uint32_t q = (act && plist) ? (uint32_t)plist[r] : 0u;
            const uint32_t wd = act ? nib8(nib, ops0 + 8 * r) : 0u;
            uint32_t pam, pdm, exm, cnt;
            nibble_counts(wd, act, pam, pdm, exm, cnt);
            const uint32_t inc = wave_incl_scan(cnt), exc = inc - cnt;
            const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
            if (act) {
                const uint32_t pv = up ? (uint32_t)up[q] : 0u;
                uint32_t nb[3], nbok = 0, lowok = 0;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const uint32_t am = a == 0 ? pmask0 : (a == 1 ? pmask1 : pmask2);
                    const bool hi = up && (q & am) != am;
                    nb[a] = hi ? (uint32_t)up[morton_inc(q, am)] : 0u;
                    nbok |= hi ? (1u << a) : 0u;
                    lowok |= (q & am) ? (1u << a) : 0u;
                }
                const VT vals = replay_children<IdxT>(wd, pv, nb, nbok, lowok, ipl + bpa + (exc & 1023u),
                                                      compact_nibble_bits(pam), compact_nibble_bits(pdm), nib,
                                                      seg + bpd + ((exc >> 10) & 1023u), P, false, bad);
                *reinterpret_cast<VT *>(cur + 8 * q) = vals;
                uint32_t ex8 = compact_nibble_bits(exm);
                cbm[q] = (uint8_t)ex8;
                if (want_list) {
                    uint32_t pos = bex + (exc >> 20);
                    while (ex8) {
                        const uint32_t k = __builtin_ctz(ex8);
                        ex8 &= ex8 - 1;
                        if (pos < list_cap) clist[pos] = (uint16_t)(8 * q + k);
                        pos++;
                    }
                }
            }
            bpa += tot & 1023u;
            bpd += (tot >> 10) & 1023u;
            bex += tot >> 20;
        }
        if (__ballot(bad) && L == 0) atomicOr(&sm->err, 1);
        __syncthreads();
        if (sm->err) return false;
        // neighbour references into this level: a reference to child k of
        // the -1 neighbour along a lands on child k | 1 << a, so a chain has
        // at most three links; a chain is followed to its end while other
        // lanes resolve in place (a reader sees either the reference or its
        // final value, and both lead to the same value)
        for (uint32_t r = tid; r < E; r += kThreadsB) {
            const uint32_t q = plist ? (uint32_t)plist[r] : 0u;
            VT vals = *reinterpret_cast<const VT *>(cur + 8 * q);
            bool dirty = false;
#pragma unroll
            for (int k = 0; k < 7; k++) {
                uint32_t v = V::get(vals, k);
                if (v >= kMark) {
                    uint32_t qq = q, kk = (uint32_t)k;
                    do {
                        const int a = (int)(v - kMark);
                        qq = morton_dec(qq, a == 0 ? pmask0 : (a == 1 ? pmask1 : pmask2));
                        kk |= 1u << a;
                        v = cur[8 * qq + kk];
                    } while (v >= kMark);
                    V::set(vals, k, v);
                    dirty = true;
                }
            }
            if (dirty) *reinterpret_cast<VT *>(cur + 8 * q) = vals;
        }
        __syncthreads();
        phase_mark(h.rq, 13 - m);
        ipl += PAtot;
        E = EXtot;
    }
    phase_mark(h.rq, 2);

    const uint32_t G = 32u >> t;
    const bool al16 = (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
    if (t >= 1) {
        // ---- output of an upper level -------------------------------------------
        const IdxT *res = lv + kLvOff[t];
        if (t == 4) {
            if (tid < 8) dst[tid] = pal_at<kG>(pal, res[tid], P);  // Morton order equals dense order on 2^3
        } else {
            const uint32_t lg = (uint32_t)(kLog2 - t);
            for (uint32_t e = 4 * tid; e < G * G * G; e += 4 * kThreadsB) {
                const uint32_t x0 = e & (G - 1), yy = (e >> lg) & (G - 1), zz = e >> (2 * lg);
                const uint32_t m0 = spread4(x0) | (spread4(yy) << 1) | (spread4(zz) << 2);
                uint4 o;
                o.x = pal_at<kG>(pal, res[m0], P);
                o.y = pal_at<kG>(pal, res[m0 | 1u], P);
                o.z = pal_at<kG>(pal, res[m0 | 8u], P);
                o.w = pal_at<kG>(pal, res[m0 | 9u], P);
                store4(dst + e, o, al16);
            }
        }
        phase_mark(h.rq, 5);
        return true;
    }

    // ---- leaf level ------------------------------------------------------------
    const uint32_t E1 = E;
    const IdxT *l1 = lv + kLvOff[1];
    const uint8_t *bm1 = bm + kBmOff[1];
    const uint64_t *bm1w = reinterpret_cast<const uint64_t *>(bm1);
    IdxT *l0x = reinterpret_cast<IdxT *>(ar + lay.l0x);
    if (w == 0) {  // rank prefix of the expanded L_1 bits, per 64-bit word
        const uint32_t c = (uint32_t)__popcll(bm1w[L]);
        bpre[L] = (uint16_t)(wave_incl_scan(c) - c);
    }
    const uint32_t seg = h.c1, seg_end = h.c0;
    if ((uint64_t)seg + 8ull * E1 > seg_end) return false;
    const uint32_t D0 = seg_end - seg - 8 * E1, ops0 = seg + D0;
    const uint32_t nch = (E1 + 63) / 64, cpw = (nch + kWavesB - 1) / kWavesB;
    const uint32_t cb = min(w * cpw, nch), ce = min(cb + cpw, nch);
    uint32_t tpa = 0, tpd = 0;
    for (uint32_t c = cb; c < ce; c++) {
        const uint32_t r = 64 * c + L;
        const bool act = r < E1;
        const uint32_t wd = act ? nib8(nib, ops0 + 8 * r) : 0u;
        uint32_t pam, pdm, exm, cnt;
        nibble_counts(wd, act, pam, pdm, exm, cnt);
        const uint32_t tot = uniform(__builtin_amdgcn_readlane(wave_incl_scan(cnt & 0xFFFFFu), 63));
        tpa += tot & 1023u;
        tpd += (tot >> 10) & 1023u;
    }
    if (L == 0) {
        sm->wt[w][0] = tpa;
        sm->wt[w][1] = tpd;
    }
    __syncthreads();
    uint32_t bpa = 0, bpd = 0, PDtot = 0;
#pragma unroll
    for (int v = 0; v < kWavesB; v++) {
        const uint32_t a0 = sm->wt[v][0], a1 = sm->wt[v][1];
        if ((uint32_t)v < w) {
            bpa += a0;
            bpd += a1;
        }
        PDtot += a1;
    }
    if (PDtot != D0) return false;
    bool bad = false;
    const uint32_t m0 = axis_mask(0, 4), m1 = axis_mask(1, 4), m2 = axis_mask(2, 4);
    for (uint32_t c = cb; c < ce; c++) {
        const uint32_t r = 64 * c + L;
        const bool act = r < E1;
        const uint32_t wd = act ? nib8(nib, ops0 + 8 * r) : 0u;
        const uint32_t p = act ? (uint32_t)list1[r] : 0u;
        uint32_t pam, pdm, exm, cnt;
        nibble_counts(wd, act, pam, pdm, exm, cnt);
        cnt &= 0xFFFFFu;
        const uint32_t inc = wave_incl_scan(cnt), exc = inc - cnt;
        const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
        if (act) {
            const uint32_t pv = l1[p];
            uint32_t nbv[3], nbok = 0, lowok = 0;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const uint32_t am = a == 0 ? m0 : (a == 1 ? m1 : m2);
                const bool hi = (p & am) != am;
                nbv[a] = hi ? (uint32_t)l1[morton_inc(p, am)] : 0u;
                nbok |= hi ? (1u << a) : 0u;
                lowok |= (p & am) ? (1u << a) : 0u;
            }
            const VT vals = replay_children<IdxT>(wd, pv, nbv, nbok, lowok, ipl + bpa + (exc & 1023u),
                                                  compact_nibble_bits(pam), compact_nibble_bits(pdm), nib,
                                                  seg + bpd + ((exc >> 10) & 1023u), P, true, bad);
            *reinterpret_cast<VT *>(l0x + 8 * r) = vals;
        }
        bpa += tot & 1023u;
        bpd += (tot >> 10) & 1023u;
    }
    if (__ballot(bad) && L == 0) atomicOr(&sm->err, 1);
    __syncthreads();
    if (sm->err) return false;
    phase_mark(h.rq, 3);
    // leaf neighbour references, resolved as on the upper levels; a chain
    // ends at a non-expanded L_1 node, whose value is final
    for (uint32_t r = tid; r < E1; r += kThreadsB) {
        VT vals = *reinterpret_cast<const VT *>(l0x + 8 * r);
        bool dirty = false;
        uint32_t p = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 7; k++) {
            uint32_t v = V::get(vals, k);
            if (v >= kMark) {
                if (p == 0xFFFFFFFFu) p = list1[r];
                uint32_t pp = p, kk = (uint32_t)k;
                do {
                    const int a = (int)(v - kMark);
                    pp = morton_dec(pp, a == 0 ? m0 : (a == 1 ? m1 : m2));
                    kk |= 1u << a;
                    if ((bm1[pp >> 3] >> (pp & 7)) & 1u) {
                        const uint32_t rk = bpre[pp >> 6] + (uint32_t)__popcll(bm1w[pp >> 6] & ((1ull << (pp & 63)) - 1ull));
                        v = l0x[8 * rk + kk];
                    } else {
                        v = l1[pp];
                    }
                } while (v >= kMark);
                V::set(vals, k, v);
                dirty = true;
            }
        }
        if (dirty) *reinterpret_cast<VT *>(l0x + 8 * r) = vals;
    }
    __syncthreads();
    phase_mark(h.rq, 4);

    // ---- leaf output: a lane covers two x-adjacent L_1 nodes, 4 rows of 16 bytes ----
    for (uint32_t it = w; it < 32; it += kWavesB) {
        const uint32_t xp = L & 7u, Y = (L >> 3) | ((it & 1u) << 3), Z = it >> 1;
        const uint32_t p0 = spread4(2 * xp) | (spread4(Y) << 1) | (spread4(Z) << 2);
        VT v8[2];
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const uint32_t p = p0 | (uint32_t)b;
            if ((bm1[p >> 3] >> (p & 7)) & 1u) {
                const uint32_t rk = bpre[p >> 6] + (uint32_t)__popcll(bm1w[p >> 6] & ((1ull << (p & 63)) - 1ull));
                v8[b] = *reinterpret_cast<const VT *>(l0x + 8 * rk);
            } else {
                v8[b] = V::splat(l1[p]);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {  // c = cy | cz << 1
            const int k0 = ((c & 1) << 1) | ((c >> 1) << 2);
            uint4 o;
            o.x = pal_at<kG>(pal, V::get(v8[0], k0), P);
            o.y = pal_at<kG>(pal, V::get(v8[0], k0 | 1), P);
            o.z = pal_at<kG>(pal, V::get(v8[1], k0), P);
            o.w = pal_at<kG>(pal, V::get(v8[1], k0 | 1), P);
            const uint32_t yy = 2 * Y + (uint32_t)(c & 1), zz = 2 * Z + (uint32_t)(c >> 1);
            store4(dst + 4 * xp + 32 * (yy + 32 * zz), o, al16);
        }
    }
    phase_mark(h.rq, 5);
    return true;
}

__global__ __launch_bounds__(kThreadsB) CSV_REPLAY_ATTR void replay_kernel(DecodeArgs a, LaunchB l) {
    extern __shared__ __align__(16) uint8_t smem[];
    SmallB *sm = reinterpret_cast<SmallB *>(smem);
    uint8_t *arena = smem + align16(sizeof(SmallB));
    uint8_t *gslot = l.scratch ? l.scratch + (size_t)blockIdx.x * l.slot_bytes : nullptr;
    const uint32_t tid = threadIdx.x;
    for (uint32_t k = 0;; k++) {
        if (tid == 0) sm->req = l.queue ? atomicAdd(l.queue, 1u) + l.base : l.base + blockIdx.x + k * gridDim.x;
        __syncthreads();
        const uint32_t req = sm->req;
        if (req >= a.n) break;
        const uint32_t rq = l.order ? l.order[req] : req;
        Hdr h;
        uint32_t *dst, count, fill;
        const ReqKind kind = load_request(a, rq, h, dst, count, fill);
        const uint8_t st = l.status[rq];
        if (kind == kReqBadLod || st == kStNone) {
            // nothing to write (reported by the entropy decoder)
        } else if (kind != kReqDecode || st == kStFail) {
            wg_fill(dst, count, (kind == kReqFill && st == kStOk) ? fill : 0u);
        } else {
            const uint32_t *nib = glob(l.nib) + (size_t)rq * l.slot_dw;
            const uint32_t S0 = h.t == 0 ? h.c0 - h.c1 : 0u;
            const LayoutB fast = make_layout_b(true, h.P, S0, 1, (h.c(h.t) + 7) / 8 + 2);
            const bool fits = h.P <= kPalFast && fast.total <= l.arena_bytes;
            bool ok;
            phase_mark(rq, 6);
            if (fits) {
                ok = replay_brick<uint8_t, false>(h, nib, arena, fast, sm, dst);
            } else if (gslot) {
                phase_mark(rq, 7);
                ok = replay_brick<uint16_t, true>(h, nib, gslot, make_layout_b(false, h.P, S0, 2, 0), sm, dst);
            } else {
                ok = false;
            }
            __syncthreads();
            if (!ok) {
                if (tid == 0) report(a.err, (fits || gslot) ? CSV_ECORRUPT : CSV_EINVAL, h.id);
                wg_fill(dst, count, 0);
            }
        }
        __syncthreads();
    }
}

// Longest-first request order: requests are binned by the log2 of their
// work (symbols to decode plus output voxels / 8), largest bin first, and
// laid out bin by bin.  ws: 2 x 32 counters.
constexpr int kBins = 32;
__device__ __forceinline__ uint32_t work_bin(const DecodeArgs &a, uint32_t r) {
    const uint32_t id = a.ids[r];
    const uint32_t t = a.lods ? (uint32_t)a.lods[r] : a.lod_scalar;
    if (id >= a.n_bricks || t > (uint32_t)kLog2) return kBins - 1;
    const uint32_t *rec = rec_at(a.rec_ptr[id]);
    const uint32_t n = t < (uint32_t)kLog2 ? rec[3 + t] : 0u;
    const uint32_t g = 32u >> t;
    const uint32_t work = n + (g * g * g) / 8 + 1;
    return (uint32_t)__builtin_clz(work);  // 32 - bit length: small for big work
}
__global__ void order_count(DecodeArgs a, uint32_t *ws) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < a.n; r += gridDim.x * blockDim.x)
        atomicAdd(&ws[work_bin(a, r)], 1u);
}
__global__ void order_scan(uint32_t *ws) {
    if (threadIdx.x == 0) {
        uint32_t o = 0;
        for (int b = 0; b < kBins; b++) {
            ws[kBins + b] = o;
            o += ws[b];
        }
    }
}
__global__ void order_scatter(DecodeArgs a, uint32_t *ws, uint32_t *order) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < a.n; r += gridDim.x * blockDim.x)
        order[atomicAdd(&ws[kBins + work_bin(a, r)], 1u)] = r;
}
__global__ void zero_words(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}


// Per-stream launch buffers: the nibble buffer and status bytes that pass
// requests from the entropy decoder to the replay, the longest-first order,
// and the two work counters.  Launches on one stream are ordered, so they
// share one set; launches on different streams get different sets.
struct LaunchBufs {
    hipStream_t stream = nullptr;
    uint64_t last_use = 0;
    uint32_t *nib = nullptr;
    uint8_t *status = nullptr;
    uint32_t *order = nullptr;
    uint32_t *small = nullptr;  // [0, 64): order bins; [64, 66): work counters
    uint32_t slot_dw = 0;
    uint32_t cap_n = 0;
    void release() {
        (void)hipFree(nib);
        (void)hipFree(status);
        (void)hipFree(order);
        (void)hipFree(small);
        nib = nullptr;
        status = nullptr;
        order = nullptr;
        small = nullptr;
        cap_n = 0;
    }
    // room for n requests of slot_dw nibble dwords each
    int reserve(uint32_t n, uint32_t dw) {
        if (nib && n <= cap_n && dw == slot_dw) return CSV_OK;
        release();
        const uint32_t cap = std::max(n, 1024u);
        if (hipMalloc(reinterpret_cast<void **>(&nib), 4ull * cap * dw + 64) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&status), cap) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&order), 4ull * cap) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&small), 4 * 66) != hipSuccess) {
            release();
            return CSV_ENOMEM;
        }
        cap_n = cap;
        slot_dw = dw;
        return CSV_OK;
    }
    uint64_t bytes() const { return nib ? (4ull * cap_n * slot_dw + 64 + 5ull * cap_n + 4 * 66) : 0; }
};
constexpr size_t kMaxStreamBufs = 16;

}  // namespace

struct csv_pool {
    int device = 0;
    int n_cu = 0;
    std::vector<void *> vol_bufs;
    std::vector<uint64_t> rec_ptr;
    std::vector<uint32_t> rec_size;
    std::vector<uint16_t> rec_vol;
    std::vector<uint32_t> luts;
    std::vector<uint32_t> lut_off;
    std::vector<uint32_t> bits;
    uint64_t *d_rec_ptr = nullptr;
    uint32_t *d_rec_size = nullptr;
    uint16_t *d_rec_vol = nullptr;
    uint32_t *d_luts = nullptr;
    uint32_t *d_lut_off = nullptr;
    uint32_t *d_bits = nullptr;
    int *d_err = nullptr;
    std::vector<LaunchBufs> bufs;             // per stream, at most kMaxStreamBufs
    uint64_t use_clock = 0;
    uint8_t *d_scratch = nullptr;             // global replay arenas
    uint32_t slot_bytes = 0;
    uint32_t n_slots = 0;
    uint32_t max_c0 = 0;                      // most symbols of any brick in the pool
    uint32_t max_fast_bytes = 0;              // largest LDS arena a brick of the pool needs
    bool any_big_palette = false;
    uint32_t generation = 0;                  // bumped when device tables move
    csv_shape shape{16, 4, 1, 0, 0.f};        // launch shape of csv_decode_bricks
    uint64_t record_bytes = 0;
    std::mutex mu;
};

namespace {

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

template <class T>
int upload(T **dptr, const std::vector<T> &h) {
    if (*dptr) {
        (void)hipFree(*dptr);
        *dptr = nullptr;
    }
    if (h.empty()) return CSV_OK;
    if (hipMalloc(reinterpret_cast<void **>(dptr), sizeof(T) * h.size()) != hipSuccess) return CSV_ENOMEM;
    if (hipMemcpy(*dptr, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return CSV_EHIP;
    return CSV_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

uint32_t lut_lds_words(const csv_pool *p) {
    const uint32_t lw = (uint32_t)p->luts.size();
    return (4 * lw <= kLutLdsCap) ? lw : 0u;
}
// nibble dwords per request: a multiple of 4, so every request's nibbles start 16-byte aligned
uint32_t slot_dw(const csv_pool *p) { return ((p->max_c0 + 7) / 8 + 4 + 3) & ~3u; }
constexpr uint32_t kSmallB = (sizeof(SmallB) + 15u) & ~15u;
constexpr uint32_t kMaxGroupsB = 8;
// replay arena when `groups` replay workgroups share a CU's LDS
uint32_t arena_b(uint32_t groups) { return ((kLdsBytes / groups) - kSmallB) & ~15u; }
uint32_t min_arena_b() { return arena_b(kMaxGroupsB); }

// the buffers of stream s, sized for n requests (pool->mu held)
int stream_bufs(csv_pool *pool, hipStream_t s, uint32_t n, LaunchBufs **out) {
    LaunchBufs *b = nullptr;
    for (auto &e : pool->bufs)
        if (e.stream == s) b = &e;
    const bool cap = capturing(s);
    if (!b) {
        if (pool->bufs.size() < kMaxStreamBufs) {
            pool->bufs.emplace_back();
            b = &pool->bufs.back();
        } else {  // hand the least recently used set to this stream once all work has finished
            if (cap) return CSV_EBUSY;
            if (hipDeviceSynchronize() != hipSuccess) return CSV_EHIP;
            b = &pool->bufs[0];
            for (auto &e : pool->bufs)
                if (e.last_use < b->last_use) b = &e;
        }
        b->stream = s;
    }
    b->last_use = ++pool->use_clock;
    const uint32_t dw = slot_dw(pool);
    if (!b->nib || n > b->cap_n || dw != b->slot_dw) {
        if (cap) return CSV_EBUSY;  // buffers cannot be re-sized inside a capture
        if (b->nib && hipStreamSynchronize(s) != hipSuccess) return CSV_EHIP;
        const int rc = b->reserve(n, dw);
        if (rc) return rc;
    }
    *out = b;
    return CSV_OK;
}

template <class F>
hipError_t set_lds_attr(F *f) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kLdsBytes);
}

template <int WPG>
void launch_a(const DecodeArgs &a, const LaunchA &l, uint32_t grid, size_t lds, hipStream_t s) {
    static std::once_flag once;
    std::call_once(once, [] {
        (void)set_lds_attr(rans_kernel<WPG, true>);
        (void)set_lds_attr(rans_kernel<WPG, false>);
    });
    if (l.lut_lds_words)
        hipLaunchKernelGGL((rans_kernel<WPG, true>), dim3(grid), dim3(64 * WPG), lds, s, a, l);
    else
        hipLaunchKernelGGL((rans_kernel<WPG, false>), dim3(grid), dim3(64 * WPG), lds, s, a, l);
}

// waves_a: entropy-decoder waves per workgroup; groups_b: replay workgroups
// per CU; fixed: buffers owned by the caller (a captured graph), else the
// stream's own set
int launch(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar, const uint64_t *out_off,
           uint32_t n, uint32_t *out, void *stream, bool plain, int waves_a, uint32_t groups_b, bool queue,
           bool lpt, LaunchBufs *fixed = nullptr) {
    if (!pool || (n && (!ids || !out))) return CSV_EINVAL;
    if (!lods && lod_scalar > (uint32_t)kLog2) return CSV_ERANGE;
    if (lods && !out_off) return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    if (pool->rec_ptr.empty() || !pool->d_err) return CSV_EINVAL;
    if (waves_a != 4 && waves_a != 8 && waves_a != 16) return CSV_EINVAL;
    if (groups_b < 1 || groups_b > kMaxGroupsB) return CSV_EINVAL;
    DeviceGuard g(pool->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    static std::once_flag once_b;
    static hipError_t attr_b = hipSuccess;
    std::call_once(once_b, [] { attr_b = set_lds_attr(replay_kernel); });
    if (attr_b != hipSuccess) return CSV_EHIP;
    std::lock_guard<std::mutex> lk(pool->mu);
    LaunchBufs *B = fixed;
    if (!B) {
        const int rc = stream_bufs(pool, s, n, &B);
        if (rc) return rc;
    } else if (n > B->cap_n) {
        return CSV_EINVAL;
    }
    DecodeArgs a;
    a.rec_ptr = pool->d_rec_ptr;
    a.rec_size = pool->d_rec_size;
    a.rec_vol = pool->d_rec_vol;
    a.luts = pool->d_luts;
    a.lut_off = pool->d_lut_off;
    a.vol_bits = pool->d_bits;
    a.n_bricks = (uint32_t)pool->rec_ptr.size();
    a.ids = ids;
    a.lods = lods;
    a.lod_scalar = lod_scalar;
    a.out_off = out_off;
    a.out = out;
    a.n = n;
    a.err = pool->d_err;
    LaunchA la;
    la.lut_lds_words = lut_lds_words(pool);
    la.queue = nullptr;
    la.order = nullptr;
    la.nib = B->nib;
    la.slot_dw = B->slot_dw;
    la.status = B->status;
    la.base = 0;
    LaunchB lb;
    lb.arena_bytes = arena_b(groups_b);
    lb.queue = nullptr;
    lb.order = nullptr;
    lb.nib = la.nib;
    lb.slot_dw = la.slot_dw;
    lb.status = la.status;
    lb.scratch = pool->d_scratch;
    lb.slot_bytes = pool->slot_bytes;
    lb.base = 0;
    const size_t lds_b = kSmallB + (size_t)lb.arena_bytes;
    const uint32_t cu = (uint32_t)std::max(1, pool->n_cu);
    // entropy decoder: as many workgroups as a CU's LDS and 32 wave slots allow
    const uint32_t lds_a = align16(4 * la.lut_lds_words) + (uint32_t)waves_a * kRingWords * 2;
    const uint32_t fit_a = std::max(1u, std::min(kLdsBytes / lds_a, 32u / (uint32_t)waves_a));
    const uint32_t grid_a = std::max(1u, std::min(cu * fit_a, (n + (uint32_t)waves_a - 1) / (uint32_t)waves_a));
    uint32_t grid_b = std::min(cu * groups_b, n);
    if (pool->d_scratch) grid_b = std::min(grid_b, pool->n_slots);
    auto go_a = [&](const DecodeArgs &aa, const LaunchA &L, uint32_t grid) {
        switch (waves_a) {
            case 4: launch_a<4>(aa, L, grid, lds_a, s); break;
            case 8: launch_a<8>(aa, L, grid, lds_a, s); break;
            default: launch_a<16>(aa, L, grid, lds_a, s); break;
        }
    };
    if (plain) {
        DecodeArgs b = a;
        for (uint32_t i = 0; i < n; i++) {
            la.base = lb.base = i;
            b.n = i + 1;
            go_a(b, la, 1);
            hipLaunchKernelGGL(replay_kernel, dim3(1), dim3(kThreadsB), lds_b, s, b, lb);
        }
    } else {
        if (lpt) {
            const uint32_t gq = std::min<uint32_t>((n + 255) / 256, 1024u);
            hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, B->small, 2u * kBins);
            hipLaunchKernelGGL(order_count, dim3(gq), dim3(256), 0, s, a, B->small);
            hipLaunchKernelGGL(order_scan, dim3(1), dim3(64), 0, s, B->small);
            hipLaunchKernelGGL(order_scatter, dim3(gq), dim3(256), 0, s, a, B->small, B->order);
            la.order = lb.order = B->order;
        }
        if (queue) {
            uint32_t *q = B->small + 2 * kBins;
            la.queue = q;
            lb.queue = q + 1;
            hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, q, 2u);
        }
        go_a(a, la, grid_a);
        hipLaunchKernelGGL(replay_kernel, dim3(grid_b), dim3(kThreadsB), lds_b, s, a, lb);
    }
    return hipGetLastError() == hipSuccess ? CSV_OK : CSV_EHIP;
}

bool valid_shape(const csv_shape &sh) {
    return (sh.waves_per_group == 4 || sh.waves_per_group == 8 || sh.waves_per_group == 16) &&
           sh.groups_per_cu >= 1 && sh.groups_per_cu <= kMaxGroupsB;
}

}  // namespace

extern "C" {

int csv_pool_create(csv_pool **pool, int device) {
    if (!pool) return CSV_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CSV_EINVAL;
    csv_pool *p = new (std::nothrow) csv_pool;
    if (!p) return CSV_ENOMEM;
    p->device = device;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete p;
        return CSV_EHIP;
    }
    p->n_cu = prop.multiProcessorCount;
    p->n_slots = (uint32_t)p->n_cu * kMaxGroupsB;  // one global replay arena per replay workgroup
    if (hipMalloc(reinterpret_cast<void **>(&p->d_err), 2 * sizeof(int)) != hipSuccess ||
        hipMemset(p->d_err, 0, 2 * sizeof(int)) != hipSuccess) {
        (void)hipFree(p->d_err);
        delete p;
        return CSV_ENOMEM;
    }
    *pool = p;
    return CSV_OK;
}

void csv_pool_destroy(csv_pool *p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    for (void *b : p->vol_bufs) (void)hipFree(b);
    (void)hipFree(p->d_rec_ptr);
    (void)hipFree(p->d_rec_size);
    (void)hipFree(p->d_rec_vol);
    (void)hipFree(p->d_luts);
    (void)hipFree(p->d_lut_off);
    (void)hipFree(p->d_bits);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_scratch);
    for (auto &b : p->bufs) b.release();
    delete p;
}

int csv_pool_add_volume(csv_pool *p, const uint8_t *blob, size_t blob_bytes, uint32_t *first_brick_id) {
    if (!p || !blob) return CSV_EINVAL;
    csv_volume_info info;
    int rc = csv_blob_info(blob, blob_bytes, &info);
    if (rc) return rc;
    if (info.brick_log2 != (uint32_t)kLog2 || info.scale_bits > (uint32_t)kLutMaxBits) return CSV_EINVAL;
    if ((uint64_t)p->rec_ptr.size() + info.n_bricks >= (1ull << 32) || p->bits.size() >= 65535) return CSV_ERANGE;
    std::lock_guard<std::mutex> lk(p->mu);
    DeviceGuard g(p->device);
    const uint64_t rs = csv::record_area_offset(info.n_bricks);
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + csv::kHeaderBytes);
    const uint32_t hdr = csv::record_header_words(kLog2);
    // every record must hold its header; offsets are 4-byte aligned and increasing
    uint32_t max_fast = p->max_fast_bytes, max_c0 = p->max_c0;
    bool big = p->any_big_palette;
    for (uint32_t i = 0; i < info.n_bricks; i++) {
        if (index[i + 1] < index[i] + 4 * hdr || (index[i] & 3)) return CSV_ECORRUPT;
        const uint32_t *w = reinterpret_cast<const uint32_t *>(blob + rs + index[i]);
        const uint32_t P = w[0], c0 = w[3], c1 = w[4];
        if (c0 == 0) continue;
        if (c1 > c0 || c0 > kMaxSym) return CSV_ECORRUPT;
        big |= P > kPalFast;
        max_c0 = std::max(max_c0, c0);
        max_fast = std::max(max_fast, make_layout_b(true, P, c0 - c1, 1, (c0 + 7) / 8 + 2).total);
    }
    // the kernels run to the end of a record; 64 bytes of slack cover their last vector loads
    void *buf = nullptr;
    const size_t rb = std::max<uint64_t>(info.record_bytes, 4) + 64;
    if (hipMalloc(&buf, rb) != hipSuccess) return CSV_ENOMEM;
    if (hipMemcpy(buf, blob + rs, info.record_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        return CSV_EHIP;
    }
    // all work that may read the tables about to move must be done
    (void)hipDeviceSynchronize();
    // a global replay arena per replay workgroup when some brick may not fit an LDS arena
    if ((big || max_fast > min_arena_b()) && !p->d_scratch) {
        p->slot_bytes = align16(make_layout_b(false, 0, kMaxSym, 2, 0).total);
        if (hipMalloc(reinterpret_cast<void **>(&p->d_scratch), (size_t)p->slot_bytes * p->n_slots) != hipSuccess) {
            (void)hipFree(buf);
            p->slot_bytes = 0;
            return CSV_ENOMEM;
        }
    }
    p->max_c0 = max_c0;
    p->max_fast_bytes = max_fast;
    p->any_big_palette = big;
    p->generation++;
    const uint32_t first = (uint32_t)p->rec_ptr.size();
    const uint16_t vol = (uint16_t)p->bits.size();
    p->vol_bufs.push_back(buf);
    p->record_bytes += info.record_bytes;
    for (uint32_t i = 0; i < info.n_bricks; i++) {
        p->rec_ptr.push_back(reinterpret_cast<uint64_t>(buf) + index[i]);
        p->rec_size.push_back((uint32_t)(index[i + 1] - index[i]));
        p->rec_vol.push_back(vol);
    }
    p->bits.push_back(info.scale_bits);
    p->lut_off.push_back((uint32_t)p->luts.size());
    for (int tb = 0; tb < 2; tb++)
        for (uint32_t s = 0; s < 16; s++)
            for (uint32_t q = 0; q < info.freq[tb][s]; q++) p->luts.push_back(csv::lut_entry(s, q, info.freq[tb][s]));
    if ((rc = upload(&p->d_rec_ptr, p->rec_ptr)) || (rc = upload(&p->d_rec_size, p->rec_size)) ||
        (rc = upload(&p->d_rec_vol, p->rec_vol)) || (rc = upload(&p->d_luts, p->luts)) ||
        (rc = upload(&p->d_lut_off, p->lut_off)) || (rc = upload(&p->d_bits, p->bits)))
        return rc;
    if (first_brick_id) *first_brick_id = first;
    return CSV_OK;
}

int csv_pool_info_get(const csv_pool *p, csv_pool_info *info) {
    if (!p || !info) return CSV_EINVAL;
    info->n_volumes = (uint32_t)p->bits.size();
    info->n_bricks = (uint32_t)p->rec_ptr.size();
    info->device = p->device;
    uint64_t lb = 0;
    for (const auto &b : p->bufs) lb += b.bytes();
    info->device_bytes = p->record_bytes + p->rec_ptr.size() * (8 + 4 + 2) + p->luts.size() * 4 +
                         (uint64_t)p->slot_bytes * (p->d_scratch ? p->n_slots : 0) + lb;
    return CSV_OK;
}

int csv_output_elems(const uint8_t *lods_host, uint32_t n, uint64_t *offsets, uint64_t *total) {
    if ((n && !lods_host) || !total) return CSV_EINVAL;
    uint64_t o = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (lods_host[i] > kLog2) return CSV_ERANGE;
        if (offsets) offsets[i] = o;
        const uint64_t g = 32u >> lods_host[i];
        o += g * g * g;
    }
    *total = o;
    return CSV_OK;
}

int csv_decode_bricks(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                      const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    if (!pool) return CSV_EINVAL;
    const csv_shape sh = pool->shape;
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, false,
                  sh.waves_per_group, (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0);
}

int csv_decode_bricks_plain(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                            const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    if (!pool) return CSV_EINVAL;
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, true,
                  pool->shape.waves_per_group, (uint32_t)pool->shape.groups_per_cu, false, false);
}

int csv_decode_bricks_shaped(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                             const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, const csv_shape *shape) {
    if (!pool || !shape || !valid_shape(*shape)) return CSV_EINVAL;
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, false,
                  shape->waves_per_group, (uint32_t)shape->groups_per_cu, shape->use_queue != 0,
                  shape->lpt_order != 0);
}

int csv_pool_set_shape(csv_pool *pool, const csv_shape *shape) {
    if (!pool || !shape || !valid_shape(*shape)) return CSV_EINVAL;
    pool->shape = *shape;
    return CSV_OK;
}

int csv_pool_get_shape(const csv_pool *pool, csv_shape *shape) {
    if (!pool || !shape) return CSV_EINVAL;
    *shape = pool->shape;
    return CSV_OK;
}

int csv_autotune(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                 const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, uint32_t reps, csv_shape *best) {
    if (!pool || !n || !reps) return CSV_EINVAL;
    DeviceGuard g(pool->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (capturing(s)) return CSV_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CSV_EHIP;
    const int waves[3] = {4, 8, 16};
    const uint32_t groups[5] = {3, 4, 5, 6, 8};
    csv_shape win{};
    win.ms = 1e30f;
    int rc = CSV_OK;
    for (int wi = 0; wi < 3 && !rc; wi++)
        for (int gi = 0; gi < 5 && !rc; gi++)
            for (int o = 0; o < 2 && !rc; o++) {
                csv_shape sh{waves[wi], groups[gi], 1, o, 0.f};
                // one warm-up launch, then reps timed launches
                rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group,
                            (uint32_t)sh.groups_per_cu, true, o != 0);
                if (rc) break;
                (void)hipEventRecord(e0, s);
                for (uint32_t r = 0; r < reps && !rc; r++)
                    rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group,
                                (uint32_t)sh.groups_per_cu, true, o != 0);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) rc = CSV_EHIP;
                float ms = 0.f;
                if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CSV_EHIP;
                sh.ms = ms / (float)reps;
                if (!rc && sh.ms < win.ms) win = sh;
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    pool->shape = win;
    if (best) *best = win;
    return CSV_OK;
}

struct csv_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t own = nullptr;
    const csv_pool *pool = nullptr;
    uint32_t generation = 0;
    LaunchBufs bufs;  // the captured launches' own buffers
    int device = 0;
};

static void graph_free(csv_graph *G) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    if (G->own) (void)hipStreamDestroy(G->own);
    G->bufs.release();
    delete G;
}

int csv_graph_create(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                     const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, csv_graph **graph) {
    if (!pool || !graph || !n) return CSV_EINVAL;
    DeviceGuard g(pool->device);
    csv_graph *G = new (std::nothrow) csv_graph;
    if (!G) return CSV_ENOMEM;
    G->device = pool->device;
    G->pool = pool;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (capturing(s)) {
        delete G;
        return CSV_EBUSY;
    }
    if (!s) {
        if (hipStreamCreateWithFlags(&G->own, hipStreamNonBlocking) != hipSuccess) {
            delete G;
            return CSV_EHIP;
        }
        s = G->own;
    }
    const csv_shape sh = pool->shape;
    int rc;
    {
        std::lock_guard<std::mutex> lk(pool->mu);
        G->generation = pool->generation;
        rc = G->bufs.reserve(n, slot_dw(pool));
    }
    if (!rc && hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = CSV_EHIP;
    if (!rc) {
        rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, s, false, sh.waves_per_group,
                    (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0, &G->bufs);
        hipGraph_t gr = nullptr;
        if (hipStreamEndCapture(s, &gr) != hipSuccess && !rc) rc = CSV_EHIP;
        G->graph = gr;
        if (!rc && hipGraphInstantiate(&G->exec, gr, nullptr, nullptr, 0) != hipSuccess) rc = CSV_EHIP;
    }
    if (rc) {
        graph_free(G);
        return rc;
    }
    *graph = G;
    return CSV_OK;
}

int csv_graph_launch(csv_graph *graph, void *stream) {
    if (!graph || !graph->exec) return CSV_EINVAL;
    // a volume added since the capture moved the tables the graph reads
    if (graph->pool->generation != graph->generation) return CSV_EBUSY;
    DeviceGuard g(graph->device);
    return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? CSV_OK : CSV_EHIP;
}

void csv_graph_destroy(csv_graph *graph) {
    if (!graph) return;
    DeviceGuard g(graph->device);
    (void)hipDeviceSynchronize();
    graph_free(graph);
}

#ifdef CSV_PHASE_TIMING
// install (or clear, with NULL) a device buffer of 16 u64 clocks per request
int csv_debug_phase_buffer(uint64_t *dev_buf) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_phase), &dev_buf, sizeof(dev_buf)) == hipSuccess ? CSV_OK : CSV_EHIP;
}
#endif

int csv_pool_last_error(csv_pool *p, int *code, uint32_t *brick_id) {
    if (!p || !code) return CSV_EINVAL;
    DeviceGuard g(p->device);
    int h[2] = {0, 0};
    if (hipDeviceSynchronize() != hipSuccess) return CSV_EHIP;
    if (hipMemcpy(h, p->d_err, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return CSV_EHIP;
    if (hipMemset(p->d_err, 0, sizeof(h)) != hipSuccess) return CSV_EHIP;
    *code = h[0];
    if (brick_id) *brick_id = (uint32_t)h[1];
    return CSV_OK;
}

}  // extern "C"
