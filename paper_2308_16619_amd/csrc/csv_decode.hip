// GPU brick decoder for gfx950 and the device pool that feeds it.
//
// A decode of n requests (brick, level of detail t; Sec. 3.4, Alg. 1) is
// two persistent launches (large batches: per chunk of requests, the chunks
// alternating between two streams):
//
// A. front kernel: one wavefront per brick, 16 per CU, 8 KB of LDS each;
//    requests by round robin (optionally in longest-first order) or from a
//    work counter.
//    - Entropy decode (Sec. 3.3).  The W interleaved states run in
//      lockstep, one per lane; a renormalising lane takes its 16-bit word at
//      the stream cursor plus the number of lower lanes that renormalise too
//      (wave ballot + mbcnt) from a 2 KB ring of the word stream.  Eight
//      lanes' 4-bit symbols are OR-ed into one dword with DPP row shifts and
//      stored to the request's slot in global memory (it stays in L2 / MALL).
//    - Replay of levels 4 .. max(t, 1) (Sec. 3.2, Alg. 1) by the same wave,
//      level by level in Morton order as palette indices in its LDS (u8 when
//      the palette has at most 253 entries, else u16 in the slot): one lane
//      per expanded parent in stream order, SWAR on its 8 (op, stop)
//      nibbles, a wave prefix sum for palette positions, delta slots and the
//      next level's expanded list.  A neighbour reference to a later node
//      reads the parent level; one to an earlier node of the same level
//      lands on a child with one more coordinate bit set, so every chain has
//      at most three links and is followed to its end.
//    - t >= 1: the level-t block goes through the palette to the output.
//      t = 0: L_1, its expansion bits and the list of expanded L_1 nodes go
//      to the slot and the request joins the leaf list.
// B. leaf kernel: one 8-wave workgroup per brick of the leaf list, 3 per CU
//    by default, bricks from a work counter: L_1, the leaf nibbles and the
//    palette staged in LDS (loaded into registers while the previous brick
//    was replayed); the leaf level as a dense 32^3 byte array, every voxel
//    first its L_1 node's index, the children of expanded nodes written over
//    it; same-level references listed, then each followed to its value; the
//    32^3 block written through the palette as dense rows of 16-byte stores.
//    Bricks whose arrays do not fit the LDS arena use the same code on an
//    arena in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/csv.h"
#include "csv_format.hpp"
#include "csv_generic.hpp"

namespace {

constexpr int kLog2 = 5;                 // 32^3 bricks
constexpr int kLutMaxBits = 12;          // largest supported table precision
constexpr uint32_t kMaxSym = 2 * 37448;  // every node an operation plus a delta nibble
constexpr uint32_t kLdsBytes = 160 * 1024;
constexpr uint32_t kLutLdsCap = 32 * 1024;  // decode tables kept in LDS when they fit (two 2^12 tables)
constexpr uint32_t kPalFast = 252;       // u8 indices 0..251; 252 marks an invalid reference, 253..255 open ones
constexpr uint32_t kRingWords = 1024;    // word ring of the entropy decoder
constexpr int kWavesLeaf = 8;            // waves of a leaf workgroup (LDS arena)
constexpr int kWavesLeafG = 4;           // waves of a leaf workgroup with a global-memory arena

// level m (1..4) offsets (entries) inside the Morton-ordered level arrays
__device__ constexpr uint32_t kLvOff[5] = {0, 0, 4096, 4608, 4672};
// expanded-node bit arrays (bytes, one per parent) for levels 1..4
__device__ constexpr uint32_t kBmOff[5] = {0, 0, 512, 576, 584};
// lists of expanded nodes (u16 entries) for levels 2..4; level 1 has its own
__device__ constexpr uint32_t kLstOff[5] = {0, 0, 72, 8, 0};

// LDS of one front-kernel wave: the word ring (2 KB plus a 128-byte mirror)
// and 512 symbol bytes during the entropy decode, then the upper levels
// (u8), their expansion bits and lists, the palette
constexpr uint32_t kWaveLds = 8192;
constexpr uint32_t kWLv = 0, kWBm = 4688, kWLst = 5280, kWPal = 6448;
constexpr uint32_t kWDeltaDw = (kWaveLds - kWPal) / 4;  // the palette area holds a level's nibbles during the replay

// Per-request slot in global memory: the packed nibbles (slot_dw dwords),
// then the levels (u16 levels 1..4 for big palettes; else u8 L_1 only, in
// Morton order), the expansion bits of levels 1..4 (L_1 first) and
// {E_1, P_a operations above L_0}.
constexpr uint32_t kSlotLv = 9376, kSlotBm = 608;
constexpr uint32_t kSlotExtra = kSlotLv + kSlotBm;

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
    const uint32_t *n_dev;  // device request count (the launch decodes min(n, *n_dev)), or nullptr
    int *err;  // [0] first error code, [1] brick id (or request index)
    // pools with level-0 detail in host memory (else nullptr): per brick the
    // word dwords held in the device record (0xFFFFFFFF: all of them) and the
    // device address of the staged remaining dwords (0: not staged)
    const uint32_t *pfx_dw;
    const uint64_t *sfx;
    // per-request status (else nullptr): a failed request rq gets its error
    // code in req_err[rq]; successful requests leave their entry untouched
    int *req_err;
    uint32_t rq_base;  // index of request 0 in the caller's whole batch (errors name requests by it)
};

// What the leaf kernel needs of a full-LOD request, written by the front
// kernel when it hands the request over (so that the leaf kernel reaches
// every address with one load)
struct LeafDesc {
    uint32_t rq, id, P, c0;
    uint32_t c1, E1, ipl, pad;
    uint64_t rec;  // record address
    uint64_t dst;  // output address
};
static_assert(sizeof(LeafDesc) == 48, "leaf descriptor");

struct LaunchA {
    uint32_t lut_lds_words;  // decode-table words in LDS (0: tables read from global memory)
    uint32_t *queue;         // work counter (nullptr: static round robin)
    const uint32_t *order;   // processing order of requests (nullptr: identity)
    uint8_t *slots;          // slot_bytes per request
    uint32_t slot_bytes;
    uint32_t slot_dw;        // nibble dwords at the start of a slot
    LeafDesc *leaf_list;     // requests left for the leaf kernel
    uint32_t *leaf_count;
    uint32_t base;           // first request index
    uint32_t *words_out;     // prefix pass (else nullptr): per request the words the decode of its
                             // level of detail consumed (0 for uniform bricks, 0xFFFFFFFF on error);
                             // nothing is written to the output
};

struct LaunchB {
    uint32_t arena_bytes;    // LDS arena per workgroup
    uint32_t *queue;         // work counter over the leaf list
    const LeafDesc *leaf_list;
    const uint32_t *leaf_count;
    LeafDesc *slow_list;     // leaf requests that do not fit the LDS arena
    uint32_t *slow_count;
    uint32_t *slow_queue;
    const uint8_t *slots;
    uint32_t slot_bytes;
    uint32_t slot_dw;
    uint8_t *scratch;        // global arena per workgroup for bricks that do not fit LDS
    uint32_t scratch_bytes;
    uint32_t ref_cap;        // longest list of same-level references (LDS room permitting)
    uint32_t *ctr;           // the launch's counters (see launch()); the last workgroup clears them
};

// ---------------------------------------------------------------------------
// wave primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// inclusive prefix sum over the 64 lanes (DPP row shifts, then row
// broadcasts); lanes shifted in from outside a row read 0, so that each
// step is one v_add_u32_dpp
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);  // row_shr:8
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
// request rq failed: the launch's error word (first error wins) and the request's status
__device__ __forceinline__ void fail(const DecodeArgs &a, uint32_t rq, int code, uint32_t who) {
    report(a.err, code, who);
    if (a.req_err) a.req_err[rq] = code;
}

// Per-brick phase clocks, only in builds with CSV_PHASE_TIMING: entry i of
// a request's 16 holds the shader clock at the end of phase i.
#ifdef CSV_PHASE_TIMING
__device__ uint64_t *g_phase = nullptr;
__device__ __forceinline__ void phase_mark(uint32_t rq, int i) {
    if (g_phase && __lane_id() == 0 && (i < 3 || i >= 9 || threadIdx.x == 0)) g_phase[16 * (size_t)rq + i] = __builtin_amdgcn_s_memtime();
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

__host__ __device__ constexpr uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }

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

// Uniform loads of data that no kernel of the launch writes, through the
// scalar cache: they count on lgkmcnt, so waiting for them does not wait for
// the wave's outstanding stores (on gfx9 vmcnt counts stores too).  p must be
// wave-uniform.  Sub-dword fields are read from their (4-byte aligned)
// dword, which lies in the same allocation.
template <class T>
__device__ __forceinline__ T ld_s(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}
__device__ __forceinline__ uint32_t ld_s_u8(const uint8_t *p) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    return (ld_s(reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3)) >> (8 * (a & 3))) & 0xFFu;
}
__device__ __forceinline__ uint32_t ld_s_u16(const uint16_t *p) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    return (ld_s(reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3)) >> (8 * (a & 2))) & 0xFFFFu;
}

// ---------------------------------------------------------------------------
// record header
// ---------------------------------------------------------------------------
struct Hdr {
    const uint32_t *rec;
    const uint32_t *sfx;  // staged word dwords from pdw on (detail in host memory), else nullptr
    uint32_t pdw;         // word dwords in the device record (0xFFFFFFFF: all)
    bool up;              // full LOD requested, level 1 decoded and written upsampled
    uint32_t P, W, nw, t, vol, rq, id;
    // cumulative symbol counts (scalars: a run-time level never indexes a private array)
    uint32_t c0, c1, c2, c3, c4;
    __device__ __forceinline__ uint32_t c(uint32_t m) const {
        return m == 0 ? c0 : (m == 1 ? c1 : (m == 2 ? c2 : (m == 3 ? c3 : c4)));
    }
};

// a hook that does nothing (the default of the kernels' optional hooks)
struct NoHook {
    __device__ void operator()() const {}
};

enum ReqKind { kReqBadLod, kReqBadId, kReqCorrupt, kReqFill, kReqDecode };

// read and check request rq; for kReqFill, fill is the value of every output label
__device__ __forceinline__ ReqKind load_request(const DecodeArgs &a, uint32_t rq, Hdr &h, uint32_t *&dst,
                                                uint32_t &count, uint32_t &fill) {
    h.rq = rq;
    h.sfx = nullptr;
    h.pdw = 0xFFFFFFFFu;
    h.up = false;
    h.id = ld_s(a.ids + rq);
    h.t = a.lods ? ld_s_u8(a.lods + rq) : a.lod_scalar;
    dst = nullptr;
    count = 0;
    fill = 0;
    if (h.t > (uint32_t)kLog2) return kReqBadLod;
    const uint32_t G = 32u >> h.t;
    count = G * G * G;
    dst = a.out + (a.out_off ? ld_s(a.out_off + rq) : (uint64_t)rq * count);
    if (h.id >= a.n_bricks) return kReqBadId;
    h.rec = rec_at(ld_s(a.rec_ptr + h.id));
    const uint32_t size = ld_s(a.rec_size + h.id);
    h.vol = ld_s_u16(a.rec_vol + h.id);
    h.P = ld_s(h.rec + 0);
    h.W = ld_s(h.rec + 1);
    h.nw = ld_s(h.rec + 2);
    h.c0 = ld_s(h.rec + 3);
    h.c1 = ld_s(h.rec + 4);
    h.c2 = ld_s(h.rec + 5);
    h.c3 = ld_s(h.rec + 6);
    h.c4 = ld_s(h.rec + 7);
    if (a.pfx_dw) {
        h.pdw = ld_s(a.pfx_dw + h.id);
        if (h.pdw != 0xFFFFFFFFu) {
            const uint64_t s = ld_s(a.sfx + h.id);
            h.sfx = s ? rec_at(s) : nullptr;
        }
    }
    const uint32_t hdr = csv::record_header_words(kLog2);
    // the record holds its words up to pdw dwords (the rest is staged)
    bool ok = h.P >= 1 && h.W <= 64 && (h.W & (h.W - 1)) == 0 && ((h.c0 > 0) == (h.W > 0)) && h.c0 <= kMaxSym &&
              4ull * ((uint64_t)hdr + h.P + h.W) + std::min<uint64_t>(2ull * h.nw, 4ull * h.pdw) <= size;
    ok = ok && h.c0 >= h.c1 && h.c1 >= h.c2 && h.c2 >= h.c3 && h.c3 >= h.c4;
    if (ok) ok = (h.c0 == 0) ? (h.P == 1) : (h.P >= 2);
    if (!ok) return kReqCorrupt;
    if (h.t == (uint32_t)kLog2 || h.c0 == 0) {  // coarsest level or uniform brick: palette[0]
        fill = ld_s(h.rec + hdr);
        return kReqFill;
    }
    if (h.t == 0 && h.pdw != 0xFFFFFFFFu && !h.sfx) {  // level 0 not on the device: level 1, upsampled
        h.t = 1;
        h.up = true;
    }
    return kReqDecode;
}

// ===========================================================================
// shared replay pieces
// ===========================================================================
// Children of one expanded parent from its 8 (op, stop) nibbles w: pv parent
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

// nibbles 0..3 of x -> bytes 0..3
__device__ __forceinline__ uint32_t nib_to_bytes(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    return (x | (x << 4)) & 0x0F0F0F0Fu;
}
// any byte of x equal to 0
__device__ __forceinline__ bool has_zero_byte(uint32_t x) { return ((x - 0x01010101u) & ~x & 0x80808080u) != 0; }
// byte selector of child k per operation code (v_perm_b32 codes over the
// candidates below): R_p -> the parent (4); R_a -> the parent level's +1
// neighbour (5 + a) if bit a of k is set, else the same-level mark (a);
// P_0, P_delta, P_a and the unused code 7 -> zero (12)
__host__ __device__ constexpr uint32_t child_selectors(int k) {
    return 4u | ((k & 1 ? 5u : 0u) << 4) | ((k & 2 ? 6u : 1u) << 8) | ((k & 4 ? 7u : 2u) << 12) | (12u << 16) |
           (12u << 20) | (12u << 24) | (12u << 28);
}
// the child replay builds these selectors as a table lookup by operation
// plus 5 where the child's bit on the operation's axis is set
constexpr bool selectors_match() {
    for (int k = 0; k < 8; k++)
        for (int o = 0; o < 8; o++) {
            const uint32_t base = o == 0 ? 4u : (o <= 3 ? (uint32_t)(o - 1) : 12u);
            const uint32_t plus = (o >= 1 && o <= 3 && ((k >> (o - 1)) & 1)) ? 5u : 0u;
            if (((child_selectors(k) >> (4 * o)) & 15u) != base + plus) return false;
        }
    return true;
}
static_assert(selectors_match(), "child selector tables");

// replay_children for u8 indices, all 8 children at once in two dwords:
// each child's copy or reference is one byte select (v_perm_b32) out of
// {marks, parent, neighbours}; the P operations add their palette position
// (ipb plus an exclusive byte-wise prefix count of the P_a children, +1 for
// P_a, -1 - delta for P_delta).  A reference that the parent's position
// does not allow selects 252, which no valid index reaches.
__device__ __forceinline__ uint2 replay_children_u8(uint32_t w, uint32_t pv, const uint32_t nb[3], uint32_t nbok,
                                                    uint32_t lowok, uint32_t ipb, const uint32_t *dnib, uint32_t db,
                                                    uint32_t P, bool leaf, bool &bad) {
    constexpr uint32_t kInv = 252u;
    const uint32_t cand_lo = ((lowok & 1u) ? 253u : kInv) | (((lowok & 2u) ? 254u : kInv) << 8) |
                             (((lowok & 4u) ? 255u : kInv) << 16) | (kInv << 24);
    const uint32_t cand_hi = pv | (((nbok & 1u) ? nb[0] : kInv) << 8) | (((nbok & 2u) ? nb[1] : kInv) << 16) |
                             (((nbok & 4u) ? nb[2] : kInv) << 24);
    // selector bytes child_selectors(k)[op_k], built for the even children
    // (0, 2, 4, 6) and the odd ones (1, 3, 5, 7) as byte vectors: a table
    // lookup by operation (R_p 4, R_x 0, R_y 1, R_z 2, P 12), plus 5 where
    // the child's k bit on the operation's axis is 1 (then its neighbour on
    // that axis is the parent-level one)
    const uint32_t ye = w & 0x07070707u, yo = (w >> 4) & 0x07070707u;
    const uint32_t be = __builtin_amdgcn_perm(0x0C0C0C0Cu, 0x02010004u, ye);
    const uint32_t bo = __builtin_amdgcn_perm(0x0C0C0C0Cu, 0x02010004u, yo);
    const uint32_t f2e = __builtin_amdgcn_perm(0u, 0x00050000u, ye), f3e = __builtin_amdgcn_perm(0u, 0x05000000u, ye);
    const uint32_t f1o = __builtin_amdgcn_perm(0u, 0x00000500u, yo), f2o = __builtin_amdgcn_perm(0u, 0x00050000u, yo),
                   f3o = __builtin_amdgcn_perm(0u, 0x05000000u, yo);
    const uint32_t se = be + ((f2e & 0xFF00FF00u) | (f3e & 0xFFFF0000u));          // ky at 2, 6; kz at 4, 6
    const uint32_t so = bo + (f1o | (f2o & 0xFF00FF00u) | (f3o & 0xFFFF0000u));    // kx at all; ky at 3, 7; kz at 5, 7
    const uint32_t sel_lo = __builtin_amdgcn_perm(so, se, 0x05010400u);            // children 0, 1, 2, 3
    const uint32_t sel_hi = __builtin_amdgcn_perm(so, se, 0x07030602u);            // children 4, 5, 6, 7
    uint32_t lo = __builtin_amdgcn_perm(cand_hi, cand_lo, sel_lo);
    uint32_t hi = __builtin_amdgcn_perm(cand_hi, cand_lo, sel_hi);
    const uint32_t y = w & 0x77777777u;
    const uint32_t pam = zero_nibbles(y ^ 0x66666666u);
    const uint32_t pa_lo = nib_to_bytes(pam), pa_hi = nib_to_bytes(pam >> 16);
    const uint32_t ip_lo = ipb * 0x01010101u + (pa_lo << 8) + (pa_lo << 16) + (pa_lo << 24);
    const uint32_t ip_hi = (ipb + (uint32_t)__builtin_popcount(pam & 0xFFFFu)) * 0x01010101u + (pa_hi << 8) +
                           (pa_hi << 16) + (pa_hi << 24);
    const uint32_t wp = (y >> 2) & 0x11111111u;  // bit 4k: operation code >= 4
    const uint32_t pb_lo = nib_to_bytes(wp), pb_hi = nib_to_bytes(wp >> 16);
    lo += (ip_lo & ((pb_lo << 8) - pb_lo)) + pa_lo;
    hi += (ip_hi & ((pb_hi << 8) - pb_hi)) + pa_hi;
    uint32_t pd = compact_nibble_bits(zero_nibbles(y ^ 0x55555555u));
    for (uint32_t j = 0; pd; j++) {
        const uint32_t k = (uint32_t)__builtin_ctz(pd);
        pd &= pd - 1;
        const uint32_t d = nib1(dnib, db + j), sh = 8 * (k & 3u);
        const uint32_t ipk = ((k < 4 ? ip_lo : ip_hi) >> sh) & 0xFFu;
        bad |= ipk < d + 1;
        if (k < 4) lo -= (d + 1) << sh;
        else hi -= (d + 1) << sh;
    }
    bad |= ipb + (uint32_t)__builtin_popcount(pam) >= P;  // the last P_a child's new entry
    bad |= zero_nibbles(y ^ 0x77777777u) != 0;
    bad |= leaf && (w & 0x88888888u) != 0;
    bad |= has_zero_byte(lo ^ 0xFCFCFCFCu) || has_zero_byte(hi ^ 0xFCFCFCFCu);
    return make_uint2(lo, hi);
}

// both index widths through one name
template <class IdxT>
__device__ __forceinline__ typename Vec8<IdxT>::T replay8(uint32_t w, uint32_t pv, const uint32_t nb[3],
                                                         uint32_t nbok, uint32_t lowok, uint32_t ipb, uint32_t pam8,
                                                         uint32_t pdm8, const uint32_t *dnib, uint32_t db, uint32_t P,
                                                         bool leaf, bool &bad) {
    if constexpr (sizeof(IdxT) == 1)
        return replay_children_u8(w, pv, nb, nbok, lowok, ipb, dnib, db, P, leaf, bad);
    else
        return replay_children<IdxT>(w, pv, nb, nbok, lowok, ipb, pam8, pdm8, dnib, db, P, leaf, bad);
}

// palette lookup; indices are checked while decoding, the clamp only keeps a
// malformed record from reading past a palette held in global memory
template <bool kG>
__device__ __forceinline__ uint32_t pal_at(const uint32_t *pal, uint32_t i, uint32_t P) {
    if constexpr (kG) return pal[i < P ? i : P - 1];
    return pal[i];
}

// four labels to dst: one non-temporal 16-byte store when dst is 16-byte
// aligned (kAl16, a compile-time choice so that the compiler keeps the wide
// store), else four dword stores (outputs of mixed levels of detail need
// not be aligned)
//
// Output stores go through global-address-space pointers, so that they are
// global (not flat) stores even where the output address was loaded from
// memory: a flat store also counts on lgkmcnt, and every LDS wait after it
// would wait for the store as well.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
__device__ __forceinline__ void store_nt(uint32_t *dst, const uint4 &o) {
    u32x4 v = {o.x, o.y, o.z, o.w};
    __builtin_nontemporal_store(v, (g_u32x4 *)dst);
}
template <bool kAl16>
__device__ __forceinline__ void store4(uint32_t *dst, const uint4 &o) {
    if constexpr (kAl16) {
        store_nt(dst, o);
    } else {
        g_u32 *g = (g_u32 *)dst;
        g[0] = o.x;
        g[1] = o.y;
        g[2] = o.z;
        g[3] = o.w;
    }
}

// count labels of value v, by kThreads threads (tid: this thread's index)
template <uint32_t kThreads>
__device__ __forceinline__ void fill_labels(uint32_t *dst, uint32_t count, uint32_t v, uint32_t tid) {
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0 && (count & 3) == 0) {
        const uint4 q = make_uint4(v, v, v, v);
        for (uint32_t e = 4 * tid; e < count; e += 4 * kThreads) store_nt(dst + e, q);
    } else {
        for (uint32_t e = tid; e < count; e += kThreads) ((g_u32 *)dst)[e] = v;
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

// ordering between the lanes of one wave: LDS (wsync) or also global memory
template <bool kG>
__device__ __forceinline__ void wave_sync() {
    if (kG) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        wsync();
    }
}

// ===========================================================================
// A. front kernel
// ===========================================================================
// Entropy decode of the first n symbols of a brick (the prefix for its
// level of detail) into packed nibbles at out (global); ring32: this wave's
// 2 KB of LDS.  False on a malformed stream.
// at_upper (with the paired front kernel) is called once, in wave-uniform
// control flow, as soon as the nibble dwords of the first c_1 symbols (the
// levels above L_0) are written, else at the end
template <bool kLutLds, class Hook = NoHook>
__device__ __forceinline__ bool entropy_decode(const DecodeArgs &a, const Hdr &h, const uint32_t *slut,
                                               uint32_t *ring32, uint32_t *out, uint32_t *lcopy, uint32_t n,
                                               uint32_t &words, Hook at_upper = Hook{}) {
    constexpr bool kHook = !std::is_same<Hook, NoHook>::value;
    const uint32_t upper = (h.c1 + 7u) & ~7u;  // whole nibble dwords
    bool fired = false;
    auto upper_done = [&](uint32_t decoded) {
        if constexpr (kHook) {
            if (!fired && decoded >= upper) {
                fired = true;
                at_upper();
            }
        }
    };
    const uint32_t L = lane();
    const uint32_t hdr = csv::record_header_words(kLog2);
    const uint16_t *ring = reinterpret_cast<const uint16_t *>(ring32);
    const uint32_t sbits = ld_s(a.vol_bits + h.vol), lutn = 1u << sbits, mask = lutn - 1u;
    const uint32_t *lut = (kLutLds ? slut : glob(a.luts)) + ld_s(a.lut_off + h.vol);
    const uint32_t W = h.W, lw = 31u - (uint32_t)__builtin_clz(W), leaf = h.c1;
    const uint32_t *wg = h.rec + hdr + h.P + W;
    const uint32_t ndw = (h.nw + 1) / 2;  // word dwords in the record (the last one padded)
    // dword d of the word stream: from the record below pdw, then from the
    // staged detail (0 past what is there: never consumed)
    const uint32_t pdw = min(h.pdw, ndw);
    const uint32_t *sfx = h.sfx;
    auto wdw = [&](uint32_t d) -> uint32_t { return d < pdw ? wg[d] : ((sfx && d < ndw) ? sfx[d - pdw] : 0u); };
    uint32_t x = L < W ? h.rec[hdr + h.P + L] : 0u;
    // the ring holds words [ring_lo, ring_lo + 1024) at positions word & 1023,
    // and positions 0..63 again after position 1023 (a read of 64 words from
    // any position needs no wrap-around); pf holds the next 512 words
    uint32_t ring_lo = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const uint32_t d = L + 64 * q;
        const uint32_t v = wdw(d);
        ring32[d] = v;
        if (q == 0 && L < 32) ring32[kRingWords / 2 + L] = v;
    }
    uint32_t pf[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t d = 512 + L + 64 * q;
        pf[q] = wdw(d);
    }
    wsync();
    uint32_t cursor = 0, acc = 0;
    bool bad = false;
    // the oldest half of the ring is consumed: refill it from pf, fetch the next
    auto refill = [&]() {
        const uint32_t hh = (ring_lo >> 9) & 1u;
        wsync();
#pragma unroll
        for (int q = 0; q < 4; q++) ring32[hh * 256 + L + 64 * q] = pf[q];
        if (hh == 0 && L < 32) ring32[kRingWords / 2 + L] = pf[0];
        ring_lo += 512;
        const uint32_t d0 = (ring_lo + 1024) >> 1;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t d = d0 + L + 64 * q;
            pf[q] = wdw(d);
        }
        wsync();
    };
    const uint32_t steps = (n + W - 1) >> lw;
    uint32_t s = 0;
    if (W == 64) {
        // steps with all 64 lanes busy: no per-lane conditions; every lane
        // reads a ring word and keeps it if it renormalises.  Steps wholly
        // before the leaf segment use the interior table without a select.
        auto step = [&](auto leaf_select) {
            const uint32_t i = (s << 6) + L;
            const uint32_t tb = decltype(leaf_select)::value ? (i >= leaf ? lutn : 0u) : 0u;
            const uint32_t e = lut[tb + (x & mask)];
            const uint32_t sym = e & 15u;
            x = __umul24(e >> 20, x >> sbits) + ((e >> 8) & 0xFFFu);
            const bool need = x < csv::kRansLower;
            const uint64_t bal = __ballot(need);
            const uint32_t wd = ring[(cursor + mbcnt(bal)) & (kRingWords - 1)];
            x = need ? ((x << 16) | wd) : x;
            cursor += (uint32_t)__popcll(bal);
            const uint32_t g = row_or<3>(sym << (4 * (L & 7u)));
            if ((L & 7u) == 7u) {
                out[(i - 7) >> 3] = g;
                if (((i - 7) >> 3) < kWDeltaDw) lcopy[(i - 7) >> 3] = g;
            }
            if (cursor >= ring_lo + 512) refill();
        };
        // blocks of 8 steps: each lane writes its symbol as a byte to LDS
        // (no address arithmetic: immediate offsets), then lane L packs the
        // block's symbols 8L .. 8L + 7 into one nibble dword
        uint8_t *sb = reinterpret_cast<uint8_t *>(ring32) + 2 * kRingWords + 128;
        auto block8 = [&](auto leaf_select) {
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint32_t i = ((s + (uint32_t)j) << 6) + L;
                const uint32_t tb = decltype(leaf_select)::value ? (i >= leaf ? lutn : 0u) : 0u;
                const uint32_t e = lut[tb + (x & mask)];
                x = __umul24(e >> 20, x >> sbits) + ((e >> 8) & 0xFFFu);
                const bool need = x < csv::kRansLower;
                const uint64_t bal = __ballot(need);
                // the wave's ring position is uniform: one scalar base plus each lane's rank
                uint32_t wd = (ring + (cursor & (kRingWords - 1)))[mbcnt(bal)];
                // every lane reads (the read is not worth a branch on the critical path)
                __asm__ volatile("" : "+v"(wd));
                x = need ? ((x << 16) | wd) : x;
                cursor += (uint32_t)__popcll(bal);
                sb[64 * j + L] = (uint8_t)e;  // the symbol (bits 4..7 of an entry are zero)
                if (cursor >= ring_lo + 512) refill();
            }
            wsync();
            const uint2 b = *reinterpret_cast<const uint2 *>(sb + 8 * L);
            const uint32_t lo = (b.x | (b.x >> 4)) & 0x00FF00FFu, hi = (b.y | (b.y >> 4)) & 0x00FF00FFu;
            const uint32_t packed = ((lo | (lo >> 8)) & 0xFFFFu) | (((hi | (hi >> 8)) & 0xFFFFu) << 16);
            out[(s << 3) + L] = packed;
            if ((s << 3) + L < kWDeltaDw) lcopy[(s << 3) + L] = packed;
            wsync();
            s += 8;
            upper_done(s << 6);
        };
        const uint32_t full = n >> 6, s_int = min(leaf >> 6, full);
        while (s + 8 <= s_int) block8(std::false_type{});
        while (s + 8 <= full) block8(std::true_type{});
        for (; s < full;) {
            step(std::true_type{});
            s++;
            upper_done(s << 6);
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
            x = __umul24(e >> 20, x >> sbits) + ((e >> 8) & 0xFFFu);
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
            if ((L & 7) == 7 && L < W && i - 7 < n) {
                out[(i - 7) >> 3] = g;
                if (((i - 7) >> 3) < kWDeltaDw) lcopy[(i - 7) >> 3] = g;
            }
        } else {
            const uint32_t g = W == 4 ? row_or<2>(v) : (W == 2 ? row_or<1>(v) : v);
            acc |= g;
            const bool full = (((s + 1) << lw) & 7) == 0;
            if (L == W - 1 && (full || s + 1 == steps)) {
                out[(s << lw) >> 3] = acc;
                if (((s << lw) >> 3) < kWDeltaDw) lcopy[(s << lw) >> 3] = acc;
            }
            if (full) acc = 0;
        }
        if (cursor >= ring_lo + 512) refill();
        upper_done((s + 1) << lw);
    }
    if constexpr (kHook) {
        if (!fired) at_upper();
    }
    // a complete decode ends in the encoder's initial states with every word read
    if (!bad && h.t == 0) bad = (__ballot(L < W && x != csv::kRansLower) != 0) || cursor != h.nw;
    words = cursor;
    return !bad;
}

// Replay of levels 4 .. max(t, 1) by one wave (Alg. 1).  lv: the level
// arrays (LDS, or the slot when kG); bm, lst: expansion bits and lists of
// levels 2..4 in LDS; nib: the brick's nibbles (global).  On return E and
// ipl hold the number of expanded L_1 nodes and the P_a operations so far.
// False on a malformed stream.
template <class IdxT, bool kG>
__device__ __forceinline__ bool upper_replay(const Hdr &h, const uint32_t *nib, IdxT *lv, uint8_t *bm, uint16_t *lst,
                                             uint32_t *dstage, uint32_t &E_out, uint32_t &ipl_out) {
    using V = Vec8<IdxT>;
    using VT = typename V::T;
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    const uint32_t L = lane(), t = h.t, P = h.P;
    const uint32_t tl = t > 1 ? t : 1u;  // finest level replayed here
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
        const bool want_list = m >= 2;  // L_1's list is rebuilt from its bits by the leaf kernel
        uint16_t *clist = lst + kLstOff[m];
        const uint32_t list_cap = 1u << (3 * (kLog2 - m));
        // children of parents that are not expanded inherit the parent's index
        if (sizeof(IdxT) == 1 && !kG && up) {
            // u8 levels in LDS: a lane takes 8 parents and writes the children
            // of all of them (the expanded ones are overwritten below)
            for (uint32_t g = L; g < np / 8; g += 64) {
                const uint2 u = *reinterpret_cast<const uint2 *>(up + 8 * g);
                *reinterpret_cast<uint2 *>(cbm + 8 * g) = make_uint2(0u, 0u);
                uint4 *o = reinterpret_cast<uint4 *>(cur + 64 * g);
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const uint32_t a = __builtin_amdgcn_perm(u.y, u.x, 0x01010101u * (uint32_t)j);
                    const uint32_t b = __builtin_amdgcn_perm(u.y, u.x, 0x01010101u * (uint32_t)(j + 1));
                    o[j / 2] = make_uint4(a, a, b, b);
                }
            }
        } else {
            for (uint32_t q = L; q < np; q += 64) {
                const bool ex = pbm ? ((pbm[q >> 3] >> (q & 7)) & 1u) : true;
                cbm[q] = 0;
                if (!ex) *reinterpret_cast<VT *>(cur + 8 * q) = V::splat(up ? (uint32_t)up[q] : 0u);
            }
        }
        wave_sync<kG>();
        const uint32_t seg = (m == kLog2 - 1) ? 0u : h.c((uint32_t)m + 1), seg_end = h.c((uint32_t)m);
        if ((uint64_t)seg + 8ull * E > seg_end) return false;
        const uint32_t D = seg_end - seg - 8 * E, ops0 = seg + D;  // deltas precede the operations
        const uint32_t pmask0 = axis_mask(0, Bp), pmask1 = axis_mask(1, Bp), pmask2 = axis_mask(2, Bp);
        // the level's nibbles (deltas, then operations) from LDS: the copy of
        // the stream's first kWDeltaDw dwords that the entropy decoder wrote,
        // else the level's segment staged (one round trip to global memory
        // per level instead of one per 64 nodes), else global memory.  src
        // holds the nibbles from position off on.
        uint32_t bpa = 0, bpd = 0, bex = 0;
        bool bad = false;
        auto run = [&](const uint32_t *src, uint32_t off) __attribute__((always_inline)) {
            for (uint32_t c = 0; c < (E + 63) / 64; c++) {
                const uint32_t r = 64 * c + L;
                const bool act = r < E;
                const uint32_t q = (act && plist) ? (uint32_t)plist[r] : 0u;
                const uint32_t wd = act ? nib8(src, ops0 - off + 8 * r) : 0u;
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
                    const VT vals = replay8<IdxT>(wd, pv, nb, nbok, lowok, ipl + bpa + (exc & 1023u),
                                                          compact_nibble_bits(pam), compact_nibble_bits(pdm), src,
                                                          seg - off + bpd + ((exc >> 10) & 1023u), P, false, bad);
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
        };
        const uint32_t s0 = seg >> 3, sn = ((seg_end + 7) >> 3) - s0 + 1;
        if (m == 1) phase_mark(h.rq, 13);
        if (((seg_end + 7) >> 3) < kWDeltaDw) {
            // every nibble up to this level's end is in the entropy decoder's copy
            run(dstage, 0);
        } else if (sn <= kWDeltaDw) {
            for (uint32_t e = L; e < sn; e += 64) dstage[e] = nib[s0 + e];
            wsync();
            run(dstage, 8 * s0);
        } else {
            run(nib, 0);
        }
        if (__ballot(bad) || bpd != D || (want_list && bex > list_cap)) return false;
        wave_sync<kG>();
        if (m == 1) phase_mark(h.rq, 14);
        // neighbour references into this level: a reference to child k of
        // the -1 neighbour along a lands on child k | 1 << a, so a chain has
        // at most three links (child 7 holds none); it is followed to its end
        // while other lanes resolve in place (a reader sees the reference or
        // its final value, and both lead to the same value).  The chains of
        // a node's children are followed together, one link each per round.
        // At level 1 (u8, in LDS) the staging area is free by now: the
        // children that hold references are listed there first, and each
        // is then followed by a lane of its own.
        bool listed = false;
        if constexpr (sizeof(IdxT) == 1 && !kG) {
            if (m == 1) {
                uint16_t *refs = reinterpret_cast<uint16_t *>(dstage);
                constexpr uint32_t kCap = 2 * kWDeltaDw;
                uint32_t nref = 0;
                for (uint32_t c = 0; c < (E + 63) / 64; c++) {
                    const uint32_t r = 64 * c + L;
                    const bool act = r < E;
                    const uint32_t q = (act && plist) ? (uint32_t)plist[r] : 0u;
                    const uint2 vv = act ? *reinterpret_cast<const uint2 *>(cur + 8 * q) : make_uint2(0u, 0u);
                    // bytes >= 253 (252 has been rejected): bit 7 of each such byte
                    const uint32_t tl = ~vv.x & 0xFCFCFCFCu, th = ~vv.y & 0xFCFCFCFCu;
                    uint32_t fl = (tl - 0x01010101u) & ~tl & 0x80808080u;
                    uint32_t fh = (th - 0x01010101u) & ~th & 0x80808080u;
                    const uint32_t cnt = (uint32_t)__builtin_popcount(fl) + (uint32_t)__builtin_popcount(fh);
                    const uint32_t inc = wave_incl_scan(cnt);
                    const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
                    if (nref + tot <= kCap) {
                        uint32_t pos = nref + inc - cnt;
                        while (fl) {
                            refs[pos++] = (uint16_t)(8 * q + ((uint32_t)__builtin_ctz(fl) >> 3));
                            fl &= fl - 1u;
                        }
                        while (fh) {
                            refs[pos++] = (uint16_t)(8 * q + 4 + ((uint32_t)__builtin_ctz(fh) >> 3));
                            fh &= fh - 1u;
                        }
                    }
                    nref += tot;
                }
                if (nref <= kCap) {
                    wsync();
                    for (uint32_t e = L; e < nref; e += 64) {
                        const uint32_t off = refs[e];
                        uint32_t qq = off >> 3, kk = off & 7u, v = cur[off];
                        while (v >= kMark) {
                            const uint32_t a = v - kMark;
                            qq = morton_dec(qq, pmask0 << a);
                            kk |= 1u << a;
                            v = cur[8 * qq + kk];
                        }
                        cur[off] = (IdxT)v;
                    }
                    listed = true;
                }
            }
        }
        for (uint32_t r = L; !listed && r < E; r += 64) {
            const uint32_t q = plist ? (uint32_t)plist[r] : 0u;
            VT vals = *reinterpret_cast<const VT *>(cur + 8 * q);
            uint32_t v[7], qq[7], kk[7];
            bool more = false;
#pragma unroll
            for (int k = 0; k < 7; k++) {
                v[k] = V::get(vals, k);
                qq[k] = q;
                kk[k] = (uint32_t)k;
                more |= v[k] >= kMark;
            }
            if (more) {
                while (more) {
#pragma unroll
                    for (int k = 0; k < 7; k++) {
                        if (v[k] >= kMark) {
                            const uint32_t a = v[k] - kMark;
                            qq[k] = morton_dec(qq[k], pmask0 << a);  // the axis masks are shifts of each other
                            kk[k] |= 1u << a;
                            v[k] = cur[8 * qq[k] + kk[k]];
                        }
                    }
                    more = false;
#pragma unroll
                    for (int k = 0; k < 7; k++) more |= v[k] >= kMark;
                }
#pragma unroll
                for (int k = 0; k < 7; k++) V::set(vals, k, v[k]);
                *reinterpret_cast<VT *>(cur + 8 * q) = vals;
            }
        }
        wave_sync<kG>();
        phase_mark(h.rq, 13 - m);
        ipl += bpa;
        E = bex;
    }
    E_out = E;
    ipl_out = ipl;
    return true;
}

// the level-t block (t >= 1) through the palette to dst, by one wave
template <class IdxT, bool kG>
__device__ __forceinline__ void upper_output(const IdxT *lv, uint32_t t, const uint32_t *pal, uint32_t P,
                                             uint32_t *dst) {
    const uint32_t L = lane(), G = 32u >> t;
    const IdxT *res = lv + kLvOff[t];
    if (t == 4) {
        if (L < 8) dst[L] = pal_at<kG>(pal, res[L], P);  // Morton order equals dense order on 2^3
        return;
    }
    const uint32_t lg = (uint32_t)(kLog2 - t);
    auto rows = [&](auto al16) {
        for (uint32_t e = 4 * L; e < G * G * G; e += 256) {
            const uint32_t x0 = e & (G - 1), yy = (e >> lg) & (G - 1), zz = e >> (2 * lg);
            const uint32_t m0 = spread4(x0) | (spread4(yy) << 1) | (spread4(zz) << 2);
            uint4 o;
            o.x = pal_at<kG>(pal, res[m0], P);
            o.y = pal_at<kG>(pal, res[m0 | 1u], P);
            o.z = pal_at<kG>(pal, res[m0 | 8u], P);
            o.w = pal_at<kG>(pal, res[m0 | 9u], P);
            store4<decltype(al16)::value>(dst + e, o);
        }
    };
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) rows(std::true_type{});
    else rows(std::false_type{});
}

// level 1 written as a 32^3 block, every voxel the value of its level-1
// node (full LOD requested, level-0 detail not on the device), by one wave
template <class IdxT, bool kG>
__device__ __forceinline__ void upper_output_up2(const IdxT *lv, const uint32_t *pal, uint32_t P, uint32_t *dst) {
    const uint32_t L = lane();
    const IdxT *res = lv + kLvOff[1];
    auto rows = [&](auto al16) {
        for (uint32_t e = 4 * L; e < 32768u; e += 256) {
            const uint32_t x0 = e & 31u, yy = (e >> 5) & 31u, zz = e >> 10;
            // x0 / 2 is even: its +1 neighbour in x differs in Morton bit 0
            const uint32_t m0 = spread4(x0 >> 1) | (spread4(yy >> 1) << 1) | (spread4(zz >> 1) << 2);
            const uint32_t a = pal_at<kG>(pal, res[m0], P), b = pal_at<kG>(pal, res[m0 | 1u], P);
            store4<decltype(al16)::value>(dst + e, make_uint4(a, a, b, b));
        }
    };
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) rows(std::true_type{});
    else rows(std::false_type{});
}

// one brick of the front kernel after its entropy decode; false on a
// malformed stream
// With e1_ipl (the paired front kernel) a t = 0 request is not yet handed to
// the leaf kernel: E_1 and ipl go to e1_ipl[0..1] for hand_off.
__device__ __forceinline__ void hand_off(const Hdr &h, const LaunchA &l, uint32_t E1, uint32_t ipl, uint32_t *dst) {
    if (lane() == 0) {
        const uint32_t at = atomicAdd(l.leaf_count, 1u);
        uint4 *d = reinterpret_cast<uint4 *>(l.leaf_list + at);
        const uint64_t ra = reinterpret_cast<uintptr_t>(h.rec), da = reinterpret_cast<uintptr_t>(dst);
        d[0] = make_uint4(h.rq, h.id, h.P, h.c0);
        d[1] = make_uint4(h.c1, E1, ipl, 0u);
        d[2] = make_uint4((uint32_t)ra, (uint32_t)(ra >> 32), (uint32_t)da, (uint32_t)(da >> 32));
    }
}

template <class IdxT, bool kG>
__device__ __forceinline__ bool front_replay(const Hdr &h, const LaunchA &l, const uint32_t *nib, uint8_t *slot,
                                             uint8_t *wl, uint32_t *dst, uint32_t *e1_ipl = nullptr) {
    const uint32_t L = lane();
    const uint32_t hdr = csv::record_header_words(kLog2);
    uint8_t *slv = slot + 4 * l.slot_dw;
    uint8_t *sbm = slv + kSlotLv;
    IdxT *lv = kG ? reinterpret_cast<IdxT *>(slv) : reinterpret_cast<IdxT *>(wl + kWLv);
    uint8_t *bm = wl + kWBm;
    uint16_t *lst = reinterpret_cast<uint16_t *>(wl + kWLst);
    uint32_t E1 = 0, ipl = 0;
    if (!upper_replay<IdxT, kG>(h, nib, lv, bm, lst, reinterpret_cast<uint32_t *>(wl + kWPal), E1, ipl)) return false;
    if (h.t >= 1) {
        const uint32_t *pal = h.rec + hdr;
        if (!kG) {  // stage the palette next to the levels
            uint32_t *sp = reinterpret_cast<uint32_t *>(wl + kWPal);
            for (uint32_t e = L; e < h.P; e += 64) sp[e] = pal[e];
            wsync();
            pal = sp;
        }
        if (h.up) upper_output_up2<IdxT, kG>(lv, pal, h.P, dst);
        else upper_output<IdxT, kG>(lv, h.t, pal, h.P, dst);
        return true;
    }
    // t = 0: hand L_1 to the leaf kernel
    if (!kG) {
        const uint4 *src = reinterpret_cast<const uint4 *>(lv);
#pragma unroll
        for (int q = 0; q < 4; q++) reinterpret_cast<uint4 *>(slv)[L + 64 * q] = src[L + 64 * q];
    }
    if (L < 32) reinterpret_cast<uint4 *>(sbm)[L] = reinterpret_cast<const uint4 *>(bm)[L];
    if (e1_ipl) {
        e1_ipl[0] = E1;
        e1_ipl[1] = ipl;
    } else {
        hand_off(h, l, E1, ipl, dst);
    }
    return true;
}

// kLutLds: the decode tables of every volume are copied to LDS (else read
// from global memory)
template <int WPG, bool kLutLds>
// 16 waves per CU at most (LDS); registers for 4 per SIMD
__global__ __launch_bounds__(WPG * 64) __attribute__((amdgpu_waves_per_eu(4))) void front_kernel(DecodeArgs a, LaunchA l) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *slut = reinterpret_cast<uint32_t *>(smem);
    if (kLutLds)
        for (uint32_t e = threadIdx.x; e < l.lut_lds_words; e += blockDim.x) slut[e] = a.luts[e];
    __syncthreads();
    const uint32_t L = lane(), wave = uniform(threadIdx.x >> 6);
    uint8_t *wl = smem + align16(4 * l.lut_lds_words) + wave * kWaveLds;
    const uint32_t wid = blockIdx.x * WPG + wave;
    const uint32_t n_req = a.n_dev ? min(a.n, ld_s(a.n_dev)) : a.n;
    // With a work counter, each request is taken one brick ahead (lane 0)
    // and its value read at the end of the brick before: a read at the top
    // of a brick would wait behind the previous brick's stores (on gfx9 one
    // counter tracks loads and stores, served in order), and then the
    // brick's own loads would wait again.  An increment, not an add: the
    // compiler rewrites a uniform-address add to read its result at once.
    uint32_t taken = 0, cur = 0;
    if (l.queue) {
        if (L == 0) taken = atomicInc(l.queue, 0xFFFFFFFFu);
        cur = uniform(taken);
        if (L == 0) taken = atomicInc(l.queue, 0xFFFFFFFFu);
    }
    for (uint32_t k = 0;; k++) {
        if (k > 0 && l.queue) {
            cur = uniform(taken);
            if (L == 0) taken = atomicInc(l.queue, 0xFFFFFFFFu);
        }
        const uint32_t req = l.base + (l.queue ? cur : wid + k * gridDim.x * WPG);
        if (req >= n_req) break;
        const uint32_t rq = l.order ? ld_s(l.order + req) : req;
        phase_mark(rq, 0);
        Hdr h;
        uint32_t *dst, count, fill;
        const ReqKind kind = load_request(a, rq, h, dst, count, fill);
        if (l.words_out && kind != kReqDecode) {
            if (L == 0) l.words_out[rq] = kind == kReqFill ? 0u : 0xFFFFFFFFu;
            continue;
        }
        if (kind == kReqBadLod) {
            if (L == 0) fail(a, rq, CSV_ERANGE, a.rq_base + rq);
            continue;
        }
        if (kind != kReqDecode) {
            if (kind != kReqFill && L == 0) fail(a, rq, kind == kReqBadId ? CSV_ERANGE : CSV_ECORRUPT,
                                                 kind == kReqBadId ? a.rq_base + rq : h.id);
            fill_labels<64>(dst, count, kind == kReqFill ? fill : 0u, L);
            continue;
        }
        if (h.up && L == 0) fail(a, rq, CSV_EDETAIL, h.id);
        const uint32_t n = h.c(h.t);
        uint8_t *slot = glob(l.slots) + (size_t)rq * l.slot_bytes;
        uint32_t *nib = reinterpret_cast<uint32_t *>(slot);
        if (n + 16 > 8 * l.slot_dw) {  // the slots are sized for the pool's largest brick
            if (L == 0) fail(a, rq, CSV_EINVAL, h.id);
            if (l.words_out) {
                if (L == 0) l.words_out[rq] = 0xFFFFFFFFu;
            } else {
                fill_labels<64>(dst, count, 0u, L);
            }
            continue;
        }
        // the packed nibbles go to the slot, and their first kWDeltaDw dwords
        // also to the wave's staging area (the upper levels read them there)
        uint32_t words = 0;
        bool ok = entropy_decode<kLutLds>(a, h, slut, reinterpret_cast<uint32_t *>(wl),
                                          nib, reinterpret_cast<uint32_t *>(wl + kWPal), n, words);
        if (l.words_out) {
            if (L == 0) l.words_out[rq] = ok ? words : 0xFFFFFFFFu;
            wsync();
            continue;
        }
        phase_mark(rq, 1);
        // this wave's nibble stores before its own loads of them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        wsync();  // the ring is reused for the levels
        if (ok) ok = h.P <= kPalFast ? front_replay<uint8_t, false>(h, l, nib, slot, wl, dst)
                                     : front_replay<uint16_t, true>(h, l, nib, slot, wl, dst);
        if (!ok) {
            if (L == 0) fail(a, rq, CSV_ECORRUPT, h.id);
            fill_labels<64>(dst, count, 0u, L);
        }
        phase_mark(rq, 2);
    }
}

// LDS of the paired kernel's decoding wave: the word ring with its mirrored
// start and the symbol bytes of a block of 8 steps (entropy_decode), then
// two verdict words
constexpr uint32_t kPairOk = 2 * kRingWords + 128 + 512;
constexpr uint32_t kPairDecLds = align16(kPairOk + 8);

// Paired front kernel for small batches (shape waves_per_group 2), where a
// decode lasts as long as its slowest brick's serial chain: a workgroup of
// two waves per brick.  Wave 0 decodes the brick's symbols; as soon as the
// symbols of the levels above L_0 are out (entropy_decode's hook, a
// workgroup barrier), wave 1 replays those levels while wave 0 decodes the
// L_0 symbols.  A second barrier ends the brick: wave 1 then hands a
// full-LOD request to the leaf kernel, or reports a malformed stream.  The
// chain becomes the upper symbols' decode plus the longer of the L_0
// decode and the replay.  Both waves take every brick of the workgroup
// (static round robin) and pass the same barriers on every path.
template <bool kLutLds>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(4))) void front_pair_kernel(DecodeArgs a,
                                                                                                LaunchA l) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *slut = reinterpret_cast<uint32_t *>(smem);
    if (kLutLds)
        for (uint32_t e = threadIdx.x; e < l.lut_lds_words; e += blockDim.x) slut[e] = a.luts[e];
    __syncthreads();
    const uint32_t L = lane(), wave = uniform(threadIdx.x >> 6);
    uint8_t *wl0 = smem + align16(4 * l.lut_lds_words);  // wave 0: the word ring
    uint8_t *wl1 = wl0 + kPairDecLds;                      // wave 1: the levels (first nibbles at kWPal)
    uint32_t *ok_word = reinterpret_cast<uint32_t *>(wl0 + kPairOk);  // wave 0's verdict, by brick parity
    const uint32_t n_req = a.n_dev ? min(a.n, ld_s(a.n_dev)) : a.n;
    for (uint32_t k = 0;; k++) {
        const uint32_t req = l.base + blockIdx.x + k * gridDim.x;
        if (req >= n_req) break;
        const uint32_t rq = l.order ? ld_s(l.order + req) : req;
        Hdr h;
        uint32_t *dst, count, fill;
        const ReqKind kind = load_request(a, rq, h, dst, count, fill);
        if (kind != kReqDecode) {
            if (wave == 0) {
                if (kind == kReqBadLod) {
                    if (L == 0) fail(a, rq, CSV_ERANGE, a.rq_base + rq);
                } else {
                    if (kind != kReqFill && L == 0)
                        fail(a, rq, kind == kReqBadId ? CSV_ERANGE : CSV_ECORRUPT,
                             kind == kReqBadId ? a.rq_base + rq : h.id);
                    fill_labels<64>(dst, count, kind == kReqFill ? fill : 0u, L);
                }
            }
            continue;
        }
        if (h.up && L == 0 && wave == 0) fail(a, rq, CSV_EDETAIL, h.id);
        const uint32_t n = h.c(h.t);
        uint8_t *slot = glob(l.slots) + (size_t)rq * l.slot_bytes;
        uint32_t *nib = reinterpret_cast<uint32_t *>(slot);
        if (n + 16 > 8 * l.slot_dw) {  // the slots are sized for the pool's largest brick
            if (wave == 0) {
                if (L == 0) fail(a, rq, CSV_EINVAL, h.id);
                fill_labels<64>(dst, count, 0u, L);
            }
            continue;
        }
        if (wave == 0) {
            uint32_t words = 0;
            const bool ok = entropy_decode<kLutLds>(a, h, slut, reinterpret_cast<uint32_t *>(wl0), nib,
                                                    reinterpret_cast<uint32_t *>(wl1 + kWPal), n, words,
                                                    [] { __syncthreads(); });
            if (L == 0) ok_word[k & 1u] = ok ? 1u : 0u;
            __syncthreads();
        } else {
            __syncthreads();  // the symbols above L_0 are out
            uint32_t e1_ipl[2] = {0u, 0u};
            bool ok = h.P <= kPalFast ? front_replay<uint8_t, false>(h, l, nib, slot, wl1, dst, e1_ipl)
                                      : front_replay<uint16_t, true>(h, l, nib, slot, wl1, dst, e1_ipl);
            __syncthreads();  // wave 0 is done with the brick
            ok = ok && ok_word[k & 1u] != 0u;
            if (ok && h.t == 0) hand_off(h, l, e1_ipl[0], e1_ipl[1], dst);
            if (!ok) {
                if (L == 0) fail(a, rq, CSV_ECORRUPT, h.id);
                fill_labels<64>(dst, count, 0u, L);
            }
        }
    }
}

// ===========================================================================
// B. leaf kernel
// ===========================================================================
struct SmallB {
    uint32_t req;
    int err;
    uint32_t nref;  // same-level references in the leaf level (list length)
    uint32_t wt[kWavesLeaf][2];  // per-wave totals of P_a, P_delta
    uint32_t desc[2][16];        // leaf descriptors (dwords 0..11) and work items (dword 12) of the
                                 // current and the next brick
    uint32_t item2;              // the work item after those
};

// Arena of a leaf brick: palette (P entries) and nib4 16-byte groups of
// nibbles (staged only in LDS), L_1 as a dense 16^3 array, its expansion
// bits (Morton order) and their rank prefix, the expanded L_1 nodes (Morton
// indices, stream order; list_cap entries) and the dense 32^3 leaf level
struct LayoutL {
    uint32_t pal, nib, l1, bm1, bpre, list1, leaf, total;
};
__host__ __device__ constexpr LayoutL make_layout_l(bool stage, uint32_t P, uint32_t nib4, uint32_t list_cap,
                                                    uint32_t idx) {
    LayoutL L{};
    uint32_t o = 0;
    L.pal = o; o += stage ? align16(4 * P) : 0;
    L.nib = o; o += stage ? 16 * nib4 : 0;
    L.l1 = o; o += 4096 * idx;
    L.bm1 = o; o += 512;
    L.bpre = o; o += 128;
    L.list1 = o; o += align16(2 * list_cap);
    L.leaf = o; o += 32768 * idx;
    L.total = o;
    return L;
}

// global arena of a leaf brick that does not fit LDS
constexpr uint32_t kArenaBytes = make_layout_l(false, 0, 0, 4096, 2).total;

// coordinates of a 12-bit Morton index (x in bits 0, 3, 6, 9)
__device__ __forceinline__ uint32_t morton_coord(uint32_t p) {
    return (p & 1u) | ((p >> 2) & 2u) | ((p >> 4) & 4u) | ((p >> 6) & 8u);
}

// children of one expanded node that the child replay leaves as same-level
// references (bit 4k for child k): R_x at kx = 0, R_y at ky = 0, R_z at
// kz = 0, each where the neighbour lies inside the brick (lowok)
__device__ __forceinline__ uint32_t ref_children(uint32_t w, uint32_t lowok) {
    const uint32_t y = w & 0x77777777u;
    return (zero_nibbles(y ^ 0x11111111u) & ((lowok & 1u) ? 0x01010101u : 0u)) |
           (zero_nibbles(y ^ 0x22222222u) & ((lowok & 2u) ? 0x00110011u : 0u)) |
           (zero_nibbles(y ^ 0x33333333u) & ((lowok & 4u) ? 0x00001111u : 0u));
}

// 4 * byte b of q in one instruction (an SDWA source select)
template <int B>
__device__ __forceinline__ uint32_t byte_x4(uint32_t q) {
    uint32_t r;
    __asm__("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_%c2"
            : "=v"(r)
            : "v"(q), "n"(B));
    return r;
}

// follow a chain of same-level references in the dense leaf level: value v
// at voxel i, a reference to the voxel at -1 along axis v - kMark
template <class IdxT>
__device__ __forceinline__ uint32_t chase(const IdxT *D, uint32_t i, uint32_t v) {
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    while (v >= kMark) {
        i -= 1u << (5 * (v - kMark));  // 1, 32 or 1024
        v = D[i];
    }
    return v;
}

// The leaf level L_0 of one brick by one workgroup, and its 32^3 output.
// nib holds the nibbles from position nib0 on; l1m (Morton order) and bm1
// come from the front kernel; pal is the palette; ar the arena.  With u8
// indices in LDS, refs (ref_cap entries) lists the voxels that hold
// same-level references; they are resolved in one pass before the output,
// which then needs no chasing (a brick with more references than fit
// chases them in the output loop).  False on a malformed stream.
//
// after_pass2() runs once pass 2 is complete and checked, on every thread,
// before the references and the output (the leaf kernel issues the next
// brick's loads there, ahead of this brick's output stores).
template <class IdxT, bool kG, int NW, class Hook = NoHook>
__device__ __forceinline__ bool leaf_replay(const Hdr &h, uint32_t E1, uint32_t ipl, const uint32_t *nib,
                                            uint32_t nib0, const IdxT *l1m, const uint64_t *bm1w,
                                            const uint32_t *pal, uint8_t *ar, const LayoutL &lay, SmallB *sm,
                                            uint32_t *dst, uint16_t *refs, uint32_t ref_cap,
                                            const uint4 *l1pre = nullptr, Hook after_pass2 = Hook{}) {
    constexpr bool kList = sizeof(IdxT) == 1 && !kG;
    using V = Vec8<IdxT>;
    using VT = typename V::T;
    const uint32_t tid = threadIdx.x, L = lane(), w = tid >> 6;
    const uint32_t P = h.P;
    IdxT *l1 = reinterpret_cast<IdxT *>(ar + lay.l1);             // X + 16 Y + 256 Z
    uint16_t *bpre = reinterpret_cast<uint16_t *>(ar + lay.bpre);
    uint16_t *list1 = reinterpret_cast<uint16_t *>(ar + lay.list1);
    IdxT *D = reinterpret_cast<IdxT *>(ar + lay.leaf);            // x + 32 y + 1024 z
    const uint32_t seg = h.c1, seg_end = h.c0;
    if ((uint64_t)seg + 8ull * E1 > seg_end || E1 > 4096) return false;
    // L_1 to dense order: Morton indices 16t .. 16t + 15 share bits 4.. of t
    for (uint32_t t = tid; t < 256; t += (64 * NW)) {
        const uint32_t base = (((t >> 2) & 1u) << 2 | ((t >> 5) & 1u) << 3) +
                              16 * (((t & 1u) << 1) | (((t >> 3) & 1u) << 2) | (((t >> 6) & 1u) << 3)) +
                              256 * ((((t >> 1) & 1u) << 1) | (((t >> 4) & 1u) << 2) | (((t >> 7) & 1u) << 3));
        IdxT v[16];
        if constexpr (sizeof(IdxT) == 1) {
            // byte j goes to x + (j & 1) + 2 ((j >> 3) & 1), y + ((j >> 1) & 1),
            // z + ((j >> 2) & 1): four dense rows of four bytes, one byte
            // permute each (bytes 0..3 of q.x / q.y, then of q.z / q.w)
            const uint4 q = l1pre ? *l1pre : reinterpret_cast<const uint4 *>(l1m)[t];
            uint32_t *o = reinterpret_cast<uint32_t *>(l1 + base);
            o[0] = __builtin_amdgcn_perm(q.z, q.x, 0x05040100u);   // j = 0, 1, 8, 9
            o[4] = __builtin_amdgcn_perm(q.z, q.x, 0x07060302u);   // j = 2, 3, 10, 11 (y + 1)
            o[64] = __builtin_amdgcn_perm(q.w, q.y, 0x05040100u);  // j = 4, 5, 12, 13 (z + 1)
            o[68] = __builtin_amdgcn_perm(q.w, q.y, 0x07060302u);  // j = 6, 7, 14, 15
            continue;
        } else {
            const uint4 q0 = reinterpret_cast<const uint4 *>(l1m)[2 * t], q1 = reinterpret_cast<const uint4 *>(l1m)[2 * t + 1];
            const uint32_t qq[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int j = 0; j < 16; j++) v[j] = (IdxT)((qq[j >> 1] >> (16 * (j & 1))) & 0xFFFFu);
        }
#pragma unroll
        for (int j = 0; j < 16; j++)
            l1[base + (j & 1) + 2 * ((j >> 3) & 1) + 16 * ((j >> 1) & 1) + 256 * ((j >> 2) & 1)] = v[j];
    }
    if (w == 0) {  // rank prefix of the expansion bits, per 64-bit word
        const uint32_t c = (uint32_t)__popcll(bm1w[L]);
        bpre[L] = (uint16_t)(wave_incl_scan(c) - c);
    }
    __syncthreads();
    phase_mark(h.rq, 8);
    // every voxel takes its L_1 node's value (expanded nodes are overwritten
    // below); pass 1: this wave's P_a and P_delta totals
    for (uint32_t e = tid; e < 2048; e += (64 * NW)) {  // half rows of 16 voxels
        const uint32_t hx = e & 1u, y = (e >> 1) & 31u, z = e >> 6;
        const IdxT *src = l1 + 8 * hx + 16 * (y >> 1) + 256 * (z >> 1);
        IdxT *o = D + 16 * hx + 32 * y + 1024 * z;
        if constexpr (sizeof(IdxT) == 1) {
            const uint2 q = *reinterpret_cast<const uint2 *>(src);
            *reinterpret_cast<uint4 *>(o) =
                make_uint4(__builtin_amdgcn_perm(q.y, q.x, 0x01010000u), __builtin_amdgcn_perm(q.y, q.x, 0x03030202u),
                           __builtin_amdgcn_perm(q.y, q.x, 0x05050404u), __builtin_amdgcn_perm(q.y, q.x, 0x07070606u));
        } else {
            const uint4 q = *reinterpret_cast<const uint4 *>(src);
            const uint32_t qq[4] = {q.x, q.y, q.z, q.w};
            uint32_t r[8];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                r[2 * j] = __builtin_amdgcn_perm(qq[j], qq[j], 0x01000100u);
                r[2 * j + 1] = __builtin_amdgcn_perm(qq[j], qq[j], 0x03020302u);
            }
            reinterpret_cast<uint4 *>(o)[0] = make_uint4(r[0], r[1], r[2], r[3]);
            reinterpret_cast<uint4 *>(o)[1] = make_uint4(r[4], r[5], r[6], r[7]);
        }
    }
    const uint32_t D0 = seg_end - seg - 8 * E1, ops0 = seg + D0 - nib0;
    const uint32_t nch = (E1 + 63) / 64, cpw = (nch + NW - 1) / NW;
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
    // the expanded L_1 nodes (Morton indices) in Morton (= stream) order,
    // from the bitmask: 8 bits per thread
    for (uint32_t t = tid; t < 512; t += (64 * NW)) {
        // recomputed per brick rather than held in registers across bricks
        __asm__ volatile("" : "+v"(t));
        const uint32_t wd = t >> 3, q = t & 7u;
        const uint64_t word = bm1w[wd];
        uint32_t bits = (uint32_t)(word >> (8 * q)) & 0xFFu;
        uint32_t pos = bpre[wd] + (uint32_t)__popcll(word & ((1ull << (8 * q)) - 1ull));
        while (bits) {
            if (pos < E1) list1[pos] = (uint16_t)(64 * wd + 8 * q + (uint32_t)__builtin_ctz(bits));
            bits &= bits - 1;
            pos++;
        }
    }
    uint32_t bpa = 0, bpd = 0, PDtot = 0;
#pragma unroll
    for (int v = 0; v < NW; v++) {
        const uint32_t a0 = sm->wt[v][0], a1 = sm->wt[v][1];
        if ((uint32_t)v < w) {
            bpa += a0;
            bpd += a1;
        }
        PDtot += a1;
    }
    __syncthreads();
    if (PDtot != D0) return false;
    phase_mark(h.rq, 3);
    // pass 2: the children of every expanded L_1 node into the dense level
    bool bad = false;
    for (uint32_t c = cb; c < ce; c++) {
        const uint32_t r = 64 * c + L;
        const bool act = r < E1;
        const uint32_t wd = act ? nib8(nib, ops0 + 8 * r) : 0u;
        const uint32_t cc = act ? (uint32_t)list1[r] : 0u;  // Morton index of the node
        const uint32_t X = morton_coord(cc), Y = morton_coord(cc >> 1), Z = morton_coord(cc >> 2);
        const uint32_t lowok = (X > 0 ? 1u : 0u) | (Y > 0 ? 2u : 0u) | (Z > 0 ? 4u : 0u);
        uint32_t pam, pdm, exm, cnt;
        nibble_counts(wd, act, pam, pdm, exm, cnt);
        uint32_t refm = 0;  // bits 20..29 of the scan: references of this lane's children
        if constexpr (kList) refm = act ? ref_children(wd, lowok) : 0u;
        cnt = (cnt & 0xFFFFFu) | ((uint32_t)__builtin_popcount(refm) << 20);
        const uint32_t inc = wave_incl_scan(cnt), exc = inc - cnt;
        const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
        // child k = kx | ky << 1 | kz << 2 at voxel (2X + kx, 2Y + ky, 2Z + kz)
        const uint32_t v0 = 2 * X + 64 * Y + 2048 * Z;
        if constexpr (kList) {
            const uint32_t tr = tot >> 20;
            if (tr) {
                uint32_t base = 0;
                if (L == 0) base = atomicAdd(&sm->nref, tr);
                base = uniform(__builtin_amdgcn_readlane(base, 0));
                if (base + tr <= ref_cap) {
                    uint32_t pos = base + (exc >> 20);
                    while (refm) {
                        const uint32_t k = (uint32_t)__builtin_ctz(refm) >> 2;
                        refm &= refm - 1u;
                        refs[pos++] = (uint16_t)(v0 + (k & 1u) + 32 * ((k >> 1) & 1u) + 1024 * (k >> 2));
                    }
                }
            }
        }
        if (act) {
            const uint32_t i = X + 16 * Y + 256 * Z;
            const uint32_t pv = l1[i];
            const uint32_t nbv[3] = {X < 15 ? (uint32_t)l1[i + 1] : 0u, Y < 15 ? (uint32_t)l1[i + 16] : 0u,
                                     Z < 15 ? (uint32_t)l1[i + 256] : 0u};
            const uint32_t nbok = (X < 15 ? 1u : 0u) | (Y < 15 ? 2u : 0u) | (Z < 15 ? 4u : 0u);
            const VT vals = replay8<IdxT>(wd, pv, nbv, nbok, lowok, ipl + bpa + (exc & 1023u),
                                          compact_nibble_bits(pam), compact_nibble_bits(pdm), nib,
                                          seg - nib0 + bpd + ((exc >> 10) & 1023u), P, true, bad);
            // x pairs of children
            if constexpr (sizeof(IdxT) == 1) {
                *reinterpret_cast<uint16_t *>(D + v0) = (uint16_t)(vals.x & 0xFFFFu);
                *reinterpret_cast<uint16_t *>(D + v0 + 32) = (uint16_t)(vals.x >> 16);
                *reinterpret_cast<uint16_t *>(D + v0 + 1024) = (uint16_t)(vals.y & 0xFFFFu);
                *reinterpret_cast<uint16_t *>(D + v0 + 1056) = (uint16_t)(vals.y >> 16);
            } else {
                *reinterpret_cast<uint32_t *>(D + v0) = vals.x;
                *reinterpret_cast<uint32_t *>(D + v0 + 32) = vals.y;
                *reinterpret_cast<uint32_t *>(D + v0 + 1024) = vals.z;
                *reinterpret_cast<uint32_t *>(D + v0 + 1056) = vals.w;
            }
        }
        bpa += tot & 1023u;
        bpd += (tot >> 10) & 1023u;
    }
    if (__ballot(bad) && L == 0) atomicOr(&sm->err, 1);
    __syncthreads();
    if (sm->err) return false;
    phase_mark(h.rq, 15);
    after_pass2();
    // the listed references, each followed to its value (concurrent chases
    // see a reference or its final value, both of which lead to the value)
    bool resolved = false;
    if constexpr (kList) {
        const uint32_t nref = sm->nref;
        if (nref <= ref_cap) {
            // two chains per thread and round, their loads in flight together
            constexpr uint32_t kMarkL = sizeof(IdxT) == 1 ? 253u : 65533u;
            uint32_t e = tid;
            for (; e + 64 * NW < nref; e += 2 * 64 * NW) {
                const uint32_t a0 = refs[e], b0 = refs[e + 64 * NW];
                uint32_t ia = a0, ib = b0, va = D[a0], vb = D[b0];
                while (va >= kMarkL || vb >= kMarkL) {
                    if (va >= kMarkL) {
                        ia -= 1u << (5 * (va - kMarkL));
                        va = D[ia];
                    }
                    if (vb >= kMarkL) {
                        ib -= 1u << (5 * (vb - kMarkL));
                        vb = D[ib];
                    }
                }
                D[a0] = (IdxT)va;
                D[b0] = (IdxT)vb;
            }
            if (e < nref) {
                const uint32_t v = refs[e];
                D[v] = (IdxT)chase<IdxT>(D, v, D[v]);
            }
            __syncthreads();
            resolved = true;
        }
    }
    phase_mark(h.rq, 4);
    // output: a wave writes 8 whole rows of a z slice per store; lane L
    // covers voxels 4 (L & 7) .. + 3 of rows (L >> 3) + 8c; references are
    // followed along the dense level (at most three links)
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    auto slices = [&](auto al16, auto refs_left) {
        for (uint32_t zz = w; zz < 32; zz += NW) {
#pragma unroll 2
            for (int c = 0; c < 4; c++) {
                const uint32_t v0 = 4 * (L & 7u) + 32 * ((L >> 3) + 8 * (uint32_t)c) + 1024 * zz;
                uint32_t idx[4];
                if constexpr (sizeof(IdxT) == 1 && !kG && !decltype(refs_left)::value) {
                    // no references left: each byte is a palette index in LDS
                    const uint32_t q = *reinterpret_cast<const uint32_t *>(D + v0);
                    const uint8_t *pb = reinterpret_cast<const uint8_t *>(pal);
                    uint4 o;
                    o.x = *reinterpret_cast<const uint32_t *>(pb + byte_x4<0>(q));
                    o.y = *reinterpret_cast<const uint32_t *>(pb + byte_x4<1>(q));
                    o.z = *reinterpret_cast<const uint32_t *>(pb + byte_x4<2>(q));
                    o.w = *reinterpret_cast<const uint32_t *>(pb + byte_x4<3>(q));
                    store4<decltype(al16)::value>(dst + v0, o);
                    continue;
                } else if constexpr (sizeof(IdxT) == 1) {
                    const uint32_t q = *reinterpret_cast<const uint32_t *>(D + v0);
#pragma unroll
                    for (int b = 0; b < 4; b++) idx[b] = (q >> (8 * b)) & 0xFFu;
                    // bytes >= 252: a reference (252 never survives the checks)
                    const uint32_t t = ~q & 0xFCFCFCFCu;
                    if (decltype(refs_left)::value && ((t - 0x01010101u) & ~t & 0x80808080u) != 0) {
#pragma unroll
                        for (int b = 0; b < 4; b++)
                            if (idx[b] >= kMark) idx[b] = chase<IdxT>(D, v0 + (uint32_t)b, idx[b]);
                    }
                } else {
                    const uint2 q = *reinterpret_cast<const uint2 *>(D + v0);
                    idx[0] = q.x & 0xFFFFu;
                    idx[1] = q.x >> 16;
                    idx[2] = q.y & 0xFFFFu;
                    idx[3] = q.y >> 16;
#pragma unroll
                    for (int b = 0; b < 4; b++)
                        if (idx[b] >= kMark) idx[b] = chase<IdxT>(D, v0 + (uint32_t)b, idx[b]);
                }
                uint4 o;
                o.x = pal_at<kG>(pal, idx[0], P);
                o.y = pal_at<kG>(pal, idx[1], P);
                o.z = pal_at<kG>(pal, idx[2], P);
                o.w = pal_at<kG>(pal, idx[3], P);
                store4<decltype(al16)::value>(dst + v0, o);
            }
        }
    };
    const bool al = (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
    if (resolved) {
        if (al) slices(std::true_type{}, std::false_type{});
        else slices(std::false_type{}, std::false_type{});
    } else {
        if (al) slices(std::true_type{}, std::true_type{});
        else slices(std::false_type{}, std::true_type{});
    }
    phase_mark(h.rq, 5);
    return true;
}

// A leaf descriptor in one VGPR: lane j (< 12) holds dword j of the
// descriptor of work item `item`, lane 12 the item itself (a vector load:
// it counts on vmcnt, not on lgkmcnt, so the LDS waits of the brick in
// progress never wait for it)
__device__ __forceinline__ uint32_t desc_lane(const LeafDesc *list, uint32_t item, uint32_t n_items) {
    uint32_t L = lane();
    // the lane's address is recomputed per call, not kept in registers
    // across the replay
    __asm__ volatile("" : "+v"(L));
    if (L == 12) return item;
    return (item < n_items && L < 12) ? glob(reinterpret_cast<const uint32_t *>(list + item))[L] : 0u;
}
struct LeafFields {
    uint32_t rq, id, P, c0, c1, E1, ipl, item;
    uint64_t rec, dst;
};
__device__ __forceinline__ LeafFields leaf_fields(uint32_t v) {
    LeafFields f;
    f.rq = __builtin_amdgcn_readlane(v, 0);
    f.id = __builtin_amdgcn_readlane(v, 1);
    f.P = __builtin_amdgcn_readlane(v, 2);
    f.c0 = __builtin_amdgcn_readlane(v, 3);
    f.c1 = __builtin_amdgcn_readlane(v, 4);
    f.E1 = __builtin_amdgcn_readlane(v, 5);
    f.ipl = __builtin_amdgcn_readlane(v, 6);
    f.item = __builtin_amdgcn_readlane(v, 12);
    // readlane returns an int: widen through uint32_t (no sign extension)
    f.rec = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 8) | (uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 9) << 32;
    f.dst = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 10) | (uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 11) << 32;
    return f;
}
// the descriptor in LDS slot k, one dword per lane
__device__ __forceinline__ LeafFields leaf_fields_lds(const SmallB *sm, uint32_t k) {
    const uint32_t L = lane();
    return leaf_fields(sm->desc[k][L < 13 ? L : 0]);
}
// How a leaf brick is staged: fast (palette, nibbles from the delta segment
// of L_0 on, from a 16-byte boundary, and the arrays in the LDS arena), lean
// (the same without the nibbles, which are then read from the slot), or
// neither (the slow list)
struct LeafKind {
    uint32_t nb0, nib4;
    bool fast, lean;
    LayoutL lay;
};
__device__ __forceinline__ LeafKind leaf_kind(const LeafFields &f, uint32_t arena_bytes) {
    LeafKind k;
    const uint32_t E1c = f.E1 < 4096 ? f.E1 : 4096u;
    k.nb0 = (f.c1 >> 5) << 2;
    k.nib4 = (((f.c0 + 7) >> 3) + 2 - k.nb0 + 3) / 4;
    const LayoutL fast = make_layout_l(true, f.P, k.nib4, E1c, 1);
    const LayoutL lean = make_layout_l(true, f.P, 0, E1c, 1);
    k.fast = f.P <= kPalFast && fast.total <= arena_bytes;
    k.lean = !k.fast && f.P <= kPalFast && lean.total <= arena_bytes;
    k.lay = k.fast ? fast : lean;
    return k;
}
// A leaf brick's staging data in registers: q is group tid of L_1 (Morton
// order) for tid < 256 and group tid - 256 of its expansion bits for
// 256 <= tid < 288; nb is nibble group tid (fast bricks); pal is palette
// entry tid
struct LeafPre {
    uint4 q, nb;
    uint32_t pal;
};
__device__ __forceinline__ void leaf_prefetch(LeafPre &p, const LeafFields &f, bool valid, const LaunchB &l,
                                              uint32_t hdr, uint32_t tid) {
    p.q = make_uint4(0u, 0u, 0u, 0u);
    p.nb = p.q;
    p.pal = 0;
    if (!valid) return;
    const LeafKind k = leaf_kind(f, l.arena_bytes);
    if (!k.fast && !k.lean) return;
    const uint8_t *slot = glob(l.slots) + (size_t)f.rq * l.slot_bytes;
    const uint8_t *slv = slot + 4 * l.slot_dw;
    if (tid < 256) p.q = reinterpret_cast<const uint4 *>(slv)[tid];
    else if (tid < 288) p.q = reinterpret_cast<const uint4 *>(slv + kSlotLv)[tid - 256];
    if (tid < f.P) p.pal = rec_at(f.rec)[hdr + tid];
    if (k.fast && tid < k.nib4) p.nb = reinterpret_cast<const uint4 *>(slot + 4 * k.nb0)[tid];
}

// Bricks that fit the LDS arena.  Each brick is staged from registers
// loaded while the workgroup replayed the previous brick, after its pass 2
// and before its output: loads issued after a brick's output stores would
// wait behind them (on gfx9 one counter tracks both, and the memory path
// serves them in order).  The work items come from a counter (after a first
// fixed round), and run ahead of the replay so that nothing waits for them:
// while brick k is replayed the workgroup loads the staging data of brick
// k + 1 and the descriptor of brick k + 2, and takes the item of brick
// k + 3.  Descriptors and items pass through LDS (two descriptor slots and
// one item), so that no register holds them during a replay.
template <int NW>
__device__ __forceinline__ void leaf_fast_bricks(const DecodeArgs &a, const LaunchB &l, SmallB *sm, uint8_t *arena,
                                                 uint32_t n_items, const LeafDesc *list) {
    constexpr uint32_t NT = 64 * NW;
    static_assert(NT >= 288, "threads below 288 hold level 1 and its expansion bits");
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t hdr = csv::record_header_words(kLog2);
    uint32_t *queue = glob(l.queue);
    // Items 0 .. 3 gridDim.x - 1 go out in a fixed order (workgroup b starts
    // with b, b + G and b + 2G), the rest from the counter, one per replayed
    // brick (thread 0).  An increment, not an add: the compiler rewrites a
    // uniform-address add so that it reads the result at once, and that
    // wait would also wait for the loads issued just before it.
    const uint32_t G = gridDim.x;
    auto take = [&]() -> uint32_t { return 3 * G + atomicInc(queue, 0xFFFFFFFFu); };
    if (tid == 0) {
        sm->desc[0][12] = blockIdx.x;
        sm->desc[1][12] = blockIdx.x + G;
        sm->item2 = blockIdx.x + 2 * G;
    }
    __syncthreads();
    // brick 0's descriptor and staging data, and brick 1's descriptor
    LeafPre pre;
    uint32_t ndv = 0, r = 0;
    {
        const uint32_t i0 = sm->desc[0][12], v0 = desc_lane(list, i0, n_items);
        leaf_prefetch(pre, leaf_fields(v0), i0 < n_items, l, hdr, tid);
        if (w == 0) ndv = desc_lane(list, sm->desc[1][12], n_items);
        __syncthreads();
        if (tid < 13) sm->desc[0][tid] = v0;
    }
    __syncthreads();
    for (uint32_t k = 0;; k++) {
        const uint32_t cur = k & 1u;
        const LeafFields f = leaf_fields_lds(sm, cur);
        if (f.item >= n_items) break;
        const uint32_t rq = f.rq;
        phase_mark(rq, 6);
#ifdef CSV_PHASE_TIMING
        if (g_phase && tid == 0) g_phase[16 * (size_t)rq + 7] = (uint64_t)blockIdx.x | (uint64_t)k << 32;
#endif
        Hdr h;
        h.rq = rq;
        h.id = f.id;
        h.P = f.P;
        h.c0 = f.c0;
        h.c1 = f.c1;
        h.rec = rec_at(f.rec);
        uint32_t *dst = reinterpret_cast<uint32_t *>(f.dst);
        const uint32_t *gnib = reinterpret_cast<const uint32_t *>(glob(l.slots) + (size_t)rq * l.slot_bytes);
        const uint8_t *slv = reinterpret_cast<const uint8_t *>(gnib) + 4 * l.slot_dw;
        const LeafKind kd = leaf_kind(f, l.arena_bytes);
        if (tid == 0) {
            sm->err = 0;
            sm->nref = 0;
            if (k > 0) sm->item2 = r;  // the item of brick k + 2, taken while brick k - 1 was replayed
        }
        if (tid < 13) sm->desc[cur ^ 1u][tid] = ndv;
        bool ok = true, done = true, pre_done = false;
        // loads for the next bricks (every thread; after a barrier that
        // follows the LDS writes above)
        auto next = [&]() {
            const LeafFields nf = leaf_fields_lds(sm, cur ^ 1u);
            leaf_prefetch(pre, nf, nf.item < n_items, l, hdr, tid);
            if (w == 0) ndv = desc_lane(list, sm->item2, n_items);
            if (tid == 0) r = take();
            pre_done = true;
        };
        if (kd.fast || kd.lean) {
            if (tid < h.P) reinterpret_cast<uint32_t *>(arena + kd.lay.pal)[tid] = pre.pal;
            if (tid >= 256 && tid < 288) reinterpret_cast<uint4 *>(arena + kd.lay.bm1)[tid - 256] = pre.q;
            if (kd.fast) {
                if (tid < kd.nib4) reinterpret_cast<uint4 *>(arena + kd.lay.nib)[tid] = pre.nb;
                for (uint32_t e = tid + NT; e < kd.nib4; e += NT)
                    reinterpret_cast<uint4 *>(arena + kd.lay.nib)[e] = reinterpret_cast<const uint4 *>(gnib + kd.nb0)[e];
            }
            const uint4 l1q = pre.q;
            __syncthreads();
            const uint32_t ref_cap = min((l.arena_bytes - kd.lay.total) / 2, l.ref_cap);
            uint16_t *refs = reinterpret_cast<uint16_t *>(arena + kd.lay.total);
            const uint64_t *bm1 = reinterpret_cast<const uint64_t *>(arena + kd.lay.bm1);
            const uint32_t *pal = reinterpret_cast<const uint32_t *>(arena + kd.lay.pal);
            if (kd.fast)
                ok = leaf_replay<uint8_t, false, NW>(h, f.E1, f.ipl, reinterpret_cast<const uint32_t *>(arena + kd.lay.nib),
                                                     8 * kd.nb0, slv, bm1, pal, arena, kd.lay, sm, dst, refs, ref_cap,
                                                     &l1q, next);
            else
                ok = leaf_replay<uint8_t, false, NW>(h, f.E1, f.ipl, gnib, 0, slv, bm1, pal, arena, kd.lay, sm, dst,
                                                     refs, ref_cap, &l1q, next);
        } else {
            __syncthreads();
            if (l.slow_list) {  // the slow kernel takes it
                done = false;
                if (tid == 0) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(glob(list + f.item));
                    uint4 *to = reinterpret_cast<uint4 *>(l.slow_list + atomicAdd(l.slow_count, 1u));
                    to[0] = src[0];
                    to[1] = src[1];
                    to[2] = src[2];
                }
            } else {  // the pool's bounds say every brick fits: a corrupt record
                ok = false;
            }
        }
        if (!pre_done) next();  // no replay, or one that stopped early
        __syncthreads();
        if (done && !ok) {
            if (tid == 0) fail(a, rq, CSV_ECORRUPT, h.id);
            fill_labels<NT>(dst, 32768u, 0u, tid);
        }
        __syncthreads();
    }
    // the last item taken has returned before this workgroup reports that it
    // is done (the last workgroup to finish clears the counter)
    __builtin_amdgcn_s_waitcnt(0);
}

// kSlow false: bricks whose arrays fit the LDS arena, the others deferred
// to the slow list; kSlow true: the slow list, on an arena in global memory
template <int NW, bool kSlow>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(kSlow ? 4 : 6))) void leaf_kernel(DecodeArgs a,
                                                                                                      LaunchB l) {
    constexpr uint32_t NT = 64 * NW;
    extern __shared__ __align__(16) uint8_t smem[];
    SmallB *sm = reinterpret_cast<SmallB *>(smem);
    uint8_t *arena = smem + align16(sizeof(SmallB));
    uint8_t *gslot = l.scratch ? glob(l.scratch) + (size_t)blockIdx.x * l.scratch_bytes : nullptr;
    const uint32_t tid = threadIdx.x;
    const uint32_t hdr = csv::record_header_words(kLog2);
    const uint32_t n_items = *glob(kSlow ? l.slow_count : l.leaf_count);
    const LeafDesc *list = kSlow ? l.slow_list : l.leaf_list;
    if constexpr (!kSlow) {
        leaf_fast_bricks<NW>(a, l, sm, arena, n_items, list);
    } else {
        uint32_t *queue = l.slow_queue;
        for (uint32_t k = 0;; k++) {
            if (tid == 0) sm->req = queue ? atomicAdd(queue, 1u) : blockIdx.x + k * gridDim.x;
            __syncthreads();
            const uint32_t item = uniform(sm->req);
            if (item >= n_items) break;
            // a request at t = 0 the front kernel has checked and decoded down
            // to level 1, whose arrays do not fit the LDS arena
            const LeafDesc *ds = list + item;
            const uint32_t rq = ld_s(&ds->rq);
            Hdr h;
            h.rq = rq;
            h.id = ld_s(&ds->id);
            h.P = ld_s(&ds->P);
            h.c0 = ld_s(&ds->c0);
            h.c1 = ld_s(&ds->c1);
            h.rec = rec_at(ld_s(&ds->rec));
            uint32_t *dst = reinterpret_cast<uint32_t *>(ld_s(&ds->dst));
            const uint32_t E1 = ld_s(&ds->E1), ipl = ld_s(&ds->ipl);
            phase_mark(rq, 6);
            const uint8_t *slot = glob(l.slots) + (size_t)rq * l.slot_bytes;
            const uint32_t *gnib = reinterpret_cast<const uint32_t *>(slot);
            const uint8_t *slv = slot + 4 * l.slot_dw;
            const uint64_t *gbm = reinterpret_cast<const uint64_t *>(slv + kSlotLv);
            if (tid == 0) {
                sm->err = 0;
                sm->nref = 0;
            }
            phase_mark(rq, 7);
            __syncthreads();
            bool ok;
            if (!gslot)
                ok = false;
            else if (h.P <= kPalFast)
                ok = leaf_replay<uint8_t, true, NW>(h, E1, ipl, gnib, 0, slv, gbm, h.rec + hdr, gslot,
                                                    make_layout_l(false, 0, 0, 4096, 1), sm, dst, nullptr, 0);
            else
                ok = leaf_replay<uint16_t, true, NW>(h, E1, ipl, gnib, 0, reinterpret_cast<const uint16_t *>(slv), gbm,
                                                     h.rec + hdr, gslot, make_layout_l(false, 0, 0, 4096, 2), sm, dst,
                                                     nullptr, 0);
            __syncthreads();
            if (!ok) {
                if (tid == 0) fail(a, rq, gslot ? CSV_ECORRUPT : CSV_EINVAL, h.id);
                fill_labels<NT>(dst, 32768u, 0u, tid);
            }
            __syncthreads();
        }
    }
    // the last workgroup to finish clears the counters this kernel was the
    // last to use, for the next launch on these buffers: every other
    // workgroup has had its last counter operation return by then.  No
    // fence: the counters only change by atomics, and the kernel boundary
    // orders them for the next launch (a device-scope fence per workgroup
    // would write back the L2).
    if (tid == 0) {
        uint32_t *ctr = glob(l.ctr);
        if (atomicAdd(ctr + (kSlow ? 6 : 5), 1u) == gridDim.x - 1) {
            if (kSlow) {
                atomicExch(ctr + 3, 0u);
                atomicExch(ctr + 4, 0u);
                atomicExch(ctr + 6, 0u);
            } else {
                atomicExch(ctr + 0, 0u);
                atomicExch(ctr + 1, 0u);
                atomicExch(ctr + 2, 0u);
                atomicExch(ctr + 5, 0u);
            }
        }
    }
}

// Longest-first request order: requests are binned by their work (symbols
// to decode plus output voxels / 8) on a log scale with 8 bins per octave
// (the bits after the leading one), largest first; the order within a bin
// is arbitrary.  Two launches of many workgroups: order_count adds up the
// bin sizes, order_place gives each request its rank (exclusive scan of
// the sizes plus a per-bin cursor).  The ranks are laid out for the front
// kernel's fixed assignment, in which round k of its W waves takes
// positions kW .. kW + W - 1: odd rounds run in reverse (snake order), so
// that the wave with the largest brick of one round gets the smallest of
// the next (a partial last round keeps its ranks).
constexpr int kBins = 128;
constexpr uint32_t kOrderWords = 2 * kBins + 8;   // bin sizes, bin cursors, done counter
constexpr uint32_t kSmallWords = kOrderWords + 8; // then the launch counters
__device__ __forceinline__ uint32_t work_bin(const DecodeArgs &a, uint32_t r) {
    const uint32_t id = a.ids[r];
    const uint32_t t = a.lods ? (uint32_t)a.lods[r] : a.lod_scalar;
    if (id >= a.n_bricks || t > (uint32_t)kLog2) return kBins - 1;
    const uint32_t *rec = rec_at(a.rec_ptr[id]);
    const uint32_t n = t < (uint32_t)kLog2 ? rec[3 + t] : 0u;
    const uint32_t g = 32u >> t;
    const uint32_t work = n + (g * g * g) / 8 + 1;
    const uint32_t lz = 31u - (uint32_t)__builtin_clz(work);  // floor(log2(work))
    const uint32_t frac = lz >= 3 ? (work >> (lz - 3)) & 7u : (work << (3 - lz)) & 7u;
    const uint32_t key = 8 * lz + frac;                       // about 8 log2(work)
    return key >= (uint32_t)kBins - 1 ? 0u : (uint32_t)kBins - 1 - key;
}
__global__ __launch_bounds__(256) void order_count(DecodeArgs a, uint32_t *cnt) {
    __shared__ uint32_t h[kBins];
    const uint32_t tid = threadIdx.x;
    for (uint32_t b = tid; b < (uint32_t)kBins; b += 256) h[b] = 0;
    __syncthreads();
    for (uint32_t r = blockIdx.x * 256 + tid; r < a.n; r += gridDim.x * 256) atomicAdd(&h[work_bin(a, r)], 1u);
    __syncthreads();
    for (uint32_t b = tid; b < (uint32_t)kBins; b += 256)
        if (h[b]) atomicAdd(cnt + b, h[b]);
}
// same grid as order_count; the last workgroup to finish clears the sizes,
// cursors and its done counter for the next launch
__global__ __launch_bounds__(256) void order_place(DecodeArgs a, uint32_t *small, uint32_t *order, uint32_t W) {
    static_assert(kBins == 128, "two waves scan the bin sizes");
    __shared__ uint32_t off[kBins], h[kBins], base[kBins], tot0, last;
    uint32_t *cnt = glob(small), *cur = cnt + kBins, *done = cnt + 2 * kBins;
    const uint32_t tid = threadIdx.x;
    // exclusive scan of the bin sizes (waves 0 and 1, 64 bins each)
    uint32_t c = 0, inc = 0;
    if (tid < (uint32_t)kBins) {
        c = cnt[tid];
        inc = wave_incl_scan(c);
        if (tid == 63) tot0 = inc;
        h[tid] = 0;
    }
    __syncthreads();
    if (tid < (uint32_t)kBins) off[tid] = inc - c + (tid >= 64 ? tot0 : 0u);
    // this workgroup's bin sizes, then its range of each bin
    for (uint32_t r = blockIdx.x * 256 + tid; r < a.n; r += gridDim.x * 256) atomicAdd(&h[work_bin(a, r)], 1u);
    __syncthreads();
    if (tid < (uint32_t)kBins) {
        base[tid] = h[tid] ? atomicAdd(cur + tid, h[tid]) : 0u;
        h[tid] = 0;
    }
    __syncthreads();
    for (uint32_t r = blockIdx.x * 256 + tid; r < a.n; r += gridDim.x * 256) {
        const uint32_t b = work_bin(a, r);
        uint32_t pos = off[b] + base[b] + atomicAdd(&h[b], 1u);
        const uint32_t rnd = pos / W, w = pos - rnd * W;
        if ((rnd & 1u) && (uint64_t)rnd * W + W <= a.n) pos = rnd * W + (W - 1 - w);
        order[pos] = r;
    }
    __syncthreads();
    if (tid == 0) last = atomicAdd(done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (last)
        for (uint32_t i = tid; i < 2 * (uint32_t)kBins + 1; i += 256) cnt[i] = 0;
}
__global__ void zero_words(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Empty-space test (Sec. 4, empty-space skipping): a brick is visible when
// some label of its palette (the brick's distinct labels) has its bit set in
// `bits`; labels >= n_bits are invisible.  One wave per request, 64 palette
// entries per step, a ballot decides.
__global__ __launch_bounds__(256) void visible_kernel(const uint64_t *rec_ptr, const uint32_t *rec_size,
                                                      uint32_t n_bricks, const uint32_t *ids, uint32_t n,
                                                      const uint32_t *bits, uint32_t n_bits, uint8_t *out,
                                                      int *err, uint32_t hdr) {
    const uint32_t L = lane(), wave = uniform(threadIdx.x >> 6);
    for (uint32_t r = blockIdx.x * 4 + wave; r < n; r += gridDim.x * 4) {
        const uint32_t id = ld_s(ids + r);
        if (id >= n_bricks) {
            if (L == 0) {
                out[r] = 0;
                report(err, CSV_ERANGE, r);
            }
            continue;
        }
        const uint32_t *rec = rec_at(ld_s(rec_ptr + id));
        const uint32_t P = ld_s(rec);
        if (P == 0 || 4ull * ((uint64_t)hdr + P) > ld_s(rec_size + id)) {
            if (L == 0) {
                out[r] = 0;
                report(err, CSV_ECORRUPT, id);
            }
            continue;
        }
        bool vis = false;
        for (uint32_t b = 0; b < P; b += 64) {
            const uint32_t e = b + L;
            const uint32_t lab = e < P ? rec[hdr + e] : 0xFFFFFFFFu;
            const bool v = lab < n_bits && ((bits[lab >> 5] >> (lab & 31u)) & 1u) != 0;
            if (__ballot(v) != 0) {
                vis = true;
                break;
            }
        }
        if (L == 0) out[r] = vis ? 1 : 0;
    }
}

// Per-stream launch buffers: the nibble buffer and status bytes that pass
// requests from the entropy decoder to the replay, the longest-first order,
// and the two work counters.  Launches on one stream are ordered, so they
// share one set; launches on different streams get different sets.
struct LaunchBufs {
    hipStream_t stream = nullptr;
    uint64_t last_use = 0;
    uint8_t *slots = nullptr;      // slot_bytes per request
    uint32_t *order = nullptr;     // longest-first order
    LeafDesc *leaf_list = nullptr; // requests for the leaf kernel
    LeafDesc *slow_list = nullptr; // ... of them for its global-arena variant
    uint32_t *small = nullptr;     // kOrderWords of order bins, then 8 launch counters
    uint8_t *arenas = nullptr;     // global arenas of the global-arena leaf kernel, one per workgroup
    uint32_t arena_groups = 0;     // workgroups they serve
    bool owned = true;             // false: a view of memory the library does not allocate
    bool dirty = false;            // counters left non-zero by a failed launch
    uint32_t slot_dw = 0;
    uint32_t cap_n = 0;
    uint8_t *gen = nullptr;        // scratch of the decoder for other brick sizes and raw nibbles
    uint64_t gen_bytes = 0;
    uint32_t slot_bytes() const { return 4 * slot_dw + kSlotExtra; }
    void release() {
        if (owned) {
            (void)hipFree(slots);
            (void)hipFree(order);
            (void)hipFree(leaf_list);
            (void)hipFree(slow_list);
            (void)hipFree(small);
            (void)hipFree(arenas);
            (void)hipFree(gen);
        }
        gen = nullptr;
        gen_bytes = 0;
        slots = nullptr;
        order = nullptr;
        leaf_list = nullptr;
        slow_list = nullptr;
        small = nullptr;
        arenas = nullptr;
        arena_groups = 0;
        cap_n = 0;
    }
    // global arenas for `groups` workgroups (kept once allocated)
    int reserve_arenas(uint32_t groups) {
        if (arenas && arena_groups >= groups) return CSV_OK;
        if (!owned) return CSV_EINVAL;
        (void)hipFree(arenas);
        arenas = nullptr;
        arena_groups = 0;
        if (hipMalloc(reinterpret_cast<void **>(&arenas), (size_t)groups * kArenaBytes) != hipSuccess) return CSV_ENOMEM;
        arena_groups = groups;
        return CSV_OK;
    }
    // room for n requests with slot_dw nibble dwords each
    int reserve(uint32_t n, uint32_t dw) {
        if (slots && n <= cap_n && dw == slot_dw) return CSV_OK;
        release();
        const uint32_t cap = std::max(n, 1024u);
        slot_dw = dw;
        if (hipMalloc(reinterpret_cast<void **>(&slots), (size_t)cap * slot_bytes()) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&order), 4ull * cap) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&leaf_list), sizeof(LeafDesc) * cap) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&slow_list), sizeof(LeafDesc) * cap) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&small), 4 * kSmallWords) != hipSuccess) {
            release();
            return CSV_ENOMEM;
        }
        cap_n = cap;
        // the counters are cleared by a kernel on the stream that uses them
        // (a memset on another stream would not be ordered with its work)
        dirty = true;
        return CSV_OK;
    }
    // HBM of the slots, lists and counters for cap requests of dw nibble dwords
    static uint64_t sized(uint32_t cap, uint32_t dw) {
        return (uint64_t)cap * (4ull * dw + kSlotExtra + 4 + 2 * sizeof(LeafDesc)) + 4 * 72;
    }
    uint64_t bytes() const {
        return (slots ? sized(cap_n, slot_dw) : 0) + (uint64_t)arena_groups * kArenaBytes + gen_bytes;
    }
};
constexpr size_t kMaxStreamBufs = 16;

// csv_decode_bricks_noalloc: the launch buffers of one decode (counters and
// order bins, global arenas, order and leaf lists, per-request slots) carved
// out of one fixed device array instead of allocated memory
constexpr size_t kNoAllocBytes = 64ull << 20;
constexpr uint32_t kNoAllocArenas = 32;
constexpr size_t kNoAllocSmall = 2048;  // order bins and counters
constexpr size_t kNoAllocHead = kNoAllocSmall + (size_t)kNoAllocArenas * kArenaBytes;  // then the arenas
static_assert(4 * kSmallWords <= kNoAllocSmall, "order bins and counters");
static_assert(kNoAllocHead % 256 == 0, "arena layout");

}  // namespace

// Scratch of csv_decode_bricks_noalloc: one copy per GPU, held until the
// process ends.  In host code this name is not a device address: host code
// uses the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

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
    uint32_t brick_log2 = 0;                  // brick edge 2^brick_log2 of every volume (0: none yet)
    bool generic = false;                     // a volume of another brick size or with raw nibbles:
                                              // every decode takes the generic decoder
    std::vector<uint8_t> vol_raw;             // per volume: symbols stored as raw nibbles
    uint8_t *d_vol_raw = nullptr;
    uint64_t use_clock = 0;
    uint32_t max_c0 = 0;                      // most symbols of any brick in the pool
    uint32_t max_fast_bytes = 0;              // largest LDS arena a brick of the pool needs (nibbles not staged)
    bool any_big_palette = false;
    uint64_t hbm_budget = 0;                  // HBM the pool may hold (0: no limit)
    uint32_t generation = 0;                  // bumped when device tables move
    csv_shape shape{16, 3, 0, 0, 4, 0.f};     // launch shape of csv_decode_bricks (untuned classes)
    bool shape_set = false;                   // shape given by csv_pool_set_shape
    std::map<uint32_t, csv_shape> tuned;      // autotuned shapes by request-set class (tune_key)
    char device_name[64] = {0};
    uint64_t record_bytes = 0;
    // level-0 detail in host memory (csv_pool_add_volume_ex, CSV_DETAIL_HOST)
    bool any_split = false;
    std::vector<uint32_t> pfx_dw;            // per brick: word dwords in the device record (~0u: all)
    std::vector<const uint8_t *> det_host;   // per brick: the remaining dwords in pinned host memory
    std::vector<uint32_t> det_bytes;
    std::vector<uint8_t> staged;             // per brick: its detail is in the staging buffer
    std::vector<void *> host_bufs;           // pinned detail buffers
    uint64_t host_bytes = 0;
    uint32_t *d_pfx_dw = nullptr;
    uint64_t *d_sfx = nullptr;               // per brick: device address of the staged detail (0: none)
    uint64_t *h_sfx = nullptr;               // its pinned host image (n_sfx entries)
    uint32_t n_sfx = 0;
    uint8_t *d_stage = nullptr, *h_stage = nullptr;  // staging buffer and its pinned host image
    uint64_t stage_cap = 8ull << 20, stage_used = 0, stage_alloc = 0;
    hipEvent_t stage_ev = nullptr;           // the last staging copies
    // pipelined decodes: per caller stream, a second stream that takes every
    // other chunk of requests, and the events that fork it from the caller's
    // stream and join it back
    struct Companion {
        hipStream_t caller = nullptr, own = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
    };
    std::vector<Companion> companions;       // reserved once: entries never move
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

// the per-brick arrays of pools with level-0 detail in host memory, sized to
// the pool's bricks (bricks of ordinary volumes keep their whole record);
// staged detail stays staged
int sync_split(csv_pool *p) {
    if (!p->any_split) return CSV_OK;
    const size_t nb = p->rec_ptr.size();
    p->pfx_dw.resize(nb, 0xFFFFFFFFu);
    p->det_host.resize(nb, nullptr);
    p->det_bytes.resize(nb, 0u);
    p->staged.resize(nb, 0u);
    int rc = upload(&p->d_pfx_dw, p->pfx_dw);
    if (rc) return rc;
    if (p->n_sfx != nb) {
        uint64_t *h = nullptr;
        if (hipHostMalloc(reinterpret_cast<void **>(&h), 8 * nb, hipHostMallocDefault) != hipSuccess) return CSV_ENOMEM;
        std::memset(h, 0, 8 * nb);
        if (p->h_sfx) {
            std::memcpy(h, p->h_sfx, 8ull * p->n_sfx);
            (void)hipHostFree(p->h_sfx);
        }
        p->h_sfx = h;
        (void)hipFree(p->d_sfx);
        p->d_sfx = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&p->d_sfx), 8 * nb) != hipSuccess) return CSV_ENOMEM;
        p->n_sfx = (uint32_t)nb;
    }
    return hipMemcpy(p->d_sfx, p->h_sfx, 8ull * p->n_sfx, hipMemcpyHostToDevice) == hipSuccess ? CSV_OK : CSV_EHIP;
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
uint32_t slot_dw(const csv_pool *p) { return ((p->max_c0 + 7) / 8 + 8 + 3) & ~3u; }
constexpr uint32_t kSmallB = (sizeof(SmallB) + 15u) & ~15u;
constexpr uint32_t kMaxGroupsB = 8;
// leaf arena when `groups` leaf workgroups share a CU's LDS (whole 4 KiB
// per workgroup: LDS is allocated in granules, and a workgroup that rounds
// up past its share would leave room for one fewer)
uint32_t arena_b(uint32_t groups) { return ((kLdsBytes / groups) & ~4095u) - kSmallB; }
// workgroups of the global-arena leaf kernel (4 per CU), each with its own arena
uint32_t slow_groups(uint32_t cu) { return 4 * cu; }

// the buffers of stream s, sized for n requests (pool->mu held)
// HBM held by the pool: records, per-brick arrays, tables, launch buffers, staging
uint64_t pool_device_bytes(const csv_pool *p) {
    uint64_t lb = 0;
    for (const auto &b : p->bufs) lb += b.bytes();
    return p->record_bytes + p->rec_ptr.size() * (8 + 4 + 2) + p->luts.size() * 4 + lb +
           (p->any_split ? p->rec_ptr.size() * (4 + 8) + p->stage_alloc : 0);
}
// would `more` bytes of HBM exceed the pool's budget?
bool over_budget(const csv_pool *p, uint64_t more) {
    return p->hbm_budget && pool_device_bytes(p) + more > p->hbm_budget;
}

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each GPU holds the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_at[kMaxDevices] = {};
int scratch_address(int dev, uint8_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        DeviceGuard g(dev);
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CSV_EHIP;
        g_scratch_at[dev] = static_cast<uint8_t *>(ptr);
    }
    *out = g_scratch_at[dev];
    return CSV_OK;
}

// the buffer set of stream s, taken over from the least recently used
// stream when all kMaxStreamBufs sets are in use (pool->mu held)
int find_bufs(csv_pool *pool, hipStream_t s, LaunchBufs **out) {
    LaunchBufs *b = nullptr;
    for (auto &e : pool->bufs)
        if (e.stream == s) b = &e;
    if (!b) {
        if (pool->bufs.size() < kMaxStreamBufs) {
            pool->bufs.emplace_back();
            b = &pool->bufs.back();
        } else {
            if (capturing(s)) return CSV_EBUSY;
            if (hipDeviceSynchronize() != hipSuccess) return CSV_EHIP;
            b = &pool->bufs[0];
            for (auto &e : pool->bufs)
                if (e.last_use < b->last_use) b = &e;
        }
        b->stream = s;
    }
    b->last_use = ++pool->use_clock;
    *out = b;
    return CSV_OK;
}

// ... with `bytes` of scratch for the generic decoder (pool->mu held)
int generic_bufs(csv_pool *pool, hipStream_t s, uint64_t bytes, LaunchBufs **out) {
    LaunchBufs *b = nullptr;
    int rc = find_bufs(pool, s, &b);
    if (rc) return rc;
    if (b->gen_bytes < bytes) {
        if (capturing(s)) return CSV_EBUSY;
        if (b->gen && hipStreamSynchronize(s) != hipSuccess) return CSV_EHIP;
        if (over_budget(pool, bytes - b->gen_bytes)) return CSV_ENOMEM;
        (void)hipFree(b->gen);
        b->gen = nullptr;
        b->gen_bytes = 0;
        if (hipMalloc(reinterpret_cast<void **>(&b->gen), bytes) != hipSuccess) return CSV_ENOMEM;
        b->gen_bytes = bytes;
    }
    *out = b;
    return CSV_OK;
}

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
    if (!b->slots || n > b->cap_n || dw != b->slot_dw) {
        if (cap) return CSV_EBUSY;  // buffers cannot be re-sized inside a capture
        if (b->slots && hipStreamSynchronize(s) != hipSuccess) return CSV_EHIP;
        const uint64_t now = b->slots ? LaunchBufs::sized(b->cap_n, b->slot_dw) : 0;
        const uint64_t want = LaunchBufs::sized(std::max(n, 1024u), dw);
        if (want > now && over_budget(pool, want - now)) return CSV_ENOMEM;
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
        (void)set_lds_attr(front_kernel<WPG, true>);
        (void)set_lds_attr(front_kernel<WPG, false>);
    });
    if (l.lut_lds_words)
        hipLaunchKernelGGL((front_kernel<WPG, true>), dim3(grid), dim3(64 * WPG), lds, s, a, l);
    else
        hipLaunchKernelGGL((front_kernel<WPG, false>), dim3(grid), dim3(64 * WPG), lds, s, a, l);
}

void launch_pair(const DecodeArgs &a, const LaunchA &l, uint32_t grid, size_t lds, hipStream_t s) {
    static std::once_flag once;
    std::call_once(once, [] {
        (void)set_lds_attr(front_pair_kernel<true>);
        (void)set_lds_attr(front_pair_kernel<false>);
    });
    if (l.lut_lds_words)
        hipLaunchKernelGGL((front_pair_kernel<true>), dim3(grid), dim3(128), lds, s, a, l);
    else
        hipLaunchKernelGGL((front_pair_kernel<false>), dim3(grid), dim3(128), lds, s, a, l);
}

// waves_a: front-kernel waves per workgroup (2: the paired kernel, two
// waves per brick); groups_b: leaf workgroups
// per CU; fixed: buffers owned by the caller (a captured graph), else the
// stream's own set
// CSV_REF_LIST_CAP (a decimal count) bounds the leaf kernel's list of
// same-level references; bricks with more chase them in the output loop.
// The default is no bound beyond the LDS arena.  Read at every launch, so
// that tests can exercise both paths in one process.
uint32_t ref_list_cap() {
    const char *e = std::getenv("CSV_REF_LIST_CAP");
    if (!e || !*e) return 0xFFFFFFFFu;
    char *end = nullptr;
    const unsigned long v = std::strtoul(e, &end, 10);
    return (end && *end == 0) ? (uint32_t)std::min<unsigned long>(v, 0xFFFFFFFFul) : 0xFFFFFFFFu;
}

int launch_one(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar, const uint64_t *out_off,
               uint32_t n, uint32_t *out, void *stream, bool plain, int waves_a, uint32_t groups_b, bool queue,
               bool lpt, LaunchBufs *fixed, uint32_t *words_out, int *req_err, uint32_t rq_base = 0,
               const uint32_t *n_dev = nullptr) {
    if (!pool || (n && (!ids || !out))) return CSV_EINVAL;
    if (!lods && lod_scalar > (uint32_t)kLog2) return CSV_ERANGE;
    if (lods && !out_off) return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    if (pool->rec_ptr.empty() || !pool->d_err) return CSV_EINVAL;
    if (waves_a != 2 && waves_a != 4 && waves_a != 8 && waves_a != 16) return CSV_EINVAL;
    if (groups_b < 1 || groups_b > kMaxGroupsB) return CSV_EINVAL;
    // the paired kernel takes no work counter and has no prefix pass
    if (waves_a == 2 && words_out) waves_a = 4;
    if (waves_a == 2) queue = false;
    DeviceGuard g(pool->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    static std::once_flag once_b;
    static hipError_t attr_b = hipSuccess;
    std::call_once(once_b, [] { attr_b = set_lds_attr(leaf_kernel<kWavesLeaf, false>); });
    if (attr_b != hipSuccess) return CSV_EHIP;
    std::lock_guard<std::mutex> lk(pool->mu);
    if (pool->generic) {
        // other brick sizes and raw nibbles: the generic decoder, one
        // workgroup per brick (no launch shape, no fixed buffers)
        if (fixed || words_out || n_dev) return CSV_EINVAL;
        // 8 workgroups per CU (few registers and 112 bytes of LDS each), 4 for
        // 64^3 bricks (1.9 MB of scratch per workgroup)
        const uint32_t cu = (uint32_t)std::max(1, pool->n_cu);
        const uint32_t groups = plain ? 1u : std::min(n, (pool->brick_log2 >= 6 ? 4u : 8u) * cu);
        csv::GenericArgs ga{};
        ga.sym_cap = pool->max_c0 + 16;
        ga.scratch_per_group = csv::generic_scratch_bytes(pool->brick_log2, ga.sym_cap);
        LaunchBufs *G = nullptr;
        const int rc = generic_bufs(pool, s, ga.scratch_per_group * groups, &G);
        if (rc) return rc;
        ga.rec_ptr = pool->d_rec_ptr;
        ga.rec_size = pool->d_rec_size;
        ga.rec_vol = pool->d_rec_vol;
        ga.luts = pool->d_luts;
        ga.lut_off = pool->d_lut_off;
        // the tables in LDS when 8 workgroups per CU still fit
        ga.lut_lds_words = 4 * pool->luts.size() <= 16 * 1024 ? (uint32_t)pool->luts.size() : 0u;
        ga.vol_bits = pool->d_bits;
        ga.vol_raw = pool->d_vol_raw;
        ga.n_bricks = (uint32_t)pool->rec_ptr.size();
        ga.log2 = pool->brick_log2;
        ga.ids = ids;
        ga.lods = lods;
        ga.lod_scalar = lod_scalar;
        ga.out_off = out_off;
        ga.out = reinterpret_cast<uint64_t>(out);
        ga.n = n;
        ga.err = pool->d_err;
        ga.req_err = req_err;
        ga.rq_base = rq_base;
        ga.scratch = reinterpret_cast<uint64_t>(G->gen);
        if (!plain) return csv::generic_launch(ga, groups, s) == hipSuccess ? CSV_OK : CSV_EHIP;
        // one launch per brick
        const uint64_t g1 = (1u << pool->brick_log2) >> (lods ? 0u : lod_scalar);
        for (uint32_t i = 0; i < n; i++) {
            csv::GenericArgs gi = ga;
            gi.ids = ids + i;
            gi.lods = lods ? lods + i : nullptr;
            gi.out_off = out_off ? out_off + i : nullptr;
            gi.out = reinterpret_cast<uint64_t>(out_off ? out : out + (uint64_t)i * g1 * g1 * g1);
            gi.n = 1;
            gi.req_err = req_err ? req_err + i : nullptr;
            gi.rq_base = rq_base + i;
            if (csv::generic_launch(gi, 1, s) != hipSuccess) return CSV_EHIP;
        }
        return CSV_OK;
    }
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
    a.n_dev = n_dev;
    a.err = pool->d_err;
    a.pfx_dw = pool->any_split ? pool->d_pfx_dw : nullptr;
    a.sfx = pool->any_split ? pool->d_sfx : nullptr;
    a.req_err = req_err;
    a.rq_base = rq_base;
    const uint32_t cu = (uint32_t)std::max(1, pool->n_cu);
    // the global-arena variant runs only for pools with bricks that may not fit the LDS arena;
    // its arenas belong to this buffer set, so launches on other streams never share them
    const bool slow = pool->any_big_palette || pool->max_fast_bytes > arena_b(groups_b);
    // buffers the library allocates get one arena per global-arena workgroup; a view of
    // memory it does not allocate brings its own, fewer ones
    const uint32_t grid_g = std::min(B->owned ? slow_groups(cu) : B->arena_groups, n);
    if (slow && (!B->arenas || B->arena_groups < grid_g)) {
        if (!B->owned || capturing(s)) return CSV_EBUSY;  // fixed buffers cannot grow
        if (over_budget(pool, (uint64_t)slow_groups(cu) * kArenaBytes)) return CSV_ENOMEM;
        const int rc = B->reserve_arenas(slow_groups(cu));
        if (rc) return rc;
    }
    // counters: 0 front queue, 1 leaf queue, 2 leaf count, 3 slow count,
    // 4 slow queue, 5 and 6 finished leaf / slow workgroups.  They are zero
    // when a launch starts: zeroed at allocation, then by the last
    // workgroup of the leaf kernels (0, 1, 2, 5) and of the global-arena
    // kernel (3, 4, 6), which only runs when the leaf kernel may defer to it.
    uint32_t *ctr = B->small + kOrderWords;
    if (B->dirty) {  // new buffers, or a launch failed part way: start from zero (a kernel, in stream order)
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, s, B->small, kSmallWords);
        B->dirty = false;
    }
    LaunchA la;
    la.lut_lds_words = lut_lds_words(pool);
    la.queue = queue ? ctr : nullptr;
    la.order = nullptr;
    la.slots = B->slots;
    la.slot_bytes = B->slot_bytes();
    la.slot_dw = B->slot_dw;
    la.leaf_list = B->leaf_list;
    la.leaf_count = ctr + 2;
    la.base = 0;
    la.words_out = words_out;
    LaunchB lb;
    lb.arena_bytes = arena_b(groups_b);
    lb.queue = ctr + 1;  // the leaf kernel always takes its bricks from a counter
    lb.leaf_list = B->leaf_list;
    lb.leaf_count = ctr + 2;
    lb.slow_count = ctr + 3;
    lb.slow_queue = ctr + 4;
    lb.slots = B->slots;
    lb.slot_bytes = B->slot_bytes();
    lb.slot_dw = B->slot_dw;
    lb.scratch = slow ? B->arenas : nullptr;
    lb.scratch_bytes = kArenaBytes;
    lb.ref_cap = ref_list_cap();
    lb.ctr = ctr;
    const size_t lds_b = kSmallB + (size_t)lb.arena_bytes;
    const size_t lds_g = kSmallB;
    lb.slow_list = slow ? B->slow_list : nullptr;
    // a small batch takes smaller front workgroups, so that its bricks spread over the CUs
    while (waves_a > 4 && (n + (uint32_t)waves_a - 1) / (uint32_t)waves_a < cu) waves_a /= 2;
    // front kernel: as many workgroups as a CU's LDS and 32 wave slots allow;
    // bricks_a of them in flight at once (one per wave, or one per paired workgroup)
    const uint32_t per_wg = waves_a == 2 ? 1u : (uint32_t)waves_a;
    const uint32_t lds_a = align16(4 * la.lut_lds_words) +
                           (waves_a == 2 ? kPairDecLds + kWaveLds : (uint32_t)waves_a * kWaveLds);
    const uint32_t fit_a = std::max(1u, std::min(kLdsBytes / lds_a, 32u / (uint32_t)waves_a));
    const uint32_t grid_a = std::max(1u, std::min(cu * fit_a, (n + per_wg - 1) / per_wg));
    const uint32_t bricks_a = grid_a * per_wg;
    const uint32_t grid_b = std::min(cu * groups_b, n);
    auto go_a = [&](const DecodeArgs &aa, const LaunchA &L, uint32_t grid) {
        switch (waves_a) {
            case 2: launch_pair(aa, L, grid, lds_a, s); break;
            case 4: launch_a<4>(aa, L, grid, lds_a, s); break;
            case 8: launch_a<8>(aa, L, grid, lds_a, s); break;
            default: launch_a<16>(aa, L, grid, lds_a, s); break;
        }
    };
    if (plain) {
        // per brick: counter reset, front kernel (one wave), leaf kernel (one workgroup)
        DecodeArgs b = a;
        for (uint32_t i = 0; i < n; i++) {
            la.base = i;
            b.n = i + 1;
            go_a(b, la, 1);
            hipLaunchKernelGGL((leaf_kernel<kWavesLeaf, false>), dim3(1), dim3(64 * kWavesLeaf), lds_b, s, b, lb);
            if (slow) hipLaunchKernelGGL((leaf_kernel<kWavesLeafG, true>), dim3(1), dim3(64 * kWavesLeafG), lds_g, s, b, lb);
        }
    } else {
        // with at most one request per front wave the order changes nothing;
        // with a device-side count the order kernels would not know it
        if (lpt && !n_dev && n > bricks_a) {
            const uint32_t grid_o = std::min(256u, (n + 255) / 256);
            hipLaunchKernelGGL(order_count, dim3(grid_o), dim3(256), 0, s, a, B->small);
            hipLaunchKernelGGL(order_place, dim3(grid_o), dim3(256), 0, s, a, B->small, B->order, bricks_a);
            la.order = B->order;
        }
        go_a(a, la, grid_a);
        hipLaunchKernelGGL((leaf_kernel<kWavesLeaf, false>), dim3(grid_b), dim3(64 * kWavesLeaf), lds_b, s, a, lb);
        if (slow) {
            hipLaunchKernelGGL((leaf_kernel<kWavesLeafG, true>), dim3(grid_g), dim3(64 * kWavesLeafG), lds_g, s, a, lb);
        }
    }
    if (hipGetLastError() != hipSuccess) {
        B->dirty = true;
        return CSV_EHIP;
    }
    return CSV_OK;
}

// Requests per chunk below which a decode is not split (a chunk should
// still fill the machine for a while).
constexpr uint32_t kMinChunk = 2048;
constexpr size_t kMaxCompanions = kMaxStreamBufs / 2;

// The companion stream of caller stream s, created on first use (nullptr
// when the pool already serves kMaxCompanions callers).  pool->mu held.
csv_pool::Companion *companion(csv_pool *pool, hipStream_t s) {
    for (auto &c : pool->companions)
        if (c.caller == s) return &c;
    if (pool->companions.size() >= kMaxCompanions) return nullptr;
    pool->companions.reserve(kMaxCompanions);
    csv_pool::Companion c;
    c.caller = s;
    if (hipStreamCreateWithFlags(&c.own, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&c.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c.join, hipEventDisableTiming) != hipSuccess) {
        if (c.fork) (void)hipEventDestroy(c.fork);
        (void)hipStreamDestroy(c.own);
        return nullptr;
    }
    pool->companions.push_back(c);
    return &pool->companions.back();
}

// A decode of n requests.  With chunks > 1 the requests are split into that
// many consecutive chunks that alternate between the caller's stream and
// its companion stream: the entropy decode of one chunk overlaps the leaf
// level of the previous one.  The companion waits for the caller's stream
// before its first chunk, and the caller's stream waits for the companion
// after its last, so the call stays ordered on `stream` as one operation.
// Fixed buffers (graphs), prefix passes, per-brick launches, stream
// captures and small batches run as one launch pair.
int launch(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar, const uint64_t *out_off,
           uint32_t n, uint32_t *out, void *stream, bool plain, int waves_a, uint32_t groups_b, bool queue,
           bool lpt, LaunchBufs *fixed = nullptr, uint32_t *words_out = nullptr, int *req_err = nullptr,
           uint32_t chunks = 1) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    chunks = std::min(chunks, n / kMinChunk);
    if (pool && pool->generic) chunks = 1;  // the generic decoder runs as one launch
    if (chunks <= 1 || !pool || plain || fixed || words_out || !ids || !out || (lods && !out_off) ||
        (!lods && lod_scalar > (uint32_t)kLog2) || capturing(s))
        return launch_one(pool, ids, lods, lod_scalar, out_off, n, out, stream, plain, waves_a, groups_b, queue,
                          lpt, fixed, words_out, req_err);
    csv_pool::Companion *c = nullptr;
    {
        std::lock_guard<std::mutex> lk(pool->mu);
        DeviceGuard g(pool->device);
        c = companion(pool, s);
    }
    if (!c)
        return launch_one(pool, ids, lods, lod_scalar, out_off, n, out, stream, plain, waves_a, groups_b, queue,
                          lpt, fixed, words_out, req_err);
    DeviceGuard g(pool->device);
    if (hipEventRecord(c->fork, s) != hipSuccess || hipStreamWaitEvent(c->own, c->fork, 0) != hipSuccess)
        return CSV_EHIP;
    const uint32_t per = (n + chunks - 1) / chunks;
    const uint64_t G = 32u >> (lods ? 0u : lod_scalar);
    const uint64_t cnt = lods ? 0 : G * G * G;
    int rc = CSV_OK;
    for (uint32_t k = 0, at = 0; at < n && rc == CSV_OK; k++, at += per) {
        const uint32_t m = std::min(per, n - at);
        rc = launch_one(pool, ids + at, lods ? lods + at : nullptr, lod_scalar, out_off ? out_off + at : nullptr, m,
                        out_off ? out : out + (uint64_t)at * cnt, (k & 1) ? (void *)c->own : stream, false, waves_a,
                        groups_b, queue, lpt, nullptr, nullptr, req_err ? req_err + at : nullptr, at);
    }
    // joined back in every case, so that nothing of the call runs unordered
    if (hipEventRecord(c->join, c->own) != hipSuccess || hipStreamWaitEvent(s, c->join, 0) != hipSuccess)
        rc = rc ? rc : CSV_EHIP;
    return rc;
}

// Class of a request set, the key of the tuned shapes: bits 0..7 the bit
// length of n, bits 8..15 how its levels of detail are given (0: all full
// LOD, 1: all one coarser LOD, 2: per request), bits 16..23 the bit length
// of the pool's mean record size.
uint32_t tune_key(const csv_pool *p, const uint8_t *lods, uint32_t lod_scalar, uint32_t n) {
    const uint32_t nb = n ? 32u - (uint32_t)__builtin_clz(n) : 0u;
    const uint32_t lc = lods ? 2u : (lod_scalar == 0 ? 0u : 1u);
    const uint64_t nr = std::max<uint64_t>(1, p->rec_ptr.size());
    const uint64_t mean = std::max<uint64_t>(1, p->record_bytes / nr);
    const uint32_t rb = 64u - (uint32_t)__builtin_clzll(mean);
    return nb | (lc << 8) | (rb << 16);
}
// The shape for a request set: the tuned one of its class, else of the
// class with the same level-of-detail kind and record size and the nearest
// n, else the pool's shape.  pool->mu held.
// Requests that the paired front kernel takes all at once: one workgroup of
// two waves per request, as many as a CU's LDS holds.
uint32_t pair_capacity(const csv_pool *p) {
    const uint32_t lds = align16(4 * lut_lds_words(p)) + kPairDecLds + kWaveLds;
    return (uint32_t)std::max(1, p->n_cu) * std::min(kLdsBytes / lds, 16u);
}

// The shape for a request set: the tuned one of its class; else, for a
// batch the paired front kernel takes all at once (there every request's
// latency is its own serial chain, which the pairing shortens) and a pool
// whose shape was not set, that of the nearest tuned class with the front
// kernel paired; else the tuned one of the class with the same
// level-of-detail kind and record size and the nearest n; else the pool's
// shape.  pool->mu held.
csv_shape shape_for(const csv_pool *p, const uint8_t *lods, uint32_t lod_scalar, uint32_t n) {
    const uint32_t key = tune_key(p, lods, lod_scalar, n);
    const auto it = p->tuned.find(key);
    if (it != p->tuned.end()) return it->second;
    const csv_shape *best = nullptr;
    uint32_t dist = 0xFFFFFFFFu;
    for (const auto &e : p->tuned)
        if ((e.first & 0xFFFF00u) == (key & 0xFFFF00u)) {
            const uint32_t a = e.first & 0xFFu, b = key & 0xFFu, d = a > b ? a - b : b - a;
            if (d < dist) {
                dist = d;
                best = &e.second;
            }
        }
    csv_shape sh = best ? *best : p->shape;
    if (!p->shape_set && n <= pair_capacity(p)) sh.waves_per_group = 2;
    return sh;
}

bool valid_shape(const csv_shape &sh) {
    return (sh.waves_per_group == 2 || sh.waves_per_group == 4 || sh.waves_per_group == 8 ||
            sh.waves_per_group == 16) &&
           sh.groups_per_cu >= 1 && sh.groups_per_cu <= kMaxGroupsB && sh.chunks >= 1 && sh.chunks <= 64;
}

}  // namespace

extern "C" {

int csv_pool_create(csv_pool **pool, int device) { return csv_pool_create_budget(pool, device, 0); }

int csv_pool_create_budget(csv_pool **pool, int device, uint64_t hbm_budget_bytes) {
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
    std::snprintf(p->device_name, sizeof(p->device_name), "%s", prop.gcnArchName);
    for (char *c = p->device_name; *c; c++)
        if (*c == ' ' || *c == '\t' || *c == '\n') *c = '_';
    p->hbm_budget = hbm_budget_bytes;
    uint8_t *scr = nullptr;  // set-up of this device's scratch address
    if (scratch_address(device, &scr) != CSV_OK) {
        delete p;
        return CSV_EHIP;
    }
    if (hipMalloc(reinterpret_cast<void **>(&p->d_err), 2 * sizeof(int)) != hipSuccess ||
        hipMemset(p->d_err, 0, 2 * sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
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
    (void)hipFree(p->d_vol_raw);
    (void)hipFree(p->d_err);
    (void)hipFree(p->d_pfx_dw);
    (void)hipFree(p->d_sfx);
    (void)hipFree(p->d_stage);
    (void)hipHostFree(p->h_sfx);
    (void)hipHostFree(p->h_stage);
    for (void *b : p->host_bufs) (void)hipHostFree(b);
    if (p->stage_ev) (void)hipEventDestroy(p->stage_ev);
    for (auto &b : p->bufs) b.release();
    for (auto &c : p->companions) {
        (void)hipEventDestroy(c.fork);
        (void)hipEventDestroy(c.join);
        (void)hipStreamDestroy(c.own);
    }
    delete p;
}

int csv_pool_add_volume(csv_pool *p, const uint8_t *blob, size_t blob_bytes, uint32_t *first_brick_id) {
    if (!p || !blob) return CSV_EINVAL;
    csv_volume_info info;
    int rc = csv_blob_info(blob, blob_bytes, &info);
    if (rc) return rc;
    if (info.scale_bits > (uint32_t)kLutMaxBits || info.coding > 1) return CSV_EINVAL;
    // one brick size per pool; other sizes and raw nibbles take the generic decoder
    if (p->brick_log2 && info.brick_log2 != p->brick_log2) return CSV_EINVAL;
    const bool gen = info.brick_log2 != (uint32_t)kLog2 || info.coding != 0;
    if (gen && p->any_split) return CSV_EINVAL;  // detail separation needs the 32^3 rANS path
    // every record is checked on the host before anything reaches the device
    if ((rc = csv_blob_check(blob, blob_bytes, nullptr))) return rc;
    if ((uint64_t)p->rec_ptr.size() + info.n_bricks >= (1ull << 32) || p->bits.size() >= 65535) return CSV_ERANGE;
    std::lock_guard<std::mutex> lk(p->mu);
    DeviceGuard g(p->device);
    const uint64_t rs = csv::record_area_offset(info.n_bricks);
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + csv::kHeaderBytes);
    uint32_t max_fast = p->max_fast_bytes, max_c0 = p->max_c0;
    bool big = p->any_big_palette;
    for (uint32_t i = 0; i < info.n_bricks; i++) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(blob + rs + index[i]);
        const uint32_t P = w[0], c0 = w[3];
        if (c0 == 0) continue;
        max_c0 = std::max(max_c0, c0);
        if (info.brick_log2 != (uint32_t)kLog2) continue;
        const uint32_t c1 = w[4];
        big |= P > kPalFast;
        const uint32_t e1 = std::min((c0 - c1) / 8, 4096u);
        // a brick whose staged nibbles do not fit reads them from its slot
        max_fast = std::max(max_fast, make_layout_l(true, P, 0, e1, 1).total);
    }
    // the kernels run to the end of a record; 64 bytes of slack cover their last vector loads
    void *buf = nullptr;
    const size_t rb = std::max<uint64_t>(info.record_bytes, 4) + 64;
    if (over_budget(p, rb + 14ull * info.n_bricks + 4ull * 2 * (1u << info.scale_bits))) return CSV_ENOMEM;
    if (hipMalloc(&buf, rb) != hipSuccess) return CSV_ENOMEM;
    if (hipMemcpy(buf, blob + rs, info.record_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        return CSV_EHIP;
    }
    // all work that may read the tables about to move must be done
    (void)hipDeviceSynchronize();
    p->max_c0 = max_c0;
    p->max_fast_bytes = max_fast;
    p->any_big_palette = big;
    p->brick_log2 = info.brick_log2;
    p->generic = p->generic || gen;
    p->vol_raw.push_back((uint8_t)info.coding);
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
        (rc = upload(&p->d_lut_off, p->lut_off)) || (rc = upload(&p->d_bits, p->bits)) ||
        (rc = upload(&p->d_vol_raw, p->vol_raw)) || (rc = sync_split(p)))
        return rc;
    if (first_brick_id) *first_brick_id = first;
    return CSV_OK;
}

int csv_pool_add_volume_ex(csv_pool *p, const uint8_t *blob, size_t blob_bytes, uint32_t flags,
                           uint32_t *first_brick_id) {
    if (!p || !blob || (flags & ~(uint32_t)CSV_DETAIL_HOST)) return CSV_EINVAL;
    if (flags & CSV_DETAIL_HOST) {  // detail separation: 32^3 rANS pools only
        csv_volume_info vi;
        const int r = csv_blob_info(blob, blob_bytes, &vi);
        if (r) return r;
        if (p->generic || vi.brick_log2 != (uint32_t)kLog2 || vi.coding != 0) return CSV_EINVAL;
    }
    uint32_t first = 0;
    int rc = csv_pool_add_volume(p, blob, blob_bytes, &first);
    if (rc) return rc;
    if (first_brick_id) *first_brick_id = first;
    if (!(flags & CSV_DETAIL_HOST)) return CSV_OK;
    csv_volume_info info;
    if ((rc = csv_blob_info(blob, blob_bytes, &info))) return rc;
    const uint32_t nb = info.n_bricks;
    if (nb == 0) return CSV_OK;
    DeviceGuard g(p->device);
    // Sec. 4.2: levels >= 1 read a prefix of a brick's word stream; a decode
    // of every brick to level 1 counts the words of that prefix
    std::vector<uint32_t> ids(nb), words(nb, 0xFFFFFFFFu);
    for (uint32_t i = 0; i < nb; i++) ids[i] = first + i;
    uint32_t *d_ids = nullptr, *d_words = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d_ids), 4ull * nb) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&d_words), 4ull * nb) != hipSuccess) {
        (void)hipFree(d_ids);
        return CSV_ENOMEM;
    }
    rc = hipMemcpy(d_ids, ids.data(), 4ull * nb, hipMemcpyHostToDevice) == hipSuccess ? CSV_OK : CSV_EHIP;
    if (!rc)
        rc = launch(p, d_ids, nullptr, 1, nullptr, nb, d_words /* not written in this mode */, nullptr, false, 16,
                    p->shape.groups_per_cu, false, false, nullptr, d_words);
    if (!rc && (hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(words.data(), d_words, 4ull * nb, hipMemcpyDeviceToHost) != hipSuccess))
        rc = CSV_EHIP;
    (void)hipFree(d_ids);
    (void)hipFree(d_words);
    if (rc) return rc;
    // bricks whose pass failed keep their whole record (the error stays in the pool's error word);
    // device records up to the end of that prefix (whole dwords); the rest in pinned host memory
    const uint64_t rs = csv::record_area_offset(nb);
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + csv::kHeaderBytes);
    const uint32_t hdr = csv::record_header_words(kLog2);
    std::vector<uint64_t> keep(nb), det(nb);
    std::vector<uint32_t> pfx(nb, 0xFFFFFFFFu);
    uint64_t dev_total = 0, host_total = 0;
    for (uint32_t i = 0; i < nb; i++) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(blob + rs + index[i]);
        const uint32_t P = w[0], W = w[1], nw = w[2], ndw = (nw + 1) / 2;
        keep[i] = index[i + 1] - index[i];
        det[i] = 0;
        // (a brick whose level-1 prefix is all its words keeps its whole record)
        if (words[i] != 0xFFFFFFFFu && words[i] <= nw && (words[i] + 1) / 2 < ndw) {
            pfx[i] = std::min((words[i] + 1) / 2, ndw);
            keep[i] = 4ull * (hdr + P + W + pfx[i]);
            det[i] = 4ull * (ndw - pfx[i]);
        }
        dev_total += keep[i];
        host_total += det[i];
    }
    std::vector<uint8_t> img(dev_total);
    uint8_t *hbuf = nullptr;
    if (host_total && hipHostMalloc(reinterpret_cast<void **>(&hbuf), host_total, hipHostMallocDefault) != hipSuccess)
        return CSV_ENOMEM;
    std::vector<uint64_t> off(nb), hoff(nb);
    uint64_t o = 0, ho = 0;
    for (uint32_t i = 0; i < nb; i++) {
        const uint8_t *r = blob + rs + index[i];
        std::memcpy(img.data() + o, r, keep[i]);
        off[i] = o;
        o += keep[i];
        if (det[i]) std::memcpy(hbuf + ho, r + keep[i], det[i]);  // the words after the kept prefix
        hoff[i] = ho;
        ho += det[i];
    }
    void *dbuf = nullptr;
    if (hipMalloc(&dbuf, dev_total + 64) != hipSuccess) {
        (void)hipHostFree(hbuf);
        return CSV_ENOMEM;
    }
    if (hipMemcpy(dbuf, img.data(), dev_total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dbuf);
        (void)hipHostFree(hbuf);
        return CSV_EHIP;
    }
    std::lock_guard<std::mutex> lk(p->mu);
    (void)hipDeviceSynchronize();  // nothing may still read the full records
    const uint64_t old_base = p->rec_ptr[first] - index[0];
    for (size_t v = 0; v < p->vol_bufs.size(); v++)
        if (reinterpret_cast<uint64_t>(p->vol_bufs[v]) == old_base) {
            (void)hipFree(p->vol_bufs[v]);
            p->vol_bufs[v] = dbuf;
        }
    p->record_bytes = p->record_bytes - info.record_bytes + dev_total;
    p->any_split = true;
    p->pfx_dw.resize(p->rec_ptr.size(), 0xFFFFFFFFu);
    p->det_host.resize(p->rec_ptr.size(), nullptr);
    p->det_bytes.resize(p->rec_ptr.size(), 0u);
    for (uint32_t i = 0; i < nb; i++) {
        p->rec_ptr[first + i] = reinterpret_cast<uint64_t>(dbuf) + off[i];
        p->rec_size[first + i] = (uint32_t)keep[i];
        p->pfx_dw[first + i] = pfx[i];
        p->det_host[first + i] = det[i] ? hbuf + hoff[i] : nullptr;
        p->det_bytes[first + i] = (uint32_t)det[i];
    }
    if (hbuf) p->host_bufs.push_back(hbuf);
    p->host_bytes += host_total;
    p->generation++;
    if ((rc = upload(&p->d_rec_ptr, p->rec_ptr)) || (rc = upload(&p->d_rec_size, p->rec_size)) ||
        (rc = sync_split(p)))
        return rc;
    return CSV_OK;
}

int csv_pool_set_detail_staging(csv_pool *p, uint64_t bytes) {
    if (!p || bytes < 4096 || bytes > (1ull << 36)) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->stage_used) return CSV_EBUSY;  // release the staged detail first
    DeviceGuard g(p->device);
    if (p->stage_ev) (void)hipEventSynchronize(p->stage_ev);
    if (p->stage_alloc != bytes) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->d_stage);
        (void)hipHostFree(p->h_stage);
        p->d_stage = p->h_stage = nullptr;
        p->stage_alloc = 0;
    }
    p->stage_cap = bytes;
    return CSV_OK;
}

int csv_pool_stage_detail(csv_pool *p, const uint32_t *ids, uint32_t n, void *stream, uint32_t *n_done) {
    if (!p || (n && !ids) || !n_done) return CSV_EINVAL;
    *n_done = 0;
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->any_split) {
        *n_done = n;
        return CSV_OK;
    }
    DeviceGuard g(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!p->d_stage) {
        if (hipMalloc(reinterpret_cast<void **>(&p->d_stage), p->stage_cap) != hipSuccess) return CSV_ENOMEM;
        if (hipHostMalloc(reinterpret_cast<void **>(&p->h_stage), p->stage_cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(p->d_stage);
            p->d_stage = nullptr;
            return CSV_ENOMEM;
        }
        p->stage_alloc = p->stage_cap;
    }
    if (!p->stage_ev && hipEventCreateWithFlags(&p->stage_ev, hipEventDisableTiming) != hipSuccess) return CSV_EHIP;
    (void)hipEventSynchronize(p->stage_ev);  // the host images are not read by earlier copies any more
    const uint64_t start = p->stage_used;
    const uint32_t nb = (uint32_t)p->rec_ptr.size();
    uint32_t i = 0;
    for (; i < n; i++) {
        const uint32_t id = ids[i];
        if (id >= nb) break;
        if (p->pfx_dw[id] == 0xFFFFFFFFu || p->staged[id] || !p->det_bytes[id]) continue;
        const uint64_t b = p->det_bytes[id], b16 = (b + 15) & ~15ull;
        if (p->stage_used + b16 > p->stage_alloc) break;
        std::memcpy(p->h_stage + p->stage_used, p->det_host[id], b);
        p->h_sfx[id] = reinterpret_cast<uint64_t>(p->d_stage) + p->stage_used;
        p->staged[id] = 1;
        p->stage_used += b16;
    }
    const bool bad_id = i < n && ids[i] >= nb;
    *n_done = i;
    if (p->stage_used > start) {
        if (hipMemcpyAsync(p->d_stage + start, p->h_stage + start, p->stage_used - start, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(p->d_sfx, p->h_sfx, 8ull * p->n_sfx, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(p->stage_ev, s) != hipSuccess)
            return CSV_EHIP;
    }
    // work on this stream sees the detail staged by earlier calls on any stream
    if (hipStreamWaitEvent(s, p->stage_ev, 0) != hipSuccess) return CSV_EHIP;
    return bad_id ? CSV_ERANGE : CSV_OK;
}

int csv_pool_detail_bytes(const csv_pool *p, uint32_t id, uint32_t *bytes, uint64_t *staging_bytes) {
    if (!p || (!bytes && !staging_bytes)) return CSV_EINVAL;
    if (staging_bytes) *staging_bytes = p->stage_cap;
    if (!bytes) return CSV_OK;
    if (id >= p->rec_ptr.size()) return CSV_ERANGE;
    // the bytes it takes in the staging buffer (16-byte granules)
    *bytes = id < p->det_bytes.size() ? (p->det_bytes[id] + 15u) & ~15u : 0u;
    return CSV_OK;
}

int csv_pool_release_detail(csv_pool *p, void *stream) {
    if (!p) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->any_split || !p->stage_used) return CSV_OK;
    DeviceGuard g(p->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    (void)hipEventSynchronize(p->stage_ev);
    for (size_t id = 0; id < p->staged.size(); id++)
        if (p->staged[id]) {
            p->staged[id] = 0;
            p->h_sfx[id] = 0;
        }
    p->stage_used = 0;
    if (hipMemcpyAsync(p->d_sfx, p->h_sfx, 8ull * p->n_sfx, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(p->stage_ev, s) != hipSuccess)
        return CSV_EHIP;
    return CSV_OK;
}

int csv_pool_info_get(const csv_pool *p, csv_pool_info *info) {
    if (!p || !info) return CSV_EINVAL;
    info->n_volumes = (uint32_t)p->bits.size();
    info->n_bricks = (uint32_t)p->rec_ptr.size();
    info->device = p->device;
    info->brick_log2 = p->brick_log2;
    info->device_bytes = pool_device_bytes(p);
    info->host_bytes = p->host_bytes;
    return CSV_OK;
}

int csv_output_elems_log2(uint32_t brick_log2, const uint8_t *lods_host, uint32_t n, uint64_t *offsets,
                          uint64_t *total) {
    if ((n && !lods_host) || !total || brick_log2 < 1 || brick_log2 > (uint32_t)csv::kMaxLog2) return CSV_EINVAL;
    uint64_t o = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (lods_host[i] > brick_log2) return CSV_ERANGE;
        if (offsets) offsets[i] = o;
        const uint64_t g = (1u << brick_log2) >> lods_host[i];
        o += g * g * g;
    }
    *total = o;
    return CSV_OK;
}

int csv_output_elems(const uint8_t *lods_host, uint32_t n, uint64_t *offsets, uint64_t *total) {
    return csv_output_elems_log2((uint32_t)kLog2, lods_host, n, offsets, total);
}

int csv_output_bytes(const uint8_t *lods_host, uint32_t n, uint64_t *offsets, uint64_t *total) {
    const int rc = csv_output_elems(lods_host, n, offsets, total);
    if (rc) return rc;
    for (uint32_t i = 0; offsets && i < n; i++) offsets[i] *= 4;
    *total *= 4;
    return CSV_OK;
}

// the launch shape a decode of these requests uses
csv_shape current_shape(const csv_pool *pool, const uint8_t *lods, uint32_t lod_scalar, uint32_t n) {
    csv_pool *p = const_cast<csv_pool *>(pool);
    std::lock_guard<std::mutex> lk(p->mu);
    return shape_for(p, lods, lod_scalar, n);
}

int csv_decode_bricks_status(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                             const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, int32_t *status) {
    if (!pool || (n && !status)) return CSV_EINVAL;
    const csv_shape sh = current_shape(pool, lods, lod_scalar, n);
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, false,
                  sh.waves_per_group, (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0, nullptr,
                  nullptr, status, sh.chunks);
}

int csv_decode_bricks(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                      const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    if (!pool) return CSV_EINVAL;
    const csv_shape sh = current_shape(pool, lods, lod_scalar, n);
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, false,
                  sh.waves_per_group, (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0, nullptr,
                  nullptr, nullptr, sh.chunks);
}

int csv_decode_bricks_devcount(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                               const uint64_t *out_off, uint32_t n_max, const uint32_t *n_dev, uint32_t *out,
                               void *stream) {
    if (!pool || !n_dev) return CSV_EINVAL;
    const csv_shape sh = current_shape(pool, lods, lod_scalar, n_max);
    return launch_one(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n_max, out, stream, false,
                      sh.waves_per_group, (uint32_t)sh.groups_per_cu, sh.use_queue != 0, false, nullptr, nullptr,
                      nullptr, 0, n_dev);
}

int csv_decode_bricks_noalloc(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                              const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    if (!pool || (n && (!ids || !out))) return CSV_EINVAL;
    if (!lods && lod_scalar > (uint32_t)kLog2) return CSV_ERANGE;
    if (lods && !out_off) return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    csv_pool *p = const_cast<csv_pool *>(pool);
    uint8_t *base = nullptr;
    int rc = scratch_address(p->device, &base);
    if (rc) return rc;
    LaunchBufs v;
    v.owned = false;
    v.stream = reinterpret_cast<hipStream_t>(stream);
    csv_shape sh;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        if (p->rec_ptr.empty() || !p->d_err || p->generic) return CSV_EINVAL;
        v.slot_dw = slot_dw(p);
        sh = shape_for(p, lods, lod_scalar, n);
    }
    // requests per launch pair: after the counters and arenas, 4 bytes of
    // order list and two 48-byte leaf descriptors plus one slot each (the
    // descriptors 16-byte, the slots 256-byte aligned: 512 bytes of slack)
    const uint64_t per = (uint64_t)v.slot_bytes() + 4 + 2 * sizeof(LeafDesc);
    const uint64_t fit = (kNoAllocBytes - kNoAllocHead - 512) / per;
    if (fit == 0) return CSV_ERANGE;  // one request's slot exceeds the scratch
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(fit, n);
    v.small = reinterpret_cast<uint32_t *>(base);
    v.arenas = base + kNoAllocSmall;
    v.arena_groups = kNoAllocArenas;
    v.order = reinterpret_cast<uint32_t *>(base + kNoAllocHead);
    v.leaf_list = reinterpret_cast<LeafDesc *>(base + kNoAllocHead + ((4ull * chunk + 15) & ~15ull));
    v.slow_list = v.leaf_list + chunk;
    const size_t lists_end = kNoAllocHead + ((4ull * chunk + 15) & ~15ull) + 2 * sizeof(LeafDesc) * chunk;
    v.slots = base + ((lists_end + 255) & ~(size_t)255);
    v.cap_n = chunk;
    // the previous call's counters and order bins may be left non-zero (a
    // failed launch): clear them with a kernel, in stream order
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, v.stream, v.small, kSmallWords);
    if (hipGetLastError() != hipSuccess) return CSV_EHIP;
    const uint64_t g = 32u >> lod_scalar;
    for (uint32_t at = 0; at < n; at += chunk) {
        const uint32_t m = std::min(chunk, n - at);
        uint32_t *o = out_off ? out : out + (uint64_t)at * g * g * g;
        rc = launch_one(p, ids + at, lods ? lods + at : nullptr, lod_scalar, out_off ? out_off + at : nullptr, m, o,
                        stream, false, sh.waves_per_group, (uint32_t)sh.groups_per_cu, sh.use_queue != 0,
                        sh.lpt_order != 0, &v, nullptr, nullptr, at);
        if (rc) return rc;
    }
    return CSV_OK;
}

int csv_bricks_visible(const csv_pool *pool, const uint32_t *ids, uint32_t n, const uint32_t *visible_bits,
                       uint32_t n_label_bits, uint8_t *visible, void *stream) {
    if (!pool) return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    if (!ids || !visible || (n_label_bits && !visible_bits)) return CSV_EINVAL;
    csv_pool *p = const_cast<csv_pool *>(pool);
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->rec_ptr.empty() || !p->d_err) return CSV_EINVAL;
    DeviceGuard g(p->device);
    const uint32_t cu = (uint32_t)std::max(1, p->n_cu);
    const uint32_t grid = std::max(1u, std::min((n + 3) / 4, cu * 8));
    hipLaunchKernelGGL(visible_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, p->d_rec_ptr, p->d_rec_size,
                       (uint32_t)p->rec_ptr.size(), ids, n, visible_bits, n_label_bits, visible, p->d_err,
                       csv::record_header_words((int)p->brick_log2));
    return hipGetLastError() == hipSuccess ? CSV_OK : CSV_EHIP;
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
                  shape->lpt_order != 0, nullptr, nullptr, nullptr, shape->chunks);
}

int csv_pool_set_shape(csv_pool *pool, const csv_shape *shape) {
    if (!pool || !shape || !valid_shape(*shape)) return CSV_EINVAL;
    std::lock_guard<std::mutex> lk(pool->mu);
    pool->shape = *shape;
    pool->shape_set = true;
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
    if (hipEventCreate(&e0) != hipSuccess) return CSV_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CSV_EHIP;
    }
    int rc = CSV_OK;
    // time of one shape: one warm-up launch, then reps timed launches
    auto time_shape = [&](csv_shape &sh) {
        rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group,
                    (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0, nullptr, nullptr, nullptr,
                    sh.chunks);
        if (rc) return;
        (void)hipEventRecord(e0, s);
        for (uint32_t r = 0; r < reps && !rc; r++)
            rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group,
                        (uint32_t)sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0, nullptr, nullptr, nullptr,
                        sh.chunks);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess && !rc) rc = CSV_EHIP;
        float ms = 0.f;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CSV_EHIP;
        sh.ms = ms / (float)reps;
    };
    csv_shape win{};
    win.ms = 1e30f;
    auto consider = [&](csv_shape sh) {
        if (rc) return;
        time_shape(sh);
        if (!rc && sh.ms < win.ms) win = sh;
    };
    // one coordinate at a time: the two kernels' shapes with the requests
    // split in up to four chunks, then the chunk count, then the work
    // counters and the longest-first order
    const uint32_t c0 = std::max(1u, std::min(4u, n / kMinChunk));
    const int waves[3] = {2, 8, 16};
    const uint32_t groups[3] = {2, 3, 4};
    for (int wi = 0; wi < 3; wi++)
        for (int gi = 0; gi < 3; gi++) consider(csv_shape{waves[wi], groups[gi], 0, 0, c0, 0.f});
    const csv_shape base = win;
    for (uint32_t c : {1u, 2u, 4u, 8u})
        if (c != c0 && (c == 1 || c <= n / kMinChunk)) {
            csv_shape sh = base;
            sh.chunks = c;
            consider(sh);
        }
    const csv_shape base2 = win;
    for (int q = 0; q < 2; q++)
        for (int o = 0; o < 2; o++)
            if (q || o) {
                csv_shape sh = base2;
                sh.use_queue = q;
                sh.lpt_order = o;
                consider(sh);
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(pool->mu);
        pool->shape = win;
        pool->tuned[tune_key(pool, lods, lod_scalar, n)] = win;
    }
    if (best) *best = win;
    return CSV_OK;
}

int csv_pool_shape_for(const csv_pool *pool, const uint8_t *lods, uint32_t lod_scalar, uint32_t n,
                       csv_shape *shape) {
    if (!pool || !shape) return CSV_EINVAL;
    *shape = current_shape(pool, lods, lod_scalar, n);
    return CSV_OK;
}

int csv_pool_tuning_save(const csv_pool *pool, const char *path) {
    if (!pool || !path) return CSV_EINVAL;
    csv_pool *p = const_cast<csv_pool *>(pool);
    std::lock_guard<std::mutex> lk(p->mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return CSV_EINVAL;
    bool ok = std::fprintf(f, "csv-tuning 1 %s %d\n", p->device_name, p->n_cu) > 0;
    for (const auto &e : p->tuned) {
        const csv_shape &sh = e.second;
        ok = ok && std::fprintf(f, "%u %u %u %d %u %d %d %u %.4f\n", e.first & 0xFFu, (e.first >> 8) & 0xFFu,
                                (e.first >> 16) & 0xFFu, sh.waves_per_group, sh.groups_per_cu, sh.use_queue,
                                sh.lpt_order, sh.chunks, (double)sh.ms) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? CSV_OK : CSV_EINVAL;
}

int csv_pool_tuning_load(csv_pool *pool, const char *path, uint32_t *n_loaded) {
    if (!pool || !path) return CSV_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return CSV_EINVAL;
    char name[64] = {0};
    int ver = 0, cu = 0;
    std::map<uint32_t, csv_shape> got;
    int rc = CSV_OK;
    if (std::fscanf(f, "csv-tuning %d %63s %d", &ver, name, &cu) != 3 || ver != 1) {
        rc = CSV_ECORRUPT;
    } else {
        unsigned nb, lc, rb, groups, chunks;
        int waves, queue, lpt;
        double ms;
        while (std::fscanf(f, "%u %u %u %d %u %d %d %u %lf", &nb, &lc, &rb, &waves, &groups, &queue, &lpt, &chunks,
                           &ms) == 9) {
            const csv_shape sh{waves, groups, queue, lpt, chunks, (float)ms};
            if (nb > 255 || lc > 2 || rb > 255 || !valid_shape(sh)) {
                rc = CSV_ECORRUPT;
                break;
            }
            got[nb | (lc << 8) | (rb << 16)] = sh;
        }
        if (rc == CSV_OK && !std::feof(f)) rc = CSV_ECORRUPT;
    }
    std::fclose(f);
    if (rc) return rc;
    uint32_t k = 0;
    {
        std::lock_guard<std::mutex> lk(pool->mu);
        // shapes tuned on another kind of device, or another CU count, do not apply
        if (std::strcmp(name, pool->device_name) == 0 && cu == pool->n_cu)
            for (const auto &e : got) {
                pool->tuned[e.first] = e.second;
                k++;
            }
    }
    if (n_loaded) *n_loaded = k;
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
    if (!pool || !graph || !n || pool->generic) return CSV_EINVAL;
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
        if (!rc && (pool->any_big_palette || pool->max_fast_bytes > arena_b((uint32_t)sh.groups_per_cu)))
            rc = G->bufs.reserve_arenas(slow_groups((uint32_t)std::max(1, pool->n_cu)));
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
    // cleared before any later work on any stream can report into it
    if (hipMemset(p->d_err, 0, sizeof(h)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return CSV_EHIP;
    *code = h[0];
    if (brick_id) *brick_id = (uint32_t)h[1];
    return CSV_OK;
}

}  // extern "C"
