// GPU brick decoder for gfx950 and the device pool that feeds it.
//
// One wavefront decodes one brick to level of detail t (Sec. 3.4, Alg. 1);
// the waves of a workgroup work on different bricks and never wait for each
// other.  Per brick:
//   1. the palette and the word stream are staged in the wave's LDS arena;
//   2. the W interleaved rANS states (Sec. 3.3) run in lockstep, one per
//      lane; a renormalising lane takes its 16-bit word at the stream cursor
//      plus the number of lower lanes that also renormalise (wave ballot +
//      mbcnt); symbols land as packed nibbles in LDS;
//   3. levels 4..max(t,1) are replayed from those nibbles (Sec. 3.2).  A level
//      is data-parallel over the expanded parents (one lane each, in
//      stream order): a wave prefix sum of the P_a / P_delta counts gives
//      every child its palette position and delta slot; a neighbour
//      reference that lands on a not-yet-known node of the same level always
//      lands on a child with one more coordinate bit set, so it is resolved
//      by three passes of decreasing child popcount;
//   4. for t = 0 the leaf segment is decoded 64 parents at a time and
//      replayed right away (rANS decode and operation replay "in one go");
//      leaf values are kept only for the expanded L_1 nodes;
//   5. the level-t block is mapped through the palette and written as
//      dense rows with 16-byte stores.
// Levels live in Morton order as palette indices (u8 when the palette has
// at most 253 entries).  Bricks that do not fit the LDS arena take the
// same code with u16 indices and an arena in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/csv.h"
#include "csv_format.hpp"

namespace {

constexpr int kLog2 = 5;                // 32^3 bricks
constexpr int kLutMaxBits = 11;         // largest supported table precision
constexpr uint32_t kMaxSym = 2 * 37448; // every node an operation plus a delta nibble
constexpr uint32_t kLdsBytes = 160 * 1024;
constexpr uint32_t kLutLdsCap = 24 * 1024;  // decode tables kept in LDS when they fit
constexpr uint32_t kPalFast = 253;      // u8 path: palette indices 0..252, 253..255 mark open references
constexpr int kMaxWaves = 8;
constexpr uint32_t kQueues = 256;  // work counters: launches in flight on one pool at a time

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

struct Launch {
    uint32_t lut_lds_words;  // decode-table words in LDS (0: tables read from global memory)
    uint32_t arena_bytes;    // LDS arena per wave
    uint32_t *queue;         // work counter (nullptr: static round robin)
    const uint32_t *order;   // processing order of requests (nullptr: identity)
    uint8_t *scratch;        // global arenas for bricks that do not fit LDS
    uint32_t slot_bytes;
    uint32_t base;           // first request index
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

// order the wave's own memory operations (LDS arena, or the global arena)
template <bool kGlobal>
__device__ __forceinline__ void wsync() {
    if constexpr (kGlobal) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Per-brick phase clocks, only in builds with CSV_PHASE_TIMING: slot i of a
// request's 8 entries holds the shader clock at the end of phase i.
#ifdef CSV_PHASE_TIMING
__device__ uint64_t *g_phase = nullptr;
__device__ __forceinline__ void phase_mark(uint32_t rq, int i) {
    if (g_phase && lane() == 0) g_phase[8 * (size_t)rq + i] = __builtin_amdgcn_s_memtime();
}
#else
__device__ __forceinline__ void phase_mark(uint32_t, int) {}
#endif

__device__ __forceinline__ void report(int *err, int code, uint32_t who) {
    if (atomicCAS(err, 0, code) == 0) atomicExch(err + 1, (int)who);
}

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

// ---------------------------------------------------------------------------
// per-brick arena layout (bytes); the same function sizes LDS and global arenas
// ---------------------------------------------------------------------------
struct Layout {
    uint32_t pal, words, lv, bm, bpre, lst, list1, chunk, region, total;
};
__host__ __device__ inline uint32_t align16(uint32_t b) { return (b + 15u) & ~15u; }
// stage: palette (P entries) and nwc words copied into the arena;
// nU upper-level symbols; S0 leaf-segment symbols (0 unless decoding to
// LOD 0); idx bytes per palette index
__host__ __device__ inline Layout make_layout(bool stage, uint32_t P, uint32_t nwc, uint32_t nU, uint32_t S0, uint32_t idx) {
    Layout L;
    uint32_t o = 0;
    L.pal = o; o += stage ? align16(4 * P) : 0;
    L.words = o; o += stage ? align16(2 * nwc + 4) : 0;
    L.lv = o; o += align16(4680 * idx);
    L.bm = o; o += 592;
    L.bpre = o; o += 160;
    L.lst = o; o += align16(2 * (8 + 64 + 512));
    L.list1 = o; o += align16(2 * (S0 / 8 < 4096 ? S0 / 8 : 4096));
    L.chunk = o; o += S0 ? 256 : 0;
    L.region = o;
    const uint32_t nib_bytes = 4 * ((nU + 7) / 8 + 2);
    uint32_t l0 = 0;
    if (S0) {
        const uint32_t e1 = S0 / 8 < 4096 ? S0 / 8 : 4096;
        l0 = align16(8 * e1 * idx) + 4 * ((S0 + 7) / 8 + 2) + 16;
    }
    o += align16(nib_bytes > l0 ? nib_bytes : l0);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// interleaved rANS (lockstep over the W states)
// ---------------------------------------------------------------------------
struct Rans {
    const uint16_t *words;
    const uint32_t *lut;
    uint32_t nw, sbits, lutn, mask, W, lw, leaf;
    uint32_t x;        // this lane's state
    uint32_t cursor;   // words consumed (uniform)
    uint32_t next;     // next symbol index (uniform)
};

// decode symbols [r.next, end) into dst (packed nibbles, position i - base);
// false if the stream runs out of words
__device__ __forceinline__ bool rans_run(Rans &r, uint32_t end, uint32_t *dst, uint32_t base) {
    if (end <= r.next) return true;
    const uint32_t L = lane();
    const uint32_t s1 = (end - 1) >> r.lw;
    for (uint32_t s = r.next >> r.lw; s <= s1; s++) {
        const uint32_t i = (s << r.lw) + L;
        const bool act = L < r.W && i >= r.next && i < end;
        uint32_t sym = 0;
        bool need = false;
        if (act) {
            const uint32_t e = r.lut[(i >= r.leaf ? r.lutn : 0u) + (r.x & r.mask)];
            sym = e & 15u;
            r.x = (e >> 16) * (r.x >> r.sbits) + ((e >> 4) & 0xFFFu);
            need = r.x < csv::kRansLower;
        }
        const uint64_t bal = __ballot(need);
        const uint32_t cnt = (uint32_t)__popcll(bal);
        if (r.cursor + cnt > r.nw) return false;
        if (need) r.x = (r.x << 16) | (uint32_t)r.words[r.cursor + mbcnt(bal)];
        r.cursor += cnt;
        if (act) atomicOr(&dst[(i - base) >> 3], sym << (4 * ((i - base) & 7)));
    }
    r.next = end;
    return true;
}

// ---------------------------------------------------------------------------
// the decode of one brick by one wave
// ---------------------------------------------------------------------------
struct Hdr {
    const uint32_t *rec;
    uint32_t P, W, nw, t, vol, rq;
    // cumulative symbol counts c0..c4 (scalars, so a run-time level never
    // indexes a private array)
    uint32_t c0, c1, c2, c3, c4;
    __device__ __forceinline__ uint32_t c(uint32_t m) const {
        return m == 0 ? c0 : (m == 1 ? c1 : (m == 2 ? c2 : (m == 3 ? c3 : c4)));
    }
};

__device__ __forceinline__ void wave_fill(uint32_t *dst, uint32_t count, uint32_t v) {
    const uint32_t L = lane();
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0 && (count & 3) == 0) {
        const uint4 q = make_uint4(v, v, v, v);
        for (uint32_t e = 4 * L; e < count; e += 256) *reinterpret_cast<uint4 *>(dst + e) = q;
    } else {
        for (uint32_t e = L; e < count; e += 64) dst[e] = v;
    }
}

// children of one expanded parent from its 8 (op, stop) nibbles w:
// pv parent index, nb[a] the parent-level neighbour at +1 along axis a
// (valid if bit a of nbok), lowok bit a: the parent is not on the low face of
// axis a; ipb palette position before the first child; pam8/pdm8 children
// with P_a / P_delta; deltas at nibble db of dnib.
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
                    v = kMark + (uint32_t)a;  // same-level neighbour at - 1, resolved later
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

template <class IdxT, bool kG>
__device__ __forceinline__ bool decode_brick(const Hdr h, Rans rs, uint8_t *ar, const Layout lay, uint32_t *dst) {
    using V = Vec8<IdxT>;
    using VT = typename V::T;
    constexpr uint32_t kMark = sizeof(IdxT) == 1 ? 253u : 65533u;
    const uint32_t L = lane();
    const uint32_t t = h.t, P = h.P;
    const uint32_t *pal = kG ? h.rec + csv::record_header_words(kLog2) : reinterpret_cast<const uint32_t *>(ar + lay.pal);
    IdxT *lv = reinterpret_cast<IdxT *>(ar + lay.lv);
    uint8_t *bm = ar + lay.bm;
    uint16_t *bpre = reinterpret_cast<uint16_t *>(ar + lay.bpre);
    uint16_t *lst = reinterpret_cast<uint16_t *>(ar + lay.lst);
    uint16_t *list1 = reinterpret_cast<uint16_t *>(ar + lay.list1);
    uint32_t *nibU = reinterpret_cast<uint32_t *>(ar + lay.region);
    const uint32_t tl = t > 1 ? t : 1u;  // finest upper level replayed
    const uint32_t nU = h.c(tl);
    const uint32_t S0 = t == 0 ? h.c0 - h.c1 : 0u;

    // ---- upper-level symbols ------------------------------------------------
    for (uint32_t e = L; e < (nU + 7) / 8 + 2; e += 64) nibU[e] = 0;
    wsync<kG>();
    if (!rans_run(rs, nU, nibU, 0)) return false;
    wsync<kG>();
    phase_mark(h.rq, 2);

    // ---- levels 4 .. tl ----------------------------------------------------
    uint32_t E = 1;        // expanded parents of the level being built (the root)
    uint32_t ipl = 0;      // P_a operations so far
    bool bad = false;
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
        const uint32_t list_cap = (m >= 2) ? (1u << (3 * (kLog2 - m))) : (S0 / 8 < 4096 ? S0 / 8 : 4096u);
        // children of parents that are not expanded inherit the parent's index
        for (uint32_t q = L; q < np; q += 64) {
            const bool ex = pbm ? ((pbm[q >> 3] >> (q & 7)) & 1u) : true;
            cbm[q] = 0;
            if (!ex) *reinterpret_cast<VT *>(cur + 8 * q) = V::splat(up ? (uint32_t)up[q] : 0u);
        }
        wsync<kG>();
        const uint32_t seg = (m == kLog2 - 1) ? 0u : h.c((uint32_t)m + 1), seg_end = h.c((uint32_t)m);
        if ((uint64_t)seg + 8ull * E > seg_end) return false;
        const uint32_t D = seg_end - seg - 8 * E, ops0 = seg + D;  // deltas precede the operations
        uint32_t ip_run = 0, d_run = 0, ex_run = 0;
        for (uint32_t r0 = 0; r0 < E; r0 += 64) {
            const uint32_t r = r0 + L;
            const bool act = r < E;
            const uint32_t q = (act && plist) ? (uint32_t)plist[r] : 0u;
            const uint32_t w = act ? nib8(nibU, ops0 + 8 * r) : 0u;
            const uint32_t y = w & 0x77777777u;
            const uint32_t pam = act ? zero_nibbles(y ^ 0x66666666u) : 0u;
            const uint32_t pdm = act ? zero_nibbles(y ^ 0x55555555u) : 0u;
            const uint32_t exm = act ? (~w >> 3) & 0x11111111u : 0u;
            const uint32_t cnt = __builtin_popcount(pam) | (__builtin_popcount(pdm) << 10) | (__builtin_popcount(exm) << 20);
            const uint32_t inc = wave_incl_scan(cnt), exc = inc - cnt;
            const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
            if (act) {
                const uint32_t pv = up ? (uint32_t)up[q] : 0u;
                uint32_t nb[3], nbok = 0, lowok = 0;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const uint32_t am = axis_mask(a, Bp);
                    const bool hi = up && (q & am) != am;
                    nb[a] = hi ? (uint32_t)up[morton_inc(q, am)] : 0u;
                    nbok |= hi ? (1u << a) : 0u;
                    lowok |= (q & am) ? (1u << a) : 0u;
                }
                const VT vals = replay_children<IdxT>(w, pv, nb, nbok, lowok, ipl + ip_run + (exc & 1023u),
                                                      compact_nibble_bits(pam), compact_nibble_bits(pdm), nibU,
                                                      seg + d_run + ((exc >> 10) & 1023u), P, false, bad);
                *reinterpret_cast<VT *>(cur + 8 * q) = vals;
                uint32_t ex8 = compact_nibble_bits(exm);
                cbm[q] = (uint8_t)ex8;
                if (want_list) {
                    uint32_t pos = ex_run + (exc >> 20);
                    while (ex8) {
                        const uint32_t k = __builtin_ctz(ex8);
                        ex8 &= ex8 - 1;
                        if (pos < list_cap) clist[pos] = (uint16_t)(8 * q + k);
                        pos++;
                    }
                }
            }
            ip_run += tot & 1023u;
            d_run += (tot >> 10) & 1023u;
            ex_run += tot >> 20;
        }
        if (d_run != D) return false;
        if (want_list && ex_run > list_cap) return false;
        wsync<kG>();
        // neighbour references into this level, by decreasing child popcount
        for (int pc = 2; pc >= 0; pc--) {
            for (uint32_t r0 = 0; r0 < E; r0 += 64) {
                const uint32_t r = r0 + L;
                if (r >= E) continue;
                const uint32_t q = plist ? (uint32_t)plist[r] : 0u;
                VT vals = *reinterpret_cast<const VT *>(cur + 8 * q);
                bool dirty = false;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    if (__builtin_popcount(k) != pc) continue;
                    const uint32_t v = V::get(vals, k);
                    if (v >= kMark) {
                        const int a = (int)(v - kMark);
                        const uint32_t q2 = morton_dec(q, axis_mask(a, Bp));
                        V::set(vals, k, (uint32_t)cur[8 * q2 + (k | (1 << a))]);
                        dirty = true;
                    }
                }
                if (dirty) *reinterpret_cast<VT *>(cur + 8 * q) = vals;
            }
            wsync<kG>();
        }
        ipl += ip_run;
        E = ex_run;
    }
    if (__ballot(bad)) return false;
    phase_mark(h.rq, 3);

    const uint32_t G = 32u >> t;
    if (t >= 1) {
        // ---- output of an upper level -------------------------------------------
        const IdxT *res = lv + kLvOff[t];
        if (t == 4) {
            if (L < 8) dst[L] = pal_at<kG>(pal, res[L], P);  // Morton order equals dense order on a 2^3 grid
        } else {
            const uint32_t lg = (uint32_t)(kLog2 - t);
            for (uint32_t e = 4 * L; e < G * G * G; e += 256) {
                const uint32_t x0 = e & (G - 1), yy = (e >> lg) & (G - 1), zz = e >> (2 * lg);
                const uint32_t m0 = spread4(x0) | (spread4(yy) << 1) | (spread4(zz) << 2);
                uint4 o;
                o.x = pal_at<kG>(pal, res[m0], P);
                o.y = pal_at<kG>(pal, res[m0 | 1u], P);
                o.z = pal_at<kG>(pal, res[m0 | 8u], P);
                o.w = pal_at<kG>(pal, res[m0 | 9u], P);
                *reinterpret_cast<uint4 *>(dst + e) = o;
            }
        }
        return true;
    }

    // ---- leaf level: fused rANS + replay, 64 expanded L_1 nodes per round --------
    const uint32_t E1 = E;
    const IdxT *l1 = lv + kLvOff[1];
    const uint8_t *bm1 = bm + kBmOff[1];
    const uint64_t *bm1w = reinterpret_cast<const uint64_t *>(bm1);
    {   // rank prefix of the expanded L_1 bits, per 64-bit word
        const uint32_t c = (uint32_t)__popcll(bm1w[L]);
        const uint32_t inc = wave_incl_scan(c);
        bpre[L] = (uint16_t)(inc - c);
    }
    const uint32_t seg = h.c1, seg_end = h.c0;
    if ((uint64_t)seg + 8ull * E1 > seg_end) return false;
    const uint32_t D0 = seg_end - seg - 8 * E1, ops0 = seg + D0;
    IdxT *l0x = reinterpret_cast<IdxT *>(ar + lay.region);
    uint32_t *dl0 = reinterpret_cast<uint32_t *>(ar + lay.region + align16(8 * E1 * (uint32_t)sizeof(IdxT)));
    uint32_t *chunk = reinterpret_cast<uint32_t *>(ar + lay.chunk);
    for (uint32_t e = L; e < (D0 + 7) / 8 + 2; e += 64) dl0[e] = 0;
    wsync<kG>();
    if (!rans_run(rs, seg + D0, dl0, seg)) return false;
    uint32_t ip_run = 0, d_run = 0;
    for (uint32_t r0 = 0; r0 < E1; r0 += 64) {
        const uint32_t nb = E1 - r0 < 64 ? E1 - r0 : 64u;
        chunk[L] = 0;
        wsync<kG>();
        if (!rans_run(rs, ops0 + 8 * (r0 + nb), chunk, ops0 + 8 * r0)) return false;
        wsync<kG>();
        const bool act = L < nb;
        const uint32_t r = r0 + L;
        const uint32_t w = act ? chunk[L] : 0u;
        const uint32_t p = act ? (uint32_t)list1[r] : 0u;
        const uint32_t y = w & 0x77777777u;
        const uint32_t pam = act ? zero_nibbles(y ^ 0x66666666u) : 0u;
        const uint32_t pdm = act ? zero_nibbles(y ^ 0x55555555u) : 0u;
        const uint32_t cnt = __builtin_popcount(pam) | (__builtin_popcount(pdm) << 10);
        const uint32_t inc = wave_incl_scan(cnt), exc = inc - cnt;
        const uint32_t tot = uniform(__builtin_amdgcn_readlane(inc, 63));
        if (act) {
            const uint32_t pv = l1[p];
            uint32_t nbv[3], nbok = 0, lowok = 0;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const uint32_t am = axis_mask(a, 4);
                const bool hi = (p & am) != am;
                nbv[a] = hi ? (uint32_t)l1[morton_inc(p, am)] : 0u;
                nbok |= hi ? (1u << a) : 0u;
                lowok |= (p & am) ? (1u << a) : 0u;
            }
            const VT vals = replay_children<IdxT>(w, pv, nbv, nbok, lowok, ipl + ip_run + (exc & 1023u),
                                                  compact_nibble_bits(pam), compact_nibble_bits(pdm), dl0,
                                                  d_run + ((exc >> 10) & 1023u), P, true, bad);
            *reinterpret_cast<VT *>(l0x + 8 * r) = vals;
        }
        ip_run += tot & 1023u;
        d_run += (tot >> 10) & 1023u;
    }
    if (d_run != D0 || __ballot(bad)) return false;
    phase_mark(h.rq, 4);
    // a complete decode ends in the encoder's initial states with every word read
    if (__ballot(L < rs.W && rs.x != csv::kRansLower) || rs.cursor != rs.nw) return false;
    wsync<kG>();
    // leaf neighbour references, by decreasing child popcount
    for (int pc = 2; pc >= 0; pc--) {
        for (uint32_t r0 = 0; r0 < E1; r0 += 64) {
            const uint32_t r = r0 + L;
            if (r >= E1) continue;
            VT vals = *reinterpret_cast<const VT *>(l0x + 8 * r);
            bool dirty = false;
            uint32_t p = 0xFFFFFFFFu;
#pragma unroll
            for (int k = 0; k < 8; k++) {
                if (__builtin_popcount(k) != pc) continue;
                const uint32_t v = V::get(vals, k);
                if (v >= kMark) {
                    if (p == 0xFFFFFFFFu) p = list1[r];
                    const int a = (int)(v - kMark);
                    const uint32_t p2 = morton_dec(p, axis_mask(a, 4));
                    const uint32_t k2 = (uint32_t)(k | (1 << a));
                    uint32_t nv;
                    if ((bm1[p2 >> 3] >> (p2 & 7)) & 1u) {
                        const uint32_t rk = bpre[p2 >> 6] + (uint32_t)__popcll(bm1w[p2 >> 6] & ((1ull << (p2 & 63)) - 1ull));
                        nv = l0x[8 * rk + k2];
                    } else {
                        nv = l1[p2];
                    }
                    V::set(vals, k, nv);
                    dirty = true;
                }
            }
            if (dirty) *reinterpret_cast<VT *>(l0x + 8 * r) = vals;
        }
        wsync<kG>();
    }

    phase_mark(h.rq, 5);
    // ---- leaf output: lane = a pair of x-adjacent L_1 nodes, 4 rows of 16 bytes ----
    for (uint32_t it = 0; it < 32; it++) {
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
            *reinterpret_cast<uint4 *>(dst + 4 * xp + 32 * (yy + 32 * zz)) = o;
        }
    }
    phase_mark(h.rq, 6);
    return true;
}

// validate a request and its record, then decode it
__device__ __forceinline__ void process(const DecodeArgs &a, const Launch &l, uint32_t rq, uint8_t *arena, uint8_t *slot,
                        const uint32_t *slut) {
    const uint32_t L = lane();
    phase_mark(rq, 0);
    const uint32_t id = uniform(a.ids[rq]);
    const uint32_t t = uniform(a.lods ? (uint32_t)a.lods[rq] : a.lod_scalar);
    if (t > (uint32_t)kLog2) {
        if (L == 0) report(a.err, CSV_ERANGE, rq);
        return;
    }
    const uint32_t G = 32u >> t, count = G * G * G;
    uint32_t *dst = a.out + (a.out_off ? a.out_off[rq] : (uint64_t)rq * count);
    if (id >= a.n_bricks) {
        if (L == 0) report(a.err, CSV_ERANGE, rq);
        wave_fill(dst, count, 0);
        return;
    }
    Hdr h;
    h.rec = reinterpret_cast<const uint32_t *>(a.rec_ptr[id]);
    const uint32_t size = a.rec_size[id];
    h.vol = a.rec_vol[id];
    h.P = h.rec[0];
    h.W = h.rec[1];
    h.nw = h.rec[2];
    h.t = t;
    h.rq = rq;
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
    if (!ok) {
        if (L == 0) report(a.err, CSV_ECORRUPT, id);
        wave_fill(dst, count, 0);
        return;
    }
    if (t == (uint32_t)kLog2 || h.c0 == 0) {  // coarsest level or uniform brick: palette[0]
        wave_fill(dst, count, h.rec[hdr]);
        return;
    }
    const uint32_t n = h.c(t);
    const uint32_t tl = t > 1 ? t : 1u;
    const uint32_t S0 = t == 0 ? h.c0 - h.c1 : 0u;
    const uint32_t nwc = h.nw < n ? h.nw : n;
    const uint32_t sbits = a.vol_bits[h.vol];
    Rans rs;
    rs.lut = (l.lut_lds_words ? slut : a.luts) + a.lut_off[h.vol];
    rs.nw = h.nw;
    rs.sbits = sbits;
    rs.lutn = 1u << sbits;
    rs.mask = rs.lutn - 1u;
    rs.W = h.W;
    rs.lw = 31u - (uint32_t)__builtin_clz(h.W);
    rs.leaf = h.c1;
    rs.cursor = 0;
    rs.next = 0;
    rs.x = L < h.W ? h.rec[hdr + h.P + L] : 0u;
    const Layout fast = make_layout(true, h.P, nwc, h.c(tl), S0, 1);
    bool done;
    if (h.P <= kPalFast && fast.total <= l.arena_bytes) {
        // stage the palette and the words this decode can read
        uint32_t *pal_s = reinterpret_cast<uint32_t *>(arena + fast.pal);
        uint32_t *wd_s = reinterpret_cast<uint32_t *>(arena + fast.words);
        const uint32_t *pal_g = h.rec + hdr, *wd_g = h.rec + hdr + h.P + h.W;
        const uint32_t nwd = (nwc + 1) / 2;
        for (uint32_t e = L; e < h.P; e += 64) pal_s[e] = pal_g[e];
        for (uint32_t e = L; e < nwd; e += 256) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) v[u] = (e + 64 * u < nwd) ? wd_g[e + 64 * u] : 0u;
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (e + 64 * u < nwd) wd_s[e + 64 * u] = v[u];
        }
        rs.words = reinterpret_cast<const uint16_t *>(wd_s);
        wsync<false>();
        phase_mark(rq, 1);
        done = decode_brick<uint8_t, false>(h, rs, arena, fast, dst);
    } else if (slot) {
        const Layout slow = make_layout(false, h.P, nwc, h.c(tl), S0, 2);
        rs.words = reinterpret_cast<const uint16_t *>(h.rec + hdr + h.P + h.W);
        phase_mark(rq, 1);
        if (L == 0) phase_mark(rq, 7);
        done = decode_brick<uint16_t, true>(h, rs, slot, slow, dst);
    } else {
        if (L == 0) report(a.err, CSV_EINVAL, id);
        wave_fill(dst, count, 0);
        return;
    }
    if (!done) {
        if (L == 0) report(a.err, CSV_ECORRUPT, id);
        wave_fill(dst, count, 0);
    }
}

template <int WPG>
__global__ __launch_bounds__(WPG * 64) void decode_kernel(DecodeArgs a, Launch l) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *slut = reinterpret_cast<uint32_t *>(smem);
    for (uint32_t e = threadIdx.x; e < l.lut_lds_words; e += blockDim.x) slut[e] = a.luts[e];
    __syncthreads();
    const uint32_t wave = threadIdx.x >> 6;
    uint8_t *arena = smem + align16(4 * l.lut_lds_words) + wave * l.arena_bytes;
    const uint32_t wid = blockIdx.x * WPG + wave;
    uint8_t *slot = l.scratch ? l.scratch + (size_t)wid * l.slot_bytes : nullptr;
    for (uint32_t k = 0;; k++) {
        uint32_t req;
        if (l.queue) {
            uint32_t v = 0;
            if (lane() == 0) v = atomicAdd(l.queue, 1u);
            req = uniform(v) + l.base;
        } else {
            req = l.base + wid + k * gridDim.x * WPG;
        }
        if (req >= a.n) break;
        process(a, l, l.order ? l.order[req] : req, arena, slot, slut);
    }
}

__global__ void zero_word(uint32_t *p) { *p = 0; }

// Longest-first request order: requests are binned by the log2 of their
// work (symbols to decode plus output voxels / 8), largest bin first, and
// laid out bin by bin.  ws: 2 x 32 counters, zeroed by the first kernel.
constexpr int kBins = 32;
__device__ __forceinline__ uint32_t work_bin(const DecodeArgs &a, uint32_t r) {
    const uint32_t id = a.ids[r];
    const uint32_t t = a.lods ? (uint32_t)a.lods[r] : a.lod_scalar;
    if (id >= a.n_bricks || t > (uint32_t)kLog2) return kBins - 1;
    const uint32_t *rec = reinterpret_cast<const uint32_t *>(a.rec_ptr[id]);
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

}  // namespace

// ---------------------------------------------------------------------------
// Pool
// ---------------------------------------------------------------------------
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
    uint32_t *d_queue = nullptr;
    uint8_t *d_scratch = nullptr;
    std::atomic<uint32_t> next_queue{0};  // launches take work counters round robin
    uint32_t *d_order = nullptr;          // longest-first request order
    uint32_t order_cap = 0;
    uint32_t *d_order_ws = nullptr;       // bin counters of the order kernels
    csv_shape shape{5, 1, 1, 0, 0.f};     // launch shape of csv_decode_bricks
    uint32_t slot_bytes = 0;
    uint32_t n_slots = 0;
    uint32_t max_fast_bytes = 0;  // largest LDS arena a brick of the pool needs
    bool any_big_palette = false;
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

uint32_t arena_for(const csv_pool *p, int wpg, uint32_t *lut_lds) {
    const uint32_t lw = (uint32_t)p->luts.size();
    *lut_lds = (4 * lw <= kLutLdsCap) ? lw : 0u;
    return ((kLdsBytes - align16(4 * *lut_lds)) / (uint32_t)wpg) & ~15u;
}

// smallest per-wave arena any launch shape can give (most waves, largest table area)
uint32_t min_arena() { return ((kLdsBytes - kLutLdsCap) / kMaxWaves) & ~15u; }

template <int WPG>
int launch_shape(csv_pool *pool, const DecodeArgs &a, uint32_t grid, bool queue, bool plain, bool lpt, hipStream_t s) {
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        attr = hipFuncSetAttribute(reinterpret_cast<const void *>(decode_kernel<WPG>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    });
    if (attr != hipSuccess) return CSV_EHIP;
    Launch l;
    l.arena_bytes = arena_for(pool, WPG, &l.lut_lds_words);
    l.queue = nullptr;
    l.order = nullptr;
    l.scratch = pool->d_scratch;
    l.slot_bytes = pool->slot_bytes;
    l.base = 0;
    const size_t lds = align16(4 * l.lut_lds_words) + (size_t)WPG * l.arena_bytes;
    if (plain) {
        DecodeArgs b = a;
        for (uint32_t i = 0; i < a.n; i++) {
            l.base = i;
            b.n = i + 1;
            hipLaunchKernelGGL(decode_kernel<WPG>, dim3(1), dim3(64 * WPG), lds, s, b, l);
        }
    } else {
        if (lpt) {
            // the order buffer only grows outside of stream capture (the autotuner or a
            // first uncaptured call sizes it)
            if (a.n > pool->order_cap) return CSV_EBUSY;
            const uint32_t g = std::min<uint32_t>((a.n + 255) / 256, 1024u);
            hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, pool->d_order_ws, 2u * kBins);
            hipLaunchKernelGGL(order_count, dim3(g), dim3(256), 0, s, a, pool->d_order_ws);
            hipLaunchKernelGGL(order_scan, dim3(1), dim3(64), 0, s, pool->d_order_ws);
            hipLaunchKernelGGL(order_scatter, dim3(g), dim3(256), 0, s, a, pool->d_order_ws, pool->d_order);
            l.order = pool->d_order;
        }
        if (queue) {
            l.queue = pool->d_queue + pool->next_queue.fetch_add(1, std::memory_order_relaxed) % kQueues;
            hipLaunchKernelGGL(zero_word, dim3(1), dim3(1), 0, s, l.queue);
        }
        hipLaunchKernelGGL(decode_kernel<WPG>, dim3(grid), dim3(64 * WPG), lds, s, a, l);
    }
    return hipGetLastError() == hipSuccess ? CSV_OK : CSV_EHIP;
}

int ensure_order(csv_pool *pool, uint32_t n) {
    if (n <= pool->order_cap) return CSV_OK;
    if (!pool->d_order_ws && hipMalloc(reinterpret_cast<void **>(&pool->d_order_ws), 8 * kBins) != hipSuccess)
        return CSV_ENOMEM;
    uint32_t *o = nullptr;
    const uint32_t cap = std::max(n, 2 * pool->order_cap);
    if (hipMalloc(reinterpret_cast<void **>(&o), 4ull * cap) != hipSuccess) return CSV_ENOMEM;
    if (pool->d_order) {
        (void)hipDeviceSynchronize();
        (void)hipFree(pool->d_order);
    }
    pool->d_order = o;
    pool->order_cap = cap;
    return CSV_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

int launch(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
           const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, bool plain, int wpg, uint32_t grid_mult,
           bool queue, bool lpt = false) {
    if (!pool || (n && (!ids || !out))) return CSV_EINVAL;
    if (!lods && lod_scalar > (uint32_t)kLog2) return CSV_ERANGE;
    if (lods && !out_off) return CSV_EINVAL;
    if (n == 0) return CSV_OK;
    if (pool->rec_ptr.empty() || !pool->d_err) return CSV_EINVAL;
    DeviceGuard g(pool->device);
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
    const uint32_t max_wgs = pool->n_slots / kMaxWaves;  // one global arena slot per wave
    uint32_t grid = (uint32_t)std::max(1, pool->n_cu) * std::max(1u, grid_mult);
    if (grid > max_wgs) grid = max_wgs;
    const uint32_t need = (n + (uint32_t)wpg - 1) / (uint32_t)wpg;
    if (grid > need) grid = need;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (lpt && !plain && n > pool->order_cap && !capturing(s)) {
        const int rc = ensure_order(pool, n);
        if (rc) return rc;
    }
    switch (wpg) {
        case 4: return launch_shape<4>(pool, a, grid, queue, plain, lpt, s);
        case 5: return launch_shape<5>(pool, a, grid, queue, plain, lpt, s);
        case 6: return launch_shape<6>(pool, a, grid, queue, plain, lpt, s);
        case 8: return launch_shape<8>(pool, a, grid, queue, plain, lpt, s);
        default: return CSV_EINVAL;
    }
}

constexpr int kDefaultWaves = 5;

bool valid_shape(const csv_shape &sh) {
    return (sh.waves_per_group == 4 || sh.waves_per_group == 5 || sh.waves_per_group == 6 ||
            sh.waves_per_group == 8) &&
           sh.groups_per_cu >= 1 && sh.groups_per_cu <= 16;
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
    p->n_slots = (uint32_t)p->n_cu * kMaxWaves;  // one resident workgroup per CU (LDS bound)
    if (hipMalloc(reinterpret_cast<void **>(&p->d_err), 2 * sizeof(int)) != hipSuccess ||
        hipMemset(p->d_err, 0, 2 * sizeof(int)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&p->d_queue), 4 * kQueues) != hipSuccess) {
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
    (void)hipFree(p->d_queue);
    (void)hipFree(p->d_scratch);
    (void)hipFree(p->d_order);
    (void)hipFree(p->d_order_ws);
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
    uint32_t max_fast = p->max_fast_bytes;
    bool big = p->any_big_palette;
    for (uint32_t i = 0; i < info.n_bricks; i++) {
        if (index[i + 1] < index[i] + 4 * hdr || (index[i] & 3)) return CSV_ECORRUPT;
        const uint32_t *w = reinterpret_cast<const uint32_t *>(blob + rs + index[i]);
        const uint32_t P = w[0], nw = w[2], c0 = w[3], c1 = w[4];
        if (c0 == 0) continue;
        if (c1 > c0 || c0 > kMaxSym) return CSV_ECORRUPT;
        big |= P > kPalFast;
        const Layout lay = make_layout(true, P, std::min(nw, c0), c1, c0 - c1, 1);
        max_fast = std::max(max_fast, lay.total);
    }
    void *buf = nullptr;
    const size_t rb = std::max<uint64_t>(info.record_bytes, 4);
    if (hipMalloc(&buf, rb) != hipSuccess) return CSV_ENOMEM;
    if (hipMemcpy(buf, blob + rs, info.record_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        return CSV_EHIP;
    }
    // a global arena per wave slot when some brick may not fit an LDS arena
    if ((big || max_fast > min_arena()) && !p->d_scratch) {
        const Layout worst = make_layout(false, 0, 0, kMaxSym, kMaxSym, 2);
        p->slot_bytes = align16(worst.total);
        if (hipMalloc(reinterpret_cast<void **>(&p->d_scratch), (size_t)p->slot_bytes * p->n_slots) != hipSuccess) {
            (void)hipFree(buf);
            p->slot_bytes = 0;
            return CSV_ENOMEM;
        }
    }
    p->max_fast_bytes = max_fast;
    p->any_big_palette = big;
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
    info->device_bytes = p->record_bytes + p->rec_ptr.size() * (8 + 4 + 2) + p->luts.size() * 4 +
                         (uint64_t)p->slot_bytes * (p->d_scratch ? p->n_slots : 0) + 72;
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
                  sh.waves_per_group, sh.groups_per_cu, sh.use_queue != 0, sh.lpt_order != 0);
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
    const int waves[4] = {4, 5, 6, 8};
    csv_shape win{};
    win.ms = 1e30f;
    int rc = CSV_OK;
    for (int wi = 0; wi < 4 && !rc; wi++)
        for (int q = 0; q < 2 && !rc; q++)
            for (int o = 0; o < 2 && !rc; o++) {
                if (o && !q) continue;  // the longest-first order only matters with the work counter
                csv_shape sh{waves[wi], 1, q, o, 0.f};
                // one warm-up launch, then reps timed launches
                rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group, 1,
                            q != 0, o != 0);
                if (rc) break;
                (void)hipEventRecord(e0, s);
                for (uint32_t r = 0; r < reps && !rc; r++)
                    rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false, sh.waves_per_group, 1,
                                q != 0, o != 0);
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

int csv_decode_bricks_plain(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                            const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, true, kDefaultWaves, 1,
                  false);
}

int csv_decode_bricks_shaped(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                             const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, const csv_shape *shape) {
    if (!pool || !shape || !valid_shape(*shape)) return CSV_EINVAL;
    return launch(const_cast<csv_pool *>(pool), ids, lods, lod_scalar, out_off, n, out, stream, false,
                  shape->waves_per_group, shape->groups_per_cu, shape->use_queue != 0, shape->lpt_order != 0);
}

struct csv_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t own = nullptr;
    int device = 0;
};

int csv_graph_create(csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                     const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, csv_graph **graph) {
    if (!pool || !graph || !n) return CSV_EINVAL;
    DeviceGuard g(pool->device);
    csv_graph *G = new (std::nothrow) csv_graph;
    if (!G) return CSV_ENOMEM;
    G->device = pool->device;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!s) {
        if (hipStreamCreateWithFlags(&G->own, hipStreamNonBlocking) != hipSuccess) {
            delete G;
            return CSV_EHIP;
        }
        s = G->own;
    }
    const csv_shape sh = pool->shape;
    int rc = CSV_OK;
    if (sh.lpt_order) rc = ensure_order(pool, n);  // size the order buffer before capture
    if (!rc && hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = CSV_EHIP;
    if (!rc) {
        rc = launch(pool, ids, lods, lod_scalar, out_off, n, out, s, false, sh.waves_per_group, sh.groups_per_cu,
                    sh.use_queue != 0, sh.lpt_order != 0);
        hipGraph_t gr = nullptr;
        if (hipStreamEndCapture(s, &gr) != hipSuccess && !rc) rc = CSV_EHIP;
        G->graph = gr;
        if (!rc && hipGraphInstantiate(&G->exec, gr, nullptr, nullptr, 0) != hipSuccess) rc = CSV_EHIP;
    }
    if (rc) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        if (G->own) (void)hipStreamDestroy(G->own);
        delete G;
        return rc;
    }
    *graph = G;
    return CSV_OK;
}

int csv_graph_launch(csv_graph *graph, void *stream) {
    if (!graph || !graph->exec) return CSV_EINVAL;
    DeviceGuard g(graph->device);
    return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? CSV_OK : CSV_EHIP;
}

void csv_graph_destroy(csv_graph *graph) {
    if (!graph) return;
    DeviceGuard g(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    if (graph->own) (void)hipStreamDestroy(graph->own);
    delete graph;
}

#ifdef CSV_PHASE_TIMING
// install (or clear, with NULL) a device buffer of 8 u64 clocks per request
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
