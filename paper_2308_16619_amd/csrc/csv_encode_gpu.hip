// GPU compressor for 32^3 bricks: the container of csv_encode_volume, byte
// for byte, built on the device from a label volume resident in HBM.
//
//   symbols kernel (a 256-thread workgroup per brick, persistent grid):
//     resolution pyramid (Sec. 3.1)    level 1 from the volume, levels 2..5
//                                      in LDS; level 0 read where needed
//     operations (Sec. 3.2, Alg. 2)    per child level, the children of the
//                                      expanded parents in Morton order: the
//                                      reuse operations (parent, neighbours)
//                                      in parallel, then the palette
//                                      operations of the remaining children
//                                      in order by one wavefront holding the
//                                      last 17 palette entries in its lanes
//     frequency tables (Sec. 3.3/3.4)  histograms of the sampled bricks'
//                                      symbols, normalised on the host
//     the symbol stream and palette of every brick go to an arena
//   rANS kernel (a wavefront per brick): interleaved rANS (Sec. 3.3), one
//     state per lane, symbols from last to first, the words of a step
//     placed by ballot; the record into a second arena
//   packing: a device scan of record sizes, one copy kernel
//
// Per-workgroup and per-wavefront scratch in global memory holds the
// symbol stream, palette and words of the bricks in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "csv.h"
#include "csv_format.hpp"

namespace csv {
// frequency normalisation of the host compressor (same arithmetic, one copy)
void normalize_counts(const uint64_t cnt[16], uint32_t M, uint32_t f[16]);
}

namespace {

constexpr int kN = 5;
constexpr uint32_t kThreads = 256;
constexpr uint32_t kPer = 3;                  // child slots per thread per chunk
constexpr uint32_t kChunk = kThreads * kPer;
constexpr uint32_t kNone = 0xFFFFFFFFu;       // no slot
constexpr uint32_t kNodes = 4681;           // levels 1..5 of a 32^3 brick
constexpr uint32_t kMaxChildren = 37448;    // 8 * (1 + 8 + 64 + 512 + 4096)
constexpr uint32_t kMaxSym = 2 * kMaxChildren;  // operations and deltas
// per-workgroup scratch (bytes)
constexpr size_t kOffSym = 0;
constexpr size_t kOffOps = 76800;           // >= kMaxSym
constexpr size_t kOffDel = kOffOps + 32768;
constexpr size_t kOffPal = kOffDel + 32768;
constexpr size_t kScratch = kOffPal + 4 * 37456;  // palette <= kMaxChildren + 1
// per-wavefront scratch of the rANS kernel: the words of one brick
constexpr size_t kWordsScratch = 2 * (size_t)kMaxSym + 64;

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0xFF0000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}
// Morton index: bit 0 of each 3-bit group is x, then y, then z
__device__ __forceinline__ uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
// offset of level l (1..5) in the LDS node arrays
__device__ __forceinline__ uint32_t lvl_off(int l) {
    return l == 1 ? 0u : (l == 2 ? 4096u : (l == 3 ? 4608u : (l == 4 ? 4672u : 4680u)));
}

// Per-workgroup phase clocks, only in builds with CSV_PHASE_TIMING: 8 u64
// per workgroup, the shader clocks its thread 0 spent in each phase.
#ifdef CSV_PHASE_TIMING
__device__ uint64_t *g_enc_phase = nullptr;
struct PhaseClock {
    uint64_t acc[8] = {}, t0 = 0;
    __device__ void start() { t0 = __builtin_amdgcn_s_memtime(); }
    __device__ void stop(int i) {
        const uint64_t t = __builtin_amdgcn_s_memtime();
        acc[i] += t - t0;
        t0 = t;
    }
    __device__ void flush() {
        if (g_enc_phase && threadIdx.x == 0)
            for (int i = 0; i < 8; i++) g_enc_phase[8 * (size_t)blockIdx.x + i] += acc[i];
    }
};
#else
struct PhaseClock {
    __device__ void start() {}
    __device__ void stop(int) {}
    __device__ void flush() {}
};
#endif

struct EncArgs {
    const uint32_t *vol;
    uint32_t nx, ny, nz, nbx, nby;
    uint32_t n_items;          // bricks
    uint32_t sample_stride;    // the frequency tables count every sample_stride-th brick
    unsigned long long *hist;  // 2 x 16 symbol counters of the sampled bricks
    uint32_t f[2][16], c[2][16];
    uint32_t bits, lane_k, lane_max;
    uint8_t *scratch;          // symbols kernel: per workgroup
    uint8_t *wscratch;         // rANS kernel: per wavefront
    uint8_t *sarena;           // symbol streams and palettes (symbols kernel -> rANS kernel)
    uint64_t sarena_cap;
    unsigned long long *sarena_top;
    uint64_t *soff;            // per brick: offset in sarena
    uint32_t *sn, *sp, *scum;  // per brick: symbols, palette entries, cum[5]
    uint8_t *arena;
    uint64_t arena_cap;
    unsigned long long *arena_top;
    uint32_t *sizes;  // per brick: record bytes
    uint64_t *aoff;   // per brick: record offset in the arena
};

struct Brick {
    uint64_t x0, y0, z0;
};

// label of voxel (cx, cy, cz) of the brick; 0 beyond the volume (padding).
// The address is clamped into the volume and the value masked, so that the
// loads of a thread need no branches and issue together.
__device__ __forceinline__ uint32_t voxel(const EncArgs &a, const Brick &b, uint32_t cx, uint32_t cy, uint32_t cz) {
    const uint64_t x = b.x0 + cx, y = b.y0 + cy, z = b.z0 + cz;
    const bool in = x < a.nx && y < a.ny && z < a.nz;
    const uint64_t xc = in ? x : 0, yc = in ? y : 0, zc = in ? z : 0;
    const uint32_t v = a.vol[xc + (uint64_t)a.nx * (yc + (uint64_t)a.ny * zc)];
    return in ? v : 0u;
}

// label of node j (Morton) on level m
__device__ __forceinline__ uint32_t label_at(const EncArgs &a, const Brick &b, const uint32_t *lab, int m, uint32_t j) {
    if (m >= 1) return lab[lvl_off(m) + j];
    return voxel(a, b, compact3(j), compact3(j >> 1), compact3(j >> 2));
}

// rank of this thread's flag among the workgroup's set flags, and their count
__device__ __forceinline__ uint32_t wg_rank(bool f, uint32_t &total, uint32_t *wcnt) {
    const uint64_t m = __ballot(f);
    const uint32_t w = threadIdx.x >> 6;
    if (lane() == 0) wcnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (uint32_t k = 0; k < kThreads / 64; k++) {
        const uint32_t c = wcnt[k];
        before += k < w ? c : 0u;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return before + mbcnt(m);
}

__device__ __forceinline__ uint32_t lanes_for(uint32_t n, uint32_t K, uint32_t Wmax) {
    if (n == 0) return 0;
    uint32_t W = 1;
    while (2 * W <= Wmax && (uint64_t)2 * W * K <= n) W *= 2;
    return W;
}

// the most frequent of 8 children, the earliest winning a tie; same: all equal
__device__ __forceinline__ uint32_t mode8(const uint32_t ch[8], bool &same) {
    same = true;
#pragma unroll
    for (int k = 1; k < 8; k++) same &= ch[k] == ch[0];
    if (same) return ch[0];
    int bestk = 0, bestn = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        int n = 0;
#pragma unroll
        for (int r = 0; r < 8; r++) n += ch[r] == ch[k];
        if (n > bestn) {
            bestn = n;
            bestk = k;
        }
    }
    uint32_t v = ch[0];
#pragma unroll
    for (int k = 1; k < 8; k++) v = k == bestk ? ch[k] : v;
    return v;
}

// Pyramid, operations and palette of one brick per workgroup; the symbol
// stream and palette go to the arena for the rANS kernel.
// (LDS under 32 KB and 5 waves per SIMD: five workgroups per CU)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void symbols_kernel(EncArgs a) {
    __shared__ uint32_t lab[kNodes];
    __shared__ uint32_t cstb[(kNodes + 31) / 32];  // constant-subtree flags, one bit per node
    __shared__ uint16_t expl[4096];
    __shared__ uint32_t c_lab[kChunk];
    __shared__ uint8_t c_op[kChunk];
    __shared__ uint32_t wcnt[kThreads / 64];
    __shared__ uint32_t wcnt4[kPer][kThreads / 64];
    __shared__ uint32_t share[8];  // 0: deltas of a level; 3: palette entries; 4, 5: arena offset
    __shared__ uint32_t s_cum[kN];
    __shared__ uint32_t hist_l[32];
    const uint32_t t = threadIdx.x, L = lane(), w = t >> 6;
    uint8_t *scr = a.scratch + (size_t)blockIdx.x * kScratch;
    uint8_t *sym = scr + kOffSym;
    uint8_t *ops = scr + kOffOps;
    uint8_t *dels = scr + kOffDel;
    uint32_t *pal = reinterpret_cast<uint32_t *>(scr + kOffPal);
    PhaseClock pc;
    for (uint32_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
        pc.start();
        const uint64_t id = item;
        Brick b;
        b.x0 = (id % a.nbx) * 32;
        b.y0 = ((id / a.nbx) % a.nby) * 32;
        b.z0 = (id / ((uint64_t)a.nbx * a.nby)) * 32;
        for (uint32_t i = t; i < (kNodes + 31) / 32; i += kThreads) cstb[i] = 0;
        __syncthreads();
        // level 1 from the volume (every level-0 node is a constant subtree)
        for (uint32_t q = t; q < 4096; q += kThreads) {
            const uint32_t x = 2 * compact3(q), y = 2 * compact3(q >> 1), z = 2 * compact3(q >> 2);
            uint32_t ch[8];
#pragma unroll
            for (int k = 0; k < 8; k++) ch[k] = voxel(a, b, x + (k & 1), y + ((k >> 1) & 1), z + (k >> 2));
            bool same;
            lab[q] = mode8(ch, same);
            // a wavefront's 64 nodes are one aligned pair of flag words
            const uint64_t bm = __ballot(same);
            if (L == 0) {
                cstb[q >> 5] = (uint32_t)bm;
                cstb[(q >> 5) + 1] = (uint32_t)(bm >> 32);
            }
        }
        __syncthreads();
        for (int l = 2; l <= kN; l++) {
            const uint32_t n = 1u << (3 * (kN - l)), lo = lvl_off(l - 1), hi = lvl_off(l);
            for (uint32_t q = t; q < n; q += kThreads) {
                uint32_t ch[8];
#pragma unroll
                for (int k = 0; k < 8; k++) ch[k] = lab[lo + 8 * q + k];
                // the 8 children's flags: one byte of a word (lo and 8q are multiples of 8)
                const uint32_t c8 = lo + 8 * q;
                const bool allc = ((cstb[c8 >> 5] >> (c8 & 31)) & 0xFFu) == 0xFFu;
                bool same;
                lab[hi + q] = mode8(ch, same);
                if (n >= 64) {  // levels 2, 3: as level 1 (their offsets are multiples of 64)
                    const uint64_t bm = __ballot(same && allc);
                    if (L == 0) {
                        cstb[(hi + q) >> 5] = (uint32_t)bm;
                        cstb[((hi + q) >> 5) + 1] = (uint32_t)(bm >> 32);
                    }
                } else if (same && allc) {  // levels 4, 5 share a word
                    atomicOr(&cstb[(hi + q) >> 5], 1u << ((hi + q) & 31));
                }
            }
            __syncthreads();
        }
        pc.stop(0);  // pyramid
        // symbol stream: child levels 4 .. 0
        uint32_t win = 0, P = 1, D = 0;  // wavefront 0: palette window (lane i: entry P-1-i), size, deltas
        if (w == 0 && L == 0) {
            win = lab[lvl_off(kN)];
            pal[0] = win;
        }
        uint32_t base = 0;
        for (int m = kN - 1; m >= 0; m--) {
            const int l = m + 1;
            const uint32_t np = 1u << (3 * (kN - l)), G = 32u >> m;
            uint32_t E = 0;
            for (uint32_t q0 = 0; q0 < np; q0 += kThreads) {
                const uint32_t q = q0 + t;
                const bool f = q < np && !((cstb[(lvl_off(l) + q) >> 5] >> ((lvl_off(l) + q) & 31)) & 1u);
                uint32_t tot;
                const uint32_t r = wg_rank(f, tot, wcnt);
                if (f) expl[E + r] = (uint16_t)q;
                E += tot;
            }
            __syncthreads();
            D = 0;
            for (uint32_t s0 = 0; s0 < 8 * E; s0 += kChunk) {
                // kPer child slots per thread (slot s0 + u * kThreads + t),
                // their label and neighbour loads all in flight together
                uint32_t opv[kPer], lblv[kPer], rk[kPer];
                uint64_t bal[kPer];
#pragma unroll
                for (uint32_t u = 0; u < kPer; u++) {
                    const uint32_t s = s0 + u * kThreads + t;
                    const bool valid = s < 8 * E;
                    uint32_t op = kNone, lbl = 0;
                    if (valid) {
                        const uint32_t q = expl[s >> 3], j = 8 * q + (s & 7);
                        const uint32_t cx = compact3(j), cy = compact3(j >> 1), cz = compact3(j >> 2);
                        lbl = label_at(a, b, lab, m, j);
                        const uint32_t par = lab[lvl_off(l) + q];
                        uint32_t nv[3];
                        bool nok[3];
#pragma unroll
                        for (uint32_t ax = 0; ax < 3; ax++) {
                            const uint32_t c = ax == 0 ? cx : (ax == 1 ? cy : cz);
                            if ((c & 1u) == 0) {  // the same-level node at -1
                                nok[ax] = c > 0;
                                const uint32_t d = nok[ax] ? 1u : 0u;
                                nv[ax] = label_at(a, b, lab, m,
                                                  morton(cx - (ax == 0 ? d : 0u), cy - (ax == 1 ? d : 0u),
                                                         cz - (ax == 2 ? d : 0u)));
                            } else {  // the parent of the node at +1
                                nok[ax] = c + 1 < G;
                                const uint32_t d = nok[ax] ? 1u : 0u;
                                nv[ax] = lab[lvl_off(l) + morton((cx + (ax == 0 ? d : 0u)) >> 1,
                                                                 (cy + (ax == 1 ? d : 0u)) >> 1,
                                                                 (cz + (ax == 2 ? d : 0u)) >> 1)];
                            }
                        }
                        op = par == lbl ? csv::kRp
                                        : (nok[0] && nv[0] == lbl
                                               ? csv::kRx
                                               : (nok[1] && nv[1] == lbl ? csv::kRy
                                                                         : (nok[2] && nv[2] == lbl ? csv::kRz : csv::kPa)));
                        const uint32_t stop =
                            (m >= 1 && ((cstb[(lvl_off(m) + j) >> 5] >> ((lvl_off(m) + j) & 31)) & 1u)) ? 1u : 0u;
                        op |= stop << 8;
                    }
                    opv[u] = op;
                    lblv[u] = lbl;
                    bal[u] = __ballot(op != kNone && (op & 0xFFu) == csv::kPa);
                    if (L == 0) wcnt4[u][w] = (uint32_t)__popcll(bal[u]);
                }
                __syncthreads();
                // candidates ranked in slot order
                uint32_t nc = 0;
#pragma unroll
                for (uint32_t u = 0; u < kPer; u++) {
                    uint32_t bw = 0, tu = 0;
#pragma unroll
                    for (uint32_t k = 0; k < kThreads / 64; k++) {
                        const uint32_t c = wcnt4[u][k];
                        bw += k < w ? c : 0u;
                        tu += c;
                    }
                    rk[u] = nc + bw + mbcnt(bal[u]);
                    nc += tu;
                    if ((bal[u] >> L) & 1ull) c_lab[rk[u]] = lblv[u];
                }
                __syncthreads();
                pc.stop(m == 0 ? 2 : 1);  // reuse operations
                if (w == 0) {
                    // palette operations in order: P_0, else the smallest delta
                    // among the 16 entries before it, else append.  Lane k
                    // holds candidate c0 + k and receives its operation.
                    for (uint32_t c0 = 0; c0 < nc; c0 += 64) {
                        const uint32_t lv = c0 + L < nc ? c_lab[c0 + L] : 0u;
                        const uint32_t cn = min(64u, nc - c0);
                        uint32_t mine = 0;
                        for (uint32_t k = 0; k < cn; k++) {
                            const uint32_t lc = (uint32_t)__builtin_amdgcn_readlane((int)lv, (int)k);
                            const uint64_t mm = __ballot(L <= 16 && L < P && win == lc);
                            uint32_t o;
                            if (mm & 1ull) {
                                o = csv::kP0;
                            } else if (mm) {
                                o = csv::kPd;
                                if (L == 0) dels[D] = (uint8_t)(__builtin_ctzll(mm) - 1);
                                D++;
                            } else {
                                o = csv::kPa;
                                // lane i takes lane i - 1's entry (DPP wave shift right by one)
                                win = (uint32_t)__builtin_amdgcn_update_dpp((int)win, (int)win, 0x138, 0xF, 0xF, false);
                                if (L == 0) {
                                    win = lc;
                                    pal[P] = lc;
                                }
                                P++;
                            }
                            mine = L == k ? o : mine;
                        }
                        if (c0 + L < nc) c_op[c0 + L] = (uint8_t)mine;
                    }
                }
                __syncthreads();
                pc.stop(3);  // palette operations
#pragma unroll
                for (uint32_t u = 0; u < kPer; u++) {
                    const uint32_t s = s0 + u * kThreads + t;
                    if (opv[u] != kNone) {
                        const uint32_t o = ((bal[u] >> L) & 1ull) ? c_op[rk[u]] : (opv[u] & 0xFFu);
                        ops[s] = (uint8_t)(o | ((opv[u] >> 8) << 3));
                    }
                }
            }
            if (t == 0) share[0] = D;
            __syncthreads();
            const uint32_t nd = share[0];
            // a level's delta nibbles precede its operation nibbles
            for (uint32_t i = t; i < nd; i += kThreads) sym[base + i] = dels[i];
            for (uint32_t i = t; i < 8 * E; i += kThreads) sym[base + nd + i] = ops[i];
            base += nd + 8 * E;
            if (t == 0) s_cum[m] = base;
            __syncthreads();
        }
        pc.stop(4);  // level ends
        const uint32_t n = base, leaf = s_cum[1];
        // the sampled bricks' symbol histograms (the frequency tables, Sec. 3.4)
        if (id % a.sample_stride == 0) {
            if (t < 32) hist_l[t] = 0;
            __syncthreads();
            for (uint32_t i = t; i < n; i += kThreads) atomicAdd(&hist_l[(i >= leaf ? 16u : 0u) + sym[i]], 1u);
            __syncthreads();
            if (t < 32 && hist_l[t]) atomicAdd(&a.hist[t], (unsigned long long)hist_l[t]);
        }
        // symbols and palette to the arena, for the rANS kernel
        if (w == 0 && L == 0) share[3] = P;
        __syncthreads();
        const uint32_t Pn = share[3];
        const uint64_t bytes = (((uint64_t)n + 3) & ~3ull) + 4ull * Pn;
        if (t == 0) {
            const uint64_t off = atomicAdd(a.sarena_top, (unsigned long long)bytes);
            a.soff[id] = off;
            a.sn[id] = n;
            a.sp[id] = Pn;
            for (int m = 0; m < kN; m++) a.scum[(size_t)kN * id + m] = s_cum[m];
            share[4] = (uint32_t)off;
            share[5] = (uint32_t)(off >> 32);
        }
        __syncthreads();
        const uint64_t off = ((uint64_t)share[5] << 32) | share[4];
        if (off + bytes <= a.sarena_cap) {
            uint8_t *d = a.sarena + off;
            // whole dwords (the arena offset and the scratch are 4-byte aligned;
            // the bytes past n are padding that the rANS kernel does not read)
            const uint32_t *sw = reinterpret_cast<const uint32_t *>(sym);
            uint32_t *dw = reinterpret_cast<uint32_t *>(d);
            for (uint32_t i = t; i < (n + 3) / 4; i += kThreads) dw[i] = sw[i];
            uint32_t *dp = reinterpret_cast<uint32_t *>(d + ((n + 3) & ~3u));
            for (uint32_t i = t; i < Pn; i += kThreads) dp[i] = pal[i];
        }
        __syncthreads();
        pc.stop(5);  // arena
    }
    pc.flush();
}

// Interleaved rANS and the record of one brick per wavefront (Sec. 3.3):
// symbol i to state i mod W, from the last symbol to the first; the words
// of a step are placed by ballot rank in descending lane order, then
// reversed into the record so that the decoder reads them in symbol order.
__global__ __launch_bounds__(kThreads) void rans_kernel(EncArgs a) {
    __shared__ uint32_t tf[2][16], tc[2][16];
    __shared__ double trcp[2][16];
    const uint32_t t = threadIdx.x, L = lane(), w = t >> 6;
    if (t < 32) {
        tf[t >> 4][t & 15] = a.f[t >> 4][t & 15];
        tc[t >> 4][t & 15] = a.c[t >> 4][t & 15];
        trcp[t >> 4][t & 15] = 1.0 / (double)a.f[t >> 4][t & 15];
    }
    __syncthreads();
    constexpr uint32_t kWaves = kThreads / 64;
    uint16_t *words = reinterpret_cast<uint16_t *>(a.wscratch + ((size_t)blockIdx.x * kWaves + w) * kWordsScratch);
    const uint64_t xmax_unit = (uint64_t)((csv::kRansLower >> a.bits) << 16);
    const uint32_t hdr = csv::record_header_words(kN);
    for (uint32_t id = blockIdx.x * kWaves + w; id < a.n_items; id += gridDim.x * kWaves) {
        const uint32_t n = a.sn[id], Pn = a.sp[id], leaf = a.scum[(size_t)kN * id + 1];
        const uint8_t *sym = a.sarena + a.soff[id];
        const uint32_t *pal = reinterpret_cast<const uint32_t *>(sym + ((n + 3) & ~3u));
        const uint32_t W = lanes_for(n, a.lane_k, a.lane_max);
        uint32_t x = csv::kRansLower, pushed = 0;
        if (n) {
            constexpr int kBlk = 16;
            for (int64_t s_hi = (int64_t)((n - 1) / W); s_hi >= 0; s_hi -= kBlk) {
                uint32_t sy[kBlk];
#pragma unroll
                for (int k = 0; k < kBlk; k++) {
                    const int64_t s = s_hi - k;
                    const uint32_t i = (uint32_t)s * W + L;
                    sy[k] = (s >= 0 && L < W && i < n) ? (uint32_t)sym[i] : 0xFFu;
                }
#pragma unroll
                for (int k = 0; k < kBlk; k++) {
                    const int64_t s = s_hi - k;
                    const uint32_t i = (uint32_t)s * W + L;
                    const bool act = sy[k] != 0xFFu;  // (false for every lane once s < 0)
                    bool emit = false;
                    uint32_t wd = 0;
                    if (act) {
                        const uint32_t tb = i >= leaf ? 1u : 0u;
                        const uint32_t f = tf[tb][sy[k]], c = tc[tb][sy[k]];
                        uint32_t v = x;
                        if ((uint64_t)v >= xmax_unit * f) {
                            emit = true;
                            wd = v & 0xFFFFu;
                            v >>= 16;
                        }
                        // v / f: a double reciprocal is within one of the
                        // quotient; the remainder corrects it
                        uint32_t q = (uint32_t)((double)v * trcp[tb][sy[k]]);
                        int64_t r = (int64_t)v - (int64_t)q * f;
                        if (r < 0) {
                            q--;
                            r += f;
                        } else if (r >= (int64_t)f) {
                            q++;
                            r -= f;
                        }
                        x = (q << a.bits) + (uint32_t)r + c;
                    }
                    // the host order within a step is descending lanes
                    const uint64_t em = __ballot(emit);
                    if (emit) words[pushed + (uint32_t)__popcll(L == 63 ? 0ull : (em >> (L + 1)))] = (uint16_t)wd;
                    pushed += (uint32_t)__popcll(em);
                }
            }
        }
        const uint32_t nw = pushed;
        const uint32_t size = (4 * (hdr + Pn + W) + 2 * nw + 3) & ~3u;
        uint32_t lo = 0, hi = 0;
        if (L == 0) {
            const uint64_t o = atomicAdd(a.arena_top, (unsigned long long)size);
            a.sizes[id] = size;
            a.aoff[id] = o;
            lo = (uint32_t)o;
            hi = (uint32_t)(o >> 32);
        }
        const uint64_t off = ((uint64_t)(uint32_t)__shfl((int)hi, 0) << 32) | (uint32_t)__shfl((int)lo, 0);
        // this wavefront's word stores before its own loads of them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (off + size <= a.arena_cap) {
            uint32_t *r = reinterpret_cast<uint32_t *>(a.arena + off);
            if (L == 0) {
                r[0] = Pn;
                r[1] = W;
                r[2] = nw;
                for (int m = 0; m < kN; m++) r[3 + m] = a.scum[(size_t)kN * id + m];
            }
            for (uint32_t i = L; i < Pn; i += 64) r[hdr + i] = pal[i];
            if (L < W) r[hdr + Pn + L] = x;
            uint16_t *wr = reinterpret_cast<uint16_t *>(r + hdr + Pn + W);
            for (uint32_t q = L; q < nw; q += 64) wr[q] = words[nw - 1 - q];
            if (L == 0 && (nw & 1u)) wr[nw] = 0;
        }
        // the words region is reused by this wavefront's next brick
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// exclusive scan of the record sizes into the container's u64 index
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *sizes, uint32_t n, uint64_t *index) {
    __shared__ uint64_t part[1024];
    const uint32_t t = threadIdx.x;
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < n; b0 += 1024) {
        const uint64_t v = b0 + t < n ? sizes[b0 + t] : 0;
        part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint64_t o = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += o;
            __syncthreads();
        }
        if (b0 + t < n) index[b0 + t] = carry + part[t] - v;
        carry += part[1023];
        __syncthreads();
    }
    if (t == 0) index[n] = carry;
}

// records from the arena to their place in the container's record area
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *arena, const uint64_t *aoff, const uint32_t *sizes,
                                                   const uint64_t *index, uint32_t n, uint8_t *records) {
    for (uint32_t id = blockIdx.x; id < n; id += gridDim.x) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(arena + aoff[id]);
        uint32_t *dst = reinterpret_cast<uint32_t *>(records + index[id]);
        const uint32_t nd = sizes[id] / 4;
        for (uint32_t i = threadIdx.x; i < nd; i += 256) dst[i] = src[i];
    }
}

// a device buffer that grows on demand
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool ensure(size_t need) {
        need = std::max<size_t>(need, 256);
        if (bytes >= need) return true;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, need) != hipSuccess) return false;
        bytes = need;
        return true;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const {
        return reinterpret_cast<T *>(p);
    }
};

// per device: the buffers of the last call, kept for the next one
struct EncCache {
    std::mutex mu;
    DevBuf scratch, wscratch, hist, sizes, aoff, top, arena, dblob, sarena, smeta;
    uint8_t *h_pin = nullptr;  // pinned staging of the container on its way to host memory
    size_t h_pin_bytes = 0;
    void release() {
        scratch.release();
        wscratch.release();
        sarena.release();
        smeta.release();
        hist.release();
        sizes.release();
        aoff.release();
        top.release();
        arena.release();
        dblob.release();
        if (h_pin) (void)hipHostFree(h_pin);
        h_pin = nullptr;
        h_pin_bytes = 0;
    }
};
constexpr int kMaxDevices = 64;
EncCache *g_cache[kMaxDevices] = {};
std::mutex g_cache_mu;

EncCache *cache_for(int device) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (!g_cache[device]) g_cache[device] = new (std::nothrow) EncCache;
    return g_cache[device];
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

extern "C" int csv_encode_volume_gpu(const uint32_t *labels, uint32_t nx, uint32_t ny, uint32_t nz,
                                     const csv_encode_opts *opts, int device, void *stream, uint8_t **blob,
                                     size_t *blob_bytes) {
    if (!labels || !blob || !blob_bytes || !nx || !ny || !nz) return CSV_EINVAL;
    csv_encode_opts o;
    csv_encode_opts_default(&o);
    if (opts) o = *opts;
    if (o.brick_log2 != (uint32_t)kN || o.scale_bits < 8 || o.scale_bits > 12 || o.lane_k < 1 || o.lane_max < 1 ||
        o.lane_max > 64 || (o.lane_max & (o.lane_max - 1)) || o.tables > 2 || o.coding != 0)
        return CSV_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev || device >= kMaxDevices)
        return CSV_EINVAL;
    const uint32_t nbx = (nx + 31) / 32, nby = (ny + 31) / 32, nbz = (nz + 31) / 32;
    const uint64_t B64 = (uint64_t)nbx * nby * nbz;
    if (B64 >= (1ull << 32)) return CSV_ERANGE;
    const uint32_t B = (uint32_t)B64;
    const uint32_t stride = o.sample_stride ? o.sample_stride : (B64 > (1ull << 20) ? 4096u : 512u);
    DeviceGuard g(device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cu < 1) cu = 1;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(B64, (uint64_t)cu * 5);  // symbols kernel: 5 workgroups per CU
    const uint64_t raw = (uint64_t)nx * ny * nz * 4;
    uint64_t cap = std::max<uint64_t>(16ull << 20, raw / 8);
    EncCache *ec = cache_for(device);
    if (!ec) return CSV_ENOMEM;
    std::lock_guard<std::mutex> lk(ec->mu);  // one compression per device at a time
    DevBuf &scratch = ec->scratch, &wscratch = ec->wscratch, &hist = ec->hist, &sizes = ec->sizes,
           &aoff = ec->aoff, &top = ec->top, &arena = ec->arena, &dblob = ec->dblob, &sarena = ec->sarena,
           &smeta = ec->smeta;
    const uint32_t waves2 = (uint32_t)std::min<uint64_t>((B64 + 3) / 4, (uint64_t)cu * 4) * 4;
    uint64_t scap = std::max<uint64_t>(16ull << 20, raw / 8);
    if (!scratch.ensure(kScratch * grid) || !wscratch.ensure(kWordsScratch * waves2) || !hist.ensure(32 * 8) ||
        !sizes.ensure(4ull * B) || !aoff.ensure(8ull * B) || !top.ensure(16) || !arena.ensure(cap) ||
        !sarena.ensure(scap) || !smeta.ensure((8ull + 4 + 4 + 4 * kN) * B))
        return CSV_ENOMEM;
    cap = arena.bytes;
    scap = sarena.bytes;
    EncArgs a;
    std::memset(&a, 0, sizeof(a));
    a.vol = labels;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.nbx = nbx;
    a.nby = nby;
    a.n_items = B;
    a.sample_stride = stride;
    a.bits = o.scale_bits;
    a.lane_k = o.lane_k;
    a.lane_max = o.lane_max;
    a.scratch = scratch.as<uint8_t>();
    a.wscratch = wscratch.as<uint8_t>();
    a.hist = hist.as<unsigned long long>();
    a.arena_top = top.as<unsigned long long>();
    a.sarena_top = top.as<unsigned long long>() + 1;
    a.sizes = sizes.as<uint32_t>();
    a.aoff = aoff.as<uint64_t>();
    a.soff = smeta.as<uint64_t>();
    a.sn = reinterpret_cast<uint32_t *>(a.soff + B);
    a.sp = a.sn + B;
    a.scum = a.sp + B;
    // symbols of every brick (and the sampled bricks' histograms); a second
    // pass with the exact arena size if they did not fit
    uint64_t used = 0;
    for (int pass = 0; pass < 2; pass++) {
        a.sarena = sarena.as<uint8_t>();
        a.sarena_cap = scap;
        if (hipMemsetAsync(a.hist, 0, 32 * 8, s) != hipSuccess || hipMemsetAsync(a.sarena_top, 0, 8, s) != hipSuccess)
            return CSV_EHIP;
        hipLaunchKernelGGL(symbols_kernel, dim3(grid), dim3(kThreads), 0, s, a);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&used, a.sarena_top, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return CSV_EHIP;
        if (used <= scap) break;
        scap = used;
        if (pass == 1 || !sarena.ensure(scap)) return CSV_ENOMEM;
    }
    uint64_t cnt[2][16];
    if (hipMemcpy(cnt, a.hist, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess) return CSV_EHIP;
    if (o.tables == 1)  // one table for all symbols
        for (int q = 0; q < 16; q++) cnt[0][q] = cnt[1][q] = cnt[0][q] + cnt[1][q];
    uint32_t f[2][16];
    for (int k = 0; k < 2; k++) {
        csv::normalize_counts(cnt[k], 1u << o.scale_bits, f[k]);
        uint32_t c = 0;
        for (int q = 0; q < 16; q++) {
            a.f[k][q] = f[k][q];
            a.c[k][q] = c;
            c += f[k][q];
        }
    }
    // rANS and records, a wavefront per brick; a second pass with the exact
    // arena size if the records did not fit
    for (int pass = 0; pass < 2; pass++) {
        a.arena = arena.as<uint8_t>();
        a.arena_cap = cap;
        if (hipMemsetAsync(a.arena_top, 0, 8, s) != hipSuccess) return CSV_EHIP;
        hipLaunchKernelGGL(rans_kernel, dim3(waves2 / 4), dim3(kThreads), 0, s, a);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&used, a.arena_top, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return CSV_EHIP;
        if (used <= cap) break;
        cap = used;
        if (pass == 1 || !arena.ensure(cap)) return CSV_ENOMEM;
    }
    // container: header (host), index (device scan), records (device copy)
    const uint64_t rs = csv::record_area_offset(B);
    const uint64_t total = rs + used;
    if (!dblob.ensure(total)) return CSV_ENOMEM;
    uint64_t *index = reinterpret_cast<uint64_t *>(dblob.as<uint8_t>() + csv::kHeaderBytes);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, a.sizes, B, index);
    hipLaunchKernelGGL(pack_kernel, dim3(std::min<uint32_t>(B, (uint32_t)cu * 8)), dim3(256), 0, s,
                       (const uint8_t *)a.arena, (const uint64_t *)a.aoff, (const uint32_t *)a.sizes,
                       (const uint64_t *)index, B, dblob.as<uint8_t>() + rs);
    if (ec->h_pin_bytes < total) {
        if (ec->h_pin) (void)hipHostFree(ec->h_pin);
        ec->h_pin = nullptr;
        ec->h_pin_bytes = 0;
        if (hipHostMalloc(reinterpret_cast<void **>(&ec->h_pin), total, hipHostMallocDefault) != hipSuccess)
            return CSV_ENOMEM;
        ec->h_pin_bytes = total;
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(ec->h_pin, dblob.p, total, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return CSV_EHIP;
    uint8_t *out = static_cast<uint8_t *>(std::malloc(total));
    if (!out) return CSV_ENOMEM;
    // into fresh host pages: several threads share the page faults and the copy
    const unsigned nt = total >= (8u << 20) ? 8u : 1u;
    const size_t chunk = (total + nt - 1) / nt;
    std::vector<std::thread> th;
    for (unsigned k = 1; k < nt; k++) {
        const size_t o = k * chunk, len = o < total ? std::min(chunk, total - o) : 0;
        if (len) th.emplace_back([=] { std::memcpy(out + o, ec->h_pin + o, len); });
    }
    std::memcpy(out, ec->h_pin, std::min(chunk, total));
    for (auto &x : th) x.join();
    csv::VolumeHeader h;
    std::memset(&h, 0, sizeof(h));
    h.magic = csv::kMagic;
    h.version = csv::kVersion;
    h.nx = nx;
    h.ny = ny;
    h.nz = nz;
    h.brick_log2 = (uint32_t)kN;
    h.nbx = nbx;
    h.nby = nby;
    h.nbz = nbz;
    h.n_bricks = B;
    h.scale_bits = o.scale_bits;
    h.lane_k = o.lane_k;
    h.lane_max = o.lane_max;
    h.sample_stride = stride;
    for (int k = 0; k < 2; k++)
        for (int q = 0; q < 16; q++) h.freq[k][q] = (uint16_t)f[k][q];
    std::memcpy(out, &h, sizeof(h));
    const uint64_t idx_end = csv::kHeaderBytes + 8ull * (B + 1);
    std::memset(out + idx_end, 0, rs - idx_end);  // padding before the record area
    *blob = out;
    *blob_bytes = total;
    return CSV_OK;
}

extern "C" int csv_encode_gpu_release(int device) {
    if (device < 0 || device >= kMaxDevices) return CSV_EINVAL;
    EncCache *ec;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        ec = g_cache[device];
    }
    if (!ec) return CSV_OK;
    DeviceGuard g(device);
    std::lock_guard<std::mutex> lk(ec->mu);
    (void)hipDeviceSynchronize();
    ec->release();
    return CSV_OK;
}

#ifdef CSV_PHASE_TIMING
// install (or clear, with NULL) a device buffer of 8 u64 clocks per workgroup
extern "C" int csv_debug_enc_phase_buffer(uint64_t *dev_buf) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_enc_phase), &dev_buf, sizeof(dev_buf)) == hipSuccess ? CSV_OK : CSV_EHIP;
}
#endif
