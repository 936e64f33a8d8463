// Decoder for every brick edge 2^N, N = 1..6, with interleaved rANS or raw
// nibbles (Sec. 3.3, Sec. 3.4, Alg. 1; Table 1's brick sizes and its
// variant without rANS).
//
// One 256-thread workgroup per request, persistent over the requests:
//   1. the record header is read and checked (as the pool's loader does);
//   2. the first c_t symbols of the brick are decoded into the workgroup's
//      scratch, one byte per symbol: rANS by wavefront 0 with the W
//      interleaved states in lockstep (symbol i -> state i mod W, words
//      handed out in lane order by ballot rank), or raw nibbles by every
//      thread;
//   3. levels N-1 .. t are replayed one after another (Alg. 1): the
//      expanded parents of a level are listed in Morton order (a block
//      scan of their flags), non-expanded parents pass their value to their
//      8 children, and each thread takes one expanded parent at a time: a
//      block scan of the P_a and P_delta counts of its 8 operations gives
//      its palette position and its first delta, so the children come out
//      in parallel.  A reference to the same-level neighbour at -1 is left
//      as a mark and followed once the level is complete (the referenced
//      child lies one coordinate step earlier, so a chain ends within three
//      links);
//   4. level t goes through the palette to the dense (b >> t)^3 output.
// Levels are u32 palette indices in a global-memory scratch area per
// workgroup (L2-resident), so that the same code covers 64^3 bricks,
// whose finest level does not fit LDS.  Malformed data is reported in the
// pool's error word and the request's output is zero-filled.
#include "csv_generic.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/csv.h"
#include "csv_format.hpp"

namespace csv {
namespace {

constexpr uint32_t kGT = 256;                 // threads per workgroup
constexpr uint32_t kGMark = 0x80000000u;      // a level entry that names a same-level node to copy

__host__ __device__ constexpr uint64_t pow8(uint32_t e) { return 1ull << (3 * e); }
// level m of a brick of edge 2^N starts at this node: levels stored finest first
__host__ __device__ constexpr uint64_t level_off(uint32_t N, uint32_t m) {
    uint64_t o = 0;
    for (uint32_t j = 0; j < m; j++) o += pow8(N - j);
    return o;
}
__host__ __device__ constexpr uint64_t all_nodes(uint32_t N) { return level_off(N, N + 1); }
__host__ __device__ constexpr uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

// Morton index of (x, y, z): bit 3i of x, bit 3i + 1 of y, bit 3i + 2 of z
__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
        m |= (((x >> i) & 1u) << (3 * i)) | (((y >> i) & 1u) << (3 * i + 1)) | (((z >> i) & 1u) << (3 * i + 2));
    return m;
}
__device__ __forceinline__ void unmorton3(uint32_t m, uint32_t c[3]) {
    c[0] = c[1] = c[2] = 0;
#pragma unroll
    for (int i = 0; i < 6; i++) {
        c[0] |= ((m >> (3 * i)) & 1u) << i;
        c[1] |= ((m >> (3 * i + 1)) & 1u) << i;
        c[2] |= ((m >> (3 * i + 2)) & 1u) << i;
    }
}

// exclusive prefix sum of v over the workgroup; *total: the sum of all.
// sh: 4 words of LDS.  Every thread must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const uint32_t L = __lane_id(), w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (L >= (uint32_t)d) x += y;
    }
    if (L == 63) sh[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t k = 0; k < kGT / 64; k++) {
        const uint32_t t = sh[k];
        before += k < w ? t : 0u;
        all += t;
    }
    __syncthreads();  // sh is reused by the next scan
    total = all;
    return before + x - v;
}

// A device address as a pointer into the global address space, so that the
// accesses compile to global (not flat) instructions: a flat access also
// counts on lgkmcnt, and the LDS waits of the block scans would wait for it.
// The addresses travel as integers (kernel arguments, the request record in
// LDS), so that nothing turns them back into generic pointers.
template <class T>
__device__ __forceinline__ T *gmem(uint64_t v) {
    return (T *)(__attribute__((address_space(1))) T *)v;
}

struct GReq {
    uint64_t rec;  // record address
    uint64_t dst;  // output address
    uint32_t P, W, nw, t, vol, id, raw, count;
    uint32_t cum[kMaxLog2];
    int err;           // first error found for this request
    uint32_t fill;     // 1: every output label is fill_v
    uint32_t fill_v;
};

__device__ __forceinline__ void g_report(const GenericArgs &a, uint32_t rq, int code, uint32_t who) {
    if (atomicCAS(a.err, 0, code) == 0) a.err[1] = (int)who;
    if (a.req_err) a.req_err[rq] = code;
}

template <uint32_t N>
__global__ __launch_bounds__(kGT) void generic_kernel(GenericArgs a) {
    constexpr uint32_t hdr = 3 + N;
    __shared__ GReq R;
    __shared__ uint32_t sh[kGT / 64];
    __shared__ int bad;
    extern __shared__ uint32_t glut[];  // the decode tables when a.lut_lds_words > 0
    const uint32_t tid = threadIdx.x;
    for (uint32_t e = tid; e < a.lut_lds_words; e += kGT) glut[e] = a.luts[e];
    __syncthreads();
    uint8_t *base = gmem<uint8_t>(a.scratch + (uint64_t)blockIdx.x * a.scratch_per_group);
    uint8_t *sym = base;
    uint32_t *lev = reinterpret_cast<uint32_t *>(base + align256(a.sym_cap));
    uint8_t *flg = reinterpret_cast<uint8_t *>(lev) + align256(4 * all_nodes(N));
    uint32_t *lst = reinterpret_cast<uint32_t *>(flg + align256(all_nodes(N)));
    // Every branch on `bad` uses this: the flag as all threads read it
    // between two barriers (so that no thread sets it while others read).
    auto agree = [&]() -> bool {
        __syncthreads();
        const bool b = bad != 0;
        __syncthreads();
        return b;
    };
    for (uint32_t rq = blockIdx.x; rq < a.n; rq += gridDim.x) {
        if (tid == 0) {
            // 1. the request and its record header
            R.err = 0;
            R.fill = 0;
            R.count = 0;
            R.dst = 0;
            R.id = a.ids[rq];
            R.t = a.lods ? (uint32_t)a.lods[rq] : a.lod_scalar;
            if (R.t > N) {
                R.err = CSV_ERANGE;
            } else {
                const uint32_t G = (1u << N) >> R.t;
                R.count = G * G * G;
                R.dst = a.out + 4 * (a.out_off ? a.out_off[rq] : (uint64_t)rq * R.count);
                if (R.id >= a.n_bricks) {
                    R.err = CSV_ERANGE;
                } else {
                    const uint32_t *rec = gmem<const uint32_t>(a.rec_ptr[R.id]);
                    const uint64_t size = a.rec_size[R.id];
                    R.rec = a.rec_ptr[R.id];
                    R.vol = a.rec_vol[R.id];
                    R.raw = a.vol_raw[R.vol];
                    R.P = rec[0];
                    R.W = rec[1];
                    R.nw = rec[2];
                    bool ok = true;
                    for (uint32_t m = 0; m < N; m++) {
                        R.cum[m] = rec[3 + m];
                        if (m > 0 && R.cum[m] > R.cum[m - 1]) ok = false;
                    }
                    const uint32_t c0 = R.cum[0];
                    ok = ok && R.P >= 1 && c0 <= a.sym_cap && (c0 == 0 ? R.P == 1 : R.P >= 2);
                    ok = ok && (R.raw ? (R.W == 0 && R.nw == (c0 + 3) / 4)
                                      : (R.W <= 64 && (R.W & (R.W - 1)) == 0 && (c0 > 0) == (R.W > 0)));
                    ok = ok && 4ull * ((uint64_t)hdr + R.P + R.W) + 2ull * R.nw <= size;
                    if (!ok) {
                        R.err = CSV_ECORRUPT;
                    } else if (R.t == N || c0 == 0) {  // coarsest level, or a uniform brick: palette[0]
                        R.fill = 1;
                        R.fill_v = rec[hdr];
                    }
                }
            }
            bad = 0;
        }
        __syncthreads();
        const uint32_t t = R.t, P = R.P, W = R.W;
        const uint32_t *rec = gmem<const uint32_t>(R.rec);
        const uint32_t *pal = rec + hdr;
        if (R.err == 0 && R.fill == 0) {
            // 2. entropy decode of the first n symbols
            const uint32_t n = t < N ? R.cum[t] : 0u;
            const uint16_t *words = reinterpret_cast<const uint16_t *>(rec + hdr + P + W);
            if (R.raw) {
                for (uint32_t i = tid; i < n; i += kGT) sym[i] = (uint8_t)((words[i >> 2] >> (4 * (i & 3))) & 15u);
                // a complete decode finds the last word's unused nibbles zero
                if (tid == 0 && t == 0 && (R.cum[0] & 3) && (words[R.nw - 1] >> (4 * (R.cum[0] & 3))) != 0) bad = 1;
            } else if (tid < 64) {
                // the rANS steps, with the decode tables in LDS or in global
                // memory (two instantiations, so that each reads one address
                // space)
                auto rans = [&](auto luts) {
                    const uint32_t L = tid, vol = R.vol;
                    const uint32_t sbits = a.vol_bits[vol], lutn = 1u << sbits, mask = lutn - 1u;
                    const auto lut = luts + a.lut_off[vol];
                    const uint32_t leaf = N >= 2 ? R.cum[1] : 0u;
                    uint32_t x = L < W ? rec[hdr + P + L] : 0u;
                    uint32_t cursor = 0;
                    bool fail = false;
                    const uint32_t steps = W ? (n + W - 1) / W : 0u;
                    for (uint32_t s = 0; s < steps; s++) {
                        const uint32_t i = s * W + L;
                        const bool act = L < W && i < n;
                        bool need = false;
                        uint32_t v = 0;
                        if (act) {
                            const uint32_t e = lut[(i >= leaf ? lutn : 0u) + (x & mask)];
                            v = e & 15u;
                            x = (e >> 20) * (x >> sbits) + ((e >> 8) & 0xFFFu);
                            need = x < kRansLower;
                        }
                        const uint64_t bal = __ballot(need);
                        const uint32_t cnt = (uint32_t)__popcll(bal);
                        if (cursor + cnt > R.nw) {  // words past the end of the stream
                            fail = true;
                            break;
                        }
                        if (need) {
                            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                            x = (x << 16) | words[cursor + rank];
                        }
                        cursor += cnt;
                        if (act) sym[i] = (uint8_t)v;
                    }
                    // a complete decode ends in the encoder's initial states with every word read
                    if (!fail && t == 0) fail = __ballot(L < W && x != kRansLower) != 0 || cursor != R.nw;
                    if (fail && L == 0) bad = 1;
                };
                if (a.lut_lds_words)
                    rans((const __attribute__((address_space(3))) uint32_t *)glut);
                else
                    rans((const __attribute__((address_space(1))) uint32_t *)a.luts);
            }
            // 3. replay, levels N-1 .. t
            if (tid == 0) {
                lev[level_off(N, N)] = 0;  // the root: palette[0]
                flg[level_off(N, N)] = 1;
            }
            bool stop = agree();
            uint32_t ipl = 0;  // P_a operations of the levels done
            for (int m = (int)N - 1; m >= (int)t && !stop; m--) {
                const uint32_t np = (uint32_t)pow8(N - (uint32_t)m - 1);  // parents
                const uint32_t *pl = lev + level_off(N, (uint32_t)m + 1);
                const uint8_t *pf = flg + level_off(N, (uint32_t)m + 1);
                uint32_t *cl = lev + level_off(N, (uint32_t)m);
                uint8_t *cf = flg + level_off(N, (uint32_t)m);
                const uint32_t seg0 = m == (int)N - 1 ? 0u : R.cum[m + 1], seg1 = R.cum[m];
                // expanded parents in Morton order
                uint32_t E = 0;
                for (uint32_t q0 = 0; q0 < np; q0 += kGT) {
                    const uint32_t q = q0 + tid;
                    const uint32_t e = q < np ? (uint32_t)pf[q] : 0u;
                    uint32_t tot;
                    const uint32_t ex = block_excl_scan(e, sh, tot);
                    if (e) lst[E + ex] = q;
                    E += tot;
                }
                // children of the other parents take the parent's value
                for (uint32_t q = tid; q < np; q += kGT)
                    if (!pf[q]) {
                        const uint32_t v = pl[q];
#pragma unroll
                        for (uint32_t k = 0; k < 8; k++) {
                            cl[8 * q + k] = v;
                            cf[8 * q + k] = 0;
                        }
                    }
                if ((uint64_t)seg0 + 8ull * E > seg1) {  // E is the same in every thread
                    if (tid == 0) bad = 1;
                    break;
                }
                const uint32_t nd = seg1 - seg0 - 8 * E, ops0 = seg0 + nd;  // deltas precede the operations
                const uint32_t G = 1u << (N - (uint32_t)m);                   // grid of the children
                uint32_t pa_c = 0, pd_c = 0;
                for (uint32_t r0 = 0; r0 < E; r0 += kGT) {
                    const uint32_t r = r0 + tid;
                    const bool act = r < E;
                    const uint32_t q = act ? lst[r] : 0u;
                    uint32_t ops[8];
                    uint32_t npa = 0, npd = 0;
#pragma unroll
                    for (uint32_t k = 0; k < 8; k++) {
                        ops[k] = act ? (uint32_t)sym[ops0 + 8 * r + k] : 0u;
                        npa += (ops[k] & 7u) == (uint32_t)kPa ? 1u : 0u;
                        npd += (ops[k] & 7u) == (uint32_t)kPd ? 1u : 0u;
                    }
                    uint32_t tot;
                    const uint32_t ex = block_excl_scan(npa | (npd << 16), sh, tot);
                    if (act) {
                        uint32_t ip = ipl + pa_c + (ex & 0xFFFFu);  // index of the last palette entry used
                        uint32_t dp = seg0 + pd_c + (ex >> 16);     // next delta nibble
                        const uint32_t pv = pl[q];
                        bool fail = false;
#pragma unroll
                        for (uint32_t k = 0; k < 8; k++) {
                            const uint32_t op = ops[k] & 7u, stop = ops[k] >> 3, j = 8 * q + k;
                            uint32_t v = 0;
                            if (stop && m == 0) fail = true;  // leaf children carry stop 0
                            if (op == (uint32_t)kRp) {
                                v = pv;
                            } else if (op >= (uint32_t)kRx && op <= (uint32_t)kRz) {
                                const uint32_t ax = op - (uint32_t)kRx;
                                uint32_t c[3];
                                unmorton3(j, c);
                                if ((c[ax] & 1u) == 0) {  // the same-level node at -1: copied once the level is done
                                    if (c[ax] == 0) fail = true;
                                    c[ax] -= 1u;
                                    v = kGMark | morton3(c[0], c[1], c[2]);
                                } else {  // the parent of the node at +1
                                    if (c[ax] + 1 >= G) fail = true;
                                    c[ax] += 1u;
                                    v = fail ? 0u : pl[morton3(c[0] >> 1, c[1] >> 1, c[2] >> 1)];
                                }
                            } else if (op == (uint32_t)kPa) {
                                ip += 1;
                                if (ip >= P) fail = true;
                                v = ip;
                            } else if (op == (uint32_t)kP0) {
                                v = ip;
                            } else if (op == (uint32_t)kPd) {
                                const uint32_t d = dp < ops0 ? (uint32_t)sym[dp] : 255u;
                                dp++;
                                if (d > 15 || ip < d + 1) fail = true;
                                v = ip - d - 1;
                            } else {
                                fail = true;  // operation code 7
                            }
                            cl[j] = fail ? 0u : v;
                            cf[j] = (m >= 1 && !stop) ? 1 : 0;
                        }
                        if (fail) bad = 1;
                    }
                    pa_c += tot & 0xFFFFu;
                    pd_c += tot >> 16;
                }
                if (pd_c != nd && tid == 0) bad = 1;
                ipl += pa_c;
                if (agree()) break;
                // same-level references, followed to their values (a reader
                // sees a mark or the final value; both lead to the value)
                for (uint32_t e = tid; e < 8 * E; e += kGT) {
                    const uint32_t j = 8 * lst[e >> 3] + (e & 7u);
                    uint32_t v = cl[j];
                    for (int hops = 0; (v & kGMark) && hops < 8; hops++) v = cl[v & ~kGMark];
                    if (v & kGMark) bad = 1;
                    cl[j] = v;
                }
                stop = agree();
            }
        }
        // 4. output
        if (R.err == 0 && !agree()) {
            const uint32_t G = (1u << N) >> t, lg = N - t;
            const uint32_t *lt = lev + level_off(N, t);
            uint32_t *dst = gmem<uint32_t>(R.dst);
            for (uint32_t v = tid; v < R.count; v += kGT) {
                uint32_t label = R.fill_v;
                if (!R.fill) {
                    const uint32_t x = v & (G - 1), y = (v >> lg) & (G - 1), z = v >> (2 * lg);
                    const uint32_t idx = lt[morton3(x, y, z)];
                    label = idx < P ? pal[idx] : 0u;
                    if (idx >= P) bad = 1;
                }
                dst[v] = label;
            }
        }
        if (R.err || agree()) {
            if (tid == 0)
                g_report(a, rq, R.err ? R.err : CSV_ECORRUPT,
                         (R.err == CSV_ERANGE) ? a.rq_base + rq : R.id);
            for (uint32_t v = tid; v < R.count; v += kGT) gmem<uint32_t>(R.dst)[v] = 0u;
        }
        __syncthreads();
    }
}

template <uint32_t N>
hipError_t go(const GenericArgs &a, uint32_t groups, hipStream_t s) {
    hipLaunchKernelGGL(generic_kernel<N>, dim3(groups), dim3(kGT), 4 * a.lut_lds_words, s, a);
    return hipGetLastError();
}

}  // namespace

uint64_t generic_scratch_bytes(uint32_t log2, uint32_t sym_cap) {
    if (log2 < 1 || log2 > (uint32_t)kMaxLog2) return 0;
    return align256(sym_cap) + align256(4 * all_nodes(log2)) + align256(all_nodes(log2)) +
           align256(4 * pow8(log2 - 1));
}

hipError_t generic_launch(const GenericArgs &a, uint32_t groups, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (a.log2) {
        case 1: return go<1>(a, groups, s);
        case 2: return go<2>(a, groups, s);
        case 3: return go<3>(a, groups, s);
        case 4: return go<4>(a, groups, s);
        case 5: return go<5>(a, groups, s);
        case 6: return go<6>(a, groups, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace csv
