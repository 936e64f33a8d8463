// GPU brick decoder for gfx950 and the device pool that feeds it.
//
// Decoding one 32^3 brick to level of detail t (Sec. 3.4, Alg. 1) in one
// 256-thread workgroup:
//   1. stage the rANS decode table, the palette and the word stream in LDS;
//   2. wave 0 runs the W interleaved rANS states in lockstep (Sec. 3.3),
//      renormalisation reads placed by a wave ballot + prefix count, and
//      writes the symbols as packed nibbles into LDS;
//   3. all waves replay the refinement operations level by level (Sec. 3.2).
//      A level is data-parallel: the rank of an expanded parent among the
//      level's expanded parents places its 8 operation nibbles, prefix
//      sums of P_a / P_delta counts give each child's palette position and
//      delta slot, and same-level neighbour reuse (which always points to a
//      child with one more coordinate bit set) is resolved in 3 passes of
//      decreasing child popcount;
//   4. the level-t block of palette indices is mapped through the palette
//      and written to HBM with 16-byte stores.
// All work happens in palette-index space (u16) in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/csv.h"
#include "csv_format.hpp"

namespace {

constexpr int kNT = 256;
constexpr int kWaves = kNT / 64;
constexpr int kLog2 = 5;                      // 32^3 bricks
constexpr int kLutBits = 11;                  // largest supported table precision
constexpr int kLutSize = 1 << kLutBits;
constexpr int kPalCap = 4096;                 // palette entries staged in LDS
constexpr int kWordCap = 32768;               // words staged in LDS
constexpr int kMaxSym = 2 * 37448;            // every node an operation plus a delta nibble
constexpr int kNibDw = kMaxSym / 8 + 2;
constexpr uint32_t kUnres = 0xFFFDu;          // kUnres + axis: same-level reference, resolved later
// level m (1..4) node arrays inside Smem::lv / Smem::fl
__device__ constexpr int kLvOff[6] = {0, 0, 4096, 4608, 4672, 4680};

struct __align__(16) Smem {
    uint32_t lut[2][kLutSize];
    uint32_t pal[kPalCap];
    uint32_t nib[kNibDw];
    union {
        uint16_t l0[32768];
        uint16_t words[kWordCap];
    } big;
    uint16_t lv[4680];
    uint8_t fl[4680];
    uint64_t red[kWaves];
    int err;
};

struct DecodeArgs {
    const uint64_t *rec_ptr;
    const uint32_t *rec_size;
    const uint16_t *rec_vol;
    const uint32_t *luts;      // [volume][2][kLutSize]
    const uint32_t *vol_bits;  // table precision per volume
    uint32_t n_bricks;
    const uint32_t *ids;
    const uint8_t *lods;
    uint32_t lod_scalar;
    const uint64_t *out_off;
    uint32_t *out;
    uint32_t n;
    int *err;  // [0] first error code, [1] brick id (or request index)
};

__device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0x030000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

__device__ inline void report(int *err, int code, uint32_t who) {
    if (atomicCAS(err, 0, code) == 0) atomicExch(err + 1, (int)who);
}

// exclusive prefix of v over the workgroup (thread order); *total gets the sum
__device__ inline uint64_t block_scan(uint64_t v, uint64_t *total, uint64_t *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t s = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = (uint64_t)__shfl_up((unsigned long long)s, d, 64);
        if (lane >= d) s += t;
    }
    if (lane == 63) red[wave] = s;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        uint64_t r = red[w];
        pre += (w < wave) ? r : 0;
        tot += r;
    }
    __syncthreads();
    *total = tot;
    return pre + s - v;
}

// 8 nibbles starting at nibble position p
__device__ inline uint32_t nib8(const uint32_t *nib, uint32_t p) {
    uint32_t lo = nib[p >> 3], hi = nib[(p >> 3) + 1];
    return __builtin_amdgcn_alignbit(hi, lo, 4 * (p & 7));
}
__device__ inline uint32_t nib1(const uint32_t *nib, uint32_t p) { return (nib[p >> 3] >> (4 * (p & 7))) & 15u; }

__device__ inline uint16_t *level_ptr(Smem &S, int m) { return m == 0 ? S.big.l0 : S.lv + kLvOff[m]; }

__device__ void fill_out(uint32_t *dst, uint32_t count, uint32_t v) {
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0 && (count & 3) == 0) {
        uint4 q = make_uint4(v, v, v, v);
        for (uint32_t e = 4 * threadIdx.x; e < count; e += 4 * kNT) *reinterpret_cast<uint4 *>(dst + e) = q;
    } else {
        for (uint32_t e = threadIdx.x; e < count; e += kNT) dst[e] = v;
    }
}

__device__ void decode_request(Smem &S, const DecodeArgs &a, uint32_t req) {
    const int tid = threadIdx.x;
    const uint32_t id = a.ids[req];
    const uint32_t t = a.lods ? (uint32_t)a.lods[req] : a.lod_scalar;
    if (t > (uint32_t)kLog2) {
        if (tid == 0) report(a.err, CSV_ERANGE, req);
        return;
    }
    const uint32_t G = 32u >> t, count = G * G * G;
    uint32_t *dst = a.out + (a.out_off ? a.out_off[req] : (uint64_t)req * count);
    if (id >= a.n_bricks) {
        if (tid == 0) report(a.err, CSV_ERANGE, req);
        fill_out(dst, count, 0);
        return;
    }
    const uint32_t *rec = reinterpret_cast<const uint32_t *>(a.rec_ptr[id]);
    const uint32_t size = a.rec_size[id];
    const uint32_t vol = a.rec_vol[id];
    const uint32_t P = rec[0], W = rec[1], nw = rec[2];
    uint32_t cum[kLog2];
#pragma unroll
    for (int m = 0; m < kLog2; m++) cum[m] = rec[3 + m];
    const uint32_t hdr = csv::record_header_words(kLog2);
    bool ok = P >= 1 && W <= 64 && (W & (W - 1)) == 0 && ((cum[0] > 0) == (W > 0)) && cum[0] <= (uint32_t)kMaxSym &&
              (uint64_t)4 * (hdr + P + W) + 2ull * nw <= size;
#pragma unroll
    for (int m = 0; m + 1 < kLog2; m++) ok = ok && cum[m] >= cum[m + 1];
    if (ok && cum[0] == 0) ok = (P == 1);
    if (ok && cum[0] > 0) ok = (P >= 2);
    if (!ok) {
        if (tid == 0) report(a.err, CSV_ECORRUPT, id);
        fill_out(dst, count, 0);
        return;
    }
    const uint32_t *pal_g = rec + hdr;
    if (t == (uint32_t)kLog2 || cum[0] == 0) {  // coarsest level / uniform brick: palette[0]
        fill_out(dst, count, pal_g[0]);
        return;
    }
    const uint32_t n = cum[t];
    const uint32_t sbits = a.vol_bits[vol];
    const uint32_t lutn = 1u << sbits;

    // ---- 1. staging ----------------------------------------------------
    {
        const uint32_t *lut_g = a.luts + (size_t)vol * 2 * kLutSize;
        const int ntab = (t == 0) ? 2 : 1;
        for (int tb = 0; tb < ntab; tb++)
            for (uint32_t e = tid; e < lutn; e += kNT) S.lut[tb][e] = lut_g[tb * kLutSize + e];
        if (P <= (uint32_t)kPalCap)
            for (uint32_t e = tid; e < P; e += kNT) S.pal[e] = pal_g[e];
        const uint32_t nwc = min(nw, n);
        if (nwc <= (uint32_t)kWordCap) {
            const uint32_t *wg = rec + hdr + P + W;
            uint32_t *wl = reinterpret_cast<uint32_t *>(S.big.words);
            for (uint32_t e = tid; e < (nwc + 1) / 2; e += kNT) wl[e] = wg[e];
        }
        for (uint32_t e = tid; e < (n + 7) / 8 + 1; e += kNT) S.nib[e] = 0;
        if (tid == 0) S.err = 0;
    }
    __syncthreads();
    const uint32_t *pal = (P <= (uint32_t)kPalCap) ? S.pal : pal_g;

    // ---- 2. interleaved rANS (wave 0) -------------------------------------
    if (tid < 64) {
        const uint32_t lane = tid;
        const uint16_t *wp = (min(nw, n) <= (uint32_t)kWordCap)
                                 ? S.big.words
                                 : reinterpret_cast<const uint16_t *>(rec + hdr + P + W);
        uint32_t x = lane < W ? rec[hdr + P + lane] : 0u;
        const uint32_t leaf_start = cum[1];
        const uint32_t mask = lutn - 1;
        const uint32_t steps = (n + W - 1) / W;
        uint32_t cursor = 0;
        bool bad = false;
        for (uint32_t s = 0; s < steps; s++) {
            const uint32_t i = s * W + lane;
            const bool act = lane < W && i < n;
            uint32_t sym = 0;
            bool need = false;
            if (act) {
                const uint32_t e = S.lut[i >= leaf_start ? 1 : 0][x & mask];
                sym = e & 15u;
                x = (e >> 16) * (x >> sbits) + ((e >> 4) & 0xFFFu);
                need = x < csv::kRansLower;
            }
            const uint64_t bal = __ballot(need);
            const uint32_t cnt = (uint32_t)__popcll(bal);
            if (cursor + cnt > nw) {
                bad = true;
                break;
            }
            if (need) {
                const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                x = (x << 16) | wp[cursor + off];
            }
            cursor += cnt;
            if (act) atomicOr(&S.nib[i >> 3], sym << (4 * (i & 7)));
        }
        if (!bad && t == 0) {
            // a complete decode ends in the encoder's initial states with every word read
            const bool fin = (lane >= W) || x == csv::kRansLower;
            bad = (__ballot(!fin) != 0) || cursor != nw;
        }
        if (bad && lane == 0) S.err = CSV_ECORRUPT;
    }
    __syncthreads();
    if (S.err) {
        if (tid == 0) report(a.err, S.err, id);
        fill_out(dst, count, 0);
        return;
    }

    // ---- 3. replay levels 4 .. t ------------------------------------------
    uint32_t ip_level = 0;  // P_a operations before the current level
    uint32_t seg = 0;       // first symbol of the current level
    for (int m = kLog2 - 1; m >= (int)t; m--) {
        const uint32_t Gp = 1u << (kLog2 - 1 - m);  // parent grid
        const uint32_t Gc = 2 * Gp;                 // child grid
        const uint32_t np = Gp * Gp * Gp;
        const uint32_t ppt = (np + kNT - 1) / kNT;
        const uint32_t q0 = min(tid * ppt, np), q1 = min(q0 + ppt, np);
        const uint16_t *up = (m + 1 <= 4) ? level_ptr(S, m + 1) : nullptr;
        const uint8_t *upf = (m + 1 <= 4) ? S.fl + kLvOff[m + 1] : nullptr;
        uint16_t *cur = level_ptr(S, m);
        uint8_t *curf = (m >= 1) ? S.fl + kLvOff[m] : nullptr;

        // ranks of expanded parents (Morton order)
        uint32_t ne = 0;
        for (uint32_t q = q0; q < q1; q++) {
            const uint32_t X = compact3(q), Y = compact3(q >> 1), Z = compact3(q >> 2);
            ne += upf ? upf[X + Gp * (Y + Gp * Z)] : 1u;
        }
        uint64_t E64;
        const uint32_t rank0 = (uint32_t)block_scan(ne, &E64, S.red);
        const uint32_t E = (uint32_t)E64;
        const uint32_t seg_end = cum[m];
        // a level's delta nibbles precede its 8 operation nibbles per expanded parent
        const bool seg_ok = (uint64_t)seg + 8ull * E <= seg_end;
        const uint32_t D = seg_ok ? seg_end - seg - 8 * E : 0;
        const uint32_t ops0 = seg + D;
        // P_a and P_delta counts of each thread's parents
        uint32_t pa = 0, pd = 0;
        {
            uint32_t r = rank0;
            for (uint32_t q = q0; q < q1; q++) {
                const uint32_t X = compact3(q), Y = compact3(q >> 1), Z = compact3(q >> 2);
                if (upf && !upf[X + Gp * (Y + Gp * Z)]) continue;
                if (seg_ok) {
                    const uint32_t w = nib8(S.nib, ops0 + 8 * r);
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        const uint32_t op = (w >> (4 * k)) & 7u;
                        pa += op == csv::kPa;
                        pd += op == csv::kPd;
                    }
                }
                r++;
            }
        }
        uint64_t tot;
        const uint64_t pre = block_scan((uint64_t)pa | ((uint64_t)pd << 32), &tot, S.red);
        const uint32_t PAtot = (uint32_t)tot, PDtot = (uint32_t)(tot >> 32);
        if (!seg_ok || PDtot != D) {
            if (tid == 0) report(a.err, CSV_ECORRUPT, id);
            fill_out(dst, count, 0);
            return;
        }
        // children values
        {
            uint32_t r = rank0;
            uint32_t ipc = ip_level + (uint32_t)pre;
            uint32_t dcur = seg + (uint32_t)(pre >> 32);
            bool bad = false;
            for (uint32_t q = q0; q < q1; q++) {
                const uint32_t X = compact3(q), Y = compact3(q >> 1), Z = compact3(q >> 2);
                const uint32_t pidx = X + Gp * (Y + Gp * Z);
                const uint32_t pv = up ? up[pidx] : 0u;
                const bool exp = upf ? upf[pidx] != 0 : true;
                if (!exp) {
#pragma unroll
                    for (int k = 0; k < 8; k++) {
                        const uint32_t c = (2 * X + (k & 1)) + Gc * ((2 * Y + ((k >> 1) & 1)) + Gc * (2 * Z + (k >> 2)));
                        cur[c] = (uint16_t)pv;
                        if (curf) curf[c] = 0;
                    }
                    continue;
                }
                const uint32_t w = nib8(S.nib, ops0 + 8 * r);
                r++;
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    const uint32_t nb = (w >> (4 * k)) & 15u, op = nb & 7u, stop = nb >> 3;
                    const uint32_t cx = 2 * X + (k & 1), cy = 2 * Y + ((k >> 1) & 1), cz = 2 * Z + (k >> 2);
                    uint32_t v = 0;
                    if (op == csv::kRp) {
                        v = pv;
                    } else if (op <= csv::kRz) {
                        const int ax = (int)op - 1;
                        const uint32_t bit = (k >> ax) & 1;
                        const uint32_t pc = ax == 0 ? X : (ax == 1 ? Y : Z);
                        if (bit == 0) {
                            const uint32_t cc = ax == 0 ? cx : (ax == 1 ? cy : cz);
                            if (cc == 0) bad = true;
                            v = kUnres + (uint32_t)ax;
                        } else {
                            if (pc + 1 >= Gp || !up) {
                                bad = true;
                            } else {
                                const uint32_t nidx = pidx + (ax == 0 ? 1u : (ax == 1 ? Gp : Gp * Gp));
                                v = up[nidx];
                            }
                        }
                    } else if (op == csv::kPa) {
                        ipc++;
                        if (ipc >= P) bad = true;
                        v = ipc;
                    } else if (op == csv::kP0) {
                        v = ipc;
                    } else if (op == csv::kPd) {
                        const uint32_t d = nib1(S.nib, dcur++);
                        if (ipc < d + 1) bad = true;
                        v = ipc - 1 - d;
                    } else {
                        bad = true;
                    }
                    if (m == 0 && stop) bad = true;
                    const uint32_t c = cx + Gc * (cy + Gc * cz);
                    cur[c] = (uint16_t)v;
                    if (curf) curf[c] = (uint8_t)(stop ^ 1u);
                }
            }
            if (bad) atomicOr(&S.err, 1);
        }
        __syncthreads();
        if (S.err) {
            if (tid == 0) report(a.err, CSV_ECORRUPT, id);
            fill_out(dst, count, 0);
            return;
        }
        // same-level references: the referenced child has one more bit set
        for (int pcnt = 2; pcnt >= 0; pcnt--) {
            for (uint32_t q = q0; q < q1; q++) {
                const uint32_t X = compact3(q), Y = compact3(q >> 1), Z = compact3(q >> 2);
#pragma unroll
                for (int k = 0; k < 8; k++) {
                    if (__builtin_popcount(k) != pcnt) continue;
                    const uint32_t c = (2 * X + (k & 1)) + Gc * ((2 * Y + ((k >> 1) & 1)) + Gc * (2 * Z + (k >> 2)));
                    const uint32_t v = cur[c];
                    if (v >= kUnres) {
                        const uint32_t ax = v - kUnres;
                        cur[c] = cur[c - (ax == 0 ? 1u : (ax == 1 ? Gc : Gc * Gc))];
                    }
                }
            }
            __syncthreads();
        }
        ip_level += PAtot;
        seg = seg_end;
    }

    // ---- 4. output ----------------------------------------------------------
    const uint16_t *res = level_ptr(S, (int)t);
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        for (uint32_t e = 4 * tid; e < count; e += 4 * kNT) {
            uint4 q;
            q.x = pal[min((uint32_t)res[e], P - 1)];
            q.y = pal[min((uint32_t)res[e + 1], P - 1)];
            q.z = pal[min((uint32_t)res[e + 2], P - 1)];
            q.w = pal[min((uint32_t)res[e + 3], P - 1)];
            *reinterpret_cast<uint4 *>(dst + e) = q;
        }
    } else {
        for (uint32_t e = tid; e < count; e += kNT) dst[e] = pal[min((uint32_t)res[e], P - 1)];
    }
}

__global__ __launch_bounds__(kNT) void decode_kernel(DecodeArgs a, uint32_t base) {
    __shared__ Smem S;
    decode_request(S, a, base + blockIdx.x);
}

}  // namespace

// ---------------------------------------------------------------------------
// Pool
// ---------------------------------------------------------------------------
struct csv_pool {
    int device = 0;
    std::vector<void *> vol_bufs;
    std::vector<uint64_t> rec_ptr;
    std::vector<uint32_t> rec_size;
    std::vector<uint16_t> rec_vol;
    std::vector<uint32_t> luts;
    std::vector<uint32_t> bits;
    uint64_t *d_rec_ptr = nullptr;
    uint32_t *d_rec_size = nullptr;
    uint16_t *d_rec_vol = nullptr;
    uint32_t *d_luts = nullptr;
    uint32_t *d_bits = nullptr;
    int *d_err = nullptr;
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

void build_lut(const uint32_t f[16], uint32_t bits, uint32_t *lut) {
    uint32_t c = 0;
    for (uint32_t s = 0; s < 16; s++) {
        for (uint32_t q = 0; q < f[s]; q++) lut[c + q] = csv::lut_entry(s, q, f[s]);
        c += f[s];
    }
    (void)bits;
}

int launch(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
           const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream, bool plain) {
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
    a.vol_bits = pool->d_bits;
    a.n_bricks = (uint32_t)pool->rec_ptr.size();
    a.ids = ids;
    a.lods = lods;
    a.lod_scalar = lod_scalar;
    a.out_off = out_off;
    a.out = out;
    a.n = n;
    a.err = pool->d_err;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (plain) {
        for (uint32_t i = 0; i < n; i++)
            hipLaunchKernelGGL(decode_kernel, dim3(1), dim3(kNT), 0, s, a, i);
    } else {
        const uint32_t chunk = 1u << 30;
        for (uint32_t b0 = 0; b0 < n; b0 += chunk)
            hipLaunchKernelGGL(decode_kernel, dim3(std::min(chunk, n - b0)), dim3(kNT), 0, s, a, b0);
    }
    return hipGetLastError() == hipSuccess ? CSV_OK : CSV_EHIP;
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
    if (hipMalloc(reinterpret_cast<void **>(&p->d_err), 2 * sizeof(int)) != hipSuccess ||
        hipMemset(p->d_err, 0, 2 * sizeof(int)) != hipSuccess) {
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
    (void)hipFree(p->d_bits);
    (void)hipFree(p->d_err);
    delete p;
}

int csv_pool_add_volume(csv_pool *p, const uint8_t *blob, size_t blob_bytes, uint32_t *first_brick_id) {
    if (!p || !blob) return CSV_EINVAL;
    csv_volume_info info;
    int rc = csv_blob_info(blob, blob_bytes, &info);
    if (rc) return rc;
    if (info.brick_log2 != (uint32_t)kLog2 || info.scale_bits > (uint32_t)kLutBits) return CSV_EINVAL;
    if ((uint64_t)p->rec_ptr.size() + info.n_bricks >= (1ull << 32) || p->bits.size() >= 65535) return CSV_ERANGE;
    std::lock_guard<std::mutex> lk(p->mu);
    DeviceGuard g(p->device);
    const uint64_t rs = csv::record_area_offset(info.n_bricks);
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + csv::kHeaderBytes);
    // every record must at least hold its header, and offsets must be 4-byte aligned and increasing
    for (uint32_t i = 0; i < info.n_bricks; i++)
        if (index[i + 1] < index[i] + 4 * csv::record_header_words(kLog2) || (index[i] & 3)) return CSV_ECORRUPT;
    void *buf = nullptr;
    const size_t rb = std::max<uint64_t>(info.record_bytes, 4);
    if (hipMalloc(&buf, rb) != hipSuccess) return CSV_ENOMEM;
    if (hipMemcpy(buf, blob + rs, info.record_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        return CSV_EHIP;
    }
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
    const size_t lo = p->luts.size();
    p->luts.resize(lo + 2 * kLutSize, 0);
    for (int tb = 0; tb < 2; tb++) build_lut(info.freq[tb], info.scale_bits, p->luts.data() + lo + tb * kLutSize);
    if ((rc = upload(&p->d_rec_ptr, p->rec_ptr)) || (rc = upload(&p->d_rec_size, p->rec_size)) ||
        (rc = upload(&p->d_rec_vol, p->rec_vol)) || (rc = upload(&p->d_luts, p->luts)) ||
        (rc = upload(&p->d_bits, p->bits)))
        return rc;
    if (first_brick_id) *first_brick_id = first;
    return CSV_OK;
}

int csv_pool_info_get(const csv_pool *p, csv_pool_info *info) {
    if (!p || !info) return CSV_EINVAL;
    info->n_volumes = (uint32_t)p->bits.size();
    info->n_bricks = (uint32_t)p->rec_ptr.size();
    info->device = p->device;
    info->device_bytes = p->record_bytes + p->rec_ptr.size() * (8 + 4 + 2) + p->luts.size() * 4 + 8;
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
    return launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, false);
}

int csv_decode_bricks_plain(const csv_pool *pool, const uint32_t *ids, const uint8_t *lods, uint32_t lod_scalar,
                            const uint64_t *out_off, uint32_t n, uint32_t *out, void *stream) {
    return launch(pool, ids, lods, lod_scalar, out_off, n, out, stream, true);
}

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
