// Host compressor: resolution pyramid (Sec. 3.1), brick encoding with the
// fixed operation test order (Sec. 3.2, Sec. 3.4, Alg. 2), two static
// frequency tables from a sampled prepass (Sec. 3.3, Sec. 3.4) and
// interleaved rANS (Sec. 3.3).  The paper's compressor is a multithreaded
// CPU program; this one distributes bricks over threads through a shared
// work counter instead of the paper's fixed T-bricks-per-round scheme.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/csv.h"
#include "csv_format.hpp"

namespace {

using namespace csv;

// Per brick size: Morton <-> dense tables and the neighbour reference of
// every node for R_x / R_y / R_z.
struct Geometry {
    int N = 0;
    uint32_t b = 0;
    std::vector<uint32_t> dense_of_leaf;  // L_0 Morton index -> offset in a dense brick
    // nbr[m][a][j] for node j (Morton) on level m, axis a:
    //   >= 0           same-level node index (the neighbour at coordinate - 1)
    //   <= -2          parent-level node index -(v + 2) (parent of the neighbour at + 1)
    //   -1             outside the brick: not applicable
    std::vector<int32_t> nbr[kMaxLog2][3];

    explicit Geometry(int n) : N(n), b(1u << n) {
        dense_of_leaf.resize((size_t)b * b * b);
        for (uint32_t m = 0; m < dense_of_leaf.size(); m++) {
            uint32_t c[3];
            coords(m, N, c);
            dense_of_leaf[m] = c[0] + b * (c[1] + b * c[2]);
        }
        for (int m = 0; m < N; m++) {
            int bits = N - m;
            uint32_t G = 1u << bits, cnt = G * G * G;
            for (int a = 0; a < 3; a++) {
                nbr[m][a].resize(cnt);
                for (uint32_t j = 0; j < cnt; j++) {
                    uint32_t c[3];
                    coords(j, bits, c);
                    int32_t v = -1;
                    if ((c[a] & 1u) == 0) {
                        if (c[a] > 0) {
                            c[a] -= 1;
                            v = (int32_t)morton(c, bits);
                        }
                    } else if (c[a] + 1 < G) {
                        c[a] += 1;
                        uint32_t p[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
                        v = -(int32_t)morton(p, bits - 1) - 2;
                    }
                    nbr[m][a][j] = v;
                }
            }
        }
    }
    static void coords(uint32_t m, int bits, uint32_t c[3]) {
        c[0] = c[1] = c[2] = 0;
        for (int i = 0; i < bits; i++)
            for (int a = 0; a < 3; a++) c[a] |= ((m >> (3 * i + a)) & 1u) << i;
    }
    static uint32_t morton(const uint32_t c[3], int bits) {
        uint32_t m = 0;
        for (int i = 0; i < bits; i++)
            for (int a = 0; a < 3; a++) m |= ((c[a] >> i) & 1u) << (3 * i + a);
        return m;
    }
};

// Scratch reused across the bricks one thread encodes.
struct BrickEncoder {
    const Geometry &g;
    std::vector<uint32_t> lab[kMaxLog2 + 1];
    std::vector<uint8_t> cst[kMaxLog2 + 1];
    std::vector<uint32_t> palette;
    std::vector<uint8_t> sym;
    std::vector<uint8_t> deltas;
    std::vector<uint8_t> ops;
    uint32_t cum[kMaxLog2] = {};

    explicit BrickEncoder(const Geometry &geo) : g(geo) {
        for (int l = 0; l <= g.N; l++) {
            size_t n = (size_t)1 << (3 * (g.N - l));
            lab[l].resize(n);
            cst[l].resize(n);
        }
    }

    void load(const uint32_t *vol, uint32_t nx, uint32_t ny, uint32_t nz, uint64_t id, uint32_t nbx, uint32_t nby) {
        uint32_t b = g.b;
        uint64_t bx = id % nbx, by = (id / nbx) % nby, bz = id / ((uint64_t)nbx * nby);
        uint64_t x0 = bx * b, y0 = by * b, z0 = bz * b;
        bool inside = x0 + b <= nx && y0 + b <= ny && z0 + b <= nz;
        for (size_t m = 0; m < lab[0].size(); m++) {
            uint32_t d = g.dense_of_leaf[m];
            uint64_t x = x0 + (d & (b - 1)), y = y0 + ((d >> g.N) & (b - 1)), z = z0 + (d >> (2 * g.N));
            uint32_t v = 0;
            if (inside || (x < nx && y < ny && z < nz)) v = vol[x + nx * (y + (uint64_t)ny * z)];
            lab[0][m] = v;
            cst[0][m] = 1;
        }
    }

    void build_pyramid() {
        for (int l = 1; l <= g.N; l++) {
            const uint32_t *ch = lab[l - 1].data();
            const uint8_t *cc = cst[l - 1].data();
            for (size_t q = 0; q < lab[l].size(); q++, ch += 8, cc += 8) {
                bool same = true, allc = true;
                for (int k = 1; k < 8; k++) same &= ch[k] == ch[0];
                for (int k = 0; k < 8; k++) allc &= cc[k] != 0;
                if (same) {
                    lab[l][q] = ch[0];
                    cst[l][q] = allc;
                    continue;
                }
                // most frequent child; the earliest child wins a tie
                int bestk = 0, bestn = 0;
                for (int k = 0; k < 8; k++) {
                    int n = 0;
                    for (int r = 0; r < 8; r++) n += ch[r] == ch[k];
                    if (n > bestn) { bestn = n; bestk = k; }
                }
                lab[l][q] = ch[bestk];
                cst[l][q] = 0;
            }
        }
    }

    void encode() {
        const int N = g.N;
        palette.assign(1, lab[N][0]);
        sym.clear();
        for (int l = N; l >= 1; l--) {
            const int m = l - 1;
            deltas.clear();
            ops.clear();
            const uint32_t *up = lab[l].data(), *cur = lab[m].data();
            for (size_t q = 0; q < lab[l].size(); q++) {
                if (cst[l][q]) continue;
                uint32_t parent = up[q];
                for (uint32_t k = 0; k < 8; k++) {
                    uint32_t j = (uint32_t)(8 * q + k), L = cur[j];
                    uint32_t stop = (m >= 1 && cst[m][j]) ? 1u : 0u;
                    uint32_t op = kPa;
                    if (parent == L) {
                        op = kRp;
                    } else {
                        for (int a = 0; a < 3 && op == kPa; a++) {
                            int32_t r = g.nbr[m][a][j];
                            if (r == -1) continue;
                            uint32_t v = r >= 0 ? cur[r] : up[-(r + 2)];
                            if (v == L) op = kRx + (uint32_t)a;
                        }
                        if (op == kPa) {
                            size_t ip = palette.size() - 1;
                            if (palette[ip] == L) {
                                op = kP0;
                            } else {
                                for (size_t d = 0; d < 16 && d + 1 <= ip; d++)
                                    if (palette[ip - 1 - d] == L) {
                                        op = kPd;
                                        deltas.push_back((uint8_t)d);
                                        break;
                                    }
                                if (op == kPa) palette.push_back(L);
                            }
                        }
                    }
                    ops.push_back((uint8_t)(op | (stop << 3)));
                }
            }
            // a level's delta nibbles precede its operation nibbles
            sym.insert(sym.end(), deltas.begin(), deltas.end());
            sym.insert(sym.end(), ops.begin(), ops.end());
            cum[m] = (uint32_t)sym.size();
        }
    }
};

struct Tables {
    uint32_t f[2][16], c[2][16];
    uint32_t bits;
};

void normalize(const uint64_t cnt[16], uint32_t M, uint32_t f[16]) {
    uint64_t tot = 0;
    for (int s = 0; s < 16; s++) tot += cnt[s] + 1;
    uint64_t sum = 0;
    for (int s = 0; s < 16; s++) {
        uint64_t v = (cnt[s] + 1) * (uint64_t)M / tot;
        f[s] = v ? (uint32_t)v : 1u;
        sum += f[s];
    }
    if (sum < M) {
        int best = 0;
        for (int s = 1; s < 16; s++)
            if (f[s] > f[best]) best = s;
        f[best] += (uint32_t)(M - sum);
    }
    while (sum > M) {
        int best = -1;
        for (int s = 0; s < 16; s++)
            if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
        f[best]--;
        sum--;
    }
}

uint32_t lanes_for(uint32_t n, uint32_t K, uint32_t Wmax) {
    if (n == 0) return 0;
    uint32_t W = 1;
    while (2 * W <= Wmax && (uint64_t)2 * W * K <= n) W *= 2;
    return W;
}

// Interleaved rANS: symbol i uses state i % W, encoded from the last symbol
// to the first so that the decoder reads words in symbol order.
void build_record(const BrickEncoder &e, const Tables &t, uint32_t K, uint32_t Wmax, std::vector<uint8_t> &rec) {
    const int N = e.g.N;
    const uint32_t n = (uint32_t)e.sym.size();
    const uint32_t W = lanes_for(n, K, Wmax);
    const uint32_t leaf_start = N >= 2 ? e.cum[1] : 0;
    uint32_t x[64];
    for (uint32_t j = 0; j < W; j++) x[j] = kRansLower;
    std::vector<uint16_t> out;
    out.reserve(n / 4 + 8);
    const uint64_t xmax_unit = (uint64_t)((kRansLower >> t.bits) << 16);
    for (uint32_t i = n; i-- > 0;) {
        const uint32_t tb = i >= leaf_start ? 1 : 0, s = e.sym[i];
        const uint32_t f = t.f[tb][s], c = t.c[tb][s];
        uint32_t &st = x[i & (W - 1)];
        uint32_t v = st;
        if (v >= xmax_unit * f) {
            out.push_back((uint16_t)v);
            v >>= 16;
        }
        st = ((v / f) << t.bits) + v % f + c;
    }
    const uint32_t hdr = record_header_words(N), P = (uint32_t)e.palette.size(), nw = (uint32_t)out.size();
    size_t size = ((size_t)4 * (hdr + P + W) + 2 * (size_t)nw + 3) & ~(size_t)3;
    rec.assign(size, 0);
    uint32_t *w = reinterpret_cast<uint32_t *>(rec.data());
    w[0] = P;
    w[1] = W;
    w[2] = nw;
    for (int m = 0; m < N; m++) w[3 + m] = e.cum[m];
    std::memcpy(w + hdr, e.palette.data(), 4 * (size_t)P);
    std::memcpy(w + hdr + P, x, 4 * (size_t)W);
    uint16_t *wd = reinterpret_cast<uint16_t *>(rec.data() + 4 * ((size_t)hdr + P + W));
    for (uint32_t q = 0; q < nw; q++) wd[q] = out[nw - 1 - q];
}

// No entropy coding: the symbols as raw nibbles, four to a 16-bit word
// (Table 1's variant without rANS).
void build_record_raw(const BrickEncoder &e, std::vector<uint8_t> &rec) {
    const int N = e.g.N;
    const uint32_t n = (uint32_t)e.sym.size();
    const uint32_t hdr = record_header_words(N), P = (uint32_t)e.palette.size(), nw = (n + 3) / 4;
    const size_t size = ((size_t)4 * (hdr + P) + 2 * (size_t)nw + 3) & ~(size_t)3;
    rec.assign(size, 0);
    uint32_t *w = reinterpret_cast<uint32_t *>(rec.data());
    w[0] = P;
    w[1] = 0;
    w[2] = nw;
    for (int m = 0; m < N; m++) w[3 + m] = e.cum[m];
    std::memcpy(w + hdr, e.palette.data(), 4 * (size_t)P);
    uint16_t *wd = reinterpret_cast<uint16_t *>(rec.data() + 4 * ((size_t)hdr + P));
    for (uint32_t q = 0; q < nw; q++) {
        uint32_t v = 0;
        for (uint32_t k = 0; k < 4 && 4 * q + k < n; k++) v |= (uint32_t)e.sym[4 * q + k] << (4 * k);
        wd[q] = (uint16_t)v;
    }
}

template <class F>
void parallel_for(uint64_t n, unsigned threads, F &&fn) {
    std::atomic<uint64_t> next{0};
    auto worker = [&](unsigned tid) {
        for (;;) {
            uint64_t i = next.fetch_add(1, std::memory_order_relaxed);
            if (i >= n) break;
            fn(i, tid);
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < threads; t++) pool.emplace_back(worker, t);
    worker(0);
    for (auto &th : pool) th.join();
}

}  // namespace

namespace csv {
void normalize_counts(const uint64_t cnt[16], uint32_t M, uint32_t f[16]) { normalize(cnt, M, f); }
}  // namespace csv

extern "C" {

uint32_t csv_abi_version(void) { return CSV_ABI_VERSION; }

const char *csv_strerror(int code) {
    switch (code) {
        case CSV_OK: return "ok";
        case CSV_EINVAL: return "invalid argument";
        case CSV_ERANGE: return "out of range";
        case CSV_ECORRUPT: return "corrupt data";
        case CSV_ENOMEM: return "out of memory";
        case CSV_EHIP: return "HIP runtime error";
        case CSV_EBUSY: return "busy";
        case CSV_EDETAIL: return "level-0 detail not on the device (level 1 upsampled)";
        default: return "unknown error";
    }
}

void csv_encode_opts_default(csv_encode_opts *o) {
    if (!o) return;
    o->brick_log2 = 5;
    o->scale_bits = 10;
    o->lane_k = 64;
    o->lane_max = 64;
    o->sample_stride = 0;
    o->threads = 0;
    o->tables = 2;
    o->coding = 0;
}

void csv_free(void *p) { std::free(p); }

int csv_encode_volume(const uint32_t *labels, uint32_t nx, uint32_t ny, uint32_t nz, const csv_encode_opts *opts,
                      uint8_t **blob, size_t *blob_bytes) {
    if (!labels || !blob || !blob_bytes || !nx || !ny || !nz) return CSV_EINVAL;
    csv_encode_opts o;
    csv_encode_opts_default(&o);
    if (opts) o = *opts;
    if (o.brick_log2 < 1 || o.brick_log2 > (uint32_t)kMaxLog2 || o.scale_bits < 8 || o.scale_bits > 12 ||
        o.lane_k < 1 || o.lane_max < 1 || o.lane_max > 64 || (o.lane_max & (o.lane_max - 1)) || o.tables > 2 ||
        o.coding > 1)
        return CSV_EINVAL;
    const bool raw = o.coding == 1;
    if (o.tables == 0) o.tables = 2;
    try {
        const int N = (int)o.brick_log2;
        const uint32_t b = 1u << N;
        const uint32_t nbx = (nx + b - 1) / b, nby = (ny + b - 1) / b, nbz = (nz + b - 1) / b;
        const uint64_t B = (uint64_t)nbx * nby * nbz;
        if (B >= (1ull << 32)) return CSV_ERANGE;
        const uint32_t stride = o.sample_stride ? o.sample_stride : (B > (1ull << 20) ? 4096u : 512u);
        unsigned threads = o.threads ? o.threads : std::max(1u, std::thread::hardware_concurrency());
        Geometry geo(N);

        // prepass: nibble histograms of the sampled bricks (none without rANS:
        // the header's tables are then uniform)
        const uint64_t n_samples = raw ? 0 : (B + stride - 1) / stride;
        std::vector<std::vector<uint64_t>> hist(threads, std::vector<uint64_t>(32, 0));
        {
            std::vector<BrickEncoder *> enc(threads, nullptr);
            parallel_for(n_samples, threads, [&](uint64_t i, unsigned tid) {
                if (!enc[tid]) enc[tid] = new BrickEncoder(geo);
                BrickEncoder &e = *enc[tid];
                e.load(labels, nx, ny, nz, i * stride, nbx, nby);
                e.build_pyramid();
                e.encode();
                const uint32_t leaf_start = N >= 2 ? e.cum[1] : 0;
                for (uint32_t q = 0; q < e.sym.size(); q++) hist[tid][(q >= leaf_start ? 16 : 0) + e.sym[q]]++;
            });
            for (auto *p : enc) delete p;
        }
        uint64_t cnt[2][16] = {};
        for (auto &h : hist)
            for (int q = 0; q < 32; q++) cnt[q / 16][q % 16] += h[q];
        if (o.tables == 1)  // one table for all symbols
            for (int q = 0; q < 16; q++) cnt[0][q] = cnt[1][q] = cnt[0][q] + cnt[1][q];
        Tables t;
        t.bits = o.scale_bits;
        for (int k = 0; k < 2; k++) {
            normalize(cnt[k], 1u << o.scale_bits, t.f[k]);
            uint32_t c = 0;
            for (int s = 0; s < 16; s++) { t.c[k][s] = c; c += t.f[k][s]; }
        }

        // all bricks
        std::vector<std::vector<uint8_t>> recs(B);
        {
            std::vector<BrickEncoder *> enc(threads, nullptr);
            parallel_for(B, threads, [&](uint64_t id, unsigned tid) {
                if (!enc[tid]) enc[tid] = new BrickEncoder(geo);
                BrickEncoder &e = *enc[tid];
                e.load(labels, nx, ny, nz, id, nbx, nby);
                e.build_pyramid();
                e.encode();
                if (raw)
                    build_record_raw(e, recs[id]);
                else
                    build_record(e, t, o.lane_k, o.lane_max, recs[id]);
            });
            for (auto *p : enc) delete p;
        }
        const uint64_t rec_start = record_area_offset(B);
        uint64_t total = rec_start;
        for (auto &r : recs) total += r.size();
        uint8_t *out = static_cast<uint8_t *>(std::calloc(total, 1));
        if (!out) return CSV_ENOMEM;
        VolumeHeader h;
        std::memset(&h, 0, sizeof(h));
        h.magic = kMagic;
        h.version = kVersion;
        h.nx = nx; h.ny = ny; h.nz = nz;
        h.brick_log2 = o.brick_log2;
        h.nbx = nbx; h.nby = nby; h.nbz = nbz;
        h.n_bricks = (uint32_t)B;
        h.scale_bits = o.scale_bits;
        h.lane_k = o.lane_k;
        h.lane_max = o.lane_max;
        h.sample_stride = stride;
        h.reserved0 = raw ? 1u : 0u;  // coding
        for (int k = 0; k < 2; k++)
            for (int s = 0; s < 16; s++) h.freq[k][s] = (uint16_t)t.f[k][s];
        std::memcpy(out, &h, sizeof(h));
        uint64_t *index = reinterpret_cast<uint64_t *>(out + kHeaderBytes);
        uint64_t off = 0;
        for (uint64_t i = 0; i < B; i++) {
            index[i] = off;
            std::memcpy(out + rec_start + off, recs[i].data(), recs[i].size());
            off += recs[i].size();
            std::vector<uint8_t>().swap(recs[i]);
        }
        index[B] = off;
        *blob = out;
        *blob_bytes = total;
        return CSV_OK;
    } catch (const std::bad_alloc &) {
        return CSV_ENOMEM;
    }
}

int csv_blob_info(const uint8_t *blob, size_t blob_bytes, csv_volume_info *info) {
    if (!blob || !info || blob_bytes < kHeaderBytes) return CSV_EINVAL;
    VolumeHeader h;
    std::memcpy(&h, blob, sizeof(h));
    if (h.magic != kMagic || h.version != kVersion) return CSV_ECORRUPT;
    if (h.brick_log2 < 1 || h.brick_log2 > (uint32_t)kMaxLog2 || h.scale_bits < 8 || h.scale_bits > 12 ||
        h.reserved0 > 1)
        return CSV_ECORRUPT;
    const uint32_t b = 1u << h.brick_log2;
    if (h.nbx != (h.nx + b - 1) / b || h.nby != (h.ny + b - 1) / b || h.nbz != (h.nz + b - 1) / b ||
        (uint64_t)h.nbx * h.nby * h.nbz != h.n_bricks)
        return CSV_ECORRUPT;
    for (int k = 0; k < 2; k++) {
        uint32_t s = 0;
        for (int q = 0; q < 16; q++) {
            if (!h.freq[k][q]) return CSV_ECORRUPT;
            s += h.freq[k][q];
        }
        if (s != (1u << h.scale_bits)) return CSV_ECORRUPT;
    }
    const uint64_t rs = record_area_offset(h.n_bricks);
    if (blob_bytes < rs) return CSV_ECORRUPT;
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + kHeaderBytes);
    if (index[0] != 0 || index[h.n_bricks] > blob_bytes - rs) return CSV_ECORRUPT;
    std::memset(info, 0, sizeof(*info));
    info->nx = h.nx; info->ny = h.ny; info->nz = h.nz;
    info->brick_log2 = h.brick_log2;
    info->nbx = h.nbx; info->nby = h.nby; info->nbz = h.nbz;
    info->n_bricks = h.n_bricks;
    info->scale_bits = h.scale_bits;
    info->lane_k = h.lane_k;
    info->lane_max = h.lane_max;
    info->sample_stride = h.sample_stride;
    for (int k = 0; k < 2; k++)
        for (int q = 0; q < 16; q++) info->freq[k][q] = h.freq[k][q];
    info->record_bytes = index[h.n_bricks];
    info->blob_bytes = rs + index[h.n_bricks];
    info->coding = h.reserved0;
    return CSV_OK;
}

int csv_blob_check(const uint8_t *blob, size_t blob_bytes, uint32_t *first_bad) {
    csv_volume_info info;
    const int rc = csv_blob_info(blob, blob_bytes, &info);
    if (rc) return rc;
    const int N = (int)info.brick_log2;
    const uint64_t hdr = record_header_words(N);
    // every node below the root carries at most one operation and one delta nibble
    uint64_t nodes = 0;
    for (int m = 1; m <= N; m++) nodes += 1ull << (3 * m);
    const uint64_t max_sym = 2 * nodes;
    const uint64_t rs = record_area_offset(info.n_bricks);
    const uint64_t *index = reinterpret_cast<const uint64_t *>(blob + kHeaderBytes);
    for (uint32_t i = 0; i < info.n_bricks; i++) {
        const uint64_t a = index[i], e = index[i + 1];
        bool ok = (a & 3) == 0 && e >= a + 4 * hdr && e <= info.record_bytes && e - a < (1ull << 32);
        if (ok) {
            const uint32_t *w = reinterpret_cast<const uint32_t *>(blob + rs + a);
            const uint64_t P = w[0], W = w[1], nw = w[2];
            uint32_t c[kMaxLog2 + 1] = {};
            for (int m = 0; m < N; m++) c[m] = w[3 + m];
            const bool shape_ok = info.coding == 1 ? (W == 0 && nw == (c[0] + 3ull) / 4)
                                                   : (W <= 64 && (W & (W - 1)) == 0 && ((c[0] > 0) == (W > 0)));
            ok = P >= 1 && shape_ok && c[0] <= max_sym && (c[0] == 0 ? P == 1 : P >= 2) &&
                 4 * (hdr + P + W) + 2 * nw <= e - a;
            for (int m = 1; ok && m < N; m++) ok = c[m] <= c[m - 1];
        }
        if (!ok) {
            if (first_bad) *first_bad = i;
            return CSV_ECORRUPT;
        }
    }
    return CSV_OK;
}

}  // extern "C"
