// Test program for the AddressSanitizer / UndefinedBehaviorSanitizer build
// of the host code (tests/test_sanitizers.py builds and runs it; no GPU):
// the library's host compressor and container checks (csv_encode.cpp) and
// the oracle, on volumes read from files.  For each volume and each format
// variant it compresses with both, requires the same bytes, decodes every
// brick at every level with the oracle and compares full LOD with the
// volume, and runs the record checker on the container and on damaged
// copies of it.  Exit status 0 when everything agrees.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/csv.h"

extern "C" {
int orc_encode_volume(const uint32_t *vol, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t brick_log2,
                      uint32_t scale_bits, uint32_t lane_k, uint32_t lane_max, uint32_t sample_stride,
                      uint32_t tables, uint8_t **blob_out, uint64_t *blob_bytes, uint64_t *op_hist_out);
int orc_decode_brick(const uint8_t *blob, uint64_t bytes, uint32_t id, uint32_t lod, uint32_t *out);
void orc_free(void *p);
}

static int fail(const char *what) {
    std::fprintf(stderr, "sanitize driver: %s\n", what);
    return 1;
}

static int run_volume(const std::vector<uint32_t> &vol, uint32_t n) {
    struct Variant {
        uint32_t log2, tables, coding, scale_bits, lane_k, lane_max;
    };
    const Variant variants[] = {{5, 2, 0, 10, 64, 64}, {4, 1, 0, 8, 1, 16}, {6, 2, 0, 12, 64, 64},
                                {5, 2, 1, 10, 64, 64}, {3, 2, 1, 10, 64, 64}, {2, 2, 0, 11, 4, 4}};
    for (const Variant &v : variants) {
        csv_encode_opts o;
        csv_encode_opts_default(&o);
        o.brick_log2 = v.log2;
        o.tables = v.tables;
        o.coding = v.coding;
        o.scale_bits = v.scale_bits;
        o.lane_k = v.lane_k;
        o.lane_max = v.lane_max;
        o.threads = 4;
        uint8_t *mine = nullptr;
        size_t mine_n = 0;
        if (csv_encode_volume(vol.data(), n, n, n, &o, &mine, &mine_n) != CSV_OK) return fail("host compressor");
        uint8_t *ref = nullptr;
        uint64_t ref_n = 0;
        if (orc_encode_volume(vol.data(), n, n, n, v.log2, v.scale_bits, v.lane_k, v.lane_max, 0,
                              v.coding ? 0u : v.tables, &ref, &ref_n, nullptr) != 0)
            return fail("oracle compressor");
        if (mine_n != ref_n || std::memcmp(mine, ref, mine_n) != 0) return fail("containers differ");
        csv_volume_info info;
        if (csv_blob_info(mine, mine_n, &info) != CSV_OK || info.coding != v.coding) return fail("blob info");
        uint32_t bad = 0;
        if (csv_blob_check(mine, mine_n, &bad) != CSV_OK) return fail("record check");
        const uint32_t b = 1u << v.log2, nb = n / b;
        std::vector<uint32_t> out((size_t)b * b * b);
        for (uint32_t id = 0; id < info.n_bricks; id++) {
            for (uint32_t t = 0; t <= v.log2; t++)
                if (orc_decode_brick(mine, mine_n, id, t, out.data()) != 0) return fail("oracle decode");
            if (orc_decode_brick(mine, mine_n, id, 0, out.data()) != 0) return fail("oracle decode");
            const uint32_t bx = id % nb, by = (id / nb) % nb, bz = id / (nb * nb);
            for (uint32_t z = 0; z < b; z++)
                for (uint32_t y = 0; y < b; y++)
                    for (uint32_t x = 0; x < b; x++)
                        if (out[x + b * (y + b * z)] !=
                            vol[(bx * b + x) + (size_t)n * ((by * b + y) + (size_t)n * (bz * b + z))])
                            return fail("full LOD differs from the volume");
        }
        // damaged copies: a palette size far past the record, a state count
        // that is not a power of two, a record offset past the end; each
        // must be refused without reading past the buffer
        const uint64_t rs = (128 + 8ull * (info.n_bricks + 1) + 15) & ~15ull;
        const uint64_t *index = reinterpret_cast<const uint64_t *>(mine + 128);
        for (int k = 0; k < 3; k++) {
            std::vector<uint8_t> dmg(mine, mine + mine_n);
            uint32_t *w = reinterpret_cast<uint32_t *>(dmg.data() + rs + index[info.n_bricks / 2]);
            if (k == 0) w[0] = 0xFFFFFFF8u;
            if (k == 1) w[1] = 3;
            if (k == 2) reinterpret_cast<uint64_t *>(dmg.data() + 128)[info.n_bricks] = 1ull << 40;
            if (csv_blob_check(dmg.data(), dmg.size(), &bad) == CSV_OK) return fail("damaged container accepted");
        }
        csv_free(mine);
        orc_free(ref);
    }
    return 0;
}

int main(int argc, char **argv) {
    for (int i = 1; i < argc; i++) {
        FILE *f = std::fopen(argv[i], "rb");
        if (!f) return fail("cannot open a volume");
        uint32_t n = 0;
        if (std::fread(&n, 4, 1, f) != 1 || n == 0 || n > 256) return fail("bad volume file");
        std::vector<uint32_t> vol((size_t)n * n * n);
        if (std::fread(vol.data(), 4, vol.size(), f) != vol.size()) return fail("short volume file");
        std::fclose(f);
        if (run_volume(vol, n)) return 1;
        std::printf("volume %s (%u^3): every variant agrees\n", argv[i], n);
    }
    return 0;
}
