// Container layout shared by the library's encoder, pool loader and kernels.
//
// Volume blob (little endian):
//   [0,128)   header: 16 x u32 {magic "CSV1", version 1, nx, ny, nz,
//             brick_log2, nbx, nby, nbz, n_bricks, scale_bits, lane_k,
//             lane_max, sample_stride, 0, 0}, then u16 freq[2][16]
//             (table 0: children on levels >= 1, table 1: children on L_0;
//             each sums to 2^scale_bits, every entry >= 1)
//   [128, ..) u64 index[n_bricks + 1]: record offsets relative to the
//             record area, which starts at the next multiple of 16
//   records   one per brick, 4-byte aligned:
//             u32 P (palette entries), u32 W (interleaved rANS states),
//             u32 n_words, u32 cum[N] (cum[m]: number of symbols in the
//             segments of child levels N-1 .. m), u32 palette[P],
//             u32 state[W], u16 words[n_words], zero padding to 4 bytes.
//
// Symbol stream of a brick (decoded order): one segment per child level m
// = N-1 .. 0; a segment holds one delta nibble per P_delta operation of
// the segment, in operation order, then 8 (op | stop << 3) nibbles per
// expanded parent in Morton order.  Symbol i belongs to interleaved state
// i mod W; words are read in symbol order.
#pragma once
#include <cstdint>

namespace csv {

constexpr uint32_t kMagic = 0x31565343u;  // "CSV1"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kRansLower = 1u << 16;
constexpr int kMaxLog2 = 6;

enum Op : uint32_t { kRp = 0, kRx = 1, kRy = 2, kRz = 3, kP0 = 4, kPd = 5, kPa = 6 };

struct VolumeHeader {
    uint32_t magic, version, nx, ny, nz, brick_log2, nbx, nby, nbz, n_bricks, scale_bits, lane_k, lane_max,
        sample_stride, reserved0, reserved1;
    uint16_t freq[2][16];
};
static_assert(sizeof(VolumeHeader) == kHeaderBytes, "header layout");

constexpr uint64_t record_area_offset(uint64_t n_bricks) { return (kHeaderBytes + 8 * (n_bricks + 1) + 15) & ~15ull; }

// u32 words before the palette in a record
constexpr uint32_t record_header_words(int N) { return 3u + (uint32_t)N; }

// Decode-table entry for one slot of a table with precision scale_bits
// (at most 11): bits 0..3 symbol, bits 4..7 zero (the low byte is the
// symbol), bits 8..19 slot - cumulative start, bits 20..31 frequency.
constexpr uint32_t lut_entry(uint32_t sym, uint32_t bias, uint32_t freq) { return sym | (bias << 8) | (freq << 20); }

}  // namespace csv
