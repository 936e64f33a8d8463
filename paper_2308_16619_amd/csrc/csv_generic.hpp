// The decoder for every brick edge 2^N (N = 1..6) and both codings (rANS
// and raw nibbles): one workgroup per brick, levels replayed one after
// another in a global-memory scratch area of the workgroup.  The 32^3
// rANS path of csv_decode.hip is the tuned one; this one serves the other
// brick sizes and the coding without rANS (Table 1's variants).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace csv {

struct GenericArgs {
    const uint64_t *rec_ptr;   // per brick: record address
    const uint32_t *rec_size;  // per brick: record bytes
    const uint16_t *rec_vol;   // per brick: volume
    const uint32_t *luts;      // decode tables of all volumes (see lut_entry)
    const uint32_t *lut_off;   // per volume: first entry of its two tables
    uint32_t lut_lds_words;    // words of luts copied to LDS per workgroup (0: read from global memory)
    const uint32_t *vol_bits;  // per volume: table precision
    const uint8_t *vol_raw;    // per volume: 1 if its symbols are stored as raw nibbles
    uint32_t n_bricks;
    uint32_t log2;             // brick edge 2^log2 of every volume of the pool
    const uint32_t *ids;
    const uint8_t *lods;
    uint32_t lod_scalar;
    const uint64_t *out_off;
    uint64_t out;              // device address of the uint32 output
    uint32_t n;
    int *err;                  // [0] first error code, [1] brick id or request index
    int *req_err;              // per-request status, or nullptr
    uint32_t rq_base;          // index of request 0 in the caller's batch
    uint64_t scratch;          // device address: scratch_per_group bytes per workgroup
    uint64_t scratch_per_group;
    uint32_t sym_cap;          // symbols a workgroup's scratch holds
};

// scratch bytes per workgroup for bricks of edge 2^log2 with at most
// sym_cap symbols
uint64_t generic_scratch_bytes(uint32_t log2, uint32_t sym_cap);

// decode a.n requests with `groups` workgroups on stream s (a.scratch holds
// groups * a.scratch_per_group bytes); hipSuccess or the launch error
hipError_t generic_launch(const GenericArgs &a, uint32_t groups, hipStream_t s);

}  // namespace csv
