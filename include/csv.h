/*
 * csv.h -- C ABI of the MI355X compressed-segmentation-volume library.
 *
 * The method is that of Piochowiak & Dachsbacher, "Fast Compressed
 * Segmentation Volumes for Scientific Visualization" (IEEE TVCG 2023):
 * a label volume is cut into 32^3 bricks (Sec. 3.1); each brick is stored as
 * a palette of labels plus a stream of 4-bit (operation, stop) nibbles that
 * rebuild the brick's resolution pyramid coarse to fine (Sec. 3.2, Alg. 1,
 * Alg. 2); the nibbles are rANS coded against two static frequency tables
 * per volume (Sec. 3.3).  Decoding a brick to level of detail t yields level
 * L_t of its pyramid: (32 >> t)^3 labels (Sec. 3.4).
 *
 * Conventions for every function:
 *   - return value: CSV_OK (0) or a negative CSV_E* code; nothing aborts or
 *     throws across this interface;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the pool's GPU; the caller owns every buffer it
 *     passes in, the library owns what it allocates (pools, blobs it
 *     returns, servers);
 *   - volumes are C order [z][y][x] with x fastest, labels uint32; brick ids
 *     run x fastest: id = bx + nbx * (by + nby * bz);
 *   - decoded bricks are dense [z][y][x] blocks of (32 >> lod)^3 uint32.
 *   - a `stream` argument is a hipStream_t (NULL = the default stream).
 */
#ifndef CSV_H
#define CSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CSV_OK = 0,
    CSV_EINVAL = -1,   /* bad argument (null pointer, unsupported parameter) */
    CSV_ERANGE = -2,   /* brick id or level of detail out of range */
    CSV_ECORRUPT = -3, /* malformed container or record */
    CSV_ENOMEM = -4,   /* host or device allocation failed */
    CSV_EHIP = -5,     /* a HIP runtime call failed */
    CSV_EBUSY = -6,    /* resource temporarily exhausted (server admission) */
    CSV_EDETAIL = -7   /* a full-LOD request whose level-0 detail is not on the device (pool with
                          detail in host memory, csv_pool_stage_detail): level 1 was decoded and
                          written upsampled 2x */
};

#define CSV_ABI_VERSION 4u
uint32_t csv_abi_version(void);

/* Human-readable name of a CSV_E* code (static string). */
const char *csv_strerror(int code);

/* ------------------------------------------------------------------ */
/* Encoding (Sec. 3.1-3.4; the paper's compressor is a CPU program)    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t brick_log2;    /* log2 of the brick edge; 5 (32^3) is what the GPU decodes; 1..6 */
    uint32_t scale_bits;    /* rANS table precision: frequencies sum to 2^scale_bits; 8..12 */
    uint32_t lane_k;        /* interleaving rule: W = largest power of two <= min(lane_max, n_symbols / lane_k) */
    uint32_t lane_max;      /* at most this many interleaved rANS states per brick (power of two <= 64) */
    uint32_t sample_stride; /* frequency-table prepass samples every sample_stride-th brick; 0 = 512,
                               or 4096 above 2^20 bricks (Sec. 3.4) */
    uint32_t threads;       /* host threads; 0 = all hardware threads */
    uint32_t tables;        /* rANS frequency tables: 2 = one for the symbols of levels >= 1 and one for L_0
                               (Sec. 3.3); 1 = one table for all symbols (stored twice; Table 1's variant);
                               0 = 2 */
    uint32_t coding;        /* 0 = interleaved rANS (Sec. 3.3); 1 = no entropy coding (Table 1's "no rANS"
                               variant): each record holds its symbols as raw nibbles, symbol i in bits
                               4 (i mod 4) .. + 3 of 16-bit word i / 4 (unused nibbles zero), no states
                               (W = 0), and the header's coding word (the first reserved word) is 1;
                               its frequency tables are uniform and unused */
} csv_encode_opts;

/* Defaults: brick_log2 5, scale_bits 10, lane_k 64, lane_max 64, sample_stride 0, threads 0, tables 2,
 * coding 0. */
void csv_encode_opts_default(csv_encode_opts *o);

/*
 * Compress a label volume (host memory, nx*ny*nz uint32, x fastest) into a
 * container blob.  Bricks that reach past the volume are padded with label
 * 0.  On success *blob points to *blob_bytes bytes allocated by the library;
 * release them with csv_free.  opts may be NULL for the defaults.
 * Errors: CSV_EINVAL (null pointers, zero dims, options out of range),
 * CSV_ERANGE (2^32 or more bricks), CSV_ENOMEM.
 */
int csv_encode_volume(const uint32_t *labels, uint32_t nx, uint32_t ny, uint32_t nz, const csv_encode_opts *opts,
                      uint8_t **blob, size_t *blob_bytes);

void csv_free(void *p);

/*
 * The same container as csv_encode_volume, byte for byte, compressed on the
 * GPU (Sec. 3: pyramid, operations, two sampled frequency tables,
 * interleaved rANS; the paper leaves a GPU encoder to future work, Sec. 5.1).
 * labels: device memory of `device`, nx*ny*nz uint32, x fastest; the work
 * runs on `stream` (NULL: the null stream) and the call returns when the
 * blob is in host memory (*blob, release with csv_free).  Only 32^3 bricks
 * (opts->brick_log2 5) and rANS coding (opts->coding 0); opts->threads is
 * ignored.  The call keeps its device
 * buffers (about 430 KiB per workgroup, 5 workgroups per CU, plus the
 * records and the container) and a pinned host buffer of the container's
 * size for later calls on the same device, until csv_encode_gpu_release;
 * calls on one device run one at a time.  Errors: CSV_EINVAL (null
 * pointers, zero dims, options out of range, a bad device), CSV_ERANGE
 * (2^32 or more bricks), CSV_ENOMEM, CSV_EHIP.
 */
int csv_encode_volume_gpu(const uint32_t *labels, uint32_t nx, uint32_t ny, uint32_t nz, const csv_encode_opts *opts,
                          int device, void *stream, uint8_t **blob, size_t *blob_bytes);
/* Free the buffers csv_encode_volume_gpu keeps for `device` (waits for the device). */
int csv_encode_gpu_release(int device);

typedef struct {
    uint32_t nx, ny, nz, brick_log2, nbx, nby, nbz, n_bricks;
    uint32_t scale_bits, lane_k, lane_max, sample_stride;
    uint32_t freq[2][16]; /* interior table (children on levels >= 1), leaf table (children on L_0) */
    uint64_t record_bytes; /* sum of all brick records */
    uint64_t blob_bytes;
    uint32_t coding;       /* 0 interleaved rANS, 1 raw nibbles (csv_encode_opts.coding) */
    uint32_t reserved;
} csv_volume_info;

/* Parse and validate a container header (host memory). */
int csv_blob_info(const uint8_t *blob, size_t blob_bytes, csv_volume_info *info);

/*
 * Validate the header and every record of a container (host memory, no
 * device needed): record offsets 4-byte aligned and increasing, each record
 * holding its header; per record P >= 1 (P = 1 exactly when the brick has no
 * symbols), W a power of two <= 64 and zero exactly when there are no
 * symbols (raw coding: W = 0 and exactly ceil(symbols / 4) words),
 * cumulative symbol counts non-increasing from the finest child
 * level and at most two per node, and header + palette + states + words
 * within the record (sums in 64 bits).  csv_pool_add_volume runs it before
 * anything reaches the device.  Errors: as csv_blob_info, CSV_ECORRUPT
 * with *first_bad (may be NULL) set to the first bad brick.
 */
int csv_blob_check(const uint8_t *blob, size_t blob_bytes, uint32_t *first_bad);

/* ------------------------------------------------------------------ */
/* Device pool: compressed volumes resident in HBM (Sec. 4)            */
/* ------------------------------------------------------------------ */
typedef struct csv_pool csv_pool;

/* Create an empty pool on HIP device `device`.  Decodes only read the pool,
 * so csv_decode_* may run concurrently on several streams: each stream gets
 * its own set of launch buffers (work counters, hand-off slots, lists and,
 * for pools that need them, global replay arenas), up to 16 sets per pool; a
 * 17th stream takes over the least recently used set after waiting for the
 * whole device.  csv_pool_add_volume must not overlap decodes. */
int csv_pool_create(csv_pool **pool, int device);
/* csv_pool_create with a limit on the HBM the pool holds (records, tables,
 * launch buffers, staging; csv_pool_info's device_bytes): adding a volume or
 * growing launch buffers past it fails with CSV_ENOMEM.  0: no limit. */
int csv_pool_create_budget(csv_pool **pool, int device, uint64_t hbm_budget_bytes);
void csv_pool_destroy(csv_pool *pool);

/*
 * Copy one container blob (host memory) into the pool's HBM.  The pool keeps
 * its own copy, so the blob may be freed afterwards.  Its bricks get the
 * global ids first_brick_id .. first_brick_id + n_bricks - 1 (volumes are
 * numbered in the order they are added; each keeps its own table pair).
 * Every volume of a pool has the same brick size (edge 2^brick_log2,
 * brick_log2 1..6; another size is CSV_EINVAL).  Pools of 32^3 rANS bricks
 * decode with the tuned kernels; a volume of another brick size or with raw
 * nibbles (csv_encode_opts.coding 1) makes every decode of the pool take the
 * generic decoder (one workgroup per brick, levels in global memory; Table
 * 1's variants), which has no launch shape, no graphs, no
 * csv_decode_bricks_noalloc, no detail separation, no serving loop and no
 * frame cache (those return CSV_EINVAL).  Every record is checked
 * first (csv_blob_check).  Synchronous, with no stream argument: the pool's
 * per-brick arrays and decode tables are re-uploaded, so the call waits for
 * every decode on the device that may read the old ones.  Errors:
 * CSV_EINVAL, CSV_ECORRUPT, CSV_ENOMEM (also past the pool's HBM budget),
 * CSV_EHIP.
 */
int csv_pool_add_volume(csv_pool *pool, const uint8_t *blob, size_t blob_bytes, uint32_t *first_brick_id);

/*
 * Detail separation (Sec. 4.2): with flags CSV_DETAIL_HOST the pool keeps
 * in HBM each record only up to the words that levels >= 1 read (the stream
 * prefix property, Sec. 3.4; found by decoding every brick to level 1 once,
 * which synchronises the device), and the rest of the words in pinned host
 * memory.  Levels of detail >= 1 decode as usual; a full-LOD request needs
 * the brick's detail staged with csv_pool_stage_detail, else level 1 is
 * decoded, written upsampled 2x and CSV_EDETAIL is recorded in the pool's
 * error word.  flags 0 is csv_pool_add_volume.  Errors as
 * csv_pool_add_volume; a brick whose level-1 decode fails keeps its whole
 * record in HBM (the error stays in the pool's error word).
 */
#define CSV_DETAIL_HOST 1u
int csv_pool_add_volume_ex(csv_pool *pool, const uint8_t *blob, size_t blob_bytes, uint32_t flags,
                           uint32_t *first_brick_id);

/*
 * Upload the level-0 detail of bricks brick_ids[0 .. n) (host memory) into
 * the pool's staging buffer in HBM (8 MiB unless csv_pool_set_detail_staging
 * says otherwise; the paper's frames upload 8 MB), asynchronously on
 * `stream`, in order, until the buffer is full.  *n_done receives how many
 * leading ids were handled (bricks of ordinary volumes and bricks already
 * staged count as handled): decodes of those at full LOD, on the same
 * stream after this call, read their detail (the stream also waits for the
 * staging copies that earlier calls made on other streams).  Staged detail
 * stays until csv_pool_release_detail, which must follow the decodes that
 * read it; not for stream capture.  Errors: CSV_EINVAL, CSV_ERANGE (an
 * id out of range: *n_done is its index), CSV_ENOMEM, CSV_EHIP.
 */
int csv_pool_stage_detail(csv_pool *pool, const uint32_t *brick_ids, uint32_t n, void *stream, uint32_t *n_done);
/* Drop all staged detail (after the decodes that used it, in stream order). */
int csv_pool_release_detail(csv_pool *pool, void *stream);
/* The bytes brick_id's level-0 detail takes in the staging buffer (0: its
 * record is whole in HBM), and the staging buffer's size; either pointer may
 * be NULL.  Errors: CSV_EINVAL, CSV_ERANGE (unknown id). */
int csv_pool_detail_bytes(const csv_pool *pool, uint32_t brick_id, uint32_t *bytes, uint64_t *staging_bytes);
/* Size of the staging buffer (bytes, 4 KiB .. 64 GiB); CSV_EBUSY while detail is staged. */
int csv_pool_set_detail_staging(csv_pool *pool, uint64_t bytes);

typedef struct {
    uint32_t n_volumes, n_bricks;
    uint64_t device_bytes; /* HBM held by the pool */
    int device;
    uint32_t brick_log2;   /* brick edge 2^brick_log2 of the pool's volumes (0: no volume yet) */
    uint64_t host_bytes;   /* pinned host memory holding level-0 detail (CSV_DETAIL_HOST volumes) */
} csv_pool_info;
int csv_pool_info_get(const csv_pool *pool, csv_pool_info *info);

/*
 * Output layout helper: for n requests at levels lods_host[i] (host memory,
 * each 0..5), offsets[i] (may be NULL) receives the element offset of
 * request i when bricks are packed back to back in request order, and
 * *total the number of uint32 elements of that packing.
 */
int csv_output_elems(const uint8_t *lods_host, uint32_t n, uint64_t *offsets, uint64_t *total);
/* The same packing in bytes (offsets[i] and *total are 4x the element figures). */
int csv_output_bytes(const uint8_t *lods_host, uint32_t n, uint64_t *offsets, uint64_t *total);
/* csv_output_elems for bricks of edge 2^brick_log2 (1..6): request i takes
 * ((2^brick_log2) >> lods_host[i])^3 elements; CSV_ERANGE for a level past
 * brick_log2. */
int csv_output_elems_log2(uint32_t brick_log2, const uint8_t *lods_host, uint32_t n, uint64_t *offsets,
                          uint64_t *total);

/*
 * THE HOT PATH: decode n bricks on the GPU, asynchronously on `stream`.
 *   brick_ids    device, uint32[n], global pool ids
 *   lods         device, uint8[n] levels of detail 0..5, or NULL: every
 *                request uses lod_scalar (Sec. 3.4: LOD t reads only the
 *                stream prefix of levels >= t; t = 5 is palette[0], Sec. 4)
 *   out_offsets  device, uint64[n] element offsets into out, or NULL: request
 *                i is written at i * (32 >> lod_scalar)^3 (requires lods NULL)
 *   out          device, uint32 destination of the decoded blocks
 * Decodes every brick bit-exactly: the result is level L_lod of the brick's
 * resolution pyramid.  Two persistent launches: an entropy decoder that
 * also replays levels 4..max(lod, 1) (a wavefront per brick, many per
 * compute unit; Sec. 3.3, Sec. 3.2) and leaves level 1 and the leaf-level
 * symbols of each full-LOD brick in a pool buffer, then the leaf-level
 * replay and output (an 8-wavefront workgroup per brick; Alg. 1),
 * plus a third launch for pools holding bricks whose leaf arrays may not
 * fit that workgroup's LDS.
 * Large batches are split into chunks that alternate between `stream` and
 * a second stream the pool creates for it (csv_shape.chunks); the call is
 * still one ordered operation on `stream`.
 * Each stream has its own intermediate buffers (up to 16 streams per pool
 * at once, second streams included; a 17th waits for all work on the
 * device), so decodes on different streams may overlap; decodes on one
 * stream run in order.  The
 * buffers grow on demand, which synchronises the stream, and cannot grow
 * inside a stream capture (CSV_EBUSY): capture with csv_graph_create.
 * Argument errors are returned synchronously.  Errors found on the device
 * (bad brick id or level, malformed record) are recorded in the pool's
 * error word (first error wins, read with csv_pool_last_error after the
 * stream is synchronised) and the affected brick's output is zero-filled.
 */
int csv_decode_bricks(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods, uint32_t lod_scalar,
                      const uint64_t *out_offsets, uint32_t n, uint32_t *out, void *stream);

/* csv_decode_bricks that also reports errors per request: status is
 * device-accessible int32[n] (device memory, or mapped pinned host memory)
 * that the caller fills with 0 beforehand; a request that fails gets its
 * CSV_E* code in status[i] (CSV_EDETAIL for a level-1 fallback), the
 * others are left untouched.  The pool's error word is set as well.
 * Errors as csv_decode_bricks. */
int csv_decode_bricks_status(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods,
                             uint32_t lod_scalar, const uint64_t *out_offsets, uint32_t n, uint32_t *out,
                             void *stream, int32_t *status);

/* csv_decode_bricks for a request list whose length is known only on the
 * device (Sec. 4.1: a frame's bricks to decode, found by a kernel):
 *   n_max   requests the arrays hold (host; bounds the launch and the
 *           intermediate buffers)
 *   n_dev   device uint32: the kernels decode requests 0 .. min(n_max,
 *           *n_dev) - 1, reading the count when they start; the output of
 *           the other requests is not written
 * Nothing waits for the device, so the call can be captured in a graph
 * once the stream's buffers are sized for n_max (a first call outside the
 * capture).  One launch pair on `stream` (no chunks, no longest-first
 * order).  Pools of other brick sizes or raw nibbles: CSV_EINVAL.  Other
 * arguments and errors as csv_decode_bricks. */
int csv_decode_bricks_devcount(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods,
                               uint32_t lod_scalar, const uint64_t *out_offsets, uint32_t n_max,
                               const uint32_t *n_dev, uint32_t *out, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): csv_decode_bricks
 * with the same arguments, results and errors, that allocates nothing.  Its
 * intermediate buffers (launch counters, request lists, the per-request
 * slots that carry level 1 and the leaf symbols from the entropy decoder to
 * the leaf kernel, and 32 global arenas for bricks too large for LDS) live
 * in one fixed device array of 64 MiB that the library holds on every GPU
 * it runs on until the process ends.  The requests are decoded in
 * consecutive chunks of as many as that array holds (about
 * (64 MiB - 2.6 MiB) / (slot + 12 bytes), where a slot is about half a byte
 * per symbol of the pool's largest brick plus 10 KB: some 2,600 requests of
 * a dense 32^3 volume), each chunk one launch pair in stream order.
 * CSV_ERANGE if a single request's slot would not fit the array.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (several
 * streams or host threads at once) race and corrupt each other's output;
 * serialise them.  Each call clears the counters it needs (with a kernel).
 * Uses the pool's launch shape (csv_pool_set_shape, csv_autotune).  The
 * caller still owns and passes the inputs and the output. */
int csv_decode_bricks_noalloc(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods,
                              uint32_t lod_scalar, const uint64_t *out_offsets, uint32_t n, uint32_t *out,
                              void *stream);

/* Baseline: the same kernels launched once per brick (a grid of one
 * wavefront, then a grid of one workgroup: 2n launches on `stream`, 3n for
 * pools that need the global-memory leaf kernel).  Same arguments and
 * results. */
int csv_decode_bricks_plain(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods, uint32_t lod_scalar,
                            const uint64_t *out_offsets, uint32_t n, uint32_t *out, void *stream);

/* Launch shape of a batched decode.  Every shape gives the same bytes. */
typedef struct {
    int waves_per_group;    /* front kernel: wavefronts per workgroup, 4, 8 or 16 (each decodes its
                               own bricks; 8 KiB of LDS per wavefront), or 2: two wavefronts per
                               brick, one decoding the symbols while the other replays the levels
                               above L_0 (shorter per-brick latency for batches too small to fill
                               the GPU; no work counter) */
    uint32_t groups_per_cu; /* leaf kernel: 8-wavefront workgroups per compute unit, 1..8; each holds
                               160 KiB / groups_per_cu of LDS (rounded down to 4 KiB; bricks
                               whose arrays do not fit take a slower path through a global-memory
                               arena) */
    int use_queue;          /* front kernel: 1: waves take requests from a device work counter;
                               0: static round robin (the leaf kernel always takes its bricks from
                               a counter after a first fixed round) */
    int lpt_order;          /* 1: requests are first ordered longest-first (binned by their symbols
                               + output voxels / 8, 8 bins per octave; two small kernels before the
                               decode) and laid out in snake rounds for the front kernel's round
                               robin; skipped when each front wavefront gets at most one request */
    uint32_t chunks;        /* 1..64: the requests are split into this many consecutive chunks that
                               alternate between the caller's stream and a second stream the pool
                               keeps for it, so that the entropy decode of one chunk overlaps the
                               leaf level of the previous one (at most n / 2048 chunks; 1: one
                               launch pair; graphs, csv_decode_bricks_noalloc and stream captures
                               use one) */
    float ms;               /* csv_autotune: the measured time per launch of this shape */
} csv_shape;

/* csv_decode_bricks with an explicit launch shape.  Errors as csv_decode_bricks. */
int csv_decode_bricks_shaped(const csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods,
                             uint32_t lod_scalar, const uint64_t *out_offsets, uint32_t n, uint32_t *out,
                             void *stream, const csv_shape *shape);

/* The shape csv_decode_bricks uses (default {16, 3, 0, 0, 4}). */
int csv_pool_set_shape(csv_pool *pool, const csv_shape *shape);
int csv_pool_get_shape(const csv_pool *pool, csv_shape *shape);

/*
 * Empty-space test of requested bricks (Sec. 4, empty-space skipping: a
 * brick none of whose palette labels the transfer function makes visible
 * need not be decoded).  For i < n:
 *   visible[i] = 1 if some label of brick brick_ids[i] (its palette: the
 *                brick's distinct labels) has bit (label & 31) of word
 *                label >> 5 set in visible_bits, else 0.
 *   brick_ids     device, uint32[n], global pool ids
 *   visible_bits  device, uint32[(n_label_bits + 31) / 32]; labels >=
 *                 n_label_bits count as invisible (n_label_bits = 0: none
 *                 is visible, and visible_bits may be NULL)
 *   visible       device, uint8[n]
 * All buffers belong to the caller; asynchronous on `stream`; n = 0 does
 * nothing.  An unknown id gives 0 and CSV_ERANGE in the pool's error word
 * (with the request index), a record whose palette does not fit its size
 * gives 0 and CSV_ECORRUPT (with the brick id); read them with
 * csv_pool_last_error.
 */
int csv_bricks_visible(const csv_pool *pool, const uint32_t *brick_ids, uint32_t n, const uint32_t *visible_bits,
                       uint32_t n_label_bits, uint8_t *visible, void *stream);

/* Autotuner: decodes the given request set (same arguments as
 * csv_decode_bricks; `out` is overwritten) with candidate shapes, one
 * coordinate at a time: front waves {8, 16} x leaf groups {2, 3, 4} (static
 * order, min(4, n / 2048) chunks), then the chunk count {1, 2, 4, 8}, then
 * work counters and longest-first order; one warm-up and `reps` timed
 * launches each (HIP events on `stream`).  Makes the fastest the pool's
 * shape and the tuned shape of this request set's class (below), and
 * returns it in *best (may be NULL).  Synchronous.  Not allowed while
 * `stream` is being captured. */
int csv_autotune(csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods, uint32_t lod_scalar,
                 const uint64_t *out_offsets, uint32_t n, uint32_t *out, void *stream, uint32_t reps,
                 csv_shape *best);

/* Tuned shapes are kept per class of request set: the bit length of n,
 * how the levels of detail are given (all full LOD; all one coarser LOD;
 * per request) and the bit length of the pool's mean record size.
 * csv_decode_bricks, _status, _devcount and _noalloc use the shape tuned
 * for the class of their request set (else the tuned class of the same kind
 * and record size with the nearest n, else the pool's shape).  Without a
 * tuned class of its own, a request set that the paired front kernel
 * (waves_per_group 2) takes all at once (one two-wave workgroup per
 * request; 2,048 requests on 256 CUs with 10-bit tables) runs paired,
 * unless the pool's shape was set with csv_pool_set_shape.
 * csv_pool_tuning_save writes them to a text file: a first line
 * "csv-tuning 1 <device architecture name> <compute units>", then one line
 * per class "<n bits> <lod kind> <record bits> <waves> <groups> <queue>
 * <lpt> <chunks> <ms>".  csv_pool_tuning_load adds the classes of such a
 * file to the pool when the device name and compute-unit count match the
 * pool's device (else none; *n_loaded, may be NULL, is the number added).
 * CSV_EINVAL if the file cannot be opened, CSV_ECORRUPT if it is malformed
 * (nothing is added then). */
int csv_pool_tuning_save(const csv_pool *pool, const char *path);
/* The shape a decode of n requests would use (lods: only whether it is NULL
 * matters; lod_scalar when it is). */
int csv_pool_shape_for(const csv_pool *pool, const uint8_t *lods, uint32_t lod_scalar, uint32_t n,
                       csv_shape *shape);
int csv_pool_tuning_load(csv_pool *pool, const char *path, uint32_t *n_loaded);

/* A decode captured once into a HIP graph and replayed.  The graph holds
 * the pointers and n given here and the pool's shape at creation; replays
 * decode the current contents of those buffers.  The graph owns its
 * intermediate buffers, sized for the pool's bricks at creation (a brick
 * added later with more symbols is reported as CSV_EINVAL).  Replays of one
 * graph must not overlap each other (they share one work counter).
 * `stream` is the capture stream (NULL: a private stream); launch on any
 * stream.  csv_graph_launch returns CSV_EBUSY once a volume has been added
 * to the pool after the capture (the pool's tables moved): create it again. */
typedef struct csv_graph csv_graph;
int csv_graph_create(csv_pool *pool, const uint32_t *brick_ids, const uint8_t *lods, uint32_t lod_scalar,
                     const uint64_t *out_offsets, uint32_t n, uint32_t *out, void *stream, csv_graph **graph);
int csv_graph_launch(csv_graph *graph, void *stream);
void csv_graph_destroy(csv_graph *graph);

/* First device-side error since the last call (synchronises the pool's
 * device and clears the word): *code is CSV_OK or a CSV_E* code,
 * *brick_id the global id it concerns (or the request index when the id
 * itself was out of range). */
int csv_pool_last_error(csv_pool *pool, int *code, uint32_t *brick_id);

/* ------------------------------------------------------------------ */
/* Serving (Sec. 4, Sec. 4.1: requested bricks are decoded into a GPU    */
/* cache in parallel; here continuously, request by request)            */
/* ------------------------------------------------------------------ */
typedef struct csv_server csv_server;

typedef struct {
    uint64_t cache_bytes;    /* decoded-brick cache in HBM (LRU per LOD class, 128 KiB pages) */
    uint64_t inflight_bytes; /* admission budget: decoded bytes of admitted, unfinished requests
                                (at most a quarter of cache_bytes is used) */
    uint32_t max_batch;      /* bricks per launch */
    uint32_t streams;        /* batches that may run on the GPU at once (1..16) */
} csv_server_opts;

/* Defaults: 1 GiB cache, 256 MiB in flight, 4096 bricks per batch, 4 streams. */
void csv_server_opts_default(csv_server_opts *o);

typedef struct {
    uint32_t brick_id;     /* global pool id */
    uint32_t lod;          /* 0..5 */
    uint64_t tag;          /* returned with the completion */
    uint64_t t_arrival_ns; /* csv_now_ns() clock */
} csv_request;

typedef struct {
    uint64_t tag;
    uint32_t brick_id, lod;
    const uint32_t *data;  /* device pointer into the cache: (32 >> lod)^3 labels, dense [z][y][x];
                              valid until the next csv_server_poll call returns */
    uint32_t elems;
    int32_t status;        /* CSV_OK, CSV_ERANGE (bad id or LOD) or a decode error */
    uint32_t hit;          /* 1: served from the cache */
    uint32_t skipped;      /* 1: invisible under the visibility table, not decoded (data NULL) */
    uint64_t t_arrival_ns, t_done_ns;
} csv_completion;

typedef struct {
    uint64_t requests, hits, misses, joined, completed, batches, evictions, rebuilds;
    uint64_t decoded_bytes, cache_bytes_used;
    double p50_us, p99_us, p50_miss_us, p99_miss_us, max_us; /* arrival -> completion */
    int32_t error;
    int32_t pad;
    uint64_t worker_busy_ns;   /* worker thread time spent on requests and batches */
    uint64_t worker_launch_ns; /* ... of which launching batches */
    uint64_t stall_batch, stall_inflight, stall_slot; /* admission rounds stopped by: no free batch,
                                                         the in-flight budget, no cache slot */
    uint64_t skipped;          /* requests completed as invisible (not in the latency figures) */
    uint64_t stall_staging;    /* admission rounds stopped by a full detail staging buffer */
    uint64_t detail_staged_bytes; /* level-0 detail promised to full-LOD misses (staging granules) */
    uint64_t detail_releases;  /* times the staged detail was dropped */
    uint64_t failed;           /* decodes that failed on the device (their requests completed with the
                                  kernel's error code, nothing cached); `error` holds the last code */
} csv_stats;

/* Clock of arrival and completion times (steady, nanoseconds). */
uint64_t csv_now_ns(void);

/* Start a server on a pool (its own worker thread, streams, HBM cache).
 * The pool must outlive the server and gain no volumes while it runs.  On a
 * pool holding level-0 detail in host memory (CSV_DETAIL_HOST, Sec. 4.2) a
 * full-LOD miss is admitted while the pool's staging buffer has room for
 * its detail; a batch stages the detail of its full-LOD bricks on its
 * stream before the decode, and the staged detail is released once no
 * launched batch reads it.  A full-LOD request whose detail exceeds the
 * staging buffer completes with CSV_EDETAIL (data NULL).  The staging
 * buffer is not resized while the server runs. */
int csv_server_create(csv_pool *pool, const csv_server_opts *opts, csv_server **server);
/* Queue n requests (host memory; thread safe; returns at once). */
int csv_server_submit(csv_server *server, const csv_request *requests, uint32_t n);
/* Take up to cap completions (host memory).  Calling poll again releases the
 * cache entries of the completions returned by the previous call; a client
 * that stops polling eventually blocks admission. */
int csv_server_poll(csv_server *server, csv_completion *completions, uint32_t cap, uint32_t *got);
int csv_server_stats(csv_server *server, csv_stats *stats);
/* Copy a completion's brick to host memory (elems uint32); valid until the
 * next csv_server_poll, like the completion itself. */
int csv_server_read(csv_server *server, const csv_completion *completion, uint32_t *host_dst);
/* Device address of the server's decoded-brick cache (a completion's data
 * lies at a byte offset below opts.cache_bytes from it); NULL for NULL. */
const uint32_t *csv_server_cache_data(const csv_server *server);
int csv_server_reset_stats(csv_server *server);
/* Empty-space skipping in serving (Sec. 4): with a visibility table set, a
 * request for a brick whose byte is 0 completes at once without a decode
 * (status CSV_OK, skipped 1, data NULL, elems 0).  visible: host, one byte
 * per global brick id (n_bricks must be the pool's brick count; e.g. from
 * csv_bricks_visible over every brick), copied; NULL clears the table (every
 * brick is decoded).  Thread safe; requests submitted after it returns are
 * admitted under the new table. */
int csv_server_set_visible(csv_server *server, const uint8_t *visible, uint32_t n_bricks);
/* Replay a trace in real time (arrival times relative to the start); see csv_server.cpp. */
int csv_server_run_trace(csv_server *server, const csv_request *requests, uint32_t n, csv_completion *done,
                         uint64_t timeout_ns, uint32_t *n_done);
void csv_server_destroy(csv_server *server);

/*
 * Frame cache of decoded bricks on the GPU (Sec. 4.1, after Shading Atlas
 * Streaming), the per-frame alternative to the serving loop's LRU cache.
 * The cache memory is a pool of base elements of 2^3 voxels; a brick at LOD
 * t (0..4) takes a block of 8^(4-t) contiguous elements.  Free blocks sit on
 * one stack per LOD; when a stack runs empty the shared top pointer
 * advances; when the top would pass the end, the cache is rebuilt (emptied,
 * then every brick of the frame decoded again).  A block keeps its LOD.
 * Each frame's request list decides the contents: entries that the frame
 * does not request, or that its visibility test rejects, are evicted and
 * their blocks pushed on their stacks.  LOD 5 is the brick's palette[0] and
 * is never stored.
 */
typedef struct csv_frame_cache csv_frame_cache;
typedef struct {
    uint32_t frame;            /* frame number, from 1 */
    uint32_t requests;         /* n */
    uint32_t distinct;         /* distinct visible (brick, LOD < 5) keys */
    uint32_t new_entries;      /* ... of which not cached before the frame */
    uint32_t decoded;          /* bricks decoded in this frame (all distinct ones after a rebuild) */
    uint32_t hits;             /* distinct - decoded */
    uint32_t evicted;          /* entries dropped at the start of the frame */
    uint32_t rebuilt;          /* 1: the cache was rebuilt */
    uint64_t used_bytes;       /* base elements handed out (top pointer), in bytes */
    uint64_t capacity_bytes;
} csv_frame_stats;

/* A cache of cache_bytes (rounded down to 32 bytes) for frames of at most
 * max_requests requests over the pool's current bricks.  The pool must
 * outlive the cache and gain no volumes while it exists.  Errors:
 * CSV_EINVAL, CSV_ENOMEM. */
int csv_frame_cache_create(csv_pool *pool, uint64_t cache_bytes, uint32_t max_requests, csv_frame_cache **cache);

/*
 * One frame: requests brick_ids[n], lods[n] (device memory); with
 * visible_bits / n_label_bits as in csv_bricks_visible (NULL and 0: no
 * test), invisible requests are not cached.  On return the bricks are being
 * decoded into the cache on `stream` and slots[i] (device uint64[n]) will
 * hold the element offset of request i's block in csv_frame_cache_data (the
 * (32 >> lod)^3 labels in x-fastest order), or UINT64_MAX for LOD 5,
 * invisible or unknown requests.  Frames of one cache run one at a time.
 * With stats (not NULL) the call waits for the stream once (the frame state
 * goes to the host between the cache update and the decode) and *stats
 * describes the frame.  With stats NULL nothing waits for the device: the
 * decode takes the number of bricks from device memory
 * (csv_decode_bricks_devcount), so the frame can be captured in a graph;
 * csv_frame_cache_last_stats gives its statistics later.  Errors:
 * CSV_EINVAL (null pointers, n above max_requests), CSV_ENOMEM (with stats:
 * the frame's distinct bricks alone exceed the cache: nothing is cached,
 * every slot UINT64_MAX; without stats the same frame returns CSV_OK and
 * csv_frame_cache_last_stats reports CSV_ENOMEM), CSV_EHIP.  A cache over a
 * pool that keeps level-0 detail in host memory takes its frames through
 * csv_frame_cache_frame_detail (this call returns CSV_EINVAL).
 */
int csv_frame_cache_frame(csv_frame_cache *cache, const uint32_t *brick_ids, const uint8_t *lods, uint32_t n,
                          const uint32_t *visible_bits, uint32_t n_label_bits, uint64_t *slots, void *stream,
                          csv_frame_stats *stats);

/*
 * Detail streaming in frames (Sec. 4.2) for caches over pools that keep
 * level-0 detail in host memory (CSV_DETAIL_HOST).  A full-LOD request for
 * a brick whose detail is not on the device, and whose full LOD is not
 * cached, is served at LOD 1, the finest level in HBM: its slot holds the
 * 16^3 block, served_lods[i] says 1, and the brick is listed as wanting its
 * detail.  The next frame of the cache first uploads that detail, then the
 * detail of predict_ids (device, uint32[n_predict], n_predict <= the
 * cache's max_requests; e.g. the bricks close to the camera, most urgent
 * first) that are not cached at full LOD after this frame, so that a
 * predicted brick is decoded at full LOD in the first frame that requests
 * it.  Uploads go through the pool's staging buffer; detail already there
 * stays while the new detail fits behind it, else all of it is dropped
 * first and the lists are staged from the start until the buffer is full.
 * While the cache exists the pool's staged detail is the cache's: no other
 * caller stages or releases detail on that pool, and its frames run on one
 * stream (the staging of a frame follows the previous frame's work in
 * stream order).  The lists reach the host after the frame's work; the
 * next frame waits for them.  Not for stream capture.  Detail the cache
 * staged stays staged after csv_frame_cache_destroy (csv_pool_release_detail
 * drops it).
 *   served_lods  device, uint8[n], or NULL: the LOD of the block slots[i]
 *                points at (0xFF when slots[i] is UINT64_MAX)
 *   stats, detail_stats  as csv_frame_cache_frame's stats; detail_stats
 *                (may be NULL; needs stats) describes the frame's detail
 * Other arguments and errors as csv_frame_cache_frame; on a cache over a
 * pool without detail in host memory the call is csv_frame_cache_frame
 * with served_lods.
 */
typedef struct {
    uint32_t fallbacks;       /* bricks requested at full LOD and served at LOD 1 in this frame */
    uint32_t wanted;          /* the previous frame's fallbacks */
    uint32_t predicted;       /* bricks of the previous frame's predictions not cached at full LOD */
    uint32_t staged;          /* of wanted + predicted (each brick once): detail on the device for this frame */
    uint32_t released;        /* 1: the staged detail was dropped to make room */
    uint32_t pad;
    uint64_t uploaded_bytes;  /* detail uploaded for this frame (staging granules) */
    uint64_t resident_bytes;  /* detail staged by the cache after the upload */
} csv_frame_detail_stats;
int csv_frame_cache_frame_detail(csv_frame_cache *cache, const uint32_t *brick_ids, const uint8_t *lods, uint32_t n,
                                 const uint32_t *visible_bits, uint32_t n_label_bits, const uint32_t *predict_ids,
                                 uint32_t n_predict, uint64_t *slots, uint8_t *served_lods, void *stream,
                                 csv_frame_stats *stats, csv_frame_detail_stats *detail_stats);
/* Statistics of the cache's last frame (waits for all work on the device).
 * Returns CSV_ENOMEM if that frame did not fit (see csv_frame_cache_frame),
 * else CSV_OK; CSV_EINVAL for null pointers, CSV_EHIP. */
int csv_frame_cache_last_stats(csv_frame_cache *cache, csv_frame_stats *stats);
/* Device address of the cache memory (uint32 labels). */
uint32_t *csv_frame_cache_data(csv_frame_cache *cache);
/* Copy n labels from element elem_offset of the cache to host memory (synchronous,
 * after all work on the device).  Errors: CSV_EINVAL (out of range), CSV_EHIP. */
int csv_frame_cache_read(csv_frame_cache *cache, uint64_t elem_offset, uint64_t n, uint32_t *host_dst);
void csv_frame_cache_destroy(csv_frame_cache *cache);

#ifdef __cplusplus
}
#endif
#endif /* CSV_H */
