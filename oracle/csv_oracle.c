/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, deliberately literal CPU implementation of compressed
 * segmentation volumes (Piochowiak & Dachsbacher, "Fast Compressed
 * Segmentation Volumes for Scientific Visualization", IEEE TVCG 2023):
 *   - the per-brick resolution pyramid            (Sec. 3.1, Sec. 3.4)
 *   - the brick encoder                           (Sec. 3.2, Alg. 2)
 *   - the two static frequency tables             (Sec. 3.3, Sec. 3.4)
 *   - rANS over the 4-bit operation nibbles       (Sec. 3.3)
 *   - the brick decoder to a level of detail t    (Sec. 3.4, Alg. 1)
 *   - the volume container that holds them        (byte layout is ours)
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this code.  It shares no source with the GPU library.
 *
 * Readings of the paper used here (each one is forced by the paper being
 * silent or self-contradictory at that point):
 *   R1  Morton order: bit 0 of every 3-bit group is x, bit 1 is y, bit 2 is
 *       z; child k of a node has offsets (k&1, k>>1&1, k>>2).
 *   R2  Mode of the 8 children; a tie goes to the tied label that occurs
 *       first in child order k = 0..7.
 *   R3  A node's stop bit ("constantChildren") means its whole subtree holds
 *       one label; children on the finest level L_0 always carry stop 0.
 *   R4  The root has no operation: it is palette[0].  A uniform brick has a
 *       one-entry palette and no symbols.
 *   R5  Neighbour reuse R_x/R_y/R_z of a child whose coordinate bit on that
 *       axis is 0 takes the same-level node at coordinate - 1; with bit 1 it
 *       takes the parent of the node at coordinate + 1 (a later node along
 *       the curve).  References leaving the brick are not applicable.
 *   R6  P_delta takes palette[i_p - delta - 1] (the prose definition; the
 *       algorithm listing's palette[i_p - delta] would duplicate P_0); the
 *       smallest matching delta in [0,15] is used.
 *   R7  Operation codes are the positions in the encoder's test order:
 *       R_p 0, R_x 1, R_y 2, R_z 3, P_0 4, P_delta 5, P_a 6 (7 is invalid);
 *       a nibble is code | stop << 3.
 *   R8  Stream layout: one segment per child level, coarse to fine.  A
 *       segment holds the delta nibbles of that level's P_delta operations
 *       (in operation order) followed by the 8 operation nibbles of every
 *       expanded parent in Morton order: the encoder emits a delta before
 *       its (op, stop) nibble, as in Alg. 2, grouped per level.  The decoder
 *       knows how many deltas precede the operations: the segment length
 *       minus 8 per expanded parent.  Segments of children at level >= 1 use
 *       the interior table, the L_0 segment uses the leaf table.
 *   R9  rANS: 32-bit state, lower bound 2^16, 16-bit renormalisation words,
 *       table precision 2^scale_bits, encoding in reverse symbol order
 *       starting from state 2^16.  W interleaved states (W a power of two)
 *       take the symbols round robin (symbol i -> state i mod W) and share
 *       one word stream that the decoder reads in symbol order.
 *   R10 Frequency tables: every nibble value gets count + 1, scaled to the
 *       table total and corrected to sum exactly to it.
 *   R11 Table 1's variant without rANS: the same symbol stream stored as
 *       raw nibbles, symbol i in bits 4(i mod 4) .. 4(i mod 4) + 3 of
 *       16-bit word i / 4, the unused high nibbles of the last word zero.
 *       The header's coding field (the first reserved word) is 1, the
 *       record has no states (W = 0), and its two frequency tables are
 *       uniform (unused).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ECORRUPT (-3)
#define ORC_ENOMEM (-4)

enum { OP_RP = 0, OP_RX = 1, OP_RY = 2, OP_RZ = 3, OP_P0 = 4, OP_PD = 5, OP_PA = 6 };

#define MAX_LOG2 6
#define RANS_L (1u << 16)

/* ------------------------------------------------------------------ */
/* Morton order inside a brick (R1)                                    */
/* ------------------------------------------------------------------ */
static uint32_t morton(uint32_t x, uint32_t y, uint32_t z, int bits) {
    uint32_t m = 0;
    for (int b = 0; b < bits; b++) {
        m |= ((x >> b) & 1u) << (3 * b);
        m |= ((y >> b) & 1u) << (3 * b + 1);
        m |= ((z >> b) & 1u) << (3 * b + 2);
    }
    return m;
}
static void unmorton(uint32_t m, int bits, uint32_t c[3]) {
    c[0] = c[1] = c[2] = 0;
    for (int b = 0; b < bits; b++) {
        c[0] |= ((m >> (3 * b)) & 1u) << b;
        c[1] |= ((m >> (3 * b + 1)) & 1u) << b;
        c[2] |= ((m >> (3 * b + 2)) & 1u) << b;
    }
}
static uint64_t pow8(int e) { return (uint64_t)1 << (3 * e); }

/* ------------------------------------------------------------------ */
/* Resolution pyramid (Sec. 3.1): L_0 = brick, L_l = mode of 8 children */
/* ------------------------------------------------------------------ */
typedef struct {
    int N;
    uint32_t *lab[MAX_LOG2 + 1]; /* level l, Morton order, 8^(N-l) nodes */
    uint8_t *cst[MAX_LOG2 + 1];  /* subtree holds one label (R3) */
} pyramid;

static void pyr_free(pyramid *p) {
    for (int l = 0; l <= p->N; l++) { free(p->lab[l]); free(p->cst[l]); }
}

/* brick: b^3 labels, x fastest */
static int pyr_build(pyramid *p, const uint32_t *brick, int N) {
    memset(p, 0, sizeof(*p));
    p->N = N;
    uint32_t b = 1u << N;
    for (int l = 0; l <= N; l++) {
        p->lab[l] = (uint32_t *)malloc(sizeof(uint32_t) * pow8(N - l));
        p->cst[l] = (uint8_t *)malloc(pow8(N - l));
        if (!p->lab[l] || !p->cst[l]) { pyr_free(p); return ORC_ENOMEM; }
    }
    for (uint32_t z = 0; z < b; z++)
        for (uint32_t y = 0; y < b; y++)
            for (uint32_t x = 0; x < b; x++) {
                uint32_t m = morton(x, y, z, N);
                p->lab[0][m] = brick[x + b * (y + b * z)];
                p->cst[0][m] = 1;
            }
    for (int l = 1; l <= N; l++) {
        for (uint64_t m = 0; m < pow8(N - l); m++) {
            const uint32_t *ch = p->lab[l - 1] + 8 * m;
            /* most frequent child label; ties to the first in child order (R2) */
            int best_k = 0, best_n = 0;
            for (int k = 0; k < 8; k++) {
                int n = 0;
                for (int q = 0; q < 8; q++) n += (ch[q] == ch[k]);
                if (n > best_n) { best_n = n; best_k = k; }
            }
            p->lab[l][m] = ch[best_k];
            int c = 1;
            for (int k = 0; k < 8; k++) c &= p->cst[l - 1][8 * m + k] && (ch[k] == ch[0]);
            p->cst[l][m] = (uint8_t)c;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Brick encoder (Alg. 2)                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t *pal; uint32_t np, cap;
} u32vec;
static int vpush(u32vec *v, uint32_t x) {
    if (v->np == v->cap) {
        uint32_t nc = v->cap ? 2 * v->cap : 64;
        uint32_t *q = (uint32_t *)realloc(v->pal, sizeof(uint32_t) * nc);
        if (!q) return ORC_ENOMEM;
        v->pal = q; v->cap = nc;
    }
    v->pal[v->np++] = x;
    return ORC_OK;
}

/*
 * bestOperation: the first applicable operation in the order
 * R_p, R_x, R_y, R_z, P_0, P_delta, P_a (Sec. 3.4).  Child j = 8m+k lies on
 * level l-1; its parent m on level l.
 */
static int best_operation(const pyramid *p, int l, uint32_t j, const u32vec *pal, int *delta) {
    int N = p->N;
    uint32_t L = p->lab[l - 1][j];
    uint32_t parent = p->lab[l][j >> 3];
    if (parent == L) return OP_RP;
    uint32_t G = 1u << (N - (l - 1)); /* grid size of level l-1 */
    uint32_t c[3];
    unmorton(j, N - (l - 1), c);
    for (int a = 0; a < 3; a++) {
        uint32_t n[3] = {c[0], c[1], c[2]};
        uint32_t v;
        if ((c[a] & 1u) == 0) { /* same-level neighbour at coordinate - 1 (R5) */
            if (c[a] == 0) continue;
            n[a] = c[a] - 1;
            v = p->lab[l - 1][morton(n[0], n[1], n[2], N - (l - 1))];
        } else { /* later neighbour at coordinate + 1: use its parent (R5) */
            if (c[a] + 1 >= G) continue;
            n[a] = c[a] + 1;
            v = p->lab[l][morton(n[0] >> 1, n[1] >> 1, n[2] >> 1, N - l)];
        }
        if (v == L) return OP_RX + a;
    }
    uint32_t ip = pal->np - 1; /* index of the last used palette entry */
    if (pal->pal[ip] == L) return OP_P0;
    for (int d = 0; d <= 15; d++) { /* R6 */
        if ((int64_t)ip - d - 1 < 0) break;
        if (pal->pal[ip - d - 1] == L) { *delta = d; return OP_PD; }
    }
    return OP_PA;
}

/* symbol stream of one brick */
typedef struct {
    uint8_t *sym; uint32_t n, cap;
    uint32_t cum[MAX_LOG2];   /* cum[m]: symbols through the segment of child level m */
    u32vec pal;
    uint64_t op_hist[8];
} brick_stream;

static int spush(brick_stream *s, uint8_t v) {
    if (s->n == s->cap) {
        uint32_t nc = s->cap ? 2 * s->cap : 1024;
        uint8_t *q = (uint8_t *)realloc(s->sym, nc);
        if (!q) return ORC_ENOMEM;
        s->sym = q; s->cap = nc;
    }
    s->sym[s->n++] = v;
    return ORC_OK;
}
static void bs_free(brick_stream *s) { free(s->sym); free(s->pal.pal); memset(s, 0, sizeof(*s)); }

static int encode_brick_stream(const uint32_t *brick, int N, brick_stream *s) {
    memset(s, 0, sizeof(*s));
    pyramid p;
    int rc = pyr_build(&p, brick, N);
    if (rc) return rc;
    rc = vpush(&s->pal, p.lab[N][0]); /* palette <- root label */
    uint8_t *dl = (uint8_t *)malloc(pow8(N) + 16); /* deltas of one level */
    uint8_t *ops = (uint8_t *)malloc(pow8(N) + 16); /* (op, stop) nibbles of one level */
    if (!dl || !ops) rc = ORC_ENOMEM;
    for (int l = N; l >= 1 && !rc; l--) {
        uint32_t nd = 0, no = 0;
        for (uint64_t m = 0; m < pow8(N - l) && !rc; m++) {
            if (p.cst[l][m]) continue; /* constant subtree: no operations below */
            for (int k = 0; k < 8 && !rc; k++) {
                uint32_t j = (uint32_t)(8 * m + k);
                uint32_t L = p.lab[l - 1][j];
                int stop = (l - 1 >= 1) ? p.cst[l - 1][j] : 0;
                int delta = 0;
                int op = best_operation(&p, l, j, &s->pal, &delta);
                if (op == OP_PA) rc = vpush(&s->pal, L);
                if (op == OP_PD) dl[nd++] = (uint8_t)delta;
                s->op_hist[op]++;
                ops[no++] = (uint8_t)(op | (stop << 3));
            }
        }
        for (uint32_t i = 0; i < nd && !rc; i++) rc = spush(s, dl[i]); /* R8 */
        for (uint32_t i = 0; i < no && !rc; i++) rc = spush(s, ops[i]);
        s->cum[l - 1] = s->n;
    }
    free(dl);
    free(ops);
    pyr_free(&p);
    if (rc) bs_free(s);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Frequency tables (Sec. 3.3, R10)                                    */
/* ------------------------------------------------------------------ */
static void normalize_table(const uint64_t cnt[16], uint32_t M, uint32_t f[16]) {
    uint64_t tot = 0;
    for (int s = 0; s < 16; s++) tot += cnt[s] + 1;
    uint64_t sum = 0;
    for (int s = 0; s < 16; s++) {
        uint64_t v = (cnt[s] + 1) * (uint64_t)M / tot;
        f[s] = v < 1 ? 1 : (uint32_t)v;
        sum += f[s];
    }
    while (sum != M) {
        int best = -1;
        for (int s = 0; s < 16; s++) {
            if (sum > M && f[s] <= 1) continue;
            if (best < 0 || f[s] > f[best]) best = s;
        }
        if (sum < M) { f[best] += (uint32_t)(M - sum); sum = M; }
        else { f[best] -= 1; sum -= 1; }
    }
}

/* ------------------------------------------------------------------ */
/* rANS (Sec. 3.3, R9)                                                 */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t f[2][16], c[2][16]; uint32_t bits; } rans_tables;

static void make_rans_tables(rans_tables *t, const uint32_t f[2][16], uint32_t bits) {
    t->bits = bits;
    for (int k = 0; k < 2; k++) {
        uint32_t c = 0;
        for (int s = 0; s < 16; s++) { t->f[k][s] = f[k][s]; t->c[k][s] = c; c += f[k][s]; }
    }
}

/* which table symbol i uses: the leaf table from the L_0 segment on */
static int table_of(uint32_t i, const uint32_t *cum, int N) {
    uint32_t leaf_start = (N >= 2) ? cum[1] : 0;
    return i >= leaf_start ? 1 : 0;
}

/* encode n symbols into W states and a word stream (words in read order) */
static int rans_encode(const uint8_t *sym, uint32_t n, const uint32_t *cum, int N, uint32_t W,
                       const rans_tables *t, uint32_t *states, uint16_t **words, uint32_t *n_words) {
    uint32_t cap = n + 16, nw = 0;
    uint16_t *tmp = (uint16_t *)malloc(sizeof(uint16_t) * cap);
    if (!tmp) return ORC_ENOMEM;
    for (uint32_t j = 0; j < W; j++) states[j] = RANS_L;
    for (int64_t i = (int64_t)n - 1; i >= 0; i--) {
        uint32_t j = (uint32_t)i % W;
        int tb = table_of((uint32_t)i, cum, N);
        uint32_t s = sym[i], f = t->f[tb][s], c = t->c[tb][s];
        uint32_t x = states[j];
        uint64_t x_max = (uint64_t)((RANS_L >> t->bits) << 16) * f;
        if (x >= x_max) { tmp[nw++] = (uint16_t)(x & 0xFFFF); x >>= 16; }
        x = ((x / f) << t->bits) + (x % f) + c;
        states[j] = x;
    }
    for (uint32_t a = 0, b = nw; a < b / 2; a++) { uint16_t q = tmp[a]; tmp[a] = tmp[b - 1 - a]; tmp[b - 1 - a] = q; }
    *words = tmp;
    *n_words = nw;
    return ORC_OK;
}

/* decode the first n symbols; returns the word cursor and final states */
static int rans_decode(uint32_t *states, uint32_t W, const uint16_t *words, uint32_t n_words, const uint32_t *cum,
                       int N, const rans_tables *t, uint32_t n, uint8_t *sym, uint32_t *cursor) {
    uint32_t M = 1u << t->bits, pos = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t j = i % W;
        int tb = table_of(i, cum, N);
        uint32_t x = states[j];
        uint32_t slot = x & (M - 1);
        uint32_t s = 0;
        while (s < 15 && t->c[tb][s + 1] <= slot) s++;
        x = t->f[tb][s] * (x >> t->bits) + slot - t->c[tb][s];
        if (x < RANS_L) {
            if (pos >= n_words) return ORC_ECORRUPT;
            x = (x << 16) | words[pos++];
        }
        states[j] = x;
        sym[i] = (uint8_t)s;
    }
    *cursor = pos;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Brick decoder (Alg. 1), in place over a Morton-ordered LOD-t array  */
/* ------------------------------------------------------------------ */
/*
 * sym: the first cum[t] symbols of the brick (all of them for t = 0).
 * out_dense: (b >> t)^3 labels, x fastest.
 */
static int replay_brick(const uint8_t *sym, const uint32_t *cum, int N, const uint32_t *pal, uint32_t P, uint32_t t,
                        uint32_t *out_dense) {
    if (t > (uint32_t)N) return ORC_ERANGE;
    uint64_t n_out = pow8(N - (int)t);
    uint32_t total = cum[0];
    if (total == 0) { /* R4: uniform brick */
        if (P != 1) return ORC_ECORRUPT;
        for (uint64_t i = 0; i < n_out; i++) out_dense[i] = pal[0];
        return ORC_OK;
    }
    if (P < 2) return ORC_ECORRUPT;
    uint32_t *out = (uint32_t *)malloc(sizeof(uint32_t) * n_out);
    uint8_t *set = (uint8_t *)calloc(n_out, 1); /* "not empty" flag for the paper's empty marker */
    if (!out || !set) { free(out); free(set); return ORC_ENOMEM; }
    int rc = ORC_OK;
    uint32_t ip = 0;
    out[0] = pal[ip]; set[0] = 1;
    for (int l = N; l >= (int)t + 1 && !rc; l--) {
        int m_lvl = l - 1;                     /* child level */
        uint64_t sp = pow8(l - (int)t);        /* spacing of level-l nodes */
        uint64_t csp = pow8(l - 1 - (int)t);   /* spacing of level-(l-1) nodes */
        uint32_t seg0 = (m_lvl + 1 <= N - 1) ? cum[m_lvl + 1] : 0, seg1 = cum[m_lvl];
        /* expanded parents of this level: their last child is still empty */
        uint64_t E = 0;
        for (uint64_t m = 0; m < pow8(N - l); m++) if (!set[m * sp + 7 * csp]) E++;
        if ((uint64_t)seg0 + 8 * E > seg1) { rc = ORC_ECORRUPT; break; }
        uint32_t nd = seg1 - seg0 - (uint32_t)(8 * E);  /* deltas precede the operations (R8) */
        uint32_t dc = seg0, opc = seg0 + nd;
        for (uint64_t m = 0; m < pow8(N - l) && !rc; m++) {
            uint64_t i = m * sp;
            if (set[i + 7 * csp]) continue; /* constant area */
            uint32_t parent = out[i];
            for (int k = 0; k < 8 && !rc; k++) {
                uint64_t j = 8 * m + k; /* child Morton index at level l-1 */
                uint8_t nib = sym[opc++];
                uint32_t op = nib & 7u, stop = nib >> 3;
                uint32_t v = 0;
                if (op == OP_RP) {
                    v = parent;
                } else if (op >= OP_RX && op <= OP_RZ) {
                    int a = (int)op - OP_RX;
                    uint32_t c[3], G = 1u << (N - m_lvl);
                    unmorton((uint32_t)j, N - m_lvl, c);
                    if ((c[a] & 1u) == 0) {
                        if (c[a] == 0) { rc = ORC_ECORRUPT; break; }
                        c[a] -= 1;
                        v = out[(uint64_t)morton(c[0], c[1], c[2], N - m_lvl) * csp];
                    } else {
                        if (c[a] + 1 >= G) { rc = ORC_ECORRUPT; break; }
                        c[a] += 1;
                        v = out[(uint64_t)morton(c[0] >> 1, c[1] >> 1, c[2] >> 1, N - l) * sp];
                    }
                } else if (op == OP_PA) {
                    if (ip + 1 >= P) { rc = ORC_ECORRUPT; break; }
                    v = pal[++ip];
                } else if (op == OP_P0) {
                    v = pal[ip];
                } else if (op == OP_PD) {
                    if (dc >= seg0 + nd) { rc = ORC_ECORRUPT; break; }
                    uint32_t d = sym[dc++];
                    if (ip < d + 1) { rc = ORC_ECORRUPT; break; }
                    v = pal[ip - d - 1];
                } else {
                    rc = ORC_ECORRUPT; break;
                }
                if (stop && m_lvl == 0) { rc = ORC_ECORRUPT; break; }
                uint64_t jo = j * csp;
                out[jo] = v; set[jo] = 1;
                if (stop) /* fill the child's whole sub-block */
                    for (uint64_t q = 0; q < csp; q++) { out[jo + q] = v; set[jo + q] = 1; }
            }
        }
        if (!rc && (opc != seg1 || dc != seg0 + nd)) rc = ORC_ECORRUPT;
    }
    if (!rc) {
        uint32_t G = 1u << (N - t);
        for (uint64_t m = 0; m < n_out; m++) {
            uint32_t c[3];
            unmorton((uint32_t)m, N - (int)t, c);
            out_dense[c[0] + (uint64_t)G * (c[1] + (uint64_t)G * c[2])] = out[m];
        }
    }
    free(out); free(set);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Volume container (byte layout is ours)                              */
/* ------------------------------------------------------------------ */
#define CSV_MAGIC 0x31565343u /* "CSV1" */
#define HDR_BYTES 128u

typedef struct {
    uint32_t magic, version, nx, ny, nz, brick_log2, nbx, nby, nbz, n_bricks, scale_bits, lane_k, lane_max,
        sample_stride, reserved0, reserved1;
    uint16_t freq[2][16];
} vol_header;

static uint32_t lane_count(uint32_t n, uint32_t K, uint32_t Wmax) {
    if (n == 0) return 0;
    uint32_t W = 1;
    while (2 * W <= Wmax && (uint64_t)2 * W * K <= n) W *= 2;
    return W;
}

static void extract_brick(const uint32_t *vol, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t bx, uint32_t by,
                          uint32_t bz, int N, uint32_t *brick) {
    uint32_t b = 1u << N;
    for (uint32_t z = 0; z < b; z++)
        for (uint32_t y = 0; y < b; y++)
            for (uint32_t x = 0; x < b; x++) {
                uint64_t gx = (uint64_t)bx * b + x, gy = (uint64_t)by * b + y, gz = (uint64_t)bz * b + z;
                uint32_t v = 0; /* padding label */
                if (gx < nx && gy < ny && gz < nz) v = vol[gx + nx * (gy + (uint64_t)ny * gz)];
                brick[x + b * (y + b * z)] = v;
            }
}

typedef struct { uint8_t *bytes; uint32_t size; } rec_buf;

/* a record whose symbols are stored as raw nibbles (R11) */
static int build_record_raw(const brick_stream *s, int N, rec_buf *r) {
    uint32_t nw = (s->n + 3) / 4;
    uint32_t hdr = 3 + (uint32_t)N;
    uint32_t size = 4 * (hdr + s->pal.np) + 2 * nw;
    size = (size + 3) & ~3u;
    uint8_t *b = (uint8_t *)calloc(size, 1);
    if (!b) return ORC_ENOMEM;
    uint32_t *w = (uint32_t *)b;
    w[0] = s->pal.np;
    w[1] = 0;
    w[2] = nw;
    for (int m = 0; m < N; m++) w[3 + m] = s->cum[m];
    memcpy(w + hdr, s->pal.pal, 4 * s->pal.np);
    uint16_t *words = (uint16_t *)(b + 4 * (hdr + s->pal.np));
    for (uint32_t i = 0; i < s->n; i++) words[i / 4] |= (uint16_t)(s->sym[i] << (4 * (i % 4)));
    r->bytes = b;
    r->size = size;
    return ORC_OK;
}

static int build_record(const brick_stream *s, int N, const rans_tables *t, uint32_t K, uint32_t Wmax, rec_buf *r) {
    uint32_t W = lane_count(s->n, K, Wmax);
    uint32_t states[64];
    uint16_t *words = NULL;
    uint32_t nw = 0;
    int rc = ORC_OK;
    if (s->n) {
        rc = rans_encode(s->sym, s->n, s->cum, N, W, t, states, &words, &nw);
        if (rc) return rc;
    }
    uint32_t hdr = 3 + (uint32_t)N;
    uint32_t size = 4 * (hdr + s->pal.np + W) + 2 * nw;
    size = (size + 3) & ~3u;
    uint8_t *b = (uint8_t *)calloc(size, 1);
    if (!b) { free(words); return ORC_ENOMEM; }
    uint32_t *w = (uint32_t *)b;
    w[0] = s->pal.np;
    w[1] = W;
    w[2] = nw;
    for (int m = 0; m < N; m++) w[3 + m] = s->cum[m];
    memcpy(w + hdr, s->pal.pal, 4 * s->pal.np);
    memcpy(w + hdr + s->pal.np, states, 4 * W);
    if (nw) memcpy(b + 4 * (hdr + s->pal.np + W), words, 2 * nw); /* a uniform brick has no words */
    free(words);
    r->bytes = b;
    r->size = size;
    return ORC_OK;
}

void orc_free(void *p) { free(p); }

/* host threads the parallel loops use */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the number of host threads of later parallel loops (n >= 1) */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
uint32_t orc_abi_version(void) { return 1; }

/*
 * Encode a whole volume.  vol: nx*ny*nz labels, x fastest.  Bricks are
 * numbered x fastest; the volume is padded with label 0 to whole bricks.
 * sample_stride 0 means: every 512th brick, every 4096th above 2^20
 * bricks (Sec. 3.4).  tables 2: one frequency table for the symbols of
 * levels >= 1 and one for L_0 (the paper's default); 1: a single table
 * from the counts of all symbols, stored twice (Table 1's variant); 0: no
 * entropy coding, the symbols stored as raw nibbles (R11; Table 1's
 * variant without rANS).
 */
int orc_encode_volume(const uint32_t *vol, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t brick_log2,
                      uint32_t scale_bits, uint32_t lane_k, uint32_t lane_max, uint32_t sample_stride,
                      uint32_t tables, uint8_t **blob_out, uint64_t *blob_bytes, uint64_t *op_hist_out) {
    if (!vol || !blob_out || !blob_bytes) return ORC_EINVAL;
    if (brick_log2 < 1 || brick_log2 > MAX_LOG2 || scale_bits < 8 || scale_bits > 12 || lane_k < 1 ||
        lane_max < 1 || lane_max > 64 || (lane_max & (lane_max - 1)) || nx == 0 || ny == 0 || nz == 0 ||
        tables > 2)
        return ORC_EINVAL;
    const int raw = tables == 0;
    int N = (int)brick_log2;
    uint32_t b = 1u << N;
    uint32_t nbx = (nx + b - 1) / b, nby = (ny + b - 1) / b, nbz = (nz + b - 1) / b;
    uint64_t B = (uint64_t)nbx * nby * nbz;
    if (B >= (1ull << 32)) return ORC_ERANGE;
    if (sample_stride == 0) sample_stride = (B > (1ull << 20)) ? 4096 : 512;
    /* prepass over every sample_stride-th brick: nibble counts per table */
    uint64_t cnt[2][16];
    memset(cnt, 0, sizeof(cnt));
    int rc = ORC_OK;
    #pragma omp parallel
    {
        uint32_t *brick = (uint32_t *)malloc(sizeof(uint32_t) * b * b * b);
        uint64_t lc[2][16];
        memset(lc, 0, sizeof(lc));
        #pragma omp for schedule(dynamic, 1)
        for (int64_t id = 0; id < (int64_t)B; id += sample_stride) {
            brick_stream s;
            extract_brick(vol, nx, ny, nz, (uint32_t)(id % nbx), (uint32_t)((id / nbx) % nby),
                          (uint32_t)(id / ((uint64_t)nbx * nby)), N, brick);
            if (encode_brick_stream(brick, N, &s)) {
                #pragma omp critical
                rc = ORC_ENOMEM;
                continue;
            }
            for (uint32_t i = 0; i < s.n; i++) lc[table_of(i, s.cum, N)][s.sym[i]]++;
            bs_free(&s);
        }
        #pragma omp critical
        for (int k = 0; k < 2; k++) for (int q = 0; q < 16; q++) cnt[k][q] += lc[k][q];
        free(brick);
    }
    if (rc) return rc;
    uint32_t f[2][16];
    if (tables == 1)
        for (int q = 0; q < 16; q++) cnt[0][q] = cnt[1][q] = cnt[0][q] + cnt[1][q];
    if (raw) /* uniform, unused */
        for (int q = 0; q < 16; q++) cnt[0][q] = cnt[1][q] = 0;
    normalize_table(cnt[0], 1u << scale_bits, f[0]);
    normalize_table(cnt[1], 1u << scale_bits, f[1]);
    rans_tables t;
    make_rans_tables(&t, f, scale_bits);
    rec_buf *recs = (rec_buf *)calloc(B, sizeof(rec_buf));
    uint64_t hist[8] = {0};
    if (!recs) return ORC_ENOMEM;
    #pragma omp parallel
    {
        uint32_t *brick = (uint32_t *)malloc(sizeof(uint32_t) * b * b * b);
        uint64_t lh[8] = {0};
        #pragma omp for schedule(dynamic, 4)
        for (int64_t id = 0; id < (int64_t)B; id++) {
            brick_stream s;
            extract_brick(vol, nx, ny, nz, (uint32_t)(id % nbx), (uint32_t)((id / nbx) % nby),
                          (uint32_t)(id / ((uint64_t)nbx * nby)), N, brick);
            int r = encode_brick_stream(brick, N, &s);
            if (!r) r = raw ? build_record_raw(&s, N, &recs[id]) : build_record(&s, N, &t, lane_k, lane_max, &recs[id]);
            for (int q = 0; q < 8; q++) lh[q] += s.op_hist[q];
            bs_free(&s);
            if (r) {
                #pragma omp critical
                rc = r;
            }
        }
        #pragma omp critical
        for (int q = 0; q < 8; q++) hist[q] += lh[q];
        free(brick);
    }
    if (op_hist_out) memcpy(op_hist_out, hist, sizeof(hist));
    uint64_t idx_bytes = 8 * (B + 1);
    uint64_t rec_start = (HDR_BYTES + idx_bytes + 15) & ~15ull;
    uint64_t total = rec_start;
    for (uint64_t i = 0; i < B && !rc; i++) total += recs[i].size;
    uint8_t *blob = rc ? NULL : (uint8_t *)calloc(total, 1);
    if (!rc && !blob) rc = ORC_ENOMEM;
    if (!rc) {
        vol_header h;
        memset(&h, 0, sizeof(h));
        h.magic = CSV_MAGIC; h.version = 1; h.nx = nx; h.ny = ny; h.nz = nz; h.brick_log2 = brick_log2;
        h.nbx = nbx; h.nby = nby; h.nbz = nbz; h.n_bricks = (uint32_t)B; h.scale_bits = scale_bits;
        h.lane_k = lane_k; h.lane_max = lane_max; h.sample_stride = sample_stride;
        h.reserved0 = raw ? 1u : 0u; /* coding (R11) */
        for (int k = 0; k < 2; k++) for (int q = 0; q < 16; q++) h.freq[k][q] = (uint16_t)f[k][q];
        memcpy(blob, &h, sizeof(h));
        uint64_t *index = (uint64_t *)(blob + HDR_BYTES);
        uint64_t off = 0;
        for (uint64_t i = 0; i < B; i++) {
            index[i] = off;
            memcpy(blob + rec_start + off, recs[i].bytes, recs[i].size);
            off += recs[i].size;
        }
        index[B] = off;
        *blob_out = blob;
        *blob_bytes = total;
    }
    for (uint64_t i = 0; i < B; i++) free(recs[i].bytes);
    free(recs);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Container parsing and brick decode                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    vol_header h;
    const uint64_t *index;
    const uint8_t *recs;
    uint64_t rec_bytes;
    rans_tables t;
} vol_view;

static int open_volume(const uint8_t *blob, uint64_t bytes, vol_view *v) {
    if (!blob || bytes < HDR_BYTES) return ORC_EINVAL;
    memcpy(&v->h, blob, sizeof(vol_header));
    if (v->h.magic != CSV_MAGIC || v->h.version != 1) return ORC_ECORRUPT;
    if (v->h.brick_log2 < 1 || v->h.brick_log2 > MAX_LOG2 || v->h.scale_bits < 8 || v->h.scale_bits > 12 ||
        v->h.reserved0 > 1)
        return ORC_ECORRUPT;
    uint64_t B = v->h.n_bricks;
    uint64_t rec_start = (HDR_BYTES + 8 * (B + 1) + 15) & ~15ull;
    if (bytes < rec_start) return ORC_ECORRUPT;
    v->index = (const uint64_t *)(blob + HDR_BYTES);
    v->recs = blob + rec_start;
    v->rec_bytes = bytes - rec_start;
    if (v->index[B] > v->rec_bytes) return ORC_ECORRUPT;
    uint32_t f[2][16];
    for (int k = 0; k < 2; k++) {
        uint32_t sum = 0;
        for (int q = 0; q < 16; q++) { f[k][q] = v->h.freq[k][q]; sum += f[k][q]; if (!f[k][q]) return ORC_ECORRUPT; }
        if (sum != (1u << v->h.scale_bits)) return ORC_ECORRUPT;
    }
    make_rans_tables(&v->t, f, v->h.scale_bits);
    return ORC_OK;
}

int orc_volume_info(const uint8_t *blob, uint64_t bytes, uint32_t *info16) {
    vol_view v;
    int rc = open_volume(blob, bytes, &v);
    if (rc) return rc;
    memcpy(info16, &v.h, 16 * sizeof(uint32_t));
    return ORC_OK;
}

static int decode_one(const vol_view *v, uint32_t id, uint32_t t, uint32_t *out, int check_end) {
    int N = (int)v->h.brick_log2;
    if (id >= v->h.n_bricks) return ORC_ERANGE;
    if (t > (uint32_t)N) return ORC_ERANGE;
    uint64_t o0 = v->index[id], o1 = v->index[id + 1];
    if (o1 < o0 || o1 > v->rec_bytes) return ORC_ECORRUPT;
    const uint8_t *rb = v->recs + o0;
    uint64_t size = o1 - o0;
    uint32_t hdr = 3 + (uint32_t)N;
    if (size < 4 * hdr) return ORC_ECORRUPT;
    const uint32_t *w = (const uint32_t *)rb;
    uint32_t P = w[0], W = w[1], nw = w[2];
    uint32_t cum[MAX_LOG2];
    for (int m = 0; m < N; m++) cum[m] = w[3 + m];
    for (int m = 0; m + 1 < N; m++) if (cum[m] < cum[m + 1]) return ORC_ECORRUPT;
    const int raw = v->h.reserved0 == 1; /* R11 */
    if (raw ? (W != 0 || nw != (cum[0] + 3) / 4)
            : (P == 0 || W > 64 || (W & (W - 1)) || (cum[0] > 0) != (W > 0)))
        return ORC_ECORRUPT;
    if (P == 0 || (uint64_t)4 * (hdr + P + W) + 2ull * nw > size) return ORC_ECORRUPT;
    const uint32_t *pal = w + hdr;
    uint32_t states[64];
    for (uint32_t j = 0; j < W; j++) states[j] = w[hdr + P + j];
    const uint16_t *words = (const uint16_t *)(rb + 4 * (hdr + P + W));
    uint32_t n = (t < (uint32_t)N) ? cum[t] : 0;
    uint8_t *sym = (uint8_t *)malloc(n + 1);
    if (!sym) return ORC_ENOMEM;
    uint32_t cursor = 0;
    int rc = ORC_OK;
    if (raw) {
        for (uint32_t i = 0; i < n; i++) sym[i] = (uint8_t)((words[i / 4] >> (4 * (i % 4))) & 15u);
        /* a complete decode finds the last word's unused nibbles zero */
        if (check_end && t == 0 && cum[0] % 4 && (words[nw - 1] >> (4 * (cum[0] % 4))) != 0) rc = ORC_ECORRUPT;
    } else if (n) {
        rc = rans_decode(states, W, words, nw, cum, N, &v->t, n, sym, &cursor);
    }
    if (!rc && !raw && check_end && t == 0 && cum[0]) {
        /* a complete decode ends in the encoder's initial states with every word read */
        for (uint32_t j = 0; j < W; j++) if (states[j] != RANS_L) rc = ORC_ECORRUPT;
        if (cursor != nw) rc = ORC_ECORRUPT;
    }
    if (!rc) {
        if (t == (uint32_t)N) out[0] = pal[0];
        else rc = replay_brick(sym, cum, N, pal, P, t, out); /* reads only segments of levels >= t */
    }
    free(sym);
    return rc;
}

int orc_decode_brick(const uint8_t *blob, uint64_t bytes, uint32_t id, uint32_t lod, uint32_t *out) {
    vol_view v;
    int rc = open_volume(blob, bytes, &v);
    if (rc) return rc;
    return decode_one(&v, id, lod, out, 1);
}

/* decode n requests, outputs packed back to back in request order */
int orc_decode_bricks(const uint8_t *blob, uint64_t bytes, const uint32_t *ids, const uint8_t *lods, uint32_t n,
                      uint32_t *out) {
    vol_view v;
    int rc = open_volume(blob, bytes, &v);
    if (rc) return rc;
    int N = (int)v.h.brick_log2;
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    if (!off) return ORC_ENOMEM;
    off[0] = 0;
    for (uint32_t i = 0; i < n; i++) {
        if (lods[i] > N) { free(off); return ORC_ERANGE; }
        off[i + 1] = off[i] + pow8(N - lods[i]);
    }
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        int r = decode_one(&v, ids[i], lods[i], out + off[i], 1);
        if (r) {
            #pragma omp critical
            rc = r;
        }
    }
    free(off);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Entry points exposing the individual steps (for the pins)           */
/* ------------------------------------------------------------------ */

/* levels packed level-major from L_0 to L_N, each in Morton order */
int orc_pyramid(const uint32_t *brick, uint32_t brick_log2, uint32_t *labels, uint8_t *consts) {
    if (brick_log2 < 1 || brick_log2 > MAX_LOG2) return ORC_EINVAL;
    pyramid p;
    int N = (int)brick_log2;
    int rc = pyr_build(&p, brick, N);
    if (rc) return rc;
    uint64_t o = 0;
    for (int l = 0; l <= N; l++) {
        memcpy(labels + o, p.lab[l], 4 * pow8(N - l));
        memcpy(consts + o, p.cst[l], pow8(N - l));
        o += pow8(N - l);
    }
    pyr_free(&p);
    return ORC_OK;
}

/* the symbol stream of one brick (before entropy coding) */
int orc_brick_symbols(const uint32_t *brick, uint32_t brick_log2, uint8_t *sym, uint32_t sym_cap, uint32_t *n_sym,
                      uint32_t *cum, uint32_t *palette, uint32_t pal_cap, uint32_t *n_pal) {
    if (brick_log2 < 1 || brick_log2 > MAX_LOG2) return ORC_EINVAL;
    brick_stream s;
    int rc = encode_brick_stream(brick, (int)brick_log2, &s);
    if (rc) return rc;
    *n_sym = s.n;
    *n_pal = s.pal.np;
    for (uint32_t m = 0; m < brick_log2; m++) cum[m] = s.cum[m];
    if (s.n > sym_cap || s.pal.np > pal_cap) { bs_free(&s); return ORC_ERANGE; }
    memcpy(sym, s.sym, s.n);
    memcpy(palette, s.pal.pal, 4 * s.pal.np);
    bs_free(&s);
    return ORC_OK;
}

/* Alg. 1 on a given symbol stream (no entropy coding) */
int orc_replay(const uint8_t *sym, const uint32_t *cum, uint32_t brick_log2, const uint32_t *palette, uint32_t P,
               uint32_t lod, uint32_t *out) {
    if (brick_log2 < 1 || brick_log2 > MAX_LOG2 || lod > brick_log2) return ORC_EINVAL;
    int N = (int)brick_log2;
    if (lod == brick_log2) { out[0] = palette[0]; return ORC_OK; }
    return replay_brick(sym, cum, N, palette, P, lod, out);
}

int orc_normalize_table(const uint64_t *counts16, uint32_t scale_bits, uint32_t *freq16) {
    if (scale_bits < 8 || scale_bits > 12) return ORC_EINVAL;
    normalize_table(counts16, 1u << scale_bits, freq16);
    return ORC_OK;
}

/*
 * rANS on an explicit symbol stream.  tab_split: index of the first symbol
 * coded with the second table.  words: capacity n + 16.
 */
int orc_rans_encode(const uint8_t *sym, uint32_t n, uint32_t tab_split, uint32_t W, const uint32_t *freq32,
                    uint32_t scale_bits, uint32_t *states, uint16_t *words, uint32_t *n_words) {
    if (W < 1 || W > 64 || scale_bits < 8 || scale_bits > 12) return ORC_EINVAL;
    uint32_t f[2][16];
    memcpy(f, freq32, sizeof(f));
    rans_tables t;
    make_rans_tables(&t, f, scale_bits);
    uint32_t cum[MAX_LOG2] = {n, tab_split, 0, 0, 0, 0};
    uint16_t *w = NULL;
    int rc = rans_encode(sym, n, cum, 2, W, &t, states, &w, n_words);
    if (rc) return rc;
    memcpy(words, w, 2 * *n_words);
    free(w);
    return ORC_OK;
}

int orc_rans_decode(uint32_t *states, uint32_t W, const uint16_t *words, uint32_t n_words, uint32_t tab_split,
                    const uint32_t *freq32, uint32_t scale_bits, uint32_t n, uint8_t *sym, uint32_t *cursor) {
    if (W < 1 || W > 64 || scale_bits < 8 || scale_bits > 12) return ORC_EINVAL;
    uint32_t f[2][16];
    memcpy(f, freq32, sizeof(f));
    rans_tables t;
    make_rans_tables(&t, f, scale_bits);
    uint32_t cum[MAX_LOG2] = {n, tab_split, 0, 0, 0, 0};
    return rans_decode(states, W, words, n_words, cum, 2, &t, n, sym, cursor);
}
