/*
 * Seeded synthetic label volumes.
 *
 * These generators produce the test and benchmark inputs: uint32 label
 * volumes in C order [z][y][x] (x fastest).  They stand in for the paper's
 * Cells, Fiber and Cortex data sets (Section 5), which are not available;
 * each one reproduces the structure of one of them: dense cell partitions
 * with noisy boundaries, smooth homogeneous blobs, and branching neurite
 * tubes with heavy-tailed sizes in a mostly empty volume.
 *
 * This module holds no part of the compression method.  It only draws
 * random numbers and paints labels.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used both as a sequential
 * stream and as a counter-based hash (mix of seed and a counter).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- SplitMix64 ------------------------------------------------------- */
static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline uint64_t sm64_next(uint64_t *s) {
    *s += 0x9E3779B97F4A7C15ull;
    return sm64_mix(*s);
}
/* counter-based: value number `ctr` of the stream keyed by `key` */
static inline uint64_t sm64_at(uint64_t key, uint64_t ctr) {
    return sm64_mix(key + (ctr + 1) * 0x9E3779B97F4A7C15ull);
}
static inline double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }
static inline double rnd(uint64_t *s) { return u01(sm64_next(s)); }
static double rnd_normal(uint64_t *s) {
    /* Box-Muller, one value per call */
    double u1 = rnd(s), u2 = rnd(s);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
static uint32_t rnd_below(uint64_t *s, uint32_t n) { return (uint32_t)(rnd(s) * n) % n; }

/* Fisher-Yates permutation of 1..n into perm[0..n-1] */
static void permute_labels(uint32_t *perm, uint32_t n, uint64_t *s) {
    for (uint32_t i = 0; i < n; i++) perm[i] = i + 1;
    for (uint32_t i = n; i > 1; i--) {
        uint32_t j = rnd_below(s, i);
        uint32_t t = perm[i - 1]; perm[i - 1] = perm[j]; perm[j] = t;
    }
}

uint32_t synth_abi_version(void) { return 1; }

/*
 * Small Voronoi volume with background.
 * n_sites sites uniform in [0,n)^3; every voxel centre (x+.5,y+.5,z+.5)
 * takes the nearest site (squared distance, ties to the lower site index);
 * site i has label i+1.  Then sites are set to background 0 in a seeded
 * random order until at least bg_frac of all voxels are 0.
 */
int synth_voronoi_bg(uint32_t *out, uint32_t n, uint32_t n_sites, double bg_frac, uint64_t seed) {
    if (!out || n == 0 || n_sites == 0) return -1;
    uint64_t s = seed;
    double *site = (double *)malloc(sizeof(double) * 3 * n_sites);
    uint64_t *count = (uint64_t *)calloc(n_sites, sizeof(uint64_t));
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * n_sites);
    if (!site || !count || !order) { free(site); free(count); free(order); return -4; }
    for (uint32_t i = 0; i < 3 * n_sites; i++) site[i] = rnd(&s) * n;
    uint64_t nv = (uint64_t)n * n * n;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)nv; v++) {
        double px = (double)(v % n) + 0.5, py = (double)((v / n) % n) + 0.5, pz = (double)(v / ((uint64_t)n * n)) + 0.5;
        double best = 1e300; uint32_t bi = 0;
        for (uint32_t i = 0; i < n_sites; i++) {
            double dx = px - site[3 * i], dy = py - site[3 * i + 1], dz = pz - site[3 * i + 2];
            double d = dx * dx + dy * dy + dz * dz;
            if (d < best) { best = d; bi = i; }
        }
        out[v] = bi + 1;
    }
    for (uint64_t v = 0; v < nv; v++) count[out[v] - 1]++;
    permute_labels(order, n_sites, &s); /* order[k]-1 = k-th site to clear */
    uint8_t *clear = (uint8_t *)calloc(n_sites, 1);
    uint64_t zeros = 0;
    for (uint32_t k = 0; k < n_sites && (double)zeros < bg_frac * (double)nv; k++) {
        clear[order[k] - 1] = 1;
        zeros += count[order[k] - 1];
    }
    for (uint64_t v = 0; v < nv; v++) if (clear[out[v] - 1]) out[v] = 0;
    free(clear); free(site); free(count); free(order);
    return 0;
}

/*
 * Dense "cells" partition: a jittered grid of grid^3 sites (one uniform
 * site per cell), nearest site found in the 27 surrounding cells, labels a
 * seeded permutation of 1..grid^3.  Then boundary noise: every voxel that
 * has an in-volume 6-neighbour with a different label takes, with
 * probability p_noise, the label of one uniformly chosen in-volume
 * 6-neighbour, read from the volume before noise.  `tmp` must hold n^3
 * values (scratch).
 */
int synth_cells(uint32_t *out, uint32_t *tmp, uint32_t n, uint32_t grid, double p_noise, uint64_t seed) {
    if (!out || !tmp || n == 0 || grid == 0) return -1;
    uint64_t s = seed;
    uint64_t ns = (uint64_t)grid * grid * grid;
    double *site = (double *)malloc(sizeof(double) * 3 * ns);
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * ns);
    if (!site || !lab) { free(site); free(lab); return -4; }
    double cs = (double)n / grid;
    for (uint64_t c = 0; c < ns; c++) {
        uint64_t cx = c % grid, cy = (c / grid) % grid, cz = c / ((uint64_t)grid * grid);
        site[3 * c] = (cx + rnd(&s)) * cs;
        site[3 * c + 1] = (cy + rnd(&s)) * cs;
        site[3 * c + 2] = (cz + rnd(&s)) * cs;
    }
    permute_labels(lab, (uint32_t)ns, &s);
    uint64_t nv = (uint64_t)n * n * n;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)nv; v++) {
        uint32_t x = v % n, y = (v / n) % n, z = v / ((uint64_t)n * n);
        double px = x + 0.5, py = y + 0.5, pz = z + 0.5;
        int gx = (int)(px / cs), gy = (int)(py / cs), gz = (int)(pz / cs);
        double best = 1e300; uint64_t bi = 0;
        for (int dz = -1; dz <= 1; dz++) for (int dy = -1; dy <= 1; dy++) for (int dx = -1; dx <= 1; dx++) {
            int cx = gx + dx, cy = gy + dy, cz = gz + dz;
            if (cx < 0 || cy < 0 || cz < 0 || cx >= (int)grid || cy >= (int)grid || cz >= (int)grid) continue;
            uint64_t c = (uint64_t)cx + grid * ((uint64_t)cy + (uint64_t)grid * cz);
            double ex = px - site[3 * c], ey = py - site[3 * c + 1], ez = pz - site[3 * c + 2];
            double d = ex * ex + ey * ey + ez * ez;
            if (d < best || (d == best && c < bi)) { best = d; bi = c; }
        }
        tmp[v] = lab[bi];
    }
    uint64_t key = sm64_next(&s);
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)nv; v++) {
        uint32_t x = v % n, y = (v / n) % n, z = v / ((uint64_t)n * n);
        int64_t nb[6]; int k = 0;
        if (x > 0) nb[k++] = v - 1;
        if (x + 1 < n) nb[k++] = v + 1;
        if (y > 0) nb[k++] = v - n;
        if (y + 1 < n) nb[k++] = v + n;
        if (z > 0) nb[k++] = v - (int64_t)n * n;
        if (z + 1 < n) nb[k++] = v + (int64_t)n * n;
        uint32_t me = tmp[v];
        int differs = 0;
        for (int i = 0; i < k; i++) differs |= (tmp[nb[i]] != me);
        uint32_t r = me;
        if (differs) {
            uint64_t h = sm64_at(key, (uint64_t)v);
            if (u01(h) < p_noise) {
                uint64_t h2 = sm64_at(key ^ 0x5bd1e995ull, (uint64_t)v);
                r = tmp[nb[(uint32_t)(u01(h2) * k) % k]];
            }
        }
        out[v] = r;
    }
    free(site); free(lab);
    return 0;
}

/*
 * Smooth blobs: n_sites sites uniform in the volume; a voxel at p takes
 * the nearest site to the warped point p + D(p), where D is the sum of 4
 * low-frequency sinusoid displacement fields, each along a random unit
 * direction with a random integer wave vector of 1..2 periods per volume
 * edge, and amplitude amp/2 (so |D| <= 2*amp).  Labels are a seeded
 * permutation of 1..n_sites.
 */
int synth_blobs(uint32_t *out, uint32_t n, uint32_t n_sites, double amp, uint64_t seed) {
    if (!out || n == 0 || n_sites == 0) return -1;
    uint64_t s = seed;
    double *site = (double *)malloc(sizeof(double) * 3 * n_sites);
    uint32_t *lab = (uint32_t *)malloc(sizeof(uint32_t) * n_sites);
    if (!site || !lab) { free(site); free(lab); return -4; }
    for (uint32_t i = 0; i < 3 * n_sites; i++) site[i] = rnd(&s) * n;
    permute_labels(lab, n_sites, &s);
    double kv[4][3], dir[4][3], ph[4];
    for (int f = 0; f < 4; f++) {
        double nn = 0;
        for (int a = 0; a < 3; a++) { kv[f][a] = (double)(1 + rnd_below(&s, 2)) * (rnd(&s) < 0.5 ? -1 : 1); }
        for (int a = 0; a < 3; a++) { dir[f][a] = rnd_normal(&s); nn += dir[f][a] * dir[f][a]; }
        nn = sqrt(nn);
        for (int a = 0; a < 3; a++) dir[f][a] /= nn;
        ph[f] = rnd(&s) * 6.283185307179586;
    }
    uint64_t nv = (uint64_t)n * n * n;
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)nv; v++) {
        double p[3] = {(double)(v % n) + 0.5, (double)((v / n) % n) + 0.5, (double)(v / ((uint64_t)n * n)) + 0.5};
        double q[3] = {p[0], p[1], p[2]};
        for (int f = 0; f < 4; f++) {
            double arg = ph[f] + 6.283185307179586 * (kv[f][0] * p[0] + kv[f][1] * p[1] + kv[f][2] * p[2]) / n;
            double w = 0.5 * amp * sin(arg);
            for (int a = 0; a < 3; a++) q[a] += w * dir[f][a];
        }
        double best = 1e300; uint32_t bi = 0;
        for (uint32_t i = 0; i < n_sites; i++) {
            double dx = q[0] - site[3 * i], dy = q[1] - site[3 * i + 1], dz = q[2] - site[3 * i + 2];
            double d = dx * dx + dy * dy + dz * dz;
            if (d < best) { best = d; bi = i; }
        }
        out[v] = lab[bi];
    }
    free(site); free(lab);
    return 0;
}

/*
 * Neurite-like volume: n_labels branching tubes in an empty (0) volume.
 *   - label of size rank r (1-based) gets a voxel budget proportional to
 *     1/r (Zipf, s = 1), scaled so the budgets sum to fill * volume;
 *   - radius uniform in {2..8};
 *   - the tube is a persistent random walk with unit steps: each step the
 *     direction becomes normalize(d + 0.3 * N(0, I)); the walk reflects at
 *     the volume faces; with probability 0.02 per step it branches, i.e. the
 *     walk continues from a uniformly chosen earlier point of the same tube
 *     with a freshly perturbed direction;
 *   - the walk takes ceil(budget / (pi r^2)) steps (one cross-section per
 *     unit of length), each painting the ball of radius r around its point;
 *   - overlaps go to the larger tube (smaller rank), which is the same as
 *     painting largest first into voxels that are still empty;
 *   - finally rank r is replaced by a seeded permutation of 1..n_labels.
 * The tubes are independent, so painting is done per z-slab in parallel
 * with a min over ranks; the result does not depend on the thread count.
 * Returns the number of painted voxels in *painted (may be NULL).
 */
typedef struct { float x, y, z; uint32_t rank_rad; } tube_pt; /* rank << 4 | radius */

static int cmp_pt_z(const void *a, const void *b) {
    float za = ((const tube_pt *)a)->z, zb = ((const tube_pt *)b)->z;
    return (za > zb) - (za < zb);
}

static inline double reflect(double p, double *d, double n) {
    if (p < 0) { p = -p; *d = -*d; }
    if (p >= n) { p = 2 * n - p - 1e-6; *d = -*d; }
    if (p < 0) p = 0;
    return p;
}

int synth_neurite(uint32_t *out, uint32_t nx, uint32_t ny, uint32_t nz, uint32_t n_labels, double fill,
                  uint64_t seed, uint64_t *painted) {
    if (!out || !nx || !ny || !nz || !n_labels) return -1;
    uint64_t s = seed;
    double V = (double)nx * ny * nz, H = 0;
    for (uint32_t r = 1; r <= n_labels; r++) H += 1.0 / r;
    uint64_t *nsteps = (uint64_t *)malloc(sizeof(uint64_t) * (n_labels + 1));
    uint32_t *rad = (uint32_t *)malloc(sizeof(uint32_t) * (n_labels + 1));
    uint64_t *first = (uint64_t *)malloc(sizeof(uint64_t) * (n_labels + 2));
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n_labels);
    if (!nsteps || !rad || !first || !perm) return -4;
    uint64_t total = 0;
    first[1] = 0;
    for (uint32_t r = 1; r <= n_labels; r++) {
        double budget = fill * V / (r * H);
        rad[r] = 2 + rnd_below(&s, 7);
        double st = ceil(budget / (3.141592653589793 * rad[r] * rad[r]));
        nsteps[r] = st < 1 ? 1 : (uint64_t)st;
        total += nsteps[r];
        first[r + 1] = total;
    }
    permute_labels(perm, n_labels, &s);
    uint64_t key = sm64_next(&s);
    tube_pt *pts = (tube_pt *)malloc(sizeof(tube_pt) * total);
    if (!pts) return -4;
    /* walk every tube with its own stream */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ri = 1; ri <= (int64_t)n_labels; ri++) {
        uint32_t r = (uint32_t)ri;
        uint64_t ts = sm64_at(key, r);
        tube_pt *tp = pts + first[r];
        double p[3] = {rnd(&ts) * nx, rnd(&ts) * ny, rnd(&ts) * nz}, d[3];
        double nn = 0;
        for (int a = 0; a < 3; a++) { d[a] = rnd_normal(&ts); nn += d[a] * d[a]; }
        nn = sqrt(nn) + 1e-12;
        for (int a = 0; a < 3; a++) d[a] /= nn;
        for (uint64_t k = 0; k < nsteps[r]; k++) {
            tp[k].x = (float)p[0]; tp[k].y = (float)p[1]; tp[k].z = (float)p[2];
            tp[k].rank_rad = (r << 4) | rad[r];
            if (k > 0 && rnd(&ts) < 0.02) { /* branch from an earlier point of this tube */
                uint64_t j = (uint64_t)(rnd(&ts) * (double)(k + 1));
                if (j > k) j = k;
                p[0] = tp[j].x; p[1] = tp[j].y; p[2] = tp[j].z;
                for (int a = 0; a < 3; a++) d[a] += 0.8 * rnd_normal(&ts);
            } else {
                for (int a = 0; a < 3; a++) d[a] += 0.3 * rnd_normal(&ts);
            }
            nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) + 1e-12;
            for (int a = 0; a < 3; a++) d[a] /= nn;
            p[0] = reflect(p[0] + d[0], &d[0], nx);
            p[1] = reflect(p[1] + d[1], &d[1], ny);
            p[2] = reflect(p[2] + d[2], &d[2], nz);
        }
    }
    /* rank buffer: 0 = empty, else min rank */
    uint64_t nv = (uint64_t)nx * ny * nz;
    memset(out, 0, sizeof(uint32_t) * nv);
    qsort(pts, total, sizeof(tube_pt), cmp_pt_z);
    int nslab = 64;
    if ((uint32_t)nslab > nz) nslab = (int)nz;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int sl = 0; sl < nslab; sl++) {
        int64_t z0 = (int64_t)nz * sl / nslab, z1 = (int64_t)nz * (sl + 1) / nslab;
        /* points whose ball can reach [z0, z1): z in (z0 - 9, z1 + 9) */
        uint64_t lo = 0, hi = total;
        while (lo < hi) { uint64_t m = (lo + hi) / 2; if (pts[m].z < (float)(z0 - 9)) lo = m + 1; else hi = m; }
        for (uint64_t k = lo; k < total && pts[k].z < (float)(z1 + 9); k++) {
            uint32_t rr = pts[k].rank_rad >> 4, R = pts[k].rank_rad & 15;
            double cx = pts[k].x, cy = pts[k].y, cz = pts[k].z, R2 = (double)R * R;
            int64_t za = (int64_t)floor(cz - R), zb = (int64_t)ceil(cz + R);
            if (za < z0) za = z0;
            if (zb > z1 - 1) zb = z1 - 1;
            for (int64_t z = za; z <= zb; z++) {
                double dz = z + 0.5 - cz, rz = R2 - dz * dz;
                if (rz < 0) continue;
                double ry = sqrt(rz);
                int64_t ya = (int64_t)ceil(cy - ry - 0.5), yb = (int64_t)floor(cy + ry - 0.5);
                if (ya < 0) ya = 0;
                if (yb > (int64_t)ny - 1) yb = ny - 1;
                for (int64_t y = ya; y <= yb; y++) {
                    double dy = y + 0.5 - cy, rx2 = rz - dy * dy;
                    if (rx2 < 0) continue;
                    double rx = sqrt(rx2);
                    int64_t xa = (int64_t)ceil(cx - rx - 0.5), xb = (int64_t)floor(cx + rx - 0.5);
                    if (xa < 0) xa = 0;
                    if (xb > (int64_t)nx - 1) xb = nx - 1;
                    uint32_t *row = out + ((uint64_t)z * ny + (uint64_t)y) * nx;
                    for (int64_t x = xa; x <= xb; x++)
                        if (row[x] == 0 || row[x] > rr) row[x] = rr;
                }
            }
        }
    }
    uint64_t cnt = 0;
    #pragma omp parallel for schedule(static) reduction(+ : cnt)
    for (int64_t v = 0; v < (int64_t)nv; v++) {
        if (out[v]) { out[v] = perm[out[v] - 1]; cnt++; }
    }
    if (painted) *painted = cnt;
    free(pts); free(nsteps); free(rad); free(first); free(perm);
    return 0;
}

/* ------------------------------------------------------------------------
 * Brick requests of a camera fly-through (the serving workload).
 *
 * Camera: closed uniform Catmull-Rom path through 8 control points drawn
 * uniformly (stream path_seed) at least 15 % of each extent inside the
 * volume, one lap per `period` seconds, looking along the path's tangent.
 * Requests: Poisson arrivals at `rate` per second over [t0, t0 + duration)
 * (stream seed).  Each picks a direction uniform in the view cone (full
 * angle cone_deg) and a distance with density proportional to d^2 up to
 * d_max, redrawn until the point lies inside the volume (after 1000 misses
 * the camera's own position is used); its brick (x fastest) is requested at
 * level 0 below d0, else at clamp(floor(log2(d / d0)) + 1, 0, max_lod).
 * Writes at most cap requests; *n_out receives the count.  Times in ns
 * relative to t0.
 * ------------------------------------------------------------------------ */
static void catmull_rom3(const double (*c)[3], int n, double u, double pos[3], double tan[3]) {
    double s = u * n;
    long i = (long)floor(s);
    double f = s - (double)i;
    i %= n;
    const double *p0 = c[(i + n - 1) % n], *p1 = c[i], *p2 = c[(i + 1) % n], *p3 = c[(i + 2) % n];
    for (int k = 0; k < 3; k++) {
        double a = -p0[k] + p2[k], b = 2 * p0[k] - 5 * p1[k] + 4 * p2[k] - p3[k];
        double cc = -p0[k] + 3 * p1[k] - 3 * p2[k] + p3[k];
        pos[k] = 0.5 * (2 * p1[k] + a * f + b * f * f + cc * f * f * f);
        tan[k] = 0.5 * (a + 2 * b * f + 3 * cc * f * f);
    }
}

static void camera_ctrl(uint32_t nx, uint32_t ny, uint32_t nz, uint64_t path_seed, double ctrl[8][3]) {
    uint64_t ps = path_seed;
    const double ext[3] = {nx, ny, nz};
    for (int i = 0; i < 8; i++)
        for (int k = 0; k < 3; k++) ctrl[i][k] = ext[k] * (0.15 + 0.7 * rnd(&ps));
}

/* the 8 control points (x, y, z) of the camera path, and the camera's
 * position and tangent at path parameter u in [0, 1) */
int synth_camera_path(uint32_t nx, uint32_t ny, uint32_t nz, uint64_t path_seed, double *ctrl24) {
    double c[8][3];
    camera_ctrl(nx, ny, nz, path_seed, c);
    memcpy(ctrl24, c, sizeof(c));
    return 0;
}

void synth_camera_pose(const double *ctrl24, double u, double *pos3, double *tan3) {
    catmull_rom3((const double(*)[3])ctrl24, 8, u, pos3, tan3);
}

int synth_camera_trace(uint32_t nx, uint32_t ny, uint32_t nz, double rate, double duration, double t0, uint64_t seed,
                       uint64_t path_seed, double period, double cone_deg, double d_max, double d0, uint32_t brick,
                       uint32_t max_lod, uint64_t cap, uint32_t *ids, uint8_t *lods, uint64_t *t_ns, uint64_t *n_out) {
    if (!ids || !lods || !t_ns || !n_out || rate <= 0 || brick == 0 || nx < brick || ny < brick || nz < brick) return 1;
    double ctrl[8][3];
    camera_ctrl(nx, ny, nz, path_seed, ctrl);
    const double ext[3] = {nx, ny, nz};
    uint64_t s = seed;
    const double cos_half = cos(cone_deg * 0.5 * 3.14159265358979323846 / 180.0);
    const uint32_t nbx = nx / brick, nby = ny / brick;
    double t = 0;
    uint64_t n = 0;
    for (;;) {
        t += -log(1.0 - rnd(&s)) / rate;
        if (t >= duration || n >= cap) break;
        double pos[3], tan[3], fw[3], e1[3], e2[3];
        double u = fmod((t + t0) / period, 1.0);
        catmull_rom3((const double(*)[3])ctrl, 8, u, pos, tan);
        double ln = sqrt(tan[0] * tan[0] + tan[1] * tan[1] + tan[2] * tan[2]);
        if (ln < 1e-9) ln = 1e-9;
        for (int k = 0; k < 3; k++) fw[k] = tan[k] / ln;
        double h[3] = {0, 0, 1};
        if (fabs(fw[2]) >= 0.9) { h[0] = 1; h[2] = 0; }
        e1[0] = fw[1] * h[2] - fw[2] * h[1];
        e1[1] = fw[2] * h[0] - fw[0] * h[2];
        e1[2] = fw[0] * h[1] - fw[1] * h[0];
        double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int k = 0; k < 3; k++) e1[k] /= l1;
        e2[0] = fw[1] * e1[2] - fw[2] * e1[1];
        e2[1] = fw[2] * e1[0] - fw[0] * e1[2];
        e2[2] = fw[0] * e1[1] - fw[1] * e1[0];
        double p[3] = {pos[0], pos[1], pos[2]}, d = 0;
        int found = 0;
        for (int tries = 0; tries < 1000 && !found; tries++) {
            double ct = cos_half + (1.0 - cos_half) * rnd(&s);
            double st = sqrt(1.0 - ct * ct), ph = 2 * 3.14159265358979323846 * rnd(&s);
            d = d_max * cbrt(rnd(&s));
            for (int k = 0; k < 3; k++) p[k] = pos[k] + d * (ct * fw[k] + st * (cos(ph) * e1[k] + sin(ph) * e2[k]));
            found = p[0] >= 0 && p[1] >= 0 && p[2] >= 0 && p[0] < nx && p[1] < ny && p[2] < nz;
        }
        if (!found) {
            for (int k = 0; k < 3; k++) {
                p[k] = pos[k] < 0 ? 0 : pos[k];
                if (p[k] > ext[k] - 1) p[k] = ext[k] - 1;
            }
            d = 0;
        }
        uint32_t bx = (uint32_t)(p[0] / brick), by = (uint32_t)(p[1] / brick), bz = (uint32_t)(p[2] / brick);
        ids[n] = bx + nbx * (by + nby * bz);
        int lod = d < d0 ? 0 : (int)floor(log2(d / d0)) + 1;
        lods[n] = (uint8_t)(lod < 0 ? 0 : (lod > (int)max_lod ? (int)max_lod : lod));
        t_ns[n] = (uint64_t)(t * 1e9);
        n++;
    }
    *n_out = n;
    return 0;
}
