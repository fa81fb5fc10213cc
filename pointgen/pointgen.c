/*
 * Seeded synthetic point clouds (16-byte XYZRGBA records), multithreaded.
 *
 * Input generators only: nothing here computes any part of the octree.
 * Output depends only on the arguments, never on the thread count:
 * randomness is counter-based (SplitMix64 of seed, stream and index, Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", 2014),
 * candidates are generated in fixed blocks and concatenated in block order.
 *
 * Aerial heightfield (the aerial-LiDAR-shaped workload):
 *   x, y uniform over [0, extent)^2; a candidate is kept with probability
 *   0.25 + 0.75 * mask(x, y), mask = one octave of value noise with a 250 m
 *   period (a 4x density variation); z = z0 + relief * fbm(x, y), fbm = 8
 *   octaves of value noise (period 400 m, lacunarity 2, gain 0.5) normalised
 *   to [0, 1]; colour is a ramp over the normalised height, alpha 255.
 *   Value noise: a hash of the integer lattice corner gives a value in
 *   [0, 1), bilinearly blended with the smoothstep weight 3t^2 - 2t^3.
 *
 * Ordering: points are sorted by the 63-bit Morton code of their 21-bit
 * integer coordinates over the given cube (LSD radix sort, stable), then cut
 * into batches whose order is shuffled (Fisher-Yates); or kept in Morton
 * order; or fully shuffled.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float x, y, z;
    uint32_t rgba;
} pg_rec;

static inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t i) {
    return splitmix64(splitmix64(seed * 0x632BE59BD9B4E019ull + stream) ^ i);
}

/* uniform in [0, 1) with 53 random bits */
static inline double unif(uint64_t seed, uint64_t stream, uint64_t i) {
    return (double)(rnd(seed, stream, i) >> 11) * (1.0 / 9007199254740992.0);
}

static inline double lattice(uint64_t seed, uint64_t octave, int64_t ix, int64_t iy) {
    uint64_t h = splitmix64(seed ^ splitmix64(octave * 0x9E3779B97F4A7C15ull ^
                                              splitmix64((uint64_t)ix * 0xD1B54A32D192ED03ull ^
                                                         (uint64_t)iy)));
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

static double value_noise(uint64_t seed, uint64_t octave, double x, double y) {
    double fx = floor(x), fy = floor(y);
    int64_t ix = (int64_t)fx, iy = (int64_t)fy;
    double tx = x - fx, ty = y - fy;
    double sx = tx * tx * (3.0 - 2.0 * tx), sy = ty * ty * (3.0 - 2.0 * ty);
    double a = lattice(seed, octave, ix, iy), b = lattice(seed, octave, ix + 1, iy);
    double c = lattice(seed, octave, ix, iy + 1), d = lattice(seed, octave, ix + 1, iy + 1);
    double ab = a + (b - a) * sx, cd = c + (d - c) * sx;
    return ab + (cd - ab) * sy;
}

static double fbm8(uint64_t seed, double x, double y, double period) {
    double f = 1.0 / period, amp = 1.0, sum = 0.0, norm = 0.0;
    for (int o = 0; o < 8; ++o) {
        sum += amp * value_noise(seed, 16 + (uint64_t)o, x * f, y * f);
        norm += amp;
        amp *= 0.5;
        f *= 2.0;
    }
    return sum / norm;
}

static uint32_t pack_rgba(double r, double g, double b, double a) {
#define PG_B(v) ((uint32_t)((v) < 0 ? 0 : ((v) > 255 ? 255 : (v))))
    return PG_B(r) | (PG_B(g) << 8) | (PG_B(b) << 16) | (PG_B(a) << 24);
#undef PG_B
}

#define PG_BLOCK 65536u

/* Generates one block of candidates; writes accepted ones to out (may be
   NULL to count only).  Returns the number accepted. */
static uint32_t aerial_block(uint64_t seed, uint64_t blk, double extent, double z0, double relief,
                             pg_rec* out) {
    uint32_t k = 0;
    for (uint32_t j = 0; j < PG_BLOCK; ++j) {
        uint64_t i = blk * PG_BLOCK + j;
        double x = unif(seed, 1, i) * extent;
        double y = unif(seed, 2, i) * extent;
        double mask = value_noise(seed, 1, x / 250.0, y / 250.0);
        if (!(unif(seed, 3, i) < 0.25 + 0.75 * mask)) continue;
        if (out) {
            double h = fbm8(seed, x, y, 400.0);
            pg_rec r;
            r.x = (float)x;
            r.y = (float)y;
            r.z = (float)(z0 + relief * h);
            double t = h;
            r.rgba = pack_rgba(30.0 + 210.0 * t, 90.0 + 150.0 * (1.0 - fabs(2.0 * t - 1.0)),
                               200.0 - 170.0 * t, 255.0);
            out[k] = r;
        }
        ++k;
    }
    return k;
}

static inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

static inline uint64_t q21(float v, float mn, float size) {
    double u = ((double)v - (double)mn) / (double)size * 2097152.0;
    if (!(u >= 0.0)) return 0;
    if (u >= 2097151.0) return 2097151;
    return (uint64_t)u;
}

/* Stable LSD radix sort of recs by 63-bit Morton code, 7 passes of 9 bits. */
static int morton_sort(pg_rec* recs, uint64_t n, const float* mn, float size, int threads) {
    uint64_t* key = (uint64_t*)malloc(n * 8);
    uint64_t* key2 = (uint64_t*)malloc(n * 8);
    pg_rec* tmp = (pg_rec*)malloc(n * sizeof(pg_rec));
    if (!key || !key2 || !tmp) {
        free(key);
        free(key2);
        free(tmp);
        return -1;
    }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        key[i] = spread3(q21(recs[i].x, mn[0], size)) | (spread3(q21(recs[i].y, mn[1], size)) << 1) |
                 (spread3(q21(recs[i].z, mn[2], size)) << 2);
    }
    const int bits = 9, buckets = 1 << 9;
    int T = threads < 1 ? 1 : threads;
    uint64_t* hist = (uint64_t*)calloc((size_t)T * buckets, 8);
    if (!hist) {
        free(key);
        free(key2);
        free(tmp);
        return -1;
    }
    for (int pass = 0; pass < 7; ++pass) {
        int sh = pass * bits;
        memset(hist, 0, (size_t)T * buckets * 8);
#pragma omp parallel num_threads(T)
        {
            int t = 0, nt = 1;
#ifdef _OPENMP
            t = omp_get_thread_num();
            nt = omp_get_num_threads();
#endif
            uint64_t lo = n * (uint64_t)t / (uint64_t)nt, hi = n * (uint64_t)(t + 1) / (uint64_t)nt;
            uint64_t* hh = hist + (size_t)t * buckets;
            for (uint64_t i = lo; i < hi; ++i) hh[(key[i] >> sh) & (buckets - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                uint64_t off = 0;
                for (int b = 0; b < buckets; ++b)
                    for (int u = 0; u < nt; ++u) {
                        uint64_t c = hist[(size_t)u * buckets + b];
                        hist[(size_t)u * buckets + b] = off;
                        off += c;
                    }
            }
            for (uint64_t i = lo; i < hi; ++i) {
                uint64_t p = hh[(key[i] >> sh) & (buckets - 1)]++;
                key2[p] = key[i];
                tmp[p] = recs[i];
            }
        }
        uint64_t* sk = key;
        key = key2;
        key2 = sk;
        memcpy(recs, tmp, n * sizeof(pg_rec));
    }
    free(hist);
    free(key);
    free(key2);
    free(tmp);
    return 0;
}

static int reorder(pg_rec* recs, uint64_t n, uint64_t seed, int order, uint64_t batch,
                   const float* mn, float size, int threads) {
    if (order == 0) return 0; /* generation order */
    if (order == 3) {         /* full random shuffle */
        for (uint64_t i = n; i > 1; --i) {
            uint64_t j = rnd(seed, 98, i) % i;
            pg_rec t = recs[i - 1];
            recs[i - 1] = recs[j];
            recs[j] = t;
        }
        return 0;
    }
    if (morton_sort(recs, n, mn, size, threads)) return -1;
    if (order == 1) return 0; /* Morton order */
    /* order 2: Morton order cut into batches, batch order shuffled */
    uint64_t nb = (n + batch - 1) / batch;
    uint64_t* perm = (uint64_t*)malloc(nb * 8);
    pg_rec* tmp = (pg_rec*)malloc(n * sizeof(pg_rec));
    if (!perm || !tmp) {
        free(perm);
        free(tmp);
        return -1;
    }
    for (uint64_t b = 0; b < nb; ++b) perm[b] = b;
    for (uint64_t i = nb; i > 1; --i) {
        uint64_t j = rnd(seed, 99, i) % i;
        uint64_t t = perm[i - 1];
        perm[i - 1] = perm[j];
        perm[j] = t;
    }
    uint64_t w = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        uint64_t lo = perm[b] * batch, hi = lo + batch < n ? lo + batch : n;
        memcpy(tmp + w, recs + lo, (hi - lo) * sizeof(pg_rec));
        w += hi - lo;
    }
    memcpy(recs, tmp, n * sizeof(pg_rec));
    free(perm);
    free(tmp);
    return 0;
}

/* Aerial heightfield cloud of exactly n points.  order: 0 generation,
   1 Morton, 2 Morton batches shuffled, 3 random.  cube_min/cube_size: the
   cube for the Morton code. */
int pg_aerial(pg_rec* out, uint64_t n, uint64_t seed, double extent, double z0, double relief,
              int order, uint64_t batch, const float* cube_min, float cube_size, int threads) {
    if (threads < 1) threads = 1;
    uint64_t nblk = (uint64_t)((double)n / (0.25 * PG_BLOCK)) + 2;
    uint32_t* acc = (uint32_t*)malloc(nblk * 4);
    uint64_t* off = (uint64_t*)malloc((nblk + 1) * 8);
    if (!acc || !off) {
        free(acc);
        free(off);
        return -1;
    }
    /* count pass, stop once enough blocks are known */
    uint64_t have = 0, used = 0;
    const uint64_t chunk = 256;
    while (have < n && used < nblk) {
        uint64_t hi = used + chunk < nblk ? used + chunk : nblk;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
        for (int64_t b = (int64_t)used; b < (int64_t)hi; ++b)
            acc[b] = aerial_block(seed, (uint64_t)b, extent, z0, relief, NULL);
        for (uint64_t b = used; b < hi && have < n; ++b) {
            off[b] = have;
            have += acc[b];
            used = b + 1;
        }
        if (have < n) used = hi;
    }
    if (have < n) {
        free(acc);
        free(off);
        return -2;
    }
    pg_rec* tmp = (pg_rec*)malloc((size_t)PG_BLOCK * sizeof(pg_rec) * (size_t)threads);
    if (!tmp) {
        free(acc);
        free(off);
        return -1;
    }
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t b = 0; b < (int64_t)used; ++b) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        pg_rec* buf = tmp + (size_t)t * PG_BLOCK;
        uint32_t k = aerial_block(seed, (uint64_t)b, extent, z0, relief, buf);
        uint64_t o = off[b];
        uint64_t m = o + k <= n ? k : n - o;
        memcpy(out + o, buf, m * sizeof(pg_rec));
    }
    free(tmp);
    free(acc);
    free(off);
    return reorder(out, n, seed, order, batch, cube_min, cube_size, threads);
}

/* ------------------------------------------------------------------------
 * Dense-scan building (the terrestrial-scan-shaped workload).
 *
 * A 60 x 60 x 15 m building, footprint [2, 62)^2, floors at z = 2 + 3.75 k,
 * inside the cube [0, 64)^3, made of 2,000 primitives:
 *   5 floor / ceiling slabs (60 x 60), 4 outer walls (60 x 15),
 *   591 interior walls (one storey high, length 1-15 m, normal along x or y),
 *   1,400 furniture boxes (0.3-2.5 m wide and deep, 0.3-2.2 m high) whose
 *   4 sides and top are scanned.
 * Density on every face is a uniform background plus 200 Gaussian hotspots
 * (sigma 0.5 m, peak 20x the background: mass 19 * 2 pi sigma^2 each), each
 * centred at an area-uniform position on an area-chosen face and spread in
 * that face's plane (truncated to the face by rejection).  The n points are
 * apportioned over faces and hotspots by mass (largest remainder).
 *
 * Scan-like order: primitives in a seeded random order; within a primitive
 * its faces' background points, each face swept in 5 cm strips along its
 * first axis (random inside a strip), then the bursts of its hotspots.
 * Colour: a random base colour per primitive plus +-16 jitter per channel,
 * alpha 255.
 * ------------------------------------------------------------------------ */

typedef struct {
    double o[3];     /* corner */
    int au, av;      /* spanning axes */
    double lu, lv;   /* extents along au, av */
    uint32_t prim;
} pg_face;

typedef struct {
    uint32_t face;
    double cu, cv;
} pg_spot;

#define PG_NPRIM 2000
#define PG_NSPOT 200
#define PG_SIGMA 0.5
#define PG_STRIP 0.05

static pg_face mkface(double x, double y, double z, int au, double lu, int av, double lv,
                      uint32_t prim) {
    pg_face f;
    f.o[0] = x;
    f.o[1] = y;
    f.o[2] = z;
    f.au = au;
    f.av = av;
    f.lu = lu;
    f.lv = lv;
    f.prim = prim;
    return f;
}

/* Faces of the building; returns their number (at most 5 + 4 + 591 + 5 * 1400). */
static uint32_t building_faces(uint64_t seed, pg_face* F) {
    uint32_t nf = 0, p = 0;
    const double lo = 2.0, span = 60.0, storey = 3.75;
    for (int k = 0; k < 5; ++k, ++p) F[nf++] = mkface(lo, lo, lo + storey * k, 0, span, 1, span, p);
    F[nf++] = mkface(lo, lo, lo, 1, span, 2, 4 * storey, p++);
    F[nf++] = mkface(lo + span, lo, lo, 1, span, 2, 4 * storey, p++);
    F[nf++] = mkface(lo, lo, lo, 0, span, 2, 4 * storey, p++);
    F[nf++] = mkface(lo, lo + span, lo, 0, span, 2, 4 * storey, p++);
    for (; p < 600; ++p) {
        double s = floor(unif(seed, 200, p) * 4.0);
        int normal_x = unif(seed, 201, p) < 0.5;
        double len = 1.0 + 14.0 * unif(seed, 202, p);
        double a = lo + (span - len) * unif(seed, 203, p);
        double c = lo + 0.1 + (span - 0.2) * unif(seed, 204, p);
        double z = lo + storey * s;
        if (normal_x) F[nf++] = mkface(c, a, z, 1, len, 2, storey, p);
        else F[nf++] = mkface(a, c, z, 0, len, 2, storey, p);
    }
    for (; p < PG_NPRIM; ++p) {
        double s = floor(unif(seed, 210, p) * 4.0);
        double w = 0.3 + 2.2 * unif(seed, 211, p), d = 0.3 + 2.2 * unif(seed, 212, p);
        double h = 0.3 + 1.9 * unif(seed, 213, p);
        double x = lo + (span - w) * unif(seed, 214, p), y = lo + (span - d) * unif(seed, 215, p);
        double z = lo + storey * s;
        F[nf++] = mkface(x, y, z, 1, d, 2, h, p);
        F[nf++] = mkface(x + w, y, z, 1, d, 2, h, p);
        F[nf++] = mkface(x, y, z, 0, w, 2, h, p);
        F[nf++] = mkface(x, y + d, z, 0, w, 2, h, p);
        F[nf++] = mkface(x, y, z + h, 0, w, 1, d, p);
    }
    return nf;
}

typedef struct {
    double frac;
    uint32_t idx;
} pg_rem;

static int rem_cmp(const void* a, const void* b) {
    const pg_rem* x = (const pg_rem*)a;
    const pg_rem* y = (const pg_rem*)b;
    if (x->frac != y->frac) return x->frac > y->frac ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static uint32_t prim_colour(uint64_t seed, uint32_t prim) {
    uint64_t h = rnd(seed, 230, prim);
    return (uint32_t)(h & 0xFFFFFFu);
}

static pg_rec face_point(const pg_face* f, double u, double v, uint32_t base, uint64_t jit) {
    double pos[3] = {f->o[0], f->o[1], f->o[2]};
    pos[f->au] += u;
    pos[f->av] += v;
    pg_rec r;
    r.x = (float)pos[0];
    r.y = (float)pos[1];
    r.z = (float)pos[2];
    double c[3];
    for (int k = 0; k < 3; ++k)
        c[k] = (double)((base >> (8 * k)) & 255u) + (double)((jit >> (8 * k)) & 31u) - 16.0;
    r.rgba = pack_rgba(c[0], c[1], c[2], 255.0);
    return r;
}

/* Dense-scan cloud of exactly n points in scan-like order (see above). */
int pg_dense_scan(pg_rec* out, uint64_t n, uint64_t seed, int threads) {
    if (threads < 1) threads = 1;
    const uint32_t max_faces = 5 + 4 + 591 + 5 * 1400;
    pg_face* F = (pg_face*)malloc(max_faces * sizeof(pg_face));
    pg_spot* H = (pg_spot*)malloc(PG_NSPOT * sizeof(pg_spot));
    uint32_t ncomp_max = max_faces + PG_NSPOT;
    uint64_t* cnt = (uint64_t*)calloc(ncomp_max, 8);
    uint64_t* off = (uint64_t*)calloc(ncomp_max, 8);
    pg_rem* rem = (pg_rem*)malloc(ncomp_max * sizeof(pg_rem));
    uint32_t* perm = (uint32_t*)malloc(PG_NPRIM * 4);
    uint32_t* first_face = (uint32_t*)malloc((PG_NPRIM + 1) * 4);
    if (!F || !H || !cnt || !off || !rem || !perm || !first_face) {
        free(F); free(H); free(cnt); free(off); free(rem); free(perm); free(first_face);
        return -1;
    }
    const uint32_t nf = building_faces(seed, F);
    const uint32_t nc = nf + PG_NSPOT;
    double area_sum = 0.0;
    for (uint32_t i = 0; i < nf; ++i) area_sum += F[i].lu * F[i].lv;
    /* hotspots: face chosen with probability proportional to area */
    for (uint32_t k = 0; k < PG_NSPOT; ++k) {
        double t = unif(seed, 220, k) * area_sum, acc = 0.0;
        uint32_t f = nf - 1;
        for (uint32_t i = 0; i < nf; ++i) {
            acc += F[i].lu * F[i].lv;
            if (t < acc) {
                f = i;
                break;
            }
        }
        H[k].face = f;
        H[k].cu = unif(seed, 221, k) * F[f].lu;
        H[k].cv = unif(seed, 222, k) * F[f].lv;
    }
    /* apportion n over components by mass, largest remainder */
    const double spot_mass = 19.0 * 2.0 * 3.14159265358979323846 * PG_SIGMA * PG_SIGMA;
    const double total = area_sum + spot_mass * PG_NSPOT;
    uint64_t given = 0;
    for (uint32_t c = 0; c < nc; ++c) {
        double m = c < nf ? F[c].lu * F[c].lv : spot_mass;
        double e = (double)n * m / total;
        double fl = floor(e);
        cnt[c] = (uint64_t)fl;
        given += cnt[c];
        rem[c].frac = e - fl;
        rem[c].idx = c;
    }
    qsort(rem, nc, sizeof(pg_rem), rem_cmp);
    for (uint64_t i = 0; given < n; ++i, ++given) cnt[rem[i % nc].idx]++;
    /* scan order: primitives permuted; faces in order, then hotspot bursts */
    for (uint32_t p = 0; p < PG_NPRIM; ++p) perm[p] = p;
    for (uint32_t i = PG_NPRIM; i > 1; --i) {
        uint32_t j = (uint32_t)(rnd(seed, 223, i) % i);
        uint32_t t = perm[i - 1];
        perm[i - 1] = perm[j];
        perm[j] = t;
    }
    for (uint32_t p = 0, i = 0; p <= PG_NPRIM; ++p) {
        while (i < nf && F[i].prim < p) ++i;
        first_face[p] = i;
    }
    uint64_t w = 0;
    for (uint32_t pi = 0; pi < PG_NPRIM; ++pi) {
        uint32_t p = perm[pi];
        for (uint32_t f = first_face[p]; f < first_face[p + 1]; ++f) {
            off[f] = w;
            w += cnt[f];
        }
        for (uint32_t k = 0; k < PG_NSPOT; ++k)
            if (F[H[k].face].prim == p) {
                off[nf + k] = w;
                w += cnt[nf + k];
            }
    }
    /* generate: work units of up to 1M points of one component */
    const uint64_t unit = 1u << 20;
    uint64_t nunits = 0;
    for (uint32_t c = 0; c < nc; ++c) nunits += (cnt[c] + unit - 1) / unit;
    uint64_t* ucomp = (uint64_t*)malloc((nunits + 1) * 16);
    if (!ucomp || w != n) {
        free(ucomp); free(F); free(H); free(cnt); free(off); free(rem); free(perm);
        free(first_face);
        return -1;
    }
    uint64_t u = 0;
    for (uint32_t c = 0; c < nc; ++c)
        for (uint64_t j = 0; j < cnt[c]; j += unit) {
            ucomp[2 * u] = c;
            ucomp[2 * u + 1] = j;
            ++u;
        }
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t ui = 0; ui < (int64_t)nunits; ++ui) {
        uint32_t c = (uint32_t)ucomp[2 * ui];
        uint64_t j0 = ucomp[2 * ui + 1], N = cnt[c];
        uint64_t j1 = j0 + unit < N ? j0 + unit : N;
        if (c < nf) {
            const pg_face* f = &F[c];
            uint64_t S = (uint64_t)(f->lu / PG_STRIP + 0.5);
            if (S < 1) S = 1;
            uint32_t base = prim_colour(seed, f->prim);
            for (uint64_t j = j0; j < j1; ++j) {
                uint64_t s = j * S / N;
                double uu = ((double)s + unif(seed, 1000 + 3 * (uint64_t)c, j)) * (f->lu / (double)S);
                double vv = unif(seed, 1001 + 3 * (uint64_t)c, j) * f->lv;
                out[off[c] + j] = face_point(f, uu, vv, base, rnd(seed, 1002 + 3 * (uint64_t)c, j));
            }
        } else {
            const pg_spot* h = &H[c - nf];
            const pg_face* f = &F[h->face];
            uint32_t base = prim_colour(seed, f->prim);
            uint64_t st = 100000 + 4 * (uint64_t)(c - nf);
            for (uint64_t j = j0; j < j1; ++j) {
                double uu = h->cu, vv = h->cv;
                for (uint64_t a = 0; a < 16; ++a) {
                    double r1 = unif(seed, st, j * 16 + a), r2 = unif(seed, st + 1, j * 16 + a);
                    double rad = PG_SIGMA * sqrt(-2.0 * log(1.0 - r1));
                    double gu = h->cu + rad * cos(2.0 * 3.14159265358979323846 * r2);
                    double gv = h->cv + rad * sin(2.0 * 3.14159265358979323846 * r2);
                    if (gu >= 0.0 && gu < f->lu && gv >= 0.0 && gv < f->lv) {
                        uu = gu;
                        vv = gv;
                        break;
                    }
                }
                out[off[c] + j] = face_point(f, uu, vv, base, rnd(seed, st + 2, j));
            }
        }
    }
    free(ucomp);
    free(F);
    free(H);
    free(cnt);
    free(off);
    free(rem);
    free(perm);
    free(first_face);
    return 0;
}
