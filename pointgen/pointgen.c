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
