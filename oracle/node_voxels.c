/*
 * Voxel sets of single inner nodes, from the definition, streamed.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  It shares no code with
 * the HIP library or with the other oracle files.
 *
 * For an inner node N at depth d, the definition of the octree LOD gives one
 * voxel per occupied cell of the R^3 grid inscribed in N (section "Voxel
 * Sampling Grid"), placed at the cell centre (section "Octree") and coloured
 * by the point of N's region with the smallest key in that cell (section
 * "Voxel Sampling": the first point that falls into an empty cell; first =
 * smallest key).  Keys are positions in the cumulative point sequence, so
 * feeding the points in key order and keeping, per cell, the first point
 * that lands there gives exactly that set.  This file does only that, for a
 * list of node paths, without building the rest of the octree, so that the
 * voxel lists of the top nodes of a very large cloud can be computed in one
 * pass over the points.  Whether N is inner at all is not decided here.
 *
 * Integer coordinates, cells and centres follow the reading stated in
 * oracle/definition.py: K = Dmax + r bits per axis,
 * q = min(floor(fl32(fl32(v - min) * scale)), 2^K - 1), 0 for negative or NaN;
 * N's region is the points whose top d bits of q (per axis) equal N's path
 * digits (octant bit 0 = x, bit 1 = y, bit 2 = z); the cell is
 * (q >> (Dmax - d)) & (R - 1) per axis; the centre of global cell g is
 * fl32(min + fl32(fl32(g + 0.5) * size * 2^-(r + d))).
 * Compile with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float x, y, z;
    uint32_t rgba;
} nv_rec;

typedef struct {
    uint64_t path;
    uint32_t depth;
    uint32_t ox, oy, oz;  /* the node's top `depth` bits per axis */
    uint32_t* first;      /* per cell: key + 1 of its first point, 0 = empty */
    uint32_t* rgba;       /* per cell: that point's colour */
    uint32_t count;       /* occupied cells */
} nv_node;

typedef struct {
    float mn[3];
    float size, scale;
    uint32_t K, r, R, Dmax;
    uint32_t nnodes;
    nv_node* nodes;
    uint64_t total; /* points fed so far = key of the next point */
} nv_state;

static uint32_t nv_quant(float v, float mn, float scale, uint32_t K) {
    float u = (v - mn) * scale;
    if (!(u >= 0.0f)) return 0u;
    float f = floorf(u);
    float qmax = (float)((1u << K) - 1u);
    if (f > qmax) f = qmax;
    return (uint32_t)f;
}

static float nv_centre(uint32_t g, float mn, float size, uint32_t r, uint32_t d) {
    float h = ldexpf(size, -(int)(r + d));
    float gf = (float)g + 0.5f;
    float prod = gf * h;
    return mn + prod;
}

void nv_destroy(nv_state* s) {
    if (!s) return;
    for (uint32_t i = 0; i < s->nnodes; ++i) {
        free(s->nodes[i].first);
        free(s->nodes[i].rgba);
    }
    free(s->nodes);
    free(s);
}

/* paths: n node paths (1 = root, parent * 8 + octant below it), each at a
 * depth below max_depth.  Returns NULL on a bad argument or allocation. */
nv_state* nv_create(const float* root_min, float root_size, uint32_t grid_bits,
                    uint32_t max_depth, const uint64_t* paths, uint32_t n) {
    if (grid_bits > 8 || max_depth + grid_bits > 24 || !(root_size > 0.0f)) return NULL;
    nv_state* s = (nv_state*)calloc(1, sizeof(nv_state));
    if (!s) return NULL;
    for (int a = 0; a < 3; ++a) s->mn[a] = root_min[a];
    s->size = root_size;
    s->K = max_depth + grid_bits;
    s->r = grid_bits;
    s->R = 1u << grid_bits;
    s->Dmax = max_depth;
    s->scale = (float)(1u << s->K) / root_size;
    s->nodes = (nv_node*)calloc(n ? n : 1, sizeof(nv_node));
    if (!s->nodes) {
        free(s);
        return NULL;
    }
    s->nnodes = n;
    const size_t cells = (size_t)s->R * s->R * s->R;
    for (uint32_t i = 0; i < n; ++i) {
        nv_node* nd = &s->nodes[i];
        uint64_t p = paths[i];
        uint32_t digits[32], d = 0;
        while (p > 1 && d < 32) {
            digits[d++] = (uint32_t)(p & 7u);
            p >>= 3;
        }
        if (paths[i] == 0 || p != 1 || d >= max_depth) {
            nv_destroy(s);
            return NULL;
        }
        nd->path = paths[i];
        nd->depth = d;
        for (uint32_t j = 0; j < d; ++j) { /* digits[d-1] is the root's octant */
            const uint32_t o = digits[d - 1 - j];
            nd->ox = (nd->ox << 1) | (o & 1u);
            nd->oy = (nd->oy << 1) | ((o >> 1) & 1u);
            nd->oz = (nd->oz << 1) | ((o >> 2) & 1u);
        }
        nd->first = (uint32_t*)calloc(cells, sizeof(uint32_t));
        nd->rgba = (uint32_t*)calloc(cells, sizeof(uint32_t));
        if (!nd->first || !nd->rgba) {
            nv_destroy(s);
            return NULL;
        }
    }
    return s;
}

/* The next n points of the sequence, in key order.  Returns -1 when the keys
 * would pass 2^32 - 1. */
int nv_feed(nv_state* s, const nv_rec* pts, uint64_t n) {
    if (s->total + n > 0xFFFFFFFFull) return -1;
    const uint32_t rm = s->R - 1u;
    for (uint64_t i = 0; i < n; ++i) {
        const nv_rec* p = &pts[i];
        const uint32_t qx = nv_quant(p->x, s->mn[0], s->scale, s->K);
        const uint32_t qy = nv_quant(p->y, s->mn[1], s->scale, s->K);
        const uint32_t qz = nv_quant(p->z, s->mn[2], s->scale, s->K);
        const uint32_t key = (uint32_t)(s->total + i);
        for (uint32_t k = 0; k < s->nnodes; ++k) {
            nv_node* nd = &s->nodes[k];
            const uint32_t top = s->K - nd->depth; /* bits below the node's prefix */
            if (nd->depth > 0 &&
                ((qx >> top) != nd->ox || (qy >> top) != nd->oy || (qz >> top) != nd->oz))
                continue;
            const uint32_t sh = s->Dmax - nd->depth;
            const size_t cell = (size_t)((qx >> sh) & rm) +
                                (size_t)s->R * ((size_t)((qy >> sh) & rm) +
                                                (size_t)s->R * (size_t)((qz >> sh) & rm));
            if (nd->first[cell] == 0u) {
                nd->first[cell] = key + 1u;
                nd->rgba[cell] = p->rgba;
                nd->count++;
            }
        }
    }
    s->total += n;
    return 0;
}

/* Voxels of node k: returns the count; with non-NULL buffers (room for the
 * count) fills the voxel records and their colouring points' keys, sorted
 * by key. */
static int nv_cmp_key(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t nv_export(const nv_state* s, uint32_t k, nv_rec* recs, uint32_t* keys) {
    if (k >= s->nnodes) return -1;
    const nv_node* nd = &s->nodes[k];
    if (!recs || !keys) return nd->count;
    const size_t cells = (size_t)s->R * s->R * s->R;
    uint64_t* order = (uint64_t*)malloc((nd->count ? nd->count : 1) * sizeof(uint64_t));
    if (!order) return -1;
    uint32_t m = 0;
    for (size_t c = 0; c < cells; ++c)
        if (nd->first[c]) order[m++] = ((uint64_t)(nd->first[c] - 1u) << 32) | (uint64_t)c;
    qsort(order, m, sizeof(uint64_t), nv_cmp_key);
    for (uint32_t i = 0; i < m; ++i) {
        const uint32_t c = (uint32_t)(order[i] & 0xFFFFFFFFu);
        const uint32_t cx = c % s->R, cy = (c / s->R) % s->R, cz = c / (s->R * s->R);
        /* global cell coordinate at depth d: the node's prefix, then the cell */
        const uint32_t gx = (nd->ox << s->r) | cx;
        const uint32_t gy = (nd->oy << s->r) | cy;
        const uint32_t gz = (nd->oz << s->r) | cz;
        recs[i].x = nv_centre(gx, s->mn[0], s->size, s->r, nd->depth);
        recs[i].y = nv_centre(gy, s->mn[1], s->size, s->r, nd->depth);
        recs[i].z = nv_centre(gz, s->mn[2], s->size, s->r, nd->depth);
        recs[i].rgba = nd->rgba[c];
        keys[i] = (uint32_t)(order[i] >> 32);
    }
    free(order);
    return m;
}
