/*
 * O2: sequential top-down octree LOD inserter (plain C, one thread).
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  It shares no code with
 * the HIP library and is never linked into it.
 *
 * This is the classic CPU approach the paper contrasts its GPU method with
 * (section "Expanding the Octree"): each point, in key order, walks from the
 * root to its leaf; at every inner node on the way it marks its cell in the
 * node's R^3 occupancy grid and, if the cell was empty, creates a voxel at
 * the cell centre with the point's colour (section "Voxel Sampling"); at the
 * leaf it is appended.  A leaf that then holds more than T points below the
 * maximum depth "spills": it becomes an inner node with 8 empty children and
 * its points are re-inserted, in key order, starting at that node.
 *
 * Points are processed in key order and spilled points are re-inserted in
 * key order before any later point arrives, so "first point into an empty
 * cell" is the point with the smallest key, and every leaf and voxel list is
 * already sorted by key when exported.
 *
 * Integer coordinates, octants, cells and voxel centres follow the reading
 * stated in oracle/definition.py; compile with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float x, y, z;
    uint32_t rgba;
} orc_rec;

typedef struct {
    int64_t child;   /* index of the first of 8 children, -1 for a leaf */
    uint64_t path;
    uint32_t depth;
    uint32_t n, cap; /* points (leaf) or voxels (inner) */
    orc_rec* rec;
    uint32_t* key;
    uint32_t* grid;  /* R^3 occupancy bits, inner nodes only */
} orc_node;

typedef struct {
    float mn[3];
    float size, scale;
    uint32_t K, r, R, Dmax, T;
    orc_node* nodes;
    int64_t nnodes, capnodes;
    uint64_t total;
    uint64_t voxels_created_last; /* voxels created by the last insert call */
    int error;
} orc_tree;

static uint32_t orc_quant(float v, float mn, float scale, uint32_t K) {
    float u = (v - mn) * scale;
    if (!(u >= 0.0f)) return 0u;
    float f = floorf(u);
    float qmax = (float)((1u << K) - 1u);
    if (f > qmax) f = qmax;
    return (uint32_t)f;
}

static float orc_centre(uint32_t g, float mn, float size, uint32_t r, uint32_t d) {
    float h = ldexpf(size, -(int)(r + d));
    float gf = (float)g + 0.5f;
    float prod = gf * h;
    return mn + prod;
}

static int orc_push(orc_node* nd, const orc_rec* rc, uint32_t key) {
    if (nd->n == nd->cap) {
        uint32_t nc = nd->cap ? nd->cap * 2 : 16;
        orc_rec* r2 = (orc_rec*)realloc(nd->rec, (size_t)nc * sizeof(orc_rec));
        if (!r2) return -1;
        nd->rec = r2;
        uint32_t* k2 = (uint32_t*)realloc(nd->key, (size_t)nc * sizeof(uint32_t));
        if (!k2) return -1;
        nd->key = k2;
        nd->cap = nc;
    }
    nd->rec[nd->n] = *rc;
    nd->key[nd->n] = key;
    nd->n++;
    return 0;
}

static int64_t orc_new_children(orc_tree* t, int64_t parent) {
    if (t->nnodes + 8 > t->capnodes) {
        int64_t nc = t->capnodes ? t->capnodes * 2 : 64;
        while (nc < t->nnodes + 8) nc *= 2;
        orc_node* n2 = (orc_node*)realloc(t->nodes, (size_t)nc * sizeof(orc_node));
        if (!n2) return -1;
        t->nodes = n2;
        t->capnodes = nc;
    }
    int64_t first = t->nnodes;
    for (int o = 0; o < 8; ++o) {
        orc_node* c = &t->nodes[first + o];
        memset(c, 0, sizeof(*c));
        c->child = -1;
        c->path = t->nodes[parent].path * 8u + (uint64_t)o;
        c->depth = t->nodes[parent].depth + 1u;
    }
    t->nnodes += 8;
    return first;
}

static int orc_insert_from(orc_tree* t, int64_t ni, const orc_rec* rc, uint32_t key);

static int orc_split(orc_tree* t, int64_t ni) {
    orc_node* nd = &t->nodes[ni];
    orc_rec* old_rec = nd->rec;
    uint32_t* old_key = nd->key;
    uint32_t old_n = nd->n;
    nd->rec = NULL;
    nd->key = NULL;
    nd->n = nd->cap = 0;
    size_t cells = (size_t)t->R * t->R * t->R;
    size_t words = (cells + 31) / 32;
    nd->grid = (uint32_t*)calloc(words, sizeof(uint32_t));
    if (!nd->grid) return -1;
    int64_t first = orc_new_children(t, ni);
    if (first < 0) return -1;
    t->nodes[ni].child = first; /* nodes may have moved */
    for (uint32_t i = 0; i < old_n; ++i) {
        if (orc_insert_from(t, ni, &old_rec[i], old_key[i])) return -1;
    }
    free(old_rec);
    free(old_key);
    return 0;
}

static int orc_insert_from(orc_tree* t, int64_t ni, const orc_rec* rc, uint32_t key) {
    uint32_t q[3];
    q[0] = orc_quant(rc->x, t->mn[0], t->scale, t->K);
    q[1] = orc_quant(rc->y, t->mn[1], t->scale, t->K);
    q[2] = orc_quant(rc->z, t->mn[2], t->scale, t->K);
    for (;;) {
        orc_node* nd = &t->nodes[ni];
        uint32_t d = nd->depth;
        if (nd->child < 0) break;
        uint32_t shift = t->Dmax - d;
        uint32_t g[3], c[3];
        for (int a = 0; a < 3; ++a) {
            g[a] = q[a] >> shift;
            c[a] = g[a] & (t->R - 1u);
        }
        size_t cell = (size_t)c[0] + (size_t)t->R * ((size_t)c[1] + (size_t)t->R * c[2]);
        uint32_t bit = 1u << (cell & 31u);
        if (!(nd->grid[cell >> 5] & bit)) {
            nd->grid[cell >> 5] |= bit;
            orc_rec v;
            v.x = orc_centre(g[0], t->mn[0], t->size, t->r, d);
            v.y = orc_centre(g[1], t->mn[1], t->size, t->r, d);
            v.z = orc_centre(g[2], t->mn[2], t->size, t->r, d);
            v.rgba = rc->rgba;
            if (orc_push(nd, &v, key)) return -1;
            t->voxels_created_last++;
        }
        uint32_t b = t->K - 1u - d;
        uint32_t oct = ((q[0] >> b) & 1u) | (((q[1] >> b) & 1u) << 1) | (((q[2] >> b) & 1u) << 2);
        ni = nd->child + (int64_t)oct;
    }
    orc_node* leaf = &t->nodes[ni];
    if (orc_push(leaf, rc, key)) return -1;
    if (leaf->n > t->T && leaf->depth < t->Dmax) return orc_split(t, ni);
    return 0;
}

/* ---- exported API (called from oracle/incremental.py through ctypes) ---- */

orc_tree* orc_create(const float* root_min, float root_size, uint32_t leaf_capacity,
                     uint32_t grid_bits, uint32_t max_depth) {
    if (grid_bits > 8 || max_depth > 21 || grid_bits + max_depth > 24 || leaf_capacity < 1)
        return NULL;
    if (!(root_size > 0.0f) || isinf(root_size)) return NULL;
    orc_tree* t = (orc_tree*)calloc(1, sizeof(orc_tree));
    if (!t) return NULL;
    for (int a = 0; a < 3; ++a) t->mn[a] = root_min[a];
    t->size = root_size;
    t->r = grid_bits;
    t->R = 1u << grid_bits;
    t->Dmax = max_depth;
    t->K = max_depth + grid_bits;
    t->T = leaf_capacity;
    t->scale = (float)(1u << t->K) / root_size; /* float32 division */
    t->capnodes = 64;
    t->nodes = (orc_node*)calloc((size_t)t->capnodes, sizeof(orc_node));
    if (!t->nodes) {
        free(t);
        return NULL;
    }
    t->nnodes = 1;
    t->nodes[0].child = -1;
    t->nodes[0].path = 1;
    return t;
}

void orc_destroy(orc_tree* t) {
    if (!t) return;
    for (int64_t i = 0; i < t->nnodes; ++i) {
        free(t->nodes[i].rec);
        free(t->nodes[i].key);
        free(t->nodes[i].grid);
    }
    free(t->nodes);
    free(t);
}

/* Inserts n 16-byte records; keys continue the cumulative sequence.
   Returns 0, or -1 on allocation failure / key overflow (tree then unusable). */
int orc_insert(orc_tree* t, const orc_rec* pts, uint64_t n) {
    if (t->error) return -1;
    if (t->total + n > 0xFFFFFFFFull) {
        t->error = 1;
        return -1;
    }
    t->voxels_created_last = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (orc_insert_from(t, 0, &pts[i], (uint32_t)(t->total + i))) {
            t->error = 1;
            return -1;
        }
    }
    t->total += n;
    return 0;
}

/* Inserts only the points of a batch that fall in the region of the node
   with `path` (1 = root, parent * 8 + octant below; depth = number of
   octant digits, at most Dmax), each with the key it has in the whole
   sequence; keys of the skipped points are consumed all the same.

   By the recursive definition, a node's subtree depends only on the points
   of its region.  Fed with exactly those points, every ancestor of the node
   holds all of them, so when they number more than T the ancestors are
   inner, the node exists, and its subtree is the one the whole sequence
   gives (provided the node exists there too); with T or fewer the root
   stays a leaf holding them, which is the node's content in the whole tree
   when the node is a leaf there.  This lets single subtrees of clouds too
   large for one oracle run be checked one at a time.
   Returns 0, -1 on allocation failure / key overflow, -2 on a bad path. */
int orc_insert_region(orc_tree* t, const orc_rec* pts, uint64_t n, uint64_t path) {
    if (t->error) return -1;
    uint32_t d = 0;
    uint64_t digits[32];
    for (uint64_t p = path; p > 1; p >>= 3) {
        if (d >= t->Dmax || d >= 32) return -2;
        digits[d++] = p & 7u;
    }
    if (path < 1) return -2;
    uint64_t p = path;
    while (p > 7) p >>= 3;
    if (p != 1) return -2;
    if (t->total + n > 0xFFFFFFFFull) {
        t->error = 1;
        return -1;
    }
    t->voxels_created_last = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const orc_rec* rc = &pts[i];
        uint32_t q[3];
        q[0] = orc_quant(rc->x, t->mn[0], t->scale, t->K);
        q[1] = orc_quant(rc->y, t->mn[1], t->scale, t->K);
        q[2] = orc_quant(rc->z, t->mn[2], t->scale, t->K);
        int inside = 1;
        for (uint32_t j = 0; j < d && inside; ++j) {
            uint32_t b = t->K - 1u - j;
            uint32_t oct = ((q[0] >> b) & 1u) | (((q[1] >> b) & 1u) << 1) | (((q[2] >> b) & 1u) << 2);
            inside = oct == digits[d - 1 - j];
        }
        if (!inside) continue;
        if (orc_insert_from(t, 0, rc, (uint32_t)(t->total + i))) {
            t->error = 1;
            return -1;
        }
    }
    t->total += n;
    return 0;
}

uint64_t orc_voxels_created_last(const orc_tree* t) { return t->voxels_created_last; }

/* Sizes of the canonical form. */
void orc_sizes(const orc_tree* t, uint64_t* num_nodes, uint64_t* num_records) {
    uint64_t rec = 0;
    for (int64_t i = 0; i < t->nnodes; ++i) rec += t->nodes[i].n;
    *num_nodes = (uint64_t)t->nnodes;
    *num_records = rec;
}

typedef struct {
    uint64_t path;
    uint64_t first;
    uint32_t count;
    uint8_t depth;
    uint8_t is_leaf;
    uint16_t reserved;
} orc_node_rec;

/* Preorder export into caller buffers sized by orc_sizes. */
int orc_export(const orc_tree* t, orc_node_rec* out_nodes, orc_rec* out_rec, uint32_t* out_keys) {
    int64_t* stack = (int64_t*)malloc((size_t)(t->nnodes + 8) * sizeof(int64_t));
    if (!stack) return -1;
    int64_t sp = 0, w = 0;
    uint64_t written = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        int64_t ni = stack[--sp];
        const orc_node* nd = &t->nodes[ni];
        orc_node_rec* o = &out_nodes[w++];
        o->path = nd->path;
        o->first = written;
        o->count = nd->n;
        o->depth = (uint8_t)nd->depth;
        o->is_leaf = nd->child < 0 ? 1 : 0;
        o->reserved = 0;
        if (nd->n) {
            memcpy(out_rec + written, nd->rec, (size_t)nd->n * sizeof(orc_rec));
            memcpy(out_keys + written, nd->key, (size_t)nd->n * sizeof(uint32_t));
        }
        written += nd->n;
        if (nd->child >= 0)
            for (int o2 = 7; o2 >= 0; --o2) stack[sp++] = nd->child + o2;
    }
    free(stack);
    return 0;
}
