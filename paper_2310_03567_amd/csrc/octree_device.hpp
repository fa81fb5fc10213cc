// Device-side layout of one octree and the wave-level helpers its kernels use.
//
// Everything an insertion pass touches lives in device memory allocated at
// creation; the kernels receive it as one by-value `DevTree`.
//
// Node table (structure of arrays, capacity max_nodes, root = node 0):
//   child[n]    first of the node's 8 consecutive children, 0 for a leaf
//               (node 0 is the root and never a child, so 0 is free)
//   count[n]    points of a leaf / voxels of an inner node; during the store
//               passes it is also the slot counter (section "Storing Points
//               and Voxels": numPoints / numVoxels)
//   cnt[n]      first-round counter (section "Expanding the Octree": point
//               counter), zero outside a pass
//   hslot[n]    histogram slot while the leaf is a pending root, else kNone
//   geo[n]      {origin x, origin y, origin z, depth}, origin in integer
//               coordinates (units of 2^-K of the root size)
//   grid[n]     arena block of the R^3 occupancy bitmap (inner nodes)
//   tab[n], tabcap[n], nchunks[n]
//               arena block, capacity and length of the node's chunk table:
//               the ids of its chunks in list order, so chunk slot/C is one
//               load away (the chunks are also linked, see below)
//   newv[n]     voxels claimed for the node in the current pass
//
// Node directory: for each depth d <= dir_depth (at most kDirMaxDepth) a
// dense table of 8^d entries indexed by the Morton code of the node's d-bit
// integer position; entry = node id, with kDirInner set once the node has
// children, or kNone where no node exists at that depth.  A point's path down
// to dir_depth is then dir_depth + 1 independent loads instead of a chain of
// dependent child-pointer loads; below dir_depth the walk follows child[].
//
// Persistent buffer ("arena", section "Persistent Buffer"): one allocation
// carved into 256-byte blocks by an atomic bump counter; chunks, occupancy
// grids and chunk tables are addressed by their first block (u32).  A chunk
// of capacity C holds C 16-byte records, then C u32 keys, then the u32 block
// id of the next chunk of the same node (0xFFFFFFFF ends the list), the
// linked list of section "Chunks and the Chunk Pool".  Freed chunks go to a
// stack of block ids (the chunk pool) and are reused before the bump counter.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace simlod {

typedef uint16_t u16;
typedef uint32_t u32;
typedef uint64_t u64;
typedef int32_t i32;

constexpr u32 kNone = 0xFFFFFFFFu;
constexpr u64 kEmptyTag = ~0ull;
constexpr u32 kBlockBytes = 256;
constexpr int kMaxRounds = 24;  // >= max_depth + 1
constexpr u32 kStripes = 8;     // claim-list stripes (one per XCD)
constexpr u32 kDirMaxDepth = 7;         // deepest level of the node directory
constexpr u32 kDirInner = 0x80000000u;  // directory entry flag: the node is inner

// Histogram of a pending root: counts of its virtual descendants at
// kHistLevels levels below it, 8^j counters at level j (j = 1..kHistLevels),
// indexed by the Morton code of the relative path.
constexpr u32 kHistLevels = 4;
constexpr u32 kHistEntries = 8u + 64u + 512u + 4096u;
__host__ __device__ __forceinline__ u32 hist_level_offset(u32 j) {  // (8^j - 8) / 7
    return ((1u << (3u * j)) - 8u) / 7u;
}

// Passes of one octree with at least this many batch points process the
// batch grouped by spatial bucket (the Morton index of a point's cell at
// kBucketBits bits per axis; buckets in Morton order, each bucket's points
// in the order their windows reserve places): the points of a region then
// share tiles, and neighbouring regions neighbouring tiles, so their voxel
// claims meet in one workgroup's LDS table and their claim-table lines and
// grid words in one L2, where in scan order (points of many regions
// interleaved) they reach global memory from many workgroups.  The order
// does not change the octree: every result is fixed by the points' keys.
constexpr u64 kGroupMinItems = 4ull << 20;
constexpr u32 kBucketBits = 8;  // per axis
constexpr u32 kBuckets = 1u << (3u * kBucketBits);
constexpr u32 kBucketChunk = 4096;  // buckets per scan chunk

// Device-resident counters of one octree.
struct Counters {
    u32 node_count;
    u32 status;          // sticky SIMLOD_OVF_* bits
    u32 arena_top;       // blocks handed out
    i32 pool_top;        // chunk ids on the pool stack (negative = empty)
    u32 spill_count;     // points moved to the spill buffer this pass
    u32 spill_jobs;      // leaves spilled this pass; with spill_count one
                         // 64-bit counter, so jobs are listed in buffer order
    u32 final_count;     // leaves finalized this pass
    u32 vtouched_count;  // inner nodes that claimed voxels this pass
    u32 touched_count;   // leaves counted in the first round
    u32 pad0;
    u32 claim_count[kStripes];  // voxels claimed this pass, per stripe
    u32 pending_count[2];       // pending roots listed by round k in [k & 1]
    u32 hist_top;        // histogram slots handed out this pass
    u32 build_rounds;    // histogram rounds that built something this pass
    u32 last_rounds, last_spilled, last_new_voxels;
    u32 max_rounds, max_spilled, max_new_voxels;
    u32 pad;
    u64 sum_spilled, sum_new_voxels, sum_rounds;
};

static_assert(offsetof(Counters, spill_count) % 8 == 0 &&
                  offsetof(Counters, spill_jobs) == offsetof(Counters, spill_count) + 4,
              "spill_count and spill_jobs form one 64-bit counter");
static_assert(offsetof(Counters, sum_spilled) % 8 == 0, "64-bit sums aligned");

// In device code the octree's tables are declared in the global address
// space: loads, stores and atomics through them then compile to global
// instructions rather than flat ones, which the hardware counts together
// with LDS operations (a wait for an LDS result would also wait for every
// outstanding memory access).  Host code sees plain pointers of the same
// size.
//
// The DevTree itself is written by the host only, never while a pass runs:
// in device code it is read through the constant address space, so that its
// fields load with scalar instructions into scalar registers.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using GPtr = __attribute__((address_space(1))) T*;
template <class T>
using CPtr = __attribute__((address_space(4))) T*;
#else
template <class T>
using GPtr = T*;
template <class T>
using CPtr = T*;
#endif

struct DevTree {
    // node table
    GPtr<u32> child;
    GPtr<u32> count;
    GPtr<u32> cnt;
    GPtr<u32> hslot;          // histogram slot of a pending root, kNone otherwise
    GPtr<uint4> geo;
    GPtr<u32> grid;
    GPtr<u32> tab;
    GPtr<u32> tabcap;
    GPtr<u32> nchunks;
    GPtr<u32> newv;
    u32 max_nodes;
    GPtr<u32> dir;
    u32 dir_depth;
    GPtr<Counters> ctr;
    // persistent buffer and chunk pool
    GPtr<uint8_t> arena;
    u32 arena_blocks;
    GPtr<u32> pool;
    u32 pool_cap;
    // per-pass work buffers
    GPtr<uint4> spill_rec;
    GPtr<u32> spill_key;
    GPtr<uint2> spill_job;    // {leaf, first spill index} of each spilled leaf
    u32 spill_cap;
    GPtr<u32> touched;        // leaves counted in the first round
    GPtr<uint2> final_list;   // {leaf, points added}
    GPtr<u32> vtouched;       // inner nodes with new voxels
    GPtr<u32> pending[2];     // pending roots (leaves that must split)
    GPtr<u32> hist;           // hist_cap slots of kHistEntries counters
    u32 hist_cap;
    GPtr<uint8_t> amask[2];   // per work item: counted in the previous round
    GPtr<u32> item_leaf;      // per batch item: its leaf in the first round
    // Large passes of one octree (kGroupMinItems points or more) process the
    // batch grouped by spatial bucket; null when max_batch is below that size.
    GPtr<uint4> grp_rec;      // batch records in the grouped order
    GPtr<u32> grp_index;      // their indices in the batch (key = base_key + index)
    GPtr<u32> grp_leaf;       // their first-round leaves
    GPtr<u32> bcnt;           // per bucket: points counted in the first round
                              // (cleared by the scan that reads them)
    GPtr<u32> bnext;          // per bucket: next place of its group (within
                              // its scan chunk; + bsum[chunk])
    GPtr<u32> bsum;           // per scan chunk of buckets: first place
    u32 active_cap;
    GPtr<u64> hent;           // voxel claim table, 16-byte entries, 8 to a bucket:
                         // [2h] = claim word (tag << 32 | key), min-reduced,
                         // [2h + 1] = (key << 32 | rgba) of spilled claimants,
                         // min-reduced (see claim_home)
    u32 hmask;
    u32 hash_bits;       // log2 of the claim table's entries
    u32 tag_bits;        // bits of a cell's identity node << 3r | cell
    GPtr<u32> claims;         // claim-table slots claimed this pass, kStripes x claim_cap
    u32 claim_cap;
    // geometry and parameters
    float mn[3];
    float size;
    float scale;
    u32 K, r, R, Dmax, T, C;
    u64 c_magic;         // ceil(2^64 / C), 0 for C = 1 (see div_C)
    u32 chunk_blocks, grid_blocks, grid_words;
};

// One octree's share of an insertion pass over a group of octrees: its
// device-resident DevTree, its batch (device memory, 16-byte records) and the
// key of the batch's first point.  A single-octree pass is a group of one.
struct Member {
    CPtr<const DevTree> tree;
    GPtr<const uint4> batch;
    u32 n;
    u32 base_key;
};

// Host side: a member from plain device pointers (C-style casts into the
// device address space where the device pass declares one).
inline Member make_member(const DevTree* tree, const uint4* batch, u32 n, u32 base_key) {
    return Member{(CPtr<const DevTree>)tree, (GPtr<const uint4>)batch, n, base_key};
}

constexpr u32 kMaxMembers = 128;  // octrees per group pass (<= two wavefronts)

// Argument of a pass's first kernel: the members inline (so that a replayed
// graph only needs this one node's arguments changed) and the device table
// it copies them to for the pass's later kernels.
struct GroupArgs {
    Member* table;
    u32 count;
    u32 pad;
    Member m[kMaxMembers];
};

__device__ __forceinline__ u64* claim_word_at(const DevTree& t, u32 h) {
    return t.hent + 2u * (u64)h;
}
__device__ __forceinline__ u64* claim_spill_at(const DevTree& t, u32 h) {
    return t.hent + 2u * (u64)h + 1u;
}

// Claim table addressing.  A cell's identity T = node << 3r | cell has
// tag_bits bits.  The table is made of buckets of 8 entries (one 128-byte
// line): the 8 cells of a 2x2x2 block of a node's grid share a bucket, each
// at its own position in it, so that the claims of neighbouring points
// (which meet neighbouring cells) share L2 lines.  T splits into the block's
// identity G (tag_bits - 3 bits) and the cell's position in the block.  An
// invertible mix of G's bits (multiply by an odd constant mod 2^n, xor-shift
// by at least n/2, multiply again) gives the home bucket (its top bits) and
// a remainder (the other bits, at most kRemBits).  A cell probes its own
// position in the home bucket and the buckets after it; an entry then holds
// (remainder << kDistBits | probe distance) as its 32-bit tag, which
// together with the entry's index determines T.  So one 64-bit word
// (tag << 32 | key) carries both the cell and the smallest key claimed for
// it, and a claim is one atomic.  (r = 0, one cell per node: buckets of 1.)
constexpr u32 kDistBits = 7;  // linear probing up to 127 buckets past home
constexpr u32 kRemBits = 24;  // the tag stays below 2^31, never the empty word's
constexpr u64 kMixA = 0x9E3779B97F4A7C15ull;
constexpr u64 kMixAinv = 0xF1DE83E19937733Dull;  // kMixA * kMixAinv = 1 mod 2^64
constexpr u64 kEmptyWord = ~0ull;

__device__ __forceinline__ u64 low_bits(u32 n) { return n >= 64u ? ~0ull : (1ull << n) - 1ull; }

__device__ __forceinline__ u64 tag_mix(u64 x, u32 n) {
    const u64 m = low_bits(n);
    x = (x * kMixA) & m;
    x ^= x >> ((n + 1u) / 2u);
    return (x * kMixA) & m;
}

__device__ __forceinline__ u64 tag_unmix(u64 x, u32 n) {
    const u64 m = low_bits(n);
    x = (x * kMixAinv) & m;
    x ^= x >> ((n + 1u) / 2u);  // an involution when the shift is >= n/2
    return (x * kMixAinv) & m;
}

__device__ __forceinline__ u32 rem_bits_of(const DevTree& t) {
    return t.tag_bits > t.hash_bits ? t.tag_bits - t.hash_bits : 0u;
}

// log2 of the entries of a bucket
__device__ __forceinline__ u32 claim_sub_bits(const DevTree& t) { return t.r ? 3u : 0u; }

// Identity T -> (block identity G, position of the cell in its 2x2x2 block).
__device__ __forceinline__ void claim_split(const DevTree& t, u64 T, u64& G, u32& sub) {
    const u32 r = t.r;
    if (!r) {
        G = T;
        sub = 0u;
        return;
    }
    const u32 m = t.R - 1u;
    const u32 cell = (u32)(T & low_bits(3u * r));
    const u64 node = T >> (3u * r);
    const u32 cx = cell & m, cy = (cell >> r) & m, cz = cell >> (2u * r);
    sub = (cx & 1u) | ((cy & 1u) << 1) | ((cz & 1u) << 2);
    const u32 q = r - 1u;
    G = (node << (3u * q)) | (u64)((cx >> 1) | ((cy >> 1) << q) | ((cz >> 1) << (2u * q)));
}

// Inverse of claim_split.
__device__ __forceinline__ u64 claim_join(const DevTree& t, u64 G, u32 sub) {
    const u32 r = t.r;
    if (!r) return G;
    const u32 q = r - 1u;
    const u32 qm = (1u << q) - 1u;
    const u32 blk = (u32)(G & low_bits(3u * q));
    const u64 node = G >> (3u * q);
    const u32 cx = ((blk & qm) << 1) | (sub & 1u);
    const u32 cy = (((blk >> q) & qm) << 1) | ((sub >> 1) & 1u);
    const u32 cz = ((blk >> (2u * q)) << 1) | (sub >> 2);
    return (node << (3u * r)) | (u64)(cx | (cy << r) | (cz << (2u * r)));
}

// Home entry (the cell's position in its home bucket) and remainder of
// identity T.
__device__ __forceinline__ void claim_home(const DevTree& t, u64 T, u32& home, u32& rem) {
    u64 G;
    u32 sub;
    claim_split(t, T, G, sub);
    const u32 sb = claim_sub_bits(t);
    const u64 m = tag_mix(G, t.tag_bits - sb);
    const u32 rb = rem_bits_of(t);
    home = (((u32)(m >> rb) & (t.hmask >> sb)) << sb) | sub;
    rem = (u32)(m & low_bits(rb));
}

// Entry at probe distance d (buckets) from home entry `home`.
__device__ __forceinline__ u32 claim_step(const DevTree& t, u32 home, u32 d) {
    return (home + (d << claim_sub_bits(t))) & t.hmask;
}

// Identity T of the cell whose claim word at entry h carries tag tg.
__device__ __forceinline__ u64 claim_identity(const DevTree& t, u32 h, u32 tg) {
    const u32 d = tg & ((1u << kDistBits) - 1u);
    const u32 sb = claim_sub_bits(t);
    const u64 hb = (u64)(((h - (d << sb)) & t.hmask) >> sb);
    const u32 rb = rem_bits_of(t);
    const u64 G = tag_unmix((hb << rb) | (u64)(tg >> kDistBits), t.tag_bits - sb);
    return claim_join(t, G, h & ((1u << sb) - 1u));
}

__device__ __forceinline__ uint8_t* block_ptr(const DevTree& t, u32 blk) {
    return t.arena + (u64)blk * kBlockBytes;
}
__device__ __forceinline__ uint4* chunk_recs(const DevTree& t, u32 blk) {
    return reinterpret_cast<uint4*>(block_ptr(t, blk));
}
__device__ __forceinline__ u32* chunk_keys(const DevTree& t, u32 blk) {
    return reinterpret_cast<u32*>(block_ptr(t, blk) + (u64)t.C * 16u);
}
__device__ __forceinline__ u32* chunk_next(const DevTree& t, u32 blk) {
    return reinterpret_cast<u32*>(block_ptr(t, blk) + (u64)t.C * 20u);
}
__device__ __forceinline__ u32* table_of(const DevTree& t, u32 node) {
    return reinterpret_cast<u32*>(block_ptr(t, t.tab[node]));
}
__device__ __forceinline__ u32* grid_of(const DevTree& t, u32 node) {
    return reinterpret_cast<u32*>(block_ptr(t, t.grid[node]));
}

// n / C for any n < 2^32 by one 64-bit multiply-high instead of an integer
// division: with m = ceil(2^64 / C), n * m / 2^64 exceeds n / C by less than
// 2^-32, too little to reach the next integer.
__device__ __forceinline__ u32 div_C(const DevTree& t, u32 n) {
    if (t.c_magic == 0ull) return n;  // C = 1
    return (u32)__umul64hi((u64)n, t.c_magic);
}

// Integer coordinate along one axis.  The subtraction and the product are
// separately rounded (explicit _rn intrinsics, so contraction can never fuse
// them); negative and NaN map to 0, everything at or beyond the far face to
// 2^K - 1.
__device__ __forceinline__ u32 quantize(float v, float mn, float scale, u32 K) {
    float u = __fmul_rn(__fsub_rn(v, mn), scale);
    if (!(u >= 0.0f)) return 0u;
    float f = floorf(u);
    float qmax = (float)((1u << K) - 1u);
    f = fminf(f, qmax);
    return (u32)f;
}

// Centre of global cell g at depth d along one axis:
// fl32(mn + fl32(fl32(g + 0.5) * h_d)), h_d = size * 2^-(r + d).
__device__ __forceinline__ float cell_centre(u32 g, float mn, float size, u32 r, u32 d) {
    float h = ldexpf(size, -(int)(r + d));
    return __fadd_rn(mn, __fmul_rn(__fadd_rn((float)g, 0.5f), h));
}

// Gathers every third bit (bit 3i -> bit i), the inverse of spread3.
__host__ __device__ __forceinline__ u32 compact3(u32 x) {
    x &= 0x09249249u;
    x = (x ^ (x >> 2)) & 0x030C30C3u;
    x = (x ^ (x >> 4)) & 0x0300F00Fu;
    x = (x ^ (x >> 8)) & 0x030000FFu;
    x = (x ^ (x >> 16)) & 0x000003FFu;
    return x;
}

// Interleaves the low 10 bits of x into every third bit (bit i -> bit 3i).
__host__ __device__ __forceinline__ u32 spread3(u32 x) {
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__host__ __device__ __forceinline__ u32 dir_offset(u32 d) { return ((1u << (3u * d)) - 1u) / 7u; }

// Morton index, at depth d, of the cell holding integer position (x, y, z):
// bit 3i = x, 3i+1 = y, 3i+2 = z, so index(d + 1) = index(d) * 8 + octant.
__device__ __forceinline__ u32 dir_index(u32 K, u32 d, u32 qx, u32 qy, u32 qz) {
    const u32 s = K - d;
    return d ? (spread3(qx >> s) | (spread3(qy >> s) << 1) | (spread3(qz >> s) << 2)) : 0u;
}

__device__ __forceinline__ u32 octant_of(u32 qx, u32 qy, u32 qz, u32 bit) {
    return ((qx >> bit) & 1u) | (((qy >> bit) & 1u) << 1) | (((qz >> bit) & 1u) << 2);
}

__device__ __forceinline__ void set_status(const DevTree& t, u32 bits) {
    atomicOr(&t.ctr->status, bits);
}

__device__ __forceinline__ u32 lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 lanes_below(u32 lane) {
    return lane == 0 ? 0ull : (~0ull >> (64u - lane));
}

// Wave-aggregated append: every lane with `pred` gets a distinct slot of
// *counter, with one atomic per wave.  Must be reached by the whole wave.
__device__ __forceinline__ u32 wave_append(u32* counter, bool pred) {
    u64 m = __ballot(pred);
    if (m == 0ull) return 0u;
    u32 lane = lane_id();
    int leader = __ffsll((long long)m) - 1;
    u32 base = 0;
    if ((int)lane == leader) base = atomicAdd(counter, (u32)__popcll(m));
    base = __shfl(base, leader);
    return base + (u32)__popcll(m & lanes_below(lane));
}

// Run-length aggregation over consecutive lanes holding equal `id`
// (ids of kNone are excluded).  Returns for each lane its run head and the
// run length at the head.  Must be reached by the whole wave.
struct Run {
    int head;
    u32 len;   // valid at the head lane
    u32 rank;  // lane - head
};
__device__ __forceinline__ Run lane_runs(u32 id) {
    u32 lane = lane_id();
    u32 prev = __shfl_up(id, 1);
    bool is_head = (lane == 0) || (prev != id);
    u64 heads = __ballot(is_head);
    u64 upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    int head = 63 - __clzll((long long)(heads & upto));
    u64 above = (lane == 63) ? 0ull : (heads >> (lane + 1));
    u32 next = above ? (lane + 1 + (u32)__ffsll((long long)above) - 1) : 64u;
    Run r;
    r.head = head;
    r.len = next - lane;
    r.rank = lane - (u32)head;
    return r;
}

// 64-bit finalizer of Austin Appleby's MurmurHash3 (fmix64, public domain):
// its published shift and multiplier constants.
__device__ __forceinline__ u64 mix64(u64 x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

}  // namespace simlod
