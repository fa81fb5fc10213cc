// gfx950 kernels of one insertion pass (section "Incrementally Updating the
// Octree").  A pass over a batch of n points runs, on one stream:
//
//   k_count_leaves, k_split_leaves   first expansion round: count the batch
//       per leaf (and, on grouped passes, per spatial bucket); a leaf whose stored plus new points exceed T (above Dmax)
//       becomes a pending root: it is listed as a spill job (its stored
//       points are copied to the spill buffer in the next kernel) and it gets
//       a histogram slot (subsection "Expanding the Octree")
//   k_bucket_scan, k_bucket_sums, k_group_batch   passes of one octree and
//                        4M points or more: the batch copied into the order
//                        grouped by spatial bucket, which the later kernels
//                        read (same octree, better locality)
//   k_count_hist, k_build   round 2: every point in a pending root adds to
//       the root's histogram of its descendants kHistLevels levels down (and
//       spilled points are copied out of their leaf's chunks); the build
//       kernel then creates that whole part of the subtree at once, and
//       descendants at the histogram's last level that still hold more than
//       T points become the next round's pending roots.  R = 1 + ceil(Dmax /
//       kHistLevels) rounds always suffice.
//   k_rounds_alloc       rounds 3..R, which usually find nothing to do, then
//                        chunks for the leaves' new points (subsection
//                        "Allocating Chunks")
//   k_sample_store       one traversal per point: voxel claims at every
//                        inner node on the path (subsection "Voxel Sampling")
//                        and the point's store into its leaf (subsection
//                        "Storing Points and Voxels")
//   k_alloc(voxels)      chunks for the inner nodes' new voxels
//   k_store_voxels       voxel records from the claim backlog, after the
//                        pass's bookkeeping
//   k_finish             group passes only: members' status words
//
// Occupancy grids need no clearing in a pass: they are carved from fresh
// blocks of the persistent buffer, which is clear up to its bump pointer.
//
// The paper repeats count/split one level at a time; counting several levels
// per round gives the same octree (a node is inner iff its region holds more
// than T points, whatever order the levels are decided in) with far fewer
// passes over the batch and kernel launches.
//
// The work list W of a pass is the spill buffer followed by the batch:
// index i < S names spilled point i (with the key it was stored with),
// index i >= S names batch point i - S with key base_key + i - S.
//
// All cross-workgroup communication inside one kernel goes through atomics;
// anything else written in one kernel is read in a later one.  Same-address
// device atomics serialize (about 11 ns each on MI355X), so counters that
// many workgroups update are aggregated in LDS first.
#include "octree_device.hpp"
#include "simlod.h"
#include "launch.hpp"

#include <algorithm>

namespace simlod {

constexpr u32 kWG = 256;  // 4 wavefronts; the LDS tables and scans assume it
static_assert(kWG == 256, "workgroup scans and LDS tables are laid out for 4 wavefronts");
constexpr u32 kLdsBits = 11;
constexpr u32 kLds = 1u << kLdsBits;
constexpr u32 kHistKey = 0x80000000u;  // LDS key flag: a histogram counter

// Renumbers the first g workgroups of the grid so that each of the 8 XCDs
// (which receive workgroups round-robin) walks a contiguous range of tiles:
// neighbouring points, and therefore the same nodes and grid words, stay in
// one XCD's L2.
__device__ __forceinline__ u32 xcd_block(u32 g) {
    u32 b = blockIdx.x;
    if (g & 7u) return b;
    return (b & 7u) * (g >> 3) + (b >> 3);
}

// Work item i: a spilled point (i < S) or a batch point.  grouped: the batch
// part of the list is in the grouped order (grp_rec, grp_index).
__device__ __forceinline__ void fetch_work(const DevTree& t, const uint4* batch, bool grouped,
                                           u32 S, u32 base_key, u32 i, uint4& rec, u32& key) {
    if (i < S) {
        rec = t.spill_rec[i];
        key = t.spill_key[i];
    } else if (grouped) {
        rec = t.grp_rec[i - S];
        key = base_key + t.grp_index[i - S];
    } else {
        rec = batch[i - S];
        key = base_key + (i - S);
    }
}

__device__ __forceinline__ void quantize3(const DevTree& t, const uint4& rec, u32& qx, u32& qy,
                                          u32& qz) {
    qx = quantize(__uint_as_float(rec.x), t.mn[0], t.scale, t.K);
    qy = quantize(__uint_as_float(rec.y), t.mn[1], t.scale, t.K);
    qz = quantize(__uint_as_float(rec.z), t.mn[2], t.scale, t.K);
}

__device__ __forceinline__ u32 cell_lin(u32 qx, u32 qy, u32 qz, u32 shift, u32 r, u32 rmask) {
    return ((qx >> shift) & rmask) | (((qy >> shift) & rmask) << r) |
           (((qz >> shift) & rmask) << (2u * r));
}

// The leaf of integer position q from its node directory entries e (depths
// 0..dir_depth); below the directory the walk continues through child[]: the
// child of a node at depth d takes bit K-1-d of each coordinate (x bit 0,
// y bit 1, z bit 2 of the octant).  Sets the leaf's depth.
__device__ __forceinline__ u32 leaf_below(const DevTree& t, const u32 (&e)[kDirMaxDepth + 1],
                                          u32 m, u32 qx, u32 qy, u32 qz, u32& depth) {
    const u32 D = t.dir_depth;
#pragma unroll
    for (u32 d = 0; d <= kDirMaxDepth; ++d) {
        if (d <= D && !(e[d] & kDirInner)) {  // a leaf at depth d
            depth = d;
            return e[d];
        }
        if (d <= D && e[d] == kNone) {  // inconsistent directory
            set_status(t, SIMLOD_OVF_INTERNAL);
            depth = 0;
            return 0u;
        }
    }
    // inner at every directory depth: e[D] again, from the directory (an
    // index into e that is not a constant would place e in scratch memory)
    u32 node = t.dir[dir_offset(D) + m] & ~kDirInner;
    u32 bit = t.K - 1u - D;
    u32 c = t.child[node];
    u32 d = D;
    for (; c != 0u && d < t.Dmax; ++d) {  // children exist only above Dmax
        node = c + octant_of(qx, qy, qz, bit);
        --bit;
        c = t.child[node];
    }
    depth = d;
    return node;
}

// Root-to-leaf walk: the directory entries in one round of independent loads,
// then leaf_below.
__device__ __forceinline__ u32 find_leaf(const DevTree& t, u32 qx, u32 qy, u32 qz, u32& depth) {
    const u32 D = t.dir_depth;
    const u32 m = dir_index(t.K, D, qx, qy, qz);
    u32 e[kDirMaxDepth + 1];
#pragma unroll
    for (u32 d = 0; d <= kDirMaxDepth; ++d)
        e[d] = d <= D ? t.dir[dir_offset(d) + (m >> (3u * (D - d)))] : kNone;
    return leaf_below(t, e, m, qx, qy, qz, depth);
}

// leaf_below without the depth.
__device__ __forceinline__ u32 leaf_from_entries(const DevTree& t, const u32 (&e)[kDirMaxDepth + 1],
                                                 u32 m, u32 qx, u32 qy, u32 qz) {
    u32 depth;
    return leaf_below(t, e, m, qx, qy, qz, depth);
}

// Workgroup-uniform early exit.  skip_if_zero (may be null): also exit when
// that counter is zero.  The status word can change while a kernel runs, so
// one thread reads and the decision is broadcast through LDS before any
// barrier is reached.
__device__ __forceinline__ bool wg_skip(const Counters* ctr, const u32* skip_if_zero) {
    __shared__ u32 s_skip;
    if (threadIdx.x == 0)
        s_skip = (ctr->status != 0u || (skip_if_zero && *skip_if_zero == 0u)) ? 1u : 0u;
    __syncthreads();
    return s_skip != 0u;
}

// ------------------------------------------------------ LDS aggregation
// Open-addressing table on u32 keys; returns the entry, or kNone after
// max_probe occupied entries (the caller then goes to global memory).  A
// miss in a nearly full table must stay cheap, so tables that can fill use
// a short probe limit; `fill` (optional) counts the entries created.
__device__ __forceinline__ u32 lds_find_or_insert(u32* keys, u32 bits, u32 key,
                                                  u32 max_probe = 0xFFFFFFFFu,
                                                  u32* fill = nullptr) {
    const u32 size = 1u << bits;
    const u32 probes = min(size, max_probe);
    u32 h = (key * 0x9E3779B1u) >> (32u - bits);
    for (u32 p = 0; p < probes; ++p) {
        const u32 k = atomicCAS(&keys[h], kNone, key);
        if (k == kNone && fill) atomicAdd(fill, 1u);
        if (k == kNone || k == key) return h;
        h = (h + 1u) & (size - 1u);
    }
    return kNone;
}

constexpr u32 kCountProbe = 32;             // probe limit of the counting tables
constexpr u32 kCountFlushAt = kLds / 2u;    // entries that trigger a flush
constexpr u32 kBucketFlushAt = kLds * 3u / 4u;  // the same for the bucket table

// Adds c to a leaf's first-round counter; the first addition lists the leaf.
__device__ __forceinline__ void count_leaf_global(const DevTree& t, u32 node, u32 c) {
    if (atomicAdd(&t.cnt[node], c) == 0u) {
        const u32 p = atomicAdd(&t.ctr->touched_count, 1u);
        if (p < t.max_nodes)
            t.touched[p] = node;
        else
            set_status(t, SIMLOD_OVF_WORK);
    }
}

// Flushes one LDS-aggregated count: a leaf counter or a histogram counter.
__device__ __forceinline__ void flush_count(const DevTree& t, u32 key, u32 c) {
    if (key & kHistKey)
        atomicAdd(&t.hist[key & ~kHistKey], c);
    else
        count_leaf_global(t, key, c);
}

// Called by the whole workgroup after each tile of a counting kernel: once
// the LDS table holds kCountFlushAt entries, or when the next tile belongs
// to another octree of the group (or there is none), its counts go to global
// memory and it starts empty, so inserts keep finding free entries within
// the probe limit however many distinct keys the workgroup meets.
__device__ __forceinline__ void count_table_tile_end(const DevTree& t, u32* lkey, u32* lval,
                                                     u32* fill, bool force) {
    __syncthreads();
    const bool flush = force || *fill >= kCountFlushAt;
    __syncthreads();  // every thread has read `fill` before it changes
    if (!flush) return;
    for (u32 e = threadIdx.x; e < kLds; e += kWG) {
        if (lkey[e] != kNone) {
            flush_count(t, lkey[e], lval[e]);
            lkey[e] = kNone;
            lval[e] = 0u;
        }
    }
    if (threadIdx.x == 0) *fill = 0u;
    __syncthreads();
}

// ------------------------------------------------------ group plumbing
// Every kernel of a pass works on a group of octrees (a single insertion is a
// group of one).  Its work space is the concatenation of the members' units
// (tiles of kWG work items, or list entries); a unit never spans two members,
// so the member, and with it the DevTree, is uniform over a workgroup's tile
// or a wavefront's entry.

// s_pre[c] = first unit of member c, s_pre[count] = total, from units(c) of
// each member; returns the total.  Whole workgroup; count <= kMaxMembers.
template <typename F>
__device__ __forceinline__ u32 member_prefix(u32 count, u32* s_pre, F units) {
    static_assert(kMaxMembers <= 2u * 64u && kMaxMembers <= kWG, "two wavefronts scan");
    const u32 tid = threadIdx.x;
    const u32 lane = lane_id();
    u32 v = tid < count ? units(tid) : 0u;
#pragma unroll
    for (u32 o = 1; o < 64u; o <<= 1) {  // inclusive scan within the wavefront
        const u32 y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    if (tid < kMaxMembers) s_pre[tid + 1u] = v;
    __syncthreads();
    if (tid >= 64u && tid < kMaxMembers) s_pre[tid + 1u] += s_pre[64];
    if (tid == 0) s_pre[0] = 0u;
    __syncthreads();
    return s_pre[count];
}

// The member whose units contain x (s_pre non-decreasing, x < s_pre[count]),
// made scalar: callers pass a workgroup- or wavefront-uniform x.
__device__ __forceinline__ u32 member_of(const u32* s_pre, u32 count, u32 x) {
    u32 lo = 0u, hi = count;  // s_pre[lo] <= x < s_pre[hi]
    while (hi - lo > 1u) {
        const u32 mid = (lo + hi) >> 1;
        if (s_pre[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Tiles are visited in runs of kRunTiles consecutive tiles, dealt to the
// workgroups in turn (XCD-aware): a workgroup meets its tiles in increasing
// order, neighbouring tiles share nodes and cells, and dense bursts still
// spread over all workgroups.  next_tile(tile) is the workgroup's next tile
// after `tile`, or kNone.  nwg: the workgroups taking part (the first nwg).
constexpr u32 kRunTiles = 4;

__device__ __forceinline__ u32 first_tile(u32 nwg) { return xcd_block(nwg) * kRunTiles; }

__device__ __forceinline__ u32 next_tile(u32 tile, u32 ntiles, u32 nwg) {
    const u32 nx = (tile + 1u) % kRunTiles ? tile + 1u
                                           : tile + 1u - kRunTiles + nwg * kRunTiles;
    return nx < ntiles ? nx : kNone;
}

// Two words after the pass's member table: arrivals and generation of the
// tail kernel's grid barrier (zeroed by the pass's first kernel).
__device__ __forceinline__ u32* pass_barrier(const Member* M, u32 count) {
    return reinterpret_cast<u32*>(const_cast<Member*>(M) + count);
}

// Reads a member of the group table into registers.
__device__ __forceinline__ DevTree tree_of(const Member* M, u32 c) { return *M[c].tree; }

// The pass processes member c's batch in the grouped order: a pass of one
// octree with at least kGroupMinItems points, and an octree that keeps the
// grouped buffers.  Every kernel of the pass decides alike (the launches of
// a pass whose capacity allows it pass grouped = 1).
__device__ __forceinline__ bool grouped_member(const Member* M, u32 count, u32 c, u32 grouped,
                                               const DevTree& t) {
    return grouped && count == 1u && M[c].n >= kGroupMinItems && t.grp_rec;
}

// Spatial bucket of integer position q: the Morton index of its cell at
// kBucketBits bits per axis.
__device__ __forceinline__ u32 bucket_of(u32 K, u32 qx, u32 qy, u32 qz) {
    const u32 x = K >= kBucketBits ? qx >> (K - kBucketBits) : qx << (kBucketBits - K);
    const u32 y = K >= kBucketBits ? qy >> (K - kBucketBits) : qy << (kBucketBits - K);
    const u32 z = K >= kBucketBits ? qz >> (K - kBucketBits) : qz << (kBucketBits - K);
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// ---------------------------------------------------------- first round
// Counts every batch point in its leaf.  All leaves are open in this round;
// a leaf's total is its stored points plus this counter.  Block 0 also
// copies the members from the kernel argument into the device table the
// pass's later kernels read.  G: the pass may take the grouped order (then
// the points are also counted per spatial bucket).
template <bool G>
__global__ __launch_bounds__(256) void k_count_leaves(GroupArgs ga) {
    __shared__ u32 lkey[kLds];
    __shared__ u32 lval[kLds];
    __shared__ u32 lfill;
    __shared__ u32 bkey[G ? kLds : 1u], bval[G ? kLds : 1u];  // points per bucket
    __shared__ u32 bfill;
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 tid = threadIdx.x;
    const u32 nwg = gridDim.x;
    const u32 count = ga.count;
    const u32 grouped = G ? 1u : 0u;
    const Member* M = ga.m;
    if (blockIdx.x == 0 && tid < count) {
        ga.table[tid] = M[tid];
        // the previous pass's voxel store has read them: clear for this pass
        Counters* c = M[tid].tree->ctr;
        for (u32 k = 0; k < kStripes; ++k) c->claim_count[k] = 0u;
    }
    if (blockIdx.x == 0 && tid < 2u) pass_barrier(ga.table, count)[tid] = 0u;
    // the bucket table is used only by a pass that may take the grouped order
    const bool any_grp = G && count == 1u && M[0].n >= kGroupMinItems;  // uniform
    for (u32 i = tid; i < kLds; i += kWG) {
        lkey[i] = kNone;
        lval[i] = 0u;
        if (any_grp) {
            bkey[i] = kNone;
            bval[i] = 0u;
        }
    }
    if (tid == 0) lfill = bfill = 0u;
    const u32 ntiles = member_prefix(count, s_pre, [&](u32 c) {
        return M[c].tree->ctr->status ? 0u : (M[c].n + kWG - 1u) / kWG;
    });
    // the tile's batch record, loaded one tile ahead
    auto load = [&](u32 tl, uint4& rec) {
        const u32 cc = member_of(s_pre, count, tl);
        const u32 jj = (tl - s_pre[cc]) * kWG + tid;
        if (jj < M[cc].n) rec = M[cc].batch[jj];
    };
    uint4 rec_n = make_uint4(0u, 0u, 0u, 0u);
    u32 tile = first_tile(nwg);
    if (tile < ntiles) load(tile, rec_n);
    while (tile < ntiles) {
        const u32 c = member_of(s_pre, count, tile);
        const DevTree t = tree_of(M, c);
        const u32 n = M[c].n;
        const u32 j = (tile - s_pre[c]) * kWG + tid;
        const uint4 rec = rec_n;
        const u32 nx = next_tile(tile, ntiles, nwg);
        const bool grp = G && grouped_member(M, count, c, grouped, t);
        u32 leaf = kNone, bucket = kNone;
        if (j < n) {
            u32 qx, qy, qz;
            quantize3(t, rec, qx, qy, qz);
            if (grp) bucket = bucket_of(t.K, qx, qy, qz);
            // directory entries first, then the next tile's record, so that
            // waiting for the entries leaves the record load in flight
            const u32 D = t.dir_depth;
            const u32 m = dir_index(t.K, D, qx, qy, qz);
            u32 e[kDirMaxDepth + 1];
#pragma unroll
            for (u32 d = 0; d <= kDirMaxDepth; ++d)
                e[d] = d <= D ? t.dir[dir_offset(d) + (m >> (3u * (D - d)))] : kNone;
            if (nx != kNone) load(nx, rec_n);
            leaf = leaf_from_entries(t, e, m, qx, qy, qz);
            t.item_leaf[j] = leaf;  // the histogram round reads it
        } else if (nx != kNone) {
            load(nx, rec_n);
        }
        const Run r = lane_runs(leaf);
        if (leaf != kNone && r.rank == 0u) {
            const u32 e = lds_find_or_insert(lkey, kLdsBits, leaf, kCountProbe, &lfill);
            if (e != kNone)
                atomicAdd(&lval[e], r.len);
            else
                count_leaf_global(t, leaf, r.len);
        }
        if (G && grp) {  // uniform
            const Run rb = lane_runs(bucket);
            if (bucket != kNone && rb.rank == 0u) {
                const u32 e = lds_find_or_insert(bkey, kLdsBits, bucket, kCountProbe, &bfill);
                if (e != kNone)
                    atomicAdd(&bval[e], rb.len);
                else
                    atomicAdd(&t.bcnt[bucket], rb.len);
            }
        }
        // both tables flush when the member ends or when one fills: the
        // bucket table's decision shares the leaf table's barriers
        const bool force = nx == kNone || nx >= s_pre[c + 1u];
        __syncthreads();
        const bool flush = force || lfill >= kCountFlushAt;
        const bool bflush = G && grp && (force || bfill >= kBucketFlushAt);
        __syncthreads();  // every thread has read the fills before they change
        if (bflush) {
            for (u32 e = tid; e < kLds; e += kWG) {
                if (bkey[e] != kNone) {
                    atomicAdd(&t.bcnt[bkey[e]], bval[e]);
                    bkey[e] = kNone;
                    bval[e] = 0u;
                }
            }
            if (tid == 0) bfill = 0u;
        }
        if (flush) {
            for (u32 e = tid; e < kLds; e += kWG) {
                if (lkey[e] != kNone) {
                    flush_count(t, lkey[e], lval[e]);
                    lkey[e] = kNone;
                    lval[e] = 0u;
                }
            }
            if (tid == 0) lfill = 0u;
        }
        if (flush || bflush) __syncthreads();
        tile = nx;
    }
}

// One workgroup per leaf counted in the first round.  A leaf whose stored
// plus counted points exceed T (and that is above Dmax) becomes a pending
// root: a zeroed histogram slot, its stored points and keys appended to the
// spill buffer (they are re-inserted with the batch) and its chunks pushed to
// the pool (section "Chunks and the Chunk Pool").  Any other counted leaf is
// final for the pass and listed with its number of new points.
__global__ __launch_bounds__(256) void k_split_leaves(const Member* M, u32 count) {
    __shared__ u32 s_dec[2];
    __shared__ i32 s_pool;
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 tid = threadIdx.x;
    const u32 total = member_prefix(count, s_pre, [&](u32 c) {
        const DevTree* tp = M[c].tree;
        return tp->ctr->status ? 0u : min(tp->ctr->touched_count, tp->max_nodes);
    });
    for (u32 it = blockIdx.x; it < total; it += gridDim.x) {
        const u32 c = member_of(s_pre, count, it);
        const DevTree t = tree_of(M, c);
        Counters* ctr = t.ctr;
        const u32 L = t.touched[it - s_pre[c]];
        if (tid == 0) {
            const u32 cn = t.cnt[L];
            const u32 stored = t.count[L];
            const u32 depth = t.geo[L].w;
            u32 pend = 0u, slot = 0u, sbase = 0u;
            if ((u64)stored + cn > (u64)t.T && depth < t.Dmax) {
                slot = atomicAdd(&ctr->hist_top, 1u);
                const u32 p = atomicAdd(&ctr->pending_count[1], 1u);
                // job index and first spill index from one atomic: the jobs
                // are listed in spill-buffer order
                u64 sj = 0ull;
                if (stored)
                    sj = atomicAdd(reinterpret_cast<unsigned long long*>(&ctr->spill_count),
                                   (1ull << 32) | stored);
                sbase = (u32)sj;
                const u32 job = (u32)(sj >> 32);
                if (slot >= t.hist_cap)
                    set_status(t, SIMLOD_OVF_HIST);
                else if (p >= t.max_nodes || job >= t.max_nodes)
                    set_status(t, SIMLOD_OVF_WORK);
                else if ((u64)sbase + stored > (u64)t.spill_cap)
                    set_status(t, SIMLOD_OVF_SPILL);
                else {
                    t.pending[1][p] = L;
                    if (stored) t.spill_job[job] = make_uint2(L, sbase);
                    pend = 1u;
                }
            } else {
                const u32 p = atomicAdd(&ctr->final_count, 1u);
                if (p < t.max_nodes)
                    t.final_list[p] = make_uint2(L, cn);
                else
                    set_status(t, SIMLOD_OVF_WORK);
            }
            t.cnt[L] = 0u;
            s_dec[0] = pend;
            s_dec[1] = slot;
        }
        __syncthreads();
        if (s_dec[0]) {
            const u32 slot = s_dec[1];
            u32* h = t.hist + (u64)slot * kHistEntries;
            for (u32 i = tid; i < kHistEntries; i += kWG) h[i] = 0u;
            // The stored points are copied to the spill buffer by the
            // histogram round (spread over its whole grid).  Their chunks
            // go to the pool now: they are handed out again only after that
            // round, and the node's chunk table stays as it is.
            const u32 stored = t.count[L];
            if (stored) {
                const u32* tab = table_of(t, L);
                const u32 nch = t.nchunks[L];
                if (tid == 0) s_pool = atomicAdd(&ctr->pool_top, (i32)nch);
                __syncthreads();
                const i32 pb = s_pool;
                for (u32 j = tid; j < nch; j += kWG)
                    if ((u64)pb + j < (u64)t.pool_cap) t.pool[pb + j] = tab[j];
            }
            __syncthreads();
            if (tid == 0) {
                t.count[L] = 0u;
                t.nchunks[L] = 0u;
                t.hslot[L] = slot;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- grouped order
// Large passes of one octree: the batch is copied into the order grouped by
// spatial bucket (buckets in Morton order; within a bucket in the order the
// windows reserve their places), with each point's batch index and
// first-round leaf; the later kernels read the batch part of the work list
// from there.  The first round counted the points per bucket; a scan of
// the counts gives each bucket's first place (and clears the counts for the
// next pass).  A workgroup then takes windows of kGroupTiles tiles: it
// counts the window's points per bucket in LDS, reserves each bucket's
// places with one atomic (same-address atomics serialize, and every window
// of a dense strip meets the same few buckets), then places the points.
constexpr u32 kGroupTiles = 8;
constexpr u32 kGroupBits = 11;  // table entries >= the points of a window
static_assert((1u << kGroupBits) >= kGroupTiles * 256u, "a window's buckets always fit");
static_assert(kBucketChunk % kWG == 0u && kBuckets % kBucketChunk == 0u, "scan layout");

__device__ u32 wg_exclusive_scan(u32* a, u32 n, u32* part);  // below

// The pass takes the grouped order (its only member, a large batch, the
// buffers, not poisoned).  One thread reads, the workgroup gets the answer:
// uniform.
__device__ __forceinline__ bool group_pass_on(const Member* M, u32 count) {
    __shared__ u32 s_on;
    if (threadIdx.x == 0) {
        const DevTree* tp = M[0].tree;
        s_on = count == 1u && M[0].n >= kGroupMinItems && tp->grp_rec && !tp->ctr->status;
    }
    __syncthreads();
    return s_on != 0u;
}

// Exclusive scan of the bucket counts, one chunk per workgroup, into bnext
// (chunk-relative) and bsum (chunk totals; scanned by the next kernel).
__global__ __launch_bounds__(256) void k_bucket_scan(const Member* M, u32 count) {
    __shared__ u32 s_wsum[kWG / 64u];
    if (!group_pass_on(M, count)) return;  // uniform
    const DevTree t = tree_of(M, 0u);
    const u32 lo = blockIdx.x * kBucketChunk;
    const u32 tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    u32 v[kBucketChunk / kWG];
#pragma unroll
    for (u32 k = 0; k < kBucketChunk / kWG; ++k) {  // coalesced, all in flight
        v[k] = t.bcnt[lo + k * kWG + tid];
        t.bcnt[lo + k * kWG + tid] = 0u;  // clear for the next pass
    }
    u32 carry = 0u;  // uniform: the sum of the rounds before
#pragma unroll
    for (u32 k = 0; k < kBucketChunk / kWG; ++k) {
        u32 x = v[k];
#pragma unroll
        for (u32 o = 1; o < 64u; o <<= 1) {  // inclusive scan within the wavefront
            const u32 y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63u) s_wsum[wave] = x;
        __syncthreads();
        u32 before = carry, round = 0u;
#pragma unroll
        for (u32 w = 0; w < kWG / 64u; ++w) {
            if (w < wave) before += s_wsum[w];
            round += s_wsum[w];
        }
        t.bnext[lo + k * kWG + tid] = before + x - v[k];
        __syncthreads();  // s_wsum read by all before the next round writes it
        carry += round;
    }
    if (tid == 0) t.bsum[blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_bucket_sums(const Member* M, u32 count) {
    __shared__ u32 s_part[4];
    if (!group_pass_on(M, count)) return;  // uniform
    const DevTree t = tree_of(M, 0u);
    (void)wg_exclusive_scan(t.bsum, kBuckets / kBucketChunk, s_part);
}

__global__ __launch_bounds__(256) void k_group_batch(const Member* M, u32 count) {
    __shared__ u32 s_key[1u << kGroupBits], s_cnt[1u << kGroupBits], s_base[1u << kGroupBits];
    const u32 tid = threadIdx.x;
    for (u32 i = tid; i < (1u << kGroupBits); i += kWG) {
        s_key[i] = kNone;
        s_cnt[i] = 0u;
    }
    if (!group_pass_on(M, count)) return;  // uniform (its barrier orders the clearing)
    const DevTree t = tree_of(M, 0u);
    const u32 n = M[0].n;
    const u32 per = kGroupTiles * kWG;
    const u32 nwin = (n + per - 1u) / per;
    for (u32 win = xcd_block(gridDim.x); win < nwin; win += gridDim.x) {
        const u32 j0 = win * per + tid;
        u32 leaf[kGroupTiles], key[kGroupTiles];
        uint4 rec[kGroupTiles];
#pragma unroll
        for (u32 k = 0; k < kGroupTiles; ++k) {
            const u32 j = j0 + k * kWG;
            leaf[k] = kNone;
            rec[k] = make_uint4(0u, 0u, 0u, 0u);
            if (j < n) {
                leaf[k] = t.item_leaf[j];
                rec[k] = M[0].batch[j];
            }
        }
#pragma unroll
        for (u32 k = 0; k < kGroupTiles; ++k) {
            key[k] = kNone;
            if (j0 + k * kWG < n) {
                u32 qx, qy, qz;
                quantize3(t, rec[k], qx, qy, qz);
                key[k] = bucket_of(t.K, qx, qy, qz);
            }
        }
        // the window's points per bucket
#pragma unroll
        for (u32 k = 0; k < kGroupTiles; ++k) {
            const Run r = lane_runs(key[k]);
            if (key[k] != kNone && r.rank == 0u)
                atomicAdd(&s_cnt[lds_find_or_insert(s_key, kGroupBits, key[k])], r.len);
        }
        __syncthreads();
        for (u32 i = tid; i < (1u << kGroupBits); i += kWG) {
            const u32 b = s_key[i];
            if (b != kNone) s_base[i] = atomicAdd(&t.bnext[b], s_cnt[i]) + t.bsum[b / kBucketChunk];
            s_cnt[i] = 0u;  // from here on: places taken within the window
        }
        __syncthreads();
#pragma unroll
        for (u32 k = 0; k < kGroupTiles; ++k) {
            const u32 j = j0 + k * kWG;
            const Run r = lane_runs(key[k]);
            u32 e = kNone, r0 = 0u;
            if (key[k] != kNone && r.rank == 0u) {
                e = lds_find_or_insert(s_key, kGroupBits, key[k]);  // present: counted above
                r0 = atomicAdd(&s_cnt[e], r.len);
            }
            e = __shfl(e, r.head);
            r0 = __shfl(r0, r.head) + r.rank;
            if (j < n) {
                const u32 pos = s_base[e] + r0;
                if (pos < n) {
                    t.grp_rec[pos] = rec[k];
                    t.grp_index[pos] = j;
                    t.grp_leaf[pos] = leaf[k];
                } else {  // the first round's counts and these disagree
                    set_status(t, SIMLOD_OVF_INTERNAL);
                }
            }
        }
        __syncthreads();
        for (u32 i = tid; i < (1u << kGroupBits); i += kWG) {
            s_key[i] = kNone;
            s_cnt[i] = 0u;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------- histogram rounds
// The histogram level counted for a pending root at depth d: kHistLevels
// levels down, or down to Dmax.
__device__ __forceinline__ u32 hist_depth(u32 d, u32 Dmax) { return min(kHistLevels, Dmax - d); }

// Relative Morton index, j levels below depth d, of integer position q.
__device__ __forceinline__ u32 rel_index(u32 K, u32 d, u32 j, u32 qx, u32 qy, u32 qz) {
    const u32 s = K - d - j;
    const u32 m = (1u << j) - 1u;
    return spread3((qx >> s) & m) | (spread3((qy >> s) & m) << 1) | (spread3((qz >> s) & m) << 2);
}

// Round k >= 2: every point whose leaf is a pending root adds one to the
// root's histogram at the deepest of the kHistLevels levels below it that
// exists (levels beyond Dmax do not); the build kernel sums the levels above
// it from that one.  Round 2 walks all of W; later rounds only the items
// counted in the round before.  Octrees without pending roots take no part.
// grouped (uniform): the pass may take the grouped order (grouped_member
// decides per member).
__device__ __forceinline__ void count_hist_body(const Member* M, u32 count, u32 round, u32 nwg,
                                                u32 grouped) {
    __shared__ u32 lkey[kLds];
    __shared__ u32 lval[kLds];
    __shared__ u32 lfill;
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < count) M[tid].tree->ctr->pending_count[round & 1u] = 0u;
    for (u32 i = tid; i < kLds; i += kWG) {
        lkey[i] = kNone;
        lval[i] = 0u;
    }
    if (tid == 0) lfill = 0u;
    const u32 ntiles = member_prefix(count, s_pre, [&](u32 c) {
        const Counters* ctr = M[c].tree->ctr;
        return ctr->status || ctr->pending_count[(round - 1u) & 1u] == 0u
                   ? 0u
                   : (ctr->spill_count + M[c].n + kWG - 1u) / kWG;
    });
    for (u32 tile = first_tile(nwg); tile < ntiles;) {
        const u32 c = member_of(s_pre, count, tile);
        const DevTree t = tree_of(M, c);
        const u32 S = t.ctr->spill_count;
        const u32 nwork = S + M[c].n;
        const uint8_t* prev = round >= 3u ? ((round & 1u) ? t.amask[0] : t.amask[1]) : nullptr;
        uint8_t* mark = (round & 1u) ? t.amask[1] : t.amask[0];
        const u32 j = (tile - s_pre[c]) * kWG + tid;
        const bool grp = grouped_member(M, count, c, grouped, t);
        u32 slot = kNone, depth = 0u, qx = 0u, qy = 0u, qz = 0u;
        if (j < S && !prev) {
            // round 2, a spilled item: its leaf is the spill job whose range
            // holds j (jobs are in buffer order); the record is copied from
            // the leaf's chunks to the spill buffer for the later kernels
            u32 lo = 0u, hi = t.ctr->spill_jobs;
            while (hi - lo > 1u) {
                const u32 mid = (lo + hi) >> 1;
                if (t.spill_job[mid].y <= j)
                    lo = mid;
                else
                    hi = mid;
            }
            const uint2 job = t.spill_job[lo];
            const u32 s = j - job.y;
            const u32 ci = div_C(t, s);
            const u32 cb = table_of(t, job.x)[ci];
            const u32 o = s - ci * t.C;
            const uint4 rec = chunk_recs(t, cb)[o];
            t.spill_rec[j] = rec;
            t.spill_key[j] = chunk_keys(t, cb)[o];
            slot = t.hslot[job.x];
            quantize3(t, rec, qx, qy, qz);
            depth = t.geo[job.x].w;
        } else if (j < nwork && !prev) {
            // round 2, a batch item: the tree has not changed since the
            // first round, so the item's leaf is the one recorded then; only
            // items of pending roots need their record
            const u32 leaf = grp ? t.grp_leaf[j - S] : t.item_leaf[j - S];
            slot = t.hslot[leaf];
            if (slot != kNone) {
                quantize3(t, grp ? t.grp_rec[j - S] : M[c].batch[j - S], qx, qy, qz);
                depth = t.geo[leaf].w;
            }
        } else if (j < nwork && prev[j]) {
            uint4 rec;
            u32 key;
            fetch_work(t, M[c].batch, grp, S, M[c].base_key, j, rec, key);
            quantize3(t, rec, qx, qy, qz);
            const u32 leaf = find_leaf(t, qx, qy, qz, depth);
            slot = t.hslot[leaf];
        }
        if (j < nwork) mark[j] = slot != kNone ? 1u : 0u;
        {
            u32 key = kNone;
            if (slot != kNone) {  // a pending root is above Dmax: lv >= 1
                const u32 lv = hist_depth(depth, t.Dmax);
                key = kHistKey | (slot * kHistEntries + hist_level_offset(lv) +
                                  rel_index(t.K, depth, lv, qx, qy, qz));
            }
            const Run r = lane_runs(key);
            if (key != kNone && r.rank == 0u) {
                const u32 e = lds_find_or_insert(lkey, kLdsBits, key, kCountProbe, &lfill);
                if (e != kNone)
                    atomicAdd(&lval[e], r.len);
                else
                    flush_count(t, key, r.len);
            }
        }
        const u32 nx = next_tile(tile, ntiles, nwg);
        count_table_tile_end(t, lkey, lval, &lfill,
                             nx == kNone || nx >= s_pre[c + 1u]);
        tile = nx;
    }
}

// Exclusive prefix sum of a[0..n) in LDS by one workgroup; returns the total.
// Each thread sums a contiguous chunk; the 256 chunk sums are scanned with
// wavefront shuffles (4 wavefronts, their totals combined through LDS).
// part: LDS scratch of kWG + 1 entries.
__device__ u32 wg_exclusive_scan(u32* a, u32 n, u32* part) {
    const u32 tid = threadIdx.x;
    const u32 lane = lane_id();
    const u32 wave = tid >> 6;
    const u32 per = (n + kWG - 1u) / kWG;
    const u32 lo = min(tid * per, n), hi = min(lo + per, n);
    u32 sum = 0u;
    for (u32 i = lo; i < hi; ++i) sum += a[i];
    u32 v = sum;  // inclusive scan within the wavefront
#pragma unroll
    for (u32 o = 1; o < 64u; o <<= 1) {
        const u32 y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    if (lane == 63u) part[wave] = v;  // wavefront totals
    __syncthreads();
    u32 before = 0u;
    for (u32 w = 0; w < wave; ++w) before += part[w];
    const u32 total = part[0] + part[1] + part[2] + part[3];
    u32 run = before + v - sum;  // exclusive prefix of this thread's chunk
    for (u32 i = lo; i < hi; ++i) {
        const u32 x = a[i];
        a[i] = run;
        run += x;
    }
    __syncthreads();  // part[] and a[] complete before anyone reuses them
    return total;
}

// Index layout of one pending root's virtual subtree in the build kernel:
// 0 = the root, 1 + hist_level_offset(j) + rel = the level-j descendant with
// relative Morton path rel.  Only levels 0..kHistLevels-1 can split.
constexpr u32 kTreeSlots = 1u + kHistEntries;
constexpr u32 kSplitSlots = 1u + 8u + 64u + 512u;  // levels 0..kHistLevels-1
constexpr u32 kFExists = 1u, kFSplit = 2u, kFPending = 4u, kFFinal = 8u;

__device__ __forceinline__ void slot_level(u32 i, u32& lv, u32& rel) {
    const u32 k = i - 1u;
    lv = k < 8u ? 1u : (k < 72u ? 2u : (k < 584u ? 3u : 4u));
    rel = k - hist_level_offset(lv);
}

__device__ __forceinline__ u32 slot_parent(u32 lv, u32 rel) {
    return lv == 1u ? 0u : 1u + hist_level_offset(lv - 1u) + (rel >> 3);
}

// Round k >= 2: one workgroup per pending root X (depth d0).  From X's
// histogram it decides the subtree kHistLevels levels down: a descendant at
// level j < kHistLevels is inner iff it holds more than T points and is above
// Dmax; one at the last level that must split becomes a pending root of the
// next round (with a fresh histogram slot); every other descendant with
// points is a final leaf listed with its point count.  X and its inner
// descendants receive 8 consecutive children each (one node-count atomic per
// root, in level order), occupancy grids (fresh blocks of the persistent
// buffer, which is clear above its bump pointer) and directory entries.
__device__ __forceinline__ void build_body(const Member* M, u32 count, u32 round, u32 nwg) {
    __shared__ u32 s_h[kHistEntries];   // the root's histogram
    __shared__ u32 s_f[kTreeSlots];     // kF* flags per virtual node
    __shared__ u32 s_sp[kSplitSlots];   // split index of inner nodes
    __shared__ u32 s_q[kTreeSlots];     // scan buffer
    __shared__ u32 s_part[kWG + 1u];
    __shared__ u32 s_alloc[8];
    __shared__ u32 s_pre[kMaxMembers + 1u];
    __shared__ u32 s_lvsplit[kHistLevels + 1u];  // level lv has a node that splits
    const u32 tid = threadIdx.x;
    const u32 total = member_prefix(count, s_pre, [&](u32 c) {
        const DevTree* tp = M[c].tree;
        const Counters* ctr = tp->ctr;
        return ctr->status ? 0u : min(ctr->pending_count[(round - 1u) & 1u], tp->max_nodes);
    });
    if (blockIdx.x == 0 && tid < count && s_pre[tid + 1u] > s_pre[tid])
        atomicAdd(&M[tid].tree->ctr->build_rounds, 1u);
    const u32 out = round & 1u;
    for (u32 it = blockIdx.x; it < total; it += nwg) {
        const u32 c = member_of(s_pre, count, it);
        const DevTree t = tree_of(M, c);
        Counters* ctr = t.ctr;
        u32* const pend_out = out ? t.pending[1] : t.pending[0];  // select: no indexed copy
        const u32 X = (out ? t.pending[0] : t.pending[1])[it - s_pre[c]];
        const uint4 gx = t.geo[X];
        const u32 d0 = gx.w;
        const u32* hsrc = t.hist + (u64)t.hslot[X] * kHistEntries;
        for (u32 i = tid; i < kHistEntries; i += kWG) s_h[i] = hsrc[i];
        if (tid == 0) s_f[0] = kFExists | kFSplit;
        if (tid <= kHistLevels) s_lvsplit[tid] = tid == 0u ? 1u : 0u;
        __syncthreads();
        // the points were counted at level L only: the levels above it are
        // the sums of their 8 children (Morton index rel -> 8 rel + o)
        for (int lv = (int)hist_depth(d0, t.Dmax) - 1; lv >= 1; --lv) {  // uniform
            const u32 off = hist_level_offset((u32)lv), offc = hist_level_offset((u32)lv + 1u);
            for (u32 rel = tid; rel < (1u << (3u * (u32)lv)); rel += kWG) {
                u32 sum = 0u;
#pragma unroll
                for (u32 o = 0; o < 8u; ++o) sum += s_h[offc + 8u * rel + o];
                s_h[off + rel] = sum;
            }
            __syncthreads();
        }
        // flags, level by level (a level exists below the level above's
        // splits); levels below the deepest one with nodes are not visited
        // and the later loops stop at slot nt
        u32 deepest = 0u;
        for (u32 lv = 1; lv <= kHistLevels && s_lvsplit[lv - 1u]; ++lv) {  // uniform
            const u32 width = 1u << (3u * lv);
            const u32 off = hist_level_offset(lv);
            for (u32 rel = tid; rel < width; rel += kWG) {
                u32 f = 0u;
                if (s_f[slot_parent(lv, rel)] & kFSplit) {
                    const u32 c = s_h[off + rel];
                    f = kFExists;
                    if (c > t.T && d0 + lv < t.Dmax)
                        f |= lv < kHistLevels ? kFSplit : kFPending;
                    else if (c > 0u)
                        f |= kFFinal;
                }
                if (f & kFSplit) s_lvsplit[lv] = 1u;
                s_f[1u + off + rel] = f;
            }
            deepest = lv;
            __syncthreads();
        }
        const u32 nt = 1u + hist_level_offset(deepest + 1u);  // slots of levels 0..deepest
        const u32 ns = 1u + hist_level_offset(deepest);       // levels 0..deepest-1 (may split)
        // split indices (level order) and per-kind counts
        for (u32 i = tid; i < ns; i += kWG) s_sp[i] = (s_f[i] & kFSplit) ? 1u : 0u;
        __syncthreads();
        const u32 nsplit = wg_exclusive_scan(s_sp, ns, s_part);
        u32 npend = 0u;
        if (deepest == kHistLevels) {  // pending roots only at the last level (uniform)
            for (u32 i = tid; i < nt; i += kWG) s_q[i] = (s_f[i] & kFPending) ? 1u : 0u;
            __syncthreads();
            npend = wg_exclusive_scan(s_q, nt, s_part);
        }
        if (tid == 0) {
            u32 ok = 1u;
            const u32 base = atomicAdd(&ctr->node_count, 8u * nsplit);
            const u32 gbase = atomicAdd(&ctr->arena_top, nsplit * t.grid_blocks);
            const u32 hb = npend ? atomicAdd(&ctr->hist_top, npend) : 0u;
            const u32 pb = npend ? atomicAdd(&ctr->pending_count[out], npend) : 0u;
            if ((u64)base + 8ull * nsplit > (u64)t.max_nodes) {
                set_status(t, SIMLOD_OVF_NODES);
                ok = 0u;
            } else if ((u64)gbase + (u64)nsplit * t.grid_blocks > (u64)t.arena_blocks) {
                set_status(t, SIMLOD_OVF_ARENA);
                ok = 0u;
            } else if ((u64)pb + npend > (u64)t.max_nodes) {
                set_status(t, SIMLOD_OVF_WORK);
                ok = 0u;
            } else if ((u64)hb + npend > (u64)t.hist_cap) {
                set_status(t, SIMLOD_OVF_HIST);
                ok = 0u;
            }
            s_alloc[0] = ok;
            s_alloc[1] = base;
            s_alloc[2] = gbase;
            s_alloc[4] = hb;
            s_alloc[5] = pb;
        }
        __syncthreads();
        if (!s_alloc[0]) continue;  // octree poisoned: later kernels skip it
        const u32 base = s_alloc[1], gbase = s_alloc[2];
        const u32 hb = s_alloc[4], pb = s_alloc[5];
        const u32 xidx = d0 <= t.dir_depth ? dir_index(t.K, d0, gx.x, gx.y, gx.z) : 0u;
        // create every existing descendant (X itself already is a node)
        for (u32 i = 1u + tid; i < nt; i += kWG) {
            const u32 f = s_f[i];
            if (!(f & kFExists)) continue;
            u32 lv, rel;
            slot_level(i, lv, rel);
            const u32 nd = base + 8u * s_sp[slot_parent(lv, rel)] + (rel & 7u);
            const u32 depth = d0 + lv;
            const u32 sh = t.K - depth;
            t.count[nd] = 0u;
            t.cnt[nd] = 0u;
            t.geo[nd] = make_uint4(gx.x | (compact3(rel) << sh), gx.y | (compact3(rel >> 1) << sh),
                                   gx.z | (compact3(rel >> 2) << sh), depth);
            t.tab[nd] = kNone;
            t.tabcap[nd] = 0u;
            t.nchunks[nd] = 0u;
            t.newv[nd] = 0u;
            if (f & kFSplit) {
                const u32 g = gbase + s_sp[i] * t.grid_blocks;
                t.child[nd] = base + 8u * s_sp[i];
                t.grid[nd] = g;
            } else {
                t.child[nd] = 0u;
                t.grid[nd] = kNone;
            }
            if (f & kFPending) {
                t.hslot[nd] = hb + s_q[i];
                pend_out[pb + s_q[i]] = nd;
            } else {
                t.hslot[nd] = kNone;
            }
            if (depth <= t.dir_depth)
                t.dir[dir_offset(depth) + ((xidx << (3u * lv)) | rel)] =
                    nd | ((f & kFSplit) ? kDirInner : 0u);
        }
        // the new pending roots' histograms start at zero
        for (u64 i = tid; i < (u64)npend * kHistEntries; i += kWG)
            t.hist[(u64)hb * kHistEntries + i] = 0u;
        // the root becomes inner (split index 0)
        if (tid == 0) {
            t.grid[X] = gbase;
            t.hslot[X] = kNone;
            t.child[X] = base;
            if (d0 <= t.dir_depth) t.dir[dir_offset(d0) + xidx] = X | kDirInner;
        }
        __syncthreads();
        // final leaves with their point counts
        for (u32 i = tid; i < nt; i += kWG) s_q[i] = (s_f[i] & kFFinal) ? 1u : 0u;
        __syncthreads();
        const u32 nfin = wg_exclusive_scan(s_q, nt, s_part);
        if (tid == 0) {
            const u32 fb = nfin ? atomicAdd(&ctr->final_count, nfin) : 0u;
            s_alloc[0] = (u64)fb + nfin <= (u64)t.max_nodes ? 1u : 0u;
            if (!s_alloc[0]) set_status(t, SIMLOD_OVF_WORK);
            s_alloc[6] = fb;
        }
        __syncthreads();
        if (!s_alloc[0]) continue;
        const u32 fb = s_alloc[6];
        for (u32 i = 1u + tid; i < nt; i += kWG) {
            if (!(s_f[i] & kFFinal)) continue;
            u32 lv, rel;
            slot_level(i, lv, rel);
            const u32 nd = base + 8u * s_sp[slot_parent(lv, rel)] + (rel & 7u);
            t.final_list[fb + s_q[i]] = make_uint2(nd, s_h[hist_level_offset(lv) + rel]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_count_hist(const Member* M, u32 count, u32 round,
                                                    u32 grouped) {
    count_hist_body(M, count, round, gridDim.x, grouped);
}

__global__ __launch_bounds__(256) void k_build(const Member* M, u32 count, u32 round) {
    build_body(M, count, round, gridDim.x);
}

// Polls before a barrier gives up: each poll is an acquire load plus a sleep
// of 8 x 64 cycles, so the wait lasts at least about 0.2 s.
constexpr u32 kBarrierSpin = 1u << 20;

// Barrier of the first n workgroups of a grid (all resident): every
// workgroup releases its writes, counts itself in and waits for the
// generation to move on.  The wait is bounded, so a grid that cannot
// complete the barrier still exits (returns false).
__device__ bool grid_barrier(u32* bar, u32 n) {
    __shared__ u32 s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const u32 gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        u32 ok = 1u;
        if (atomicAdd(&bar[0], 1u) == n - 1u) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            u32 spin = 0u;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++spin == kBarrierSpin) {
                    ok = 0u;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0u;
}

// ---------------------------------------------------------------- allocation
// One wavefront per listed node: the node needs ceil((old + added) / C)
// chunks in total (subsection "Allocating Chunks"); missing ones come from
// the pool first, then from the persistent buffer (section "Chunks and the
// Chunk Pool"), are appended to the node's chunk table (grown by doubling)
// and linked after its last chunk.
// nwg: the workgroups taking part (the first nwg of the grid).
__device__ __forceinline__ void alloc_body(const Member* M, u32 count, u32 voxels, u32 nwg) {
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 ntotal = member_prefix(count, s_pre, [&](u32 c) {
        const DevTree* tp = M[c].tree;
        const Counters* ctr = tp->ctr;
        return ctr->status ? 0u
                           : min(voxels ? ctr->vtouched_count : ctr->final_count, tp->max_nodes);
    });
    const u32 lane = lane_id();
    const u32 wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
    const u32 nwaves = nwg * (kWG >> 6);
    for (u32 ew = wave; ew < ntotal; ew += nwaves) {
        const u32 c = member_of(s_pre, count, ew);
        const DevTree t = tree_of(M, c);
        Counters* ctr = t.ctr;
        const u32 e = ew - s_pre[c];
        u32 node, added;
        if (voxels) {
            node = t.vtouched[e];
            added = t.newv[node];
        } else {
            uint2 fl = t.final_list[e];
            node = fl.x;
            added = fl.y;
        }
        const u32 old = t.count[node];
        const u32 have = t.nchunks[node];
        const u32 total = (u32)(((u64)old + added + t.C - 1u) / t.C);
        if (voxels && lane == 0) t.newv[node] = 0u;
        if (total <= have) continue;
        const u32 need = total - have;

        u32 tabblk = t.tab[node];
        const u32 cap = t.tabcap[node];
        if (total > cap) {
            u32 ncap = max(total, max(cap * 2u, 16u));
            u32 nb = (ncap * 4u + kBlockBytes - 1u) / kBlockBytes;
            u32 nblk = 0u;
            if (lane == 0) nblk = atomicAdd(&ctr->arena_top, nb);
            nblk = __shfl(nblk, 0);
            if ((u64)nblk + nb > (u64)t.arena_blocks) {
                if (lane == 0) set_status(t, SIMLOD_OVF_ARENA);
                continue;
            }
            u32* nt = reinterpret_cast<u32*>(block_ptr(t, nblk));
            if (cap) {
                const u32* ot = reinterpret_cast<const u32*>(block_ptr(t, tabblk));
                for (u32 j = lane; j < have; j += 64u) nt[j] = ot[j];
            }
            tabblk = nblk;
            if (lane == 0) {
                t.tab[node] = nblk;
                t.tabcap[node] = ncap;
            }
        }
        u32* table = reinterpret_cast<u32*>(block_ptr(t, tabblk));

        i32 top = 0;
        if (lane == 0) top = atomicSub(&ctr->pool_top, (i32)need);
        top = __shfl(top, 0);
        const u32 from_pool = top <= 0 ? 0u : min((u32)top, need);
        const u32 rest = need - from_pool;
        u32 abase = 0u;
        if (rest) {
            if (lane == 0) abase = atomicAdd(&ctr->arena_top, rest * t.chunk_blocks);
            abase = __shfl(abase, 0);
            if ((u64)abase + (u64)rest * t.chunk_blocks > (u64)t.arena_blocks) {
                if (lane == 0) set_status(t, SIMLOD_OVF_ARENA);
                continue;
            }
        }
        const u32 pool_lo = (u32)(top - (i32)from_pool);
        auto id_of = [&](u32 j) -> u32 {
            return j < from_pool ? t.pool[pool_lo + j] : abase + (j - from_pool) * t.chunk_blocks;
        };
        for (u32 j = lane; j < need; j += 64u) {
            u32 id = id_of(j);
            table[have + j] = id;
            *chunk_next(t, id) = (j + 1u < need) ? id_of(j + 1u) : kNone;
        }
        if (lane == 0) {
            if (have) *chunk_next(t, table[have - 1u]) = id_of(0);
            t.nchunks[node] = total;
        }
    }
}

__global__ __launch_bounds__(256) void k_alloc(const Member* M, u32 count, u32 voxels) {
    alloc_body(M, count, voxels, gridDim.x);
}

// Expansion rounds first..last, then the chunks of the final leaves, in one
// launch.  After the second round a pass rarely has pending roots left (only
// where one pass splits a region more than kHistLevels levels deep), so the
// whole grid usually goes straight to the allocation, instead of launches
// that each find nothing.  When there are, only the first `tail` workgroups
// run the rounds, separated by barriers among themselves, and then the
// allocation.  The host sizes `tail` to half of what the device holds of this
// kernel at once (occupancy x compute units), so the first `tail` workgroups
// are resident together even beside other work.  A barrier that still times
// out (the device so shared that they are not) poisons every member of the
// pass: its later rounds did not run.
constexpr u32 kTailWGs = 256;  // upper bound of `tail`

__device__ __forceinline__ u32 any_pending(const Member* M, u32 count, u32 round) {
    u32 any = 0u;
    for (u32 c = 0; c < count && !any; ++c)
        any = M[c].tree->ctr->pending_count[(round - 1u) & 1u] != 0u;
    return any;
}

__global__ __launch_bounds__(256) void k_rounds_alloc(const Member* M, u32 count, u32 first,
                                                      u32 last, u32 tail, u32 grouped) {
    __shared__ u32 s_any;
    // pending roots from the round before: the same for every workgroup
    // (written before the last barrier or launch, read after it)
    if (threadIdx.x == 0) s_any = first <= last ? any_pending(M, count, first) : 0u;
    __syncthreads();
    const bool rounds = s_any != 0u;  // uniform over the grid
    if (rounds) {
        if (blockIdx.x >= tail) return;
        u32* bar = pass_barrier(M, count);
        for (u32 round = first; round <= last; ++round) {
            if (round > first) {
                if (threadIdx.x == 0) s_any = any_pending(M, count, round);
                __syncthreads();
                if (!s_any) break;  // uniform
            }
            count_hist_body(M, count, round, tail, grouped);
            bool ok = grid_barrier(bar, tail);
            if (ok) {
                build_body(M, count, round, tail);
                ok = grid_barrier(bar, tail);
            }
            if (!ok) {
                if (threadIdx.x < count)
                    atomicOr(&M[threadIdx.x].tree->ctr->status, SIMLOD_OVF_INTERNAL);
                return;
            }
        }
    }
    alloc_body(M, count, 0u, rounds ? tail : gridDim.x);
}

// ------------------------------------------------------- voxel claim table
// Identity of a cell in the claim table: node << 3r | cell.
__device__ __forceinline__ u64 cell_identity(const DevTree& t, u64 ltag) {
    return ((ltag >> 24) << (3u * t.r)) | (ltag & 0xFFFFFFull);
}

// Claims cell T (home entry, remainder) for `key`, probing from distance d0
// on: an empty entry takes the claim word, an entry holding the cell keeps
// the smaller key (atomic min only when ours is smaller).  Returns false if
// no entry was found (status set); fresh = this call created the entry.
__device__ __forceinline__ bool claim_probe(const DevTree& t, u32 home, u32 rem, u32 key, u32 d0,
                                            u32& slot, bool& fresh) {
    for (u32 d = d0; d < (1u << kDistBits); ++d) {
        const u32 h = claim_step(t, home, d);
        const u32 tg = (rem << kDistBits) | d;
        const u64 mine = ((u64)tg << 32) | key;
        u64* w = claim_word_at(t, h);
        u64 cur = *w;
        if (cur == kEmptyWord)
            cur = atomicCAS((unsigned long long*)w, (unsigned long long)kEmptyWord,
                            (unsigned long long)mine);
        if (cur == kEmptyWord) {
            slot = h;
            fresh = true;
            return true;
        }
        if ((u32)(cur >> 32) == tg) {
            if ((u32)cur > key) atomicMin((unsigned long long*)w, (unsigned long long)mine);
            slot = h;
            fresh = false;
            return true;
        }
    }
    set_status(t, SIMLOD_OVF_HASH);
    return false;
}

// A claim by a spilled point (key below the batch's first key) also
// min-reduces (key << 32 | rgba) in the entry's side word: spilled records
// cannot be found from their keys, batch records can (batch[key - base]).
__device__ __forceinline__ void claim_spill_colour(const DevTree& t, u32 slot, u64 val) {
    atomicMin((unsigned long long*)claim_spill_at(t, slot), (unsigned long long)val);
}

// ------------------------------------------------------- sample and store
constexpr u32 kClaimBuf = 2048;  // claims staged per workgroup before one flush
constexpr u32 kSlotBits = 9;     // > 256 distinct leaves per tile
constexpr u32 kNodeBits = 8;     // inner nodes with new voxels per workgroup

constexpr u32 kCandBits = 10;  // claim candidates per tile, deduplicated in LDS
constexpr u32 kCands = 1u << kCandBits;
// Candidates the tile's table has no entry for (an overfull table: scans
// where every point meets fresh cells on many levels) wait in an overflow
// list and are claimed in the same round trip as the table's entries; only
// beyond kOvf per tile is a candidate claimed at once.
constexpr u32 kOvf = 256;

// Stages a claim the calling lane created: the claim-table slot goes to the
// workgroup's LDS buffer (straight to the stripe when that is full) and the
// node's new-voxel count is summed in LDS.
__device__ __forceinline__ void stage_claim(const DevTree& t, u32 hslot, u32 node, u32 stripe,
                                            u32* s_claims, u32* s_nclaims, u32* s_vkey,
                                            u32* s_vcnt, u32* s_vfill) {
    const u32 off = atomicAdd(s_nclaims, 1u);
    if (off < kClaimBuf) {
        s_claims[off] = hslot;
    } else {
        const u32 pos = atomicAdd(&t.ctr->claim_count[stripe], 1u);
        if (pos < t.claim_cap)
            t.claims[(u64)stripe * t.claim_cap + pos] = hslot;
        else
            set_status(t, SIMLOD_OVF_BACKLOG);
    }
    const u32 e = lds_find_or_insert(s_vkey, kNodeBits, node, kCountProbe, s_vfill);
    if (e != kNone) {
        atomicAdd(&s_vcnt[e], 1u);
    } else if (atomicAdd(&t.newv[node], 1u) == 0u) {
        const u32 p = atomicAdd(&t.ctr->vtouched_count, 1u);
        if (p < t.max_nodes)
            t.vtouched[p] = node;
        else
            set_status(t, SIMLOD_OVF_WORK);
    }
}

// Candidate table of a workgroup.  A live entry maps (node << 24 | cell) to
// the minimum (key << 32 | rgba) of the current tile; an entry flagged
// kSubmitted remembers a cell the workgroup already claimed in an earlier
// tile, with a smaller key than any batch item it meets later (its tiles run
// in increasing work index, batch keys increase with the index, and spilled
// items carry keys below every batch key).  A batch item on such a cell is
// dominated: its claim could not lower the cell's minimum, so it is dropped
// without touching global memory.  Submitted entries are only a cache: any
// may be overwritten by a new live entry.  Returns false when no entry was
// found within the probe limit.
constexpr u64 kSubmitted = 1ull << 63;  // tags use bits 0..55
// Probes of a candidate insert before the candidate goes to the overflow
// list: in an overfull table (dense scans) long probe chains of LDS atomics
// cost more than the global claim they save.
constexpr u32 kCandProbe = 2;

// Home entry of a cell in the LDS candidate table: a 32-bit multiplicative
// hash of (node, cell), cheaper than a 64-bit mix; any spread will do, the
// table only deduplicates within a workgroup.
__device__ __forceinline__ u32 cand_home(u64 tag) {
    const u32 x = (u32)(tag >> 24) * 0x9E3779B1u ^ (u32)tag * 0x85EBCA77u;
    return (x ^ (x >> 15)) >> (32u - kCandBits);
}

// Every probe is a compare-and-swap (from empty, or from the marker found
// there), so the common cases (a new entry, or the cell's own) cost one LDS
// round trip.  The lane that makes an entry live appends its index to the
// tile's live list (live, nlive), which is all the claim step visits.
__device__ __forceinline__ bool cand_insert(u64* ctag, u64* cval, u16* live, u32* nlive, u64 tag,
                                            u64 val, bool batch_item) {
    u32 h = cand_home(tag);
    u64 expect = kEmptyTag;
    for (u32 p = 0; p < kCandProbe;) {
        const u64 cur = atomicCAS((unsigned long long*)&ctag[h], (unsigned long long)expect,
                                  (unsigned long long)tag);
        if (cur == expect) {  // made live here (from empty or from a marker)
            live[atomicAdd(nlive, 1u)] = (u16)h;
            atomicMin((unsigned long long*)&cval[h], (unsigned long long)val);
            return true;
        }
        if (cur == tag) {
            atomicMin((unsigned long long*)&cval[h], (unsigned long long)val);
            return true;
        }
        if (batch_item && cur == (tag | kSubmitted)) return true;  // dominated
        if (cur == kEmptyTag || (cur & kSubmitted)) {  // free or a marker: take it
            expect = cur;  // entries only become live within a tile: bounded
            continue;
        }
        h = (h + 1u) & (kCands - 1u);  // another cell's live entry
        expect = kEmptyTag;
        ++p;
    }
    return false;
}

// A candidate the LDS table has no entry for is claimed in the global claim
// table at once.
__device__ __forceinline__ void claim_now(const DevTree& t, u64 tag, u32 key, u64 val, u32 stripe,
                                          u32 base_key, u32* s_claims, u32* s_nclaims,
                                          u32* s_vkey, u32* s_vcnt, u32* s_vfill) {
    u32 home, rem, slot;
    bool fresh;
    claim_home(t, cell_identity(t, tag), home, rem);
    if (claim_probe(t, home, rem, key, 0u, slot, fresh)) {
        if (key < base_key) claim_spill_colour(t, slot, val);
        if (fresh)
            stage_claim(t, slot, (u32)(tag >> 24), stripe, s_claims, s_nclaims, s_vkey, s_vcnt,
                        s_vfill);
    }
}

// One level of voxel sampling for a wave: every lane whose node at depth d is
// inner tests its cell's bit (word = the grid word holding it, loaded by the
// caller); a clear bit makes the cell a candidate.  Consecutive lanes on the
// same cell with increasing keys add it once; candidates are merged in the
// tile's LDS table (smallest key per cell), or else listed in the overflow
// list, and claimed globally, all at once, after the traversal.  Must be
// reached by the whole wave.  use_table (uniform): merge in the LDS table at
// all; without it every candidate goes to the overflow list, which a small
// pass's tiles (a few dozen candidates each, few of them repeated) fill at
// less cost than the table's compare-and-swap inserts.
__device__ __forceinline__ void level_candidates(const DevTree& t, bool inner, u32 node, u32 d,
                                                 u32 word, u32 qx, u32 qy, u32 qz, u32 key,
                                                 u32 rgba, bool batch_item, u32 lane,
                                                 bool use_table, u64* ctag,
                                                 u64* cval, u16* s_live, u32* s_nlive,
                                                 u64* s_ovf, u32* s_novf,
                                                 u32 stripe, u32 base_key,
                                                 u32* s_claims, u32* s_nclaims, u32* s_vkey,
                                                 u32* s_vcnt, u32* s_vfill) {
    u64 tag = kEmptyTag;
    if (inner) {
        const u32 lin = cell_lin(qx, qy, qz, t.Dmax - d, t.r, t.R - 1u);
        if (!((word >> (lin & 31u)) & 1u)) tag = ((u64)node << 24) | lin;
    }
    if (__ballot(tag != kEmptyTag) == 0ull) return;  // no candidate in the wave
    const u64 ptag = __shfl_up(tag, 1);
    const u32 pkey = __shfl_up(key, 1);
    const bool cand = tag != kEmptyTag && !(lane > 0u && ptag == tag && pkey < key);
    const u64 val = ((u64)key << 32) | (u64)rgba;
    if (cand && !(use_table && cand_insert(ctag, cval, s_live, s_nlive, tag, val, batch_item))) {
        const u32 o = atomicAdd(s_novf, 1u);
        if (o < kOvf) {  // claimed with the table's entries
            s_ovf[2u * o] = tag;
            s_ovf[2u * o + 1u] = val;
        } else {  // overflow list full too: claim now
            claim_now(t, tag, key, val, stripe, base_key, s_claims, s_nclaims, s_vkey, s_vcnt,
                      s_vfill);
        }
    }
}

// Claims of one tile, in two halves so that other global atomics can share
// the round trip: claim_issue takes a thread's entries of the LDS candidate
// table (and of the overflow list) and loads each one's home entry of the
// claim table with a plain load; claim_resolve then drops the candidates
// whose cell is already claimed with a smaller key, issues a CAS where the
// entry was empty, and handles what that found (an entry created, the
// cell's entry holding a larger key: atomic min, another cell's entry:
// probe on), and stages the claims this workgroup created.
//
// The plain load may return a stale copy of the entry, but within a pass an
// entry only goes from empty to one cell's claim word, whose key only
// decreases: a stale copy shows an empty entry (the CAS then finds the
// truth) or a key at least the current one, so a candidate it shows as
// dominated is dominated.  In a dense scan most candidates meet a cell
// another workgroup claimed earlier in the pass; the load answers them
// without a device-scope atomic (which is performed past the L2 and
// writes a whole line).
constexpr u32 kCandPer = kCands / 256u;
constexpr u32 kClaimPer = kCandPer + kOvf / 256u;  // + the overflow list's
static_assert(kOvf % 256u == 0u, "overflow entries are dealt one per thread and slot");
struct ClaimBatch {
    u64 tg[kClaimPer], vl[kClaimPer], cur[kClaimPer];
    u32 hh[kClaimPer], rm[kClaimPer];
};

// keep: the workgroup's next tile belongs to the same octree, so submitted
// cells stay in the table as dominance markers; otherwise it starts empty.
// Whole workgroup, after a barrier that follows the tile's inserts.
__device__ __forceinline__ void claim_issue(const DevTree& t, u64* ctag, u64* cval,
                                            const u16* s_live, u32 nlive, const u64* s_ovf,
                                            u32 novf, ClaimBatch& b, bool keep) {
#pragma unroll
    for (u32 k = 0; k < kCandPer; ++k) {
        const u32 i = threadIdx.x + k * 256u;
        b.tg[k] = kEmptyTag;
        b.vl[k] = ~0ull;
        b.hh[k] = b.rm[k] = 0u;
        if (i < nlive) {
            const u32 h = s_live[i];
            b.tg[k] = ctag[h];
            b.vl[k] = cval[h];
            ctag[h] = b.tg[k] | kSubmitted;
            cval[h] = ~0ull;
            claim_home(t, cell_identity(t, b.tg[k]), b.hh[k], b.rm[k]);
        }
    }
#pragma unroll
    for (u32 k = kCandPer; k < kClaimPer; ++k) {  // the overflow list
        const u32 i = threadIdx.x + (k - kCandPer) * 256u;
        b.tg[k] = kEmptyTag;
        b.vl[k] = ~0ull;
        b.hh[k] = b.rm[k] = 0u;
        if (i < min(novf, kOvf)) {
            b.tg[k] = s_ovf[2u * i];
            b.vl[k] = s_ovf[2u * i + 1u];
            claim_home(t, cell_identity(t, b.tg[k]), b.hh[k], b.rm[k]);
        }
    }
    if (!keep) {  // uniform: every entry, markers included, cleared
        __syncthreads();
        for (u32 i = threadIdx.x; i < kCands; i += kWG) {
            ctag[i] = kEmptyTag;
            cval[i] = ~0ull;
        }
    }
#pragma unroll
    for (u32 k = 0; k < kClaimPer; ++k)
        b.cur[k] = b.tg[k] != kEmptyTag ? *claim_word_at(t, b.hh[k]) : 0ull;
}

__device__ __forceinline__ void claim_resolve(const DevTree& t, const ClaimBatch& b, u32 stripe,
                                              u32 base_key, u32* s_claims, u32* s_nclaims,
                                              u32* s_vkey, u32* s_vcnt, u32* s_vfill) {
    u64 cur[kClaimPer];
#pragma unroll
    for (u32 k = 0; k < kClaimPer; ++k)
        cur[k] = (b.tg[k] != kEmptyTag && b.cur[k] == kEmptyWord)
                     ? atomicCAS((unsigned long long*)claim_word_at(t, b.hh[k]),
                                 (unsigned long long)kEmptyWord,
                                 (unsigned long long)(((u64)(b.rm[k] << kDistBits) << 32) |
                                                      (b.vl[k] >> 32)))
                     : b.cur[k];
#pragma unroll
    for (u32 k = 0; k < kClaimPer; ++k) {
        if (b.tg[k] == kEmptyTag) continue;
        const u32 key = (u32)(b.vl[k] >> 32);
        const u32 tg0 = b.rm[k] << kDistBits;
        bool fresh = false, found = true;
        u32 slot = b.hh[k];
        if ((u32)(cur[k] >> 32) == tg0 && (u32)cur[k] <= key) continue;  // dominated
        if (cur[k] == kEmptyWord) {
            fresh = true;
        } else if ((u32)(cur[k] >> 32) == tg0) {
            if ((u32)cur[k] > key)
                atomicMin((unsigned long long*)claim_word_at(t, slot),
                          (unsigned long long)(((u64)tg0 << 32) | key));
        } else {  // another cell's entry: probe on
            found = claim_probe(t, b.hh[k], b.rm[k], key, 1u, slot, fresh);
        }
        if (!found) continue;
        if (key < base_key) claim_spill_colour(t, slot, b.vl[k]);
        if (fresh)
            stage_claim(t, slot, (u32)(b.tg[k] >> 24), stripe, s_claims, s_nclaims, s_vkey,
                        s_vcnt, s_vfill);
    }
}

constexpr u32 kClaimFlushAt = kClaimBuf - kCands - kOvf - kWG;  // room for one more tile
constexpr u32 kNodeFlushAt = (1u << kNodeBits) / 2u;

// Appends the workgroup's staged claims to its stripe's list (one atomic)
// and adds its per-node new-voxel counts to the nodes (listing each node the
// first time); leaves the LDS buffers empty.  Whole workgroup.
__device__ __forceinline__ void flush_staged(const DevTree& t, u32 stripe, u32* s_claims, u32* s_nclaims,
                             u32* s_vkey, u32* s_vcnt, u32* s_vfill, u32* s_flush) {
    Counters* ctr = t.ctr;
    const u32 tid = threadIdx.x;
    __syncthreads();
    const u32 nc = min(*s_nclaims, kClaimBuf);
    if (tid == 0) *s_flush = nc ? atomicAdd(&ctr->claim_count[stripe], nc) : 0u;
    __syncthreads();
    u32* dst = t.claims + (u64)stripe * t.claim_cap;
    for (u32 i = tid; i < nc; i += kWG) {
        const u32 pos = *s_flush + i;
        if (pos < t.claim_cap)
            dst[pos] = s_claims[i];
        else
            set_status(t, SIMLOD_OVF_BACKLOG);
    }
    for (u32 i = tid; i < (1u << kNodeBits); i += kWG) {
        const u32 node = s_vkey[i];
        if (node != kNone && atomicAdd(&t.newv[node], s_vcnt[i]) == 0u) {
            const u32 p = atomicAdd(&ctr->vtouched_count, 1u);
            if (p < t.max_nodes)
                t.vtouched[p] = node;
            else
                set_status(t, SIMLOD_OVF_WORK);
        }
        s_vkey[i] = kNone;
        s_vcnt[i] = 0u;
    }
    __syncthreads();
    if (tid == 0) {
        *s_nclaims = 0u;
        *s_vfill = 0u;
    }
    __syncthreads();
}

// Walks each point of W once more from the root.  At every inner node it
// projects the point into the node's R^3 grid (cell = (q >> (Dmax - d)) &
// (R - 1) per axis); a cell whose bit is still clear from earlier passes is
// claimed in the claim table with the point's key, the smallest key winning.
// Consecutive lanes that hit the same cell with increasing keys claim once.
// At the leaf the point takes the next slot of the leaf and is written, with
// its key, into the chunk slot / C.
//
// Same-address device atomics serialize (about 11 ns each on MI355X), so
// nothing here issues one per wave on a shared counter: leaf slots are
// reserved per (workgroup, leaf) after an LDS histogram of the tile, per-node
// voxel counts are summed in LDS and flushed once per workgroup, and claimed
// cells are staged in LDS and appended with one atomic per workgroup on one
// of kStripes counters (workgroup id mod kStripes, i.e. one per XCD).
template <bool G>  // the pass may take the grouped order
__global__ __launch_bounds__(256) void k_sample_store(const Member* M, u32 count, u32 use_table) {
    const u32 grouped = G ? 1u : 0u;
    __shared__ u32 s_claims[kClaimBuf];
    __shared__ u32 s_lkey[1u << kSlotBits], s_lcnt[1u << kSlotBits], s_lbase[1u << kSlotBits];
    __shared__ u32 s_vkey[1u << kNodeBits], s_vcnt[1u << kNodeBits];
    __shared__ u64 s_ctag[kCands], s_cval[kCands];
    __shared__ u16 s_live[kCands];  // live entries of the tile's candidate table
    __shared__ u64 s_ovf[2u * kOvf];  // overflow list: (tag, value) pairs
    __shared__ u32 s_nclaims, s_flush, s_vfill, s_nlive, s_novf;
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 tid = threadIdx.x;
    const u32 nwg = gridDim.x;
    for (u32 i = tid; i < kCands; i += kWG) {
        s_ctag[i] = kEmptyTag;
        s_cval[i] = ~0ull;
    }
    for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
        s_lkey[i] = kNone;
        s_lcnt[i] = 0u;
    }
    for (u32 i = tid; i < (1u << kNodeBits); i += kWG) {
        s_vkey[i] = kNone;
        s_vcnt[i] = 0u;
    }
    if (tid == 0) {
        s_nclaims = 0u;
        s_vfill = 0u;
        s_nlive = 0u;
        s_novf = 0u;
    }
    const u32 ntiles = member_prefix(count, s_pre, [&](u32 c) {
        const Counters* ctr = M[c].tree->ctr;
        return ctr->status ? 0u : (ctr->spill_count + M[c].n + kWG - 1u) / kWG;
    });
    const u32 lane = lane_id();
    const u32 stripe = blockIdx.x % kStripes;
    // work item j of member c's tile: its record and key
    auto fetch = [&](u32 c, u32 tile, uint4& rec, u32& key) {
        const DevTree* tp = M[c].tree;
        const u32 S = tp->ctr->spill_count;
        const u32 j = (tile - s_pre[c]) * kWG + tid;
        if (j < S + M[c].n)
            fetch_work(*tp, M[c].batch, grouped_member(M, count, c, grouped, *tp), S,
                       M[c].base_key, j, rec, key);
    };
    u32 tile = first_tile(nwg);
    uint4 rec_n = make_uint4(0u, 0u, 0u, 0u);
    u32 key_n = 0u;
    if (tile < ntiles) fetch(member_of(s_pre, count, tile), tile, rec_n, key_n);
    while (tile < ntiles) {
        const u32 c = member_of(s_pre, count, tile);
        const DevTree t = tree_of(M, c);
        const u32 S = t.ctr->spill_count;
        const u32 base_key = M[c].base_key;
        const u32 j = (tile - s_pre[c]) * kWG + tid;
        const bool valid = j < S + M[c].n;
        const bool batch_item = j >= S;
        const u32 rmask = t.R - 1u;
        const uint4 rec = rec_n;
        const u32 key = key_n;
        u32 qx = 0u, qy = 0u, qz = 0u;
        if (valid) quantize3(t, rec, qx, qy, qz);
        // Path through the node directory: all entries, then all grid blocks,
        // then all grid words are loaded as independent batches.
        const u32 D = t.dir_depth;
        const u32 m = dir_index(t.K, D, qx, qy, qz);
        u32 e[kDirMaxDepth + 1], w[kDirMaxDepth + 1];
#pragma unroll
        for (u32 d = 0; d <= kDirMaxDepth; ++d)
            e[d] = (valid && d <= D) ? t.dir[dir_offset(d) + (m >> (3u * (D - d)))] : kNone;
#pragma unroll
        for (u32 d = 0; d <= kDirMaxDepth; ++d)
            w[d] = (e[d] != kNone && (e[d] & kDirInner)) ? t.grid[e[d] & ~kDirInner] : kNone;
#pragma unroll
        for (u32 d = 0; d <= kDirMaxDepth; ++d) {
            const u32 lin = d <= t.Dmax ? cell_lin(qx, qy, qz, t.Dmax - d, t.r, rmask) : 0u;
            w[d] = w[d] != kNone ? reinterpret_cast<const u32*>(block_ptr(t, w[d]))[lin >> 5] : ~0u;
        }
        u32 leaf = kNone;
        bool desc = valid;
#pragma unroll
        for (u32 d = 0; d <= kDirMaxDepth; ++d) {  // unrolled: constant indices into e, w
            if (d > D) break;                        // uniform
            const u32 ed = e[d], wd = w[d];
            const bool inner = desc && ed != kNone && (ed & kDirInner);
            if (desc && !inner) {
                if (ed == kNone) set_status(t, SIMLOD_OVF_INTERNAL);
                leaf = ed == kNone ? 0u : ed;
                desc = false;
            }
            level_candidates(t, inner, ed & ~kDirInner, d, wd, qx, qy, qz, key, rec.w,
                             batch_item, lane, use_table != 0u, s_ctag, s_cval, s_live,
                             &s_nlive, s_ovf, &s_novf, stripe, base_key, s_claims, &s_nclaims,
                             s_vkey, s_vcnt, &s_vfill);
        }
        // Below the directory: dependent walk through child[].
        u32 node = 0u;
        if (desc) node = t.child[e[D] & ~kDirInner] + octant_of(qx, qy, qz, t.K - 1u - D);
        for (u32 d = D + 1u; d <= t.Dmax; ++d) {
            const u32 ch = desc && d < t.Dmax ? t.child[node] : 0u;
            const bool inner = desc && ch != 0u;
            if (desc && !inner) {
                leaf = node;
                desc = false;
            }
            if (__ballot(inner) == 0ull) break;
            u32 word = ~0u;
            if (inner) word = grid_of(t, node)[cell_lin(qx, qy, qz, t.Dmax - d, t.r, rmask) >> 5];
            level_candidates(t, inner, node, d, word, qx, qy, qz, key, rec.w, batch_item, lane,
                             use_table != 0u, s_ctag, s_cval, s_live, &s_nlive, s_ovf, &s_novf,
                             stripe, base_key, s_claims, &s_nclaims, s_vkey, s_vcnt, &s_vfill);
            if (inner) node = ch + octant_of(qx, qy, qz, t.K - 1u - d);
        }
        if (desc) leaf = node;
        // leaf slots: LDS histogram of the tile
        if (!valid) leaf = kNone;
        const Run r = lane_runs(leaf);
        u32 le = kNone, r0 = 0u;
        if (leaf != kNone && r.rank == 0u) {
            le = lds_find_or_insert(s_lkey, kSlotBits, leaf);  // never full: <= 256 keys
            r0 = atomicAdd(&s_lcnt[le], r.len);
        }
        le = __shfl(le, r.head);
        r0 = __shfl(r0, r.head) + r.rank;
        // the leaf's chunk count and chunk table (written by the allocation
        // kernel) load now, so that only the chunk id waits for the slot
        const u32 nch = valid ? t.nchunks[leaf] : 0u;
        const u32* ltab = valid ? table_of(t, leaf) : nullptr;
        const u32 nx = next_tile(tile, ntiles, nwg);
        const u32 cn = nx == kNone ? kNone : member_of(s_pre, count, nx);
        __syncthreads();
        // one round trip for the tile: claim CASes, one slot reservation per
        // leaf, and the next tile's records
        ClaimBatch cb;
        // dominance markers need keys increasing along the workgroup's tiles,
        // which the grouped order does not keep
        claim_issue(t, s_ctag, s_cval, s_live, s_nlive, s_ovf, s_novf, cb,
                    cn == c && !grouped_member(M, count, c, grouped, t));
        for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
            const u32 k = s_lkey[i];
            if (k != kNone) s_lbase[i] = atomicAdd(&t.count[k], s_lcnt[i]);
            s_lkey[i] = kNone;
            s_lcnt[i] = 0u;
        }
        if (nx != kNone) fetch(cn, nx, rec_n, key_n);
        claim_resolve(t, cb, stripe, base_key, s_claims, &s_nclaims, s_vkey, s_vcnt, &s_vfill);
        __syncthreads();
        if (tid == 0) {  // every thread read them in claim_issue, before the barrier
            s_nlive = 0u;
            s_novf = 0u;
        }
        if (valid) {
            const u32 slot = s_lbase[le] + r0;
            const u32 ci = div_C(t, slot);
            if (ci < nch) {
                const u32 cbk = ltab[ci];
                const u32 o = slot - ci * t.C;
                chunk_recs(t, cbk)[o] = rec;
                chunk_keys(t, cbk)[o] = key;
            } else {
                set_status(t, SIMLOD_OVF_ARENA);
            }
        }
        // Staged claims and node counts go out before the buffers can
        // overflow in the next tile, and before the workgroup moves on to
        // another octree (or has no tile left).  The decision is read by
        // every thread before the barrier and changed by none until after
        // it: uniform.
        const bool flush = cn != c || s_nclaims > kClaimFlushAt || s_vfill >= kNodeFlushAt;
        __syncthreads();
        if (flush) flush_staged(t, stripe, s_claims, &s_nclaims, s_vkey, s_vcnt, &s_vfill, &s_flush);
        tile = nx;
    }
}

// ------------------------------------------------------- bookkeeping
// Statistics of the pass added and its counters cleared for the next one,
// by one thread per member at the start of the voxel store kernel: none of
// these counters is read by that kernel or written before the next pass.
// The claim counters, which the voxel store reads, are cleared by the next
// pass's first kernel instead.
__device__ __forceinline__ void pass_bookkeeping(const Member& mb) {
    const DevTree& t = *mb.tree;
    Counters* c = t.ctr;
    if (c->status || mb.n == 0u) return;  // an empty share did no work
    if (c->pool_top < 0) c->pool_top = 0;
    u32 claims = 0u;
    for (u32 k = 0; k < kStripes; ++k) claims += min(c->claim_count[k], t.claim_cap);
    const u32 rounds = 1u + c->build_rounds;
    c->last_rounds = rounds;
    c->last_spilled = c->spill_count;
    c->last_new_voxels = claims;
    c->max_rounds = max(c->max_rounds, rounds);
    c->max_spilled = max(c->max_spilled, c->spill_count);
    c->max_new_voxels = max(c->max_new_voxels, claims);
    c->sum_spilled += c->spill_count;
    c->sum_new_voxels += claims;
    c->sum_rounds += rounds;
    c->spill_count = 0u;
    c->spill_jobs = 0u;
    c->final_count = 0u;
    c->vtouched_count = 0u;
    c->touched_count = 0u;
    c->pending_count[0] = c->pending_count[1] = 0u;
    c->hist_top = 0u;
    c->build_rounds = 0u;
}

// ------------------------------------------------------- voxel stores
constexpr u32 kWordBits = 9;  // grid words touched per tile, merged in LDS

// One thread per claimed cell: the voxel (cell centre, colour of the
// smallest-key point) goes to the node's next voxel slot, the cell's bit is
// set, and the claim-table entry is cleared for the next pass.  Slots are
// reserved per (workgroup, node) after an LDS histogram of the tile, and the
// tile's bits are OR-ed per grid word in LDS before one atomic per word.
__global__ __launch_bounds__(256) void k_store_voxels(const Member* M, u32 count) {
    __shared__ u32 s_nkey[1u << kSlotBits], s_ncnt[1u << kSlotBits], s_nbase[1u << kSlotBits];
    __shared__ u64 s_wkey[1u << kWordBits];
    __shared__ u32 s_wbits[1u << kWordBits];
    __shared__ u32 s_pre[kMaxMembers + 1u];
    const u32 tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < count) pass_bookkeeping(M[tid]);
    for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
        s_nkey[i] = kNone;
        s_ncnt[i] = 0u;
    }
    for (u32 i = tid; i < (1u << kWordBits); i += kWG) {
        s_wkey[i] = kEmptyTag;
        s_wbits[i] = 0u;
    }
    // tiles of each octree's claims (all stripes, in stripe order)
    const u32 ntiles = member_prefix(count, s_pre, [&](u32 c) {
        const DevTree* tp = M[c].tree;
        const Counters* ctr = tp->ctr;
        if (ctr->status) return 0u;
        u32 n = 0u;
        for (u32 s = 0; s < kStripes; ++s) n += min(ctr->claim_count[s], tp->claim_cap);
        return (n + kWG - 1u) / kWG;
    });
    for (u32 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const u32 c = member_of(s_pre, count, tile);
        const DevTree t = tree_of(M, c);
        Counters* ctr = t.ctr;
        u32 pre[kStripes + 1];
        pre[0] = 0u;
        for (u32 s = 0; s < kStripes; ++s)
            pre[s + 1] = pre[s] + min(ctr->claim_count[s], t.claim_cap);
        const u32 n = pre[kStripes];
        const u32 rmask = t.R - 1u;
        const u32 base = (tile - s_pre[c]) * kWG;
        const u32 i = base + tid;
        const bool valid = i < n;
        u32 h = 0u, node = kNone, lin = 0u;
        u64 val = 0ull;
        if (valid) {
            u32 s = 0;
            while (i >= pre[s + 1]) ++s;
            h = t.claims[(u64)s * t.claim_cap + (i - pre[s])];
            const ulonglong2 ent = *reinterpret_cast<const ulonglong2*>(claim_word_at(t, h));
            const u64 T = claim_identity(t, h, (u32)(ent.x >> 32));
            const u32 key = (u32)ent.x;
            node = (u32)(T >> (3u * t.r));
            lin = (u32)(T & low_bits(3u * t.r));
            // the winner's colour: from the batch record, or (a spilled
            // point) from the side word
            const u32 rgba = key >= M[c].base_key ? M[c].batch[key - M[c].base_key].w : (u32)ent.y;
            val = ((u64)key << 32) | rgba;
        }
        // slot reservation: LDS histogram per node, one global atomic per node
        const Run r = lane_runs(node);
        u32 ne = kNone, r0 = 0u;
        if (node != kNone && r.rank == 0u) {
            ne = lds_find_or_insert(s_nkey, kSlotBits, node);  // never full: <= 256 keys
            r0 = atomicAdd(&s_ncnt[ne], r.len);
        }
        ne = __shfl(ne, r.head);
        r0 = __shfl(r0, r.head) + r.rank;
        // the node's geometry, chunk count and chunk table load now
        uint4 g = make_uint4(0u, 0u, 0u, 0u);
        u32 nch = 0u;
        const u32* ntab = nullptr;
        if (valid) {
            g = t.geo[node];
            nch = t.nchunks[node];
            ntab = table_of(t, node);
        }
        // grid bits: OR per word in LDS
        if (valid) {
            const u64 wkey = ((u64)node << 32) | (lin >> 5);
            u32 we = (u32)(mix64(wkey) >> (64u - kWordBits));
            bool done = false;
            for (u32 p = 0; p < (1u << kWordBits) && !done; ++p) {
                const u64 cur = atomicCAS((unsigned long long*)&s_wkey[we],
                                          (unsigned long long)kEmptyTag, (unsigned long long)wkey);
                if (cur == kEmptyTag || cur == wkey) {
                    atomicOr(&s_wbits[we], 1u << (lin & 31u));
                    done = true;
                } else {
                    we = (we + 1u) & ((1u << kWordBits) - 1u);
                }
            }
            if (!done) atomicOr(&grid_of(t, node)[lin >> 5], 1u << (lin & 31u));
        }
        __syncthreads();
        for (u32 e = tid; e < (1u << kSlotBits); e += kWG) {
            const u32 k = s_nkey[e];
            if (k != kNone) s_nbase[e] = atomicAdd(&t.count[k], s_ncnt[e]);
        }
        for (u32 e = tid; e < (1u << kWordBits); e += kWG) {
            const u64 wk = s_wkey[e];
            if (wk != kEmptyTag) {
                atomicOr(&grid_of(t, (u32)(wk >> 32))[(u32)wk], s_wbits[e]);
                s_wkey[e] = kEmptyTag;
                s_wbits[e] = 0u;
            }
        }
        __syncthreads();
        if (valid) {
            const u32 slot = s_nbase[ne] + r0;
            const u32 d = g.w;
            const u32 shift = t.Dmax - d;
            const u32 cx = lin & rmask, cy = (lin >> t.r) & rmask, cz = lin >> (2u * t.r);
            uint4 v;
            v.x = __float_as_uint(cell_centre((g.x >> shift) + cx, t.mn[0], t.size, t.r, d));
            v.y = __float_as_uint(cell_centre((g.y >> shift) + cy, t.mn[1], t.size, t.r, d));
            v.z = __float_as_uint(cell_centre((g.z >> shift) + cz, t.mn[2], t.size, t.r, d));
            v.w = (u32)val;
            const u32 ci = div_C(t, slot);
            if (ci < nch) {
                const u32 cb = ntab[ci];
                const u32 o = slot - ci * t.C;
                chunk_recs(t, cb)[o] = v;
                chunk_keys(t, cb)[o] = (u32)(val >> 32);
            } else {
                set_status(t, SIMLOD_OVF_ARENA);
            }
            *reinterpret_cast<ulonglong2*>(claim_word_at(t, h)) = make_ulonglong2(kEmptyWord, ~0ull);
        }
        __syncthreads();
        for (u32 e = tid; e < (1u << kSlotBits); e += kWG) {
            s_nkey[e] = kNone;
            s_ncnt[e] = 0u;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- status words
// Group passes only: each member's status word after the pass, for the
// host's copy.
__global__ void k_finish(const Member* M, u32 count, u32* status_out) {
    const u32 m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < count) status_out[m] = M[m].tree->ctr->status;
}

// ------------------------------------------------------- reset / export
// n pairs (a, b) of u64.
__global__ void k_fill_pairs(u64* p, u64 n, u64 a, u64 b) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        reinterpret_cast<ulonglong2*>(p)[i] = make_ulonglong2(a, b);
}

__global__ void k_fill_u32(u32* p, u64 n, u32 v) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        p[i] = v;
}

// Clears the blocks of the persistent buffer handed out since the last
// reset.  Occupancy grids are only ever carved from fresh blocks (the bump
// pointer; the pool recycles chunks only), so a buffer that is zero up to
// the bump pointer gives every new inner node a clear grid without a pass
// having to clear it.
__global__ void k_zero_arena(DevTree t) {
    const u64 n = (u64)min(t.ctr->arena_top, t.arena_blocks) * (kBlockBytes / 16u);
    uint4* a = reinterpret_cast<uint4*>(block_ptr(t, 0u));
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        a[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_reset(DevTree t) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Counters* c = t.ctr;
    u32* raw = reinterpret_cast<u32*>(c);
    for (u32 i = 0; i < sizeof(Counters) / 4u; ++i) raw[i] = 0u;
    c->node_count = 1u;
    t.child[0] = 0u;
    t.count[0] = 0u;
    t.cnt[0] = 0u;
    t.hslot[0] = kNone;
    t.geo[0] = make_uint4(0u, 0u, 0u, 0u);
    t.grid[0] = kNone;
    t.tab[0] = kNone;
    t.tabcap[0] = 0u;
    t.nchunks[0] = 0u;
    t.newv[0] = 0u;
    t.dir[0] = 0u;  // the root, a leaf
}

// Copies the records and keys of the listed nodes to out[first[i] ...].
__global__ __launch_bounds__(256) void k_gather(DevTree t, const u32* nodes, const u64* first,
                                                u32 nn, uint4* out_rec, u32* out_key) {
    for (u32 i = blockIdx.x; i < nn; i += gridDim.x) {
        const u32 node = nodes[i];
        const u32 cnt = t.count[node];
        if (cnt == 0u) continue;
        const u64 f = first[i];
        const u32* tab = table_of(t, node);
        for (u32 s = threadIdx.x; s < cnt; s += kWG) {
            const u32 ci = div_C(t, s);
            const u32 cb = tab[ci];
            const u32 o = s - ci * t.C;
            out_rec[f + s] = chunk_recs(t, cb)[o];
            out_key[f + s] = chunk_keys(t, cb)[o];
        }
    }
}

// The same copy through the chunk lists, the layout's reader: one
// workgroup per node starts at the node's first chunk and follows each
// chunk's next link, copying a chunk's records together (section "Chunks
// and the Chunk Pool").  A list that ends early or runs past the node's
// last chunk sets *err.
__global__ __launch_bounds__(256) void k_walk(DevTree t, const u32* nodes, const u64* first,
                                              u32 nn, uint4* out_rec, u32* out_key, u32* err) {
    for (u32 i = blockIdx.x; i < nn; i += gridDim.x) {
        const u32 node = nodes[i];
        const u32 cnt = t.count[node];
        if (cnt == 0u) continue;
        const u64 f = first[i];
        u32 chunk = table_of(t, node)[0];
        for (u32 base = 0; base < cnt; base += t.C) {
            if (chunk == kNone || (u64)chunk + t.chunk_blocks > (u64)t.arena_blocks) {
                if (threadIdx.x == 0) atomicOr(err, 1u);
                break;
            }
            const u32 m = min(t.C, cnt - base);
            for (u32 s = threadIdx.x; s < m; s += kWG) {
                out_rec[f + base + s] = chunk_recs(t, chunk)[s];
                out_key[f + base + s] = chunk_keys(t, chunk)[s];
            }
            chunk = *chunk_next(t, chunk);
        }
        if (chunk != kNone && threadIdx.x == 0) atomicOr(err, 2u);  // list continues
    }
}

// ------------------------------------------------------- host launchers
static inline u32 grid_for(u64 items, u32 lo, u32 hi) {
    u64 g = (items + kWG - 1) / kWG;
    if (g < lo) g = lo;
    if (g > hi) g = hi;
    return (u32)((g + 7u) & ~7ull);
}

u32 expansion_rounds(u32 max_depth) { return 1u + (max_depth + kHistLevels - 1u) / kHistLevels; }

bool is_count_leaves_kernel(const void* f) {
    return f == reinterpret_cast<const void*>(&k_count_leaves<false>) ||
           f == reinterpret_cast<const void*>(&k_count_leaves<true>);
}

// Grid sizes depend only on `items`, the pass's batch points summed over the
// group (or a capacity for a pass captured in a graph), and the launch shape,
// never on device-side counts: every kernel loops over whatever work it finds.

hipError_t launch_count_leaves(const GroupArgs& ga, u64 items, const LaunchShape& sh,
                               hipStream_t s) {
    const u32 g = grid_for(items, 8, sh.cap[kShapeCount]);
    if (grouped_pass(ga.count, items))
        hipLaunchKernelGGL(k_count_leaves<true>, dim3(g), dim3(kWG), 0, s, ga);
    else
        hipLaunchKernelGGL(k_count_leaves<false>, dim3(g), dim3(kWG), 0, s, ga);
    return hipGetLastError();
}
// Passes whose launches let the device take the grouped order: one octree,
// a large batch (or capacity; each kernel checks the batch itself).  In
// group passes the members' batches are smaller, many of them already in
// good order, and the copy cost more than it saved.
u32 grouped_pass(u32 count, u64 items) {
    return count == 1u && items >= kGroupMinItems ? 1u : 0u;
}

hipError_t launch_split_leaves(const Member* m, u32 count, u64 items, hipStream_t s) {
    hipLaunchKernelGGL(k_split_leaves, dim3(grid_for(items / 64u, 64, 1024)), dim3(kWG), 0, s, m,
                       count);
    return hipGetLastError();
}
hipError_t launch_group_batch(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                              hipStream_t s) {
    if (!grouped_pass(count, items)) return hipSuccess;
    hipLaunchKernelGGL(k_bucket_scan, dim3(kBuckets / kBucketChunk), dim3(kWG), 0, s, m, count);
    hipLaunchKernelGGL(k_bucket_sums, dim3(1), dim3(kWG), 0, s, m, count);
    const u32 g = grid_for(items / kGroupTiles, 8, sh.cap[kShapeCount]);
    hipLaunchKernelGGL(k_group_batch, dim3(g), dim3(kWG), 0, s, m, count);
    return hipGetLastError();
}
hipError_t launch_count_hist(const Member* m, u32 count, u64 items, u32 round,
                             const LaunchShape& sh, hipStream_t s) {
    // Round 2 of a large pass (a 10M-point batch) has every point of a
    // pending root to histogram and about 11 tiles per workgroup even at
    // 4096 workgroups, which hide each other's latency; below 4M items the
    // launch shape's cap holds (more workgroups only add set-up there).
    const u32 cap = sh.cap[kShapeHist];
    const u32 cap2 = items >= (4ull << 20) ? std::max<u32>(cap, 4096u) : cap;
    const u32 g = round == 2u ? grid_for(items + 65536u, 64, cap2)
                              : grid_for(items / 4u, 32, std::max<u32>(cap / 2u, 32u));
    hipLaunchKernelGGL(k_count_hist, dim3(g), dim3(kWG), 0, s, m, count, round,
                       grouped_pass(count, items));
    return hipGetLastError();
}
hipError_t launch_build(const Member* m, u32 count, u32 round, hipStream_t s) {
    hipLaunchKernelGGL(k_build, dim3(128), dim3(kWG), 0, s, m, count, round);
    return hipGetLastError();
}
// Workgroups of the later expansion rounds: half of what the device holds of
// k_rounds_alloc at once (occupancy per compute unit x compute units), at
// most kTailWGs and at least 8; queried once per device.
static u32 tail_workgroups() {
    static u32 cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64u;
    if (cached[dev]) return cached[dev];
    int per_cu = 0, cus = 0;
    u32 tail = 64u;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rounds_alloc, kWG, 0) ==
            hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        per_cu > 0 && cus > 0)
        tail = std::max<u32>(8u, std::min<u32>(kTailWGs, (u32)(per_cu * cus) / 2u) & ~7u);
    cached[dev] = tail;
    return tail;
}

hipError_t launch_rounds_alloc(const Member* m, u32 count, u64 items, u32 first, u32 last,
                               hipStream_t s) {
    const u32 tail = tail_workgroups();
    hipLaunchKernelGGL(k_rounds_alloc, dim3(std::max<u32>(tail, 1024u)), dim3(kWG), 0, s, m,
                       count, first, last, tail, grouped_pass(count, items));
    return hipGetLastError();
}
hipError_t launch_alloc(const Member* m, u32 count, u32 voxels, hipStream_t s) {
    hipLaunchKernelGGL(k_alloc, dim3(voxels ? 256 : 1024), dim3(kWG), 0, s, m, count, voxels);
    return hipGetLastError();
}
hipError_t launch_sample_store(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                               hipStream_t s) {
    const u32 g = grid_for(items + 4096u, 64, sh.cap[kShapeSample]);
    // the LDS candidate table pays on large passes (a 10M-point scan's tiles
    // meet hundreds of repeated cells), not on 1M-point ones
    const u32 use_table = items >= (4ull << 20) ? 1u : 0u;
    if (grouped_pass(count, items))
        hipLaunchKernelGGL(k_sample_store<true>, dim3(g), dim3(kWG), 0, s, m, count, use_table);
    else
        hipLaunchKernelGGL(k_sample_store<false>, dim3(g), dim3(kWG), 0, s, m, count, use_table);
    return hipGetLastError();
}
hipError_t launch_store_voxels(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                               hipStream_t s) {
    const u32 g = grid_for(items, 64, sh.cap[kShapeStore]);
    hipLaunchKernelGGL(k_store_voxels, dim3(g), dim3(kWG), 0, s, m, count);
    return hipGetLastError();
}
hipError_t launch_finish(const Member* m, u32 count, u32* status_out, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kMaxMembers), 0, s, m, count, status_out);
    return hipGetLastError();
}
hipError_t launch_reset(const DevTree& t, u64 hash_entries, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_arena, dim3(4096), dim3(kWG), 0, s, t);  // before the counters
    u32 g = (u32)std::min<u64>((hash_entries + kWG - 1) / kWG, 4096);
    hipLaunchKernelGGL(k_fill_pairs, dim3(g), dim3(kWG), 0, s, t.hent, hash_entries, kEmptyTag,
                       ~0ull);
    const u64 dir_entries = dir_offset(t.dir_depth + 1u);
    const u32 gd = (u32)std::min<u64>((dir_entries + kWG - 1) / kWG, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(gd), dim3(kWG), 0, s, t.dir, dir_entries, kNone);
    if (t.bcnt) hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(kWG), 0, s, t.bcnt, (u64)kBuckets, 0u);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_walk(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                       uint4* out_rec, u32* out_key, u32* err, hipStream_t s) {
    const u32 g = std::max<u32>(1u, std::min<u32>(nn, 4096u));
    hipLaunchKernelGGL(k_walk, dim3(g), dim3(kWG), 0, s, t, nodes, first, nn, out_rec, out_key, err);
    return hipGetLastError();
}
hipError_t launch_gather(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                         uint4* out_rec, u32* out_key, hipStream_t s) {
    u32 g = std::min<u32>(std::max<u32>(nn, 1u), 4096u);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kWG), 0, s, t, nodes, first, nn, out_rec, out_key);
    return hipGetLastError();
}

}  // namespace simlod
