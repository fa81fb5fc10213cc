// gfx950 kernels of one insertion pass (section "Incrementally Updating the
// Octree").  A pass over a batch of n points runs, on one stream:
//
//   k_count / k_split, round k = 1..Dmax+1   expansion (subsection
//       "Expanding the Octree"); rounds after the first that finds no leaf
//       to split exit at once on a device flag, so the host never waits
//   k_alloc(points)      chunks for the leaves' new points (subsection
//                        "Allocating Chunks")
//   k_sample_store       one traversal per point: voxel claims at every
//                        inner node on the path (subsection "Voxel Sampling")
//                        and the point's store into its leaf (subsection
//                        "Storing Points and Voxels")
//   k_alloc(voxels)      chunks for the inner nodes' new voxels
//   k_store_voxels       voxel records from the claim backlog
//   k_finish             per-pass bookkeeping
//
// The work list W of a pass is the spill buffer followed by the batch:
// index i < S names spilled point i (with the key it was stored with),
// index i >= S names batch point i - S with key base_key + i - S.
//
// All cross-workgroup communication inside one kernel goes through atomics;
// anything else written in one kernel is read in a later one.
#include "octree_device.hpp"
#include "simlod.h"
#include "launch.hpp"

namespace simlod {

constexpr u32 kWG = 256;
constexpr u32 kLdsBits = 11;
constexpr u32 kLds = 1u << kLdsBits;
constexpr u32 kMaxProbe = 4096;

// Renumbers workgroups so that each of the 8 XCDs (which receive workgroups
// round-robin) walks a contiguous range of tiles: neighbouring points, and
// therefore the same nodes and grid words, stay in one XCD's L2.
__device__ __forceinline__ u32 xcd_block() {
    u32 b = blockIdx.x, g = gridDim.x;
    if (g & 7u) return b;
    return (b & 7u) * (g >> 3) + (b >> 3);
}

__device__ __forceinline__ void fetch_work(const DevTree& t, const uint4* batch, u32 S,
                                           u32 base_key, u32 i, uint4& rec, u32& key) {
    if (i < S) {
        rec = t.spill_rec[i];
        key = t.spill_key[i];
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

// Root-to-leaf walk: the child of a node at depth d takes bit K-1-d of each
// integer coordinate (x bit 0, y bit 1, z bit 2 of the octant).
__device__ __forceinline__ u32 find_leaf(const DevTree& t, u32 qx, u32 qy, u32 qz) {
    u32 node = 0;
    u32 bit = t.K - 1u;
    u32 c = t.child[0];
    for (u32 d = 0; c != 0u && d < t.Dmax; ++d) {  // children exist only above Dmax
        node = c + octant_of(qx, qy, qz, bit);
        --bit;
        c = t.child[node];
    }
    return node;
}

// Adds c to a leaf's round counter; the first addition of the round lists
// the leaf for the split kernel.
__device__ __forceinline__ void count_global(const DevTree& t, u32 node, u32 c, u32 round) {
    u32 old = atomicAdd(&t.cnt[node], c);
    if (old == 0u) {
        u32 p = atomicAdd(&t.ctr->touched_count[round & 1u], 1u);
        if (p < t.max_nodes)
            t.touched[round & 1u][p] = node;
        else
            set_status(t, SIMLOD_OVF_WORK);
    }
}

// Per-workgroup histogram in LDS (open addressing); false when full.
__device__ __forceinline__ bool count_lds(u32* lkey, u32* lval, u32 node, u32 c) {
    u32 h = (node * 0x9E3779B1u) >> (32u - kLdsBits);
    for (u32 p = 0; p < 32u; ++p) {
        u32 k = atomicCAS(&lkey[h], kNone, node);
        if (k == kNone || k == node) {
            atomicAdd(&lval[h], c);
            return true;
        }
        h = (h + 1u) & (kLds - 1u);
    }
    return false;
}

// Workgroup-uniform early exit: the handle is poisoned, or the previous
// round split nothing.  The status word can change while the kernel runs, so
// one thread reads it and the decision is broadcast through LDS before any
// barrier is reached.
__device__ __forceinline__ bool wg_skip(const Counters* ctr, u32 round) {
    __shared__ u32 s_skip;
    if (threadIdx.x == 0)
        s_skip = (ctr->status != 0u || (round > 1u && ctr->split_any[round - 1u] == 0u)) ? 1u : 0u;
    __syncthreads();
    return s_skip != 0u;
}

// ---------------------------------------------------------------- counting
// Round 1 counts every batch point in its leaf (all leaves are open; a
// leaf's counter adds to the points it already stores).  Round k >= 2 counts
// only points whose leaf was created by round k-1's splits: round 2 walks all
// of W, later rounds only the items marked in the previous round's mask.
// Counts go to a per-workgroup LDS histogram first and reach the global
// counters once per (workgroup, leaf).
__global__ __launch_bounds__(256) void k_count(DevTree t, const uint4* batch, u32 n,
                                               u32 base_key, u32 round, u32 epoch) {
    __shared__ u32 lkey[kLds];
    __shared__ u32 lval[kLds];
    Counters* ctr = t.ctr;
    if (wg_skip(ctr, round)) return;
    for (u32 i = threadIdx.x; i < kLds; i += kWG) {
        lkey[i] = kNone;
        lval[i] = 0u;
    }
    __syncthreads();

    const u32 S = ctr->spill_count;
    const u32 nwork = round == 1u ? n : S + n;
    const uint8_t* prev = round >= 3u ? t.amask[(round - 1u) & 1u] : nullptr;
    uint8_t* mark = round >= 2u ? t.amask[round & 1u] : nullptr;
    const u32 open_epoch = epoch - 1u;

    const u32 step = gridDim.x * kWG;
    for (u32 base = xcd_block() * kWG; base < nwork; base += step) {
        const u32 j = base + threadIdx.x;
        u32 leaf = kNone;
        if (j < nwork && (!prev || prev[j])) {
            uint4 rec;
            u32 key, qx, qy, qz;
            fetch_work(t, batch, S, base_key, j, rec, key);
            quantize3(t, rec, qx, qy, qz);
            leaf = find_leaf(t, qx, qy, qz);
            if (round > 1u && t.birth[leaf] != open_epoch) leaf = kNone;
        }
        if (mark && j < nwork) mark[j] = leaf != kNone ? 1u : 0u;
        const Run r = lane_runs(leaf);
        if (leaf != kNone && r.rank == 0u) {
            if (!count_lds(lkey, lval, leaf, r.len)) count_global(t, leaf, r.len, round);
        }
    }
    __syncthreads();
    for (u32 e = threadIdx.x; e < kLds; e += kWG) {
        const u32 node = lkey[e];
        if (node != kNone) count_global(t, node, lval[e], round);
    }
}

// ---------------------------------------------------------------- splitting
// One workgroup per leaf counted this round.  A leaf whose stored plus
// counted points exceed T (and that is above Dmax) becomes inner: 8 empty
// children, a zeroed occupancy grid, its stored points and keys appended to
// the spill buffer and its chunks pushed to the pool.  Any other counted leaf
// is final for the pass and listed with its number of new points.
__global__ __launch_bounds__(256) void k_split(DevTree t, u32 round, u32 epoch) {
    __shared__ u32 s_dec[4];
    __shared__ i32 s_pool;
    Counters* ctr = t.ctr;
    if (wg_skip(ctr, round)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->touched_count[(round + 1u) & 1u] = 0u;
    u32 nt = min(ctr->touched_count[round & 1u], t.max_nodes);
    const u32* touched = t.touched[round & 1u];
    const u32 tid = threadIdx.x;
    for (u32 it = blockIdx.x; it < nt; it += gridDim.x) {
        u32 L = touched[it];
        if (tid == 0) {
            u32 c = t.cnt[L];
            u32 stored = t.count[L];
            u32 depth = t.geo[L].w;
            u32 split = 0u, first = 0u, gblk = 0u, sbase = 0u;
            if ((u64)stored + c > (u64)t.T && depth < t.Dmax) {
                first = atomicAdd(&ctr->node_count, 8u);
                if ((u64)first + 8u > (u64)t.max_nodes) {
                    set_status(t, SIMLOD_OVF_NODES);
                } else {
                    gblk = atomicAdd(&ctr->arena_top, t.grid_blocks);
                    if ((u64)gblk + t.grid_blocks > (u64)t.arena_blocks) {
                        set_status(t, SIMLOD_OVF_ARENA);
                    } else {
                        sbase = stored ? atomicAdd(&ctr->spill_count, stored) : 0u;
                        if ((u64)sbase + stored > (u64)t.spill_cap)
                            set_status(t, SIMLOD_OVF_SPILL);
                        else
                            split = 1u;
                    }
                }
            } else {
                u32 p = atomicAdd(&ctr->final_count, 1u);
                if (p < t.max_nodes)
                    t.final_list[p] = make_uint2(L, c);
                else
                    set_status(t, SIMLOD_OVF_WORK);
                t.cnt[L] = 0u;
            }
            s_dec[0] = split;
            s_dec[1] = first;
            s_dec[2] = gblk;
            s_dec[3] = sbase;
        }
        __syncthreads();
        if (s_dec[0]) {
            const u32 first = s_dec[1], gblk = s_dec[2], sbase = s_dec[3];
            const uint4 g = t.geo[L];
            const u32 depth = g.w;
            const u32 bit = t.K - 1u - depth;
            if (tid < 8u) {
                u32 nd = first + tid;
                t.child[nd] = 0u;
                t.count[nd] = 0u;
                t.cnt[nd] = 0u;
                t.birth[nd] = epoch;
                t.geo[nd] = make_uint4(g.x | ((tid & 1u) << bit), g.y | (((tid >> 1) & 1u) << bit),
                                       g.z | (((tid >> 2) & 1u) << bit), depth + 1u);
                t.grid[nd] = kNone;
                t.tab[nd] = kNone;
                t.tabcap[nd] = 0u;
                t.nchunks[nd] = 0u;
                t.newv[nd] = 0u;
            }
            uint4* gw = reinterpret_cast<uint4*>(block_ptr(t, gblk));
            const u32 n16 = t.grid_blocks * (kBlockBytes / 16u);
            for (u32 w = tid; w < n16; w += kWG) gw[w] = make_uint4(0u, 0u, 0u, 0u);
            const u32 stored = t.count[L];
            if (stored) {
                const u32* tab = table_of(t, L);
                for (u32 s = tid; s < stored; s += kWG) {
                    u32 ci = s / t.C;
                    u32 cb = tab[ci];
                    u32 o = s - ci * t.C;
                    t.spill_rec[sbase + s] = chunk_recs(t, cb)[o];
                    t.spill_key[sbase + s] = chunk_keys(t, cb)[o];
                }
                const u32 nch = t.nchunks[L];
                if (tid == 0) s_pool = atomicAdd(&ctr->pool_top, (i32)nch);
                __syncthreads();
                const i32 pb = s_pool;
                for (u32 j = tid; j < nch; j += kWG) {
                    if ((u64)pb + j < (u64)t.pool_cap) t.pool[pb + j] = tab[j];
                }
            }
            __syncthreads();
            if (tid == 0) {
                t.count[L] = 0u;
                t.nchunks[L] = 0u;
                t.grid[L] = gblk;
                t.cnt[L] = 0u;
                t.child[L] = first;
                ctr->split_any[round] = 1u;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- allocation
// One wavefront per listed node: the node needs ceil((old + added) / C)
// chunks in total (subsection "Allocating Chunks"); missing ones come from
// the pool first, then from the persistent buffer (section "Chunks and the
// Chunk Pool"), are appended to the node's chunk table (grown by doubling)
// and linked after its last chunk.
__global__ __launch_bounds__(256) void k_alloc(DevTree t, u32 voxels) {
    Counters* ctr = t.ctr;
    if (__builtin_amdgcn_readfirstlane(ctr->status)) return;  // wave-uniform
    u32 n = voxels ? ctr->vtouched_count : ctr->final_count;
    n = min(n, t.max_nodes);
    const u32 lane = lane_id();
    const u32 wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
    const u32 nwaves = gridDim.x * (kWG >> 6);
    for (u32 e = wave; e < n; e += nwaves) {
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

// ------------------------------------------------------- voxel claim table
// Inserts (node, cell) and min-reduces (key << 32 | rgba) into its value.
// Returns true for the call that created the entry.
__device__ __forceinline__ bool claim_cell(const DevTree& t, u64 tag, u64 val, u32& slot) {
    u32 h = (u32)mix64(tag) & t.hmask;
    for (u32 p = 0; p < kMaxProbe; ++p) {
        u64 cur = t.htag[h];
        if (cur == kEmptyTag)
            cur = atomicCAS((unsigned long long*)&t.htag[h], (unsigned long long)kEmptyTag,
                            (unsigned long long)tag);
        if (cur == kEmptyTag || cur == tag) {
            atomicMin((unsigned long long*)&t.hval[h], (unsigned long long)val);
            slot = h;
            return cur == kEmptyTag;
        }
        h = (h + 1u) & t.hmask;
    }
    set_status(t, SIMLOD_OVF_HASH);
    return false;
}

// ------------------------------------------------------- sample and store
// LDS tables of one workgroup (open addressing on u32 node ids).  The tables
// are sized above the number of distinct keys a workgroup can insert, except
// where a caller falls back to a global atomic when a table is full.
__device__ __forceinline__ u32 lds_find_or_insert(u32* keys, u32 bits, u32 key) {
    const u32 size = 1u << bits;
    u32 h = (key * 0x9E3779B1u) >> (32u - bits);
    for (u32 p = 0; p < size; ++p) {
        const u32 k = atomicCAS(&keys[h], kNone, key);
        if (k == kNone || k == key) return h;
        h = (h + 1u) & (size - 1u);
    }
    return kNone;
}

constexpr u32 kClaimBuf = 2048;  // claims staged per workgroup before one flush
constexpr u32 kSlotBits = 9;     // > 256 distinct leaves per tile
constexpr u32 kNodeBits = 8;     // inner nodes with new voxels per workgroup

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
__global__ __launch_bounds__(256) void k_sample_store(DevTree t, const uint4* batch, u32 n,
                                                      u32 base_key) {
    __shared__ u32 s_claims[kClaimBuf];
    __shared__ u32 s_lkey[1u << kSlotBits], s_lcnt[1u << kSlotBits], s_lbase[1u << kSlotBits];
    __shared__ u32 s_vkey[1u << kNodeBits], s_vcnt[1u << kNodeBits];
    __shared__ u32 s_nclaims, s_flush;
    Counters* ctr = t.ctr;
    if (wg_skip(ctr, 1u)) return;
    const u32 tid = threadIdx.x;
    for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
        s_lkey[i] = kNone;
        s_lcnt[i] = 0u;
    }
    for (u32 i = tid; i < (1u << kNodeBits); i += kWG) {
        s_vkey[i] = kNone;
        s_vcnt[i] = 0u;
    }
    if (tid == 0) s_nclaims = 0u;
    __syncthreads();

    const u32 S = ctr->spill_count;
    const u32 nwork = S + n;
    const u32 lane = lane_id();
    const u32 rmask = t.R - 1u;
    const u32 stripe = blockIdx.x % kStripes;
    const u32 step = gridDim.x * kWG;
    for (u32 base = xcd_block() * kWG; base < nwork; base += step) {
        const u32 j = base + tid;
        const bool valid = j < nwork;
        uint4 rec = make_uint4(0u, 0u, 0u, 0u);
        u32 key = 0u, qx = 0u, qy = 0u, qz = 0u;
        if (valid) {
            fetch_work(t, batch, S, base_key, j, rec, key);
            quantize3(t, rec, qx, qy, qz);
        }
        u32 node = 0u;
        bool desc = valid;
        for (u32 d = 0; d <= t.Dmax; ++d) {  // inner nodes exist only above Dmax
            const u32 c = desc && d < t.Dmax ? t.child[node] : 0u;
            const bool inner = desc && c != 0u;
            if (__ballot(inner) == 0ull) break;
            u64 tag = kEmptyTag;
            if (inner) {
                const u32 shift = t.Dmax - d;
                const u32 lin = ((qx >> shift) & rmask) | (((qy >> shift) & rmask) << t.r) |
                                (((qz >> shift) & rmask) << (2u * t.r));
                const u32 word = grid_of(t, node)[lin >> 5];
                if (!((word >> (lin & 31u)) & 1u)) tag = ((u64)node << 24) | lin;
            }
            const u64 ptag = __shfl_up(tag, 1);
            const u32 pkey = __shfl_up(key, 1);
            const bool cand = tag != kEmptyTag && !(lane > 0u && ptag == tag && pkey < key);
            bool fresh = false;
            u32 hslot = 0u;
            if (cand) fresh = claim_cell(t, tag, ((u64)key << 32) | (u64)rec.w, hslot);
            // stage the claim in LDS (one LDS atomic per wave)
            const u64 fm = __ballot(fresh);
            if (fm) {
                const int leader = __ffsll((long long)fm) - 1;
                u32 off = 0u;
                if ((int)lane == leader) off = atomicAdd(&s_nclaims, (u32)__popcll(fm));
                off = __shfl(off, leader) + (u32)__popcll(fm & lanes_below(lane));
                if (fresh) {
                    if (off < kClaimBuf) {
                        s_claims[off] = hslot;
                    } else {  // staging full: append straight to the stripe
                        const u32 pos = atomicAdd(&ctr->claim_count[stripe], 1u);
                        if (pos < t.claim_cap)
                            t.claims[(u64)stripe * t.claim_cap + pos] = hslot;
                        else
                            set_status(t, SIMLOD_OVF_BACKLOG);
                    }
                }
            }
            // count new voxels per node in LDS
            const Run vr = lane_runs(fresh ? node : kNone);
            if (fresh && vr.rank == 0u) {
                const u32 e = lds_find_or_insert(s_vkey, kNodeBits, node);
                if (e != kNone) {
                    atomicAdd(&s_vcnt[e], vr.len);
                } else if (atomicAdd(&t.newv[node], vr.len) == 0u) {
                    const u32 p = atomicAdd(&ctr->vtouched_count, 1u);
                    if (p < t.max_nodes)
                        t.vtouched[p] = node;
                    else
                        set_status(t, SIMLOD_OVF_WORK);
                }
            }
            if (inner)
                node = c + octant_of(qx, qy, qz, t.K - 1u - d);
            else
                desc = false;
        }
        // leaf slots: LDS histogram of the tile, one global atomic per leaf
        const u32 leaf = valid ? node : kNone;
        const Run r = lane_runs(leaf);
        u32 e = kNone, r0 = 0u;
        if (leaf != kNone && r.rank == 0u) {
            e = lds_find_or_insert(s_lkey, kSlotBits, leaf);  // never full: <= 256 keys
            r0 = atomicAdd(&s_lcnt[e], r.len);
        }
        e = __shfl(e, r.head);
        r0 = __shfl(r0, r.head) + r.rank;
        __syncthreads();
        for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
            const u32 k = s_lkey[i];
            if (k != kNone) s_lbase[i] = atomicAdd(&t.count[k], s_lcnt[i]);
        }
        __syncthreads();
        if (valid) {
            const u32 slot = s_lbase[e] + r0;
            const u32 ci = slot / t.C;
            if (ci < t.nchunks[leaf]) {
                const u32 cb = table_of(t, leaf)[ci];
                const u32 o = slot - ci * t.C;
                chunk_recs(t, cb)[o] = rec;
                chunk_keys(t, cb)[o] = key;
            } else {
                set_status(t, SIMLOD_OVF_ARENA);
            }
        }
        __syncthreads();
        for (u32 i = tid; i < (1u << kSlotBits); i += kWG) {
            s_lkey[i] = kNone;
            s_lcnt[i] = 0u;
        }
        __syncthreads();
    }
    // flush staged claims (one atomic per workgroup) and per-node counts
    const u32 nc = min(s_nclaims, kClaimBuf);
    if (tid == 0) s_flush = nc ? atomicAdd(&ctr->claim_count[stripe], nc) : 0u;
    __syncthreads();
    u32* dst = t.claims + (u64)stripe * t.claim_cap;
    for (u32 i = tid; i < nc; i += kWG) {
        const u32 pos = s_flush + i;
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
    }
}

// ------------------------------------------------------- voxel stores
// One thread per claimed cell: the voxel (cell centre, colour of the
// smallest-key point) goes to the node's next voxel slot, the cell's bit is
// set, and the claim-table entry is cleared for the next pass.
__global__ __launch_bounds__(256) void k_store_voxels(DevTree t) {
    Counters* ctr = t.ctr;
    if (__builtin_amdgcn_readfirstlane(ctr->status)) return;  // wave-uniform
    u32 pre[kStripes + 1];
    pre[0] = 0u;
    for (u32 s = 0; s < kStripes; ++s) pre[s + 1] = pre[s] + min(ctr->claim_count[s], t.claim_cap);
    const u32 n = pre[kStripes];
    const u32 rmask = t.R - 1u;
    const u32 step = gridDim.x * kWG;
    for (u32 base = blockIdx.x * kWG; base < n; base += step) {
        const u32 i = base + threadIdx.x;
        const bool valid = i < n;
        u32 h = 0u, node = kNone, lin = 0u;
        u64 val = 0ull;
        if (valid) {
            u32 s = 0;
            while (i >= pre[s + 1]) ++s;
            h = t.claims[(u64)s * t.claim_cap + (i - pre[s])];
            const u64 tag = t.htag[h];
            val = t.hval[h];
            node = (u32)(tag >> 24);
            lin = (u32)tag & 0xFFFFFFu;
        }
        const Run r = lane_runs(node);
        u32 sb = 0u;
        if (valid && r.rank == 0u) sb = atomicAdd(&t.count[node], r.len);
        sb = __shfl(sb, r.head);
        if (valid) {
            const u32 slot = sb + r.rank;
            const uint4 g = t.geo[node];
            const u32 d = g.w;
            const u32 shift = t.Dmax - d;
            const u32 cx = lin & rmask, cy = (lin >> t.r) & rmask, cz = lin >> (2u * t.r);
            uint4 v;
            v.x = __float_as_uint(cell_centre((g.x >> shift) + cx, t.mn[0], t.size, t.r, d));
            v.y = __float_as_uint(cell_centre((g.y >> shift) + cy, t.mn[1], t.size, t.r, d));
            v.z = __float_as_uint(cell_centre((g.z >> shift) + cz, t.mn[2], t.size, t.r, d));
            v.w = (u32)val;
            const u32 ci = slot / t.C;
            if (ci < t.nchunks[node]) {
                const u32 cb = table_of(t, node)[ci];
                const u32 o = slot - ci * t.C;
                chunk_recs(t, cb)[o] = v;
                chunk_keys(t, cb)[o] = (u32)(val >> 32);
            } else {
                set_status(t, SIMLOD_OVF_ARENA);
            }
            atomicOr(&grid_of(t, node)[lin >> 5], 1u << (lin & 31u));
            t.htag[h] = kEmptyTag;
            t.hval[h] = ~0ull;
        }
    }
}

// ------------------------------------------------------- bookkeeping
__global__ void k_finish(DevTree t) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Counters* c = t.ctr;
    if (c->status) return;
    if (c->pool_top < 0) c->pool_top = 0;
    u32 rounds = 1u;
    for (u32 k = 1; k <= (u32)kMaxRounds; ++k)
        if (c->split_any[k]) rounds = k + 1u;
    u32 claims = 0u;
    for (u32 k = 0; k < kStripes; ++k) claims += min(c->claim_count[k], t.claim_cap);
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
    c->final_count = 0u;
    c->vtouched_count = 0u;
    for (u32 k = 0; k < kStripes; ++k) c->claim_count[k] = 0u;
    c->touched_count[0] = c->touched_count[1] = 0u;
    for (u32 k = 0; k < (u32)kMaxRounds + 2u; ++k) c->split_any[k] = 0u;
}

// ------------------------------------------------------- reset / export
__global__ void k_fill_u64(u64* p, u64 n, u64 v) {
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
        p[i] = v;
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
    t.birth[0] = 0u;
    t.geo[0] = make_uint4(0u, 0u, 0u, 0u);
    t.grid[0] = kNone;
    t.tab[0] = kNone;
    t.tabcap[0] = 0u;
    t.nchunks[0] = 0u;
    t.newv[0] = 0u;
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
            const u32 ci = s / t.C;
            const u32 cb = tab[ci];
            const u32 o = s - ci * t.C;
            out_rec[f + s] = chunk_recs(t, cb)[o];
            out_key[f + s] = chunk_keys(t, cb)[o];
        }
    }
}

// ------------------------------------------------------- host launchers
static inline u32 grid_for(u64 items, u32 lo, u32 hi) {
    u64 g = (items + kWG - 1) / kWG;
    if (g < lo) g = lo;
    if (g > hi) g = hi;
    return (u32)((g + 7u) & ~7ull);
}

hipError_t launch_count(const DevTree& t, const uint4* batch, u32 n, u32 base_key, u32 round,
                        u32 epoch, hipStream_t s) {
    u32 g = round == 1u ? grid_for(n, 8, 4096) : (round == 2u ? grid_for(n, 64, 2048)
                                                            : grid_for(n / 4u, 32, 512));
    hipLaunchKernelGGL(k_count, dim3(g), dim3(kWG), 0, s, t, batch, n, base_key, round, epoch);
    return hipGetLastError();
}
hipError_t launch_split(const DevTree& t, u32 round, u32 epoch, u32 n, hipStream_t s) {
    u32 g = round == 1u ? grid_for((u64)n / 64u, 64, 1024) : 256u;
    hipLaunchKernelGGL(k_split, dim3(g), dim3(kWG), 0, s, t, round, epoch);
    return hipGetLastError();
}
hipError_t launch_alloc(const DevTree& t, u32 voxels, hipStream_t s) {
    hipLaunchKernelGGL(k_alloc, dim3(256), dim3(kWG), 0, s, t, voxels);
    return hipGetLastError();
}
hipError_t launch_sample_store(const DevTree& t, const uint4* batch, u32 n, u32 base_key,
                               hipStream_t s) {
    u32 g = grid_for((u64)n + 4096u, 64, 4096);
    hipLaunchKernelGGL(k_sample_store, dim3(g), dim3(kWG), 0, s, t, batch, n, base_key);
    return hipGetLastError();
}
hipError_t launch_store_voxels(const DevTree& t, u32 n, hipStream_t s) {
    u32 g = grid_for(n, 64, 2048);
    hipLaunchKernelGGL(k_store_voxels, dim3(g), dim3(kWG), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_finish(const DevTree& t, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_reset(const DevTree& t, u64 hash_entries, hipStream_t s) {
    u32 g = (u32)std::min<u64>((hash_entries + kWG - 1) / kWG, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kWG), 0, s, t.htag, hash_entries, kEmptyTag);
    hipLaunchKernelGGL(k_fill_u64, dim3(g), dim3(kWG), 0, s, t.hval, hash_entries, ~0ull);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_gather(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                         uint4* out_rec, u32* out_key, hipStream_t s) {
    u32 g = std::min<u32>(std::max<u32>(nn, 1u), 4096u);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kWG), 0, s, t, nodes, first, nn, out_rec, out_key);
    return hipGetLastError();
}

}  // namespace simlod
