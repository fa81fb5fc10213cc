// Host side of the C ABI declared in include/simlod.h: creation, the launch
// sequence of one insertion pass, canonical export, counters, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "launch.hpp"
#include "octree_device.hpp"
#include "simlod.h"

using namespace simlod;

// Per-kernel HIP-event timing of the passes a handle or group enqueues.
struct Timing {
    uint32_t mask = 0;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    simlod_kernel_times acc;
};

struct simlod_octree {
    simlod_config cfg;
    DevTree t;
    DevTree* d_tree = nullptr;   // device copy of t, read by the kernels
    Member* d_members = nullptr; // the handle's one-member table for its own passes
    int device = 0;
    u64 hash_entries = 0;
    u64 total_points = 0;
    u64 passes = 0;
    u32 epoch = 1;
    int poisoned = 0;
    int sticky = SIMLOD_OK;
    u32* h_status = nullptr;  // pinned host copy of the device status word
    hipEvent_t status_ev = nullptr;
    bool status_pending = false;
    hipStream_t last_stream = nullptr;
    bool has_work = false;             // work was enqueued on last_stream
    hipEvent_t order_ev = nullptr;     // orders a new stream after last_stream
    uint4* staging = nullptr;
    u64 staging_cap = 0;
    std::vector<void*> dev_allocs;
    LaunchShape shape = default_shape();
    Timing tm;
    u64 dev_bytes = 0;     // device memory held
    u64* dry = nullptr;    // set: dalloc only adds up sizes
    simlod_config alloc_cfg{};  // the configuration its buffers were sized for
};

namespace {

// Events that only order streams of one device need no system-scope fence.
constexpr unsigned kOrderingEvent = hipEventDisableTiming | hipEventDisableSystemFence;

thread_local char g_last_error[512] = "";

void note_error(const char* what, hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e),
                  (int)e);
}

// Any error left by earlier HIP calls of the process (torch's included) would
// otherwise be reported by the next hipGetLastError after our own launches.
void clear_stale_error() { (void)hipGetLastError(); }

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard() {
        if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }

  private:
    int prev_ = -1, dev_ = 0;
};

template <typename T>
bool dalloc(simlod_octree* h, T** p, u64 count) {
    void* v = nullptr;
    u64 bytes = std::max<u64>(count * sizeof(T), 256);
    if (h->dry) {  // sizing only
        *h->dry += bytes;
        *p = nullptr;
        return true;
    }
    h->dev_bytes += bytes;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
        note_error("hipMalloc", e);
        return false;
    }
    h->dev_allocs.push_back(v);
    *p = (T*)v;  // a C-style cast: T may carry the device address space
    return true;
}

u64 next_pow2(u64 v) {
    u64 p = 1;
    while (p < v) p <<= 1;
    return p;
}

u32 bit_length(u64 v) {
    u32 b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Bits of a cell identity node << 3r | cell.
u32 tag_bits_for(const simlod_config* c) {
    return bit_length((u64)c->max_nodes - 1u) + 3u * c->grid_bits;
}

// Claim-table entries: twice the backlog (at least one 8-entry bucket), and
// enough that a cell identity's bits beyond the table index fit the claim
// word's tag (kRemBits).
u64 hash_entries_for(const simlod_config* c) {
    u64 e = std::max<u64>(next_pow2(2 * c->backlog_capacity), 8u);
    const u32 tb = tag_bits_for(c);
    if (tb > kRemBits) e = std::max<u64>(e, 1ull << (tb - kRemBits));
    return e;
}

bool cfg_valid(const simlod_config* c) {
    if (c->grid_bits > 8 || c->max_depth > 21 || c->grid_bits + c->max_depth > 24) return false;
    if (c->max_depth + 1 > (u32)kMaxRounds) return false;
    if (c->leaf_capacity < 1 || c->chunk_capacity < 1 || c->chunk_capacity > (1u << 24)) return false;
    if (c->max_nodes < 9 || c->max_nodes > (1u << 31)) return false;
    if (!(c->root_size > 0.0f) || std::isinf(c->root_size)) return false;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->root_min[a])) return false;
    if (c->max_batch < 1 || c->max_batch > 0xFFFFFFFFull) return false;
    if (c->spill_capacity > 0xFFFFFFFFull || c->max_batch + c->spill_capacity > 0xFFFFFFFFull)
        return false;
    if (c->backlog_capacity < 1 || c->backlog_capacity > (1ull << 31)) return false;
    if (c->hist_capacity > (1u << 31) / kHistEntries) return false;
    // a caller-owned persistent buffer: a size, and block alignment
    if (c->arena_ptr && (c->arena_bytes < kBlockBytes ||
                         reinterpret_cast<uintptr_t>(c->arena_ptr) % kBlockBytes))
        return false;
    return true;
}

void free_timing(Timing& tm) {
    for (auto& p : tm.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : tm.free_events) (void)hipEventDestroy(e);
    tm.pending.clear();
    tm.free_events.clear();
}

void free_all(simlod_octree* h) {
    for (void* p : h->dev_allocs) (void)hipFree(p);
    h->dev_allocs.clear();
    if (h->h_status) (void)hipHostFree(h->h_status);
    h->h_status = nullptr;
    if (h->status_ev) (void)hipEventDestroy(h->status_ev);
    if (h->order_ev) (void)hipEventDestroy(h->order_ev);
    free_timing(h->tm);
}

// Reads the status word copied after the last pass.  wait: block until it
// has arrived; otherwise only look if the copy already completed.
int poll_status(simlod_octree* h, bool wait) {
    if (h->poisoned) return SIMLOD_ERR_POISONED;
    if (h->status_pending) {
        hipError_t e = wait ? hipEventSynchronize(h->status_ev) : hipEventQuery(h->status_ev);
        if (e == hipErrorNotReady) return SIMLOD_OK;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->poisoned = 1;
            h->sticky = SIMLOD_ERR_HIP;
            return SIMLOD_ERR_HIP;
        }
        h->status_pending = false;
        if (*h->h_status) {
            h->poisoned = 1;
            h->sticky = SIMLOD_ERR_CAPACITY;
            return SIMLOD_ERR_CAPACITY;
        }
    }
    return SIMLOD_OK;
}

// Orders stream s after everything enqueued on the handle so far: a call on
// another stream than the previous call's waits for that stream's work (the
// passes share the octree's counters, claim table, spill buffers and staging
// buffer).  Then s becomes the handle's stream.
hipError_t order_after_last(simlod_octree* h, hipStream_t s) {
    if (h->has_work && h->last_stream != s) {
        hipError_t e = hipEventRecord(h->order_ev, h->last_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, h->order_ev, 0);
        if (e != hipSuccess) return e;
    }
    h->last_stream = s;
    h->has_work = true;
    return hipSuccess;
}

hipEvent_t take_event(Timing& tm) {
    if (!tm.free_events.empty()) {
        hipEvent_t e = tm.free_events.back();
        tm.free_events.pop_back();
        return e;
    }
    // Timing only: without the system-scope fence an event costs no L2
    // writeback and invalidation (several microseconds of idle GPU, and a
    // cold L2 for the next kernel).
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}

template <typename F>
hipError_t timed(Timing* tm, int kind, hipStream_t s, F&& launch) {
    if (!tm || !((tm->mask >> kind) & 1u)) return launch();
    hipEvent_t a = take_event(*tm), b = take_event(*tm);
    (void)hipEventRecord(a, s);
    hipError_t e = launch();
    (void)hipEventRecord(b, s);
    tm->pending.push_back({kind, a, b});
    return e;
}

void drain_timing(Timing& tm) {
    for (auto& p : tm.pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            tm.acc.launches[p.kind] += 1;
            tm.acc.total_ms[p.kind] += ms;
        }
        tm.free_events.push_back(p.a);
        tm.free_events.push_back(p.b);
    }
    tm.pending.clear();
}

bool is_device_ptr(const void* p) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// One insertion pass over a group of octrees, each member's share of at most
// its max_batch device-resident points (a single octree is a group of one).
// items: batch points summed over the members (for a captured pass: their
// capacity); rounds: the largest member's expansion rounds; tm: timing (may
// be null); status_out: per-member status words (may be null).
hipError_t enqueue_group_pass(const GroupArgs& ga, u64 items, u32 rounds, const LaunchShape& sh,
                              Timing* tm, u32* status_out, hipStream_t s) {
    const Member* M = ga.table;
    const u32 cnt = ga.count;
    hipError_t e = timed(tm, SIMLOD_KERNEL_COUNT, s,
                         [&] { return launch_count_leaves(ga, items, sh, s); });
    if (e == hipSuccess)
        e = timed(tm, SIMLOD_KERNEL_SPLIT, s, [&] { return launch_split_leaves(M, cnt, items, s); });
    if (e == hipSuccess && cnt == 1u && items >= kGroupMinItems)
        e = timed(tm, SIMLOD_KERNEL_GROUP_BATCH, s,
                  [&] { return launch_group_batch(M, cnt, items, sh, s); });
    if (rounds >= 2u && e == hipSuccess) {
        e = timed(tm, SIMLOD_KERNEL_COUNT_HIST, s,
                  [&] { return launch_count_hist(M, cnt, items, 2u, sh, s); });
        if (e == hipSuccess)
            e = timed(tm, SIMLOD_KERNEL_BUILD, s, [&] { return launch_build(M, cnt, 2u, s); });
    }
    // the rare later rounds share the leaves' chunk allocation's launch
    if (e == hipSuccess)
        e = timed(tm, SIMLOD_KERNEL_ALLOC_POINTS, s,
                  [&] { return launch_rounds_alloc(M, cnt, items, 3u, rounds, s); });
    if (e == hipSuccess)
        e = timed(tm, SIMLOD_KERNEL_SAMPLE_STORE, s,
                  [&] { return launch_sample_store(M, cnt, items, sh, s); });
    if (e == hipSuccess)
        e = timed(tm, SIMLOD_KERNEL_ALLOC_VOXELS, s, [&] { return launch_alloc(M, cnt, 1u, s); });
    if (e == hipSuccess)
        e = timed(tm, SIMLOD_KERNEL_STORE_VOXELS, s,
                  [&] { return launch_store_voxels(M, cnt, items, sh, s); });
    if (e == hipSuccess && status_out)  // a group's status words for the host
        e = timed(tm, SIMLOD_KERNEL_FINISH, s,
                  [&] { return launch_finish(M, cnt, status_out, s); });
    return e;
}

// One pass of a single handle over n <= max_batch device-resident points.
hipError_t enqueue_pass(simlod_octree* h, const uint4* batch, u32 n, u32 base_key, hipStream_t s) {
    GroupArgs ga{};
    ga.table = h->d_members;
    ga.count = 1;
    ga.m[0] = make_member(h->d_tree, batch, n, base_key);
    hipError_t e = enqueue_group_pass(ga, n, expansion_rounds(h->cfg.max_depth), h->shape, &h->tm,
                                      nullptr, s);
    // At most one status copy in flight: the status word is sticky, so a
    // later copy reports every earlier error, and a copy with its event
    // (a system-scope fence) per pass would cost more than a short kernel.
    if (e == hipSuccess && !h->status_pending) {
        e = hipMemcpyAsync(h->h_status, &h->t.ctr->status, sizeof(u32), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(h->status_ev, s);
        if (e == hipSuccess) h->status_pending = true;
    }
    return e;
}

struct HostNodes {
    std::vector<u32> child, count, nchunks;
    std::vector<uint4> geo;
    Counters ctr;
};

int read_nodes(simlod_octree* h, HostNodes& hn, bool full) {
    if (hipMemcpy(&hn.ctr, h->t.ctr, sizeof(Counters), hipMemcpyDeviceToHost) != hipSuccess)
        return SIMLOD_ERR_HIP;
    u32 nn = std::min(hn.ctr.node_count, h->t.max_nodes);
    hn.child.resize(nn);
    hn.count.resize(nn);
    if (hipMemcpy(hn.child.data(), h->t.child, nn * 4ull, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hn.count.data(), h->t.count, nn * 4ull, hipMemcpyDeviceToHost) != hipSuccess)
        return SIMLOD_ERR_HIP;
    if (full) {
        hn.nchunks.resize(nn);
        hn.geo.resize(nn);
        if (hipMemcpy(hn.nchunks.data(), h->t.nchunks, nn * 4ull, hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(hn.geo.data(), h->t.geo, nn * 16ull, hipMemcpyDeviceToHost) != hipSuccess)
            return SIMLOD_ERR_HIP;
    }
    return SIMLOD_OK;
}

int sync_handle(simlod_octree* h) {
    const hipError_t e = hipStreamSynchronize(h->last_stream);
    if (e != hipSuccess) {
        note_error("hipStreamSynchronize", e);
        clear_stale_error();
        h->poisoned = 1;
        h->sticky = SIMLOD_ERR_HIP;
        return SIMLOD_ERR_HIP;
    }
    const int rc = poll_status(h, true);
    if (rc) return rc;
    // group passes leave no host copy of the status word: read it
    u32 st = 0;
    if (hipMemcpy(&st, &h->t.ctr->status, sizeof(u32), hipMemcpyDeviceToHost) != hipSuccess) {
        note_error("status read", hipGetLastError());
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    if (st) {
        h->poisoned = 1;
        h->sticky = SIMLOD_ERR_CAPACITY;
        return SIMLOD_ERR_CAPACITY;
    }
    return SIMLOD_OK;
}

}  // namespace

// Every device buffer of an octree (the same sequence sizes a configuration
// when h->dry is set).  arena_bytes: 0 = 90% of the free memory.
// Sets every scalar of the handle's DevTree (capacities, geometry, derived
// sizes) from *cfg; the buffer pointers stay.  arena_bytes: the arena size
// to use.
static void configure_tree(simlod_octree* h, const simlod_config* cfg, u64 arena_bytes) {
    DevTree& t = h->t;
    h->cfg = *cfg;
    h->hash_entries = hash_entries_for(cfg);
    t.dir_depth = std::min<u32>(cfg->max_depth, kDirMaxDepth);
    t.max_nodes = cfg->max_nodes;
    t.hist_cap = cfg->hist_capacity ? cfg->hist_capacity : 8192u;
    t.spill_cap = (u32)cfg->spill_capacity;
    t.active_cap = (u32)(cfg->max_batch + cfg->spill_capacity);
    t.hmask = (u32)(h->hash_entries - 1);
    t.hash_bits = bit_length(h->hash_entries) - 1u;
    t.tag_bits = tag_bits_for(cfg);
    t.claim_cap = (u32)cfg->backlog_capacity;
    const u64 chunk_bytes = (u64)cfg->chunk_capacity * 20u + 4u;
    t.chunk_blocks = (u32)((chunk_bytes + kBlockBytes - 1) / kBlockBytes);
    const u64 cells = 1ull << (3 * cfg->grid_bits);
    t.grid_words = (u32)std::max<u64>(1, cells / 32);
    t.grid_blocks = (u32)((t.grid_words * 4ull + kBlockBytes - 1) / kBlockBytes);
    t.arena_blocks = (u32)std::min<u64>(arena_bytes / kBlockBytes, 0xFFFFFFF0ull);
    t.pool_cap = t.arena_blocks / t.chunk_blocks + 1;
    for (int a = 0; a < 3; ++a) t.mn[a] = cfg->root_min[a];
    t.size = cfg->root_size;
    t.K = cfg->max_depth + cfg->grid_bits;
    t.r = cfg->grid_bits;
    t.R = 1u << cfg->grid_bits;
    t.Dmax = cfg->max_depth;
    t.T = cfg->leaf_capacity;
    t.C = cfg->chunk_capacity;
    t.c_magic = t.C == 1u ? 0ull : ~0ull / t.C + 1ull;
    t.scale = (float)(1u << t.K) / cfg->root_size;  // float32 division
}

// Element counts of every buffer a configuration needs; a handle allocated
// for A can serve B when each of B's counts is at most A's.
struct Footprint {
    u64 v[9];
};

static Footprint footprint_of(const simlod_config* c) {
    const u64 chunk_bytes = (u64)c->chunk_capacity * 20u + 4u;
    const u64 chunk_blocks = (chunk_bytes + kBlockBytes - 1) / kBlockBytes;
    const u64 arena_blocks = std::min<u64>(c->arena_bytes / kBlockBytes, 0xFFFFFFF0ull);
    Footprint f;
    f.v[0] = c->max_nodes;
    f.v[1] = dir_offset(std::min<u32>(c->max_depth, kDirMaxDepth) + 1u);
    f.v[2] = c->spill_capacity;
    f.v[3] = c->hist_capacity ? c->hist_capacity : 8192u;
    f.v[4] = c->max_batch + c->spill_capacity;
    f.v[5] = hash_entries_for(c);
    f.v[6] = c->backlog_capacity * kStripes;
    f.v[7] = arena_blocks;
    f.v[8] = arena_blocks / chunk_blocks + 1;
    return f;
}

static bool footprint_fits(const Footprint& have, const Footprint& need) {
    for (int i = 0; i < 9; ++i)
        if (need.v[i] > have.v[i]) return false;
    return true;
}

static bool allocate_all(simlod_octree* h, const simlod_config* cfg, u64 arena_bytes) {
    DevTree& t = h->t;
    std::memset(&t, 0, sizeof(t));
    const u64 N = cfg->max_nodes;
    const u64 work = cfg->max_batch + cfg->spill_capacity;
    h->hash_entries = hash_entries_for(cfg);
    t.dir_depth = std::min<u32>(cfg->max_depth, kDirMaxDepth);
    const u32 hist_slots = cfg->hist_capacity ? cfg->hist_capacity : 8192u;
    bool ok = dalloc(h, &t.child, N) && dalloc(h, &t.count, N) && dalloc(h, &t.cnt, N) &&
              dalloc(h, &t.hslot, N) && dalloc(h, &t.geo, N) && dalloc(h, &t.grid, N) &&
              dalloc(h, &t.tab, N) && dalloc(h, &t.tabcap, N) && dalloc(h, &t.nchunks, N) &&
              dalloc(h, &t.newv, N) && dalloc(h, &t.ctr, 1) &&
              dalloc(h, &t.dir, dir_offset(t.dir_depth + 1u)) &&
              dalloc(h, &t.spill_rec, cfg->spill_capacity) &&
              dalloc(h, &t.spill_key, cfg->spill_capacity) &&
              dalloc(h, &t.spill_job, N) && dalloc(h, &t.touched, N) &&
              dalloc(h, &t.pending[0], N) && dalloc(h, &t.pending[1], N) &&
              dalloc(h, &t.hist, (u64)hist_slots * kHistEntries) && dalloc(h, &t.final_list, N) &&
              dalloc(h, &t.vtouched, N) && dalloc(h, &t.amask[0], work) &&
              dalloc(h, &t.amask[1], work) && dalloc(h, &t.item_leaf, cfg->max_batch) &&
              (cfg->max_batch < kGroupMinItems ||
               (dalloc(h, &t.grp_rec, cfg->max_batch) && dalloc(h, &t.grp_index, cfg->max_batch) &&
                dalloc(h, &t.grp_leaf, cfg->max_batch) && dalloc(h, &t.bcnt, kBuckets) &&
                dalloc(h, &t.bnext, kBuckets) && dalloc(h, &t.bsum, kBuckets / kBucketChunk))) &&
              dalloc(h, &t.hent, 2 * h->hash_entries) &&
              dalloc(h, &t.claims, cfg->backlog_capacity * kStripes) &&
              dalloc(h, &h->d_tree, 1) && dalloc(h, &h->d_members, 2);  // + pass barrier words
    const u32 C = cfg->chunk_capacity;
    const u64 chunk_bytes = (u64)C * 20u + 4u;
    t.chunk_blocks = (u32)((chunk_bytes + kBlockBytes - 1) / kBlockBytes);
    const u64 cells = 1ull << (3 * cfg->grid_bits);
    t.grid_words = (u32)std::max<u64>(1, cells / 32);
    t.grid_blocks = (u32)((t.grid_words * 4ull + kBlockBytes - 1) / kBlockBytes);
    if (arena_bytes == 0) arena_bytes = cfg->arena_bytes;
    if (ok && arena_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) ok = false;
        // pool entries need 4 bytes per chunk of the arena as well
        arena_bytes = (u64)((double)fr * 0.9 * (double)chunk_bytes / (double)(chunk_bytes + 4));
    }
    u64 blocks = std::min<u64>(arena_bytes / kBlockBytes, 0xFFFFFFF0ull);
    t.arena_blocks = (u32)blocks;
    t.pool_cap = t.arena_blocks / t.chunk_blocks + 1;
    if (cfg->arena_ptr) {  // the caller's buffer: used, never freed
        if (!h->dry) t.arena = (GPtr<uint8_t>)cfg->arena_ptr;
        ok = ok && blocks > 0 && dalloc(h, &t.pool, t.pool_cap);
    } else {
        ok = ok && blocks > 0 && dalloc(h, &t.arena, blocks * (u64)kBlockBytes) &&
             dalloc(h, &t.pool, t.pool_cap);
    }
    return ok;
}

// A caller-owned persistent buffer must be device memory of `device`.
static bool arena_ptr_ok(const void* p, int device) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice && attr.device == device;
}

extern "C" {

int simlod_default_config(simlod_config* cfg) {
    if (!cfg) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->root_min[0] = cfg->root_min[1] = cfg->root_min[2] = 0.0f;
    cfg->root_size = 1.0f;
    cfg->leaf_capacity = 50000;
    cfg->grid_bits = 7;
    cfg->max_depth = 16;
    cfg->chunk_capacity = 1000;
    cfg->max_nodes = 1u << 20;
    cfg->hist_capacity = 8192;
    cfg->arena_bytes = 0;
    cfg->max_batch = 10000000ull;
    cfg->spill_capacity = 16000000ull;
    cfg->backlog_capacity = 10000000ull;
    cfg->device = 0;
    return SIMLOD_OK;
}

int simlod_create(const simlod_config* cfg, simlod_octree** out) {
    if (!cfg || !out || !cfg_valid(cfg)) return SIMLOD_ERR_INVALID_ARGUMENT;
    clear_stale_error();
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev == 0) {
        note_error("hipGetDeviceCount", de);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    if (cfg->device < 0 || cfg->device >= ndev) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(cfg->device);
    if (cfg->arena_ptr && !arena_ptr_ok(cfg->arena_ptr, cfg->device)) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "arena_ptr is not device memory of device %d", cfg->device);
        return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    simlod_octree* h = new (std::nothrow) simlod_octree();
    if (!h) return SIMLOD_ERR_OUT_OF_MEMORY;
    h->cfg = *cfg;
    h->device = cfg->device;
    std::memset(&h->tm.acc, 0, sizeof(h->tm.acc));
    bool ok = allocate_all(h, cfg, 0);
    if (ok && hipHostMalloc((void**)&h->h_status, sizeof(u32), hipHostMallocDefault) != hipSuccess)
        ok = false;
    if (ok && hipEventCreateWithFlags(&h->status_ev, hipEventDisableTiming) != hipSuccess)
        ok = false;
    if (ok && hipEventCreateWithFlags(&h->order_ev, kOrderingEvent) != hipSuccess) ok = false;
    if (!ok) {
        std::snprintf(g_last_error, sizeof(g_last_error), "device allocation failed (%s)",
                      hipGetErrorString(hipGetLastError()));
        free_all(h);
        delete h;
        return SIMLOD_ERR_OUT_OF_MEMORY;
    }
    *h->h_status = 0;
    DevTree& t = h->t;
    configure_tree(h, cfg, (u64)t.arena_blocks * kBlockBytes);
    h->alloc_cfg = *cfg;
    h->alloc_cfg.arena_bytes = (u64)t.arena_blocks * kBlockBytes;
    clear_stale_error();
    hipError_t re = hipMemcpy(h->d_tree, &t, sizeof(DevTree), hipMemcpyHostToDevice);
    if (re != hipSuccess) note_error("device tree copy", re);
    // a fresh persistent buffer starts all zero (the reset clears only what
    // earlier passes used: below the bump pointer, zero here)
    if (re == hipSuccess) re = hipMemset(t.ctr, 0, sizeof(Counters));
    if (re == hipSuccess) re = hipMemset(t.arena, 0, (u64)t.arena_blocks * kBlockBytes);
    if (re != hipSuccess) note_error("initial clear", re);
    if (re == hipSuccess) re = launch_reset(t, h->hash_entries, nullptr);
    if (re != hipSuccess) note_error("reset kernels (launch)", re);
    if (re == hipSuccess) {
        re = hipStreamSynchronize(nullptr);
        if (re != hipSuccess) note_error("reset kernels (execution)", re);
    }
    if (re != hipSuccess) {
        clear_stale_error();
        free_all(h);
        delete h;
        return SIMLOD_ERR_HIP;
    }
    *out = h;
    return SIMLOD_OK;
}

int simlod_insert_batch(simlod_octree* h, const simlod_point* pts, uint64_t n, void* stream) {
    if (!h || (n && !pts)) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    int rc = poll_status(h, false);
    if (rc) return rc;
    if (n == 0) return SIMLOD_OK;
    clear_stale_error();
    if (h->total_points + n > 0xFFFFFFFFull) return SIMLOD_ERR_KEY_SPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool dev = is_device_ptr(pts);
    if (dev && (reinterpret_cast<uintptr_t>(pts) & 15u)) return SIMLOD_ERR_INVALID_ARGUMENT;
    const u64 maxb = h->cfg.max_batch;
    const hipError_t oe = order_after_last(h, s);
    if (oe != hipSuccess) {
        note_error("stream ordering", oe);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    if (!dev && h->staging_cap < std::min<u64>(n, maxb)) {
        if (h->staging) {
            (void)hipStreamSynchronize(h->last_stream);
            (void)hipFree(h->staging);
            h->staging = nullptr;
            h->staging_cap = 0;
        }
        u64 cap = std::min<u64>(std::max<u64>(n, 1u << 20), maxb);
        if (hipMalloc((void**)&h->staging, cap * 16ull) != hipSuccess) {
            (void)hipGetLastError();
            return SIMLOD_ERR_OUT_OF_MEMORY;
        }
        h->staging_cap = cap;
    }
    u64 done = 0;
    while (done < n) {
        const u64 m = std::min<u64>(n - done, maxb);
        const uint4* src = reinterpret_cast<const uint4*>(pts + done);
        if (!dev) {
            const hipError_t ce = hipMemcpyAsync(h->staging, src, m * 16ull, hipMemcpyHostToDevice, s);
            if (ce != hipSuccess) {
                note_error("host-to-device copy", ce);
                clear_stale_error();
                return SIMLOD_ERR_HIP;
            }
            src = h->staging;
        }
        const hipError_t pe = enqueue_pass(h, src, (u32)m, (u32)h->total_points, s);
        if (pe != hipSuccess) {
            note_error("insertion pass launch", pe);
            clear_stale_error();
            h->poisoned = 1;
            h->sticky = SIMLOD_ERR_HIP;
            return SIMLOD_ERR_HIP;
        }
        h->total_points += m;
        h->passes += 1;
        done += m;
    }
    return SIMLOD_OK;
}

}  // extern "C"

// ------------------------------------------------ static staging (no allocation)
// simlod_insert_batch_static stages host input through this array instead of
// a buffer the library allocates.  In host code `scratch` names only a
// host-side stand-in: its device address, one per device (each device holds
// its own copy of the array until the process ends), comes from
// hipGetSymbolAddress at the device's first call and is what the copies and
// kernels use.
constexpr u64 kStaticStageRecords = 1ull << 20;  // 16 MiB: 1,048,576 points
static __device__ __align__(256) uint4 scratch[kStaticStageRecords];

namespace {

constexpr int kMaxStageDevices = 64;

struct StaticStage {
    std::mutex mu;
    bool ready = false;
    uint4* ptr = nullptr;             // device address of `scratch` on this device
    hipEvent_t free_ev = nullptr;     // after the last pass that read it
    bool used = false;
};
StaticStage g_stage[kMaxStageDevices];

// Set-up of device `dev` (current): the array's device address and the
// event that orders later calls after the passes reading it.  Lock held.
hipError_t stage_setup(StaticStage& st) {
    if (st.ready) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&st.free_ev, kOrderingEvent);
    if (e != hipSuccess) return e;
    st.ptr = static_cast<uint4*>(p);
    st.ready = true;
    return hipSuccess;
}

// Passes over n device-resident points at src, cut at max_batch.
int enqueue_passes(simlod_octree* h, const uint4* src, u64 n, hipStream_t s) {
    const u64 maxb = h->cfg.max_batch;
    for (u64 done = 0; done < n;) {
        const u64 m = std::min<u64>(n - done, maxb);
        const hipError_t pe = enqueue_pass(h, src + done, (u32)m, (u32)h->total_points, s);
        if (pe != hipSuccess) {
            note_error("insertion pass launch", pe);
            clear_stale_error();
            h->poisoned = 1;
            h->sticky = SIMLOD_ERR_HIP;
            return SIMLOD_ERR_HIP;
        }
        h->total_points += m;
        h->passes += 1;
        done += m;
    }
    return SIMLOD_OK;
}

}  // namespace

extern "C" {

int simlod_insert_batch_static(simlod_octree* h, const simlod_point* pts, uint64_t n,
                               void* stream) {
    if (!h || (n && !pts)) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    int rc = poll_status(h, false);
    if (rc) return rc;
    if (n == 0) return SIMLOD_OK;
    clear_stale_error();
    if (h->total_points + n > 0xFFFFFFFFull) return SIMLOD_ERR_KEY_SPACE;
    if (h->device < 0 || h->device >= kMaxStageDevices) return SIMLOD_ERR_INVALID_ARGUMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool dev = is_device_ptr(pts);
    if (dev && (reinterpret_cast<uintptr_t>(pts) & 15u)) return SIMLOD_ERR_INVALID_ARGUMENT;
    if (!dev && n > kStaticStageRecords) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "host input of %llu points exceeds the static staging buffer (%llu points)",
                      (unsigned long long)n, (unsigned long long)kStaticStageRecords);
        return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    hipError_t e = order_after_last(h, s);
    if (e != hipSuccess) {
        note_error("stream ordering", e);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    if (dev) return enqueue_passes(h, reinterpret_cast<const uint4*>(pts), n, s);
    StaticStage& st = g_stage[h->device];
    std::lock_guard<std::mutex> lk(st.mu);
    e = stage_setup(st);
    if (e != hipSuccess) {
        note_error("static staging set-up", e);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    // the previous call's passes on this device must have read the array
    if (st.used) e = hipStreamWaitEvent(s, st.free_ev, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(st.ptr, pts, n * 16ull, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        note_error("host-to-device copy", e);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    rc = enqueue_passes(h, st.ptr, n, s);
    e = hipEventRecord(st.free_ev, s);
    if (e != hipSuccess) {
        note_error("static staging event", e);
        clear_stale_error();
        return rc ? rc : SIMLOD_ERR_HIP;
    }
    st.used = true;
    return rc;
}

int simlod_sync(simlod_octree* h) {
    if (!h) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    if (h->poisoned) return SIMLOD_ERR_POISONED;
    return sync_handle(h);
}

namespace {

// Canonical export of the subtree rooted at the node with `root_path`;
// linked: read every node through its chunk list instead of its chunk table;
// single: that node alone, without its descendants.
int export_subtree(simlod_octree* h, u64 root_path, simlod_snapshot_buffers* s,
                   bool linked = false, bool single = false) {
    if (!h || !s) return SIMLOD_ERR_INVALID_ARGUMENT;
    const int nulls = (s->nodes == nullptr) + (s->records == nullptr) + (s->keys == nullptr);
    const bool nodes_only = nulls == 2 && s->nodes != nullptr;
    if (nulls != 0 && nulls != 3 && !nodes_only) return SIMLOD_ERR_INVALID_ARGUMENT;
    // path: a leading 1, then one octant digit per level below the root
    u32 depth = 0;
    u32 digits[32];
    for (u64 p = root_path; p > 1; p >>= 3) {
        if (depth >= h->cfg.max_depth) {
            std::snprintf(g_last_error, sizeof(g_last_error), "path %llu is deeper than max_depth",
                          (unsigned long long)root_path);
            return SIMLOD_ERR_INVALID_ARGUMENT;
        }
        digits[depth++] = (u32)(p & 7u);
    }
    if (root_path == 0 || (root_path >> (3 * depth)) != 1) {
        std::snprintf(g_last_error, sizeof(g_last_error), "%llu is not a node path",
                      (unsigned long long)root_path);
        return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    DeviceGuard guard(h->device);
    if (h->poisoned) return SIMLOD_ERR_POISONED;
    int rc = sync_handle(h);
    if (rc) return rc;
    clear_stale_error();
    HostNodes hn;
    rc = read_nodes(h, hn, true);
    if (rc) return rc;
    const u32 nn = (u32)hn.child.size();
    u32 root = 0;
    for (u32 j = 0; j < depth; ++j) {
        if (root >= nn) return SIMLOD_ERR_HIP;
        if (!hn.child[root]) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "no node with path %llu (a leaf at depth %u)",
                          (unsigned long long)root_path, j);
            return SIMLOD_ERR_NOT_FOUND;
        }
        root = hn.child[root] + digits[depth - 1 - j];
    }
    // Preorder, children in octant order.
    std::vector<u32> order;
    std::vector<u64> first;
    std::vector<u64> path;
    std::vector<std::pair<u32, u64>> stack;
    stack.push_back({root, root_path});
    u64 written = 0, npts = 0, nvox = 0;
    while (!stack.empty()) {
        auto [node, p] = stack.back();
        stack.pop_back();
        if (node >= nn || order.size() >= nn) return SIMLOD_ERR_HIP;
        order.push_back(node);
        first.push_back(written);
        path.push_back(p);
        written += hn.count[node];
        (hn.child[node] ? nvox : npts) += hn.count[node];
        if (hn.child[node] && !single)
            for (int o = 7; o >= 0; --o) stack.push_back({hn.child[node] + (u32)o, p * 8 + (u64)o});
    }
    const u32 ns = (u32)order.size();
    s->num_nodes = ns;
    s->num_points = npts;
    s->num_voxels = nvox;
    s->num_records = written;
    auto fill_nodes = [&]() {
        for (u32 i = 0; i < ns; ++i) {
            const u32 node = order[i];
            simlod_node_record& r = s->nodes[i];
            r.path = path[i];
            r.first = first[i];
            r.count = hn.count[node];
            r.depth = (uint8_t)hn.geo[node].w;
            r.is_leaf = hn.child[node] ? 0 : 1;
            r.reserved = 0;
        }
    };
    if (nulls == 3) return SIMLOD_OK;
    if (nodes_only) {
        fill_nodes();
        return SIMLOD_OK;
    }
    u32* d_nodes = nullptr;
    u64* d_first = nullptr;
    uint4* d_rec = nullptr;
    u32* d_key = nullptr;
    u32* d_err = nullptr;
    u32 walk_err = 0;
    const u64 nrec = std::max<u64>(written, 1);
    bool ok = hipMalloc((void**)&d_nodes, ns * 4ull) == hipSuccess &&
              hipMalloc((void**)&d_first, ns * 8ull) == hipSuccess &&
              hipMalloc((void**)&d_rec, nrec * 16ull) == hipSuccess &&
              hipMalloc((void**)&d_key, nrec * 4ull) == hipSuccess &&
              hipMalloc((void**)&d_err, sizeof(u32)) == hipSuccess &&
              hipMemset(d_err, 0, sizeof(u32)) == hipSuccess;
    std::vector<uint4> rec;
    std::vector<u32> key;
    if (ok) {
        rec.resize(written);
        key.resize(written);
        ok = hipMemcpy(d_nodes, order.data(), ns * 4ull, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_first, first.data(), ns * 8ull, hipMemcpyHostToDevice) == hipSuccess &&
             (linked ? launch_walk(h->t, d_nodes, d_first, ns, d_rec, d_key, d_err, nullptr)
                     : launch_gather(h->t, d_nodes, d_first, ns, d_rec, d_key, nullptr)) ==
                 hipSuccess &&
             hipMemcpy(rec.data(), d_rec, written * 16ull, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(key.data(), d_key, written * 4ull, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(&walk_err, d_err, sizeof(u32), hipMemcpyDeviceToHost) == hipSuccess;
    }
    const hipError_t ge = ok ? hipSuccess : hipGetLastError();
    if (!ok) note_error("snapshot gather", ge);
    const bool oom = ge == hipErrorOutOfMemory;
    (void)hipFree(d_nodes);
    (void)hipFree(d_first);
    (void)hipFree(d_rec);
    (void)hipFree(d_key);
    (void)hipFree(d_err);
    if (!ok) return oom ? SIMLOD_ERR_OUT_OF_MEMORY : SIMLOD_ERR_HIP;
    if (walk_err) {
        std::snprintf(g_last_error, sizeof(g_last_error), "chunk list inconsistent (%u)", walk_err);
        return SIMLOD_ERR_HIP;
    }
    fill_nodes();
    // Canonical order inside a node: by key.  Nodes are independent; large
    // exports sort them on several host threads.
    auto sort_nodes = [&](u32 lo, u32 hi) {
        std::vector<u32> perm;
        for (u32 i = lo; i < hi; ++i) {
            const u64 f = first[i];
            const u32 c = hn.count[order[i]];
            bool sorted = true;
            for (u32 j = 1; j < c && sorted; ++j) sorted = key[f + j - 1] < key[f + j];
            if (sorted) {
                std::memcpy(s->records + f, rec.data() + f, c * 16ull);
                std::memcpy(s->keys + f, key.data() + f, c * 4ull);
                continue;
            }
            perm.resize(c);
            std::iota(perm.begin(), perm.end(), 0u);
            std::sort(perm.begin(), perm.end(),
                      [&](u32 a, u32 b) { return key[f + a] < key[f + b]; });
            for (u32 j = 0; j < c; ++j) {
                std::memcpy(s->records + f + j, &rec[f + perm[j]], 16);
                s->keys[f + j] = key[f + perm[j]];
            }
        }
    };
    const u32 hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const u32 nthreads = written >= (1u << 22) ? std::min<u32>(hw, ns) : 1u;
    if (nthreads <= 1) {
        sort_nodes(0, ns);
    } else {
        // split the node range into pieces of about equal record counts
        std::vector<std::thread> pool;
        u32 lo = 0;
        for (u32 t = 0; t < nthreads && lo < ns; ++t) {
            const u64 target = written * (t + 1) / nthreads;
            u32 hi = lo;
            while (hi < ns && (t + 1 == nthreads || first[hi] < target)) ++hi;
            if (hi == lo) hi = lo + 1;
            pool.emplace_back(sort_nodes, lo, hi);
            lo = hi;
        }
        for (auto& th : pool) th.join();
        if (lo < ns) sort_nodes(lo, ns);
    }
    return SIMLOD_OK;
}

}  // namespace

int simlod_snapshot(simlod_octree* h, simlod_snapshot_buffers* s) {
    return export_subtree(h, 1, s);
}

int simlod_snapshot_subtree(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s) {
    return export_subtree(h, path, s);
}

int simlod_snapshot_linked(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s) {
    return export_subtree(h, path, s, true);
}

int simlod_snapshot_node(simlod_octree* h, uint64_t path, simlod_snapshot_buffers* s) {
    return export_subtree(h, path, s, false, true);
}

int simlod_stats(simlod_octree* h, simlod_stats_data* st) {
    if (!h || !st) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    std::memset(st, 0, sizeof(*st));
    if (!h->poisoned) sync_handle(h);
    else (void)hipStreamSynchronize(h->last_stream);
    HostNodes hn;
    if (read_nodes(h, hn, false)) return SIMLOD_ERR_HIP;
    const u32 C = h->cfg.chunk_capacity;
    for (u32 i = 0; i < hn.child.size(); ++i) {
        if (hn.child[i]) {
            st->num_inner++;
            st->num_voxels += hn.count[i];
        } else {
            st->num_leaves++;
            st->num_points += hn.count[i];
        }
        st->chunks_in_use += (hn.count[i] + C - 1) / C;
    }
    st->num_nodes = hn.child.size();
    st->chunks_pooled = (u64)std::max<i32>(hn.ctr.pool_top, 0);
    st->arena_bytes_used = (u64)std::min(hn.ctr.arena_top, h->t.arena_blocks) * kBlockBytes;
    st->arena_bytes_total = (u64)h->t.arena_blocks * kBlockBytes;
    st->batches = h->passes;
    st->points_inserted = h->total_points;
    st->last_rounds = hn.ctr.last_rounds;
    st->last_spilled = hn.ctr.last_spilled;
    st->last_new_voxels = hn.ctr.last_new_voxels;
    st->max_rounds = hn.ctr.max_rounds;
    st->max_spilled = hn.ctr.max_spilled;
    st->max_new_voxels = hn.ctr.max_new_voxels;
    st->sum_rounds = hn.ctr.sum_rounds;
    st->sum_spilled = hn.ctr.sum_spilled;
    st->sum_new_voxels = hn.ctr.sum_new_voxels;
    st->status_bits = hn.ctr.status;
    st->poisoned = h->poisoned;
    return SIMLOD_OK;
}

int simlod_reset(simlod_octree* h, void* stream) {
    if (!h) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h->poisoned) (void)hipStreamSynchronize(h->last_stream);
    clear_stale_error();
    hipError_t re = order_after_last(h, s);
    if (re == hipSuccess) re = launch_reset(h->t, h->hash_entries, s);
    if (re != hipSuccess) {
        note_error("reset kernels (launch)", re);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    h->total_points = 0;
    h->passes = 0;
    h->poisoned = 0;
    h->sticky = SIMLOD_OK;
    h->status_pending = false;
    return SIMLOD_OK;
}

int simlod_destroy(simlod_octree* h) {
    if (!h) return SIMLOD_OK;
    DeviceGuard guard(h->device);
    hipError_t e = hipStreamSynchronize(h->last_stream);
    (void)hipGetLastError();
    if (h->staging) (void)hipFree(h->staging);
    free_all(h);
    delete h;
    return e == hipSuccess ? SIMLOD_OK : SIMLOD_ERR_HIP;
}

int simlod_set_kernel_timing(simlod_octree* h, uint32_t kernel_mask) {
    if (!h) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    drain_timing(h->tm);
    std::memset(&h->tm.acc, 0, sizeof(h->tm.acc));
    h->tm.mask = kernel_mask & ((1u << SIMLOD_NUM_KERNELS) - 1u);
    return SIMLOD_OK;
}

int simlod_get_kernel_times(simlod_octree* h, simlod_kernel_times* out) {
    if (!h || !out) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    drain_timing(h->tm);
    *out = h->tm.acc;
    return SIMLOD_OK;
}

// ------------------------------------------------------------------ groups
}  // extern "C"

namespace {

constexpr u32 kTuneCaps[] = {256u, 512u, 1024u, 2048u, 4096u};
constexpr u32 kTuneCands = sizeof(kTuneCaps) / sizeof(kTuneCaps[0]);
constexpr int kShapeKernel[kNumShapes] = {SIMLOD_KERNEL_COUNT, SIMLOD_KERNEL_COUNT_HIST,
                                          SIMLOD_KERNEL_SAMPLE_STORE, SIMLOD_KERNEL_STORE_VOXELS};

}  // namespace

struct simlod_group {
    std::vector<simlod_octree*> members;
    int device = 0;
    uint32_t flags = 0;
    Member* d_table = nullptr;   // member table the pass's later kernels read
    u32* d_status = nullptr;     // members' status words after the last pass
    u32* h_status = nullptr;     // pinned copy
    hipEvent_t status_ev = nullptr;
    bool status_pending = false;
    hipStream_t last_stream = nullptr;
    u32 rounds = 1;
    u64 cap_items = 0;           // summed max_batch: the captured pass's launch shape
    LaunchShape shape = default_shape();
    Timing tm;
    // launch-shape tuning
    Timing tune_tm;
    u32 tune_pass = 0;
    bool tuned = false;
    double tune_cost[kNumShapes][kTuneCands] = {};
    // graph replay
    hipStream_t gs = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t head = nullptr;
    hipKernelNodeParams head_params{};
    GroupArgs args{};            // argument of the replayed first kernel
    void* arg_ptrs[1] = {nullptr};
};

namespace {

void group_free(simlod_group* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->fork) (void)hipEventDestroy(g->fork);
    if (g->join) (void)hipEventDestroy(g->join);
    if (g->status_ev) (void)hipEventDestroy(g->status_ev);
    if (g->gs) (void)hipStreamDestroy(g->gs);
    if (g->d_table) (void)hipFree(g->d_table);
    if (g->d_status) (void)hipFree(g->d_status);
    if (g->h_status) (void)hipHostFree(g->h_status);
    free_timing(g->tm);
    free_timing(g->tune_tm);
}

// Marks members whose status word in h_status is non-zero as poisoned.
int group_apply_status(simlod_group* g) {
    int rc = SIMLOD_OK;
    for (size_t i = 0; i < g->members.size(); ++i) {
        simlod_octree* h = g->members[i];
        if (g->h_status[i] && !h->poisoned) {
            h->poisoned = 1;
            h->sticky = SIMLOD_ERR_CAPACITY;
            rc = SIMLOD_ERR_CAPACITY;
        }
    }
    return rc;
}

// Evaluates the status copy in flight, if it has arrived (wait: block
// until it has).
int group_poll(simlod_group* g, bool wait) {
    if (!g->status_pending) return SIMLOD_OK;
    const hipError_t e = wait ? hipEventSynchronize(g->status_ev) : hipEventQuery(g->status_ev);
    if (e == hipErrorNotReady) return SIMLOD_OK;
    g->status_pending = false;
    if (e != hipSuccess) {
        note_error("group status event", e);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    return group_apply_status(g);
}

// Captures one pass (shape fixed, grid sizes from the members' capacity) on
// the group's own stream and finds the first kernel's node.
hipError_t group_capture(simlod_group* g, const GroupArgs& ga) {
    hipError_t e = hipStreamBeginCapture(g->gs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t pe = enqueue_group_pass(ga, g->cap_items, g->rounds, g->shape, nullptr, g->d_status,
                                       g->gs);
    e = hipStreamEndCapture(g->gs, &g->graph);
    if (pe != hipSuccess) return pe;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    size_t num = 0;
    e = hipGraphGetNodes(g->graph, nullptr, &num);
    if (e != hipSuccess) return e;
    std::vector<hipGraphNode_t> nodes(num);
    e = hipGraphGetNodes(g->graph, nodes.data(), &num);
    if (e != hipSuccess) return e;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams p{};
        if (hipGraphKernelNodeGetParams(nd, &p) != hipSuccess) continue;
        if (is_count_leaves_kernel(p.func)) {
            g->head = nd;
            g->head_params = p;
        }
    }
    return g->head ? hipSuccess : hipErrorInvalidValue;
}

// One pass: replayed from the graph when one is captured, else launched
// (with the tuning shape and timing while tuning).
hipError_t group_pass(simlod_group* g, const GroupArgs& ga, u64 items, hipStream_t s) {
    const u32 cnt = (u32)g->members.size();
    const bool tuning = (g->flags & SIMLOD_GROUP_AUTOTUNE) && !g->tuned;
    if ((g->flags & SIMLOD_GROUP_GRAPH) && !tuning && !g->exec) {
        const hipError_t ce = group_capture(g, ga);
        if (ce != hipSuccess) {
            note_error("group graph capture", ce);
            return ce;
        }
    }
    hipError_t e;
    if (g->exec) {
        g->args = ga;
        g->arg_ptrs[0] = &g->args;
        g->head_params.kernelParams = g->arg_ptrs;
        g->head_params.extra = nullptr;
        e = hipGraphExecKernelNodeSetParams(g->exec, g->head, &g->head_params);
        if (e == hipSuccess) e = hipEventRecord(g->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(g->gs, g->fork, 0);
        if (e == hipSuccess) e = hipGraphLaunch(g->exec, g->gs);
        if (e == hipSuccess) e = hipEventRecord(g->join, g->gs);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, g->join, 0);
    } else {
        LaunchShape sh = g->shape;
        Timing* tm = &g->tm;
        u32 cand = 0;
        if (tuning) {
            cand = g->tune_pass % kTuneCands;
            for (u32 k = 0; k < kNumShapes; ++k) sh.cap[k] = kTuneCaps[cand];
            g->tune_tm.mask = 0;
            for (u32 k = 0; k < kNumShapes; ++k) g->tune_tm.mask |= 1u << kShapeKernel[k];
            std::memset(&g->tune_tm.acc, 0, sizeof(g->tune_tm.acc));
            tm = &g->tune_tm;
        }
        e = enqueue_group_pass(ga, items, g->rounds, sh, tm, g->d_status, s);
        if (e == hipSuccess && tuning) {
            drain_timing(g->tune_tm);  // waits for this pass
            const double per = 1.0 / (double)std::max<u64>(items, 1);
            for (u32 k = 0; k < kNumShapes; ++k)
                g->tune_cost[k][cand] += g->tune_tm.acc.total_ms[kShapeKernel[k]] * per;
            if (++g->tune_pass >= SIMLOD_TUNE_PASSES) {
                for (u32 k = 0; k < kNumShapes; ++k) {
                    u32 best = 0;
                    for (u32 c = 1; c < kTuneCands; ++c)
                        if (g->tune_cost[k][c] < g->tune_cost[k][best]) best = c;
                    g->shape.cap[k] = kTuneCaps[best];
                }
                g->tuned = true;
            }
        }
    }
    // one status copy in flight at most (the words are sticky)
    if (e == hipSuccess && !g->status_pending) {
        e = hipMemcpyAsync(g->h_status, g->d_status, cnt * sizeof(u32), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(g->status_ev, s);
        if (e == hipSuccess) g->status_pending = true;
    }
    return e;
}

}  // namespace

extern "C" {

int simlod_group_create(simlod_octree* const* members, uint32_t count, uint32_t flags,
                        simlod_group** out) {
    if (!members || !out || count == 0 || count > SIMLOD_MAX_GROUP || count > kMaxMembers ||
        (flags & ~(SIMLOD_GROUP_GRAPH | SIMLOD_GROUP_AUTOTUNE)))
        return SIMLOD_ERR_INVALID_ARGUMENT;
    u64 nodes = 0;
    for (u32 i = 0; i < count; ++i) {
        simlod_octree* h = members[i];
        if (!h || h->poisoned || h->device != members[0]->device) return SIMLOD_ERR_INVALID_ARGUMENT;
        for (u32 j = 0; j < i; ++j)
            if (members[j] == h) return SIMLOD_ERR_INVALID_ARGUMENT;
        nodes += h->cfg.max_nodes;
    }
    if (nodes >= (1ull << 32)) return SIMLOD_ERR_INVALID_ARGUMENT;  // member prefix sums are u32
    DeviceGuard guard(members[0]->device);
    clear_stale_error();
    simlod_group* g = new (std::nothrow) simlod_group();
    if (!g) return SIMLOD_ERR_OUT_OF_MEMORY;
    g->members.assign(members, members + count);
    g->device = members[0]->device;
    g->flags = flags;
    std::memset(&g->tm.acc, 0, sizeof(g->tm.acc));
    std::memset(&g->tune_tm.acc, 0, sizeof(g->tune_tm.acc));
    for (simlod_octree* h : g->members) {
        g->rounds = std::max(g->rounds, expansion_rounds(h->cfg.max_depth));
        g->cap_items += h->cfg.max_batch;
    }
    // one entry more: the pass barrier's two words follow the members
    bool ok = hipMalloc((void**)&g->d_table, (count + 1u) * sizeof(Member)) == hipSuccess &&
              hipMalloc((void**)&g->d_status, count * sizeof(u32)) == hipSuccess &&
              hipHostMalloc((void**)&g->h_status, count * sizeof(u32), hipHostMallocDefault) ==
                  hipSuccess &&
              hipEventCreateWithFlags(&g->status_ev, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&g->fork, kOrderingEvent) == hipSuccess &&
              hipEventCreateWithFlags(&g->join, kOrderingEvent) == hipSuccess &&
              hipStreamCreateWithFlags(&g->gs, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        note_error("group allocation", hipGetLastError());
        clear_stale_error();
        group_free(g);
        delete g;
        return SIMLOD_ERR_OUT_OF_MEMORY;
    }
    std::memset(g->h_status, 0, count * sizeof(u32));
    *out = g;
    return SIMLOD_OK;
}

int simlod_group_insert(simlod_group* g, const simlod_point* const* pts, const uint64_t* n,
                        void* stream) {
    if (!g || !pts || !n) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(g->device);
    const u32 cnt = (u32)g->members.size();
    int rc = group_poll(g, false);
    if (rc) return rc;
    u64 passes = 0;
    for (u32 i = 0; i < cnt; ++i) {
        simlod_octree* h = g->members[i];
        rc = poll_status(h, false);
        if (rc) return rc;
        if (n[i] == 0) continue;
        if (!pts[i] || (reinterpret_cast<uintptr_t>(pts[i]) & 15u) || !is_device_ptr(pts[i]))
            return SIMLOD_ERR_INVALID_ARGUMENT;
        if (h->total_points + n[i] > 0xFFFFFFFFull) return SIMLOD_ERR_KEY_SPACE;
        passes = std::max<u64>(passes, (n[i] + h->cfg.max_batch - 1) / h->cfg.max_batch);
    }
    clear_stale_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (u32 i = 0; i < cnt && passes; ++i) {
        const hipError_t oe = order_after_last(g->members[i], s);
        if (oe != hipSuccess) {
            note_error("stream ordering", oe);
            clear_stale_error();
            return SIMLOD_ERR_HIP;
        }
    }
    for (u64 p = 0; p < passes; ++p) {
        GroupArgs ga{};
        ga.table = g->d_table;
        ga.count = cnt;
        u64 items = 0;
        for (u32 i = 0; i < cnt; ++i) {
            simlod_octree* h = g->members[i];
            const u64 maxb = h->cfg.max_batch;
            const u64 off = p * maxb;
            const u64 m = off < n[i] ? std::min<u64>(maxb, n[i] - off) : 0u;
            ga.m[i] = make_member(h->d_tree,
                                  m ? reinterpret_cast<const uint4*>(pts[i] + off) : nullptr,
                                  (u32)m, (u32)(h->total_points + off));
            items += m;
        }
        const hipError_t e = group_pass(g, ga, items, s);
        if (e != hipSuccess) {
            note_error("group pass launch", e);
            clear_stale_error();
            for (simlod_octree* h : g->members) {
                h->poisoned = 1;
                h->sticky = SIMLOD_ERR_HIP;
            }
            return SIMLOD_ERR_HIP;
        }
    }
    for (u32 i = 0; i < cnt; ++i) {
        simlod_octree* h = g->members[i];
        h->total_points += n[i];
        h->passes += (n[i] + h->cfg.max_batch - 1) / h->cfg.max_batch;
    }
    g->last_stream = s;
    return SIMLOD_OK;
}

int simlod_group_shape(simlod_group* g, uint32_t caps[4], uint32_t* state) {
    if (!g || !caps) return SIMLOD_ERR_INVALID_ARGUMENT;
    for (u32 k = 0; k < kNumShapes; ++k) caps[k] = g->shape.cap[k];
    if (state) *state = (g->tuned ? 1u : 0u) | (g->exec ? 2u : 0u);
    return SIMLOD_OK;
}

int simlod_group_set_kernel_timing(simlod_group* g, uint32_t kernel_mask) {
    if (!g) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(g->device);
    drain_timing(g->tm);
    std::memset(&g->tm.acc, 0, sizeof(g->tm.acc));
    g->tm.mask = kernel_mask & ((1u << SIMLOD_NUM_KERNELS) - 1u);
    return SIMLOD_OK;
}

int simlod_group_get_kernel_times(simlod_group* g, simlod_kernel_times* out) {
    if (!g || !out) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(g->device);
    drain_timing(g->tm);
    *out = g->tm.acc;
    return SIMLOD_OK;
}

int simlod_group_sync(simlod_group* g) {
    if (!g) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(g->device);
    const hipError_t e = hipStreamSynchronize(g->last_stream);
    if (e != hipSuccess) {
        note_error("hipStreamSynchronize", e);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    int rc = group_poll(g, true);
    if (rc) return rc;
    // the last passes may have left no status copy: read the words
    const hipError_t ce = hipMemcpy(g->h_status, g->d_status, g->members.size() * sizeof(u32),
                                    hipMemcpyDeviceToHost);
    if (ce != hipSuccess) {
        note_error("group status read", ce);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    return group_apply_status(g);
}

int simlod_group_destroy(simlod_group* g) {
    if (!g) return SIMLOD_OK;
    DeviceGuard guard(g->device);
    hipError_t e = hipStreamSynchronize(g->last_stream);
    if (g->gs) (void)hipStreamSynchronize(g->gs);
    (void)hipGetLastError();
    group_free(g);
    delete g;
    return e == hipSuccess ? SIMLOD_OK : SIMLOD_ERR_HIP;
}

int simlod_tune_chunk_capacity(const simlod_config* cfg, const simlod_point* sample, uint64_t n,
                               const uint32_t* candidates, uint32_t count, void* stream,
                               uint32_t* best, double* best_ms) {
    if (!cfg || !candidates || count == 0 || !best || (n && !sample))
        return SIMLOD_ERR_INVALID_ARGUMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double best_t = 0.0;
    u32 best_c = 0;
    for (u32 i = 0; i < count; ++i) {
        simlod_config c = *cfg;
        c.chunk_capacity = candidates[i];
        simlod_octree* h = nullptr;
        int rc = simlod_create(&c, &h);
        if (rc) return rc;
        DeviceGuard guard(h->device);
        hipEvent_t a = nullptr, b = nullptr;
        float ms = 0.f;
        bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
                  hipEventRecord(a, s) == hipSuccess;
        if (ok) rc = simlod_insert_batch(h, sample, n, stream);
        ok = ok && rc == SIMLOD_OK && hipEventRecord(b, s) == hipSuccess &&
             hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
        if (ok) rc = simlod_sync(h);
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)simlod_destroy(h);
        if (rc) return rc;
        if (!ok) {
            note_error("chunk tuning", hipGetLastError());
            clear_stale_error();
            return SIMLOD_ERR_HIP;
        }
        if (i == 0 || ms < best_t) {
            best_t = ms;
            best_c = candidates[i];
        }
    }
    *best = best_c;
    if (best_ms) *best_ms = best_t;
    return SIMLOD_OK;
}

// ------------------------------------------------------------------ serving
}  // extern "C"

namespace {

using Clock = std::chrono::steady_clock;

constexpr u32 kServerInflight = 2;  // passes enqueued ahead of the device
constexpr u32 kStatusRing = 4;      // pinned status arrays, > kServerInflight

struct ServerRequest {
    u64 ticket;
    u32 slot;
    const uint4* pts;             // device points (staging area for host requests)
    u32 n;
    Clock::time_point t_submit;
    const void* host = nullptr;   // host points, for requests in host memory
    bool ready = true;            // host requests: the copy has been enqueued
    u64 stage_off = 0, stage_len = 0;  // staging range of a host request
    hipEvent_t up_ev = nullptr;   // host requests: after the copy
    // pass budget: points of a queued request already given to passes; in a
    // pass, whether this part is the request's last (the one that completes it)
    u32 taken = 0;
    bool last = true;
};

struct ServerSlot {
    simlod_octree* h = nullptr;
    u64 bytes = 0;
    bool open = false, opening = false, closing = false;
    std::deque<ServerRequest> queue;
    u64 queued_points = 0;
    u32 inflight = 0;  // requests of this slot on the device
};

struct ServerPass {
    hipEvent_t done = nullptr;
    std::vector<ServerRequest> reqs;  // member i of the pass = reqs[i]
    u32 ring = 0;
};

struct RequestResult {
    int done = 0;
    int status = SIMLOD_OK;
    double latency_ms = 0.0;
};

}  // namespace

struct simlod_server {
    simlod_server_config cfg{};
    std::mutex mu;
    // uploads of requests in host memory (section "Overview": an uploader
    // thread copies loaded batches to a GPU-side queue)
    uint8_t* staging = nullptr;       // staging_bytes of device memory
    std::map<u64, u64> stage_free;    // free ranges: offset -> length
    std::deque<u64> upload_q;         // tickets of host requests to copy, in order
    std::condition_variable cv_upload;
    hipStream_t copy_stream = nullptr;
    std::vector<hipEvent_t> free_up_events;
    std::thread uploader;
    std::condition_variable cv_work;  // scheduler: requests queued or a pass retired
    std::condition_variable cv_done;  // callers: requests completed
    std::condition_variable cv_retire;  // completion thread: a pass was enqueued
    std::vector<ServerSlot> slots;
    std::deque<ServerPass*> inflight;
    std::vector<hipEvent_t> free_events;
    std::vector<RequestResult> results;  // by ticket - 1
    u64 budget_used = 0;
    u64 submitted = 0, completed = 0, passes = 0, points = 0;
    u32 ring_next = 0;
    hipStream_t stream = nullptr;
    Member* d_table = nullptr;
    u32* d_status = nullptr;  // kMaxMembers words
    u32* h_status = nullptr;  // pinned, kStatusRing x kMaxMembers
    bool stop = false;
    std::deque<u32> reap;            // closed slots waiting for their last requests
    std::condition_variable cv_reap;
    struct Pooled {
        simlod_octree* h;
        u64 bytes;
    };
    std::vector<Pooled> pool;        // closed octrees kept for reuse (budget still held)
    std::thread scheduler, completer, reaper;
};

namespace {

constexpr u64 kStageAlign = 256;

// Staging ranges for requests in host memory: first fit over the free
// ranges (lock held).
bool stage_alloc(simlod_server* sv, u64 len, u64* off) {
    for (auto it = sv->stage_free.begin(); it != sv->stage_free.end(); ++it) {
        if (it->second < len) continue;
        *off = it->first;
        const u64 rest = it->second - len, at = it->first + len;
        sv->stage_free.erase(it);
        if (rest) sv->stage_free[at] = rest;
        return true;
    }
    return false;
}

void stage_release(simlod_server* sv, u64 off, u64 len) {
    auto it = sv->stage_free.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != sv->stage_free.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        sv->stage_free.erase(nx);
    }
    if (it != sv->stage_free.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            sv->stage_free.erase(it);
        }
    }
}

// A host request's staging range and event go back once its copy is done
// (lock held; the copy has completed or completes shortly).
void release_upload(simlod_server* sv, ServerRequest& r) {
    if (!r.stage_len) return;
    if (r.up_ev) {
        (void)hipEventSynchronize(r.up_ev);
        sv->free_up_events.push_back(r.up_ev);
    }
    stage_release(sv, r.stage_off, r.stage_len);
    r.stage_len = 0;
    r.up_ev = nullptr;
    sv->cv_upload.notify_all();
}

ServerRequest* find_queued(simlod_server* sv, u64 ticket) {
    for (ServerSlot& sl : sv->slots)
        for (ServerRequest& r : sl.queue)
            if (r.ticket == ticket) return &r;
    return nullptr;
}

// Uploader thread: copies the requests in host memory, in submission order,
// into free staging ranges on the server's copy stream, while the passes of
// earlier requests run on the pass stream; a request becomes eligible for a
// pass once its copy is enqueued, and the pass waits for the copy's event.
void server_upload(simlod_server* sv) {
    (void)hipSetDevice(sv->cfg.device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_upload.wait(lk, [&] { return sv->stop || !sv->upload_q.empty(); });
        if (sv->stop) return;
        const u64 tk = sv->upload_q.front();
        ServerRequest* r = find_queued(sv, tk);
        if (!r) {  // its stream was poisoned and its requests completed
            sv->upload_q.pop_front();
            continue;
        }
        const u64 len = ((u64)r->n * 16u + kStageAlign - 1) / kStageAlign * kStageAlign;
        u64 off = 0;
        if (!stage_alloc(sv, len, &off)) {  // wait until completed passes free space
            sv->cv_upload.wait(lk);
            continue;
        }
        sv->upload_q.pop_front();
        hipEvent_t ev = nullptr;
        if (!sv->free_up_events.empty()) {
            ev = sv->free_up_events.back();
            sv->free_up_events.pop_back();
        } else {
            (void)hipEventCreateWithFlags(&ev, kOrderingEvent);
        }
        r->stage_off = off;
        r->stage_len = len;
        r->up_ev = ev;
        const void* src = r->host;
        const u64 bytes = (u64)r->n * 16u;
        lk.unlock();
        hipError_t e = hipMemcpyAsync(sv->staging + off, src, bytes, hipMemcpyHostToDevice,
                                      sv->copy_stream);
        if (e == hipSuccess) e = hipEventRecord(ev, sv->copy_stream);
        lk.lock();
        r = find_queued(sv, tk);
        if (!r) {  // completed as poisoned meanwhile: the range is ours to free
            ServerRequest gone{};
            gone.stage_off = off;
            gone.stage_len = len;
            gone.up_ev = ev;
            release_upload(sv, gone);
            continue;
        }
        if (e != hipSuccess) {
            note_error("server upload", e);
            (void)hipGetLastError();
            simlod_octree* h = sv->slots[r->slot].h;
            if (h && !h->poisoned) {
                h->poisoned = 1;
                h->sticky = SIMLOD_ERR_HIP;
            }
        }
        r->pts = reinterpret_cast<const uint4*>(sv->staging + off);
        r->ready = true;
        sv->cv_work.notify_all();
    }
}

// Chooses the next pass's requests (lock held): the head request of every
// open stream that has one ready (max_per_pass 0), else the max_per_pass
// oldest ready heads.  Requests of poisoned streams complete at once with
// POISONED.
std::vector<ServerRequest> server_pick(simlod_server* sv) {
    std::vector<u32> heads;
    for (u32 i = 0; i < sv->slots.size(); ++i) {
        ServerSlot& sl = sv->slots[i];
        while (!sl.queue.empty() && (sl.h == nullptr || sl.h->poisoned)) {
            ServerRequest& r = sl.queue.front();
            sv->results[r.ticket - 1] = RequestResult{1, SIMLOD_ERR_POISONED, 0.0};
            if (r.ready) release_upload(sv, r);  // else the uploader frees it
            sl.queued_points -= r.n - r.taken;
            sl.queue.pop_front();
            ++sv->completed;
        }
        if (!sl.queue.empty() && sl.queue.front().ready) heads.push_back(i);
    }
    const u32 lim = sv->cfg.max_per_pass ? sv->cfg.max_per_pass : kMaxMembers;
    if (heads.size() > lim) {
        std::sort(heads.begin(), heads.end(), [&](u32 a, u32 b) {
            return sv->slots[a].queue.front().ticket < sv->slots[b].queue.front().ticket;
        });
        heads.resize(lim);
    }
    // the pass budget cuts a request in device memory into parts of at most
    // pass_points points, one per pass, in order; it stays at the head of its
    // stream's queue until its last part is taken
    const u32 budget = sv->cfg.pass_points;
    std::vector<ServerRequest> out;
    for (u32 i : heads) {
        ServerSlot& sl = sv->slots[i];
        ServerRequest& head = sl.queue.front();
        const u32 rest = head.n - head.taken;
        const u32 take = (budget && !head.host) ? std::min(rest, budget) : rest;
        ServerRequest part = head;
        part.pts = head.pts + head.taken;
        part.n = take;
        part.last = take == rest;
        if (part.last)
            sl.queue.pop_front();
        else
            head.taken += take;
        sl.queued_points -= take;
        sl.inflight += 1;
        out.push_back(part);
    }
    return out;
}

void server_schedule(simlod_server* sv) {
    (void)hipSetDevice(sv->cfg.device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_work.wait(lk, [&] {
            if (sv->stop) return true;
            if (sv->inflight.size() >= kServerInflight) return false;
            for (const ServerSlot& sl : sv->slots)
                if (!sl.queue.empty() &&
                    (sl.queue.front().ready || sl.h == nullptr || sl.h->poisoned))
                    return true;
            return false;
        });
        if (sv->stop) return;
        std::vector<ServerRequest> reqs = server_pick(sv);
        if (reqs.empty()) {
            sv->cv_done.notify_all();
            sv->cv_reap.notify_all();
            continue;
        }
        ServerPass* ps = new ServerPass();
        ps->reqs = std::move(reqs);
        ps->ring = sv->ring_next++ % kStatusRing;
        if (!sv->free_events.empty()) {
            ps->done = sv->free_events.back();
            sv->free_events.pop_back();
        } else {
            (void)hipEventCreateWithFlags(&ps->done, hipEventDisableTiming);
        }
        GroupArgs ga{};
        ga.table = sv->d_table;
        ga.count = (u32)ps->reqs.size();
        u64 items = 0;
        u32 rounds = 1;
        for (u32 i = 0; i < ga.count; ++i) {
            const ServerRequest& r = ps->reqs[i];
            simlod_octree* h = sv->slots[r.slot].h;
            ga.m[i] = make_member(h->d_tree, r.pts, r.n, (u32)h->total_points);
            h->total_points += r.n;
            h->passes += 1;
            h->last_stream = sv->stream;
            h->has_work = true;
            items += r.n;
            rounds = std::max(rounds, expansion_rounds(h->cfg.max_depth));
        }
        u32* hs = sv->h_status + (u64)ps->ring * kMaxMembers;
        std::memset(hs, 0, ga.count * sizeof(u32));
        hipError_t e = hipSuccess;
        for (const ServerRequest& r : ps->reqs)  // uploads of host requests first
            if (e == hipSuccess && r.up_ev) e = hipStreamWaitEvent(sv->stream, r.up_ev, 0);
        if (e == hipSuccess)
            e = enqueue_group_pass(ga, items, rounds, default_shape(), nullptr, sv->d_status,
                                   sv->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hs, sv->d_status, ga.count * sizeof(u32), hipMemcpyDeviceToHost,
                               sv->stream);
        if (e == hipSuccess) e = hipEventRecord(ps->done, sv->stream);
        if (e != hipSuccess) {
            note_error("server pass launch", e);
            (void)hipGetLastError();
            for (const ServerRequest& r : ps->reqs) {
                sv->slots[r.slot].h->poisoned = 1;
                sv->slots[r.slot].h->sticky = SIMLOD_ERR_HIP;
            }
            for (u32 i = 0; i < ga.count; ++i) hs[i] = 1u;
            (void)hipEventRecord(ps->done, sv->stream);
        }
        sv->passes += 1;
        sv->points += items;
        sv->inflight.push_back(ps);
        sv->cv_retire.notify_all();
    }
}

void server_complete(simlod_server* sv) {
    (void)hipSetDevice(sv->cfg.device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_retire.wait(lk, [&] { return sv->stop || !sv->inflight.empty(); });
        if (sv->inflight.empty()) return;  // stopping, nothing on the device
        ServerPass* ps = sv->inflight.front();
        lk.unlock();
        const hipError_t e = hipEventSynchronize(ps->done);
        const Clock::time_point now = Clock::now();
        lk.lock();
        sv->inflight.pop_front();
        const u32* hs = sv->h_status + (u64)ps->ring * kMaxMembers;
        for (u32 i = 0; i < ps->reqs.size(); ++i) {
            const ServerRequest& r = ps->reqs[i];
            ServerSlot& sl = sv->slots[r.slot];
            int st = SIMLOD_OK;
            if (e != hipSuccess) {
                st = SIMLOD_ERR_HIP;
            } else if (hs[i]) {
                st = SIMLOD_ERR_CAPACITY;
            }
            if (st && sl.h && !sl.h->poisoned) {
                sl.h->poisoned = 1;
                sl.h->sticky = st;
            }
            sl.inflight -= 1;
            if (!r.last) {  // an earlier part of a request cut by the pass budget
                RequestResult& rr = sv->results[r.ticket - 1];
                if (st && !rr.done) rr.status = st;  // reported with the last part
                continue;
            }
            const double ms =
                std::chrono::duration<double, std::milli>(now - r.t_submit).count();
            const int prior = sv->results[r.ticket - 1].status;  // an earlier part's error
            sv->results[r.ticket - 1] = RequestResult{1, st ? st : prior, ms};
            ++sv->completed;
            if (r.stage_len) release_upload(sv, ps->reqs[i]);
        }
        sv->free_events.push_back(ps->done);
        delete ps;
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
        sv->cv_reap.notify_all();
    }
}

// Moves the octrees of closed streams, once their requests have completed,
// to the pool: device memory is neither freed nor allocated while requests
// flow (either would synchronize the device and stall the passes); a later
// open reuses a pooled octree whose buffers are large enough.
void server_reap(simlod_server* sv) {
    (void)hipSetDevice(sv->cfg.device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_reap.wait(lk, [&] {
            if (sv->stop && sv->reap.empty()) return true;
            for (u32 id : sv->reap) {
                const ServerSlot& sl = sv->slots[id];
                if (sl.queue.empty() && sl.inflight == 0) return true;
            }
            return false;
        });
        if (sv->stop && sv->reap.empty()) return;
        u32 id = kNone;
        for (auto it = sv->reap.begin(); it != sv->reap.end(); ++it) {
            const ServerSlot& sl = sv->slots[*it];
            if (sl.queue.empty() && sl.inflight == 0) {
                id = *it;
                sv->reap.erase(it);
                break;
            }
        }
        if (id == kNone) continue;
        ServerSlot& sl = sv->slots[id];
        sv->pool.push_back({sl.h, sl.bytes});
        sl = ServerSlot{};
        sv->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int simlod_config_device_bytes(const simlod_config* cfg, uint64_t* bytes) {
    if (!cfg || !bytes || !cfg_valid(cfg) || cfg->arena_bytes == 0)
        return SIMLOD_ERR_INVALID_ARGUMENT;
    simlod_octree dry;
    u64 total = 0;
    dry.dry = &total;
    dry.cfg = *cfg;
    (void)allocate_all(&dry, cfg, cfg->arena_bytes);
    *bytes = total;
    return SIMLOD_OK;
}

int simlod_server_create(const simlod_server_config* cfg, simlod_server** out) {
    if (!cfg || !out || cfg->max_streams == 0 || cfg->max_streams > SIMLOD_MAX_GROUP ||
        cfg->max_streams > kMaxMembers || cfg->max_per_pass > kMaxMembers)
        return SIMLOD_ERR_INVALID_ARGUMENT;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) {
        clear_stale_error();
        return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    DeviceGuard guard(cfg->device);
    clear_stale_error();
    simlod_server* sv = new (std::nothrow) simlod_server();
    if (!sv) return SIMLOD_ERR_OUT_OF_MEMORY;
    sv->cfg = *cfg;
    sv->slots.resize(cfg->max_streams);
    bool ok = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void**)&sv->d_table, (kMaxMembers + 1u) * sizeof(Member)) == hipSuccess &&
              hipMalloc((void**)&sv->d_status, kMaxMembers * sizeof(u32)) == hipSuccess &&
              hipHostMalloc((void**)&sv->h_status, kStatusRing * kMaxMembers * sizeof(u32),
                            hipHostMallocDefault) == hipSuccess;
    const u64 stage = cfg->staging_bytes / kStageAlign * kStageAlign;
    if (ok && stage)
        ok = hipMalloc((void**)&sv->staging, stage) == hipSuccess &&
             hipStreamCreateWithFlags(&sv->copy_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        note_error("server allocation", hipGetLastError());
        clear_stale_error();
        if (sv->staging) (void)hipFree(sv->staging);
        if (sv->copy_stream) (void)hipStreamDestroy(sv->copy_stream);
        if (sv->stream) (void)hipStreamDestroy(sv->stream);
        if (sv->d_table) (void)hipFree(sv->d_table);
        if (sv->d_status) (void)hipFree(sv->d_status);
        if (sv->h_status) (void)hipHostFree(sv->h_status);
        delete sv;
        return SIMLOD_ERR_OUT_OF_MEMORY;
    }
    if (stage) sv->stage_free[0] = stage;
    sv->scheduler = std::thread(server_schedule, sv);
    sv->completer = std::thread(server_complete, sv);
    sv->reaper = std::thread(server_reap, sv);
    if (stage) sv->uploader = std::thread(server_upload, sv);
    *out = sv;
    return SIMLOD_OK;
}

int simlod_server_open(simlod_server* sv, const simlod_config* cfg, uint32_t* id) {
    if (!sv || !cfg || !id || cfg->device != sv->cfg.device) return SIMLOD_ERR_INVALID_ARGUMENT;
    if (cfg->arena_ptr) {  // the server owns (and pools) its octrees' memory
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "simlod_server_open: arena_ptr must be NULL");
        return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    u64 bytes = 0;
    int rc = simlod_config_device_bytes(cfg, &bytes);
    if (rc) return rc;
    const Footprint need = footprint_of(cfg);
    u32 slot = 0;
    simlod_octree* reuse = nullptr;
    u64 reuse_bytes = 0;
    std::vector<simlod_octree*> evict;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        while (slot < sv->slots.size() &&
               (sv->slots[slot].open || sv->slots[slot].opening || sv->slots[slot].closing))
            ++slot;
        if (slot == sv->slots.size()) return SIMLOD_ERR_BUSY;
        // the smallest pooled octree whose buffers are large enough
        size_t best = sv->pool.size();
        for (size_t i = 0; i < sv->pool.size(); ++i)
            if (footprint_fits(footprint_of(&sv->pool[i].h->alloc_cfg), need) &&
                (best == sv->pool.size() || sv->pool[i].bytes < sv->pool[best].bytes))
                best = i;
        if (best < sv->pool.size()) {
            reuse = sv->pool[best].h;
            reuse_bytes = sv->pool[best].bytes;
            sv->pool.erase(sv->pool.begin() + (long)best);
        } else {
            // make room by releasing pooled octrees, largest first
            std::sort(sv->pool.begin(), sv->pool.end(),
                      [](const simlod_server::Pooled& a, const simlod_server::Pooled& b) {
                          return a.bytes < b.bytes;
                      });
            while (sv->budget_used + bytes > sv->cfg.hbm_budget && !sv->pool.empty()) {
                evict.push_back(sv->pool.back().h);
                sv->budget_used -= sv->pool.back().bytes;
                sv->pool.pop_back();
            }
            if (sv->budget_used + bytes > sv->cfg.hbm_budget) {
                for (simlod_octree* h : evict) (void)simlod_destroy(h);
                return SIMLOD_ERR_BUSY;
            }
            sv->budget_used += bytes;
        }
        sv->slots[slot].opening = true;
    }
    for (simlod_octree* h : evict) (void)simlod_destroy(h);
    simlod_octree* h = reuse;
    if (reuse) {
        // same buffers, new configuration; the reset is ordered on the
        // server's stream before the stream's first pass
        DeviceGuard guard(sv->cfg.device);
        configure_tree(h, cfg, cfg->arena_bytes);
        hipError_t e = hipMemcpyAsync(h->d_tree, &h->t, sizeof(DevTree), hipMemcpyHostToDevice,
                                      sv->stream);
        if (e == hipSuccess) e = launch_reset(h->t, h->hash_entries, sv->stream);
        h->total_points = 0;
        h->passes = 0;
        h->poisoned = 0;
        h->sticky = SIMLOD_OK;
        h->status_pending = false;
        h->last_stream = sv->stream;
        h->has_work = true;
        if (e != hipSuccess) {
            note_error("pooled octree reset", e);
            clear_stale_error();
            rc = SIMLOD_ERR_HIP;
        }
        bytes = reuse_bytes;
    } else {
        rc = simlod_create(cfg, &h);
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    ServerSlot& sl = sv->slots[slot];
    sl.opening = false;
    if (rc) {
        if (h) {
            sv->pool.push_back({h, bytes});
        } else {
            sv->budget_used -= bytes;
        }
        return rc;
    }
    sl.h = h;
    sl.bytes = bytes;
    sl.open = true;
    sl.queued_points = 0;
    sl.inflight = 0;
    *id = slot;
    return SIMLOD_OK;
}

int simlod_server_submit(simlod_server* sv, uint32_t id, const simlod_point* pts, uint64_t n,
                         uint64_t* ticket) {
    if (!sv || !ticket || (n && !pts)) return SIMLOD_ERR_INVALID_ARGUMENT;
    bool on_host = false;
    if (n) {
        DeviceGuard guard(sv->cfg.device);
        on_host = !is_device_ptr(pts);
        clear_stale_error();
        if (on_host ? (!sv->staging || n * 16u > sv->cfg.staging_bytes / kStageAlign * kStageAlign)
                    : (reinterpret_cast<uintptr_t>(pts) & 15u) != 0u)
            return SIMLOD_ERR_INVALID_ARGUMENT;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (id >= sv->slots.size() || !sv->slots[id].open || sv->slots[id].closing)
        return SIMLOD_ERR_INVALID_ARGUMENT;
    ServerSlot& sl = sv->slots[id];
    if (sl.h->poisoned) return SIMLOD_ERR_POISONED;
    if (n > sl.h->cfg.max_batch) return SIMLOD_ERR_INVALID_ARGUMENT;
    if (sl.h->total_points + sl.queued_points + n > 0xFFFFFFFFull) return SIMLOD_ERR_KEY_SPACE;
    const u64 t = sv->results.size() + 1;
    sv->results.push_back(RequestResult{});
    *ticket = t;
    ++sv->submitted;
    if (n == 0) {
        sv->results[t - 1] = RequestResult{1, SIMLOD_OK, 0.0};
        ++sv->completed;
        return SIMLOD_OK;
    }
    ServerRequest rq{t, id, reinterpret_cast<const uint4*>(pts), (u32)n, Clock::now()};
    if (on_host) {
        rq.pts = nullptr;
        rq.host = pts;
        rq.ready = false;
        sv->upload_q.push_back(t);
        sv->cv_upload.notify_one();
    }
    sl.queue.push_back(rq);
    sl.queued_points += n;
    sv->cv_work.notify_one();
    return SIMLOD_OK;
}

int simlod_server_poll(simlod_server* sv, uint64_t ticket, int* done, double* latency_ms) {
    if (!sv || !done) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (ticket == 0 || ticket > sv->results.size()) return SIMLOD_ERR_INVALID_ARGUMENT;
    const RequestResult& r = sv->results[ticket - 1];
    *done = r.done;
    if (latency_ms) *latency_ms = r.latency_ms;
    return r.done ? r.status : SIMLOD_OK;
}

int simlod_server_drain(simlod_server* sv) {
    if (!sv) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_work.notify_all();
    sv->cv_done.wait(lk, [&] { return sv->completed == sv->submitted; });
    return SIMLOD_OK;
}

simlod_octree* simlod_server_octree(simlod_server* sv, uint32_t id) {
    if (!sv) return nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    return id < sv->slots.size() && sv->slots[id].open ? sv->slots[id].h : nullptr;
}

int simlod_server_close(simlod_server* sv, uint32_t id) {
    if (!sv) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (id >= sv->slots.size() || !sv->slots[id].open || sv->slots[id].closing)
        return SIMLOD_ERR_INVALID_ARGUMENT;
    sv->slots[id].closing = true;
    sv->reap.push_back(id);
    sv->cv_work.notify_all();
    sv->cv_reap.notify_all();
    return SIMLOD_OK;
}

int simlod_server_wait_closed(simlod_server* sv) {
    if (!sv) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_reap.notify_all();
    sv->cv_done.wait(lk, [&] {
        for (const ServerSlot& sl : sv->slots)
            if (sl.closing) return false;
        return true;
    });
    return SIMLOD_OK;
}

int simlod_server_counters(simlod_server* sv, uint64_t out[4]) {
    if (!sv || !out) return SIMLOD_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(sv->mu);
    out[0] = sv->passes;
    out[1] = sv->completed;
    out[2] = sv->points;
    out[3] = sv->budget_used;
    return SIMLOD_OK;
}

int simlod_server_destroy(simlod_server* sv) {
    if (!sv) return SIMLOD_OK;
    (void)simlod_server_drain(sv);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    sv->cv_retire.notify_all();
    sv->cv_reap.notify_all();
    sv->cv_upload.notify_all();
    sv->scheduler.join();
    sv->completer.join();
    sv->reaper.join();
    if (sv->uploader.joinable()) sv->uploader.join();
    DeviceGuard guard(sv->cfg.device);
    (void)hipStreamSynchronize(sv->stream);
    int rc = SIMLOD_OK;
    for (ServerSlot& sl : sv->slots)
        if (sl.h && simlod_destroy(sl.h) != SIMLOD_OK) rc = SIMLOD_ERR_HIP;
    for (auto& p : sv->pool)
        if (simlod_destroy(p.h) != SIMLOD_OK) rc = SIMLOD_ERR_HIP;
    for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : sv->free_up_events) (void)hipEventDestroy(e);
    if (sv->copy_stream) (void)hipStreamSynchronize(sv->copy_stream);
    if (sv->copy_stream) (void)hipStreamDestroy(sv->copy_stream);
    if (sv->staging) (void)hipFree(sv->staging);
    (void)hipStreamDestroy(sv->stream);
    (void)hipFree(sv->d_table);
    (void)hipFree(sv->d_status);
    (void)hipHostFree(sv->h_status);
    delete sv;
    return rc;
}

const char* simlod_last_error(void) { return g_last_error; }

const char* simlod_status_string(int code) {
    switch (code) {
        case SIMLOD_OK: return "ok";
        case SIMLOD_ERR_INVALID_ARGUMENT: return "invalid argument";
        case SIMLOD_ERR_OUT_OF_MEMORY: return "out of memory";
        case SIMLOD_ERR_HIP: return "HIP runtime error";
        case SIMLOD_ERR_CAPACITY: return "device-side capacity exceeded (handle poisoned)";
        case SIMLOD_ERR_POISONED: return "handle poisoned by an earlier error";
        case SIMLOD_ERR_KEY_SPACE: return "more than 2^32-1 points in one octree";
        case SIMLOD_ERR_NOT_FOUND: return "no node with that path";
        case SIMLOD_ERR_BUSY: return "no stream slot or device-memory budget free";
        default: return "unknown status";
    }
}

}  // extern "C"
