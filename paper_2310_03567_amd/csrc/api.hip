// Host side of the C ABI declared in include/simlod.h: creation, the launch
// sequence of one insertion pass, canonical export, counters, timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "launch.hpp"
#include "octree_device.hpp"
#include "simlod.h"

using namespace simlod;

struct simlod_octree {
    simlod_config cfg;
    DevTree t;
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
    uint4* staging = nullptr;
    u64 staging_cap = 0;
    std::vector<void*> dev_allocs;
    // kernel timing
    uint32_t timing_mask = 0;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    simlod_kernel_times acc;
};

namespace {

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
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
        note_error("hipMalloc", e);
        return false;
    }
    h->dev_allocs.push_back(v);
    *p = static_cast<T*>(v);
    return true;
}

u64 next_pow2(u64 v) {
    u64 p = 1;
    while (p < v) p <<= 1;
    return p;
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
    return true;
}

void free_all(simlod_octree* h) {
    for (void* p : h->dev_allocs) (void)hipFree(p);
    h->dev_allocs.clear();
    if (h->h_status) (void)hipHostFree(h->h_status);
    h->h_status = nullptr;
    if (h->status_ev) (void)hipEventDestroy(h->status_ev);
    for (auto& p : h->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->free_events) (void)hipEventDestroy(e);
    h->pending.clear();
    h->free_events.clear();
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

hipEvent_t take_event(simlod_octree* h) {
    if (!h->free_events.empty()) {
        hipEvent_t e = h->free_events.back();
        h->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

template <typename F>
hipError_t timed(simlod_octree* h, int kind, hipStream_t s, F&& launch) {
    if (!((h->timing_mask >> kind) & 1u)) return launch();
    hipEvent_t a = take_event(h), b = take_event(h);
    (void)hipEventRecord(a, s);
    hipError_t e = launch();
    (void)hipEventRecord(b, s);
    h->pending.push_back({kind, a, b});
    return e;
}

void drain_timing(simlod_octree* h) {
    for (auto& p : h->pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            h->acc.launches[p.kind] += 1;
            h->acc.total_ms[p.kind] += ms;
        }
        h->free_events.push_back(p.a);
        h->free_events.push_back(p.b);
    }
    h->pending.clear();
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

// One insertion pass over n <= max_batch device-resident points.
hipError_t enqueue_pass(simlod_octree* h, const uint4* batch, u32 n, u32 base_key, hipStream_t s) {
    const DevTree& t = h->t;
    const u32 rounds = expansion_rounds(h->cfg.max_depth);
    hipError_t e = timed(h, SIMLOD_KERNEL_COUNT, s, [&] { return launch_count_leaves(t, batch, n, s); });
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_SPLIT, s, [&] { return launch_split_leaves(t, n, s); });
    for (u32 k = 2; k <= rounds && e == hipSuccess; ++k) {
        e = timed(h, SIMLOD_KERNEL_COUNT_HIST, s,
                  [&] { return launch_count_hist(t, batch, n, base_key, k, s); });
        if (e == hipSuccess)
            e = timed(h, SIMLOD_KERNEL_BUILD, s, [&] { return launch_build(t, k, s); });
    }
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_ALLOC_POINTS, s, [&] { return launch_alloc(t, 0u, s); });
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_SAMPLE_STORE, s,
                  [&] { return launch_sample_store(t, batch, n, base_key, s); });
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_ALLOC_VOXELS, s, [&] { return launch_alloc(t, 1u, s); });
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_STORE_VOXELS, s, [&] { return launch_store_voxels(t, n, s); });
    if (e == hipSuccess)
        e = timed(h, SIMLOD_KERNEL_FINISH, s, [&] { return launch_finish(t, s); });
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->h_status, &h->t.ctr->status, sizeof(u32), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(h->status_ev, s);
    if (e == hipSuccess) h->status_pending = true;
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
    return poll_status(h, true);
}

}  // namespace

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
    simlod_octree* h = new (std::nothrow) simlod_octree();
    if (!h) return SIMLOD_ERR_OUT_OF_MEMORY;
    h->cfg = *cfg;
    h->device = cfg->device;
    std::memset(&h->acc, 0, sizeof(h->acc));
    DevTree& t = h->t;
    std::memset(&t, 0, sizeof(t));
    const u64 N = cfg->max_nodes;
    const u64 work = cfg->max_batch + cfg->spill_capacity;
    h->hash_entries = next_pow2(2 * cfg->backlog_capacity);
    t.dir_depth = std::min<u32>(cfg->max_depth, kDirMaxDepth);
    const u32 hist_slots = cfg->hist_capacity ? cfg->hist_capacity : 8192u;
    bool ok = dalloc(h, &t.child, N) && dalloc(h, &t.count, N) && dalloc(h, &t.cnt, N) &&
              dalloc(h, &t.hslot, N) && dalloc(h, &t.geo, N) && dalloc(h, &t.grid, N) &&
              dalloc(h, &t.tab, N) && dalloc(h, &t.tabcap, N) && dalloc(h, &t.nchunks, N) &&
              dalloc(h, &t.newv, N) && dalloc(h, &t.ctr, 1) &&
              dalloc(h, &t.dir, dir_offset(t.dir_depth + 1u)) &&
              dalloc(h, &t.spill_rec, cfg->spill_capacity) &&
              dalloc(h, &t.spill_key, cfg->spill_capacity) && dalloc(h, &t.touched, N) &&
              dalloc(h, &t.pending[0], N) && dalloc(h, &t.pending[1], N) &&
              dalloc(h, &t.zero_list, N) &&
              dalloc(h, &t.hist, (u64)hist_slots * kHistEntries) && dalloc(h, &t.final_list, N) &&
              dalloc(h, &t.vtouched, N) && dalloc(h, &t.amask[0], work) &&
              dalloc(h, &t.amask[1], work) && dalloc(h, &t.htag, h->hash_entries) &&
              dalloc(h, &t.hval, h->hash_entries) &&
              dalloc(h, &t.claims, cfg->backlog_capacity * kStripes);
    const u32 C = cfg->chunk_capacity;
    const u64 chunk_bytes = (u64)C * 20u + 4u;
    t.chunk_blocks = (u32)((chunk_bytes + kBlockBytes - 1) / kBlockBytes);
    const u64 cells = 1ull << (3 * cfg->grid_bits);
    t.grid_words = (u32)std::max<u64>(1, cells / 32);
    t.grid_blocks = (u32)((t.grid_words * 4ull + kBlockBytes - 1) / kBlockBytes);
    u64 arena_bytes = cfg->arena_bytes;
    if (ok && arena_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) ok = false;
        // pool entries need 4 bytes per chunk of the arena as well
        arena_bytes = (u64)((double)fr * 0.9 * (double)chunk_bytes / (double)(chunk_bytes + 4));
    }
    u64 blocks = std::min<u64>(arena_bytes / kBlockBytes, 0xFFFFFFF0ull);
    t.arena_blocks = (u32)blocks;
    t.pool_cap = t.arena_blocks / t.chunk_blocks + 1;
    ok = ok && blocks > 0 && dalloc(h, &t.arena, blocks * (u64)kBlockBytes) &&
         dalloc(h, &t.pool, t.pool_cap);
    if (ok && hipHostMalloc((void**)&h->h_status, sizeof(u32), hipHostMallocDefault) != hipSuccess)
        ok = false;
    if (ok && hipEventCreateWithFlags(&h->status_ev, hipEventDisableTiming) != hipSuccess)
        ok = false;
    if (!ok) {
        std::snprintf(g_last_error, sizeof(g_last_error), "device allocation failed (%s)",
                      hipGetErrorString(hipGetLastError()));
        free_all(h);
        delete h;
        return SIMLOD_ERR_OUT_OF_MEMORY;
    }
    *h->h_status = 0;
    t.max_nodes = cfg->max_nodes;
    t.hist_cap = hist_slots;
    t.spill_cap = (u32)cfg->spill_capacity;
    t.active_cap = (u32)work;
    t.hmask = (u32)(h->hash_entries - 1);
    t.claim_cap = (u32)cfg->backlog_capacity;
    for (int a = 0; a < 3; ++a) t.mn[a] = cfg->root_min[a];
    t.size = cfg->root_size;
    t.K = cfg->max_depth + cfg->grid_bits;
    t.r = cfg->grid_bits;
    t.R = 1u << cfg->grid_bits;
    t.Dmax = cfg->max_depth;
    t.T = cfg->leaf_capacity;
    t.C = C;
    t.scale = (float)(1u << t.K) / cfg->root_size;  // float32 division
    clear_stale_error();
    hipError_t re = launch_reset(t, h->hash_entries, nullptr);
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
    h->last_stream = s;
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

int simlod_sync(simlod_octree* h) {
    if (!h) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    if (h->poisoned) return SIMLOD_ERR_POISONED;
    return sync_handle(h);
}

namespace {

// Canonical export of the subtree rooted at the node with `root_path`.
int export_subtree(simlod_octree* h, u64 root_path, simlod_snapshot_buffers* s) {
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
        if (hn.child[node])
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
    const u64 nrec = std::max<u64>(written, 1);
    bool ok = hipMalloc((void**)&d_nodes, ns * 4ull) == hipSuccess &&
              hipMalloc((void**)&d_first, ns * 8ull) == hipSuccess &&
              hipMalloc((void**)&d_rec, nrec * 16ull) == hipSuccess &&
              hipMalloc((void**)&d_key, nrec * 4ull) == hipSuccess;
    std::vector<uint4> rec;
    std::vector<u32> key;
    if (ok) {
        rec.resize(written);
        key.resize(written);
        ok = hipMemcpy(d_nodes, order.data(), ns * 4ull, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(d_first, first.data(), ns * 8ull, hipMemcpyHostToDevice) == hipSuccess &&
             launch_gather(h->t, d_nodes, d_first, ns, d_rec, d_key, nullptr) == hipSuccess &&
             hipMemcpy(rec.data(), d_rec, written * 16ull, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(key.data(), d_key, written * 4ull, hipMemcpyDeviceToHost) == hipSuccess;
    }
    const hipError_t ge = ok ? hipSuccess : hipGetLastError();
    if (!ok) note_error("snapshot gather", ge);
    const bool oom = ge == hipErrorOutOfMemory;
    (void)hipFree(d_nodes);
    (void)hipFree(d_first);
    (void)hipFree(d_rec);
    (void)hipFree(d_key);
    if (!ok) return oom ? SIMLOD_ERR_OUT_OF_MEMORY : SIMLOD_ERR_HIP;
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
    const hipError_t re = launch_reset(h->t, h->hash_entries, s);
    if (re != hipSuccess) {
        note_error("reset kernels (launch)", re);
        clear_stale_error();
        return SIMLOD_ERR_HIP;
    }
    h->last_stream = s;
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
    drain_timing(h);
    std::memset(&h->acc, 0, sizeof(h->acc));
    h->timing_mask = kernel_mask & ((1u << SIMLOD_NUM_KERNELS) - 1u);
    return SIMLOD_OK;
}

int simlod_get_kernel_times(simlod_octree* h, simlod_kernel_times* out) {
    if (!h || !out) return SIMLOD_ERR_INVALID_ARGUMENT;
    DeviceGuard guard(h->device);
    drain_timing(h);
    *out = h->acc;
    return SIMLOD_OK;
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
        default: return "unknown status";
    }
}

}  // extern "C"
