// Host-side launchers of the insertion kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "octree_device.hpp"

namespace simlod {

// Largest workgroup count of each per-point kernel (the launch shape a group
// autotunes); each launch uses min(cap, what its items need).
enum ShapeKind : u32 { kShapeCount = 0, kShapeHist, kShapeSample, kShapeStore, kNumShapes };
struct LaunchShape {
    u32 cap[kNumShapes];
};
inline LaunchShape default_shape() { return LaunchShape{{1024u, 1024u, 1024u, 1024u}}; }

u32 expansion_rounds(u32 max_depth);
// 1 when a pass of `count` octrees over `items` points (or capacity) may take
// the grouped order (GroupArgs.grouped of its first kernel).
u32 grouped_pass(u32 count, u64 items);
bool is_count_leaves_kernel(const void* f);  // the pass's first kernel (graph replay)
hipError_t launch_count_leaves(const GroupArgs& ga, u64 items, const LaunchShape& sh,
                               hipStream_t s);
hipError_t launch_split_leaves(const Member* m, u32 count, u64 items, hipStream_t s);
// Passes of one octree with at least kGroupMinItems points: the first
// round's bucket counts scanned, then the batch copied into the order
// grouped by spatial bucket (nothing launched otherwise).  After the first
// round.
hipError_t launch_group_batch(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                              hipStream_t s);
hipError_t launch_count_hist(const Member* m, u32 count, u64 items, u32 round,
                             const LaunchShape& sh, hipStream_t s);
hipError_t launch_build(const Member* m, u32 count, u32 round, hipStream_t s);
// Rounds first..last (skipped at once when nothing is pending), then the
// chunks of the final leaves (launch_alloc with voxels = 0), in one launch.
// The member table must have room for two barrier words after its `count`
// entries.
hipError_t launch_rounds_alloc(const Member* m, u32 count, u64 items, u32 first, u32 last,
                               hipStream_t s);
hipError_t launch_alloc(const Member* m, u32 count, u32 voxels, hipStream_t s);
hipError_t launch_sample_store(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                               hipStream_t s);
hipError_t launch_store_voxels(const Member* m, u32 count, u64 items, const LaunchShape& sh,
                               hipStream_t s);
hipError_t launch_finish(const Member* m, u32 count, u32* status_out, hipStream_t s);
hipError_t launch_reset(const DevTree& t, u64 hash_entries, hipStream_t s);
hipError_t launch_walk(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                       uint4* out_rec, u32* out_key, u32* err, hipStream_t s);
hipError_t launch_gather(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                         uint4* out_rec, u32* out_key, hipStream_t s);

}  // namespace simlod
