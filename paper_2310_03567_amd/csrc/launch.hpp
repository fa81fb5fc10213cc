// Host-side launchers of the insertion kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "octree_device.hpp"

namespace simlod {

u32 expansion_rounds(u32 max_depth);
hipError_t launch_count_leaves(const DevTree& t, const uint4* batch, u32 n, hipStream_t s);
hipError_t launch_split_leaves(const DevTree& t, u32 n, hipStream_t s);
hipError_t launch_count_hist(const DevTree& t, const uint4* batch, u32 n, u32 base_key, u32 round,
                             hipStream_t s);
hipError_t launch_build(const DevTree& t, u32 round, hipStream_t s);
hipError_t launch_alloc(const DevTree& t, u32 voxels, hipStream_t s);
hipError_t launch_sample_store(const DevTree& t, const uint4* batch, u32 n, u32 base_key,
                               hipStream_t s);
hipError_t launch_store_voxels(const DevTree& t, u32 n, hipStream_t s);
hipError_t launch_finish(const DevTree& t, hipStream_t s);
hipError_t launch_reset(const DevTree& t, u64 hash_entries, hipStream_t s);
hipError_t launch_gather(const DevTree& t, const u32* nodes, const u64* first, u32 nn,
                         uint4* out_rec, u32* out_key, hipStream_t s);

}  // namespace simlod
