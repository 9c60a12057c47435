// Internal interfaces between the C ABI (hv_api.hip), the index build
// (hv_build.hip) and the query kernels (hv_query.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hv.h"

namespace hv {

constexpr int kLeaf = 16;        // objects per leaf
constexpr int kFan = 16;         // children per inner node
constexpr int kMaxLevels = 16;   // node levels (2e9 objects need 8)
constexpr int kLevelShift = 27;  // stack entry: level << 27 | node index
constexpr uint32_t kIdxMask = (1u << kLevelShift) - 1;
constexpr double kCullPad = 1e-5;  // px beyond r for every cull box

// Device view of an index, passed to kernels by value.
struct DevIndex {
    const double *obj;           // Hilbert order; 2 (points) or 4 (segments) doubles each
    const double4 *nodes;        // all levels, level 0 (leaves) first; (minX, minY, maxX, maxY)
    const int64_t *meta;         // [0, kMaxLevels): level offsets; [kMaxLevels, 2*kMaxLevels): counts
    int64_t n;
    int32_t levels;
    int32_t seg;                 // 0 points, 1 segments / edges
};

// A request as the kernels see it: one tile of one index with its own
// radius / half-width.  `index` selects an entry of the batch's index table.
struct DevReq {
    int32_t z, x, y, index;
    double r;
};

struct BuildResult {
    int status;                  // HV_OK / HV_EINVAL / HV_ENOMEM / HV_EHIP
    const char *msg;
};

// Device arrays owned by one index (freed by free_index_arrays).
struct IndexArrays {
    double *obj = nullptr;
    double4 *nodes = nullptr;
    uint32_t *order = nullptr;
    int64_t *meta = nullptr;     // device copy of level_off / level_cnt
    int64_t n = 0;
    int32_t seg = 0;
    int32_t levels = 0;
    int32_t key_bits = 0;
    int64_t level_off[kMaxLevels] = {};
    int64_t level_cnt[kMaxLevels] = {};
    int64_t nodes_total = 0;
    int64_t device_bytes = 0;
};

// Builds the index on `stream` and synchronises.  `objects` is a device
// pointer; validation of coordinates happens on the device.
BuildResult build_index(const double *objects, int kind_flags, int64_t n, hipStream_t stream,
                        IndexArrays *out);
void free_index_arrays(IndexArrays *a);

struct LaunchShape {
    int block;        // 8 or 16
    int cand_cap;     // staged candidates per wave
    int waves;        // waves per workgroup
    int grid;         // workgroups of the persistent query kernel (0: fill the GPU)
    int region;       // 0: one wave per block; 32 or 64: one workgroup per region of that side
    int opl;          // region mode: objects loaded per lane at a leaf step (1, 2 or 4)
};

// LDS bytes per workgroup for a shape and the deepest index of a batch.
size_t query_lds_bytes(const LaunchShape &s, int max_levels);

// Device workspace of one batch of n requests over n_ix indexes.  The first
// staged_bytes() bytes (index table, requests, a zeroed counter) are copied
// from the host; the rest (frontiers, compacted tile list) is written by the
// kernels.
struct Workspace {
    size_t table_off, req_off, counter_off, frontier_off, fmeta_off, list_off, total;
    size_t staged_bytes() const { return frontier_off; }
};
Workspace workspace_layout(int64_t n_req, int n_ix);

// Fills the host part of a workspace (index table, requests, zero counter).
void stage_host(const Workspace &w, const DevIndex *ixs, int n_ix, const DevReq *reqs, int64_t n_req,
                unsigned char *host);

// Launches the tile-frontier and persistent query kernels for a staged
// workspace `dws` (device) on `stream`.  Masks go to out + k * 8192.
hipError_t launch_query(const Workspace &w, unsigned char *dws, int64_t n_req, int max_levels, uint8_t *out,
                        const LaunchShape &s, hipStream_t stream);

// Workgroups that fill the current device for a shape (occupancy x CUs).
int persistent_grid(const LaunchShape &s, int max_levels);

}  // namespace hv
