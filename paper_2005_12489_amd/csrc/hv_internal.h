// Internal interfaces between the C ABI (hv_api.hip), the index build
// (hv_build.hip) and the query kernels (hv_query.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hv.h"

namespace hv {

constexpr int kLeaf = 16;        // objects per leaf
constexpr int kFan = 16;         // children per inner node
constexpr int kEdgeChunk = 8;    // polygon edges per chunk box (filling)
constexpr int kChunkSuper = 8;   // chunk boxes per super-chunk box (filling)
constexpr int kFrontier = 256;   // most nodes in a tile's frontier
constexpr int kMaxLevels = 16;   // node levels (2e9 objects need 8)
constexpr int kLevelShift = 27;  // stack entry: level << 27 | node index
constexpr uint32_t kIdxMask = (1u << kLevelShift) - 1;
constexpr double kCullPad = 1e-5;  // px beyond r for every cull box

// Device view of an index, passed to kernels by value.
struct DevIndex {
    const double *obj;           // Hilbert order; 2 (points) or 4 (segments) doubles each
    const double4 *nodes;        // all levels, level 0 (leaves) first; (minX, minY, maxX, maxY)
    const double2 *rep;          // per node, same order: the first vertex of its first object
    const int64_t *meta;         // [0, kMaxLevels): level offsets; [kMaxLevels, 2*kMaxLevels): counts
    int64_t n;
    int32_t levels;
    int32_t seg;                 // 0 points, 1 segments / edges
    // polygon indexes only (filling): the tree above holds the polygons'
    // bounding boxes as diagonals, in sorted order
    const uint32_t *order;       // sorted position -> polygon
    const double *pedges;        // edges, 4 doubles each, polygon after polygon in sorted order
    const int64_t *pfirst;       // the polygon at sorted position k owns edges [pfirst[k], pfirst[k + 1])
    const float4 *pchunk;        // chunk c: a box holding edges [kEdgeChunk c, kEdgeChunk (c + 1))
    const float4 *psuper;        // super-chunk s: a box holding chunks [kChunkSuper s, kChunkSuper (s + 1))
    int64_t npoly;
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
    double2 *rep = nullptr;      // per node: the first vertex of its first object
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

// Device arrays of a polygon index beyond its box tree (freed by
// free_poly_arrays).
struct PolyArrays {
    double *edges = nullptr;     // projected, polygon after polygon in the tree's sorted order
    int64_t *first = nullptr;    // npoly + 1 offsets into edges, by sorted position
    float4 *chunks = nullptr;    // ceil(n_edges / kEdgeChunk) conservative float boxes
    float4 *supers = nullptr;    // ceil(chunks / kChunkSuper) unions of chunk boxes
    int64_t npoly = 0, n_edges = 0;
};

// Builds a polygon index: projects `edges` (device, n x 4 lon0, lat0, lon1,
// lat1, or normalised with HV_INPUT_MERC01 in flags; polygon p owns edges
// [first[p], first[p + 1]), `first` on the host), computes each polygon's
// bounding box, builds the Hilbert R-tree over those boxes (as diagonal
// segments), then stores the edges polygon after polygon in the tree's
// order, with a conservative box per kEdgeChunk edges.
BuildResult build_polygons(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int flags,
                           hipStream_t stream, IndexArrays *tree, PolyArrays *poly);
void free_poly_arrays(PolyArrays *p);

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
    int fill = 0;     // 1: polygon filling (region mode) instead of the distance masks
    int aa = 0;       // 1: anti-aliased values 0-4 (region mode, HV_AA_BYTES per request)
    int cull = kFrontier;  // frontier cap of the per-tile pass (cull depth)
};

// LDS bytes per workgroup for a shape and the deepest index of a batch.
size_t query_lds_bytes(const LaunchShape &s, int max_levels);

// Header of a batch, in device memory and staged from the host each launch,
// so that a captured graph's kernel arguments never change.
struct BatchHeader {
    int64_t n_req;      // live requests
    uint8_t *out;       // request k at out + k * 8192 (anti-aliased values: k * 65536)
    int32_t counter;    // tiles appended to the compacted list (0 when staged)
    int32_t ecounter;   // tiles with no data within r, listed for zero-filling (0 when staged)
    uint64_t t_start;   // wall clock when the batch started on the device
};

// Device addresses of one batch's workspace (a kernel argument).
struct DevBatch {
    BatchHeader *hdr;
    const DevIndex *ixs;
    const DevReq *reqs;
    const uint32_t *order;  // the requests by zoom, lowest first: the tile-frontier kernel's order
    uint32_t *frontier;  // per request: up to 256 frontier nodes
    int32_t *fmeta;      // per request: frontier size, frontier level, 64 bits of regions it reaches
    uint32_t *list;      // compacted list of requests with data nearby
    uint32_t *elist;     // requests whose tile has no data within r
    uint32_t *done;      // per request: parts finished
    uint64_t *ts;        // per request: wall clock at completion
};

// Device workspace of one batch of up to n_req requests over n_ix indexes.
// Its first staged_bytes() bytes (header, index table, requests) are copied
// from the host; the rest is written by the kernels.
struct Workspace {
    int64_t n_req;
    size_t hdr_off, table_off, req_off, order_off, frontier_off, fmeta_off, list_off, elist_off, done_off, ts_off,
        total;
    size_t staged_bytes() const { return frontier_off; }
};
Workspace workspace_layout(int64_t n_req, int n_ix);

// Fills the host part of a workspace: header, index table, requests, and
// their order by zoom (lowest first, stable), in which the tile-frontier
// kernel lists them for the query kernel, so that dense low-zoom tiles start
// first and the short high-zoom ones fill the end of the launch.
void stage_host(const Workspace &w, const DevIndex *ixs, int n_ix, const DevReq *reqs, int64_t n_req, uint8_t *out,
                unsigned char *host);

DevBatch device_batch(const Workspace &w, unsigned char *dws);

// Launches the tile-frontier and query kernels for a staged workspace `dws`
// (device) on `stream`; the grids cover w.n_req requests.  With `marks`
// (three events, or NULL) it records marks[0] before the frontier kernel,
// marks[1] between the two and marks[2] after the query kernel.
hipError_t launch_query(const Workspace &w, unsigned char *dws, int max_levels, const LaunchShape &s,
                        hipStream_t stream, hipEvent_t *marks = nullptr);


// Workgroups that fill the current device for a shape (occupancy x CUs).
int persistent_grid(const LaunchShape &s, int max_levels);

// Anti-aliased values of n requests (HV_AA_BYTES each at out) from child
// masks or one-pass values: map[k] >= 0 takes the 2 x 2 bit counts of the
// four 8192-byte masks at kids + 4 map[k] * 8192 (child (2x + a, 2y + b)
// at index 2b + a), map[k] < 0 copies request -1 - map[k] of `whole`.  map,
// kids, whole and out are device memory.
hipError_t launch_aa_assemble(const int32_t *map, int64_t n, const uint8_t *kids, const uint8_t *whole,
                              uint8_t *out, hipStream_t stream);

}  // namespace hv

// An index as the C ABI hands it out.
struct hv_index {
    hv::IndexArrays a;
    hv::PolyArrays p;   // polygon indexes only
    int kind = 0;
    int device = 0;     // -1 for an empty index (no device memory)
    double root[4] = {0, 0, 0, 0};
    double build_ms = 0;
};
