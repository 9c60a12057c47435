// C ABI of the tile-mask engine: argument validation (on the host, before
// any device call), ownership, errors and streams.  The operations
// themselves are in hv_build.hip (index) and hv_query.hip (masks).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <cmath>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hv.h"
#include "hv_internal.h"


namespace {

thread_local std::string t_err;
thread_local hipStream_t t_stream = nullptr;

int fail(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

int hip_status(hipError_t e, const char *where) {
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return fail(HV_ENOMEM, std::string(where) + ": out of device memory");
    return fail(HV_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// True when p is device (or managed) memory usable by kernels.
bool is_device_pointer(const void *p) {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
           at.type == hipMemoryTypeUnified;
}

hv::DevIndex dev_view(const hv_index *ix) {
    hv::DevIndex d;
    d.obj = ix->a.obj;
    d.nodes = ix->a.nodes;
    d.rep = ix->a.rep;
    d.meta = ix->a.meta;
    d.n = ix->a.n;
    d.levels = ix->a.levels;
    d.seg = ix->a.seg;
    d.order = ix->a.order;
    d.pedges = ix->p.edges;
    d.pfirst = ix->p.first;
    d.pchunk = ix->p.chunks;
    d.psuper = ix->p.supers;
    d.npoly = ix->p.npoly;
    return d;
}

int validate_tiles(const hv_tile *tiles, int64_t n_tiles) {
    for (int64_t k = 0; k < n_tiles; ++k) {
        const hv_tile &t = tiles[k];
        if (t.z < 0 || t.z > HV_MAX_ZOOM)
            return fail(HV_EINVAL, "tile " + std::to_string(k) + ": zoom outside [0, 22]");
        const int64_t side = int64_t(1) << t.z;
        if (t.x < 0 || t.y < 0 || t.x >= side || t.y >= side)
            return fail(HV_EINVAL, "tile " + std::to_string(k) + ": x or y outside [0, 2^z)");
    }
    return HV_OK;
}

int validate_style(const hv_style *style) {
    if (!style) return fail(HV_EINVAL, "style is NULL");
    const double r = style->r_px;
    if (!std::isfinite(r) || !(r > 0.0) || r > HV_MAX_RADIUS)
        return fail(HV_EINVAL, "r_px must be finite and in (0, 64]");
    return HV_OK;
}

// Wavefronts per workgroup of the default shape for a batch of n requests:
// in small batches the few heaviest regions set the time, and more waves on
// each region shorten them; in large ones the GPU is full anyway and one wave
// per region (occupancy bound by registers) does the least work per pixel.
int default_waves(int64_t n) { return n < 1024 ? 4 : n < 4096 ? 2 : 1; }

int resolve_shape(const hv_launch *l, int max_levels, hv::LaunchShape *s, int64_t n) {
    // default: one workgroup per 32x32 region with default_waves(n) waves,
    // two objects per lane at a leaf step and the smallest queue that allows
    // (small LDS); hv_launch selects any other shape
    s->block = 16;
    s->waves = default_waves(n);
    s->cand_cap = 64 * s->waves * 2;
    s->grid = 0;
    s->region = 32;
    s->opl = 2;
    if (l) {
        s->block = l->block ? l->block : 16;
        s->waves = l->waves_per_wg ? l->waves_per_wg : (l->region ? 1 : 2);
        s->grid = l->grid_wgs;
        s->region = l->region;
        s->opl = l->objs_per_lane ? l->objs_per_lane : 1;
        s->cand_cap = l->cand_cap ? l->cand_cap : (l->region ? 64 * s->waves * s->opl : 64);
    }
    if (s->opl != 1 && s->opl != 2 && s->opl != 4) return fail(HV_EINVAL, "launch.objs_per_lane must be 1, 2 or 4");
    s->cull = l && l->cull_nodes ? l->cull_nodes : hv::kFrontier;
    if (s->cull < 1 || s->cull > hv::kFrontier) return fail(HV_EINVAL, "launch.cull_nodes must be in [0, 256]");
    if (s->region != 0 && s->region != 32 && s->region != 64)
        return fail(HV_EINVAL, "launch.region must be 0, 32 or 64");
    if (s->region && s->cand_cap < 64 * s->waves)
        return fail(HV_EINVAL, "launch.cand_cap must be at least 64 * waves_per_wg in region mode");
    if (s->block != 8 && s->block != 16 && s->block != 32)
        return fail(HV_EINVAL, "launch.block must be 8, 16 or 32");
    if (s->cand_cap < 64 || s->cand_cap > 4096) return fail(HV_EINVAL, "launch.cand_cap must be in [64, 4096]");
    if (s->waves != 1 && s->waves != 2 && s->waves != 4)
        return fail(HV_EINVAL, "launch.waves_per_wg must be 1, 2 or 4");
    if (s->grid < 0 || s->grid > (1 << 20)) return fail(HV_EINVAL, "launch.grid_wgs must be in [0, 2^20]");
    if (l && (l->aa_split < -2 || l->aa_split > 62)) return fail(HV_EINVAL, "launch.aa_split must be in [-2, 62]");
    if (hv::query_lds_bytes(*s, max_levels) > 65536)
        return fail(HV_EINVAL, "launch shape needs more than 64 KiB of LDS per workgroup");
    return HV_OK;
}

// Per-thread pinned staging buffer for the host part of a workspace.  An
// event guards it: it is only refilled once the previous copy from it has
// completed.
struct HostStage {
    unsigned char *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    ~HostStage() {
        if (pending) (void)hipEventSynchronize(ev);
        if (ev) (void)hipEventDestroy(ev);
        if (p) (void)hipHostFree(p);
    }
    hipError_t acquire(size_t bytes) {
        if (pending) {
            const hipError_t e = hipEventSynchronize(ev);
            if (e != hipSuccess) return e;
            pending = false;
        }
        if (!ev) {
            const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (bytes > cap) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
            const size_t want = bytes < 65536 ? 65536 : bytes + bytes / 2;
            const hipError_t e = hipHostMalloc((void **)&p, want, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap = want;
        }
        return hipSuccess;
    }
};
thread_local HostStage t_stage;
// the second sub-batch and the request map of an anti-aliased batch split
// into child tiles and one-pass requests
thread_local HostStage t_stage_b, t_stage_map;

// Copies the staged workspace to a fresh stream-ordered device allocation
// and launches the query; the allocation is released in stream order.
int run_batch(const hv::DevIndex *ixs, int n_ix, int max_levels, const hv::DevReq *reqs, int64_t n_req,
              uint8_t *out, const hv::LaunchShape &shape, const char *who, hipEvent_t *marks = nullptr,
              HostStage &st = t_stage) {
    const hv::Workspace w = hv::workspace_layout(n_req, n_ix);
    hipError_t e = st.acquire(w.staged_bytes());
    if (e != hipSuccess) return hip_status(e, who);
    hv::stage_host(w, ixs, n_ix, reqs, n_req, out, st.p);
    unsigned char *dws = nullptr;
    e = hipMallocAsync((void **)&dws, w.total, t_stream);
    if (e != hipSuccess) return hip_status(e, who);
    e = hipMemcpyAsync(dws, st.p, w.staged_bytes(), hipMemcpyHostToDevice, t_stream);
    if (e == hipSuccess) e = hipEventRecord(st.ev, t_stream);
    if (e == hipSuccess) {
        st.pending = true;
        e = hv::launch_query(w, dws, max_levels, shape, t_stream, marks);
    }
    const hipError_t ef = hipFreeAsync(dws, t_stream);
    if (e != hipSuccess) return hip_status(e, who);
    if (ef != hipSuccess) return hip_status(ef, who);
    return HV_OK;
}

int validate_tile(int32_t z, int32_t x, int32_t y, int64_t k) {
    if (z < 0 || z > HV_MAX_ZOOM) return fail(HV_EINVAL, "request " + std::to_string(k) + ": zoom outside [0, 22]");
    const int64_t side = int64_t(1) << z;
    if (x < 0 || y < 0 || x >= side || y >= side)
        return fail(HV_EINVAL, "request " + std::to_string(k) + ": x or y outside [0, 2^z)");
    return HV_OK;
}

int validate_r(double r, int64_t k) {
    if (!std::isfinite(r) || !(r > 0.0) || r > HV_MAX_RADIUS)
        return fail(HV_EINVAL, "request " + std::to_string(k) + ": r_px must be finite and in (0, 64]");
    return HV_OK;
}

int validate_out(uint8_t *out) {
    if (!out) return fail(HV_EINVAL, "out_masks is NULL");
    if (reinterpret_cast<uintptr_t>(out) % 16 != 0) return fail(HV_EINVAL, "out_masks must be 16-byte aligned");
    if (!is_device_pointer(out)) return fail(HV_EINVAL, "out_masks must be device memory");
    return HV_OK;
}

// The distinct indexes of a batch (its index table) and its requests in
// kernel form.
struct BatchPlan {
    std::vector<hv::DevIndex> table;
    std::vector<const hv_index *> owners;
    std::vector<hv::DevReq> reqs;
    int max_levels = 0;
};

int plan_batch(const hv_request *reqs, int64_t n, BatchPlan *p) {
    if (n < 0) return fail(HV_EINVAL, "n < 0");
    if (n > 0 && !reqs) return fail(HV_EINVAL, "reqs is NULL with n > 0");
    int dev = -1;
    bool have_dev = false;
    p->reqs.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        const hv_request &q = reqs[k];
        if (!q.index) return fail(HV_EINVAL, "request " + std::to_string(k) + ": index is NULL");
        if (q.index->kind == HV_POLYGONS)
            return fail(HV_EINVAL, "request " + std::to_string(k) + ": a polygon index renders with hv_render_fill");
        int rc = validate_tile(q.z, q.x, q.y, k);
        if (rc) return rc;
        if ((rc = validate_r(q.r_px, k))) return rc;
        int slot = -1;
        for (int j = (int)p->owners.size() - 1; j >= 0; --j)
            if (p->owners[(size_t)j] == q.index) {
                slot = j;
                break;
            }
        if (slot < 0) {
            if (q.index->device >= 0) {
                if (!have_dev) {
                    if (hipGetDevice(&dev) != hipSuccess) return hip_status(hipGetLastError(), "hipGetDevice");
                    have_dev = true;
                }
                if (dev != q.index->device)
                    return fail(HV_EINVAL, "request " + std::to_string(k) + ": index lives on another device");
            }
            slot = (int)p->owners.size();
            p->owners.push_back(q.index);
            p->table.push_back(dev_view(q.index));
            if (q.index->a.levels > p->max_levels) p->max_levels = q.index->a.levels;
        }
        p->reqs[(size_t)k] = hv::DevReq{q.z, q.x, q.y, slot, q.r_px};
    }
    return HV_OK;
}

// ---------------------------------------------------------------- tuning cache
struct TuneKey {
    int kind, zband, rband, nband;
    bool operator==(const TuneKey &o) const {
        return kind == o.kind && zband == o.zband && rband == o.rband && nband == o.nband;
    }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, hv_launch>> g_tune;

// zs, rs: host scratch of n entries each (the medians are taken in place).
TuneKey batch_key_in(const hv_request *reqs, int64_t n, int *zs, double *rs) {
    int64_t seg = 0;
    for (int64_t k = 0; k < n; ++k) {
        seg += reqs[k].index->kind != HV_POINTS;
        zs[k] = reqs[k].z;
        rs[k] = reqs[k].r_px;
    }
    std::nth_element(zs, zs + n / 2, zs + n);
    std::nth_element(rs, rs + n / 2, rs + n);
    const double rm = rs[n / 2];
    return TuneKey{seg * 2 >= n ? 1 : 0, zs[n / 2] / 4, rm <= 1.0 ? 0 : rm <= 2.0 ? 1 : rm <= 4.0 ? 2 : 3,
                   default_waves(n)};
}

TuneKey batch_key(const hv_request *reqs, int64_t n) {
    std::vector<int> zs((size_t)n);
    std::vector<double> rs((size_t)n);
    return batch_key_in(reqs, n, zs.data(), rs.data());
}

bool tuned_for_key(const TuneKey &key, hv_launch *out) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (auto &e : g_tune)
        if (e.first == key) {
            *out = e.second;
            return true;
        }
    return false;
}

bool tuned_for(const hv_request *reqs, int64_t n, hv_launch *out) {
    if (n <= 0) return false;
    return tuned_for_key(batch_key(reqs, n), out);
}

}  // namespace

extern "C" {

const char *hv_last_error(void) { return t_err.c_str(); }

int hv_set_stream(void *hip_stream) {
    t_stream = reinterpret_cast<hipStream_t>(hip_stream);
    return HV_OK;
}

hv_index *hv_index_build(const double *objects, int kind, int64_t n) {
    const int k = kind & ~HV_INPUT_MERC01;
    if (k != HV_POINTS && k != HV_SEGMENTS && k != HV_POLYGON_EDGES) {
        fail(HV_EINVAL, "unknown kind");
        return nullptr;
    }
    if (n < 0 || n > HV_MAX_OBJECTS) {
        fail(HV_EINVAL, "n outside [0, 2e9]");
        return nullptr;
    }
    if (n > 0 && !objects) {
        fail(HV_EINVAL, "objects is NULL with n > 0");
        return nullptr;
    }
    if (n > 0 && !is_device_pointer(objects)) {
        fail(HV_EINVAL, "objects must be device memory");
        return nullptr;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hv_index *ix = new (std::nothrow) hv_index;
    if (!ix) {
        fail(HV_ENOMEM, "host allocation failed");
        return nullptr;
    }
    ix->kind = k;
    if (n == 0) {  // an empty index owns no device memory and renders all-zero masks
        ix->device = -1;
        t_err.clear();
        return ix;
    }
    if (hipGetDevice(&ix->device) != hipSuccess) {
        hip_status(hipGetLastError(), "hipGetDevice");
        delete ix;
        return nullptr;
    }
    const hv::BuildResult br = hv::build_index(objects, kind, n, t_stream, &ix->a);
    if (br.status != HV_OK) {
        fail(br.status, std::string("hv_index_build: ") + br.msg);
        hv::free_index_arrays(&ix->a);
        delete ix;
        return nullptr;
    }
    if (ix->a.levels > 0) {
        double4 rb;
        const hipError_t e = hipMemcpy(&rb, ix->a.nodes + ix->a.level_off[ix->a.levels - 1], sizeof rb,
                                       hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            hip_status(e, "hv_index_build");
            hv::free_index_arrays(&ix->a);
            delete ix;
            return nullptr;
        }
        ix->root[0] = rb.x; ix->root[1] = rb.y; ix->root[2] = rb.z; ix->root[3] = rb.w;
    }
    ix->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    t_err.clear();
    return ix;
}

void hv_free(hv_index *index) {
    if (!index) return;
    hv::free_index_arrays(&index->a);
    hv::free_poly_arrays(&index->p);
    delete index;
}

hv_index *hv_polygon_index_build(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int flags) {
    if ((flags & ~HV_INPUT_MERC01) != 0) {
        fail(HV_EINVAL, "flags must be 0 or HV_INPUT_MERC01");
        return nullptr;
    }
    if (n < 0 || n > HV_MAX_OBJECTS || npoly < 0 || npoly > n / 3) {
        fail(HV_EINVAL, "n outside [0, 2e9] or npoly outside [0, n / 3]");
        return nullptr;
    }
    if (npoly > 0 && (!edges || !first)) {
        fail(HV_EINVAL, "edges or first is NULL");
        return nullptr;
    }
    if (npoly == 0 && n != 0) {
        fail(HV_EINVAL, "edges without polygons");
        return nullptr;
    }
    for (int64_t p = 0; p < npoly; ++p) {
        if ((p == 0 && first[0] != 0) || first[p + 1] - first[p] < 3) {
            fail(HV_EINVAL, "polygon " + std::to_string(p) + ": first[0] must be 0 and a polygon needs >= 3 edges");
            return nullptr;
        }
    }
    if (npoly > 0 && first[npoly] != n) {
        fail(HV_EINVAL, "first[npoly] must equal n");
        return nullptr;
    }
    if (n > 0 && !is_device_pointer(edges)) {
        fail(HV_EINVAL, "edges must be device memory");
        return nullptr;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hv_index *ix = new (std::nothrow) hv_index;
    if (!ix) {
        fail(HV_ENOMEM, "host allocation failed");
        return nullptr;
    }
    ix->kind = HV_POLYGONS;
    if (npoly == 0) {
        ix->device = -1;
        t_err.clear();
        return ix;
    }
    if (hipGetDevice(&ix->device) != hipSuccess) {
        hip_status(hipGetLastError(), "hipGetDevice");
        delete ix;
        return nullptr;
    }
    const hv::BuildResult br = hv::build_polygons(edges, n, first, npoly, flags, t_stream, &ix->a, &ix->p);
    if (br.status != HV_OK) {
        fail(br.status, std::string("hv_polygon_index_build: ") + br.msg);
        hv::free_index_arrays(&ix->a);
        hv::free_poly_arrays(&ix->p);
        delete ix;
        return nullptr;
    }
    if (ix->a.levels > 0) {
        double4 rb;
        const hipError_t e = hipMemcpy(&rb, ix->a.nodes + ix->a.level_off[ix->a.levels - 1], sizeof rb,
                                       hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            hip_status(e, "hv_polygon_index_build");
            hv_free(ix);
            return nullptr;
        }
        ix->root[0] = rb.x; ix->root[1] = rb.y; ix->root[2] = rb.z; ix->root[3] = rb.w;
    }
    ix->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    t_err.clear();
    return ix;
}

}  // extern "C"

namespace {

// Checks a fill call and resolves its shape; *empty is set for n_tiles = 0
// (nothing to launch).
int prepare_fill(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, uint8_t *out_masks,
                 const hv_launch *launch, hv::LaunchShape *shape, bool *empty) {
    *empty = false;
    if (!index) return fail(HV_EINVAL, "index is NULL");
    if (index->kind != HV_POLYGONS) return fail(HV_EINVAL, "hv_render_fill needs a polygon index");
    if (n_tiles < 0) return fail(HV_EINVAL, "n_tiles < 0");
    if (n_tiles > 0 && (!tiles || !out_masks)) return fail(HV_EINVAL, "tiles or out_masks is NULL");
    int rc = validate_tiles(tiles, n_tiles);
    if (rc) return rc;
    if ((rc = resolve_shape(launch, index->a.levels, shape, n_tiles))) return rc;
    if (!launch) {
        // filling's default at every batch size: two waves per 32 x 32 region
        shape->waves = 2;
        shape->cand_cap = 256;
    }
    if (shape->region == 0) return fail(HV_EINVAL, "filling runs in region mode: launch.region must be 32 or 64");
    shape->fill = 1;
    if (hv::query_lds_bytes(*shape, index->a.levels) > 65536)
        return fail(HV_EINVAL, "launch shape needs more than 64 KiB of LDS per workgroup");
    if (n_tiles == 0) {
        *empty = true;
        return HV_OK;
    }
    if ((rc = validate_out(out_masks))) return rc;
    if (index->device >= 0) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess) return hip_status(hipGetLastError(), "hipGetDevice");
        if (dev != index->device) return fail(HV_EINVAL, "the index lives on another device");
    }
    return HV_OK;
}

std::vector<hv::DevReq> fill_requests(const hv_tile *tiles, int64_t n_tiles) {
    std::vector<hv::DevReq> reqs((size_t)n_tiles);
    for (int64_t k = 0; k < n_tiles; ++k) reqs[(size_t)k] = hv::DevReq{tiles[k].z, tiles[k].x, tiles[k].y, 0, 0.0};
    return reqs;
}

}  // namespace

extern "C" {

int hv_render_fill(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, uint8_t *out_masks,
                   const hv_launch *launch) {
    hv::LaunchShape shape;
    bool empty = false;
    int rc = prepare_fill(index, tiles, n_tiles, out_masks, launch, &shape, &empty);
    if (rc) return rc;
    if (empty) {
        t_err.clear();
        return HV_OK;
    }
    const std::vector<hv::DevReq> reqs = fill_requests(tiles, n_tiles);
    const hv::DevIndex dv = dev_view(index);
    rc = run_batch(&dv, 1, index->a.levels, reqs.data(), n_tiles, out_masks, shape, "hv_render_fill");
    if (rc) return rc;
    t_err.clear();
    return HV_OK;
}

int hv_time_fill(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, uint8_t *out_masks,
                 const hv_launch *launch, int32_t reps, double *ms) {
    if (!ms) return fail(HV_EINVAL, "ms is NULL");
    if (reps < 1 || reps > 100000) return fail(HV_EINVAL, "reps must be in [1, 100000]");
    if (n_tiles <= 0) return fail(HV_EINVAL, "the batch is empty");
    hv::LaunchShape shape;
    bool empty = false;
    int rc = prepare_fill(index, tiles, n_tiles, out_masks, launch, &shape, &empty);
    if (rc) return rc;
    const std::vector<hv::DevReq> reqs = fill_requests(tiles, n_tiles);
    const hv::DevIndex dv = dev_view(index);
    hipEvent_t m[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreate(&m[k]);
    double sum[2] = {0.0, 0.0};
    for (int rep = 0; rep < reps && e == hipSuccess && rc == HV_OK; ++rep) {
        rc = run_batch(&dv, 1, index->a.levels, reqs.data(), n_tiles, out_masks, shape, "hv_time_fill", m);
        if (rc) break;
        if ((e = hipEventSynchronize(m[2])) != hipSuccess) break;
        float a = 0, b = 0;
        if ((e = hipEventElapsedTime(&a, m[0], m[1])) != hipSuccess) break;
        if ((e = hipEventElapsedTime(&b, m[1], m[2])) != hipSuccess) break;
        sum[0] += a;
        sum[1] += b;
    }
    for (int k = 0; k < 3; ++k)
        if (m[k]) (void)hipEventDestroy(m[k]);
    if (rc) return rc;
    if (e != hipSuccess) return hip_status(e, "hv_time_fill");
    ms[0] = sum[0] / reps;
    ms[1] = sum[1] / reps;
    t_err.clear();
    return HV_OK;
}

int hv_render_tiles_ex(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, const hv_style *style,
                       uint8_t *out_masks, const hv_launch *launch) {
    if (!index) return fail(HV_EINVAL, "index is NULL");
    if (index->kind == HV_POLYGONS) return fail(HV_EINVAL, "a polygon index renders with hv_render_fill");
    if (n_tiles < 0) return fail(HV_EINVAL, "n_tiles < 0");
    int rc = validate_style(style);
    if (rc) return rc;
    if (n_tiles > 0 && (!tiles || !out_masks)) return fail(HV_EINVAL, "tiles or out_masks is NULL");
    if ((rc = validate_tiles(tiles, n_tiles))) return rc;
    hv::LaunchShape shape;
    if ((rc = resolve_shape(launch, index->a.levels, &shape, n_tiles))) return rc;
    if (n_tiles == 0) {
        t_err.clear();
        return HV_OK;
    }
    if (reinterpret_cast<uintptr_t>(out_masks) % 16 != 0) return fail(HV_EINVAL, "out_masks must be 16-byte aligned");
    if (!is_device_pointer(out_masks)) return fail(HV_EINVAL, "out_masks must be device memory");
    int dev = -1;
    if (index->device >= 0 && (hipGetDevice(&dev) != hipSuccess || dev != index->device))
        return fail(HV_EINVAL, "the current device is not the index's device");
    std::vector<hv::DevReq> reqs((size_t)n_tiles);
    for (int64_t k = 0; k < n_tiles; ++k)
        reqs[(size_t)k] = hv::DevReq{tiles[k].z, tiles[k].x, tiles[k].y, 0, style->r_px};
    const hv::DevIndex ix = dev_view(index);
    rc = run_batch(&ix, 1, index->a.levels, reqs.data(), n_tiles, out_masks, shape, "hv_render_tiles");
    if (rc) return rc;
    t_err.clear();
    return HV_OK;
}

int hv_render_tiles(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, const hv_style *style,
                    uint8_t *out_masks) {
    return hv_render_tiles_ex(index, tiles, n_tiles, style, out_masks, nullptr);
}

int hv_index_info(const hv_index *index, hv_info *info) {
    if (!index || !info) return fail(HV_EINVAL, "NULL argument");
    info->kind = index->kind;
    info->levels = index->a.levels;
    info->n = index->a.n;
    info->nodes = index->a.nodes_total;
    info->leaf_size = hv::kLeaf;
    info->fanout = hv::kFan;
    info->key_bits = index->a.key_bits;
    info->pad = 0;
    for (int k = 0; k < 4; ++k) info->root[k] = index->root[k];
    info->device_bytes = index->a.device_bytes;
    info->build_ms = index->build_ms;
    return HV_OK;
}

int hv_index_read(const hv_index *index, int what, int level, void *host_dst, int64_t bytes) {
    if (!index || !host_dst) return fail(HV_EINVAL, "NULL argument");
    const void *src = nullptr;
    int64_t need = 0;
    const int w = index->a.seg ? 4 : 2;
    switch (what) {
    case HV_READ_ORDER:
        src = index->a.order;
        need = (int64_t)sizeof(uint32_t) * index->a.n;
        break;
    case HV_READ_OBJECTS:
        src = index->a.obj;
        need = (int64_t)sizeof(double) * w * index->a.n;
        break;
    case HV_READ_NODES:
        if (level < 0 || level >= index->a.levels) return fail(HV_EINVAL, "level out of range");
        src = index->a.nodes + index->a.level_off[level];
        need = (int64_t)sizeof(double4) * index->a.level_cnt[level];
        break;
    default:
        return fail(HV_EINVAL, "unknown array");
    }
    if (bytes != need) return fail(HV_EINVAL, "bytes does not match the array's size");
    if (need == 0) return HV_OK;
    const hipError_t e = hipMemcpy(host_dst, src, (size_t)need, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e, "hv_index_read");
    return HV_OK;
}


int hv_render_batch(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch) {
    BatchPlan p;
    int rc = plan_batch(reqs, n, &p);
    if (rc) return rc;
    hv_launch tuned;
    if (!launch && tuned_for(reqs, n, &tuned)) launch = &tuned;
    hv::LaunchShape shape;
    if ((rc = resolve_shape(launch, p.max_levels, &shape, n))) return rc;
    if (n == 0) {
        t_err.clear();
        return HV_OK;
    }
    if ((rc = validate_out(out_masks))) return rc;
    rc = run_batch(p.table.data(), (int)p.table.size(), p.max_levels, p.reqs.data(), n, out_masks, shape,
                   "hv_render_batch");
    if (rc) return rc;
    t_err.clear();
    return HV_OK;
}

}  // extern "C"

namespace {

// The shape of an anti-aliased batch: one pass in region mode, four
// sub-sample masks per region.
int aa_shape(const hv_launch *launch, int max_levels, int64_t n, hv::LaunchShape *shape) {
    int rc = resolve_shape(launch, max_levels, shape, n);
    if (rc) return rc;
    if (shape->region == 0) {
        shape->region = 32;
        if (!launch || !launch->cand_cap) shape->cand_cap = 64 * shape->waves * shape->opl;
        if (shape->cand_cap < 64 * shape->waves * shape->opl) shape->cand_cap = 64 * shape->waves * shape->opl;
    }
    shape->aa = 1;
    if (hv::query_lds_bytes(*shape, max_levels) > 65536)
        return fail(HV_EINVAL, "launch shape needs more than 64 KiB of LDS per workgroup");
    return HV_OK;
}

// An anti-aliased batch split by launch->aa_split: the requests rendered as
// child tiles (map[k] = s >= 0: children 4s .. 4s + 3 of `kids`, child
// (2x + a, 2y + b) at 4s + 2b + a, binary at 2r) and the others (map[k] =
// -1 - s: request s of `whole`, one pass).
struct AaPlan {
    std::vector<hv::DevReq> kids, whole;
    std::vector<int32_t> map;
};

bool aa_by_children(const hv_index *ix, const hv::DevReq &q, int split) {
    if (split == -1 || q.z >= HV_MAX_ZOOM || 2.0 * q.r > HV_MAX_RADIUS) return false;
    if (split == -2) return true;
    const int k = split ? split : HV_AA_SPLIT_DEFAULT;
    return (double)ix->a.n >= std::ldexp(1.0, k + 2 * q.z);
}

void plan_aa(const BatchPlan &p, int split, AaPlan *a) {
    const int64_t n = (int64_t)p.reqs.size();
    a->map.resize((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        const hv::DevReq &q = p.reqs[(size_t)k];
        if (aa_by_children(p.owners[(size_t)q.index], q, split)) {
            a->map[(size_t)k] = (int32_t)(a->kids.size() / 4);
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    a->kids.push_back(hv::DevReq{q.z + 1, 2 * q.x + c, 2 * q.y + b, q.index, 2.0 * q.r});
        } else {
            a->map[(size_t)k] = -1 - (int32_t)a->whole.size();
            a->whole.push_back(q);
        }
    }
}

// Renders an anti-aliased batch: one pass (shape sa) for every request, or,
// with requests in the child form, their child tiles in binary form (shape
// sb) and the one-pass rest into stream-ordered scratch, then the values
// assembled into out.  marks: six events (child tiles, then one pass; see
// run_batch) or NULL.
int run_aa(const BatchPlan &p, int64_t n, uint8_t *out, const hv::LaunchShape &sa, const hv::LaunchShape &sb,
           int split, const char *who, hipEvent_t *marks = nullptr) {
    AaPlan a;
    plan_aa(p, split, &a);
    const int n_ix = (int)p.table.size();
    if (a.kids.empty())
        return run_batch(p.table.data(), n_ix, p.max_levels, p.reqs.data(), n, out, sa, who,
                         marks ? marks + 3 : nullptr);
    const size_t nw = a.whole.size();
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t kid_bytes = a.kids.size() * (size_t)HV_MASK_BYTES, whole_bytes = nw * (size_t)HV_AA_BYTES;
    const size_t map_bytes = (size_t)n * sizeof(int32_t);
    uint8_t *tmp = nullptr;
    hipError_t e = t_stage_map.acquire(map_bytes);
    if (e != hipSuccess) return hip_status(e, who);
    std::memcpy(t_stage_map.p, a.map.data(), map_bytes);
    if ((e = hipMallocAsync((void **)&tmp, up(kid_bytes) + up(whole_bytes) + map_bytes, t_stream)) != hipSuccess)
        return hip_status(e, who);
    uint8_t *kids = tmp, *whole = tmp + up(kid_bytes);
    int32_t *map = reinterpret_cast<int32_t *>(tmp + up(kid_bytes) + up(whole_bytes));
    int rc = HV_OK;
    e = hipMemcpyAsync(map, t_stage_map.p, map_bytes, hipMemcpyHostToDevice, t_stream);
    if (e == hipSuccess) e = hipEventRecord(t_stage_map.ev, t_stream);
    if (e == hipSuccess) {
        t_stage_map.pending = true;
        rc = run_batch(p.table.data(), n_ix, p.max_levels, a.kids.data(), (int64_t)a.kids.size(), kids, sb, who,
                       marks);
        if (!rc && nw)
            rc = run_batch(p.table.data(), n_ix, p.max_levels, a.whole.data(), (int64_t)nw, whole, sa, who,
                           marks ? marks + 3 : nullptr, t_stage_b);
        if (!rc) e = hv::launch_aa_assemble(map, n, kids, whole, out, t_stream);
    }
    const hipError_t ef = hipFreeAsync(tmp, t_stream);
    if (rc) return rc;
    if (e != hipSuccess) return hip_status(e, who);
    if (ef != hipSuccess) return hip_status(ef, who);
    return HV_OK;
}

}  // namespace

extern "C" {

int hv_render_batch_aa(const hv_request *reqs, int64_t n, uint8_t *out_values, const hv_launch *launch) {
    BatchPlan p;
    int rc = plan_batch(reqs, n, &p);
    if (rc) return rc;
    hv::LaunchShape sa, sb;
    if ((rc = aa_shape(launch, p.max_levels, n, &sa))) return rc;
    if ((rc = resolve_shape(launch, p.max_levels, &sb, 4 * n))) return rc;
    if (n == 0) {
        t_err.clear();
        return HV_OK;
    }
    if ((rc = validate_out(out_values))) return rc;
    rc = run_aa(p, n, out_values, sa, sb, launch ? launch->aa_split : 0, "hv_render_batch_aa");
    if (rc) return rc;
    t_err.clear();
    return HV_OK;
}

}  // extern "C"

namespace {

// Kernel timing of a batch (binary masks, or anti-aliased values with aa).
int time_batch(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch, int32_t reps,
               double *ms, bool aa, const char *who) {
    if (!ms) return fail(HV_EINVAL, "ms is NULL");
    if (reps < 1 || reps > 100000) return fail(HV_EINVAL, "reps must be in [1, 100000]");
    if (n <= 0) return fail(HV_EINVAL, "the batch is empty");
    BatchPlan p;
    int rc = plan_batch(reqs, n, &p);
    if (rc) return rc;
    hv_launch tuned;
    if (!aa && !launch && tuned_for(reqs, n, &tuned)) launch = &tuned;
    hv::LaunchShape shape, sb;
    if ((rc = aa ? aa_shape(launch, p.max_levels, n, &shape) : resolve_shape(launch, p.max_levels, &shape, n)))
        return rc;
    if (aa && (rc = resolve_shape(launch, p.max_levels, &sb, 4 * n))) return rc;
    if ((rc = validate_out(out_masks))) return rc;
    // six marks: around the frontier and query kernels of the child tiles,
    // then of the one-pass requests (binary batches use the second three)
    hipEvent_t m[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 6 && e == hipSuccess; ++k) e = hipEventCreate(&m[k]);
    double sum[2] = {0.0, 0.0};
    for (int rep = 0; rep < reps && e == hipSuccess && rc == HV_OK; ++rep) {
        // a mark no kernel follows in this call stays unrecorded: record all
        // six first, so that unused pairs time zero
        for (int k = 0; k < 6 && e == hipSuccess; ++k) e = hipEventRecord(m[k], t_stream);
        if (e != hipSuccess) break;
        rc = aa ? run_aa(p, n, out_masks, shape, sb, launch ? launch->aa_split : 0, who, m)
                : run_batch(p.table.data(), (int)p.table.size(), p.max_levels, p.reqs.data(), n, out_masks, shape,
                            who, m + 3);
        if (rc) break;
        if ((e = hipStreamSynchronize(t_stream)) != hipSuccess) break;
        for (int s = 0; s < 2 && e == hipSuccess; ++s) {
            float a = 0, b = 0;
            if ((e = hipEventElapsedTime(&a, m[3 * s], m[3 * s + 1])) != hipSuccess) break;
            if ((e = hipEventElapsedTime(&b, m[3 * s + 1], m[3 * s + 2])) != hipSuccess) break;
            sum[0] += a;
            sum[1] += b;
        }
    }
    for (int k = 0; k < 6; ++k)
        if (m[k]) (void)hipEventDestroy(m[k]);
    if (rc) return rc;
    if (e != hipSuccess) return hip_status(e, who);
    ms[0] = sum[0] / reps;
    ms[1] = sum[1] / reps;
    t_err.clear();
    return HV_OK;
}

}  // namespace

extern "C" {

int hv_time_kernels(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch, int32_t reps,
                    double *ms) {
    return time_batch(reqs, n, out_masks, launch, reps, ms, false, "hv_time_kernels");
}

int hv_time_aa(const hv_request *reqs, int64_t n, uint8_t *out_values, const hv_launch *launch, int32_t reps,
               double *ms) {
    return time_batch(reqs, n, out_values, launch, reps, ms, true, "hv_time_aa");
}

int64_t hv_estimate_bytes(const hv_index *index, const hv_tile *tile, const hv_style *style) {
    if (!index || !tile) return fail(HV_EINVAL, "index or tile is NULL");
    int rc = validate_tiles(tile, 1);
    if (rc) return rc;
    if (index->kind != HV_POLYGONS && (rc = validate_style(style))) return rc;
    // A request's records in a batch workspace (request, tile frontier, its
    // size, level and region bits, list entries, part counter, completion
    // stamp), taken from the layout itself: two batch sizes that are
    // multiples of 256 leave no alignment padding between them.
    const hv::Workspace a = hv::workspace_layout(256, 1), b = hv::workspace_layout(512, 1);
    const int64_t per_request = (int64_t)(b.total - a.total) / 256;
    t_err.clear();
    return per_request + HV_MASK_BYTES;
}

int64_t hv_estimate_batch_bytes(int64_t n_requests, int32_t n_indexes) {
    static_assert(sizeof(hv::DevIndex) == 96, "hv.h documents 96 bytes per index of a batch");
    if (n_requests < 0 || n_indexes < 0 || n_indexes > 4096)
        return fail(HV_EINVAL, "n_requests < 0 or n_indexes outside [0, 4096]");
    const hv::Workspace w = hv::workspace_layout(n_requests, n_indexes);
    t_err.clear();
    return (int64_t)w.total + n_requests * (int64_t)HV_MASK_BYTES;
}

int hv_tuned_launch(const hv_request *reqs, int64_t n, hv_launch *out) {
    if (!out || n <= 0 || !reqs) return fail(HV_EINVAL, "NULL argument or empty batch");
    for (int64_t k = 0; k < n; ++k)
        if (!reqs[k].index) return fail(HV_EINVAL, "request " + std::to_string(k) + ": index is NULL");
    if (!tuned_for(reqs, n, out)) return fail(HV_EINVAL, "no tuned shape for this batch class");
    return HV_OK;
}

int hv_autotune(const hv_request *sample, int64_t n, uint8_t *scratch_masks, hv_launch *best, double *best_ms) {
    if (!best) return fail(HV_EINVAL, "best is NULL");
    if (n <= 0) return fail(HV_EINVAL, "the sample is empty");
    // Candidates are timed on growing, evenly spread parts of the sample (16
    // requests, 128, then all of it) and dropped as soon as one part takes
    // more than four times the best time seen on it, so that a shape that is
    // very slow on this kind of batch costs one short run, not a full one.
    // (Not tighter: the best shape for a small part -- more waves per region
    // -- can be twice as fast there as the best one for the whole sample.)
    constexpr int kStages = 3;
    constexpr double kDrop = 4.0;
    const int64_t sizes[kStages] = {std::min<int64_t>(n, 16), std::min<int64_t>(n, 128), n};
    BatchPlan plans[kStages];
    for (int st = 0; st < kStages; ++st) {
        std::vector<hv_request> part((size_t)sizes[st]);
        for (int64_t i = 0; i < sizes[st]; ++i) part[(size_t)i] = sample[i * n / sizes[st]];
        int rc = plan_batch(part.data(), sizes[st], &plans[st]);
        if (rc) return rc;
    }
    const BatchPlan &p = plans[kStages - 1];
    int rc = HV_OK;
    if ((rc = validate_out(scratch_masks))) return rc;
    // Candidate shapes, all in region mode: side, waves, objects per lane,
    // queue, and the cull depth in the last field (0 = 256 frontier nodes).
    // The default's three shapes come first (queues at their minimum, 64 x
    // waves x objects per lane: larger queues cost occupancy); grid 2^20
    // gives each region its own workgroup, which helps batches whose regions
    // differ widely in cost; a queue of 64 or 96 x waves (a leaf step's
    // objects taken 64 x waves at a time) frees LDS for more workgroups per
    // CU.
    // One wavefront per pixel block (region 0) is
    // not a candidate: it never won, and without the accept pass a single
    // run of it on a few dense low-zoom tiles can take seconds.
    static const hv_launch cands[] = {
        {0, 128, 1, 0, 32, 2, 0}, {0, 256, 2, 0, 32, 2, 0}, {0, 512, 4, 0, 32, 2, 0}, {0, 128, 1, 0, 32, 2, 128},
        {0, 128, 1, 0, 32, 2, 32}, {0, 512, 4, 0, 32, 2, 32}, {0, 128, 1, 1 << 20, 32, 2, 0},
        {0, 96, 1, 1 << 20, 32, 2, 0}, {0, 64, 1, 1 << 20, 32, 2, 0}, {0, 96, 1, 0, 32, 2, 0}, {0, 64, 1, 0, 32, 2, 0},
        {0, 64, 1, 0, 32, 1}, {0, 256, 1, 0, 32, 4},
        {0, 128, 2, 0, 32, 1}, {0, 256, 4, 0, 32, 1}, {0, 128, 1, 0, 64, 2}, {0, 256, 2, 0, 64, 2},
        {0, 256, 4, 0, 64, 1}, {0, 512, 4, 0, 64, 2},
    };
    // events around the two kernels only: staging and the workspace
    // allocation are the same for every shape and only add noise
    hipEvent_t m[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreate(&m[k]);
    if (e != hipSuccess) {
        for (int k = 0; k < 3; ++k)
            if (m[k]) (void)hipEventDestroy(m[k]);
        return hip_status(e, "hv_autotune");
    }
    double stage_best[kStages] = {1e300, 1e300, 1e300};
    constexpr double kMargin = 0.03;
    double chosen_ms = 1e300;
    int best_k = -1;
    for (int k = 0; k < (int)(sizeof(cands) / sizeof(cands[0])) && rc == HV_OK && e == hipSuccess; ++k) {
        hv::LaunchShape shape;
        if (resolve_shape(&cands[k], p.max_levels, &shape, n)) continue;  // does not fit this batch
        for (int st = 0; st < kStages; ++st) {
            if (st < kStages - 1 && sizes[st] == sizes[st + 1]) continue;
            const BatchPlan &q = plans[st];
            const int reps = st == kStages - 1 ? 4 : 2;
            float ms_min = 1e30f;
            for (int rep = 0; rep < reps; ++rep) {
                rc = run_batch(q.table.data(), (int)q.table.size(), q.max_levels, q.reqs.data(), sizes[st],
                               scratch_masks, shape, "hv_autotune", m);
                if (rc) break;
                if ((e = hipEventSynchronize(m[2])) != hipSuccess) break;
                float ms = 0;
                if ((e = hipEventElapsedTime(&ms, m[0], m[2])) != hipSuccess) break;
                if (rep > 0 && ms < ms_min) ms_min = ms;  // the first run warms up
                if (rep == 0 && ms > kDrop * stage_best[st]) {
                    ms_min = ms;  // far behind already: no need to repeat
                    break;
                }
            }
            if (rc || e != hipSuccess) break;
            if (ms_min > kDrop * stage_best[st]) break;
            // on the whole sample a later candidate must beat the chosen one
            // by kMargin, so that shapes within noise of each other do not
            // trade places from run to run (the default shapes come first)
            if (st == kStages - 1 && (best_k < 0 || ms_min < (1.0 - kMargin) * chosen_ms)) {
                best_k = k;
                chosen_ms = ms_min;
            }
            if (ms_min < stage_best[st]) stage_best[st] = ms_min;
        }
    }
    for (int k = 0; k < 3; ++k) (void)hipEventDestroy(m[k]);
    if (rc) return rc;
    if (e != hipSuccess) return hip_status(e, "hv_autotune");
    if (best_k < 0) return fail(HV_EINVAL, "no candidate shape fits this batch");
    *best = cands[best_k];
    if (best_ms) *best_ms = chosen_ms;
    const TuneKey key = batch_key(sample, n);
    std::lock_guard<std::mutex> g(g_tune_mu);
    bool found = false;
    for (auto &x : g_tune)
        if (x.first == key) {
            x.second = *best;
            found = true;
        }
    if (!found) g_tune.push_back({key, *best});
    t_err.clear();
    return HV_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batcher
struct hv_batcher {
    struct Slot {
        unsigned char *host = nullptr;  // pinned staging
        unsigned char *dev = nullptr;   // device workspace
        hipGraph_t graph[3] = {nullptr, nullptr, nullptr};  // one per shape class
        hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
        hipEvent_t done = nullptr;
        bool pending = false;
        int64_t n = 0;
    };
    int64_t max_req = 0;
    int max_ix = 0, max_levels = 0, device = 0;
    // shape class k runs batches of up to limit[k] requests (a given launch:
    // one class; NULL: the default's classes by batch size)
    int n_shapes = 0;
    int64_t limit[3] = {0, 0, 0};
    hv::LaunchShape shape[3]{};
    hv::Workspace w{};
    hipStream_t capture = nullptr;
    Slot slot[2];
    int next = 0, last = -1;
    double khz = 0;  // wall clock rate
};

namespace {

void batcher_release(hv_batcher *b) {
    for (auto &s : b->slot) {
        if (s.pending) (void)hipEventSynchronize(s.done);
        for (int k = 0; k < 3; ++k) {
            if (s.exec[k]) (void)hipGraphExecDestroy(s.exec[k]);
            if (s.graph[k]) (void)hipGraphDestroy(s.graph[k]);
        }
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.dev) (void)hipFree(s.dev);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

}  // namespace

extern "C" {

hv_batcher *hv_batcher_create(int64_t max_requests, int32_t max_indexes, int32_t max_levels,
                              const hv_launch *launch) {
    if (max_requests < 1 || max_requests > (int64_t(1) << 24)) {
        fail(HV_EINVAL, "max_requests must be in [1, 2^24]");
        return nullptr;
    }
    if (max_indexes < 1 || max_indexes > 4096) {
        fail(HV_EINVAL, "max_indexes must be in [1, 4096]");
        return nullptr;
    }
    if (max_levels < 1 || max_levels > hv::kMaxLevels) {
        fail(HV_EINVAL, "max_levels must be in [1, 16]");
        return nullptr;
    }
    hv::LaunchShape shape[3];
    int64_t limit[3] = {max_requests, max_requests, max_requests};
    int n_shapes = 0;
    if (launch) {
        if (resolve_shape(launch, max_levels, &shape[0], max_requests)) return nullptr;
        n_shapes = 1;
    } else {
        // the default's shape classes this batcher can meet: below 1024
        // requests, below 4096, and beyond
        static const int64_t bounds[3] = {1023, 4095, int64_t(1) << 24};
        for (int k = 0; k < 3; ++k) {
            const int64_t hi = std::min(bounds[k], max_requests);
            if (resolve_shape(nullptr, max_levels, &shape[n_shapes], hi)) return nullptr;
            limit[n_shapes++] = hi;
            if (hi == max_requests) break;
        }
    }
    hv_batcher *b = new (std::nothrow) hv_batcher;
    if (!b) {
        fail(HV_ENOMEM, "host allocation failed");
        return nullptr;
    }
    b->max_req = max_requests;
    b->max_ix = max_indexes;
    b->max_levels = max_levels;
    b->n_shapes = n_shapes;
    for (int k = 0; k < n_shapes; ++k) {
        b->shape[k] = shape[k];
        b->limit[k] = limit[k];
    }
    b->w = hv::workspace_layout(max_requests, max_indexes);
    hipError_t e = hipGetDevice(&b->device);
    int khz = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device);
    b->khz = khz;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    for (int k = 0; k < n_shapes; ++k)
        (void)hv::persistent_grid(shape[k], max_levels);  // occupancy queries outside the captures
    for (auto &s : b->slot) {
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.host, b->w.staged_bytes(), hipHostMallocDefault);
        if (e == hipSuccess) {
            std::memset(s.host, 0, b->w.staged_bytes());
            e = hipMalloc((void **)&s.dev, b->w.total);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        for (int k = 0; k < n_shapes && e == hipSuccess; ++k) {
            e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t ec = hipMemcpyAsync(s.dev, s.host, b->w.staged_bytes(), hipMemcpyHostToDevice, b->capture);
                if (ec == hipSuccess) ec = hv::launch_query(b->w, s.dev, max_levels, shape[k], b->capture);
                e = hipStreamEndCapture(b->capture, &s.graph[k]);
                if (ec != hipSuccess) e = ec;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&s.exec[k], s.graph[k], nullptr, nullptr, 0);
        }
    }
    if (e != hipSuccess) {
        hip_status(e, "hv_batcher_create");
        batcher_release(b);
        return nullptr;
    }
    t_err.clear();
    return b;
}

int hv_batcher_run(hv_batcher *b, const hv_request *reqs, int64_t n, uint8_t *out_masks) {
    if (!b) return fail(HV_EINVAL, "batcher is NULL");
    if (n > b->max_req) return fail(HV_EINVAL, "n exceeds the batcher's max_requests");
    BatchPlan p;
    int rc = plan_batch(reqs, n, &p);
    if (rc) return rc;
    if ((int)p.table.size() > b->max_ix) return fail(HV_EINVAL, "the batch names more indexes than max_indexes");
    if (p.max_levels > b->max_levels) return fail(HV_EINVAL, "an index is deeper than max_levels");
    if (n > 0 && (rc = validate_out(out_masks))) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(HV_EINVAL, "the current device is not the batcher's device");
    hv_batcher::Slot &s = b->slot[b->next];
    if (s.pending) {
        const hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return hip_status(e, "hv_batcher_run");
        s.pending = false;
    }
    hv::stage_host(b->w, p.table.data(), (int)p.table.size(), p.reqs.data(), n, out_masks, s.host);
    int k = 0;
    while (k + 1 < b->n_shapes && n > b->limit[k]) ++k;
    hipError_t e = hipGraphLaunch(s.exec[k], t_stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, t_stream);
    if (e != hipSuccess) return hip_status(e, "hv_batcher_run");
    s.pending = true;
    s.n = n;
    b->last = b->next;
    b->next ^= 1;
    t_err.clear();
    return HV_OK;
}

int hv_batcher_latency(hv_batcher *b, double *latency_us, int64_t n) {
    if (!b || (!latency_us && n > 0)) return fail(HV_EINVAL, "NULL argument");
    if (b->last < 0) return fail(HV_EINVAL, "the batcher has not run");
    hv_batcher::Slot &s = b->slot[b->last];
    if (n != s.n) return fail(HV_EINVAL, "n differs from the last run's size");
    hipError_t e = s.pending ? hipEventSynchronize(s.done) : hipSuccess;
    if (e != hipSuccess) return hip_status(e, "hv_batcher_latency");
    s.pending = false;
    if (n == 0) return HV_OK;
    hv::BatchHeader h;
    std::vector<uint64_t> ts((size_t)n);
    e = hipMemcpy(&h, s.dev + b->w.hdr_off, sizeof h, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ts.data(), s.dev + b->w.ts_off, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e, "hv_batcher_latency");
    for (int64_t k = 0; k < n; ++k) {
        const double ticks = ts[(size_t)k] > h.t_start ? (double)(ts[(size_t)k] - h.t_start) : 0.0;
        latency_us[k] = ticks / b->khz * 1e3;
    }
    return HV_OK;
}

void hv_batcher_free(hv_batcher *b) {
    if (b) batcher_release(b);
}

}  // extern "C"

// ---------------------------------------------------------------- no allocation
// hv_render_batch_noalloc runs the kernels of hv_render_batch on a batch
// workspace held in `scratch`, a file-scope device array, instead of a
// stream-ordered allocation.  Each device holds its own copy of the array for
// the life of the process; its address on a device is looked up once, with
// that device current, and kept in g_scratch_dev.  Host code never uses the
// array's name as an address (on the host it only names the symbol).
// The workspace's counters start at zero because the staged header copied in
// by every call holds them; everything else in it is written by the kernels
// before it is read.
namespace {
constexpr size_t kScratchBytes = size_t(5) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_noalloc_mu;                    // guards everything below
void *g_scratch_dev[kMaxDevices] = {};      // per device: the address of its `scratch`
// host staging of one call: the staged part of the workspace, the requests in
// kernel form, and the medians' scratch of the tuned-shape lookup
alignas(256) unsigned char g_noalloc_host[size_t(128) << 10];
hv::DevReq g_noalloc_reqs[HV_NOALLOC_MAX_REQUESTS];
int g_noalloc_z[HV_NOALLOC_MAX_REQUESTS];
double g_noalloc_r[HV_NOALLOC_MAX_REQUESTS];

// The address of `scratch` on device dev (current); looked up on first use.
int scratch_on(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HV_EINVAL, "hv_render_batch_noalloc: device ordinal above 63");
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hv_render_batch_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return fail(HV_EHIP, "hv_render_batch_noalloc: hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_dev[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_dev[dev]);
    return HV_OK;
}

}  // namespace

extern "C" {

int hv_render_batch_noalloc(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch) {
    if (n < 0) return fail(HV_EINVAL, "n < 0");
    if (n > HV_NOALLOC_MAX_REQUESTS)
        return fail(HV_EINVAL, "n = " + std::to_string(n) + " exceeds HV_NOALLOC_MAX_REQUESTS (" +
                                   std::to_string(HV_NOALLOC_MAX_REQUESTS) + "), the static scratch's capacity");
    if (n > 0 && !reqs) return fail(HV_EINVAL, "reqs is NULL with n > 0");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    // validation and the index table, as plan_batch does, into static storage
    hv::DevIndex table[HV_NOALLOC_MAX_INDEXES];
    const hv_index *owners[HV_NOALLOC_MAX_INDEXES];
    int n_ix = 0, max_levels = 0, dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_status(hipGetLastError(), "hipGetDevice");
    for (int64_t k = 0; k < n; ++k) {
        const hv_request &q = reqs[k];
        if (!q.index) return fail(HV_EINVAL, "request " + std::to_string(k) + ": index is NULL");
        if (q.index->kind == HV_POLYGONS)
            return fail(HV_EINVAL, "request " + std::to_string(k) + ": a polygon index renders with hv_render_fill");
        int rc = validate_tile(q.z, q.x, q.y, k);
        if (rc) return rc;
        if ((rc = validate_r(q.r_px, k))) return rc;
        int slot = -1;
        for (int j = n_ix - 1; j >= 0; --j)
            if (owners[j] == q.index) {
                slot = j;
                break;
            }
        if (slot < 0) {
            if (q.index->device >= 0 && q.index->device != dev)
                return fail(HV_EINVAL, "request " + std::to_string(k) + ": index lives on another device");
            if (n_ix == HV_NOALLOC_MAX_INDEXES)
                return fail(HV_EINVAL, "the batch names more than HV_NOALLOC_MAX_INDEXES (" +
                                           std::to_string(HV_NOALLOC_MAX_INDEXES) + ") indexes");
            slot = n_ix++;
            owners[slot] = q.index;
            table[slot] = dev_view(q.index);
            if (q.index->a.levels > max_levels) max_levels = q.index->a.levels;
        }
        g_noalloc_reqs[k] = hv::DevReq{q.z, q.x, q.y, slot, q.r_px};
    }
    hv_launch tuned;
    if (!launch && n > 0 && tuned_for_key(batch_key_in(reqs, n, g_noalloc_z, g_noalloc_r), &tuned)) launch = &tuned;
    hv::LaunchShape shape;
    int rc = resolve_shape(launch, max_levels, &shape, n);
    if (rc) return rc;
    if (n == 0) {
        t_err.clear();
        return HV_OK;
    }
    if ((rc = validate_out(out_masks))) return rc;
    const hv::Workspace w = hv::workspace_layout(n, n_ix);
    if (w.total > kScratchBytes || w.staged_bytes() > sizeof(g_noalloc_host))
        return fail(HV_EINVAL, "hv_render_batch_noalloc: the batch's workspace exceeds the static scratch");
    unsigned char *ws = nullptr;
    if ((rc = scratch_on(dev, &ws))) return rc;
    hv::stage_host(w, table, n_ix, g_noalloc_reqs, n, out_masks, g_noalloc_host);
    // The staged bytes travel from pageable static memory; the wait makes sure
    // the copy has read them before the next call may overwrite them.  The
    // copy is ordered after earlier work on this stream, so a call never
    // overwrites a workspace that an earlier call on the same stream still uses.
    hipError_t e = hipMemcpyAsync(ws, g_noalloc_host, w.staged_bytes(), hipMemcpyHostToDevice, t_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t_stream);
    if (e == hipSuccess) e = hv::launch_query(w, ws, max_levels, shape, t_stream);
    if (e != hipSuccess) return hip_status(e, "hv_render_batch_noalloc");
    t_err.clear();
    return HV_OK;
}

}  // extern "C"
