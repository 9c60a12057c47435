// C ABI of the tile-mask engine: argument validation (on the host, before
// any device call), ownership, errors and streams.  The operations
// themselves are in hv_build.hip (index) and hv_query.hip (masks).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/hv.h"
#include "hv_internal.h"

struct hv_index {
    hv::IndexArrays a;
    int kind = 0;
    int device = 0;
    double root[4] = {0, 0, 0, 0};
    double build_ms = 0;
};

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
    d.meta = ix->a.meta;
    d.n = ix->a.n;
    d.levels = ix->a.levels;
    d.seg = ix->a.seg;
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

int resolve_shape(const hv_launch *l, int max_levels, hv::LaunchShape *s) {
    // default: one single-wave workgroup per 32x32 region (fastest on the
    // benchmark workload); hv_launch selects any other shape
    s->block = 16;
    s->cand_cap = 64;
    s->waves = 1;
    s->grid = 0;
    s->region = 32;
    s->opl = 1;
    if (l) {
        s->block = l->block ? l->block : 16;
        s->cand_cap = l->cand_cap ? l->cand_cap : 64;
        s->waves = l->waves_per_wg ? l->waves_per_wg : (l->region ? 1 : 2);
        s->grid = l->grid_wgs;
        s->region = l->region;
        s->opl = l->objs_per_lane ? l->objs_per_lane : 1;
    }
    if (s->opl != 1 && s->opl != 2 && s->opl != 4) return fail(HV_EINVAL, "launch.objs_per_lane must be 1, 2 or 4");
    if (s->region != 0 && s->region != 32 && s->region != 64)
        return fail(HV_EINVAL, "launch.region must be 0, 32 or 64");
    if (s->region && s->cand_cap < 64 * s->waves * s->opl)
        return fail(HV_EINVAL, "launch.cand_cap must be at least 64 * waves_per_wg * objs_per_lane in region mode");
    if (s->block != 8 && s->block != 16 && s->block != 32)
        return fail(HV_EINVAL, "launch.block must be 8, 16 or 32");
    if (s->cand_cap < 64 || s->cand_cap > 4096) return fail(HV_EINVAL, "launch.cand_cap must be in [64, 4096]");
    if (s->waves != 1 && s->waves != 2 && s->waves != 4)
        return fail(HV_EINVAL, "launch.waves_per_wg must be 1, 2 or 4");
    if (s->grid < 0 || s->grid > (1 << 20)) return fail(HV_EINVAL, "launch.grid_wgs must be in [0, 2^20]");
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

// Copies the staged workspace to a fresh stream-ordered device allocation
// and launches the query; the allocation is released in stream order.
int run_batch(const hv::DevIndex *ixs, int n_ix, int max_levels, const hv::DevReq *reqs, int64_t n_req,
              uint8_t *out, const hv::LaunchShape &shape, const char *who) {
    const hv::Workspace w = hv::workspace_layout(n_req, n_ix);
    hipError_t e = t_stage.acquire(w.staged_bytes());
    if (e != hipSuccess) return hip_status(e, who);
    hv::stage_host(w, ixs, n_ix, reqs, n_req, t_stage.p);
    unsigned char *dws = nullptr;
    e = hipMallocAsync((void **)&dws, w.total, t_stream);
    if (e != hipSuccess) return hip_status(e, who);
    e = hipMemcpyAsync(dws, t_stage.p, w.staged_bytes(), hipMemcpyHostToDevice, t_stream);
    if (e == hipSuccess) e = hipEventRecord(t_stage.ev, t_stream);
    if (e == hipSuccess) {
        t_stage.pending = true;
        e = hv::launch_query(w, dws, n_req, max_levels, out, shape, t_stream);
    }
    const hipError_t ef = hipFreeAsync(dws, t_stream);
    if (e != hipSuccess) return hip_status(e, who);
    if (ef != hipSuccess) return hip_status(ef, who);
    return HV_OK;
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
    delete index;
}

int hv_render_tiles_ex(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, const hv_style *style,
                       uint8_t *out_masks, const hv_launch *launch) {
    if (!index) return fail(HV_EINVAL, "index is NULL");
    if (n_tiles < 0) return fail(HV_EINVAL, "n_tiles < 0");
    int rc = validate_style(style);
    if (rc) return rc;
    if (n_tiles > 0 && (!tiles || !out_masks)) return fail(HV_EINVAL, "tiles or out_masks is NULL");
    if ((rc = validate_tiles(tiles, n_tiles))) return rc;
    hv::LaunchShape shape;
    if ((rc = resolve_shape(launch, index->a.levels, &shape))) return rc;
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

}  // extern "C"
