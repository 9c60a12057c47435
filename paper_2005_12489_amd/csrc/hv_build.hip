// GPU index build: project -> Hilbert keys -> LSD radix sort -> gather ->
// bottom-up packing of a Hilbert-packed R-tree.
//
// The paper keeps one R-tree per object kind, whose entries are points,
// segments or polygon edges rather than whole objects (Sec. 3.1), built
// with Boost on the CPU.  Here the tree is packed on the GPU: objects are
// ordered along a Hilbert curve through their bounding-box centres (the
// Hilbert-packed R-tree of Kamel and Faloutsos, 1993), cut into leaves of
// kLeaf consecutive objects, and each upper level groups kFan consecutive
// nodes.  Children are implicit (node i of level k owns nodes
// i*kFan .. i*kFan+kFan-1 of level k-1), so the tree has no pointers and
// every level is one contiguous array of FP64 boxes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "hv_internal.h"

namespace hv {
namespace {

constexpr int kRT = 256;            // radix-sort threads per block
constexpr int kRIPT = 16;           // keys per thread
constexpr int kRTile = kRT * kRIPT; // keys per block
constexpr double kMaxLat = 85.0511287798066;
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------ projection
// lon/lat (deg) -> normalised Web-Mercator X (east), Y (south, 0 = north).
__device__ inline void mercator(double lon, double lat, double &X, double &Y) {
    lat = fmin(fmax(lat, -kMaxLat), kMaxLat);
    const double phi = lat * (kPi / 180.0);
    X = (lon + 180.0) / 360.0;
    Y = 0.5 - log(tan(kPi / 4.0 + phi / 2.0)) / (2.0 * kPi);
}

// Hilbert index of (x, y) on a 2^bits grid (xy -> d: at each level take the
// quadrant's position along the curve, then rotate / reflect the remaining
// low bits into that quadrant's frame).
__device__ inline uint64_t hilbert_d(uint32_t x, uint32_t y, int bits) {
    uint64_t d = 0;
    for (int b = bits - 1; b >= 0; --b) {
        const uint32_t rx = (x >> b) & 1u, ry = (y >> b) & 1u;
        d |= (uint64_t)((3u * rx) ^ ry) << (2 * b);
        if (ry == 0) {
            if (rx == 1) { x = ~x; y = ~y; }
            const uint32_t t = x; x = y; y = t;
        }
    }
    return d;
}

__device__ inline uint32_t quantise(double c, int bits) {
    const double s = ldexp(1.0, bits);
    double q = floor(c * s);
    q = fmin(fmax(q, 0.0), s - 1.0);
    return (uint32_t)q;
}

template <int W>
__global__ __launch_bounds__(256) void k_project_key(const double *__restrict__ in, int64_t n, int merc,
                                                     double *__restrict__ proj, uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ ids, int bits, int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[W];
#pragma unroll
    for (int c = 0; c < W; ++c) v[c] = in[i * W + c];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < W; ++c) bad |= !isfinite(v[c]);
    if (!merc) {
#pragma unroll
        for (int c = 0; c < W; c += 2) bad |= fabs(v[c]) > 180.0 || fabs(v[c + 1]) > 90.0;
    }
    if (bad) atomicOr(err, 1);
    double p[W];
#pragma unroll
    for (int c = 0; c < W; c += 2) {
        if (merc) { p[c] = v[c]; p[c + 1] = v[c + 1]; }
        else mercator(v[c], v[c + 1], p[c], p[c + 1]);
    }
#pragma unroll
    for (int c = 0; c < W; ++c) proj[i * W + c] = p[c];
    double cx = p[0], cy = p[1];
    if constexpr (W == 4) {
        cx = 0.5 * (fmin(p[0], p[2]) + fmax(p[0], p[2]));
        cy = 0.5 * (fmin(p[1], p[3]) + fmax(p[1], p[3]));
    }
    keys[i] = hilbert_d(quantise(cx, bits), quantise(cy, bits), bits);
    ids[i] = (uint32_t)i;
}

// Projects polygon edges (4 doubles each) in their given order; flags
// coordinates that are not finite or outside [-180, 180] x [-90, 90].
__global__ __launch_bounds__(256) void k_project_edges(const double *__restrict__ in, int64_t n, int merc,
                                                       double *__restrict__ out, int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = in[i * 4 + c];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) bad |= !isfinite(v[c]);
    if (!merc) bad |= fabs(v[0]) > 180.0 || fabs(v[1]) > 90.0 || fabs(v[2]) > 180.0 || fabs(v[3]) > 90.0;
    if (bad) atomicOr(err, 1);
    double p[4] = {v[0], v[1], v[2], v[3]};
    if (!merc) {
        mercator(v[0], v[1], p[0], p[1]);
        mercator(v[2], v[3], p[2], p[3]);
    }
    reinterpret_cast<double4 *>(out)[i] = make_double4(p[0], p[1], p[2], p[3]);
}

// Bounding box of each polygon's edges, written as the diagonal segment
// (min X, min Y) - (max X, max Y), whose own box is the polygon's box.
__global__ __launch_bounds__(256) void k_polygon_boxes(const double *__restrict__ edges,
                                                       const int64_t *__restrict__ first, int64_t npoly,
                                                       double *__restrict__ diag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npoly) return;
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int64_t e = first[p]; e < first[p + 1]; ++e) {
        const double4 g = reinterpret_cast<const double4 *>(edges)[e];
        x0 = fmin(x0, fmin(g.x, g.z)); x1 = fmax(x1, fmax(g.x, g.z));
        y0 = fmin(y0, fmin(g.y, g.w)); y1 = fmax(y1, fmax(g.y, g.w));
    }
    reinterpret_cast<double4 *>(diag)[p] = make_double4(x0, y0, x1, y1);
}

// Conservative float box of each run of kEdgeChunk consecutive edges of the
// edge array (runs may straddle polygons): min rounded down, max rounded up,
// so that every edge of the run lies inside it exactly.
__device__ inline float float_down(double d) {
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ inline float float_up(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, INFINITY);
    return f;
}

__global__ __launch_bounds__(256) void k_edge_chunks(const double *__restrict__ edges, int64_t n,
                                                     float4 *__restrict__ chunks) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (n + kEdgeChunk - 1) / kEdgeChunk) return;
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    const int64_t e1 = min(n, (c + 1) * kEdgeChunk);
    for (int64_t e = c * kEdgeChunk; e < e1; ++e) {
        const double4 g = reinterpret_cast<const double4 *>(edges)[e];
        x0 = fmin(x0, fmin(g.x, g.z)); x1 = fmax(x1, fmax(g.x, g.z));
        y0 = fmin(y0, fmin(g.y, g.w)); y1 = fmax(y1, fmax(g.y, g.w));
    }
    chunks[c] = make_float4(float_down(x0), float_down(y0), float_up(x1), float_up(y1));
}

// Union of each run of kChunkSuper chunk boxes (already outward-rounded):
// the upper level of the two-level box hierarchy over a polygon's edges.
__global__ __launch_bounds__(256) void k_super_chunks(const float4 *__restrict__ chunks, int64_t nchunk,
                                                      float4 *__restrict__ supers) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (nchunk + kChunkSuper - 1) / kChunkSuper) return;
    float4 b = chunks[s * kChunkSuper];
    const int64_t c1 = min(nchunk, (s + 1) * kChunkSuper);
    for (int64_t c = s * kChunkSuper + 1; c < c1; ++c) {
        const float4 q = chunks[c];
        b = make_float4(fminf(b.x, q.x), fminf(b.y, q.y), fmaxf(b.z, q.z), fmaxf(b.w, q.w));
    }
    supers[s] = b;
}

// Copies each polygon's edges from input order to the tree's order: wave w
// of the grid moves sorted polygon w, whose edges start at src_first[order[w]]
// in `src` and at dst_first[w] in `dst`.
__global__ __launch_bounds__(256) void k_permute_polygons(const double4 *__restrict__ src,
                                                          const int64_t *__restrict__ src_first,
                                                          const uint32_t *__restrict__ order,
                                                          const int64_t *__restrict__ dst_first, int64_t npoly,
                                                          double4 *__restrict__ dst) {
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (k >= npoly) return;
    const int64_t p = order[k];
    const int64_t s0 = src_first[p], cnt = src_first[p + 1] - s0, d0 = dst_first[k];
    for (int64_t e = lane; e < cnt; e += 64) dst[d0 + e] = src[s0 + e];
}

// ------------------------------------------------------------ scans
__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Exclusive scan over the block (blockDim a multiple of 64, <= 1024).
// ws: 16 words of LDS.  All threads must call it.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *ws) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    if (w == 0) {
        uint32_t s = lane < nw ? ws[lane] : 0u;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const uint32_t y = __shfl_up(s, o, 64);
            if (lane >= o) s += y;
        }
        if (lane < nw) ws[lane] = s;
    }
    __syncthreads();
    const uint32_t off = w ? ws[w - 1] : 0u;
    *total = ws[nw - 1];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ a, int64_t m,
                                                     uint32_t *__restrict__ part) {
    __shared__ uint32_t ws[16];
    const int64_t base = (int64_t)blockIdx.x * kRTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kRIPT; ++k) {
        const int64_t idx = base + k * kRT + threadIdx.x;
        if (idx < m) s += a[idx];
    }
    uint32_t tot;
    block_excl_scan(s, &tot, ws);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *part, int64_t np) {
    __shared__ uint32_t ws[16];
    uint32_t carry = 0;
    for (int64_t b = 0; b < np; b += 1024) {
        const int64_t idx = b + threadIdx.x;
        const uint32_t v = idx < np ? part[idx] : 0u;
        uint32_t tot;
        const uint32_t e = block_excl_scan(v, &tot, ws);
        if (idx < np) part[idx] = carry + e;
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(uint32_t *__restrict__ a, int64_t m,
                                                   const uint32_t *__restrict__ part) {
    __shared__ uint32_t ws[16];
    const int64_t base = (int64_t)blockIdx.x * kRTile + (int64_t)threadIdx.x * kRIPT;
    uint32_t v[kRIPT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kRIPT; ++k) {
        v[k] = base + k < m ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t e = block_excl_scan(s, &tot, ws) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kRIPT; ++k) {
        if (base + k < m) a[base + k] = e;
        e += v[k];
    }
}

// ------------------------------------------------------------ radix sort
// Digit histogram of one block's tile; counts are digit-major so that one
// exclusive scan gives every (digit, block) its output offset.
__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                    uint32_t *__restrict__ counts, int64_t nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kRTile;
#pragma unroll
    for (int k = 0; k < kRIPT; ++k) {
        const int64_t idx = t0 + k * kRT + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Keys of a tile are visited in input order (k, wave,
// lane); within a wave, lanes holding the same digit find each other with
// eight ballots, and per-digit running bases carry the order across waves
// and across k.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                       int64_t n, int shift, const uint32_t *__restrict__ offs,
                                                       int64_t nb) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wc[4][256];
    const int tid = threadIdx.x, w = tid >> 6;
    base[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * kRTile;
    for (int k = 0; k < kRIPT; ++k) {
#pragma unroll
        for (int q = 0; q < 4; ++q) wc[q][tid] = 0;
        __syncthreads();
        const int64_t idx = t0 + k * kRT + tid;
        const bool valid = idx < n;
        const uint64_t key = valid ? kin[idx] : 0ull;
        const uint32_t val = valid ? vin[idx] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = lanes_below(m);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(m);
        __syncthreads();
        {
            uint32_t run = base[tid];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t c = wc[q][tid];
                wc[q][tid] = run;
                run += c;
            }
            base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wc[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ gather + pack
template <int W>
__global__ __launch_bounds__(256) void k_gather(const double *__restrict__ proj, const uint32_t *__restrict__ order,
                                                int64_t n, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = order[i];
#pragma unroll
    for (int c = 0; c < W; ++c) out[i * W + c] = proj[s * W + c];
}

template <int W>
__global__ __launch_bounds__(256) void k_leaf_boxes(const double *__restrict__ obj, int64_t n,
                                                    double4 *__restrict__ leaf, int64_t nleaf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int64_t lo = i * kLeaf, hi = min<int64_t>(lo + kLeaf, n);
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int64_t k = lo; k < hi; ++k) {
#pragma unroll
        for (int c = 0; c < W; c += 2) {
            const double x = obj[k * W + c], y = obj[k * W + c + 1];
            x0 = fmin(x0, x); x1 = fmax(x1, x);
            y0 = fmin(y0, y); y1 = fmax(y1, y);
        }
    }
    leaf[i] = make_double4(x0, y0, x1, y1);
}

__global__ __launch_bounds__(256) void k_level_boxes(const double4 *__restrict__ child, int64_t nchild,
                                                     double4 *__restrict__ parent, int64_t nparent) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nparent) return;
    const int64_t lo = i * kFan, hi = min<int64_t>(lo + kFan, nchild);
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int64_t k = lo; k < hi; ++k) {
        const double4 b = child[k];
        x0 = fmin(x0, b.x); y0 = fmin(y0, b.y);
        x1 = fmax(x1, b.z); y1 = fmax(y1, b.w);
    }
    parent[i] = make_double4(x0, y0, x1, y1);
}

// Node i of level l owns the sorted objects [i * 16^(l + 1), (i + 1) *
// 16^(l + 1)); its representative is the first vertex of the first of them,
// a point of an object inside the node's box.
template <int W>
__global__ __launch_bounds__(256) void k_node_reps(const double *__restrict__ obj, int shift,
                                                   double2 *__restrict__ rep, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t o = i << shift;
    rep[i] = make_double2(obj[o * W], obj[o * W + 1]);
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bits per axis of the Hilbert grid: enough for ~16 cells per object on
// average, a multiple of 4 so that the key is a whole number of digits.
int key_bits_for(int64_t n) {
    int lg = 0;
    while ((int64_t(1) << lg) < n && lg < 62) ++lg;
    int kb = (lg + 1) / 2 + 4;
    kb = (kb + 3) / 4 * 4;
    return std::min(32, std::max(8, kb));
}

struct Scratch {
    void *p[8] = {};
    int k = 0;
    ~Scratch() {
        for (int i = 0; i < k; ++i)
            if (p[i]) (void)hipFree(p[i]);
    }
    template <class T>
    hipError_t alloc(T **out, size_t bytes) {
        hipError_t e = hipMalloc((void **)out, bytes ? bytes : 1);
        if (e == hipSuccess) p[k++] = *out;
        return e;
    }
};

BuildResult hip_fail(hipError_t e) {
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return {HV_ENOMEM, "out of device memory"};
    return {HV_EHIP, hipGetErrorString(e)};
}

}  // namespace

void free_poly_arrays(PolyArrays *p) {
    if (p->edges) (void)hipFree(p->edges);
    if (p->first) (void)hipFree(p->first);
    if (p->chunks) (void)hipFree(p->chunks);
    if (p->supers) (void)hipFree(p->supers);
    p->supers = nullptr;
    p->edges = nullptr;
    p->first = nullptr;
    p->chunks = nullptr;
}

BuildResult build_polygons(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int flags,
                           hipStream_t st, IndexArrays *tree, PolyArrays *poly) {
    const int merc = (flags & HV_INPUT_MERC01) != 0;
    poly->npoly = npoly;
    poly->n_edges = n;
    tree->n = 0;
    tree->seg = 1;
    tree->levels = 0;
    if (npoly == 0) return {HV_OK, ""};
    // projected edges and offsets in input order first; once the tree has
    // sorted the polygons, both are rewritten in the tree's order so that the
    // polygons of one region lie close together in memory
    double *proj = nullptr, *diag = nullptr;
    int64_t *in_first = nullptr;
    int *err = nullptr;
    auto release = [&]() {
        if (proj) (void)hipFree(proj);
        if (in_first) (void)hipFree(in_first);
        if (diag) (void)hipFree(diag);
        if (err) (void)hipFree(err);
        proj = diag = nullptr;
        in_first = nullptr;
        err = nullptr;
    };
    auto bail = [&](hipError_t e) {
        release();
        free_poly_arrays(poly);
        free_index_arrays(tree);
        return hip_fail(e);
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&proj, sizeof(double) * 4 * (size_t)n)) != hipSuccess) return bail(e);
    if ((e = hipMalloc((void **)&in_first, sizeof(int64_t) * (size_t)(npoly + 1))) != hipSuccess) return bail(e);
    if ((e = hipMalloc((void **)&diag, sizeof(double) * 4 * (size_t)npoly)) != hipSuccess) return bail(e);
    if ((e = hipMalloc((void **)&err, sizeof(int))) != hipSuccess) return bail(e);
    if ((e = hipMemcpyAsync(in_first, first, sizeof(int64_t) * (size_t)(npoly + 1), hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return bail(e);
    if ((e = hipMemsetAsync(err, 0, sizeof(int), st)) != hipSuccess) return bail(e);
    hipLaunchKernelGGL(k_project_edges, dim3((uint32_t)cdiv(n, 256)), dim3(256), 0, st, edges, n, merc, proj, err);
    hipLaunchKernelGGL(k_polygon_boxes, dim3((uint32_t)cdiv(npoly, 256)), dim3(256), 0, st, proj, in_first, npoly,
                       diag);
    if ((e = hipGetLastError()) != hipSuccess) return bail(e);
    int herr = 0;
    if ((e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return bail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e);
    if (herr) {
        release();
        free_poly_arrays(poly);
        return {HV_EINVAL, "edges hold a non-finite coordinate, |lon| > 180 or |lat| > 90"};
    }
    const BuildResult r = build_index(diag, HV_SEGMENTS | HV_INPUT_MERC01, npoly, st, tree);
    if (r.status != HV_OK) {
        release();
        free_poly_arrays(poly);
        return r;
    }
    // offsets in the tree's order (host prefix sums over the sorted counts)
    std::vector<uint32_t> order((size_t)npoly);
    std::vector<int64_t> sorted_first((size_t)npoly + 1);
    if ((e = hipMemcpy(order.data(), tree->order, sizeof(uint32_t) * (size_t)npoly, hipMemcpyDeviceToHost)) !=
        hipSuccess)
        return bail(e);
    sorted_first[0] = 0;
    for (int64_t k = 0; k < npoly; ++k) {
        const uint32_t p = order[(size_t)k];
        sorted_first[(size_t)k + 1] = sorted_first[(size_t)k] + (first[p + 1] - first[p]);
    }
    const int64_t nchunk = cdiv(n, kEdgeChunk);
    if ((e = hipMalloc((void **)&poly->edges, sizeof(double) * 4 * (size_t)n)) != hipSuccess) return bail(e);
    if ((e = hipMalloc((void **)&poly->first, sizeof(int64_t) * (size_t)(npoly + 1))) != hipSuccess) return bail(e);
    const int64_t nsuper = cdiv(nchunk, kChunkSuper);
    if (nchunk > 0 && (e = hipMalloc((void **)&poly->chunks, sizeof(float4) * (size_t)nchunk)) != hipSuccess)
        return bail(e);
    if (nsuper > 0 && (e = hipMalloc((void **)&poly->supers, sizeof(float4) * (size_t)nsuper)) != hipSuccess)
        return bail(e);
    if ((e = hipMemcpyAsync(poly->first, sorted_first.data(), sizeof(int64_t) * (size_t)(npoly + 1),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e);
    hipLaunchKernelGGL(k_permute_polygons, dim3((uint32_t)cdiv(npoly, 4)), dim3(256), 0, st,
                       reinterpret_cast<const double4 *>(proj), in_first, tree->order, poly->first, npoly,
                       reinterpret_cast<double4 *>(poly->edges));
    if (nchunk > 0) {
        hipLaunchKernelGGL(k_edge_chunks, dim3((uint32_t)cdiv(nchunk, 256)), dim3(256), 0, st, poly->edges, n,
                           poly->chunks);
        hipLaunchKernelGGL(k_super_chunks, dim3((uint32_t)cdiv(nsuper, 256)), dim3(256), 0, st, poly->chunks,
                           nchunk, poly->supers);
    }
    if ((e = hipGetLastError()) != hipSuccess) return bail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e);
    release();
    tree->device_bytes += (int64_t)(sizeof(double) * 4 * (size_t)n + sizeof(int64_t) * (size_t)(npoly + 1) +
                                    sizeof(float4) * (size_t)(nchunk + nsuper));
    return r;
}

void free_index_arrays(IndexArrays *a) {
    if (a->obj) (void)hipFree(a->obj);
    if (a->nodes) (void)hipFree(a->nodes);
    if (a->rep) (void)hipFree(a->rep);
    if (a->order) (void)hipFree(a->order);
    if (a->meta) (void)hipFree(a->meta);
    a->obj = nullptr;
    a->nodes = nullptr;
    a->rep = nullptr;
    a->order = nullptr;
    a->meta = nullptr;
}

#define HV_TRY(expr)                          \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) {               \
            free_index_arrays(out);           \
            return hip_fail(e_);              \
        }                                     \
    } while (0)

BuildResult build_index(const double *objects, int kind_flags, int64_t n, hipStream_t st, IndexArrays *out) {
    const int kind = kind_flags & 0xff;
    const int merc = (kind_flags & HV_INPUT_MERC01) != 0;
    const int seg = kind != HV_POINTS;
    const int W = seg ? 4 : 2;
    out->n = n;
    out->seg = seg;
    out->levels = 0;
    out->nodes_total = 0;
    out->device_bytes = 0;
    if (n == 0) return {HV_OK, ""};  // empty index: no device memory at all
    {
        hipError_t e = hipMalloc((void **)&out->meta, sizeof(int64_t) * 2 * kMaxLevels);
        if (e != hipSuccess) return hip_fail(e);
    }

    // node-level sizes
    int levels = 0;
    int64_t cnt = cdiv(n, kLeaf), total = 0;
    for (;;) {
        if (levels == kMaxLevels) return {HV_EINVAL, "too many tree levels"};
        out->level_off[levels] = total;
        out->level_cnt[levels] = cnt;
        total += cnt;
        ++levels;
        if (cnt == 1) break;
        cnt = cdiv(cnt, kFan);
    }
    out->levels = levels;
    out->nodes_total = total;
    const int bits = key_bits_for(n);
    out->key_bits = bits;
    const int passes = (2 * bits + 7) / 8;
    const int64_t nb = cdiv(n, kRTile);
    const int64_t ncount = 256 * nb;
    const int64_t npart = cdiv(ncount, kRTile);

    Scratch s;
    double *proj;
    uint64_t *k0, *k1;
    uint32_t *v0, *v1, *counts, *part;
    int *err;
    HV_TRY(s.alloc(&proj, sizeof(double) * W * n));
    HV_TRY(s.alloc(&k0, sizeof(uint64_t) * n));
    HV_TRY(s.alloc(&k1, sizeof(uint64_t) * n));
    HV_TRY(s.alloc(&v1, sizeof(uint32_t) * n));
    HV_TRY(s.alloc(&counts, sizeof(uint32_t) * ncount));
    HV_TRY(s.alloc(&part, sizeof(uint32_t) * npart));
    HV_TRY(s.alloc(&err, sizeof(int)));
    HV_TRY(hipMalloc((void **)&out->obj, sizeof(double) * W * n));
    HV_TRY(hipMalloc((void **)&out->order, sizeof(uint32_t) * n));
    HV_TRY(hipMalloc((void **)&out->nodes, sizeof(double4) * total));
    HV_TRY(hipMalloc((void **)&out->rep, sizeof(double2) * total));
    v0 = out->order;  // the sort's value buffer doubles as the stored order
    out->device_bytes = (int64_t)(sizeof(double) * W * n + sizeof(uint32_t) * n +
                                  (sizeof(double4) + sizeof(double2)) * total);

    {
        int64_t meta[2 * kMaxLevels] = {};
        for (int l = 0; l < levels; ++l) {
            meta[l] = out->level_off[l];
            meta[kMaxLevels + l] = out->level_cnt[l];
        }
        HV_TRY(hipMemcpy(out->meta, meta, sizeof(meta), hipMemcpyHostToDevice));
    }
    HV_TRY(hipMemsetAsync(err, 0, sizeof(int), st));
    const int64_t g = cdiv(n, 256);
    if (seg)
        hipLaunchKernelGGL(k_project_key<4>, dim3((uint32_t)g), dim3(256), 0, st, objects, n, merc, proj, k0, v0, bits, err);
    else
        hipLaunchKernelGGL(k_project_key<2>, dim3((uint32_t)g), dim3(256), 0, st, objects, n, merc, proj, k0, v0, bits, err);
    HV_TRY(hipGetLastError());

    uint64_t *kin = k0, *kout = k1;
    uint32_t *vin = v0, *vout = v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((uint32_t)nb), dim3(kRT), 0, st, kin, n, shift, counts, nb);
        hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)npart), dim3(kRT), 0, st, counts, ncount, part);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, npart);
        hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)npart), dim3(kRT), 0, st, counts, ncount, part);
        hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)nb), dim3(kRT), 0, st, kin, vin, kout, vout, n, shift,
                           counts, nb);
        HV_TRY(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (vin != out->order)
        HV_TRY(hipMemcpyAsync(out->order, vin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));

    if (seg)
        hipLaunchKernelGGL(k_gather<4>, dim3((uint32_t)g), dim3(256), 0, st, proj, out->order, n, out->obj);
    else
        hipLaunchKernelGGL(k_gather<2>, dim3((uint32_t)g), dim3(256), 0, st, proj, out->order, n, out->obj);
    const int64_t nl = out->level_cnt[0];
    if (seg)
        hipLaunchKernelGGL(k_leaf_boxes<4>, dim3((uint32_t)cdiv(nl, 256)), dim3(256), 0, st, out->obj, n, out->nodes, nl);
    else
        hipLaunchKernelGGL(k_leaf_boxes<2>, dim3((uint32_t)cdiv(nl, 256)), dim3(256), 0, st, out->obj, n, out->nodes, nl);
    for (int l = 1; l < levels; ++l) {
        const int64_t np = out->level_cnt[l];
        hipLaunchKernelGGL(k_level_boxes, dim3((uint32_t)cdiv(np, 256)), dim3(256), 0, st,
                           out->nodes + out->level_off[l - 1], out->level_cnt[l - 1], out->nodes + out->level_off[l], np);
    }
    for (int l = 0; l < levels; ++l) {
        const int64_t np = out->level_cnt[l];
        if (seg)
            hipLaunchKernelGGL(k_node_reps<4>, dim3((uint32_t)cdiv(np, 256)), dim3(256), 0, st, out->obj, 4 * (l + 1),
                               out->rep + out->level_off[l], np);
        else
            hipLaunchKernelGGL(k_node_reps<2>, dim3((uint32_t)cdiv(np, 256)), dim3(256), 0, st, out->obj, 4 * (l + 1),
                               out->rep + out->level_off[l], np);
    }
    HV_TRY(hipGetLastError());
    int herr = 0;
    HV_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HV_TRY(hipStreamSynchronize(st));
    if (herr) {
        free_index_arrays(out);
        return {HV_EINVAL, "objects hold a non-finite coordinate, |lon| > 180 or |lat| > 90"};
    }
    return {HV_OK, ""};
}

}  // namespace hv
