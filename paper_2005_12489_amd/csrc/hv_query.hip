// Per-pixel tile-mask query (binary form of the paper's Algorithm 1).
//
// Display-driven computing makes each pixel a unit of work whose value comes
// from index queries about nearby objects (Sec. 3).  On the GPU a wavefront
// owns one square block of pixels (8x8 with one pixel per lane, or 16x16
// with four): it walks the tree once with the block's box grown by r (the
// OuterBox filter of Algorithm 1, shared by the block's pixels), stages the
// objects that pass in LDS, and then every lane measures the exact FP64
// distance from its own pixel centres to each staged object.  As soon as
// every pixel of the block is lit the wavefront stops (Algorithm 1 likewise
// returns as soon as one object is found within the radius).
//
// The tree walk is wavefront-uniform: the stack lives in LDS, each step pops
// up to four nodes of the same level and the 64 lanes test their 4 x 16
// children at once; hits are pushed with one ballot.
#include <hip/hip_runtime.h>

#include "hv_internal.h"

namespace hv {
namespace {

__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Keeps a tile's workgroups on one XCD: workgroup b is dispatched to XCD
// b % 8, so consecutive logical ids are dealt out XCD by XCD.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7u, l = b >> 3, per = n >> 3, rem = n & 7u;
    return x * per + min(x, rem) + l;
}

__host__ __device__ constexpr int stack_words(int levels) { return 64 * (levels > 0 ? levels : 1); }

template <int SEG>
__host__ __device__ constexpr int cand_bytes() { return SEG ? 40 : 16; }

__host__ __device__ inline size_t wave_lds_bytes(int cap, int levels, int seg) {
    const size_t b = (size_t)stack_words(levels) * 4 + (size_t)cap * (seg ? 40 : 16);
    return (b + 15) / 16 * 16;
}

template <int BS, int SEG>
__global__ __launch_bounds__(256) void k_query_tiles(DevIndex ix, const DevTile *__restrict__ tiles,
                                                     int64_t n_tiles, double r, uint8_t *__restrict__ out,
                                                     int cap, int xcd) {
    extern __shared__ double4 smem[];
    constexpr int NB = 256 / BS;      // blocks per tile row
    constexpr int BPT = NB * NB;      // blocks per tile
    constexpr int PPL = BS * BS / 64; // pixels per lane
    constexpr int ROWSTEP = 64 / BS;  // rows between a lane's pixels
    constexpr uint32_t FULL = (1u << PPL) - 1u;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const size_t wave_bytes = wave_lds_bytes(cap, ix.levels, SEG);
    unsigned char *wbase = reinterpret_cast<unsigned char *>(smem) + wv * wave_bytes;
    uint32_t *stk = reinterpret_cast<uint32_t *>(wbase);
    double2 *ca = reinterpret_cast<double2 *>(wbase + stack_words(ix.levels) * 4);
    double2 *cd = ca + cap;                                  // segments only
    double *ci = reinterpret_cast<double *>(cd + cap);       // segments only

    const uint32_t bid = xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int64_t wid = (int64_t)bid * wpb + wv;
    if (wid >= n_tiles * BPT) return;
    const int64_t t = wid / BPT;
    const int b = (int)(wid - t * BPT);
    const int bx = b % NB, by = b / NB;
    const DevTile tl = tiles[t];

    const double S = ldexp(256.0, tl.z);       // world size in pixels
    const double iS = ldexp(1.0, -8 - tl.z);   // 1 / S, exact
    const double ox = 256.0 * (double)tl.x, oy = 256.0 * (double)tl.y;
    const double i0 = (double)(bx * BS), j0 = (double)(by * BS);
    const double m = r + kCullPad;
    // cull box (normalised): first pixel centre - m .. last pixel centre + m
    const double qx0 = ((ox + i0) + (0.5 - m)) * iS;
    const double qx1 = ((ox + i0) + ((BS - 0.5) + m)) * iS;
    const double qy0 = ((oy + j0) + (0.5 - m)) * iS;
    const double qy1 = ((oy + j0) + ((BS - 0.5) + m)) * iS;
    const double r2 = r * r;

    // this lane's pixel centres, tile-local pixels
    const double px = i0 + (double)(lane % BS) + 0.5;
    const double py0 = j0 + (double)(lane / BS) + 0.5;
    uint32_t lit = 0;

    int sp = 0;
    int ncand = 0;
    bool all_lit = false;
    if (ix.levels > 0) {
        // data bounding box test first: blocks (and tiles) that miss it
        // write zeros without a traversal
        const double4 rb = ix.nodes[ix.meta[ix.levels - 1]];
        if (rb.x <= qx1 && rb.z >= qx0 && rb.y <= qy1 && rb.w >= qy0) {
            if (lane == 0) stk[0] = ((uint32_t)(ix.levels - 1) << kLevelShift);
            sp = 1;
        }
    }
    __builtin_amdgcn_wave_barrier();

    auto flush = [&]() {
        for (int c = 0; c < ncand; ++c) {
            if (SEG) {
                const double2 a = ca[c];
                const double2 d = cd[c];
                const double inv = ci[c];
                const double wx = px - a.x;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const double wy = (py0 + (double)(k * ROWSTEP)) - a.y;
                    double tt = (wx * d.x + wy * d.y) * inv;
                    tt = fmin(fmax(tt, 0.0), 1.0);
                    const double ex = wx - tt * d.x, ey = wy - tt * d.y;
                    if (ex * ex + ey * ey <= r2) lit |= 1u << k;
                }
            } else {
                const double2 a = ca[c];
                const double dx = px - a.x;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const double dy = (py0 + (double)(k * ROWSTEP)) - a.y;
                    if (dx * dx + dy * dy <= r2) lit |= 1u << k;
                }
            }
            if ((c & 3) == 3 && __ballot(lit != FULL) == 0) break;
        }
        ncand = 0;
        all_lit = __ballot(lit != FULL) == 0;
    };

    while (sp > 0) {
        const uint32_t top = stk[sp - 1];
        const int lvl = (int)(top >> kLevelShift);
        const int j = lane >> 4;   // which popped node (kFan = kLeaf = 16)
        const int c = lane & 15;   // which child of it
        bool nv = false;
        uint32_t node = 0;
        if (j < sp) {
            const uint32_t e = stk[sp - 1 - j];
            nv = (int)(e >> kLevelShift) == lvl;
            node = e & kIdxMask;
        }
        const int npop = __popcll(__ballot(nv && c == 0));
        bool hit = false;
        if (lvl > 0) {
            const int cl = lvl - 1;
            const int64_t child = (int64_t)node * kFan + c;
            if (nv && child < ix.meta[kMaxLevels + cl]) {
                const double4 nb = ix.nodes[ix.meta[cl] + child];
                hit = nb.x <= qx1 && nb.z >= qx0 && nb.y <= qy1 && nb.w >= qy0;
            }
            sp -= npop;
            __builtin_amdgcn_wave_barrier();
            const uint64_t hm = __ballot(hit);
            if (hit) stk[sp + (int)lanes_below(hm)] = ((uint32_t)cl << kLevelShift) | (uint32_t)child;
            sp += __popcll(hm);
            __builtin_amdgcn_wave_barrier();
        } else {
            const int64_t o = (int64_t)node * kLeaf + c;
            double ax = 0, ay = 0, bxx = 0, byy = 0;
            if (nv && o < ix.n) {
                if (SEG) {
                    const double4 s = reinterpret_cast<const double4 *>(ix.obj)[o];
                    ax = s.x; ay = s.y; bxx = s.z; byy = s.w;
                    hit = fmin(ax, bxx) <= qx1 && fmax(ax, bxx) >= qx0 && fmin(ay, byy) <= qy1 && fmax(ay, byy) >= qy0;
                } else {
                    const double2 p = reinterpret_cast<const double2 *>(ix.obj)[o];
                    ax = p.x; ay = p.y;
                    hit = ax <= qx1 && ax >= qx0 && ay <= qy1 && ay >= qy0;
                }
            }
            sp -= npop;
            const uint64_t hm = __ballot(hit);
            if (hit) {
                const int slot = ncand + (int)lanes_below(hm);
                // tile-local pixel frame; scaling by S is exact
                const double ua = ax * S - ox, va = ay * S - oy;
                ca[slot] = make_double2(ua, va);
                if (SEG) {
                    const double dx = (bxx * S - ox) - ua, dy = (byy * S - oy) - va;
                    const double l2 = dx * dx + dy * dy;
                    cd[slot] = make_double2(dx, dy);
                    ci[slot] = l2 > 0.0 ? 1.0 / l2 : 0.0;
                }
            }
            ncand += __popcll(hm);
            __builtin_amdgcn_wave_barrier();
            if (ncand > cap - 64) {
                flush();
                if (all_lit) break;
            }
        }
    }
    if (!all_lit && ncand > 0) flush();

    // mask write: row-major, 32 bytes per row, column i = bit (i & 7) of byte i >> 3
    uint8_t *tm = out + t * (int64_t)HV_MASK_BYTES;
    if (BS == 8) {
        const uint64_t bal = __ballot(lit & 1u);
        if (lane < 8) tm[(by * 8 + lane) * 32 + bx] = (uint8_t)(bal >> (8 * lane));
    } else {
        uint64_t bal[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) bal[k] = __ballot((lit >> k) & 1u);
        if (lane < 16) {
            const int k = lane >> 2, q = lane & 3;
            uint64_t v = bal[0];
#pragma unroll
            for (int kk = 1; kk < PPL; ++kk) v = k == kk ? bal[kk] : v;
            const int row = by * BS + k * ROWSTEP + q;
            *reinterpret_cast<uint16_t *>(tm + row * 32 + bx * 2) = (uint16_t)(v >> (16 * q));
        }
    }
}

}  // namespace

size_t query_lds_bytes(const LaunchShape &s, int levels, int seg) {
    return (size_t)s.waves * wave_lds_bytes(s.cand_cap, levels, seg);
}

hipError_t launch_query_tiles(const DevIndex &ix, const DevTile *tiles, int64_t n_tiles, double r, uint8_t *out,
                              const LaunchShape &s, hipStream_t st) {
    const int64_t bpt = (256 / s.block) * (256 / s.block);
    const size_t lds = query_lds_bytes(s, ix.levels, ix.seg);
    const dim3 b((uint32_t)(64 * s.waves));
    // at most 2^20 tiles per launch keeps the grid far below 2^31 workgroups
    constexpr int64_t kChunk = int64_t(1) << 20;
    for (int64_t off = 0; off < n_tiles; off += kChunk) {
        const int64_t nt = n_tiles - off < kChunk ? n_tiles - off : kChunk;
        const DevTile *tp = tiles + off;
        uint8_t *op = out + off * (int64_t)HV_MASK_BYTES;
        const dim3 g((uint32_t)((nt * bpt + s.waves - 1) / s.waves));
        if (s.block == 8) {
            if (ix.seg) hipLaunchKernelGGL((k_query_tiles<8, 1>), g, b, lds, st, ix, tp, nt, r, op, s.cand_cap, s.xcd_remap);
            else hipLaunchKernelGGL((k_query_tiles<8, 0>), g, b, lds, st, ix, tp, nt, r, op, s.cand_cap, s.xcd_remap);
        } else {
            if (ix.seg) hipLaunchKernelGGL((k_query_tiles<16, 1>), g, b, lds, st, ix, tp, nt, r, op, s.cand_cap, s.xcd_remap);
            else hipLaunchKernelGGL((k_query_tiles<16, 0>), g, b, lds, st, ix, tp, nt, r, op, s.cand_cap, s.xcd_remap);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hv
