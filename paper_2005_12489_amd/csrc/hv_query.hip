// Per-pixel tile-mask query (binary form of the paper's Algorithm 1).
//
// Display-driven computing makes each pixel a unit of work whose value comes
// from index queries about nearby objects (Sec. 3).  On the GPU:
//
//  1. k_tile_frontier -- one wavefront per tile walks the tree breadth-first
//     with the tile's box grown by r and keeps the deepest level at which at
//     most 64 nodes meet it.  A tile whose frontier is empty misses all data
//     and its blocks write zeros at once (Sec. 4.1: such tiles make no task).
//  2. k_query_tiles -- one wavefront per square block of pixels (8x8, one
//     pixel per lane, or 16x16, four per lane) starts from its tile's
//     frontier and walks down with the block's box grown by r: the OuterBox
//     filter of Algorithm 1, shared by the block's pixels.  Objects that pass
//     are staged in LDS in tile-local pixel coordinates together with the
//     range of block pixels their box grown by r covers.  Small ranges are
//     tested object-parallel (one lane per object, only its own pixels: the
//     per-pixel box filter of Algorithm 1 seen from the object's side);
//     large ones pixel-parallel (every lane tests its own pixels).  Every
//     test is the exact FP64 distance against r, inclusive.  Once every
//     pixel of the block is lit the wavefront stops, as Algorithm 1 returns
//     as soon as one object lies within the radius.
//
// The tree walk is wavefront-uniform: the stack lives in LDS, each step pops
// up to four nodes of the same level and the 64 lanes test their 4 x 16
// children at once; hits are pushed with one ballot.
#include <hip/hip_runtime.h>

#include "hv_internal.h"

namespace hv {
namespace {

constexpr int kFrontier = 64;             // nodes per tile frontier
constexpr uint32_t kBigFlag = 0x80000000u;  // staged object tested pixel-parallel
constexpr int kSmallArea = 48;            // largest pixel range tested object-parallel
constexpr double kRangeEps = 1e-7;        // px, widens every pixel range

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

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// LDS of one wavefront: stack | staged objects (SoA) | block mask rows.
__host__ __device__ inline size_t wave_lds_bytes(int cap, int levels, int seg, int bs) {
    const size_t per = seg ? (16 + 16 + 8 + 4) : (16 + 4);
    return align16((size_t)stack_words(levels) * 4) + align16((size_t)cap * per) + align16((size_t)bs * 4);
}

__global__ __launch_bounds__(256) void k_tile_frontier(DevIndex ix, const DevTile *__restrict__ tiles,
                                                       int64_t n_tiles, double r, uint32_t *__restrict__ frontier,
                                                       int32_t *__restrict__ fmeta) {
    __shared__ uint32_t buf[4][2][kFrontier];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * 4 + wv;
    if (t >= n_tiles) return;
    const DevTile tl = tiles[t];
    const double iS = ldexp(1.0, -8 - tl.z);
    const double ox = 256.0 * (double)tl.x, oy = 256.0 * (double)tl.y;
    const double m = r + kCullPad;
    const double qx0 = (ox + (0.5 - m)) * iS, qx1 = (ox + (255.5 + m)) * iS;
    const double qy0 = (oy + (0.5 - m)) * iS, qy1 = (oy + (255.5 + m)) * iS;
    uint32_t *cur = buf[wv][0], *nxt = buf[wv][1];
    int ncur = 0, lvl = ix.levels - 1;
    if (ix.levels > 0) {
        const double4 rb = ix.nodes[ix.meta[ix.levels - 1]];
        if (rb.x <= qx1 && rb.z >= qx0 && rb.y <= qy1 && rb.w >= qy0) {
            if (lane == 0) cur[0] = 0;
            ncur = 1;
        }
    }
    __builtin_amdgcn_wave_barrier();
    while (lvl > 0 && ncur > 0) {
        const int cl = lvl - 1;
        const int64_t cnt = ix.meta[kMaxLevels + cl], off = ix.meta[cl];
        int nn = 0;
        for (int base = 0; base < ncur * kFan; base += 64) {
            const int k = base + lane;
            bool hit = false;
            int64_t child = 0;
            if (k < ncur * kFan) {
                child = (int64_t)cur[k / kFan] * kFan + (k % kFan);
                if (child < cnt) {
                    const double4 nb = ix.nodes[off + child];
                    hit = nb.x <= qx1 && nb.z >= qx0 && nb.y <= qy1 && nb.w >= qy0;
                }
            }
            const uint64_t hm = __ballot(hit);
            const int pos = nn + (int)lanes_below(hm);
            if (hit && pos < kFrontier) nxt[pos] = (uint32_t)child;
            nn += __popcll(hm);
            if (nn > kFrontier) break;
        }
        __builtin_amdgcn_wave_barrier();
        if (nn > kFrontier) break;
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        ncur = nn;
        --lvl;
    }
    if (lane < ncur) frontier[t * kFrontier + lane] = cur[lane];
    if (lane == 0) {
        fmeta[2 * t] = ncur;
        fmeta[2 * t + 1] = lvl;
    }
}

template <int BS, int SEG>
__global__ __launch_bounds__(256) void k_query_tiles(DevIndex ix, const DevTile *__restrict__ tiles,
                                                     const uint32_t *__restrict__ frontier,
                                                     const int32_t *__restrict__ fmeta, int64_t n_tiles, double r,
                                                     uint8_t *__restrict__ out, int cap, int xcd) {
    extern __shared__ double4 smem[];
    constexpr int NB = 256 / BS;      // blocks per tile row
    constexpr int BPT = NB * NB;      // blocks per tile
    constexpr int PPL = BS * BS / 64; // pixels per lane (pixel-parallel layout)
    constexpr int ROWSTEP = 64 / BS;  // rows between a lane's pixels
    constexpr uint32_t FULL = (1u << PPL) - 1u;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char *wbase = reinterpret_cast<unsigned char *>(smem) + wv * wave_lds_bytes(cap, ix.levels, SEG, BS);
    uint32_t *stk = reinterpret_cast<uint32_t *>(wbase);
    unsigned char *cbase = wbase + align16((size_t)stack_words(ix.levels) * 4);
    double2 *ca = reinterpret_cast<double2 *>(cbase);              // first point (tile-local px)
    double2 *cd = ca + cap;                                         // segment direction (segments only)
    double *ci = reinterpret_cast<double *>(cd + cap);              // 1 / |direction|^2 (segments only)
    uint32_t *crng = SEG ? reinterpret_cast<uint32_t *>(ci + cap)   // pixel range | big flag
                         : reinterpret_cast<uint32_t *>(ca + cap);
    uint32_t *mrow = reinterpret_cast<uint32_t *>(cbase + align16((size_t)cap * (SEG ? 44 : 20)));

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

    // pixel-parallel layout: this lane's pixel centres, tile-local pixels
    const double px = i0 + (double)(lane % BS) + 0.5;
    const double py0 = j0 + (double)(lane / BS) + 0.5;
    uint32_t lit = 0;
    if (lane < BS) mrow[lane] = 0;

    int sp = 0;
    int ncand = 0;
    bool all_lit = false;
    {
        const int fcount = fmeta[2 * t], flevel = fmeta[2 * t + 1];
        bool hit = false;
        uint32_t node = 0;
        if (lane < fcount) {
            node = frontier[t * kFrontier + lane];
            const double4 nb = ix.nodes[ix.meta[flevel] + node];
            hit = nb.x <= qx1 && nb.z >= qx0 && nb.y <= qy1 && nb.w >= qy0;
        }
        const uint64_t hm = __ballot(hit);
        if (hit) stk[lanes_below(hm)] = ((uint32_t)flevel << kLevelShift) | node;
        sp = __popcll(hm);
    }
    __builtin_amdgcn_wave_barrier();

    auto flush = [&]() {
        // object-parallel: lane k takes staged object base + k and tests
        // only the block pixels in its range
        for (int base = 0; base < ncand; base += 64) {
            const int c = base + lane;
            if (c < ncand) {
                const uint32_t rg = crng[c];
                if (!(rg & kBigFlag)) {
                    const int ilo = rg & 15, ihi = (rg >> 4) & 15, jlo = (rg >> 8) & 15, jhi = (rg >> 12) & 15;
                    const double2 a = ca[c];
                    double2 d = make_double2(0.0, 0.0);
                    double inv = 0.0;
                    if (SEG) {
                        d = cd[c];
                        inv = ci[c];
                    }
                    for (int jj = jlo; jj <= jhi; ++jj) {
                        const double wy = (j0 + (double)jj + 0.5) - a.y;
                        uint32_t bits = 0;
                        for (int ii = ilo; ii <= ihi; ++ii) {
                            const double wx = (i0 + (double)ii + 0.5) - a.x;
                            double d2;
                            if (SEG) {
                                double tt = (wx * d.x + wy * d.y) * inv;
                                tt = fmin(fmax(tt, 0.0), 1.0);
                                const double ex = wx - tt * d.x, ey = wy - tt * d.y;
                                d2 = ex * ex + ey * ey;
                            } else {
                                d2 = wx * wx + wy * wy;
                            }
                            if (d2 <= r2) bits |= 1u << ii;
                        }
                        if (bits) atomicOr(&mrow[jj], bits);
                    }
                }
            }
        }
        // pixel-parallel: every lane tests its own pixels against each large object
        for (int c = 0; c < ncand; ++c) {
            if (!(crng[c] & kBigFlag)) continue;
            const double2 a = ca[c];
            if (SEG) {
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
                const double dx = px - a.x;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const double dy = (py0 + (double)(k * ROWSTEP)) - a.y;
                    if (dx * dx + dy * dy <= r2) lit |= 1u << k;
                }
            }
        }
        ncand = 0;
        __builtin_amdgcn_wave_barrier();
        uint32_t mine = lit;
#pragma unroll
        for (int k = 0; k < PPL; ++k)
            if ((mrow[lane / BS + k * ROWSTEP] >> (lane % BS)) & 1u) mine |= 1u << k;
        all_lit = __ballot(mine != FULL) == 0;
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
        if (lvl > 0) {
            bool hit = false;
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
            bool keep = false;
            double ua = 0, va = 0, ub = 0, vb = 0;
            uint32_t rg = 0;
            if (nv && o < ix.n) {
                double ax, ay, bxx, byy;
                if (SEG) {
                    const double4 s = reinterpret_cast<const double4 *>(ix.obj)[o];
                    ax = s.x; ay = s.y; bxx = s.z; byy = s.w;
                } else {
                    const double2 p = reinterpret_cast<const double2 *>(ix.obj)[o];
                    ax = bxx = p.x; ay = byy = p.y;
                }
                if (fmin(ax, bxx) <= qx1 && fmax(ax, bxx) >= qx0 && fmin(ay, byy) <= qy1 && fmax(ay, byy) >= qy0) {
                    // tile-local pixel frame; scaling by S is exact
                    ua = ax * S - ox; va = ay * S - oy;
                    ub = bxx * S - ox; vb = byy * S - oy;
                    // block pixels whose centre lies within r of the object's box
                    const double flo_i = fmax(ceil(fmin(ua, ub) - r - 0.5 - i0 - kRangeEps), 0.0);
                    const double fhi_i = fmin(floor(fmax(ua, ub) + r - 0.5 - i0 + kRangeEps), BS - 1.0);
                    const double flo_j = fmax(ceil(fmin(va, vb) - r - 0.5 - j0 - kRangeEps), 0.0);
                    const double fhi_j = fmin(floor(fmax(va, vb) + r - 0.5 - j0 + kRangeEps), BS - 1.0);
                    if (flo_i <= fhi_i && flo_j <= fhi_j) {
                        keep = true;
                        const int ilo = (int)flo_i, ihi = (int)fhi_i, jlo = (int)flo_j, jhi = (int)fhi_j;
                        rg = (uint32_t)ilo | ((uint32_t)ihi << 4) | ((uint32_t)jlo << 8) | ((uint32_t)jhi << 12);
                        if ((ihi - ilo + 1) * (jhi - jlo + 1) > kSmallArea) rg |= kBigFlag;
                    }
                }
            }
            sp -= npop;
            const uint64_t hm = __ballot(keep);
            if (keep) {
                const int slot = ncand + (int)lanes_below(hm);
                ca[slot] = make_double2(ua, va);
                if (SEG) {
                    const double dx = ub - ua, dy = vb - va;
                    const double l2 = dx * dx + dy * dy;
                    cd[slot] = make_double2(dx, dy);
                    ci[slot] = l2 > 0.0 ? 1.0 / l2 : 0.0;
                }
                crng[slot] = rg;
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
    __builtin_amdgcn_wave_barrier();

    // mask write: row-major, 32 bytes per row, column i = bit (i & 7) of byte i >> 3
    uint8_t *tm = out + t * (int64_t)HV_MASK_BYTES;
    if (BS == 8) {
        const uint64_t bal = __ballot(lit & 1u);
        if (lane < 8) tm[(by * 8 + lane) * 32 + bx] = (uint8_t)((bal >> (8 * lane)) | mrow[lane]);
    } else {
        uint64_t bal[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) bal[k] = __ballot((lit >> k) & 1u);
        if (lane < 16) {
            const int k = lane >> 2, q = lane & 3;
            uint64_t v = bal[0];
#pragma unroll
            for (int kk = 1; kk < PPL; ++kk) v = k == kk ? bal[kk] : v;
            const uint32_t row = (uint32_t)((v >> (16 * q)) & 0xffffu) | mrow[lane];
            *reinterpret_cast<uint16_t *>(tm + (by * BS + lane) * 32 + bx * 2) = (uint16_t)row;
        }
    }
}

}  // namespace

size_t query_lds_bytes(const LaunchShape &s, int levels, int seg) {
    return (size_t)s.waves * wave_lds_bytes(s.cand_cap, levels, seg, s.block);
}

size_t query_scratch_bytes(int64_t n_tiles) {
    return (size_t)n_tiles * (sizeof(uint32_t) * kFrontier + 2 * sizeof(int32_t));
}

hipError_t launch_query_tiles(const DevIndex &ix, const DevTile *tiles, int64_t n_tiles, double r, uint8_t *out,
                              const LaunchShape &s, void *scratch, hipStream_t st) {
    const int64_t bpt = (256 / s.block) * (256 / s.block);
    const size_t lds = query_lds_bytes(s, ix.levels, ix.seg);
    const dim3 b((uint32_t)(64 * s.waves));
    uint32_t *frontier = reinterpret_cast<uint32_t *>(scratch);
    int32_t *fmeta = reinterpret_cast<int32_t *>(frontier + n_tiles * kFrontier);
    // at most 2^20 tiles per launch keeps the grid far below 2^31 workgroups
    constexpr int64_t kChunk = int64_t(1) << 20;
    for (int64_t off = 0; off < n_tiles; off += kChunk) {
        const int64_t nt = n_tiles - off < kChunk ? n_tiles - off : kChunk;
        const DevTile *tp = tiles + off;
        uint32_t *fp = frontier + off * kFrontier;
        int32_t *mp = fmeta + 2 * off;
        uint8_t *op = out + off * (int64_t)HV_MASK_BYTES;
        hipLaunchKernelGGL(k_tile_frontier, dim3((uint32_t)((nt + 3) / 4)), dim3(256), 0, st, ix, tp, nt, r, fp, mp);
        const dim3 g((uint32_t)((nt * bpt + s.waves - 1) / s.waves));
        if (s.block == 8) {
            if (ix.seg) hipLaunchKernelGGL((k_query_tiles<8, 1>), g, b, lds, st, ix, tp, fp, mp, nt, r, op, s.cand_cap, s.xcd_remap);
            else hipLaunchKernelGGL((k_query_tiles<8, 0>), g, b, lds, st, ix, tp, fp, mp, nt, r, op, s.cand_cap, s.xcd_remap);
        } else {
            if (ix.seg) hipLaunchKernelGGL((k_query_tiles<16, 1>), g, b, lds, st, ix, tp, fp, mp, nt, r, op, s.cand_cap, s.xcd_remap);
            else hipLaunchKernelGGL((k_query_tiles<16, 0>), g, b, lds, st, ix, tp, fp, mp, nt, r, op, s.cand_cap, s.xcd_remap);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hv
