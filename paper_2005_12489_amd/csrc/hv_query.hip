// Per-pixel tile-mask query (binary form of the paper's Algorithm 1).
//
// Display-driven computing makes each pixel a unit of work whose value comes
// from index queries about nearby objects (Sec. 3).  A batch of requests --
// each one tile of one index with its own radius -- runs as two kernels:
//
//  1. k_tile_frontier -- one wavefront per request walks the tree breadth-
//     first with the tile's box grown by r and keeps the deepest level at
//     which at most 256 nodes meet it.  A tile whose frontier is empty misses
//     all data and takes no further work (Sec. 4.1: tiles outside the data's
//     bounds make no task); it goes to a list of tiles whose masks the query
//     kernel zero-fills.  The others are appended to a compacted work list.
//  2. k_query -- a persistent grid (as many workgroups as the GPU holds at
//     once) strides over the (tile, pixel block) items of that list, one
//     wavefront per block (8x8, 16x16 or 32x32: 1, 4 or 16 pixels per lane),
//     the way the paper's engine hands tiles to idle processes (Sec. 4.3).
//     A block starts from its tile's frontier and walks down with the
//     block's box grown by r: the OuterBox filter of Algorithm 1, shared by
//     the block's pixels.  Objects that pass are staged in LDS in tile-local
//     pixel coordinates with the range of block pixels their box grown by r
//     covers.  Small ranges are tested object-parallel (one lane per object,
//     only its own pixels: Algorithm 1's per-pixel box filter seen from the
//     object's side); large ones pixel-parallel (every lane its own pixels).
//     Every test is the exact FP64 distance against r, inclusive.  Once all
//     pixels of the block are lit the wavefront stops, as Algorithm 1 returns
//     as soon as one object lies within the radius.
//
// The tree walk is wavefront-uniform: the stack lives in LDS, each step pops
// up to four nodes of the same level and the 64 lanes test their 4 x 16
// children at once; hits are pushed with one ballot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "hv_internal.h"

namespace hv {
namespace {

constexpr uint32_t kBigFlag = 0x80000000u;  // staged object tested pixel-parallel
constexpr int kSmallArea = 48;              // largest pixel range tested object-parallel
constexpr double kRangeEps = 1e-7;          // px, widens every pixel range
constexpr double kAcceptMargin = 1e-3;      // px: accepts in FP32 use the radius r - kAcceptMargin
constexpr int kCandBytes = 16 + 16 + 8 + 4; // staged object: a, d, 1/|d|^2, range

__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// The frontier level holds at most kFrontier entries, every level below it at
// most 64 (a level is pushed only when none of its entries remain).
__host__ __device__ constexpr int stack_words(int levels) { return 64 * (levels > 0 ? levels : 1) + kFrontier; }

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

__host__ __device__ inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// LDS of one wavefront: stack | staged objects (SoA) | block mask rows.
__host__ __device__ inline size_t wave_lds_bytes(int cap, int levels, int bs) {
    return align16((size_t)stack_words(levels) * 4) + align16((size_t)cap * kCandBytes) + align16((size_t)bs * 4);
}

__device__ inline bool meets(const double4 &nb, double qx0, double qx1, double qy0, double qy1) {
    return nb.x <= qx1 && nb.z >= qx0 && nb.y <= qy1 && nb.w >= qy0;
}

// Regions of side rs (32 or 64) of a tile whose query box -- pixel centres
// grown by m -- a node box meets: bit ry * (256 / rs) + rx.  The region
// kernel makes the same test in normalised coordinates; this one, in tile
// pixels, is widened by 1e-6 px so that it never misses a region that test
// would find (rounding differs by at most ~1e-7 px up to zoom 22).
__device__ inline uint64_t region_bits(const double4 &nb, double S, double ox, double oy, double m, int rs) {
    const double nr = 256.0 / rs, e = 1e-6;
    const double fx0 = fmax(ceil((nb.x * S - ox - (rs - 0.5) - m - e) / rs), 0.0);
    const double fx1 = fmin(floor((nb.z * S - ox - 0.5 + m + e) / rs), nr - 1.0);
    const double fy0 = fmax(ceil((nb.y * S - oy - (rs - 0.5) - m - e) / rs), 0.0);
    const double fy1 = fmin(floor((nb.w * S - oy - 0.5 + m + e) / rs), nr - 1.0);
    if (!(fx0 <= fx1 && fy0 <= fy1)) return 0;
    const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1, n = (int)nr;
    const uint64_t row = ((1ull << (x1 - x0 + 1)) - 1ull) << x0;
    uint64_t bits = 0;
    for (int y = y0; y <= y1; ++y) bits |= row << (y * n);
    return bits;
}

__device__ inline uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        v |= (uint64_t)lo | ((uint64_t)hi << 32);
    }
    return v;
}

// rs: region side of the query kernel that follows (32 or 64), for which the
// frontier records the regions its nodes can reach; 0 marks every part.
// cull (1..kFrontier): the cull depth -- the walk goes one level deeper only
// while that level holds at most cull nodes meeting the tile.
// grow (px) widens the tile's box beyond r on every side: 1/4 for
// anti-aliased output, whose sub-samples lie 1/4 px from the pixel centres.
__global__ __launch_bounds__(256) void k_tile_frontier(DevBatch B, int rs, int cull, double grow) {
    __shared__ uint32_t buf[4][2][kFrontier];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: keeps per-tile values scalar
    if (blockIdx.x == 0 && threadIdx.x == 0) B.hdr->t_start = wall_clock64();
    const int64_t i = (int64_t)blockIdx.x * 4 + wv;
    if (i >= B.hdr->n_req) return;
    const int64_t t = B.order[i];  // requests by zoom, lowest first: the list follows this order
    const DevReq rq = B.reqs[t];
    const DevIndex ix = B.ixs[rq.index];
    const double iS = ldexp(1.0, -8 - rq.z), S = ldexp(256.0, rq.z);
    const double ox = 256.0 * (double)rq.x, oy = 256.0 * (double)rq.y;
    const double m = rq.r + grow + kCullPad;
    const double qx0 = (ox + (0.5 - m)) * iS, qx1 = (ox + (255.5 + m)) * iS;
    const double qy0 = (oy + (0.5 - m)) * iS, qy1 = (oy + (255.5 + m)) * iS;
    uint32_t *cur = buf[wv][0], *nxt = buf[wv][1];
    int ncur = 0, lvl = ix.levels - 1;
    uint64_t cbits = ~0ull;  // regions the current frontier level can reach
    if (ix.levels > 0) {
        const double4 root = ix.nodes[ix.meta[ix.levels - 1]];
        if (meets(root, qx0, qx1, qy0, qy1)) {
            if (lane == 0) cur[0] = 0;
            ncur = 1;
            if (rs) cbits = region_bits(root, S, ox, oy, m, rs);
        }
    }
    __builtin_amdgcn_wave_barrier();
    while (lvl > 0 && ncur > 0) {
        const int cl = lvl - 1;
        const int64_t cnt = ix.meta[kMaxLevels + cl], off = ix.meta[cl];
        int nn = 0;
        uint64_t nbits = 0;
        for (int base = 0; base < ncur * kFan; base += 64) {
            const int k = base + lane;
            bool hit = false;
            int64_t child = 0;
            if (k < ncur * kFan) {
                child = (int64_t)cur[k / kFan] * kFan + (k % kFan);
                if (child < cnt) {
                    const double4 nb = ix.nodes[off + child];
                    hit = meets(nb, qx0, qx1, qy0, qy1);
                    if (hit && rs) nbits |= region_bits(nb, S, ox, oy, m, rs);
                }
            }
            const uint64_t hm = __ballot(hit);
            const int pos = nn + (int)lanes_below(hm);
            if (hit && pos < cull) nxt[pos] = (uint32_t)child;
            nn += __popcll(hm);
            if (nn > cull) break;
        }
        __builtin_amdgcn_wave_barrier();
        if (nn > cull) break;
        uint32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        ncur = nn;
        if (rs) cbits = wave_or64(nbits);
        --lvl;
    }
    if (ncur == 0) {
        // no data within r of the tile: its mask is all zero, written by the
        // query kernel
        if (lane == 0) B.elist[atomicAdd(&B.hdr->ecounter, 1)] = (uint32_t)t;
        return;
    }
    for (int k = lane; k < ncur; k += 64) B.frontier[t * kFrontier + k] = cur[k];
    if (lane == 0) {
        reinterpret_cast<int4 *>(B.fmeta)[t] = make_int4(ncur, lvl, (int)(uint32_t)cbits, (int)(uint32_t)(cbits >> 32));
        B.done[t] = 0;
        B.list[atomicAdd(&B.hdr->counter, 1)] = (uint32_t)t;
    }
}

// Writes the zero masks of the requests whose tile has no data within r
// (listed by the tile-frontier kernel); workgroups take them in turn.
__device__ inline void zero_empty_tiles(const DevBatch &B, uint8_t *out, int tile_bytes = HV_MASK_BYTES) {
    const int ne = B.hdr->ecounter;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const int64_t t = B.elist[e];
        uint4 *m4 = reinterpret_cast<uint4 *>(out + t * (int64_t)tile_bytes);
        for (int k = threadIdx.x; k < tile_bytes / 16; k += blockDim.x) m4[k] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        if (threadIdx.x == 0) B.ts[t] = wall_clock64();
    }
}

// Counts one finished part of request t; the last part stamps its completion.
__device__ inline void part_done(const DevBatch &B, int64_t t, uint32_t parts) {
    if (atomicAdd(&B.done[t], 1u) == parts - 1u) B.ts[t] = wall_clock64();
}

struct WaveLds {
    uint32_t *stk;
    double2 *ca;     // first point of the staged object (tile-local px)
    double2 *cd;     // segment direction
    double *ci;      // 1 / |direction|^2 (0 for a point or a zero-length segment)
    uint32_t *crng;  // block pixel range | kBigFlag
    uint32_t *mrow;  // block rows lit object-parallel
};

// Work items are (position in the compacted tile list, part of the tile).
// Workgroup b runs on XCD b % 8; dealing list positions to XCDs the same way
// keeps all parts of a tile on one XCD, so the partial cache lines its mask
// rows are written in merge in that XCD's L2 before they reach HBM.
struct ItemMap {
    int64_t first, step, n;  // local items first, first + step, ... < n
    int x;                   // XCD slot (-1: no dealing)
    __device__ inline ItemMap(int64_t count, int per_tile) {
        const int64_t g = gridDim.x, b = blockIdx.x;
        // small batches keep every XCD busy instead (a lone tile would
        // otherwise land on one XCD)
        if (g >= 8 && count >= 32) {
            x = (int)(b & 7);
            const int64_t gx = g / 8 + ((b & 7) < (g & 7) ? 1 : 0);
            first = b >> 3;
            step = gx;
            const int64_t tiles_x = count > x ? (count - x + 7) / 8 : 0;
            n = tiles_x * per_tile;
        } else {
            x = -1;
            first = b;
            step = g;
            n = count * per_tile;
        }
    }
    // list position and part of local item u
    __device__ inline int64_t pos(int64_t u, int per_tile) const {
        return x < 0 ? u / per_tile : x + 8 * (u / per_tile);
    }
};

// One pixel block of tile t: traversal, staging, tests, mask write.
template <int BS, int SEG>
__device__ __forceinline__ void block_query(const DevIndex &ix, const DevReq &rq, int64_t t, int b,
                                            const uint32_t *__restrict__ frontier,
                                            const int32_t *__restrict__ fmeta, uint8_t *__restrict__ out,
                                            int cap, const WaveLds &L, int lane) {
    constexpr int NB = 256 / BS;      // blocks per tile row
    constexpr int PPL = BS * BS / 64; // pixels per lane (pixel-parallel layout)
    constexpr int ROWSTEP = 64 / BS;  // rows between a lane's pixels
    constexpr uint32_t FULL = (1u << PPL) - 1u;
    uint32_t *stk = L.stk;
    double2 *ca = L.ca;
    double2 *cd = L.cd;
    double *ci = L.ci;
    uint32_t *crng = L.crng;
    uint32_t *mrow = L.mrow;

    const int bx = b % NB, by = b / NB;
    const double r = rq.r;
    const double S = ldexp(256.0, rq.z);       // world size in pixels
    const double iS = ldexp(1.0, -8 - rq.z);   // 1 / S, exact
    const double ox = 256.0 * (double)rq.x, oy = 256.0 * (double)rq.y;
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
        // the tile's frontier, tested against the block's box in rounds of 64
        const int fcount = fmeta[4 * t], flevel = fmeta[4 * t + 1];
        for (int base = 0; base < fcount; base += 64) {
            bool hit = false;
            uint32_t node = 0;
            if (base + lane < fcount) {
                node = frontier[t * kFrontier + base + lane];
                hit = meets(ix.nodes[ix.meta[flevel] + node], qx0, qx1, qy0, qy1);
            }
            const uint64_t hm = __ballot(hit);
            if (hit) stk[sp + (int)lanes_below(hm)] = ((uint32_t)flevel << kLevelShift) | node;
            sp += __popcll(hm);
        }
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
                    const int ilo = rg & 31, ihi = (rg >> 5) & 31, jlo = (rg >> 10) & 31, jhi = (rg >> 15) & 31;
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
            const int cl = lvl - 1;
            const int64_t child = (int64_t)node * kFan + c;
            const bool hit = nv && child < ix.meta[kMaxLevels + cl] &&
                             meets(ix.nodes[ix.meta[cl] + child], qx0, qx1, qy0, qy1);
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
                        rg = (uint32_t)ilo | ((uint32_t)ihi << 5) | ((uint32_t)jlo << 10) | ((uint32_t)jhi << 15);
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
    uint64_t bal[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) bal[k] = __ballot((lit >> k) & 1u);
    if (lane < BS) {
        // ballot k holds rows k * ROWSTEP .. k * ROWSTEP + ROWSTEP - 1, BS bits each
        const int k = lane / ROWSTEP, q = lane % ROWSTEP;
        uint64_t v = bal[0];
#pragma unroll
        for (int kk = 1; kk < PPL; ++kk) v = k == kk ? bal[kk] : v;
        const uint32_t row = (uint32_t)((v >> (BS * q)) & ((BS == 64 ? 0ull : (1ull << BS)) - 1ull)) | mrow[lane];
        uint8_t *dst = tm + (by * BS + lane) * 32 + bx * (BS / 8);
        if (BS == 8) *dst = (uint8_t)row;
        else if (BS == 16) *reinterpret_cast<uint16_t *>(dst) = (uint16_t)row;
        else *reinterpret_cast<uint32_t *>(dst) = row;
    }
    __builtin_amdgcn_wave_barrier();
}

template <int BS>
__global__ __launch_bounds__(256) void k_query(DevBatch B, int cap, int max_levels) {
    extern __shared__ double4 smem[];
    constexpr int BPT = (256 / BS) * (256 / BS);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: keeps per-block values scalar
    const int wpb = blockDim.x >> 6;
    unsigned char *wbase = reinterpret_cast<unsigned char *>(smem) + wv * wave_lds_bytes(cap, max_levels, BS);
    WaveLds L;
    L.stk = reinterpret_cast<uint32_t *>(wbase);
    unsigned char *cbase = wbase + align16((size_t)stack_words(max_levels) * 4);
    L.ca = reinterpret_cast<double2 *>(cbase);
    L.cd = L.ca + cap;
    L.ci = reinterpret_cast<double *>(L.cd + cap);
    L.crng = reinterpret_cast<uint32_t *>(L.ci + cap);
    L.mrow = reinterpret_cast<uint32_t *>(cbase + align16((size_t)cap * kCandBytes));

    // a workgroup's waves take consecutive blocks of one tile
    const int per_wg = (BPT + wpb - 1) / wpb;
    uint8_t *const out = B.hdr->out;
    zero_empty_tiles(B, out);
    const ItemMap im(B.hdr->counter, per_wg);
    for (int64_t u = im.first; u < im.n; u += im.step) {
        const int b = (int)(u % per_wg) * wpb + wv;
        if (b >= BPT) continue;
        const int64_t t = B.list[im.pos(u, per_wg)];
        const DevReq rq = B.reqs[t];
        const DevIndex ix = B.ixs[rq.index];
        if (ix.seg) block_query<BS, 1>(ix, rq, t, b, B.frontier, B.fmeta, out, cap, L, lane);
        else block_query<BS, 0>(ix, rq, t, b, B.frontier, B.fmeta, out, cap, L, lane);
        if (lane == 0) part_done(B, t, BPT);
    }
}

// ------------------------------------------------------------ region mode
// One workgroup per RS x RS region of a tile.  It walks the tree once with
// the region's box grown by r, all lanes testing children together, and
// queues every object that meets the box in LDS with the range of region
// pixels within r of the object's box (the per-pixel box filter of
// Algorithm 1 seen from the object's side).  The queue is then dealt out as
// work cells -- (object, pixel row, group of 8 columns) -- evenly over all
// lanes, whatever the objects' sizes: each cell tests at most 8 pixels
// with the exact FP64 distance and sets the lit ones with one LDS OR.

// Most children an inner traversal step of a region tests (16 popped nodes).
constexpr int kInnerWidth = 256;

// A traversal step pops nodes of one level -- the lowest on the stack -- and
// pushes at most min(threads * per_lane, kInnerWidth) of their children
// (per_lane children tested by each thread), so every level below the
// frontier holds at most that many entries at a time.
__host__ __device__ inline int region_stack_words(int levels, int threads, int per_lane = 1) {
    const int width = threads * per_lane < kInnerWidth ? threads * per_lane : kInnerWidth;
    return kFrontier + width * (levels > 0 ? levels : 1);
}

// The distance query's walk starts from a frontier at level levels - 1 (the
// root's) at most, so at most levels - 1 levels lie below the frontier.
__host__ __device__ inline int query_stack_words(int levels, int threads, int per_lane) {
    const int width = threads * per_lane < kInnerWidth ? threads * per_lane : kInnerWidth;
    return kFrontier + width * (levels > 1 ? levels - 1 : 0);
}

// stack | queued objects (SoA) | cell prefix sums | mask rows (four sets for
// anti-aliased output, one per sub-sample) | control | scan scratch
__host__ __device__ inline size_t region_lds_bytes(int cap, int levels, int threads, int rs, int opl, int aa = 0) {
    return align16((size_t)query_stack_words(levels, threads, opl) * 4) + align16((size_t)cap * kCandBytes) +
           align16((size_t)(cap + 1) * 4) + align16((size_t)rs * (rs / 32) * 4 * (aa ? 4 : 1)) + 16 + 64;
}

struct RegionLds {
    uint32_t *stk;
    double2 *ca, *cd;
    double *ci;
    uint32_t *crng;  // ilo | ihi << 6 | jlo << 12 | jhi << 18 (region pixels)
    uint32_t *cpre;  // exclusive prefix sums of work cells per queued object
    uint32_t *mask;  // RS rows x RS/32 words (x4 for anti-aliased output: sub-sample m at m * RS * RS/32)
    int *ctl;        // [0] stack size, [1] queued objects
    uint32_t *scan;  // 16 words
};

// Reserves popcount(hm) consecutive slots of *counter for the wave's set lanes.
__device__ inline int wave_alloc(int *counter, uint64_t hm, int lane) {
    int base = 0;
    if (hm) {
        const int first = __ffsll((unsigned long long)hm) - 1;
        if (lane == first) base = atomicAdd(counter, __popcll(hm));
        base = __shfl(base, first, 64);
    }
    return base + (int)lanes_below(hm);
}

// Exclusive scan over the workgroup (blockDim a multiple of 64, at most
// 1024); `scan` holds 16 words of LDS.  Every thread must call it.
__device__ inline uint32_t wg_excl_scan(uint32_t v, uint32_t *total, uint32_t *scan) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scan[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        const uint32_t sk = scan[k];
        if (k < w) off += sk;
        tot += sk;
    }
    *total = tot;
    __syncthreads();
    return off + x - v;
}

// Region pixels whose centre lies within r, per axis, of the box
// [x0, x1] x [y0, y1] (tile-local px), widened by kRangeEps; false if none.
template <int RS>
__device__ inline bool px_range(double x0, double x1, double y0, double y1, double r, double i0, double j0, int &ilo,
                                int &ihi, int &jlo, int &jhi) {
    const double flo_i = fmax(ceil(x0 - r - 0.5 - i0 - kRangeEps), 0.0);
    const double fhi_i = fmin(floor(x1 + r - 0.5 - i0 + kRangeEps), RS - 1.0);
    const double flo_j = fmax(ceil(y0 - r - 0.5 - j0 - kRangeEps), 0.0);
    const double fhi_j = fmin(floor(y1 + r - 0.5 - j0 + kRangeEps), RS - 1.0);
    if (!(flo_i <= fhi_i && flo_j <= fhi_j)) return false;
    ilo = (int)flo_i;
    ihi = (int)fhi_i;
    jlo = (int)flo_j;
    jhi = (int)fhi_j;
    return true;
}

// True when every region pixel of the range is already lit.  Pixels are
// only ever set, so a node or object whose whole range is lit can be
// skipped without changing the mask.
template <int W>
__device__ inline bool range_lit(const uint32_t *mask, int ilo, int ihi, int jlo, int jhi) {
    for (int jj = jlo; jj <= jhi; ++jj)
        for (int w = ilo >> 5; w <= (ihi >> 5); ++w) {
            const int c0 = max(ilo, 32 * w) - 32 * w, c1 = min(ihi, 32 * w + 31) - 32 * w;
            const uint32_t want = (c1 == 31 ? 0xffffffffu : ((1u << (c1 + 1)) - 1u)) & ~((1u << c0) - 1u);
            if ((mask[jj * W + w] & want) != want) return false;
        }
    return true;
}

__device__ inline int region_cells(uint32_t rg) {
    const int ilo = rg & 63, ihi = (rg >> 6) & 63, jlo = (rg >> 12) & 63, jhi = (rg >> 18) & 63;
    return (jhi - jlo + 1) * ((ihi >> 3) - (ilo >> 3) + 1);
}

// AA = 0: one bit per pixel, [D(centre) <= r].  AA = 1: Algorithm 1's value
// 0-4, the number of the pixel's four sub-samples (centre +- 1/4 px in x and
// y) within r, each against its own nearest object; the region keeps one
// mask per sub-sample, culls with the samples' reach r + 1/4 px per axis,
// makes its edge accepts on each sub-sample grid and tests the four
// sub-samples of every pixel it drains.
template <int RS, int SEG, int OPL, int AA>
__device__ __forceinline__ void region_query(const DevIndex &ix, const DevReq &rq, int64_t t, int reg,
                                             const uint32_t *__restrict__ frontier,
                                             const int32_t *__restrict__ fmeta, uint8_t *__restrict__ out,
                                             int cap, const RegionLds &L) {
    constexpr int NR = 256 / RS;
    constexpr int W = RS / 32;   // mask words per region row
    constexpr int MW = RS * W;   // words of one mask
    constexpr int NM = AA ? 4 : 1;
    const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
    uint32_t *stk = L.stk;
    uint32_t *mask = L.mask;
    int *ctl = L.ctl;

    const int rx = reg % NR, ry = reg / NR;
    const double r = rq.r, r2 = r * r;
    const double rreach = AA ? r + 0.25 : r;  // per axis, how far from a pixel centre an object can matter
    // anti-aliased output: centre-distance bounds (Algorithm 1's R1 and R2,
    // r -+ sqrt(2)/4, each moved 1e-7 px inwards); rin2 < 0 when R1 <= 0
    const double rin = r - 0.35355339059327373 - 1e-7, rout = r + 0.35355339059327373 + 1e-7;
    const double rin2 = rin > 0.0 ? rin * rin : -1.0, rout2 = rout * rout;
    const bool centre_first = AA && r >= 1.0;
    const double S = ldexp(256.0, rq.z);
    const double iS = ldexp(1.0, -8 - rq.z);
    const double ox = 256.0 * (double)rq.x, oy = 256.0 * (double)rq.y;
    const double i0 = (double)(rx * RS), j0 = (double)(ry * RS);
    const double m = rreach + kCullPad;
    const double qx0 = ((ox + i0) + (0.5 - m)) * iS;
    const double qx1 = ((ox + i0) + ((RS - 0.5) + m)) * iS;
    const double qy0 = ((oy + j0) + (0.5 - m)) * iS;
    const double qy1 = ((oy + j0) + ((RS - 0.5) + m)) * iS;
    uint8_t *tm = out + t * (int64_t)(AA ? HV_AA_BYTES : HV_MASK_BYTES);

    const int4 fm = reinterpret_cast<const int4 *>(fmeta)[t];
    const int fcount = fm.x, flevel = fm.y;
    const uint64_t reach = (uint64_t)(uint32_t)fm.z | ((uint64_t)(uint32_t)fm.w << 32);
    if (!((reach >> reg) & 1ull)) {
        // no frontier node comes within r of this region: all zero
        if (AA) {
            for (int k = tid; k < RS * RS / 4; k += nthr)
                *reinterpret_cast<uint32_t *>(tm + (ry * RS + k / (RS / 4)) * 256 + rx * RS + 4 * (k % (RS / 4))) = 0u;
        } else {
            for (int k = tid; k < RS * W; k += nthr)
                *reinterpret_cast<uint32_t *>(tm + (ry * RS + k / W) * 32 + rx * (RS / 8) + 4 * (k % W)) = 0u;
        }
        return;
    }

    for (int k = tid; k < NM * MW; k += nthr) mask[k] = 0;
    // a range is done once every pixel in it is set in every mask
    auto range_done = [&](int ilo, int ihi, int jlo, int jhi) -> bool {
        bool d = range_lit<W>(mask, ilo, ihi, jlo, jhi);
#pragma unroll
        for (int mm = 1; mm < NM; ++mm) d = d && range_lit<W>(mask + mm * MW, ilo, ihi, jlo, jhi);
        return d;
    };
    if (tid == 0) {
        ctl[0] = 0;
        ctl[1] = 0;
    }
    __syncthreads();
    // accepts keep a margin so that they never claim a sample whose distance
    // could round to just above r
    const double racc = r - 1e-7, racc2 = racc * racc;
    // Pushes the frontier nodes that meet the region; true when one of them
    // is worth an accept pass: its leaves, at about 4^-level of its size,
    // could be small enough to light pixels by themselves.
    auto push_frontier = [&]() -> bool {
        bool promising = false;
        for (int base = 0; base < fcount; base += nthr) {
            bool hit = false;
            uint32_t node = 0;
            if (base + tid < fcount) {
                node = frontier[t * kFrontier + base + tid];
                const double4 nb = ix.nodes[ix.meta[flevel] + node];
                hit = meets(nb, qx0, qx1, qy0, qy1);
                const double w = (nb.z - nb.x) * S, h = (nb.w - nb.y) * S;
                promising |= hit && w * w + h * h <= ldexp(16.0 * racc2, 4 * flevel);
            }
            const int pos = wave_alloc(&ctl[0], __ballot(hit), lane);
            if (hit) stk[pos] = ((uint32_t)flevel << kLevelShift) | node;
        }
        return __syncthreads_or(promising);
    };
    const bool promising = push_frontier();

    // Tests every queued object against its pixels; returns true once the
    // whole region is lit.
    auto drain = [&]() -> bool {
        const int nq = ctl[1];
        const int per = (nq + nthr - 1) / nthr;
        const int q0 = min(nq, tid * per), q1 = min(nq, q0 + per);
        uint32_t cnt = 0;
        for (int q = q0; q < q1; ++q) cnt += (uint32_t)region_cells(L.crng[q]);
        uint32_t tot;
        uint32_t off = wg_excl_scan(cnt, &tot, L.scan);
        for (int q = q0; q < q1; ++q) {
            L.cpre[q] = off;
            off += (uint32_t)region_cells(L.crng[q]);
        }
        __syncthreads();
        for (uint32_t cell = tid; cell < tot; cell += nthr) {
            int lo = 0, hi = nq - 1;  // last object whose first cell is <= cell
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.cpre[mid] <= cell) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t rg = L.crng[lo];
            const int ilo = rg & 63, ihi = (rg >> 6) & 63, jlo = (rg >> 12) & 63;
            const int g0 = ilo >> 3, ng = (ihi >> 3) - g0 + 1;
            const int local = (int)(cell - L.cpre[lo]);
            // local / ng by reciprocal: exact here (local < 2^10, ng <= 9)
            const int dq = (int)(((float)local + 0.5f) * __builtin_amdgcn_rcpf((float)ng));
            const int row = jlo + dq, g = g0 + (local - dq * ng);
            if (row >= RS || g < g0 || g >= g0 + ng) continue;  // never taken: the quotient is exact
            const int c0 = max(ilo, 8 * g), c1 = min(ihi, 8 * g + 7);
            const double2 a = L.ca[lo];
            double2 d = make_double2(0.0, 0.0);
            double inv = 0.0;
            if (SEG) {
                d = L.cd[lo];
                inv = L.ci[lo];
            }
            // exact FP64 squared distance from a sample (tile-local px) to the object
            auto dist2 = [&](double px, double py) -> double {
                const double wx = px - a.x, wy = py - a.y;
                if (SEG) {
                    double tt = (wx * d.x + wy * d.y) * inv;
                    tt = fmin(fmax(tt, 0.0), 1.0);
                    const double ex = wx - tt * d.x, ey = wy - tt * d.y;
                    return ex * ex + ey * ey;
                }
                return wx * wx + wy * wy;
            };
            const double cy = j0 + (double)row + 0.5;
            // only the cell's pixels not done yet (bits are only ever set)
            const int wbase = c0 & ~31, widx = row * W + (wbase >> 5);
            uint32_t done = mask[widx];
#pragma unroll
            for (int mm = 1; mm < NM; ++mm) done &= mask[mm * MW + widx];
            uint32_t todo = (((2u << (c1 - c0)) - 1u) << (c0 - wbase)) & ~done;
            uint32_t bits[NM];
#pragma unroll
            for (int mm = 0; mm < NM; ++mm) bits[mm] = 0;
            while (todo) {
                const int ii = wbase + __builtin_ctz(todo);
                const uint32_t bit = 1u << (ii & 31);
                todo &= todo - 1u;
                const double cx = i0 + (double)ii + 0.5;
                if (AA) {
                    // From r >= 1 on, Algorithm 1's thresholds on the centre's
                    // distance first: a sub-sample lies sqrt(2)/4 px from it,
                    // so within rin of the object every sub-sample is within r,
                    // beyond rout none is (both kept 1e-7 px inside the exact
                    // bounds).  Otherwise (and for smaller r, where the band
                    // between them holds nearly every pixel in reach)
                    // sub-sample mm at (cx -+ 1/4, cy -+ 1/4) is tested itself
                    // (bit 0 of mm picks +x, bit 1 picks +y).
                    auto each = [&]() {
#pragma unroll
                        for (int mm = 0; mm < NM; ++mm)
                            if (dist2(cx + ((mm & 1) ? 0.25 : -0.25), cy + ((mm & 2) ? 0.25 : -0.25)) <= r2)
                                bits[mm] |= bit;
                    };
                    if (centre_first) {
                        const double dc2 = dist2(cx, cy);
                        if (dc2 <= rin2) {
#pragma unroll
                            for (int mm = 0; mm < NM; ++mm) bits[mm] |= bit;
                        } else if (dc2 <= rout2) {
                            each();
                        }
                    } else {
                        each();
                    }
                } else if (dist2(cx, cy) <= r2) {
                    bits[0] |= bit;
                }
            }
#pragma unroll
            for (int mm = 0; mm < NM; ++mm)
                if (bits[mm]) atomicOr(&mask[mm * MW + widx], bits[mm]);
        }
        __syncthreads();
        bool full = true;
        for (int k = tid; k < NM * MW; k += nthr) full &= mask[k] == 0xffffffffu;
        const bool all = __syncthreads_and(full);
        if (tid == 0) ctl[1] = 0;
        __syncthreads();
        return all;
    };

    // Two walks.  The first (accept pass) descends only until nodes are small
    // enough for their edge accepts to cover the pixels around them, makes
    // those accepts and reads no objects; it skips subtrees whose leaves are
    // unlikely to be that small.  In dense data it lights most pixels, so
    // that the second, full walk finds most ranges lit and reads few objects.
    // A frontier made of leaves, or of nodes whose leaves cannot be small,
    // takes the full walk only.
    bool accept_pass = racc > 0.0 && flevel > 0 && promising;
    bool done = false;
    for (;;) {
        const int sp = ctl[0];
        if (sp == 0) {
            if (!accept_pass) break;
            accept_pass = false;
            // every wave has read the empty stack before any pushes to it
            __syncthreads();
            (void)push_frontier();
            continue;
        }
        bool accepted = false;
        const int lvl = (int)(stk[sp - 1] >> kLevelShift);
        // a step tests OPL objects per thread at a leaf level, and up to OPL
        // children per thread, kInnerWidth in all, at an inner one: 16 per
        // popped node either way
        const int per_step = (lvl > 0 ? min(nthr * OPL, kInnerWidth) : nthr * OPL) / kFan;
        const bool top = tid < per_step && tid < sp && (int)(stk[sp - 1 - tid] >> kLevelShift) == lvl;
        const int npop = __syncthreads_count(top);
        if (lvl > 0) {
            const int cl = lvl - 1;
            const int64_t ccount = ix.meta[kMaxLevels + cl], coff = ix.meta[cl];
            // issue all OPL child-box loads first so that they are in flight
            // together, in the accept pass each with the child's
            // representative (the first vertex of its first object), stored
            // beside the boxes so that a node's children read it contiguously
            double4 nbk[OPL];
            double2 repk[OPL];
            uint32_t childk[OPL];
            bool havek[OPL];
#pragma unroll
            for (int k = 0; k < OPL; ++k) {
                const int q = k * nthr + tid, j = q >> 4, c = q & 15;  // popped node, child of it
                havek[k] = false;
                childk[k] = 0;
                nbk[k] = make_double4(0.0, 0.0, 0.0, 0.0);
                repk[k] = make_double2(0.0, 0.0);
                if (j < npop) {
                    const int64_t child = (int64_t)(stk[sp - 1 - j] & kIdxMask) * kFan + c;
                    if (child < ccount) {
                        havek[k] = true;
                        childk[k] = (uint32_t)child;
                        nbk[k] = ix.nodes[coff + child];
                        if (accept_pass) repk[k] = ix.rep[coff + child];
                    }
                }
            }
            if (tid == 0) ctl[0] = sp - npop;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < OPL; ++k) {
                const double4 nb = nbk[k];
                bool push = false;
                if (havek[k] && meets(nb, qx0, qx1, qy0, qy1)) {
                    const double bx0 = nb.x * S - ox, bx1 = nb.z * S - ox;
                    const double by0 = nb.y * S - oy, by1 = nb.w * S - oy;
                    int ilo, ihi, jlo, jhi;
                    push = px_range<RS>(bx0, bx1, by0, by1, rreach, i0, j0, ilo, ihi, jlo, jhi);
                    const double bw = bx1 - bx0, bh = by1 - by0;
                    const double diag2 = bw * bw + bh * bh;
                    const bool small = racc > 0.0 && bw <= 2.0 * racc && bh <= 2.0 * racc;
                    // a child whose pixel range is all lit can add nothing:
                    // neither accepts nor objects
                    if (push && range_done(ilo, ihi, jlo, jhi)) push = false;
                    // Accepts light sample rows in FP32 with the radius ra = r -
                    // 1e-3 px.  Tile-local coordinates stay below a few hundred px,
                    // where one FP32 rounding is at most 3e-5 px, so the squared
                    // distance a claimed sample is known to have is off by less
                    // than 2 r 1e-4 + r^2 3e-7 px^2 (runs are shrunk by 1e-4 px for
                    // their own rounding): under a tenth of the room r^2 - ra^2 =
                    // 2 r 1e-3 - 1e-6 for every r in (1e-3, 64].  No accept claims a
                    // sample beyond r; samples near an accept's edge fall to the
                    // exact FP64 test.  For anti-aliased output every accept runs
                    // on the four sub-sample grids (centres shifted by -+1/4 px in
                    // x and y) and lights that sub-sample's mask.
                    const float ra = (float)(r - kAcceptMargin);
                    const float ra2 = ra * ra;
                    // with one mask word per row: the child's columns as row
                    // bits, so that rows already lit there (in both masks a
                    // sample row serves, for anti-aliased output) are skipped
                    const uint32_t rowwant = (uint32_t)(((2ull << (ihi - ilo)) - 1ull) << ilo);
                    // the columns of [ilo, ihi] whose sample x (column 0's sample
                    // at fc0) lies in [lo, hi], as row bits
                    auto run = [&](float fc0, float lo, float hi) -> uint64_t {
                        const int a0 = max((int)ceilf(lo - fc0 + 1e-4f), ilo);
                        const int a1 = min((int)floorf(hi - fc0 - 1e-4f), ihi);
                        if (a0 > a1) return 0ull;
                        return (a1 - a0 == 63 ? ~0ull : ((1ull << (a1 - a0 + 1)) - 1ull)) << a0;
                    };
                    // sets row bits in mask mm's row jj (one LDS atomic per word)
                    auto light = [&](int mm, int jj, uint64_t bits) {
#pragma unroll
                        for (int wd = 0; wd < W; ++wd) {
                            const uint32_t wb = (uint32_t)(bits >> (32 * wd));
                            if (wb) {
                                atomicOr(&mask[mm * MW + jj * W + wd], wb);
                                accepted = true;
                            }
                        }
                    };
                    if (push && ra > 0.0f && accept_pass) {
                        // Disk accept (accept pass): the child's representative is a
                        // vertex of an object of the index, so every sample within ra
                        // of it is lit.  Any node, however large, lights a disk this
                        // way, so that coarse levels already prune the nodes below.
                        const double pu = repk[k].x * S - ox, pv = repk[k].y * S - oy;
                        const float fpu = (float)pu, fpv = (float)pv;
                        const int r0 = max(jlo, (int)ceil(pv - (double)ra - 0.75 - j0));
                        const int r1 = min(jhi, (int)floor(pv + (double)ra - 0.25 - j0));
#pragma unroll
                        for (int sy = 0; sy < (AA ? 2 : 1); ++sy) {
                            const float syo = AA ? (sy ? 0.25f : -0.25f) : 0.0f;
                            for (int jj = r0; jj <= r1; ++jj) {
                                if (W == 1 && (mask[(AA ? 2 * sy : 0) * MW + jj] & rowwant) == rowwant &&
                                    (!AA || (mask[(2 * sy + 1) * MW + jj] & rowwant) == rowwant))
                                    continue;
                                const float dy = (float)(j0 + (double)jj + 0.5) + syo - fpv;
                                const float rn = ra2 - dy * dy;
                                if (rn < 0.0f) continue;
                                const float h = __builtin_amdgcn_sqrtf(rn);
#pragma unroll
                                for (int sx = 0; sx < (AA ? 2 : 1); ++sx)
                                    light(AA ? 2 * sy + sx : 0, jj,
                                          run((float)(i0 + 0.5) + (AA ? (sx ? 0.25f : -0.25f) : 0.0f), fpu - h, fpu + h));
                            }
                        }
                    }
                    if (push && small) {
                        // Edge accept.  A node box is the exact bounding box of
                        // its objects' coordinates (points, segment endpoints),
                        // so each of its four sides holds a point of some object.
                        // A pixel centre within ra of both ends of one side is
                        // within ra of that point, hence lit, without looking
                        // at the objects.  Per pixel row at height cy, with dyn
                        // and dyf the distances to the nearer and farther
                        // horizontal side, that holds for the centres cx with
                        //   |cx - bx0| <= a or |cx - bx1| <= a,  a = sqrt(ra^2 - dyf^2)
                        //     (both ends of the vertical side at bx0 or bx1), or
                        //   bx1 - b <= cx <= bx0 + b,            b = sqrt(ra^2 - dyn^2)
                        //     (both ends of the nearer horizontal side),
                        // so the row's accepted pixels are at most three runs.
                        const float fx0 = (float)bx0, fx1 = (float)bx1, fy0 = (float)by0, fy1 = (float)by1;
                        // rows of samples: one per pixel row, or two (-+1/4) for
                        // anti-aliased output, each serving its two sub-sample
                        // columns (-+1/4), which share the row's runs
#pragma unroll
                        for (int sy = 0; sy < (AA ? 2 : 1); ++sy) {
                            const float syo = AA ? (sy ? 0.25f : -0.25f) : 0.0f;
                            for (int jj = jlo; jj <= jhi && ra > 0.0f; ++jj) {
                                if (W == 1 && (mask[(AA ? 2 * sy : 0) * MW + jj] & rowwant) == rowwant &&
                                    (!AA || (mask[(2 * sy + 1) * MW + jj] & rowwant) == rowwant))
                                    continue;
                                const float cy = (float)(j0 + (double)jj + 0.5) + syo;  // exact
                                const float ey0 = fabsf(cy - fy0), ey1 = fabsf(cy - fy1);
                                const float dyn = fminf(ey0, ey1), dyf = fmaxf(ey0, ey1);
                                const float rn = ra2 - dyn * dyn;
                                if (rn < 0.0f) continue;
                                const float b = __builtin_amdgcn_sqrtf(rn);
                                const float rf = ra2 - dyf * dyf;
                                const float a = rf >= 0.0f ? __builtin_amdgcn_sqrtf(rf) : -1.0f;
#pragma unroll
                                for (int sx = 0; sx < (AA ? 2 : 1); ++sx) {
                                    // sample of region column 0 (exact)
                                    const float fc0 = (float)(i0 + 0.5) + (AA ? (sx ? 0.25f : -0.25f) : 0.0f);
                                    uint64_t bits = run(fc0, fx1 - b, fx0 + b);
                                    if (a >= 0.0f) bits |= run(fc0, fx0 - a, fx0 + a) | run(fc0, fx1 - a, fx1 + a);
                                    light(AA ? 2 * sy + sx : 0, jj, bits);
                                }
                            }
                        }
                        // (a child the accept pass stops at needs no second look)
                        if (!(accept_pass && (diag2 <= 2.25 * racc2 || cl == 0)) && range_done(ilo, ihi, jlo, jhi))
                            push = false;
                    }
                    // The accept pass stops at leaves and at nodes whose diagonal
                    // is at most 1.5 racc.  A box's edge accepts light every pixel
                    // centre inside it once its diagonal is at most 2 racc (the
                    // centre of the box is the farthest from the ends of its
                    // edges, at half the diagonal), so such nodes, spread over an
                    // area, light all of it; stopping well below 2 racc keeps the
                    // accepts of their children for the ring of pixels around
                    // them, which would otherwise fall to the full walk.  It
                    // enters a larger node only if its leaves, at about
                    // 4^-level of its size, could be small.
                    if (accept_pass && push && (diag2 <= 2.25 * racc2 || cl == 0 || diag2 > ldexp(16.0 * racc2, 4 * cl)))
                        push = false;
                }
                const int pos = wave_alloc(&ctl[0], __ballot(push), lane);
                if (push) stk[pos] = ((uint32_t)cl << kLevelShift) | childk[k];
            }
        } else {
            // issue all OPL loads first so that they are in flight together
            double4 ob[OPL];
            bool have[OPL];
#pragma unroll
            for (int k = 0; k < OPL; ++k) {
                const int q = k * nthr + tid, j = q >> 4, c = q & 15;
                have[k] = false;
                ob[k] = make_double4(0.0, 0.0, 0.0, 0.0);
                if (j < npop) {
                    const int64_t o = (int64_t)(stk[sp - 1 - j] & kIdxMask) * kLeaf + c;
                    if (o < ix.n) {
                        have[k] = true;
                        if (SEG) {
                            ob[k] = reinterpret_cast<const double4 *>(ix.obj)[o];
                        } else {
                            const double2 p = reinterpret_cast<const double2 *>(ix.obj)[o];
                            ob[k] = make_double4(p.x, p.y, p.x, p.y);
                        }
                    }
                }
            }
            if (tid == 0) ctl[0] = sp - npop;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < OPL; ++k) {
                // a queue smaller than a step's OPL * threads objects takes
                // them threads at a time, draining in between
                if (k > 0 && cap < nthr * OPL) {
                    __syncthreads();
                    if (ctl[1] > cap - nthr && drain()) {
                        done = true;
                        break;
                    }
                }
                const double ax = ob[k].x, ay = ob[k].y, bxx = ob[k].z, byy = ob[k].w;
                bool keep = false;
                double ua = 0, va = 0, ub = 0, vb = 0;
                uint32_t rg = 0;
                if (have[k] && fmin(ax, bxx) <= qx1 && fmax(ax, bxx) >= qx0 && fmin(ay, byy) <= qy1 &&
                    fmax(ay, byy) >= qy0) {
                    // tile-local pixel frame; scaling by S is exact
                    ua = ax * S - ox; va = ay * S - oy;
                    ub = bxx * S - ox; vb = byy * S - oy;
                    // region pixels that have a sample within r of the object's box
                    const double flo_i = fmax(ceil(fmin(ua, ub) - rreach - 0.5 - i0 - kRangeEps), 0.0);
                    const double fhi_i = fmin(floor(fmax(ua, ub) + rreach - 0.5 - i0 + kRangeEps), RS - 1.0);
                    const double flo_j = fmax(ceil(fmin(va, vb) - rreach - 0.5 - j0 - kRangeEps), 0.0);
                    const double fhi_j = fmin(floor(fmax(va, vb) + rreach - 0.5 - j0 + kRangeEps), RS - 1.0);
                    if (flo_i <= fhi_i && flo_j <= fhi_j &&
                        !range_done((int)flo_i, (int)fhi_i, (int)flo_j, (int)fhi_j)) {
                        keep = true;
                        rg = (uint32_t)flo_i | ((uint32_t)fhi_i << 6) | ((uint32_t)flo_j << 12) |
                             ((uint32_t)fhi_j << 18);
                    }
                }
                const int slot = wave_alloc(&ctl[1], __ballot(keep), lane);
                if (keep) {
                    L.ca[slot] = make_double2(ua, va);
                    if (SEG) {
                        const double dx = ub - ua, dy = vb - va;
                        const double l2 = dx * dx + dy * dy;
                        L.cd[slot] = make_double2(dx, dy);
                        // 1 / l2: the hardware reciprocal and two Newton steps
                        // (each doubles its correct bits), within an ulp or so
                        // of the quotient at a fraction of a division's cost
                        double iv = __builtin_amdgcn_rcp(l2);
                        iv = fma(iv, fma(-l2, iv, 1.0), iv);
                        iv = fma(iv, fma(-l2, iv, 1.0), iv);
                        L.ci[slot] = l2 > 0.0 ? iv : 0.0;
                    }
                    L.crng[slot] = rg;
                }
            }
        }
        if (done) break;
        if (__syncthreads_or(accepted)) {
            // accepts may have lit the whole region
            bool full = true;
            for (int k = tid; k < NM * MW; k += nthr) full &= mask[k] == 0xffffffffu;
            if (__syncthreads_and(full)) {
                done = true;
                break;
            }
        }
        // room for what the next leaf step queues at once
        if (ctl[1] > cap - (cap >= nthr * OPL ? nthr * OPL : nthr) && drain()) {
            done = true;
            break;
        }
    }
    if (!done && ctl[1] > 0) drain();
    __syncthreads();
    if (AA) {
        // one byte per pixel: the number of its sub-samples within r; a
        // thread writes four neighbouring pixels
        for (int k = tid; k < RS * RS / 4; k += nthr) {
            const int row = k / (RS / 4), col = 4 * (k % (RS / 4)), widx = row * W + (col >> 5);
            uint32_t v = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t c = 0;
#pragma unroll
                for (int mm = 0; mm < NM; ++mm) c += (mask[mm * MW + widx] >> ((col + q) & 31)) & 1u;
                v |= c << (8 * q);
            }
            *reinterpret_cast<uint32_t *>(tm + (ry * RS + row) * 256 + rx * RS + col) = v;
        }
    } else {
        for (int k = tid; k < RS * W; k += nthr) {
            const int row = k / W, wd = k % W;
            *reinterpret_cast<uint32_t *>(tm + (ry * RS + row) * 32 + rx * (RS / 8) + 4 * wd) = mask[k];
        }
    }
    __syncthreads();
}

template <int RS, int OPL, int AA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_query_region(DevBatch B, int cap, int max_levels) {
    extern __shared__ double4 smem[];
    constexpr int RPT = (256 / RS) * (256 / RS);
    unsigned char *base = reinterpret_cast<unsigned char *>(smem);
    RegionLds L;
    L.stk = reinterpret_cast<uint32_t *>(base);
    unsigned char *cb = base + align16((size_t)query_stack_words(max_levels, blockDim.x, OPL) * 4);
    L.ca = reinterpret_cast<double2 *>(cb);
    L.cd = L.ca + cap;
    L.ci = reinterpret_cast<double *>(L.cd + cap);
    L.crng = reinterpret_cast<uint32_t *>(L.ci + cap);
    L.cpre = reinterpret_cast<uint32_t *>(cb + align16((size_t)cap * kCandBytes));
    L.mask = reinterpret_cast<uint32_t *>(reinterpret_cast<unsigned char *>(L.cpre) + align16((size_t)(cap + 1) * 4));
    L.ctl = reinterpret_cast<int *>(L.mask + RS * (RS / 32) * (AA ? 4 : 1));
    L.scan = reinterpret_cast<uint32_t *>(L.ctl + 4);
    uint8_t *const out = B.hdr->out;
    zero_empty_tiles(B, out, AA ? HV_AA_BYTES : HV_MASK_BYTES);
    const ItemMap im(B.hdr->counter, RPT);
    for (int64_t u = im.first; u < im.n; u += im.step) {
        const int64_t t = B.list[im.pos(u, RPT)];
        const int reg = (int)(u % RPT);
        const DevReq rq = B.reqs[t];
        const DevIndex ix = B.ixs[rq.index];
        if (ix.seg) region_query<RS, 1, OPL, AA>(ix, rq, t, reg, B.frontier, B.fmeta, out, cap, L);
        else region_query<RS, 0, OPL, AA>(ix, rq, t, reg, B.frontier, B.fmeta, out, cap, L);
        if (threadIdx.x == 0) part_done(B, t, RPT);
    }
}

// ------------------------------------------------------------ polygon filling
// SIBF (Algorithm 2) per region of RS x RS pixels.  The index's tree holds
// the polygons' bounding boxes; the walk collects the polygons whose box
// meets the region's pixel centres (Algorithm 2's RtreeMBR query).  For
// each, every edge toggles, in every region row whose centre line it
// crosses (half-open in y: an edge is crossed when exactly one endpoint lies
// below the line, so a vertex on it counts once and edges parallel to x
// never, which is what IsLevel and segment cutting achieve in the paper),
// the pixels whose centre lies right of the crossing.  After all its edges a
// pixel's bit is the parity of the crossings left of it: inside that polygon
// (even-odd rule, holes included).  The fill is the OR over polygons.
// Casting the ray towards -x instead of towards the nearer side of the box
// gives the same parity for closed rings.
// Queued polygons are tested in groups of up to kFillGroup: the edge chunks
// of the whole group are dealt out over all lanes, each polygon toggling its
// own parity rows, and the rows are ORed into the fill after the group.  A
// chunk's conservative box decides whether any of its edges can cross a row
// centre line of the region left of its last pixel centre; only then are its
// edges read.  A polygon (or a subtree) whose pixel centres in the region are
// all filled already cannot change the OR and is skipped.
constexpr int kFillGroup = 32;
constexpr int64_t kFillGrid = 262144;  // default workgroups of a filling launch (at most one per region)

struct FillLds {
    uint32_t *stk;
    uint32_t *cand;   // candidate polygons
    uint32_t *crng;   // their pixel-centre ranges in the region: ilo | ihi << 6 | jlo << 12 | jhi << 18
    uint32_t *mask;   // RS rows x RS/32 words: filled so far
    uint32_t *par;    // kFillGroup x RS rows x RS/32 words: parity rows of the group (zero between groups)
    int64_t *efirst;  // edge range [efirst, eend) of each polygon of the group
    int64_t *eend;
    int64_t *cpre;    // kFillGroup + 1 prefix sums of the group's chunk counts
    int64_t *lc;      // one per thread: chunks that passed their box test this round
    uint8_t *lq;      // and the group polygon each belongs to
    uint8_t *ldir;    // kFillGroup: bit w set when the group polygon's rays in mask word column w run towards +x
    int64_t *spre;    // kFillGroup + 1 prefix sums of the group's super-chunk counts
    int64_t *ls;      // one per thread: super-chunks that passed their box test this round
    uint8_t *lsq;     // and the group polygon each belongs to
    int *ctl;         // [0] stack size, [1] candidates, [2], [3] passed chunks (alternate rounds), [4] passed supers
};

// A group whose polygons hold at most this many chunk boxes per thread tests
// them all; beyond, it tests the super-chunk boxes first.
constexpr int kFlatChunkRounds = 4;

__host__ __device__ inline size_t fill_lds_bytes(int cap, int levels, int threads, int rs) {
    const size_t rows = (size_t)rs * (rs / 32) * 4;
    return align16((size_t)region_stack_words(levels, threads) * 4) + 2 * align16((size_t)cap * 4) + align16(rows) +
           align16(kFillGroup * rows) + 2 * align16(kFillGroup * 8) + align16((kFillGroup + 1) * 8) +
           align16((size_t)threads * 8) + align16((size_t)threads) + align16(kFillGroup) +
           align16((kFillGroup + 1) * 8) + align16((size_t)threads * 8) + align16((size_t)threads) + 32;
}

template <int RS>
__device__ __forceinline__ void fill_query(const DevIndex &ix, const DevReq &rq, int64_t t, int reg,
                                           const uint32_t *__restrict__ frontier, const int32_t *__restrict__ fmeta,
                                           uint8_t *__restrict__ out, int cap, const FillLds &L) {
    constexpr int NR = 256 / RS;
    constexpr int W = RS / 32;
    const int tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
    uint32_t *stk = L.stk, *mask = L.mask, *par = L.par;
    int *ctl = L.ctl;
    const int rx = reg % NR, ry = reg / NR;
    const double S = ldexp(256.0, rq.z), iS = ldexp(1.0, -8 - rq.z);
    const double ox = 256.0 * (double)rq.x, oy = 256.0 * (double)rq.y;
    const double i0 = (double)(rx * RS), j0 = (double)(ry * RS);
    const double m = kCullPad;
    const double qx0 = ((ox + i0) + (0.5 - m)) * iS, qx1 = ((ox + i0) + ((RS - 0.5) + m)) * iS;
    const double qy0 = ((oy + j0) + (0.5 - m)) * iS, qy1 = ((oy + j0) + ((RS - 0.5) + m)) * iS;
    uint8_t *tm = out + t * (int64_t)HV_MASK_BYTES;

    const int4 fm = reinterpret_cast<const int4 *>(fmeta)[t];
    const int fcount = fm.x, flevel = fm.y;
    const uint64_t reach = (uint64_t)(uint32_t)fm.z | ((uint64_t)(uint32_t)fm.w << 32);
    if (!((reach >> reg) & 1ull)) {
        for (int k = tid; k < RS * W; k += nthr)
            *reinterpret_cast<uint32_t *>(tm + (ry * RS + k / W) * 32 + rx * (RS / 8) + 4 * (k % W)) = 0u;
        return;
    }
    for (int k = tid; k < RS * W; k += nthr) mask[k] = 0;
    if (tid == 0) {
        ctl[0] = 0;
        ctl[1] = 0;
        ctl[2] = 0;
        ctl[3] = 0;
        ctl[4] = 0;
    }
    __syncthreads();
    for (int base = 0; base < fcount; base += nthr) {
        bool hit = false;
        uint32_t node = 0;
        if (base + tid < fcount) {
            node = frontier[t * kFrontier + base + tid];
            hit = meets(ix.nodes[ix.meta[flevel] + node], qx0, qx1, qy0, qy1);
        }
        const int pos = wave_alloc(&ctl[0], __ballot(hit), lane);
        if (hit) stk[pos] = ((uint32_t)flevel << kLevelShift) | node;
    }
    __syncthreads();

    // Tests the queued polygons, a group at a time; true once the region is
    // all filled.
    auto test = [&]() -> bool {
        const int nc = ctl[1];
        for (int c0 = 0; c0 < nc; c0 += kFillGroup) {
            const int nb = min(kFillGroup, nc - c0);
            if (tid < 64) {  // edge ranges of the group and the prefix sums of their chunk counts
                int64_t f = 0, fe = 0;
                long long x = 0, xs = 0;
                uint8_t dir = 0;
                // a polygon whose pixel centres in the region are all filled
                // already cannot change the fill: it gets no chunks
                const uint32_t rg = lane < nb ? L.crng[c0 + lane] : 0u;
                if (lane < nb && !range_lit<W>(mask, rg & 63, (rg >> 6) & 63, (rg >> 12) & 63, (rg >> 18) & 63)) {
                    const int64_t pid = L.cand[c0 + lane];
                    f = ix.pfirst[pid];
                    fe = ix.pfirst[pid + 1];
                    x = fe > f ? (fe - 1) / kEdgeChunk - f / kEdgeChunk + 1 : 0;
                    constexpr int kSuperEdges = kEdgeChunk * kChunkSuper;
                    xs = fe > f ? (fe - 1) / kSuperEdges - f / kSuperEdges + 1 : 0;
                    // Algorithm 2 casts each pixel's ray to the nearer x side of
                    // the polygon's box.  Here the centre of each 32-pixel word
                    // column picks the side for its pixels (the parity of a
                    // closed ring is the same either way; a fixed column width
                    // keeps centres on an edge alike in every launch shape), so
                    // pixels in the right half of a polygon need only the edges
                    // right of them
                    const double4 bb = reinterpret_cast<const double4 *>(ix.obj)[pid];
#pragma unroll
                    for (int wd = 0; wd < W; ++wd) {
                        const double wcx = i0 + 32.0 * wd + 16.0;
                        if (wcx - (bb.x * S - ox) >= (bb.z * S - ox) - wcx) dir |= (uint8_t)(1u << wd);
                    }
                }
#pragma unroll
                for (int o = 1; o < kFillGroup; o <<= 1) {
                    const long long y = __shfl_up(x, o, 64);
                    const long long ys = __shfl_up(xs, o, 64);
                    if (lane >= o) {
                        x += y;
                        xs += ys;
                    }
                }
                if (lane < nb) {
                    L.efirst[lane] = f;
                    L.eend[lane] = fe;
                    L.cpre[lane + 1] = x;
                    L.spre[lane + 1] = xs;
                    L.ldir[lane] = dir;
                }
                if (lane == 0) {
                    L.cpre[0] = 0;
                    L.spre[0] = 0;
                }
            }
            __syncthreads();
            // A chunk or super-chunk box of group polygon q can hold an edge the
            // edge stage below would use: on the ray side of some centre (left
            // of a word column's last centre for rays to -x, right of its first
            // for rays to +x) and spanning a region row.  The boxes bound every
            // edge's pixel coordinates (S is a power of two and rounding is
            // monotonic), so such an edge's box always passes.
            auto box_pass = [&](const float4 cb, int q) -> bool {
                const double cx0 = (double)cb.x * S - ox, cx1 = (double)cb.z * S - ox;
                bool side = false;
#pragma unroll
                for (int wd = 0; wd < W; ++wd)
                    side |= (L.ldir[q] >> wd) & 1u ? cx1 > i0 + 32.0 * wd + 0.5 : cx0 < i0 + 32.0 * wd + 31.5;
                return side && fmax(ceil((double)cb.y * S - oy - j0 - 0.5) - 1.0, 0.0) <=
                                   fmin(ceil((double)cb.w * S - oy - j0 - 0.5), RS - 1.0);
            };
            // the edges of the np chunks listed in L.lc / L.lq, one per lane
            auto edges_of = [&](int np) {
                for (int it = tid; it < np * kEdgeChunk; it += nthr) {
                    const int sl = it / kEdgeChunk;
                    const int qq = L.lq[sl];
                    const int64_t e = L.lc[sl] * kEdgeChunk + it % kEdgeChunk;
                    if (e < L.efirst[qq] || e >= L.eend[qq]) continue;
                    const double4 gd = reinterpret_cast<const double4 *>(ix.pedges)[e];
                    const double ax = gd.x * S - ox, ay = gd.y * S - oy, bx = gd.z * S - ox, by = gd.w * S - oy;
                    const uint32_t dir = L.ldir[qq];
                    if (ay == by) continue;
                    // no crossing on the ray side of any centre
                    bool side = false;
#pragma unroll
                    for (int wd = 0; wd < W; ++wd)
                        side |= (dir >> wd) & 1u ? fmax(ax, bx) > i0 + 32.0 * wd + 0.5
                                                 : fmin(ax, bx) < i0 + 32.0 * wd + 31.5;
                    if (!side) continue;
                    uint32_t *pq = par + qq * (RS * W);
                    // candidate rows, one wider on each side; each is checked exactly
                    const int jlo = (int)fmax(ceil(fmin(ay, by) - j0 - 0.5) - 1.0, 0.0);
                    const int jhi = (int)fmin(ceil(fmax(ay, by) - j0 - 0.5), RS - 1.0);
                    for (int j = jlo; j <= jhi; ++j) {
                        const double yc = j0 + (double)j + 0.5;
                        if ((ay > yc) == (by > yc)) continue;
                        const double xc = ax + (yc - ay) * (bx - ax) / (by - ay);
                        // the first pixel strictly right of xc and the last
                        // strictly left of it, clamped to [-1, RS]
                        const int k0 = (int)fmin(fmax(floor(xc - i0 - 0.5) + 1.0, -1.0), (double)RS);
                        const int k1 = (int)fmin(fmax(ceil(xc - i0 - 0.5) - 1.0, -1.0), (double)RS);
#pragma unroll
                        for (int wd = 0; wd < W; ++wd) {
                            uint32_t bits;
                            if ((dir >> wd) & 1u) {
                                // rays to +x: the crossing counts for the centres left of it
                                const int hi = k1 - 32 * wd;
                                bits = hi < 0 ? 0u : hi >= 31 ? 0xffffffffu : ((2u << hi) - 1u);
                            } else {
                                // rays to -x: for the centres right of it
                                const int lo = k0 - 32 * wd;
                                bits = lo <= 0 ? 0xffffffffu : lo >= 32 ? 0u : (0xffffffffu << lo);
                            }
                            if (bits) atomicXor(&pq[j * W + wd], bits);
                        }
                    }
                }
            };
            // One round: each lane tests the chunk its index gives (if any),
            // the passing chunks are listed, and their edges dealt out.
            int round = 0;
            auto chunk_round = [&](bool have, int64_t c, int q) {
                int *npass = &ctl[2 + (round & 1)];
                const bool pass = have && box_pass(ix.pchunk[c], q);
                const int slot = wave_alloc(npass, __ballot(pass), lane);
                if (pass) {
                    L.lc[slot] = c;
                    L.lq[slot] = (uint8_t)q;
                }
                __syncthreads();
                edges_of(*npass);
                __syncthreads();
                // this round's counter is free again (the next round uses the
                // other one, cleared before this round's first barrier)
                if (tid == 0) *npass = 0;
                ++round;
            };
            const int64_t tot = L.cpre[nb];
            if (tot <= (int64_t)kFlatChunkRounds * nthr) {
                // few chunks: every chunk box is tested, nthr per round
                for (int64_t base = 0; base < tot; base += nthr) {
                    const int64_t g = base + tid;
                    int q = 0;
                    int64_t c = 0;
                    if (g < tot) {
                        // the group's polygon holding chunk g: largest q with cpre[q] <= g
#pragma unroll
                        for (int h = kFillGroup / 2; h > 0; h >>= 1)
                            if (q + h < nb && L.cpre[q + h] <= g) q += h;
                        c = L.efirst[q] / kEdgeChunk + (g - L.cpre[q]);
                    }
                    chunk_round(g < tot, c, q);
                }
            } else {
                // many chunks (polygons with many edges): the super-chunk boxes
                // first, nthr per round, then only the chunks of those that pass
                const int64_t stot = L.spre[nb];
                for (int64_t base = 0; base < stot; base += nthr) {
                    const int64_t g = base + tid;
                    bool pass = false;
                    int q = 0;
                    int64_t sc = 0;
                    if (g < stot) {
#pragma unroll
                        for (int h = kFillGroup / 2; h > 0; h >>= 1)
                            if (q + h < nb && L.spre[q + h] <= g) q += h;
                        sc = L.efirst[q] / (kEdgeChunk * kChunkSuper) + (g - L.spre[q]);
                        pass = box_pass(ix.psuper[sc], q);
                    }
                    const int slot = wave_alloc(&ctl[4], __ballot(pass), lane);
                    if (pass) {
                        L.ls[slot] = sc;
                        L.lsq[slot] = (uint8_t)q;
                    }
                    __syncthreads();
                    const int ns = ctl[4];
                    for (int cb = 0; cb < ns * kChunkSuper; cb += nthr) {
                        const int it = cb + tid;
                        bool have = false;
                        int q2 = 0;
                        int64_t c = 0;
                        if (it < ns * kChunkSuper) {
                            const int sl = it / kChunkSuper;
                            q2 = L.lsq[sl];
                            c = L.ls[sl] * kChunkSuper + it % kChunkSuper;
                            // only the polygon's own chunks of the super-chunk
                            have = c >= L.efirst[q2] / kEdgeChunk && c <= (L.eend[q2] - 1) / kEdgeChunk;
                        }
                        chunk_round(have, c, q2);
                    }
                    // every lane has read ctl[4] and the list before it is reset
                    __syncthreads();
                    if (tid == 0) ctl[4] = 0;
                    __syncthreads();
                }
            }
            __syncthreads();
            bool full = true;
            for (int k = tid; k < RS * W; k += nthr) {
                uint32_t v = mask[k];
                for (int q = 0; q < nb; ++q) {
                    v |= par[q * (RS * W) + k];
                    par[q * (RS * W) + k] = 0;
                }
                mask[k] = v;
                full &= v == 0xffffffffu;
            }
            if (__syncthreads_and(full)) return true;
        }
        if (tid == 0) ctl[1] = 0;
        __syncthreads();
        return false;
    };

    bool done = false;
    for (;;) {
        const int sp = ctl[0];
        if (sp == 0) break;
        const int lvl = (int)(stk[sp - 1] >> kLevelShift);
        const int per_step = lvl > 0 ? nthr / kFan : nthr / kLeaf;
        const bool top = tid < per_step && tid < sp && (int)(stk[sp - 1 - tid] >> kLevelShift) == lvl;
        const int npop = __syncthreads_count(top);
        const int j = tid >> 4, c = tid & 15;
        const uint32_t node = j < npop ? (stk[sp - 1 - j] & kIdxMask) : 0u;
        if (tid == 0) ctl[0] = sp - npop;
        __syncthreads();
        if (lvl > 0) {
            const int cl = lvl - 1;
            const int64_t child = (int64_t)node * kFan + c;
            bool push = false;
            if (j < npop && child < ix.meta[kMaxLevels + cl]) {
                const double4 nb = ix.nodes[ix.meta[cl] + child];
                if (meets(nb, qx0, qx1, qy0, qy1)) {
                    // the same test as for a polygon below: the node's box
                    // holds every box of its subtree, and its range of pixel
                    // centres (rounded the same way) every range of theirs
                    const double cx0 = fmax(ceil(nb.x * S - ox - i0 - 0.5), 0.0);
                    const double cx1 = fmin(floor(nb.z * S - ox - i0 - 0.5), RS - 1.0);
                    const double cy0 = fmax(ceil(nb.y * S - oy - j0 - 0.5), 0.0);
                    const double cy1 = fmin(floor(nb.w * S - oy - j0 - 0.5), RS - 1.0);
                    push = cx0 <= cx1 && cy0 <= cy1 &&
                           !range_lit<W>(mask, (int)cx0, (int)cx1, (int)cy0, (int)cy1);
                }
            }
            const int pos = wave_alloc(&ctl[0], __ballot(push), lane);
            if (push) stk[pos] = ((uint32_t)cl << kLevelShift) | (uint32_t)child;
        } else {
            // a polygon whose box holds no pixel centre of the region holds
            // none, and one whose centres are all filled adds nothing
            const int64_t o = (int64_t)node * kLeaf + c;
            bool keep = false;
            uint32_t rg = 0;
            if (j < npop && o < ix.n) {
                const double4 bb = reinterpret_cast<const double4 *>(ix.obj)[o];
                const double cx0 = fmax(ceil(bb.x * S - ox - i0 - 0.5), 0.0);
                const double cx1 = fmin(floor(bb.z * S - ox - i0 - 0.5), RS - 1.0);
                const double cy0 = fmax(ceil(bb.y * S - oy - j0 - 0.5), 0.0);
                const double cy1 = fmin(floor(bb.w * S - oy - j0 - 0.5), RS - 1.0);
                if (cx0 <= cx1 && cy0 <= cy1) {
                    rg = (uint32_t)cx0 | ((uint32_t)cx1 << 6) | ((uint32_t)cy0 << 12) | ((uint32_t)cy1 << 18);
                    keep = !range_lit<W>(mask, (int)cx0, (int)cx1, (int)cy0, (int)cy1);
                }
            }
            const int slot = wave_alloc(&ctl[1], __ballot(keep), lane);
            if (keep) {
                L.cand[slot] = (uint32_t)o;  // edges and offsets are stored by sorted position
                L.crng[slot] = rg;
            }
        }
        __syncthreads();
        if (ctl[1] > cap - nthr && test()) {
            done = true;
            break;
        }
    }
    if (!done && ctl[1] > 0) test();
    __syncthreads();
    for (int k = tid; k < RS * W; k += nthr) {
        const int row = k / W, wd = k % W;
        *reinterpret_cast<uint32_t *>(tm + (ry * RS + row) * 32 + rx * (RS / 8) + 4 * wd) = mask[k];
    }
    __syncthreads();
}

template <int RS>
__global__ __launch_bounds__(256) void k_fill_region(DevBatch B, int cap, int max_levels) {
    extern __shared__ double4 smem[];
    constexpr int RPT = (256 / RS) * (256 / RS);
    unsigned char *base = reinterpret_cast<unsigned char *>(smem);
    FillLds L;
    L.stk = reinterpret_cast<uint32_t *>(base);
    unsigned char *cb = base + align16((size_t)region_stack_words(max_levels, blockDim.x) * 4);
    constexpr size_t kRows = (size_t)RS * (RS / 32) * 4;
    L.cand = reinterpret_cast<uint32_t *>(cb);
    L.crng = reinterpret_cast<uint32_t *>(cb + align16((size_t)cap * 4));
    L.mask = reinterpret_cast<uint32_t *>(cb + 2 * align16((size_t)cap * 4));
    L.par = L.mask + align16(kRows) / 4;
    L.efirst = reinterpret_cast<int64_t *>(L.par + align16(kFillGroup * kRows) / 4);
    L.eend = L.efirst + align16(kFillGroup * 8) / 8;
    L.cpre = L.eend + align16(kFillGroup * 8) / 8;
    L.lc = L.cpre + align16((kFillGroup + 1) * 8) / 8;
    L.lq = reinterpret_cast<uint8_t *>(L.lc + blockDim.x);
    L.ldir = L.lq + align16(blockDim.x);
    L.spre = reinterpret_cast<int64_t *>(L.ldir + align16(kFillGroup));
    L.ls = L.spre + align16((kFillGroup + 1) * 8) / 8;
    L.lsq = reinterpret_cast<uint8_t *>(L.ls + blockDim.x);
    L.ctl = reinterpret_cast<int *>(L.lsq + align16(blockDim.x));
    // the group parity rows start at zero and every group clears what it used
    for (int k = threadIdx.x; k < kFillGroup * RS * (RS / 32); k += blockDim.x) L.par[k] = 0;
    __syncthreads();
    uint8_t *const out = B.hdr->out;
    zero_empty_tiles(B, out);
    const ItemMap im(B.hdr->counter, RPT);
    for (int64_t u = im.first; u < im.n; u += im.step) {
        const int64_t t = B.list[im.pos(u, RPT)];
        const int reg = (int)(u % RPT);
        const DevReq rq = B.reqs[t];
        const DevIndex ix = B.ixs[rq.index];
        fill_query<RS>(ix, rq, t, reg, B.frontier, B.fmeta, out, cap, L);
        if (threadIdx.x == 0) part_done(B, t, RPT);
    }
}

using RegionKernel = void (*)(DevBatch, int, int);

template <int AA>
RegionKernel region_kernel_aa(const LaunchShape &s) {
    if (s.region == 32)
        return s.opl == 4 ? k_query_region<32, 4, AA> : s.opl == 2 ? k_query_region<32, 2, AA> : k_query_region<32, 1, AA>;
    return s.opl == 4 ? k_query_region<64, 4, AA> : s.opl == 2 ? k_query_region<64, 2, AA> : k_query_region<64, 1, AA>;
}

RegionKernel region_kernel(const LaunchShape &s) { return s.aa ? region_kernel_aa<1>(s) : region_kernel_aa<0>(s); }

struct GridKey {
    int device, block, waves, region, opl, fill, aa;
    size_t lds;
    int grid;
};

}  // namespace

size_t query_lds_bytes(const LaunchShape &s, int max_levels) {
    if (s.fill) return fill_lds_bytes(s.cand_cap, max_levels, 64 * s.waves, s.region);
    if (s.region) return region_lds_bytes(s.cand_cap, max_levels, 64 * s.waves, s.region, s.opl, s.aa);
    return (size_t)s.waves * wave_lds_bytes(s.cand_cap, max_levels, s.block);
}

Workspace workspace_layout(int64_t n_req, int n_ix) {
    static_assert(sizeof(BatchHeader) <= 256, "the header must fit before the index table");
    Workspace w;
    w.n_req = n_req;
    w.hdr_off = 0;
    w.table_off = 256;
    w.req_off = w.table_off + align256(sizeof(DevIndex) * (size_t)n_ix);
    w.order_off = w.req_off + align256(sizeof(DevReq) * (size_t)n_req);
    w.frontier_off = w.order_off + align256(sizeof(uint32_t) * (size_t)n_req);
    w.fmeta_off = w.frontier_off + align256(sizeof(uint32_t) * kFrontier * (size_t)n_req);
    w.list_off = w.fmeta_off + align256(sizeof(int32_t) * 4 * (size_t)n_req);
    w.elist_off = w.list_off + align256(sizeof(uint32_t) * (size_t)n_req);
    w.done_off = w.elist_off + align256(sizeof(uint32_t) * (size_t)n_req);
    w.ts_off = w.done_off + align256(sizeof(uint32_t) * (size_t)n_req);
    w.total = w.ts_off + align256(sizeof(uint64_t) * (size_t)n_req);
    return w;
}

void stage_host(const Workspace &w, const DevIndex *ixs, int n_ix, const DevReq *reqs, int64_t n_req, uint8_t *out,
                unsigned char *host) {
    BatchHeader h;
    memset(&h, 0, sizeof h);
    h.n_req = n_req;
    h.out = out;
    memcpy(host + w.hdr_off, &h, sizeof h);
    memcpy(host + w.table_off, ixs, sizeof(DevIndex) * (size_t)n_ix);
    memcpy(host + w.req_off, reqs, sizeof(DevReq) * (size_t)n_req);
    // counting sort by zoom, stable (zooms are validated; the clamp only
    // keeps the buckets in bounds)
    auto bucket = [&](int64_t k) { return std::min(std::max(reqs[k].z, 0), (int32_t)HV_MAX_ZOOM); };
    int64_t start[HV_MAX_ZOOM + 2] = {};
    for (int64_t k = 0; k < n_req; ++k) ++start[bucket(k) + 1];
    for (int z = 0; z <= HV_MAX_ZOOM; ++z) start[z + 1] += start[z];
    uint32_t *order = reinterpret_cast<uint32_t *>(host + w.order_off);
    for (int64_t k = 0; k < n_req; ++k) order[start[bucket(k)]++] = (uint32_t)k;
}

DevBatch device_batch(const Workspace &w, unsigned char *dws) {
    DevBatch b;
    b.hdr = reinterpret_cast<BatchHeader *>(dws + w.hdr_off);
    b.ixs = reinterpret_cast<const DevIndex *>(dws + w.table_off);
    b.reqs = reinterpret_cast<const DevReq *>(dws + w.req_off);
    b.order = reinterpret_cast<const uint32_t *>(dws + w.order_off);
    b.frontier = reinterpret_cast<uint32_t *>(dws + w.frontier_off);
    b.fmeta = reinterpret_cast<int32_t *>(dws + w.fmeta_off);
    b.list = reinterpret_cast<uint32_t *>(dws + w.list_off);
    b.elist = reinterpret_cast<uint32_t *>(dws + w.elist_off);
    b.done = reinterpret_cast<uint32_t *>(dws + w.done_off);
    b.ts = reinterpret_cast<uint64_t *>(dws + w.ts_off);
    return b;
}

int persistent_grid(const LaunchShape &s, int max_levels) {
    static std::mutex mu;
    static GridKey cache[16];
    static int ncache = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    const size_t lds = query_lds_bytes(s, max_levels);
    std::lock_guard<std::mutex> g(mu);
    for (int k = 0; k < ncache; ++k)
        if (cache[k].device == dev && cache[k].block == s.block && cache[k].waves == s.waves &&
            cache[k].region == s.region && cache[k].opl == s.opl && cache[k].fill == s.fill && cache[k].aa == s.aa &&
            cache[k].lds == lds)
            return cache[k].grid;
    int per_cu = 0, cus = 0;
    const int thr = 64 * s.waves;
    hipError_t e;
    if (s.fill)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, s.region == 64 ? k_fill_region<64> : k_fill_region<32>,
                                                         thr, lds);
    else if (s.region) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, region_kernel(s), thr, lds);
    else if (s.block == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query<8>, thr, lds);
    else if (s.block == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query<16>, thr, lds);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query<32>, thr, lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    (void)hipGetLastError();
    // ten times what fits at once: the dispatcher then hands out the
    // remaining workgroups as others finish, which evens out uneven blocks
    const int grid = 10 * per_cu * cus;
    if (ncache < 16) cache[ncache++] = GridKey{dev, s.block, s.waves, s.region, s.opl, s.fill, s.aa, lds, grid};
    return grid;
}

hipError_t launch_query(const Workspace &w, unsigned char *dws, int max_levels, const LaunchShape &s,
                        hipStream_t st, hipEvent_t *marks) {
    const int64_t n_req = w.n_req;  // requests the grids cover; the header holds how many are live
    if (n_req == 0) return hipSuccess;
    const DevBatch B = device_batch(w, dws);
    hipError_t e;
    if (marks && (e = hipEventRecord(marks[0], st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_frontier, dim3((uint32_t)((n_req + 3) / 4)), dim3(256), 0, st, B, s.region, s.cull,
                       s.aa ? 0.25 : 0.0);
    if (marks && (e = hipEventRecord(marks[1], st)) != hipSuccess) return e;
    const size_t lds = query_lds_bytes(s, max_levels);
    // never more workgroups than there are blocks (or regions) to render
    const int64_t per_tile = s.region ? (256 / s.region) * (256 / s.region)
                                      : ((256 / s.block) * (256 / s.block) + s.waves - 1) / s.waves;
    // (the item count per XCD is rounded up to whole tiles)
    const int64_t need = n_req * per_tile;
    // filling's regions differ in cost by orders of magnitude (clusters of
    // small polygons next to empty sea), so by default each gets its own
    // workgroup and the dispatcher balances them; the distance kernels keep a
    // persistent grid
    int64_t grid = s.grid > 0 ? s.grid : s.fill ? kFillGrid : persistent_grid(s, max_levels);
    if (grid > need) grid = need;
    const dim3 g((uint32_t)grid), b((uint32_t)(64 * s.waves));
    if (s.fill && s.region == 64) hipLaunchKernelGGL(k_fill_region<64>, g, b, lds, st, B, s.cand_cap, max_levels);
    else if (s.fill) hipLaunchKernelGGL(k_fill_region<32>, g, b, lds, st, B, s.cand_cap, max_levels);
    else if (s.region) hipLaunchKernelGGL(region_kernel(s), g, b, lds, st, B, s.cand_cap, max_levels);
    else if (s.block == 8) hipLaunchKernelGGL(k_query<8>, g, b, lds, st, B, s.cand_cap, max_levels);
    else if (s.block == 16) hipLaunchKernelGGL(k_query<16>, g, b, lds, st, B, s.cand_cap, max_levels);
    else hipLaunchKernelGGL(k_query<32>, g, b, lds, st, B, s.cand_cap, max_levels);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (marks && (e = hipEventRecord(marks[2], st)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace hv
