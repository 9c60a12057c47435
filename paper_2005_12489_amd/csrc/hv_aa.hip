// Anti-aliased values assembled from child-tile masks (Algorithm 1,
// Sec. 3.2.1).  The four sub-samples of pixel (i, j) of tile (z, x, y), its
// centre +- 1/4 px in x and y, are the centres of pixels (2i mod 256 + a',
// 2j mod 256 + b'), a', b' in {0, 1}, of the child tile (z + 1, 2x + i / 128,
// 2y + j / 128); at zoom z + 1 every length in pixels doubles, so a binary
// mask of the child at radius 2 r holds the sub-samples' bits.
#include "hv_internal.h"

namespace hv {

// One thread per 16 output bytes (pixel row j, columns 16c .. 16c + 15) of
// request k.  map[k] >= 0: the request's child masks are kids[4 map[k] +
// 2 b + a] (8192 bytes each, a and b the column and row halves);
// map[k] < 0: its values are request -1 - map[k] of `whole`, copied.
__global__ __launch_bounds__(256) void k_aa_assemble(const int32_t *__restrict__ map, int64_t n,
                                                     const uint32_t *__restrict__ kids,
                                                     const uint4 *__restrict__ whole, uint4 *__restrict__ out) {
    const int64_t total = n * 4096;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256) {
        const int64_t k = g >> 12;
        const int q = (int)(g & 4095), j = q >> 4, c = q & 15;
        const int32_t m = map[k];
        uint4 v;
        if (m < 0) {
            v = whole[(int64_t)(-1 - m) * 4096 + q];
        } else {
            // child rows 2j mod 256 and the next, columns 32c mod 256 .. +31:
            // word c mod 8 of each 8-word row
            const uint32_t *t = kids + ((int64_t)m * 4 + 2 * (j >> 7) + (c >> 3)) * 2048;
            const int row = 2 * (j & 127);
            const uint32_t w0 = t[row * 8 + (c & 7)], w1 = t[(row + 1) * 8 + (c & 7)];
            // bits per 2-bit field (pixel p: child columns 2p, 2p + 1), 0..2
            const uint32_t p0 = (w0 & 0x55555555u) + ((w0 >> 1) & 0x55555555u);
            const uint32_t p1 = (w1 & 0x55555555u) + ((w1 >> 1) & 0x55555555u);
            uint32_t o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t acc = 0;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const int sh = 2 * (4 * e + f);
                    acc |= (((p0 >> sh) & 3u) + ((p1 >> sh) & 3u)) << (8 * f);
                }
                o[e] = acc;
            }
            v = make_uint4(o[0], o[1], o[2], o[3]);
        }
        out[g] = v;
    }
}

hipError_t launch_aa_assemble(const int32_t *map, int64_t n, const uint8_t *kids, const uint8_t *whole,
                              uint8_t *out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n * 4096 + 255) / 256;
    const int grid = (int)(blocks < 262144 ? blocks : 262144);
    hipLaunchKernelGGL(k_aa_assemble, dim3(grid), dim3(256), 0, stream, map, n,
                       reinterpret_cast<const uint32_t *>(kids), reinterpret_cast<const uint4 *>(whole),
                       reinterpret_cast<uint4 *>(out));
    return hipGetLastError();
}

}  // namespace hv
