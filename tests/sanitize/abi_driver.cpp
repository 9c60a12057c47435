// Calls every host-side path of the C ABI that needs no GPU -- argument
// validation of every entry point, empty indexes, the byte estimates, error
// messages -- so that a host build of the library with AddressSanitizer and
// UndefinedBehaviorSanitizer can report any out-of-bounds access, leak or
// undefined operation in it.  Exit 0: every call returned what the header
// promises (the sanitizers abort on their own findings).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/hv.h"

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, \
                         hv_last_error());                                         \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

int main() {
    // index build
    CHECK(hv_index_build(nullptr, 7, 3) == nullptr && std::strlen(hv_last_error()) > 0);
    CHECK(hv_index_build(nullptr, HV_POINTS, -1) == nullptr);
    CHECK(hv_index_build(nullptr, HV_SEGMENTS, 3000000000LL) == nullptr);
    CHECK(hv_index_build(nullptr, HV_POINTS, 3) == nullptr);
    std::vector<double> host(8, 0.0);
    CHECK(hv_index_build(host.data(), HV_POINTS, 4) == nullptr);          // host memory: rejected
    hv_index *e = hv_index_build(nullptr, HV_SEGMENTS, 0);                 // empty index, no device
    CHECK(e != nullptr);
    hv_info info;
    CHECK(hv_index_info(e, &info) == HV_OK && info.n == 0 && info.levels == 0 && info.device_bytes == 0);
    CHECK(hv_index_info(nullptr, &info) == HV_EINVAL);
    CHECK(hv_index_read(e, HV_READ_ORDER, 0, host.data(), 0) == HV_OK);
    CHECK(hv_index_read(e, HV_READ_NODES, 0, host.data(), 0) == HV_EINVAL);
    CHECK(hv_index_read(e, 9, 0, host.data(), 0) == HV_EINVAL);
    // tiles and styles
    const hv_style st{1.0}, bad_r[] = {{0.0}, {-1.0}, {NAN}, {INFINITY}, {64.5}};
    const hv_tile ok_tiles[] = {{0, 0, 0, 0}, {22, (1 << 22) - 1, 0, 0}}, bad_tiles[] = {{23, 0, 0, 0}, {-1, 0, 0, 0},
                                                                                     {3, 8, 0, 0}, {3, 0, -1, 0}};
    uint8_t *dummy = reinterpret_cast<uint8_t *>(16);                      // never touched: rejected first
    for (const hv_tile &t : bad_tiles) CHECK(hv_render_tiles(e, &t, 1, &st, dummy) == HV_EINVAL);
    for (const hv_style &s : bad_r) CHECK(hv_render_tiles(e, ok_tiles, 1, &s, dummy) == HV_EINVAL);
    CHECK(hv_render_tiles(e, ok_tiles, 0, &st, nullptr) == HV_OK);
    CHECK(hv_render_tiles(e, ok_tiles, -1, &st, dummy) == HV_EINVAL);
    CHECK(hv_render_tiles(nullptr, ok_tiles, 1, &st, dummy) == HV_EINVAL);
    CHECK(hv_render_tiles(e, ok_tiles, 2, &st, host.data() ? reinterpret_cast<uint8_t *>(host.data()) : dummy) ==
          HV_EINVAL);                                                      // host output
    hv_launch L{};
    static_assert(sizeof(hv_launch) == 8 * sizeof(int), "hv_launch is eight int32 fields");
    const int bad_fields[][8] = {{12, 0, 0, 0, 0, 0, 0, 0}, {0, 32, 0, 0, 0, 0, 0, 0}, {0, 5000, 0, 0, 0, 0, 0, 0},
                                 {0, 0, 3, 0, 0, 0, 0, 0},  {0, 0, 0, -1, 0, 0, 0, 0}, {0, 0, 0, 0, 16, 0, 0, 0},
                                 {0, 0, 0, 0, 32, 3, 0, 0}, {0, 0, 0, 0, 0, 0, 300, 0}, {0, 64, 4, 0, 64, 4, 0, 0},
                                 {0, 0, 0, 0, 0, 0, 0, -3}, {0, 0, 0, 0, 0, 0, 0, 63}};
    for (const auto &f : bad_fields) {
        std::memcpy(&L, f, sizeof L);
        CHECK(hv_render_tiles_ex(e, ok_tiles, 1, &st, dummy, &L) == HV_EINVAL);
    }
    // batches
    hv_request rq[3] = {{e, 3, 1, 1, 0, 1.0}, {e, 5, 2, 2, 0, 2.0}, {nullptr, 1, 0, 0, 0, 1.0}};
    CHECK(hv_render_batch(rq, 3, dummy, nullptr) == HV_EINVAL);            // NULL index
    rq[2] = hv_request{e, 23, 0, 0, 0, 1.0};
    CHECK(hv_render_batch(rq, 3, dummy, nullptr) == HV_EINVAL);            // zoom
    CHECK(hv_render_batch(rq, -1, dummy, nullptr) == HV_EINVAL);
    CHECK(hv_render_batch(nullptr, 2, dummy, nullptr) == HV_EINVAL);
    CHECK(hv_render_batch(rq, 0, nullptr, nullptr) == HV_OK);
    CHECK(hv_render_batch_aa(rq, 3, dummy, nullptr) == HV_EINVAL);
    rq[2] = hv_request{e, 22, 0, 0, 0, 1.0};
    CHECK(hv_render_batch_aa(rq, 3, dummy, nullptr) == HV_EINVAL);         // output not device memory
    CHECK(hv_render_batch_aa(rq, 0, nullptr, nullptr) == HV_OK);
    std::vector<hv_request> many(HV_NOALLOC_MAX_REQUESTS + 1, hv_request{e, 3, 1, 1, 0, 1.0});
    CHECK(hv_render_batch_noalloc(many.data(), (int64_t)many.size(), dummy, nullptr) == HV_EINVAL);
    CHECK(hv_render_batch_noalloc(rq, -1, dummy, nullptr) == HV_EINVAL);
    CHECK(hv_batcher_create(0, 1, 4, nullptr) == nullptr);
    CHECK(hv_batcher_create(10, 0, 4, nullptr) == nullptr);
    CHECK(hv_batcher_create(10, 1, 17, nullptr) == nullptr);
    CHECK(hv_batcher_run(nullptr, rq, 1, dummy) == HV_EINVAL);
    CHECK(hv_batcher_latency(nullptr, nullptr, 0) == HV_EINVAL);
    hv_batcher_free(nullptr);
    hv_launch best;
    double ms = 0;
    CHECK(hv_autotune(rq, 0, dummy, &best, &ms) == HV_EINVAL);
    CHECK(hv_autotune(rq, 2, dummy, nullptr, &ms) == HV_EINVAL);
    CHECK(hv_tuned_launch(rq, 2, &best) == HV_EINVAL);                     // nothing tuned
    double km[2];
    CHECK(hv_time_kernels(rq, 0, dummy, nullptr, 1, km) == HV_EINVAL);
    CHECK(hv_time_kernels(rq, 2, dummy, nullptr, 0, km) == HV_EINVAL);
    // byte estimates
    const int64_t per = hv_estimate_bytes(e, &ok_tiles[0], &st);
    CHECK(per > HV_MASK_BYTES);
    CHECK(hv_estimate_bytes(e, &bad_tiles[0], &st) == HV_EINVAL);
    CHECK(hv_estimate_bytes(e, &ok_tiles[0], &bad_r[0]) == HV_EINVAL);
    CHECK(hv_estimate_bytes(nullptr, &ok_tiles[0], &st) == HV_EINVAL);
    for (int64_t n : {0LL, 1LL, 255LL, 4096LL, 1LL << 24}) {
        const int64_t b = hv_estimate_batch_bytes(n, 5);
        CHECK(b >= n * per && b <= n * per + 2304 + 96 * 5);
    }
    CHECK(hv_estimate_batch_bytes(-1, 1) == HV_EINVAL);
    CHECK(hv_estimate_batch_bytes(1, 5000) == HV_EINVAL);
    // polygon indexes
    const int64_t first_bad[3] = {0, 2, 6};
    CHECK(hv_polygon_index_build(host.data(), 6, first_bad, 2, 0) == nullptr);
    CHECK(hv_polygon_index_build(host.data(), 6, first_bad, 2, 7) == nullptr);
    hv_index *ep = hv_polygon_index_build(nullptr, 0, nullptr, 0, 0);
    CHECK(ep != nullptr);
    CHECK(hv_render_fill(ep, ok_tiles, 0, nullptr, nullptr) == HV_OK);
    CHECK(hv_render_fill(e, ok_tiles, 1, dummy, nullptr) == HV_EINVAL);     // not a polygon index
    CHECK(hv_render_tiles(ep, ok_tiles, 1, &st, dummy) == HV_EINVAL);       // polygon index
    CHECK(hv_estimate_bytes(ep, &ok_tiles[0], nullptr) > HV_MASK_BYTES);
    CHECK(hv_set_stream(nullptr) == HV_OK);
    hv_free(ep);
    hv_free(e);
    hv_free(nullptr);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("abi driver ok\n");
    return 0;
}
