/*
 * hv.h -- per-pixel tile masks from spatial-index queries on MI355X (gfx950).
 *
 * Display-driven computing after HiVision (arXiv 2005.12489): every pixel of
 * a 256x256 Web-Mercator tile is an independent unit of work, and its value
 * comes from index queries about the objects near it (Sec. 1 and Sec. 3).
 * This library computes the binary form of the paper's Algorithm 1 (SIBV):
 * pixel (i, j) of tile (z, x, y) is lit iff some indexed point, segment or
 * polygon edge lies within r pixels of the pixel's centre, where the
 * distance is Euclidean in world pixels of zoom z (one pixel is the
 * resolution R_z of Algorithm 1 and the style radius is R = N * R_z), and
 * the comparison is inclusive.
 *
 * Conventions used by every entry point:
 *   - Space: Web-Mercator normalised to [0,1]^2 with y = 0 at the north edge;
 *     latitude is clamped to +-85.0511287798066 deg; there is no
 *     antimeridian wrap.  Zoom z has 4^z tiles (XYZ scheme, rows from the
 *     north, Sec. 2.1 and Sec. 4) of 256x256 pixels.
 *   - Masks: one tile is 8192 bytes, row-major from the north-west pixel,
 *     32 bytes per row; pixel column i is bit (i & 7), least significant
 *     first, of byte (i >> 3) of its row.  Masks are fully overwritten.
 *   - Precision: coordinates, distances and comparisons are FP64.
 *   - Work is issued asynchronously on the calling thread's current stream
 *     (hv_set_stream; default: the null stream).  Device outputs are valid
 *     once that stream has reached the call.
 *   - Errors: every call validates its arguments on the host before any
 *     device work; on error nothing is launched, outputs are untouched, a
 *     negative status is returned (NULL for hv_index_build) and
 *     hv_last_error() describes the problem.  All entry points are
 *     thread-safe; the error message and current stream are per thread.
 */
#ifndef HV_H
#define HV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Index kinds (Sec. 3.1: RtreeP for points, RtreeL for linestring segments,
 * RtreeE for polygon edges; linestrings and polygons are split into segments
 * and edges before indexing). */
enum {
    HV_POINTS = 0,
    HV_SEGMENTS = 1,
    HV_POLYGON_EDGES = 2,
    /* A polygon index for filling (hv_polygon_index_build, hv_render_fill). */
    HV_POLYGONS = 3,
    /* OR-ed into kind: inputs are already normalised Mercator X,Y. */
    HV_INPUT_MERC01 = 0x100
};

enum { HV_OK = 0, HV_EINVAL = -1, HV_ENOMEM = -2, HV_EHIP = -3 };

/* Largest zoom accepted; 1 ulp of a world coordinate at z = 22 is 2.4e-7 px. */
#define HV_MAX_ZOOM 22
/* Largest style radius / half-width, px. */
#define HV_MAX_RADIUS 64.0
/* Largest object count (sorted positions are 32-bit). */
#define HV_MAX_OBJECTS 2000000000LL
#define HV_MASK_BYTES 8192
/* Bytes of one anti-aliased tile: one value 0-4 per pixel. */
#define HV_AA_BYTES 65536

typedef struct hv_index hv_index;

/* A tile request in the XYZ scheme: 0 <= z <= HV_MAX_ZOOM, 0 <= x, y < 2^z. */
typedef struct { int32_t z, x, y, pad; } hv_tile;

/* Style: point radius, or line / edge half-width (= width / 2), in pixels;
 * 0 < r_px <= HV_MAX_RADIUS (Algorithm 1's radius N). */
typedef struct { double r_px; } hv_style;

/* Build an index over `n` objects (Sec. 3.1 data organisation; the paper's
 * R-trees are replaced by a Hilbert-packed R-tree built on the GPU).
 *   objects  device pointer owned by the caller, FP64 array-of-structures:
 *            points (n,2) = lon, lat; segments / edges (n,4) =
 *            lon0, lat0, lon1, lat1 (degrees; with HV_INPUT_MERC01 the
 *            values are normalised X, Y instead).  Polygon rings arrive as
 *            their edges, the closing edge included.  Only read during the
 *            call; the caller may free it once the call returns.
 *   kind     HV_POINTS, HV_SEGMENTS or HV_POLYGON_EDGES, optionally
 *            | HV_INPUT_MERC01.
 *   n        0 <= n <= HV_MAX_OBJECTS; n = 0 builds an empty index whose
 *            masks are all zero.
 * Synchronous.  Returns an index that owns all of its device memory and is
 * immutable (renders on several streams may share it), or NULL: HV_EINVAL
 * for a NULL pointer with n > 0, a bad kind or n, a non-finite coordinate,
 * |lon| > 180 or |lat| > 90; HV_ENOMEM when device memory runs out; HV_EHIP
 * for another HIP error. */
hv_index *hv_index_build(const double *objects, int kind, int64_t n);

/* Render the masks of `n_tiles` tiles of one index with one style
 * (Algorithm 1 per pixel, binary form).  One launch covers every tile.
 *   tiles      host array of n_tiles requests (copied during the call).
 *   style      host pointer.
 *   out_masks  device buffer of n_tiles * 8192 bytes owned by the caller,
 *              16-byte aligned; it must not alias the index.  Tile k's
 *              mask is at k * 8192.
 * Tiles that miss the data's bounding box (grown by r) come out all zero
 * without a traversal (Sec. 4.1: such tiles create no task).
 * Returns HV_OK, or HV_EINVAL for a NULL index/style/pointer with
 * n_tiles > 0, n_tiles < 0, z outside [0, 22], x or y outside [0, 2^z),
 * r_px not finite or outside (0, 64], or out_masks not 16-byte aligned
 * device memory; HV_EHIP on a launch failure. */
int hv_render_tiles(const hv_index *index, const hv_tile *tiles, int64_t n_tiles,
                    const hv_style *style, uint8_t *out_masks);

/* Release an index and its device memory (NULL-safe).  The caller must make
 * sure no render using it is still in flight. */
void hv_free(hv_index *index);

/* Message describing the calling thread's most recent error ("" if none). */
const char *hv_last_error(void);

/* Set the calling thread's stream (a hipStream_t; NULL = null stream). */
int hv_set_stream(void *hip_stream);

/* Launch shape of the query kernel.  The default (a NULL launch) follows
 * the batch size n: region = 32, objs_per_lane 2, waves_per_wg 4 for
 * n < 1024, 2 for n < 4096 and 1 beyond (in a small batch the heaviest
 * regions set the time and more waves shorten them; a large one fills the
 * GPU with single-wave groups), cand_cap 128 * waves_per_wg and cull_nodes
 * 256.  Anti-aliased output takes the same default; filling has its own
 * (hv_render_fill).  In a given shape, zero
 * fields take block 16, waves_per_wg 2 (1 in region mode), objs_per_lane
 * 1, cand_cap 64 * waves_per_wg * objs_per_lane in region mode (64
 * otherwise), cull_nodes 256 and a grid that fills the GPU; region = 0
 * selects one wavefront per pixel block. */
typedef struct {
    int32_t block;          /* pixel block per wavefront: 8, 16 or 32 (1, 4 or 16 px/lane) */
    int32_t cand_cap;       /* LDS candidate capacity per wavefront, >= 64 */
    int32_t waves_per_wg;   /* wavefronts per workgroup: 1, 2 or 4 */
    int32_t grid_wgs;       /* workgroups of the persistent query kernel; 0 = ten times as many as fit on
                               the GPU (filling: one per region, at most 262,144) */
    int32_t region;         /* 0: one wavefront per pixel block; 32 or 64: one workgroup per region of
                               that side whose queued objects are dealt out over all lanes (block is
                               then unused and cand_cap sizes the queue) */
    int32_t objs_per_lane;  /* region mode: objects each lane loads per leaf step, 1, 2 or 4;
                               cand_cap must be >= 64 * waves_per_wg; below 64 * waves_per_wg *
                               objs_per_lane the queue takes a step's objects 64 * waves_per_wg at
                               a time, draining in between (less LDS: more workgroups per CU) */
    int32_t cull_nodes;     /* cull depth of the per-tile pass: it descends the tree while the next
                               level holds at most this many nodes that meet the tile, 1..256
                               (0 = 256); blocks and regions then walk on from those nodes */
    int32_t aa_split;       /* anti-aliased output only (hv_render_batch_aa): which requests render
                               as their four child tiles instead of in one pass.  k in [1, 62]: those
                               whose index holds at least 2^k * 4^z objects; -1: none; -2: all;
                               0: k = HV_AA_SPLIT_DEFAULT.  Only requests with z < HV_MAX_ZOOM and
                               2 r <= HV_MAX_RADIUS qualify.  Other entry points ignore it. */
} hv_launch;

/* Default of hv_launch.aa_split: requests whose index holds at least
 * 2^HV_AA_SPLIT_DEFAULT objects per tile of their zoom (as if spread
 * evenly) render anti-aliased output as child tiles. */
#define HV_AA_SPLIT_DEFAULT 12

/* hv_render_tiles with an explicit launch shape (autotuning and variant
 * tests).  Every valid shape produces identical masks.  Extra HV_EINVAL
 * cases: block not 8, 16 or 32, cand_cap < 64 or > 4096, waves_per_wg not 1,
 * 2 or 4, grid_wgs outside [0, 2^20], region not 0, 32 or 64,
 * objs_per_lane not 1, 2 or 4, cand_cap below 64 * waves_per_wg in region
 * mode, cull_nodes outside [0, 256], or a shape
 * needing more than 64 KiB of LDS per workgroup. */
int hv_render_tiles_ex(const hv_index *index, const hv_tile *tiles, int64_t n_tiles,
                       const hv_style *style, uint8_t *out_masks, const hv_launch *launch);

/* Facts about a built index. */
typedef struct {
    int32_t kind;           /* HV_POINTS / HV_SEGMENTS / HV_POLYGON_EDGES */
    int32_t levels;         /* node levels, leaves = level 0 */
    int64_t n;              /* objects */
    int64_t nodes;          /* nodes over all levels */
    int32_t leaf_size;      /* objects per leaf */
    int32_t fanout;         /* children per inner node */
    int32_t key_bits;       /* Hilbert order used for sorting (bits per axis) */
    int32_t pad;
    double root[4];         /* data bounding box: min X, min Y, max X, max Y (normalised) */
    int64_t device_bytes;   /* device memory held by the index */
    double build_ms;        /* wall time of hv_index_build */
} hv_info;

/* Fill *info.  Returns HV_OK or HV_EINVAL for a NULL argument. */
int hv_index_info(const hv_index *index, hv_info *info);

/* Copy one of the index's device arrays to host memory (synchronous; for
 * tests and tools).  what: HV_READ_ORDER = sorted position -> input index
 * (uint32, n entries); HV_READ_OBJECTS = projected objects in sorted order
 * (FP64, n*2 or n*4); HV_READ_NODES = node boxes of `level` (FP64 min X,
 * min Y, max X, max Y per node).  `bytes` must equal the array's size.
 * Returns HV_OK, HV_EINVAL, or HV_EHIP. */
enum { HV_READ_ORDER = 0, HV_READ_OBJECTS = 1, HV_READ_NODES = 2 };
int hv_index_read(const hv_index *index, int what, int level, void *host_dst, int64_t bytes);

/* ------------------------------------------------------------------ batches
 * Many heterogeneous requests -- tiles of different indexes, zooms and
 * styles -- rendered by one launch of the query, the way the paper's engine
 * hands queued tile tasks to whichever process is idle (Sec. 4.2, 4.3). */

/* One request: a tile of `index` with its own radius / half-width. */
typedef struct {
    const hv_index *index;
    int32_t z, x, y, pad;
    double r_px;
} hv_request;

/* Render n requests in one launch.  reqs: host array (copied during the
 * call); out_masks: device, n * 8192 bytes, 16-byte aligned, request k at
 * k * 8192.  launch: NULL takes the autotuned shape for the batch's class
 * (see hv_autotune) or the default.  Every index must live on the current
 * device.  Errors as hv_render_tiles_ex, plus HV_EINVAL for a NULL index in
 * a request. */
int hv_render_batch(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch);

/* A reusable batch executor.  It owns, twice over, a device workspace for
 * up to max_requests requests over up to max_indexes distinct indexes of at
 * most max_levels tree levels, and a pinned host staging buffer; for each
 * it captures one HIP graph [copy staged requests -> frontier kernel ->
 * query kernel] at creation, so a run is one graph launch.  Runs use the
 * two slots in turn; a run waits (on the host) until the run that last used
 * its slot has finished.  launch: the query shape baked into the graphs;
 * NULL = the default, which then captures one graph per size class of the
 * default shape that max_requests reaches, and a run launches the one for
 * its batch size.  Returns NULL on error (hv_last_error). */
typedef struct hv_batcher hv_batcher;
hv_batcher *hv_batcher_create(int64_t max_requests, int32_t max_indexes, int32_t max_levels,
                              const hv_launch *launch);

/* Launch one batch on the calling thread's stream (asynchronous).  Same
 * arguments and errors as hv_render_batch, plus HV_EINVAL when n exceeds
 * max_requests, the batch names more than max_indexes indexes, or an index
 * is deeper than max_levels. */
int hv_batcher_run(hv_batcher *b, const hv_request *reqs, int64_t n, uint8_t *out_masks);

/* Wait until the last run has finished, then write each of its requests'
 * completion time, in microseconds after the batch started on the device,
 * to latency_us (host, n entries; n must equal that run's size).  A
 * request completes when the last part of its tile has been written. */
int hv_batcher_latency(hv_batcher *b, double *latency_us, int64_t n);

/* Release a batcher (NULL-safe); waits for its runs first. */
void hv_batcher_free(hv_batcher *b);

/* Time a set of launch shapes on a sample batch and return the fastest in
 * *best (and its time per launch in *best_ms, may be NULL: the frontier and
 * query kernels between HIP events, the fastest of the repeats).  Each shape
 * runs first on 16, then 128 evenly spread requests of the sample, then on
 * all of it, and is dropped once a part takes more than four times the
 * best time seen on that part; on the whole sample a shape replaces the one
 * chosen so far only if it is at least 3% faster (the candidates start with
 * the default shapes).  The result is also cached under the
 * sample's class -- dominant kind, zoom band (z / 4), radius band (r <= 1,
 * <= 2, <= 4, > 4) and size band (n < 1024, < 4096, larger) -- which
 * hv_render_batch with launch == NULL then uses for batches of that class.  scratch_masks:
 * device, n * 8192 bytes.  Synchronous. */
int hv_autotune(const hv_request *sample, int64_t n, uint8_t *scratch_masks, hv_launch *best, double *best_ms);

/* The cached shape for a batch's class: HV_OK and *out filled, or HV_EINVAL
 * if that class has not been tuned. */
int hv_tuned_launch(const hv_request *reqs, int64_t n, hv_launch *out);

/* Anti-aliased output: Algorithm 1's value 0-4 per pixel (Sec. 3.2.1), the
 * number of the pixel's four sub-samples -- its centre +- 1/4 px in x and y
 * -- that lie within r of some object of the request's index, each
 * sub-sample measured against its own nearest object (Algorithm 1 as
 * printed measures all four against the object nearest the centre, which
 * can count fewer).  One pass of the region kernel, with four sub-sample
 * masks per region: it culls with the samples' reach (r + 1/4 px per axis),
 * lights sub-samples near node boxes and representatives on each sub-sample
 * grid without reading objects (the binary kernel's accepts), and from
 * r = 1 px on sets all four sub-samples of a pixel whose centre lies
 * within r - sqrt(2)/4 px of an object (Algorithm 1's R1) and none of one
 * beyond r + sqrt(2)/4 (R2); it tests the four sub-samples of every other
 * pixel in reach exactly (FP64, inclusive).
 * reqs: host array as for hv_render_batch (0 <= z <= HV_MAX_ZOOM).
 * out_values: device, n * HV_AA_BYTES bytes, 16-byte aligned; the value of
 * pixel (i, j) of request k is at k * HV_AA_BYTES + j * 256 + i.
 * A request can instead render as its four child tiles, (z + 1, 2x + a,
 * 2y + b) for a, b in {0, 1}, in binary form at radius 2 r, each pixel's
 * value then being the number of set bits among its 2 x 2 child pixels: the
 * centres of those pixels are exactly its sub-samples, and doubling every
 * length in pixels at the next zoom leaves each comparison unchanged, so
 * both forms give the same values (up to rounding where a sub-sample's
 * distance lies within rounding error of r).  The child form does four times the
 * pixel work but none of the one-pass form's four-grid accepts; it is faster
 * on dense tiles, where accepts decide most pixels.  launch->aa_split picks
 * the requests that take it (default: HV_AA_SPLIT_DEFAULT).  A batch with
 * such requests allocates 32 KiB of child masks per such request, plus
 * 64 KiB per other request when both forms are present, in stream order
 * on the calling thread's stream.
 * launch: the query shape (NULL = the default shape for n requests; a shape
 * with region = 0 runs with region 32, the one-pass form needing region
 * mode; the child tiles run in the shape as given, or with NULL in the
 * default shape for their number).  Asynchronous on the
 * calling thread's stream.  Errors as hv_render_batch, and HV_EINVAL for
 * aa_split outside [-2, 62]; nothing is launched on error. */
int hv_render_batch_aa(const hv_request *reqs, int64_t n, uint8_t *out_values, const hv_launch *launch);

/* Polygon index for filling (Sec. 3.1, the multi-level index for polygons:
 * the polygons' bounding boxes in a tree -- the paper's RtreeMBR -- and each
 * polygon's edges).  edges: device, n x 4 doubles (lon0, lat0, lon1, lat1,
 * or normalised Mercator with flags = HV_INPUT_MERC01), grouped by polygon:
 * polygon p owns edges first[p] .. first[p + 1] - 1, which must form closed
 * rings (several rings make holes, even-odd).  first: host, npoly + 1
 * entries, first[0] = 0, first[npoly] = n, at least 3 edges per polygon.
 * Edges are copied; the caller keeps ownership of both arrays.  Synchronous.
 * Returns NULL on error (hv_last_error): HV_EINVAL for a bad first[], NULL
 * pointers, host edges, or a coordinate that is not finite or outside
 * [-180, 180] x [-90, 90]; HV_ENOMEM / HV_EHIP as hv_index_build.  npoly = 0
 * gives an empty index (all masks zero).  hv_info reports kind HV_POLYGONS
 * and n = npoly. */
hv_index *hv_polygon_index_build(const double *edges, int64_t n, const int64_t *first, int64_t npoly, int flags);

/* Fill masks (SIBF, Sec. 3.2.2, Algorithm 2): pixel (i, j) is set when its
 * centre lies inside some polygon of the index, by the even-odd rule (an
 * edge counts when exactly one endpoint lies below the centre's row line, so
 * vertices on the line count once and edges parallel to x never).  tiles,
 * out_masks as for hv_render_tiles (8192 bytes per tile, same bit layout).
 * launch: region mode only (region 32 or 64; NULL = region 32 with two
 * waves per workgroup, objs_per_lane 2, cand_cap 256, at any batch size).
 * Each region's candidate polygons are those whose bounding box holds one
 * of its pixel centres not filled yet; their edges are tested in groups of up to 32
 * polygons, and only the edges of 8-edge runs whose stored bounding box can
 * cross one of the region's pixel-centre rows are read.
 * Errors as hv_render_tiles_ex, plus HV_EINVAL for an index that is not a
 * polygon index or a launch with region 0.  The distance-mask entry points
 * reject polygon indexes. */
int hv_render_fill(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, uint8_t *out_masks,
                   const hv_launch *launch);

/* Device memory a request holds while it is in a batch (the task pool's
 * admission unit, Sec. 4.2: the task pool and result pool live within a
 * memory limit): its records in the batch workspace -- the request, its
 * tile frontier of up to 256 nodes (the candidate buffer its regions start
 * from), the frontier's size, level and region bits, its work-list entries,
 * part counter and completion stamp -- plus its 8192-byte mask.  The value
 * is the library's own and follows its workspace layout.  index, tile and
 * style are validated as hv_render_batch validates a request (style may be
 * NULL for a polygon index).  Returns the bytes (> 0), or HV_EINVAL. */
int64_t hv_estimate_bytes(const hv_index *index, const hv_tile *tile, const hv_style *style);

/* Device memory of a whole batch of n_requests requests over n_indexes
 * distinct indexes: its workspace (header, index table, requests and
 * per-request records, each array aligned to 256 bytes) plus the masks.  It
 * is at most n_requests * hv_estimate_bytes(...) + 2304 + 96 * n_indexes
 * bytes.  Returns the bytes, or HV_EINVAL for a negative count or more than
 * 4096 indexes. */
int64_t hv_estimate_batch_bytes(int64_t n_requests, int32_t n_indexes);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Renders a
 * batch exactly as hv_render_batch does (same arguments, kernels and masks)
 * but calls no allocating routine: the batch's device workspace lives in a
 * static device array of the library (5 MiB on each device the library runs
 * on, held until the process ends) and its host staging in static host
 * memory.  Limits: n <= HV_NOALLOC_MAX_REQUESTS requests over at most
 * HV_NOALLOC_MAX_INDEXES distinct indexes; larger batches are rejected with
 * HV_EINVAL before any device call.  All calls on one device share that
 * array: calls are serialised on the host, and the copy of each call's
 * requests is ordered after earlier work on the calling thread's stream, so
 * consecutive calls on one stream are safe, but calls on different streams
 * of one device whose kernels overlap race on the array.  The call waits
 * until its requests have reached the device (a stream synchronisation);
 * the kernels then run asynchronously on the calling thread's stream.
 * Errors as hv_render_batch. */
#define HV_NOALLOC_MAX_REQUESTS 4096
#define HV_NOALLOC_MAX_INDEXES 16
int hv_render_batch_noalloc(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch);

/* Kernel timing for roofline figures.  Renders the batch reps times, as
 * hv_render_batch would (same arguments; launch NULL takes the tuned shape
 * or the default), each time recording HIP events on the calling thread's
 * stream before the tile-frontier kernel, between it and the query kernel,
 * and after the query kernel.  ms (host, 2 entries) receives the mean
 * duration in milliseconds of the frontier kernel (ms[0]) and of the query
 * kernel (ms[1]).  Synchronous.  HV_EINVAL for an empty batch, reps outside
 * [1, 100000] or ms NULL, before any device call. */
int hv_time_kernels(const hv_request *reqs, int64_t n, uint8_t *out_masks, const hv_launch *launch, int32_t reps,
                    double *ms);

/* Kernel timing of anti-aliased batches, for their roofline: hv_time_kernels
 * for hv_render_batch_aa (out_values as there; launch NULL takes that
 * call's default shape).  ms[0] is the frontier kernel, ms[1] the query
 * kernel: with requests in the child form (launch->aa_split), each is the
 * sum over the two sub-batches (child tiles, one pass), and the small kernel
 * that assembles the values is not counted.  Errors as hv_time_kernels. */
int hv_time_aa(const hv_request *reqs, int64_t n, uint8_t *out_values, const hv_launch *launch, int32_t reps,
               double *ms);

/* Kernel timing of polygon filling, for its roofline: hv_render_fill's
 * arguments, rendered reps times, with HIP events on the calling thread's
 * stream around the tile-frontier kernel and the fill kernel.  ms (host, 2
 * entries) receives their mean durations in milliseconds (frontier, fill).
 * Synchronous.  Errors as hv_render_fill, and HV_EINVAL for n_tiles < 1, reps
 * outside [1, 100000] or ms NULL, before any device call. */
int hv_time_fill(const hv_index *index, const hv_tile *tiles, int64_t n_tiles, uint8_t *out_masks,
                 const hv_launch *launch, int32_t reps, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* HV_H */
