// Host side of the C ABI: argument checks, the view table, the workspace
// layout and the launch sequence preprocess -> pair count -> scan -> pair
// write -> radix sort -> tile ranges -> blend (and the backward pair of
// kernels).  A single-view render is the batch of one view.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "aaa_internal.h"
#include "../../include/aaa.h"

namespace {

constexpr int kMaxViews = 256;

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(AAA_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int tiles_of(const aaa_camera *cam, int *tx, int *ty)
{
    *tx = (cam->width + aaa::kTile - 1) / aaa::kTile;
    *ty = (cam->height + aaa::kTile - 1) / aaa::kTile;
    return (*tx) * (*ty);
}

struct Shape {
    int64_t n;
    int nviews;
    int64_t total_tiles;
    int64_t total_pixels;
};

Shape shape_of(const aaa_scene *scene, int nviews, const aaa_camera *cams)
{
    Shape sh;
    sh.n = scene->n;
    sh.nviews = nviews;
    sh.total_tiles = 0;
    sh.total_pixels = 0;
    for (int v = 0; v < nviews; ++v) {
        int tx, ty;
        sh.total_tiles += tiles_of(&cams[v], &tx, &ty);
        sh.total_pixels += (int64_t)cams[v].width * cams[v].height;
    }
    return sh;
}

// Candidate tile tests a workspace can take: 8 per pair of the pair buffer
// (per 64 tests: item, keep bits, count and offset, 24 bytes).  A batch with
// more is reported as a pair overflow asking for a larger buffer.
uint64_t keep_cap_of(uint64_t max_pairs) { return ((max_pairs > 0 ? max_pairs : 1) * 8 + 63) / 64 * 64; }

struct Layout {
    size_t hdr, views, status, rect, bbox, pending, pending_n, area, area_off, rec, cull, bwd_list, keep_bits, chunk_item, chunk_cnt, kept_before, chunk_scan_tmp, scan_tmp, keys, keys_alt, vals, vals_alt, sort_tmp,
        ranges, seg_long, long_tiles, tile_order, masks, summary, n_done, n_ins, wave_caps, wave_off, wave_scan_tmp, grad_rec, total;
};

uint64_t summary_words(const Shape &sh, uint64_t mp) { return ((mp / 64 + (uint64_t)sh.total_tiles + 2) / 64 + 1) * 256; }

Layout layout(const Shape &sh, uint64_t max_pairs)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const int64_t items = sh.n * sh.nviews > 0 ? sh.n * sh.nviews : 1;
    L.hdr = take(1024);
    L.views = take(sizeof(aaa::ViewDev) * (size_t)(sh.nviews > 0 ? sh.nviews : 1));
    L.status = take(items * 4);
    L.rect = take(items * 16);
    L.bbox = take(items * 16);
    L.pending = take(items * 4);
    L.pending_n = take((items + 255) / 256 * 4);
    L.area = take(items * 4);
    L.area_off = take((items + 1) * 8);
    L.rec = take(items * 16 * aaa::kRecQuads);
    L.cull = take(items * 16 * aaa::kCullQuads);
    L.bwd_list = take(items * 4);  // K6b: the Gaussians with a visible item
    const uint64_t chunks = keep_cap_of(max_pairs) / 64;
    L.keep_bits = take(chunks * 8);
    L.chunk_item = take(chunks * 4);
    L.chunk_cnt = take(chunks * 4);
    L.kept_before = take((chunks + 1) * 8);
    L.chunk_scan_tmp = take(aaa::scan_tmp_bytes((int64_t)chunks));
    L.scan_tmp = take(aaa::scan_tmp_bytes(items));
    uint64_t mp = max_pairs > 0 ? max_pairs : 1;
    L.keys = take(mp * 8);
    L.keys_alt = take(mp * 8);
    L.vals = take(mp * 4);
    L.vals_alt = take(mp * 4);
    L.sort_tmp = take(aaa::sort_tmp_bytes(mp));
    L.ranges = take((size_t)sh.total_tiles * 4 * 8);  // per tile, or per 8x8 sub-tile with AAA_SUBTILE_SORT
    L.seg_long = take((size_t)sh.total_tiles * 8 * 4);  // the two queues of lists for the longer per-list sorts
    L.long_tiles = take((size_t)sh.total_tiles * 4);
    L.tile_order = take((size_t)sh.total_tiles * 8);  // the forward blend's tiles, longest lists first; tile keys
    L.masks = take((mp / 64 + (uint64_t)sh.total_tiles + 2) * 256 * 8);  // per-pixel masks of long lists
    L.summary = take(summary_words(sh, mp) * 8);
    L.n_done = take((size_t)sh.total_pixels * 4);
    L.n_ins = take((size_t)sh.total_pixels * 4);
    const int64_t quads = 4 * sh.total_tiles > 0 ? 4 * sh.total_tiles : 1;  // 8x8 pixel quadrants of the tiles
    L.wave_caps = take((size_t)quads * 4);
    L.wave_off = take(((size_t)quads + 1) * 8);
    L.wave_scan_tmp = take(aaa::scan_tmp_bytes(quads));
    L.grad_rec = take(items * 4 * aaa::kGradStride);
    L.total = o;
    return L;
}

int key_bits(int64_t ntiles)
{
    int b = 0;
    while ((1ll << b) < ntiles) ++b;
    return 32 + b;
}

// The pair sort runs ceil(list bits / 8) LSD passes over the high word,
// ping-ponging between the two buffers, then sorts each list in place (with
// very long lists, global passes over the whole key follow, and a copy if
// their number was odd): the result is in the buffer this parity names.
bool sorted_in_alt(int64_t ntiles) { return ((key_bits(ntiles) - 32 + 7) / 8) % 2 == 1; }

int check_camera(const aaa_camera *cam)
{
    if (cam->width <= 0 || cam->height <= 0 || cam->width > 32768 || cam->height > 32768)
        return fail(AAA_ERR_INVALID, "image size %dx%d out of range", cam->width, cam->height);
    if (!(cam->fx > 0) || !(cam->fy > 0) || !(cam->znear > 0))
        return fail(AAA_ERR_INVALID, "focal lengths and znear must be positive");
    return AAA_OK;
}

int check_common(const aaa_scene *sc, int nviews, const aaa_camera *cams, const aaa_settings *st)
{
    if (!sc || !cams || !st) return fail(AAA_ERR_INVALID, "null scene/camera/settings");
    if (nviews < 1 || nviews > kMaxViews) return fail(AAA_ERR_INVALID, "n_views %d not in 1..%d", nviews, kMaxViews);
    if (sc->n < 0 || sc->n * (int64_t)nviews >= (1ll << 32))
        return fail(AAA_ERR_INVALID, "scene size %lld x %d views out of range", (long long)sc->n, nviews);
    if (sc->sh_degree < 0 || sc->sh_degree > 3) return fail(AAA_ERR_UNSUPPORTED, "sh_degree %d not in 0..3", sc->sh_degree);
    if (sc->n > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return fail(AAA_ERR_INVALID, "null scene array");
    int64_t tiles = 0;
    for (int v = 0; v < nviews; ++v) {
        int rc = check_camera(&cams[v]);
        if (rc) return rc;
        int tx, ty;
        tiles += tiles_of(&cams[v], &tx, &ty);
    }
    if (tiles >= (1ll << 30)) return fail(AAA_ERR_INVALID, "too many tiles in the batch");
    int K = st->ray_window;
    if (!(K == 0 || K == 1 || K == 2 || K == 4 || K == 8 || K == 16 || K == 32))
        return fail(AAA_ERR_INVALID, "ray_window %d not one of 0,1,2,4,8,16,32", K);
    // alpha_max < 1 in float: the kernels blend with 1 - alpha and the
    // backward divides by it, so an opaque clamp is not representable
    if (!((float)st->alpha_min > 0 && st->alpha_min < st->alpha_max && (float)st->alpha_max < 1.0f && st->t_min >= 0 &&
          st->t_min < 1))
        return fail(AAA_ERR_INVALID, "need 0 < alpha_min < alpha_max < 1 (as float) and 0 <= t_min < 1");
    if (!(st->filter_k >= 0)) return fail(AAA_ERR_INVALID, "filter_k must be >= 0");
    return AAA_OK;
}

aaa::CamDev cam_dev(const aaa_camera *cam)
{
    aaa::CamDev c;
    c.fx = cam->fx;
    c.fy = cam->fy;
    c.cx = cam->cx;
    c.cy = cam->cy;
    c.width = cam->width;
    c.height = cam->height;
    c.tiles_x = (cam->width + aaa::kTile - 1) / aaa::kTile;
    c.tiles_y = (cam->height + aaa::kTile - 1) / aaa::kTile;
    c.znear = cam->znear;
    return c;
}

void fill_views(int nviews, const aaa_camera *cams, float *const *out_rgb, float *const *out_T,
                const float *const *dL_drgb, aaa::ViewDev *vd)
{
    int32_t tile_base = 0;
    int64_t pix_base = 0;
    for (int v = 0; v < nviews; ++v) {
        const aaa_camera *cam = &cams[v];
        aaa::ViewDev &w = vd[v];
        memset(&w, 0, sizeof w);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) w.RV[3 * r + c] = cam->viewmat[4 * r + c];
            w.tV[r] = cam->viewmat[4 * r + 3];
        }
        // camera centre o = -R_V^T t_V
        for (int r = 0; r < 3; ++r) w.o[r] = -(w.RV[r] * w.tV[0] + w.RV[3 + r] * w.tV[1] + w.RV[6 + r] * w.tV[2]);
        w.cam = cam_dev(cam);
        w.tile_base = tile_base;
        w.pix_base = pix_base;
        for (int k = 0; k < 3; ++k) w.bg[k] = (float)cam->bg[k];
        w.out_rgb = out_rgb ? out_rgb[v] : nullptr;
        w.out_T = out_T ? out_T[v] : nullptr;
        w.dL_drgb = dL_drgb ? dL_drgb[v] : nullptr;
        tile_base += w.cam.tiles_x * w.cam.tiles_y;
        pix_base += (int64_t)cam->width * cam->height;
    }
}

template <typename T>
T *at(void *ws, size_t off) { return (T *)((char *)ws + off); }

aaa::PreArgs pre_args(const aaa_scene *scene, int nviews, const aaa_settings *settings, void *ws, const Layout &L)
{
    aaa::PreArgs pa;
    pa.means = scene->means;
    pa.log_scales = scene->log_scales;
    pa.quats = scene->quats;
    pa.logits = scene->opacity_logits;
    pa.sh = scene->sh;
    pa.v_train = scene->v_train;
    pa.n = scene->n;
    pa.sh_degree = scene->sh_degree;
    pa.views = at<aaa::ViewDev>(ws, L.views);
    pa.nviews = nviews;
    pa.filter_k = settings->filter_k;
    pa.alpha_min = settings->alpha_min;
    pa.alpha_max = settings->alpha_max;
    pa.filter_mode = (settings->flags & AAA_FILTER_OFF) ? 1 : ((settings->flags & AAA_FILTER_VOLUME) ? 2 : 0);
    pa.status = at<int32_t>(ws, L.status);
    pa.rect = at<int4>(ws, L.rect);
    pa.area = at<uint32_t>(ws, L.area);
    pa.rec = at<float4>(ws, L.rec);
    pa.cull = at<float4>(ws, L.cull);
    pa.bbox = at<float4>(ws, L.bbox);
    pa.pending = at<uint32_t>(ws, L.pending);
    pa.pending_n = at<uint32_t>(ws, L.pending_n);
    return pa;
}

// Sorted values carry quadrant bits when the Gaussian index fits below them
// (and not in the ablation without tile culling, which keeps the plain 2D
// rectangle of tiles and nothing finer).
bool quad_values(int64_t n, const aaa_settings *st)
{
    return n < aaa::kQuadMaxGaussians && (st->flags & AAA_NO_TILE_CULL) == 0;
}

// The middle level of the hierarchical sort: one list per 8x8 sub-tile.
bool subtile_lists(const aaa_settings *st) { return (st->flags & AAA_SUBTILE_SORT) != 0; }

// Lists the sort keys number: tiles, or their 8x8 sub-tiles.
int64_t list_count(int64_t ntiles, const aaa_settings *st) { return subtile_lists(st) ? 4 * ntiles : ntiles; }

void set_value_bits(aaa::BlendArgs &ba, bool quads)
{
    ba.id_mask = quads ? aaa::kQuadIdMask : 0xffffffffu;
    ba.quad_on = quads ? 0u : ~aaa::kQuadIdMask;
}

}  // namespace

// Backward slots of aaa_render_backward_noalloc: one array per device, held
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels, copies and fills take the address that
// hipGetSymbolAddress returns for the current device (slot_array_address).
constexpr size_t kStaticSlotBytes = AAA_STATIC_SLOT_BYTES;
static_assert(kStaticSlotBytes == ((size_t)64 << 20), "slot array size");
static __device__ __align__(256) unsigned char scratch[kStaticSlotBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_slot_addr_mu;
void *g_slot_addr[kMaxDevices];
// calls of the allocation-free backward on one device run one at a time
std::mutex g_slot_mu[kMaxDevices];

// Device address of the static slot array on `device` (which is current),
// looked up once per device.
hipError_t slot_array_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_slot_addr_mu);
    if (!g_slot_addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_slot_addr[device] = p;
    }
    *out = g_slot_addr[device];
    return hipSuccess;
}

}  // namespace

struct aaa_ctx {
    int device;
    // pinned staging for the view table (copied to the workspace per call)
    aaa::ViewDev *views_host;
    // training-camera table of K7: pinned staging and its device copy
    aaa::TrainCam *train_host, *train_dev;
    // coherent pinned words the device publishes before the host's one wait
    // per call ([0], [1] values, [2] the call's sequence number)
    uint64_t *sync_host;
    uint64_t sync_seq;
    // second stream for the long-list blend, forked from and joined back to
    // the caller's stream with these events
    hipStream_t side;
    hipEvent_t fork, join;
    // this device's static slot array (aaa_render_backward_noalloc)
    void *slots_static;
    // AAA_TIMING: two sets of stage events (frame i uses set i % 2); a set is
    // folded into the totals once a later frame has synchronised past it.
    static constexpr int kEvents = 10;
    hipEvent_t ev[2][kEvents];
    bool pending[2];
    int cur;
    double total_ms[AAA_NUM_STAGES];
    uint64_t frames;
};

namespace {

// Publishing device words to the host: a kernel writes two words (and, with
// a note word, that word, which it then clears), then the publication's
// sequence number, into coherent pinned memory; the host spins on the number
// for up to 2 ms (a blocking stream wait adds its wake-up latency, tens of
// microseconds, to every frame) and then falls back to the blocking wait,
// which also reports stream errors.  In stream order the kernel follows
// everything enqueued before it.
hipError_t publish(aaa_ctx *c, const uint64_t *a, const uint64_t *b, hipStream_t s, uint64_t *seq,
                   uint32_t *note = nullptr)
{
    *seq = ++c->sync_seq;
    return aaa::launch_publish2(a, b, c->sync_host, *seq, note, s);
}

hipError_t wait_published(aaa_ctx *c, hipStream_t s, uint64_t seq)
{
    volatile uint64_t *flag = c->sync_host + 2;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned k = 0; *flag != seq; ++k) {
        if ((k & 255u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
            return hipStreamSynchronize(s);
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return hipSuccess;
}

hipError_t publish_and_wait(aaa_ctx *c, const uint64_t *a, const uint64_t *b, hipStream_t s)
{
    uint64_t seq = 0;
    hipError_t e = publish(c, a, b, s, &seq);
    return e != hipSuccess ? e : wait_published(c, s, seq);
}

void fold_events(aaa_ctx *c, int set)
{
    if (!c->pending[set]) return;
    hipEvent_t *e = c->ev[set];
    // e0 start | preprocess | e1 | count | e2 | scan | e3 | publish | e4 | write | e5 .. host wait .. | sort (list bits) | e6 |
    // ranges | e7 | sort (within lists) | e8 | blend | e9
    const int a[AAA_NUM_STAGES] = {0, 1, 2, 4, 5, 6, 8, 0};
    const int b[AAA_NUM_STAGES] = {1, 2, 3, 5, 6, 7, 9, 9};
    for (int k = 0; k < AAA_NUM_STAGES; ++k) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e[a[k]], e[b[k]]) == hipSuccess) c->total_ms[k] += t;
    }
    float t2 = 0.f;  // the sort's second phase
    if (hipEventElapsedTime(&t2, e[7], e[8]) == hipSuccess) c->total_ms[4] += t2;
    c->frames++;
    c->pending[set] = false;
}

}  // namespace

extern "C" {

const char *aaa_last_error(void) { return g_err.c_str(); }

const char *aaa_version(void) { return "aaa-gfx950 0.2"; }

int aaa_create(aaa_ctx **out, int device)
{
    if (!out) return fail(AAA_ERR_INVALID, "null out");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(AAA_ERR_INVALID, "device %d of %d", device, count);
    if (device >= kMaxDevices) return fail(AAA_ERR_INVALID, "device %d: at most %d devices", device, kMaxDevices);
    HIP_TRY(hipSetDevice(device));
    void *slots = nullptr;
    HIP_TRY(slot_array_address(device, &slots));
    aaa_ctx *c = new aaa_ctx;
    c->slots_static = slots;
    c->device = device;
    c->views_host = nullptr;
    c->train_host = nullptr;
    c->train_dev = nullptr;
    c->sync_host = nullptr;
    c->sync_seq = 0;
    c->side = nullptr;
    c->fork = c->join = nullptr;
    hipError_t e = hipHostMalloc((void **)&c->views_host, sizeof(aaa::ViewDev) * kMaxViews, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->train_host, sizeof(aaa::TrainCam) * AAA_MAX_TRAIN_CAMERAS, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)&c->train_dev, sizeof(aaa::TrainCam) * AAA_MAX_TRAIN_CAMERAS);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->sync_host, 64, hipHostMallocCoherent);
    if (e == hipSuccess) memset(c->sync_host, 0, 64);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->views_host) (void)hipHostFree(c->views_host);
        if (c->train_host) (void)hipHostFree(c->train_host);
        if (c->train_dev) (void)hipFree(c->train_dev);
        if (c->sync_host) (void)hipHostFree(c->sync_host);
        if (c->fork) (void)hipEventDestroy(c->fork);
        if (c->side) (void)hipStreamDestroy(c->side);
        delete c;
        return fail(AAA_ERR_HIP, "context allocation: %s", hipGetErrorString(e));
    }
    for (int s_ = 0; s_ < 2; ++s_) {
        c->pending[s_] = false;
        for (int k = 0; k < aaa_ctx::kEvents; ++k) {
            e = hipEventCreate(&c->ev[s_][k]);
            if (e != hipSuccess) {
                (void)hipHostFree(c->views_host);
                (void)hipHostFree(c->train_host);
                (void)hipFree(c->train_dev);
                (void)hipHostFree(c->sync_host);
                (void)hipEventDestroy(c->fork);
                (void)hipEventDestroy(c->join);
                (void)hipStreamDestroy(c->side);
                delete c;
                return fail(AAA_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
            }
        }
    }
    c->cur = 0;
    c->frames = 0;
    for (int k = 0; k < AAA_NUM_STAGES; ++k) c->total_ms[k] = 0.0;
    *out = c;
    return AAA_OK;
}

void aaa_destroy(aaa_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (int s_ = 0; s_ < 2; ++s_)
        for (int k = 0; k < aaa_ctx::kEvents; ++k) (void)hipEventDestroy(ctx->ev[s_][k]);
    (void)hipHostFree(ctx->views_host);
    (void)hipHostFree(ctx->train_host);
    (void)hipFree(ctx->train_dev);
    (void)hipHostFree(ctx->sync_host);
    (void)hipEventDestroy(ctx->fork);
    (void)hipEventDestroy(ctx->join);
    (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

int aaa_stage_times(aaa_ctx *ctx, double *ms, uint64_t *frames, int reset)
{
    if (!ctx || !ms || !frames) return fail(AAA_ERR_INVALID, "null argument");
    HIP_TRY(hipSetDevice(ctx->device));
    for (int k = 0; k < 2; ++k) {
        int set = (ctx->cur + k) % 2;  // oldest first
        if (ctx->pending[set]) HIP_TRY(hipEventSynchronize(ctx->ev[set][aaa_ctx::kEvents - 1]));
        fold_events(ctx, set);
    }
    for (int k = 0; k < AAA_NUM_STAGES; ++k) ms[k] = ctx->total_ms[k];
    *frames = ctx->frames;
    if (reset) {
        for (int k = 0; k < AAA_NUM_STAGES; ++k) ctx->total_ms[k] = 0.0;
        ctx->frames = 0;
    }
    return AAA_OK;
}

int aaa_workspace_size_batch(const aaa_scene *scene, int n_views, const aaa_camera *cams, const aaa_settings *settings,
                             uint64_t max_pairs, size_t *bytes_out)
{
    int rc = check_common(scene, n_views, cams, settings);
    if (rc) return rc;
    if (!bytes_out) return fail(AAA_ERR_INVALID, "null bytes_out");
    if (max_pairs >= (1ull << 32)) return fail(AAA_ERR_INVALID, "max_pairs must be < 2^32");
    *bytes_out = layout(shape_of(scene, n_views, cams), max_pairs).total;
    return AAA_OK;
}

int aaa_workspace_size(const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings, uint64_t max_pairs,
                       size_t *bytes_out)
{
    return aaa_workspace_size_batch(scene, 1, cam, settings, max_pairs, bytes_out);
}

int aaa_render_batch(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                     const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream,
                     float *const *out_rgb, float *const *out_T, aaa_stats *stats)
{
    if (!ctx) return fail(AAA_ERR_INVALID, "null context");
    int rc = check_common(scene, n_views, cams, settings);
    if (rc) return rc;
    if (max_pairs >= (1ull << 32)) return fail(AAA_ERR_INVALID, "max_pairs must be < 2^32");
    if (!ws || !out_rgb || !out_T) return fail(AAA_ERR_INVALID, "null workspace or output");
    for (int v = 0; v < n_views; ++v)
        if (!out_rgb[v] || !out_T[v]) return fail(AAA_ERR_INVALID, "null output of view %d", v);
    if (((uintptr_t)ws & 255) != 0) return fail(AAA_ERR_INVALID, "workspace must be 256-byte aligned");
    const Shape sh = shape_of(scene, n_views, cams);
    Layout L = layout(sh, max_pairs);
    if (ws_bytes < L.total) return fail(AAA_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = scene->n;
    const int64_t ntiles = sh.total_tiles;
    const bool want_stats = (settings->flags & AAA_STATS) != 0;
    unsigned long long *ctr = at<unsigned long long>(ws, L.hdr);  // [0] visible [1] tests [2] evals [3] contribs [4] near [5..7] wave steps
    const bool timing = (settings->flags & AAA_TIMING) != 0;
    hipEvent_t *ev = ctx->ev[ctx->cur];
    if (timing) {
        // the set was last used two frames ago; the previous frame's host
        // wait already ordered it, so its events are complete
        fold_events(ctx, ctx->cur);
        HIP_TRY(hipEventRecord(ev[0], s));
    }
#define STAGE_MARK(k) \
    do { if (timing) HIP_TRY(hipEventRecord(ev[k], s)); } while (0)
    // view table: pinned staging -> workspace (the previous call's copy has
    // completed: every call waits on its stream once before returning)
    fill_views(n_views, cams, out_rgb, out_T, nullptr, ctx->views_host);
    HIP_TRY(hipMemcpyAsync(at<void>(ws, L.views), ctx->views_host, sizeof(aaa::ViewDev) * n_views,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(ctr, 0, 384, s));  // counters [0..7], long-tile count [8], the sort's queue counts
                                             // [11..12], the tile order's class counts [16..47]

    aaa::PreArgs pa = pre_args(scene, n_views, settings, ws, L);
    HIP_TRY(aaa::launch_preprocess(pa, s));
    STAGE_MARK(1);

    const bool tile_cull = (settings->flags & AAA_NO_TILE_CULL) == 0;
    const int64_t items = n * n_views;
    uint64_t *area_off = at<uint64_t>(ws, L.area_off);
    uint64_t *keep_bits = at<uint64_t>(ws, L.keep_bits);
    uint32_t *chunk_item = at<uint32_t>(ws, L.chunk_item);
    uint32_t *chunk_cnt = at<uint32_t>(ws, L.chunk_cnt);
    uint64_t *kept_before = at<uint64_t>(ws, L.kept_before);
    const uint64_t keep_cap = keep_cap_of(max_pairs), chunks = keep_cap / 64;
    // candidate tests numbered by the scan of the areas, which also records
    // the item of every 64th test
    HIP_TRY(aaa::launch_exclusive_scan(pa.area, area_off, items, at<void>(ws, L.scan_tmp), s, nullptr, chunk_item,
                                       chunks));
    const bool subtile = subtile_lists(settings);
    const int64_t nlists = list_count(ntiles, settings);
    HIP_TRY(aaa::launch_count_pairs(pa.rect, pa.rec, pa.cull, area_off, items, pa.views, n_views, tile_cull,
                                    want_stats ? ctr : nullptr, keep_bits, chunk_cnt, chunk_item, keep_cap, pa.bbox,
                                    subtile, s));
    STAGE_MARK(2);
    // the chunks of this batch's C tests only (the host does not know C yet)
    HIP_TRY(aaa::launch_exclusive_scan(chunk_cnt, kept_before, (int64_t)chunks, at<void>(ws, L.chunk_scan_tmp), s,
                                       area_off + items));
    STAGE_MARK(3);
    uint64_t count_seq = 0;
    HIP_TRY(publish(ctx, kept_before + chunks, area_off + items, s, &count_seq));
    uint64_t *keys = at<uint64_t>(ws, L.keys), *keys_alt = at<uint64_t>(ws, L.keys_alt);
    uint32_t *vals = at<uint32_t>(ws, L.vals), *vals_alt = at<uint32_t>(ws, L.vals_alt);
    STAGE_MARK(4);
    // The writer needs no count from the host (a fixed grid; it stores no
    // pair at or past max_pairs and does nothing when the tests overflow
    // keep_cap), so it runs while the host waits for the count.
    const bool quads = quad_values(n, settings) && !subtile;
    HIP_TRY(aaa::launch_write_pairs(pa.rect, pa.rec, pa.cull, area_off, items, pa.views, n_views, keep_bits,
                                    chunk_item, kept_before, keep_cap, max_pairs, keys, vals, pa.bbox, quads,
                                    tile_cull, subtile, s));
    STAGE_MARK(5);
    HIP_TRY(wait_published(ctx, s, count_seq));
    uint64_t P = ctx->sync_host[0];
    const uint64_t C = ctx->sync_host[1];
    if (C > keep_cap) P = std::max<uint64_t>(max_pairs + 1, (C + 7) / 8);  // buffer too small to even count
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->pairs = P;
    }
    if (P > max_pairs) return fail(AAA_ERR_PAIR_OVERFLOW, "%llu pairs exceed max_pairs %llu", (unsigned long long)P,
                                   (unsigned long long)max_pairs);
    // Pair sort.  Phase 1: LSD passes over the list bits (the high word);
    // phase 2 (below) sorts each list by the depth word.
    bool in_alt = false;
    uint32_t *ranges = at<uint32_t>(ws, L.ranges);  // cleared by the first pass
    HIP_TRY(aaa::radix_sort_pairs(keys, vals, keys_alt, vals_alt, P, 32, key_bits(nlists), at<void>(ws, L.sort_tmp),
                                  s, &in_alt, ranges, 2 * (uint64_t)nlists));
    if (P > 1 && in_alt != sorted_in_alt(nlists)) return fail(AAA_ERR_HIP, "internal: sort parity");
    uint64_t *skeys = (P > 1 && in_alt) ? keys_alt : keys;
    uint32_t *svals = (P > 1 && in_alt) ? vals_alt : vals;
    if (P <= 1 && sorted_in_alt(nlists)) {
        // keep the invariant "sorted pairs live where sorted_in_alt says"
        HIP_TRY(hipMemcpyAsync(keys_alt, keys, P * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(vals_alt, vals, P * 4, hipMemcpyDeviceToDevice, s));
        skeys = keys_alt;
        svals = vals_alt;
    }
    STAGE_MARK(6);
    HIP_TRY(aaa::launch_tile_ranges(skeys, P, ranges, (int)nlists, s, true));
    // the blend starts the tiles with the longest lists first (sub-tile
    // lists: tile order); phase 2's filing workgroups rank the tiles by
    // length class
    uint32_t *tile_order = subtile ? nullptr : at<uint32_t>(ws, L.tile_order);
    static_assert(aaa::kOrderClasses <= 64, "class counts and starts in header words 16..79");
    const aaa::TileOrderScratch order_scratch{tile_order ? tile_order + ntiles : nullptr, (uint32_t *)(ctr + 16),
                                              (uint32_t *)(ctr + 48)};
    STAGE_MARK(7);
    // Phase 2: each list sorted by the depth word in place (the other pair
    // buffer is scratch for long lists).  Its first kernel sorts the lists
    // of up to 512 entries, queues the longer ones, notes lists longer than
    // kLongList and kSortNoteList and leaves the latter out (far views: most
    // pairs in a few lists, which one workgroup each would sort far below
    // the chip's bandwidth); it publishes the note once every list is filed,
    // while its sorts still run.  With such a list, global passes over the whole key
    // sort all pairs from the current order (stable: the order of a full
    // sort; tile boundaries, and so the ranges, are unchanged).
    uint64_t *okeys = skeys == keys ? keys_alt : keys;
    uint32_t *ovals = svals == vals ? vals_alt : vals;
    uint32_t *queues = at<uint32_t>(ws, L.seg_long), *n_queued = (uint32_t *)(ctr + 11);
    uint32_t *list_note = (uint32_t *)(ctr + 13), *list_done = list_note + 1;  // zeroed with the counters
    // the host reads the note while the short lists sort, then enqueues only
    // the tiers that have lists
    const uint64_t seq = ++ctx->sync_seq;
    HIP_TRY(aaa::launch_segment_sort_first(skeys, svals, P, ranges, nlists, queues, n_queued, list_note, list_done,
                                           aaa::SortPublish{kept_before + chunks, area_off + items, ctx->sync_host, seq},
                                           order_scratch, s));
    HIP_TRY(wait_published(ctx, s, seq));
    const uint32_t lists = P > 1 ? (uint32_t)ctx->sync_host[3] : 0u;
    if (!(lists & aaa::kNoteSortWide))
        HIP_TRY(aaa::launch_segment_sort_rest(skeys, svals, okeys, ovals, P, ranges, nlists, queues, n_queued, lists,
                                              s));
    else {
        bool moved = false;
        HIP_TRY(aaa::radix_sort_pairs(skeys, svals, okeys, ovals, P, 0, key_bits(nlists), at<void>(ws, L.sort_tmp), s,
                                      &moved));
        if (moved) {  // an odd number of passes (more than 65536 lists): back into place
            HIP_TRY(hipMemcpyAsync(skeys, okeys, P * 8, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(svals, ovals, P * 4, hipMemcpyDeviceToDevice, s));
        }
    }
    if (tile_order)
        HIP_TRY(aaa::launch_tile_order(order_scratch.tile_key, order_scratch.class_start, (int)ntiles, tile_order, s));
    STAGE_MARK(8);

    aaa::BlendArgs ba;
    ba.rec = pa.rec;
    ba.vals = svals;
    set_value_bits(ba, quads);
    ba.ranges = ranges;
    ba.quad_lists = subtile;
    ba.views = pa.views;
    ba.nviews = n_views;
    ba.total_tiles = (int)ntiles;
    ba.alpha_min = (float)settings->alpha_min;
    ba.alpha_max = (float)settings->alpha_max;
    ba.t_min = (float)settings->t_min;
    ba.n_done = at<uint32_t>(ws, L.n_done);
    ba.n_ins = at<uint32_t>(ws, L.n_ins);
    ba.counters = ctr + 2;
    ba.grad_rec = nullptr;
    ba.wave_off = nullptr;
    ba.slots = nullptr;
    ba.rank16 = false;
    ba.tile_order = tile_order;
    const int K = settings->ray_window;
    const bool long_all = (settings->flags & AAA_LONG_ALL) != 0;
    // the long-list route walks whole tiles: not with sub-tile lists
    // the long-list route needs a side stream, its own list scan and a
    // fork and join (~20 us): set up only when this call has a list that
    // long (the note of phase 2)
    ba.long_list = (K > 16 || subtile) ? 0xffffffffu
                   : long_all ? 0u
                   : (lists & aaa::kNoteLongRoute) ? aaa::kLongList
                   : 0xffffffffu;
    uint32_t *n_long = (uint32_t *)(ctr + 8);  // zeroed with the counters
    ba.n_long = n_long;
    if (ba.long_list != 0xffffffffu && P > ba.long_list) {
        // tiles with long lists render concurrently on the side stream
        uint32_t *long_tiles = at<uint32_t>(ws, L.long_tiles);
        HIP_TRY(aaa::launch_find_long(ba, long_tiles, n_long, s));
        uint64_t bound = P / ((uint64_t)ba.long_list + 1);
        if (bound > (uint64_t)ntiles) bound = (uint64_t)ntiles;
        if (bound > aaa::kMaxLongTiles) bound = aaa::kMaxLongTiles;
        const unsigned grid = (unsigned)bound;
        HIP_TRY(hipEventRecord(ctx->fork, s));
        HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->fork, 0));
        HIP_TRY(aaa::launch_blend_long(ba, K, want_stats, long_tiles, n_long, grid, at<uint64_t>(ws, L.masks),
                                       at<uint64_t>(ws, L.summary), summary_words(sh, max_pairs), ctx->side));
        HIP_TRY(hipEventRecord(ctx->join, ctx->side));
        HIP_TRY(aaa::launch_blend(ba, K, want_stats, false, s));
        HIP_TRY(hipStreamWaitEvent(s, ctx->join, 0));
    } else {
        HIP_TRY(aaa::launch_blend(ba, K, want_stats, false, s));
    }
    if (timing) {
        STAGE_MARK(9);
        ctx->pending[ctx->cur] = true;
        ctx->cur ^= 1;
    }
#undef STAGE_MARK
    if (stats && want_stats) {
        unsigned long long h[8];
        HIP_TRY(hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        stats->visible = h[0];
        stats->candidate_tiles = h[1];
        stats->evaluations = h[2];
        stats->contributors = h[3];
        stats->near = h[4];
        stats->wave_steps = h[5];
        stats->wave_near_steps = h[6];
        stats->wave_contrib_steps = h[7];
    }
    return AAA_OK;
}

int aaa_render(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings, void *ws,
               size_t ws_bytes, uint64_t max_pairs, void *stream, float *out_rgb, float *out_T, aaa_stats *stats)
{
    return aaa_render_batch(ctx, scene, 1, cam, settings, ws, ws_bytes, max_pairs, stream, &out_rgb, &out_T, stats);
}

// Slots of the backward: each 8x8 quadrant of a tile gets one row of 64
// slots (a lane each) per contributor rank of its busiest pixel, placed by an
// exclusive scan of those row counts.  *rank16: every pixel has at most 65536
// contributors (ranks 0..65535).
static int backward_slots(aaa_ctx *ctx, const Shape &sh, const Layout &L, void *ws, hipStream_t s, uint64_t *total,
                          bool *rank16 = nullptr)
{
    const int64_t quads = 4 * sh.total_tiles;
    uint32_t *max_big = (uint32_t *)(at<unsigned long long>(ws, L.hdr) + 10);
    HIP_TRY(hipMemsetAsync(max_big, 0, 4, s));
    HIP_TRY(aaa::launch_wave_caps(at<aaa::ViewDev>(ws, L.views), sh.nviews, (int)sh.total_tiles,
                                  at<uint32_t>(ws, L.n_ins), at<uint32_t>(ws, L.wave_caps), max_big, s));
    HIP_TRY(aaa::launch_exclusive_scan(at<uint32_t>(ws, L.wave_caps), at<uint64_t>(ws, L.wave_off), quads,
                                       at<void>(ws, L.wave_scan_tmp), s));
    HIP_TRY(publish_and_wait(ctx, at<uint64_t>(ws, L.wave_off) + quads, (const uint64_t *)max_big, s));
    const uint64_t rows = ctx->sync_host[0];
    const uint32_t big = (uint32_t)ctx->sync_host[1];  // the low word of the 8 bytes at max_big
    *total = rows * 64;
    if (rank16) *rank16 = big == 0;
    return AAA_OK;
}

int aaa_backward_scratch_size(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                              const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                              void *stream, size_t *bytes_out)
{
    if (!ctx || !bytes_out) return fail(AAA_ERR_INVALID, "null context or bytes_out");
    int rc = check_common(scene, n_views, cams, settings);
    if (rc) return rc;
    if (!ws) return fail(AAA_ERR_INVALID, "null workspace");
    const Shape sh = shape_of(scene, n_views, cams);
    Layout L = layout(sh, max_pairs);
    if (ws_bytes < L.total) return fail(AAA_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    HIP_TRY(hipSetDevice(ctx->device));
    uint64_t total = 0;
    rc = backward_slots(ctx, sh, L, ws, (hipStream_t)stream, &total);
    if (rc) return rc;
    *bytes_out = (size_t)total * sizeof(float2) + 256;
    return AAA_OK;
}

// Backward of the last render into `ws`.  `scratch` holds the per-contributor
// slots; with `fixed` it is the context's device's static slot array, whose
// size is checked here instead of being the caller's.
static int backward_run(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                        const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream,
                        const float *const *out_rgb, const float *const *dL_drgb, void *scratch, size_t scratch_bytes,
                        bool fixed, aaa_scene_grad *grad)
{
    if (!ctx) return fail(AAA_ERR_INVALID, "null context");
    int rc = check_common(scene, n_views, cams, settings);
    if (rc) return rc;
    if (!ws || !out_rgb || !dL_drgb || !grad) return fail(AAA_ERR_INVALID, "null workspace, image or gradient");
    for (int v = 0; v < n_views; ++v)
        if (!out_rgb[v] || !dL_drgb[v]) return fail(AAA_ERR_INVALID, "null image or gradient of view %d", v);
    const Shape sh = shape_of(scene, n_views, cams);
    Layout L = layout(sh, max_pairs);
    if (ws_bytes < L.total) return fail(AAA_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = scene->n;
    if (n == 0) return AAA_OK;
    uint64_t total = 0;
    bool rank16 = false;
    rc = backward_slots(ctx, sh, L, ws, s, &total, &rank16);
    if (rc) return rc;
    if (fixed && total * sizeof(float2) > scratch_bytes)
        return fail(AAA_ERR_WORKSPACE,
                    "this frame needs %zu bytes of backward slots; the static slot array holds %zu "
                    "(use aaa_render_backward with caller scratch)",
                    (size_t)(total * sizeof(float2)), scratch_bytes);
    if (total > 0 && (!scratch || scratch_bytes < total * sizeof(float2)))
        return fail(AAA_ERR_WORKSPACE, "backward scratch %zu < %zu bytes (aaa_backward_scratch_size)", scratch_bytes,
                    (size_t)(total * sizeof(float2)));
    const int64_t ntiles = sh.total_tiles;
    float *grad_rec = at<float>(ws, L.grad_rec);
    HIP_TRY(hipMemsetAsync(grad_rec, 0, (size_t)n * n_views * 4 * aaa::kGradStride, s));
    // the view table gains the backward's image and gradient pointers
    fill_views(n_views, cams, const_cast<float *const *>(out_rgb), nullptr, dL_drgb, ctx->views_host);
    HIP_TRY(hipMemcpyAsync(at<void>(ws, L.views), ctx->views_host, sizeof(aaa::ViewDev) * n_views,
                           hipMemcpyHostToDevice, s));
    aaa::PreArgs pa = pre_args(scene, n_views, settings, ws, L);
    const bool subtile = subtile_lists(settings);
    const bool alt = sorted_in_alt(list_count(ntiles, settings));
    aaa::BlendArgs ba;
    ba.rec = pa.rec;
    ba.vals = at<uint32_t>(ws, alt ? L.vals_alt : L.vals);
    set_value_bits(ba, quad_values(n, settings) && !subtile);
    ba.ranges = at<uint32_t>(ws, L.ranges);
    ba.quad_lists = subtile;
    ba.views = pa.views;
    ba.nviews = n_views;
    ba.total_tiles = (int)ntiles;
    ba.alpha_min = (float)settings->alpha_min;
    ba.alpha_max = (float)settings->alpha_max;
    ba.t_min = (float)settings->t_min;
    ba.n_done = at<uint32_t>(ws, L.n_done);
    ba.n_ins = at<uint32_t>(ws, L.n_ins);
    ba.counters = nullptr;
    ba.grad_rec = grad_rec;
    ba.wave_off = at<uint64_t>(ws, L.wave_off);
    ba.slots = (float2 *)scratch;
    ba.rank16 = rank16 && (settings->flags & AAA_WIDE_RANKS) == 0;
    ba.long_list = 0xffffffffu;
    ba.n_long = nullptr;
    ba.tile_order = subtile ? nullptr : at<uint32_t>(ws, L.tile_order);  // the forward's, longest lists first
    HIP_TRY(aaa::launch_blend(ba, settings->ray_window, false, true, s));  // pass 1: window replay
    HIP_TRY(aaa::launch_grad(ba, s));                                     // pass 2: list order, wave sums
    aaa::GradOut go;
    go.means = grad->means;
    go.log_scales = grad->log_scales;
    go.quats = grad->quats;
    go.logits = grad->opacity_logits;
    go.sh = grad->sh;
    // K6b over the Gaussians with a visible item (listed in bwd_list; the
    // count sits beside the frame counters)
    uint32_t *bwd_count = (uint32_t *)(at<unsigned long long>(ws, L.hdr) + 9);
    HIP_TRY(hipMemsetAsync(bwd_count, 0, 4, s));
    HIP_TRY(aaa::launch_preprocess_bwd(pa, grad_rec, go, at<uint32_t>(ws, L.bwd_list), bwd_count, s));
    // the pinned view table is reused by the next call on this context
    HIP_TRY(hipStreamSynchronize(s));
    return AAA_OK;
}

int aaa_render_backward_batch(aaa_ctx *ctx, const aaa_scene *scene, int n_views, const aaa_camera *cams,
                              const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                              void *stream, const float *const *out_rgb, const float *const *dL_drgb,
                              void *scratch, size_t scratch_bytes, aaa_scene_grad *grad)
{
    return backward_run(ctx, scene, n_views, cams, settings, ws, ws_bytes, max_pairs, stream, out_rgb, dL_drgb,
                        scratch, scratch_bytes, false, grad);
}

int aaa_render_backward_noalloc(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam,
                                const aaa_settings *settings, void *ws, size_t ws_bytes, uint64_t max_pairs,
                                void *stream, const float *out_rgb, const float *dL_drgb, aaa_scene_grad *grad)
{
    if (!ctx) return fail(AAA_ERR_INVALID, "null context");
    // one call at a time per device: every call on a device shares its array
    std::lock_guard<std::mutex> lock(g_slot_mu[ctx->device]);
    return backward_run(ctx, scene, 1, cam, settings, ws, ws_bytes, max_pairs, stream, &out_rgb, &dL_drgb,
                        ctx->slots_static, kStaticSlotBytes, true, grad);
}

int aaa_render_backward(aaa_ctx *ctx, const aaa_scene *scene, const aaa_camera *cam, const aaa_settings *settings,
                        void *ws, size_t ws_bytes, uint64_t max_pairs, void *stream, const float *out_rgb,
                        const float *dL_drgb, void *scratch, size_t scratch_bytes, aaa_scene_grad *grad)
{
    return aaa_render_backward_batch(ctx, scene, 1, cam, settings, ws, ws_bytes, max_pairs, stream, &out_rgb, &dL_drgb,
                                     scratch, scratch_bytes, grad);
}

int aaa_read_gaussians(const aaa_scene *scene, const aaa_camera *cam, uint64_t max_pairs, const void *ws,
                       size_t ws_bytes, void *stream, int32_t *status, float *alpha_t, float *tau, float *color,
                       int32_t *rect)
{
    if (!scene || !cam || !ws) return fail(AAA_ERR_INVALID, "null argument");
    Layout L = layout(shape_of(scene, 1, cam), max_pairs);
    if (ws_bytes < L.total) return fail(AAA_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = scene->n;
    if (n == 0) return AAA_OK;
    const char *w = (const char *)ws;
    if (status) HIP_TRY(hipMemcpyAsync(status, w + L.status, n * 4, hipMemcpyDeviceToDevice, s));
    // strided fields of the records: rec[i].q5.w = alpha~, rec[i].q6.y = tau, rec[i].q7.xyz = colour
    const size_t stride = 16 * aaa::kRecQuads;
    if (alpha_t) HIP_TRY(hipMemcpy2DAsync(alpha_t, 4, w + L.rec + 5 * 16 + 12, stride, 4, n, hipMemcpyDeviceToDevice, s));
    if (tau) HIP_TRY(hipMemcpy2DAsync(tau, 4, w + L.rec + 6 * 16 + 4, stride, 4, n, hipMemcpyDeviceToDevice, s));
    if (color)
        for (int c = 0; c < 3; ++c)
            HIP_TRY(hipMemcpy2DAsync(color + c * n, 4, w + L.rec + 7 * 16 + 4 * c, stride, 4, n,
                                     hipMemcpyDeviceToDevice, s));
    if (rect)
        for (int c = 0; c < 4; ++c)
            HIP_TRY(hipMemcpy2DAsync(rect + c * n, 4, w + L.rect + 4 * c, 16, 4, n, hipMemcpyDeviceToDevice, s));
    return AAA_OK;
}

int aaa_read_pairs(const aaa_scene *scene, const aaa_camera *cam, uint64_t max_pairs, const void *ws, size_t ws_bytes,
                   void *stream, uint64_t *keys, uint32_t *values, uint32_t *ranges, uint64_t cap, uint64_t *n_pairs)
{
    if (!scene || !cam || !ws || !n_pairs) return fail(AAA_ERR_INVALID, "null argument");
    const Shape sh = shape_of(scene, 1, cam);
    Layout L = layout(sh, max_pairs);
    if (ws_bytes < L.total) return fail(AAA_ERR_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    const char *w = (const char *)ws;
    uint64_t P = 0;
    HIP_TRY(hipMemcpyAsync(&P, w + L.kept_before + 8 * (keep_cap_of(max_pairs) / 64), 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_pairs = P;
    if (P > max_pairs) return fail(AAA_ERR_PAIR_OVERFLOW, "last frame overflowed");
    if (P > cap) return fail(AAA_ERR_INVALID, "cap %llu < %llu pairs", (unsigned long long)cap, (unsigned long long)P);
    const bool alt = sorted_in_alt(sh.total_tiles);
    if (keys && P) HIP_TRY(hipMemcpyAsync(keys, w + (alt ? L.keys_alt : L.keys), P * 8, hipMemcpyDeviceToDevice, s));
    if (values && P) {
        HIP_TRY(hipMemcpyAsync(values, w + (alt ? L.vals_alt : L.vals), P * 4, hipMemcpyDeviceToDevice, s));
        // indices only (below 2^28 the mask also clears any quadrant bits)
        if (scene->n < aaa::kQuadMaxGaussians) HIP_TRY(aaa::launch_and_u32(values, P, aaa::kQuadIdMask, s));
    }
    if (ranges) HIP_TRY(hipMemcpyAsync(ranges, w + L.ranges, (size_t)sh.total_tiles * 8, hipMemcpyDeviceToDevice, s));
    return AAA_OK;
}

int aaa_sort_tmp_size(uint64_t n, size_t *bytes_out)
{
    if (!bytes_out) return fail(AAA_ERR_INVALID, "null bytes_out");
    if (n >= (1ull << 32)) return fail(AAA_ERR_INVALID, "n must be < 2^32");
    *bytes_out = align256(n * 8) + align256(n * 4) + align256(aaa::sort_tmp_bytes(n > 0 ? n : 1));
    return AAA_OK;
}

int aaa_sort_pairs(uint64_t *keys, uint32_t *values, uint64_t n, int key_bits_, void *tmp, size_t tmp_bytes, void *stream)
{
    if (n >= (1ull << 32)) return fail(AAA_ERR_INVALID, "n must be < 2^32");
    if (key_bits_ < 1 || key_bits_ > 64) return fail(AAA_ERR_INVALID, "key_bits %d not in 1..64", key_bits_);
    size_t need = 0;
    aaa_sort_tmp_size(n, &need);
    if (n > 0 && (!keys || !values || !tmp)) return fail(AAA_ERR_INVALID, "null argument");
    if (tmp_bytes < need) return fail(AAA_ERR_WORKSPACE, "tmp %zu < %zu bytes", tmp_bytes, need);
    if (((uintptr_t)tmp & 255) != 0) return fail(AAA_ERR_INVALID, "tmp must be 256-byte aligned");
    if (n <= 1) return AAA_OK;
    hipStream_t s = (hipStream_t)stream;
    char *t = (char *)tmp;
    uint64_t *ka = (uint64_t *)t;
    uint32_t *va = (uint32_t *)(t + align256(n * 8));
    void *st = t + align256(n * 8) + align256(n * 4);
    bool in_alt = false;
    HIP_TRY(aaa::radix_sort_pairs(keys, values, ka, va, n, 0, key_bits_, st, s, &in_alt));
    if (in_alt) {
        HIP_TRY(hipMemcpyAsync(keys, ka, n * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(values, va, n * 4, hipMemcpyDeviceToDevice, s));
    }
    return AAA_OK;
}

}  // extern "C"

int aaa_training_frequency(aaa_ctx *ctx, const float *means, int64_t n, const aaa_camera *cams, int n_cams,
                           void *stream, float *v_train)
{
    if (!ctx || (n > 0 && (!means || !v_train)) || (n_cams > 0 && !cams))
        return fail(AAA_ERR_INVALID, "null context, means, cameras or output");
    if (n < 0) return fail(AAA_ERR_INVALID, "n must be >= 0");
    if (n_cams < 0 || n_cams > AAA_MAX_TRAIN_CAMERAS)
        return fail(AAA_ERR_INVALID, "n_cams %d not in 0..%d", n_cams, AAA_MAX_TRAIN_CAMERAS);
    for (int c = 0; c < n_cams; ++c) {
        int rc = check_camera(&cams[c]);
        if (rc) return rc;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    for (int c = 0; c < n_cams; ++c) {
        aaa::TrainCam &t = ctx->train_host[c];
        for (int k = 0; k < 12; ++k) t.V[k] = cams[c].viewmat[k];
        t.fx = cams[c].fx;
        t.fy = cams[c].fy;
        t.cx = cams[c].cx;
        t.cy = cams[c].cy;
        t.w = (double)cams[c].width;
        t.h = (double)cams[c].height;
        t.znear = cams[c].znear;
    }
    if (n_cams > 0)
        HIP_TRY(hipMemcpyAsync(ctx->train_dev, ctx->train_host, sizeof(aaa::TrainCam) * n_cams, hipMemcpyHostToDevice, s));
    HIP_TRY(aaa::launch_train_freq(means, n, ctx->train_dev, n_cams, v_train, s));
    // the pinned staging is reused by the next call
    HIP_TRY(hipStreamSynchronize(s));
    return AAA_OK;
}

int aaa_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int64_t step, double lr, double beta1,
                  double beta2, double eps, void *stream)
{
    if (n < 0) return fail(AAA_ERR_INVALID, "n must be >= 0");
    if (n > 0 && (!param || !grad || !m || !v)) return fail(AAA_ERR_INVALID, "null array");
    if (step < 1) return fail(AAA_ERR_INVALID, "step must be >= 1");
    if (!(beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
        return fail(AAA_ERR_INVALID, "need 0 <= beta1, beta2 < 1 and eps > 0");
    const double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
    HIP_TRY(aaa::launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
    return AAA_OK;
}
