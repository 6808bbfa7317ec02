// lens_runtime.cpp -- host runtime behind include/lens_api.h.
//
// Context, resident lens registry with HBM-budget accounting, per-stream
// scratch, the blocking and device-buffer likelihood calls, the multi-lens
// call, and the serving scheduler (continuous batching of proposal tiles from
// many concurrent requests onto several HIP streams).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lens_api.h"
#include "lens_internal.h"

using lensk::LensGeom;

namespace {

constexpr size_t kAlign = 256;
constexpr int kServeStreams = 2;            // serving batches alternate over these streams
constexpr size_t kLatencyWindow = 4096;   // completed requests kept for the latency quantiles
// Serving batches: the work of many requests on many lenses in one prep step
// and one persistent launch per lens group.  At most kServeDepth batches are
// in flight, so the next one is queued on the device while the last one's
// tail drains.  A batch holds at most kBatchMax proposals from at most
// kBatchPieces request pieces, and stops taking work past kBatchWork sub-pixel
// evaluations (about 10 ms of the device at ~2e11 evaluations/s): large
// enough that the launch tail is a small share, small enough that a request
// arriving behind a full batch waits about that long.
constexpr int kServeDepth = 2;
constexpr int64_t kBatchMax = 32768;
constexpr int kBatchPieces = 256;
constexpr double kBatchWork = 2.0e9;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Lens {
    lens_id id = 0;
    LensGeom g{};
    int precision = 0;
    int amplitudes = 0;     // LENS_AMP_*
    int light_model = 0;    // LENS_LIGHT_*
    int mass_model = 0;     // LENS_MASS_*
    int prep_code = 0;      // the prep step's model code: light model | mass << kMassShift
    int64_t masked = 0, needed = 0;
    int psf_given = 0;      // PSF side as loaded (g.k is the side after the tail crop)
    void *slab = nullptr;   // one device allocation holding every array
    size_t bytes = 0;
    int users = 0;          // blocking calls in progress
    int requests = 0;       // serving requests queued or running
};

// Per-stream device scratch.  Its mutex is held from the moment a call takes
// the buffer until that call has enqueued every launch that uses it, so that
// calls sharing a stream neither interleave their launches on one buffer nor
// free it under each other (a grow drains the stream first).
struct Scratch {
    std::mutex mu;
    void *p = nullptr;
    size_t bytes = 0;
};

enum class RState { Queued, Running, Done, Error, Canceled };

struct Request {
    lens_req id = 0;
    Lens *lens = nullptr;
    int64_t n = 0;
    std::vector<double> params;   // host copy taken at submit
    double *out = nullptr;        // caller's buffer
    RState state = RState::Queued;
    lens_status status = LENS_PENDING;
    int64_t next_tile = 0;        // first proposal not yet placed in a batch
    int64_t done = 0;             // proposals finished
    int tiles_running = 0;        // pieces in batches on the device
    bool resident = false;        // has had work on the device (counts against max_inflight)
    bool cancel = false;
    std::vector<double> result;   // assembled here, copied to out when complete
    std::chrono::steady_clock::time_point t_submit;
};

// A contiguous range of one request's proposals inside a serving batch.
struct Piece {
    Request *req = nullptr;
    int64_t off = 0, n = 0;       // request proposals [off, off + n)
    int64_t at = 0;               // pooled position in the batch
};

// One serving batch in flight: its pieces, its slot of the serving buffers
// and the event recorded behind its result copy.
struct SBatch {
    std::vector<Piece> pieces;
    int slot = 0;
    int64_t n = 0;
    hipEvent_t ev = nullptr;
};

thread_local std::unordered_map<const void *, std::string> t_err;

// One multi-lens call shape (lens ids and proposal counts) captured as a
// hipGraph: H2D params -> prep -> one persistent launch per (mode, workgroup
// size) group -> D2H results.  Replayed for every call with the same shape.
struct Ensemble;   // a sampler ensemble (defined with its entry points)

struct Plan {
    std::vector<lens_id> ids;
    std::vector<int64_t> counts;
    int64_t tot = 0;
    void *dev = nullptr;
    size_t bytes = 0;
    double *h_params = nullptr, *h_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
    // the same sequence without a graph: used when the capture was invalidated
    // by another thread (an operation on the legacy default stream while it ran)
    std::function<hipError_t(hipStream_t)> eager;
};

// One multi-lens call shape of the device-buffer entry point: the launch
// groups and their read-only device tables (lens descriptors, item starts,
// output offsets, and the per-lens prep model table when models differ).  The
// prepared constants and the work counters live in the caller stream's
// scratch.  Created and dropped under sync_mu; dropped only after the device
// has drained, since launches on callers' streams may still read the tables.
struct DPlan;

// round-to-nearest-even FP32 -> BF16 and back
uint16_t bf16_rn_host(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_to_float(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// round-to-nearest-even FP32 -> IEEE half (subnormals kept) and back
uint16_t f16_rn_host(float f)
{
    const _Float16 h = (_Float16)f;
    uint16_t u;
    memcpy(&u, &h, 2);
    return u;
}

float f16_to_float(uint16_t u)
{
    _Float16 h;
    memcpy(&h, &u, 2);
    return (float)h;
}

// The flipped PSF Kf[a][b] = K[k-1-a][k-1-b], times scale (a power of two),
// as npl 16-bit planes per tap ([k*k][npl]; BF16, or IEEE half if f16), each
// plane the nearest value to what the earlier ones leave of the FP32 tap,
// except that the last plane of some taps is rounded to its other neighbour so
// that the planes sum, over the whole kernel, to the FP64 sum of scale K.  The kernel's rounding would otherwise scale every model pixel by
// a common factor 1 + sum(K - planes)/sum(K), off by up to ~2^-17 for two
// planes, an error that the chi-square does not average away.  Taps are
// flipped in the order of the least added error, each only when that brings
// the residual sum closer to zero; no tap's error exceeds one unit of its last
// plane.
std::vector<uint16_t> split_psf_planes(const double *psf, int k, int npl, bool f16 = false, double scale = 1.0)
{
    uint16_t (*rn)(float) = f16 ? f16_rn_host : bf16_rn_host;
    float (*val)(uint16_t) = f16 ? f16_to_float : bf16_to_float;
    const int n = k * k;
    std::vector<uint16_t> out((size_t)n * npl);
    std::vector<double> e(n), ealt(n);
    std::vector<uint16_t> alt(n);
    double E = 0.0;
    for (int t = 0; t < n; ++t) {
        const int a = t / k, b = t % k;
        const double K = scale * psf[(size_t)(k - 1 - a) * k + (k - 1 - b)];
        float v = (float)K;
        double sum = 0.0;
        for (int q = 0; q < npl; ++q) {
            const uint16_t h = rn(v);
            out[(size_t)t * npl + q] = h;
            if (q + 1 < npl) v -= val(h);   // exact: v and its nearest 16-bit value share the leading bits
            sum += (double)val(h);
        }
        e[t] = K - sum;
        E += e[t];
        // the other 16-bit neighbour of the last plane's target v
        const uint16_t h = out[(size_t)t * npl + npl - 1];
        const float fh = val(h);
        alt[t] = h;
        ealt[t] = e[t];
        if (v != 0.0f && fh != 0.0f && std::isfinite(fh) && fh != v) {
            // one unit towards v: +1 in the magnitude bits moves away from 0 (both formats)
            const bool up_mag = std::fabs(v) > std::fabs(fh);
            const uint16_t o = up_mag ? (uint16_t)(h + 1) : (uint16_t)(h - 1);
            const float fo = val(o);
            if (std::isfinite(fo) && (fo > 0.0f) == (fh > 0.0f)) {
                alt[t] = o;
                ealt[t] = e[t] + (double)fh - (double)fo;
            }
        }
    }
    std::vector<int> order(n);
    for (int t = 0; t < n; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::fabs(ealt[x]) - std::fabs(e[x]) < std::fabs(ealt[y]) - std::fabs(e[y]);
    });
    for (int t : order) {
        if (alt[t] == out[(size_t)t * npl + npl - 1]) continue;
        const double E2 = E - e[t] + ealt[t];
        if (std::fabs(E2) < std::fabs(E)) {
            out[(size_t)t * npl + npl - 1] = alt[t];
            E = E2;
        }
    }
    return out;
}

// Strip height H and workgroup size of one lens: the LDS ring holds H + k - 1
// binned rows.  False if even H = 1 does not fit.
bool set_tiles(LensGeom &g, int H, int nt, size_t lds_max)
{
    if (H < 1) return false;
    H = std::min(H, g.ny);
    const size_t bytes = (size_t)(H + 2 * g.r) * lensk::ring_row_bytes(g.mode, g.k, g.span);
    if (bytes > lds_max) return false;
    if (lensk::mode_base(g.mode) == lensk::MODE_SPLIT && H + 2 * g.r > lensk::kRingRowsMax) return false;
    g.nt = nt;
    g.strip_h = H;
    g.ring_rows = H + 2 * g.r;
    g.plane = g.ring_rows * g.ring_w;
    g.nstrips = (g.ny + H - 1) / H;
    return true;
}

// Default shape, from full-batch timings on MI355X:
// - FP32 convolution whose ring for 16-row strips fits a quarter of a CU's LDS:
//   256 threads, 16 rows (the most resident workgroups);
// - otherwise 512 threads and the tallest strip of min(32, ny), 16, 8 or 4 rows
//   whose ring lets two workgroups share a CU (powers of two keep the MFMA
//   convolution's 16-segment tiles spread evenly over the 8 waves);
// - failing that, the tallest strip that fits one workgroup's LDS.
// Each resident workgroup also holds its kernel's static LDS (the SIE
// deflection table and the reduction slots).
int default_strip(const LensGeom &g, size_t lds_max, size_t lds_cu, int *nt)
{
    const size_t row_b = lensk::ring_row_bytes(g.mode, g.k, g.span);
    const auto ring = [&](int H) { return (size_t)(H + 2 * g.r) * row_b; };
    const auto share = [&](size_t n, int threads) {
        const size_t st = lensk::batch_static_lds(g.mode, threads);
        return lds_cu / n > st ? lds_cu / n - st : 0;
    };
    if (lensk::mode_base(g.mode) == lensk::MODE_FP32 && ring(std::min(16, g.ny)) <= std::min(lds_max, share(4, 256))) {
        *nt = 256;
        return std::min(16, g.ny);
    }
    *nt = 512;
    const size_t half = std::min(lds_max, share(2, 512));
    for (int H : {std::min(32, g.ny), 16, 8, 4})
        if (H <= g.ny && ring(H) <= half) return H;
    for (int H = std::min(32, g.ny); H >= 1; --H)
        if (ring(H) <= lds_max) return H;
    return 0;
}

}  // namespace

struct lens_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    lens_dev_alloc_fn alloc = nullptr;
    lens_dev_free_fn dfree = nullptr;
    void *user = nullptr;
    int64_t budget = 0;
    size_t lds_max = 65536;               // dynamic LDS one workgroup may use
    size_t lds_cu = 65536;                // LDS of one compute unit
    std::atomic<int64_t> used{0};
    std::atomic<int> dev_error{0};

    std::mutex mu;                        // registry, scratch, budget
    std::map<lens_id, Lens *> lenses;
    lens_id next_id = 1;
    std::unordered_map<hipStream_t, std::unique_ptr<Scratch>> scratch;

    std::mutex sync_mu;                   // staging of the blocking calls
    double *h_params = nullptr, *h_out = nullptr;
    size_t h_cap = 0;                     // proposals
    void *d_sync = nullptr;               // params | pc | out for the blocking calls
    size_t d_sync_bytes = 0;

    // autotuner: (strip height, workgroup size) per shape bucket
    bool autotune = false;
    std::mutex tune_mu;
    std::map<std::string, std::pair<int, int>> tune_cache;
    std::string tune_file;
    int num_cus = 256;

    // sampler ensembles (registry guarded by mu; each ensemble by its own mutex)
    std::map<int64_t, Ensemble *> ensembles;
    int64_t next_ens = 1;

    // multi-lens plans (graph-captured persistent launches), guarded by sync_mu
    std::map<std::string, struct Plan *> plans;
    uint64_t plan_clock = 0;
    // multi-lens shapes of the device-buffer entry point, guarded by sync_mu
    std::map<std::string, struct DPlan *> dplans;

    // serving
    int max_inflight = 64;
    bool nonblocking = false;
    std::mutex smu;
    std::condition_variable scv;          // wakes the scheduler
    std::condition_variable dcv;          // request finished
    std::deque<Request *> queue;          // requests with tiles still to launch
    std::map<lens_req, Request *> reqs;
    lens_req next_req = 1;
    std::vector<SBatch> running;          // batches in flight
    int resident = 0;                     // requests with work placed on the device, not finished
    bool slot_busy[kServeDepth] = {};
    void *d_serve = nullptr;              // kServeDepth slots: tables | params | prep | out
    char *h_serve = nullptr;              // kServeDepth slots: tables | params | out (pinned)
    hipStream_t sstreams[kServeStreams] = {};
    // batch-plan capture, under sync_mu only: no other thread enqueues on a
    // stream while it is being captured
    hipStream_t cap_stream = nullptr;
    std::thread sched;
    bool stop = false;
    lens_stats stats{};
    // latencies (us) of the most recent completed requests, a ring (guarded by smu)
    std::vector<double> lat_ring;
    size_t lat_pos = 0;
    int log = 0;                          // LENS_LOG at init: 1 = one stderr line per event
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// One line to stderr when the context was created with LENS_LOG=1.
void log_line(const lens_ctx *c, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void log_line(const lens_ctx *c, const char *fmt, ...)
{
    if (!c || !c->log) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fprintf(stderr, "[lens %p] %s\n", (const void *)c, buf);
}

lens_status fail(lens_ctx *c, lens_status st, const std::string &msg)
{
    t_err[c] = msg;
    log_line(c, "error %d (%s): %s", (int)st, lens_strerror(st), msg.c_str());
    return st;
}

lens_status hip_fail(lens_ctx *c, hipError_t e, const char *what)
{
    c->dev_error.store(1);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    return fail(c, LENS_EDEVICE, buf);
}

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
    } while (0)

void *dev_alloc(lens_ctx *c, size_t bytes)
{
    if (c->alloc) return c->alloc(bytes, (void *)c->stream, c->user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(lens_ctx *c, void *p)
{
    if (!p) return;
    if (c->dfree) c->dfree(p, (void *)c->stream, c->user);
    else (void)hipFree(p);
}

bool charge(lens_ctx *c, int64_t bytes)
{
    int64_t cur = c->used.load();
    while (true) {
        if (cur + bytes > c->budget) return false;
        if (c->used.compare_exchange_weak(cur, cur + bytes)) return true;
    }
}

void uncharge(lens_ctx *c, int64_t bytes) { c->used.fetch_sub(bytes); }

Lens *acquire(lens_ctx *c, lens_id id)
{
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->lenses.find(id);
    if (it == c->lenses.end()) return nullptr;
    it->second->users++;
    return it->second;
}

void release(lens_ctx *c, Lens *L)
{
    std::lock_guard<std::mutex> lk(c->mu);
    L->users--;
}

lens_status check_ctx(lens_ctx *c)
{
    if (!c) return LENS_EINVAL;
    if (c->dev_error.load()) return fail(c, LENS_EDEVICE, "context is in the device-error state");
    return LENS_OK;
}

// Device scratch of at least `bytes` private to `stream` (grown by re-allocation
// after the stream has drained).  On return `hold` owns the buffer's lock: keep
// it until every launch that uses the buffer has been enqueued.
lens_status stream_scratch(lens_ctx *c, hipStream_t st, size_t bytes, void **out, std::unique_lock<std::mutex> *hold)
{
    Scratch *sp = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        std::unique_ptr<Scratch> &e = c->scratch[st];
        if (!e) e.reset(new Scratch());
        sp = e.get();
    }
    *hold = std::unique_lock<std::mutex>(sp->mu);
    Scratch &s = *sp;
    if (s.bytes >= bytes) {
        *out = s.p;
        return LENS_OK;
    }
    size_t want = align_up(std::max(bytes, s.bytes * 3 / 2), 1 << 20);
    if (s.p) {
        HIPCHK(c, hipStreamSynchronize(st));
        dev_free(c, s.p);
        uncharge(c, (int64_t)s.bytes);
        s.p = nullptr;
        s.bytes = 0;
    }
    if (!charge(c, (int64_t)want)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (scratch)");
    s.p = dev_alloc(c, want);
    if (!s.p) {
        uncharge(c, (int64_t)want);
        return fail(c, LENS_ENOMEM, "device allocation failed (scratch)");
    }
    s.bytes = want;
    *out = s.p;
    return LENS_OK;
}

struct ScratchLayout {
    double *params;
    lensk::PropBlock *pc;
    double *out;
    double *amp;   // [n][N] solved amplitudes (N <= 4), right after out
};

size_t scratch_bytes(int64_t n, bool with_params_out)
{
    size_t b = align_up((size_t)n * lensk::kPCBytes, kAlign);
    if (with_params_out)
        b += align_up((size_t)n * lensk::kStride * sizeof(double), kAlign) + align_up((size_t)n * 5 * sizeof(double), kAlign);
    return b;
}

ScratchLayout carve(void *base, int64_t n, bool with_params_out)
{
    ScratchLayout L{};
    char *p = (char *)base;
    L.pc = (lensk::PropBlock *)p;
    p += align_up((size_t)n * lensk::kPCBytes, kAlign);
    if (with_params_out) {
        L.params = (double *)p;
        p += align_up((size_t)n * lensk::kStride * sizeof(double), kAlign);
        L.out = (double *)p;
        L.amp = L.out + n;
    }
    return L;
}

hipError_t launch_lens(const Lens *L, const double *d_params, lensk::PropBlock *d_pc, int64_t n, double *d_out,
                       hipStream_t st, double *d_amp = nullptr)
{
    hipError_t e = lensk::launch_prep(d_params, n, d_pc, L->prep_code, nullptr, nullptr, 0, st);
    if (e != hipSuccess) return e;
    return lensk::launch_loglike(L->g, d_pc, n, d_out, d_amp, st);
}

// A walker ensemble resident on the device (lens_ensemble_*).  It holds a
// user reference on its lens until destroyed.
struct Ensemble {
    int64_t id = 0;
    Lens *L = nullptr;
    int W = 0, d = 0;             // walkers, free slots
    double a = 2.0;               // stretch scale
    uint64_t seed = 0;
    int64_t t = 0;                // iterations done
    void *slab = nullptr;         // lo | hi | walkers | lnp | accepted | Y | aux | pc | out
    size_t bytes = 0;
    double *lo = nullptr, *hi = nullptr, *walkers = nullptr, *lnp = nullptr, *Y = nullptr, *aux = nullptr,
           *out = nullptr;
    int64_t *accepted = nullptr;
    lensk::PropBlock *pc = nullptr;
    std::mutex mu;                // one call on an ensemble at a time
    int users = 0;                // calls in progress (guarded by the context's mu)
};

void scheduler_main(lens_ctx *c);
lens_status tune_lens(lens_ctx *c, Lens *L);
void drop_plan(lens_ctx *c, Plan *pl);
void drop_dplan(lens_ctx *c, DPlan *pl);
bool dplan_uses(const DPlan *pl, lens_id id);
void free_dplan_now(lens_ctx *c, DPlan *pl);

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" lens_status lens_init(const lens_init_opts *opts, lens_ctx **out)
{
    if (!out) return LENS_EINVAL;
    *out = nullptr;
    lens_init_opts o{};
    if (opts) o = *opts;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return LENS_EDEVICE;
    if (o.device < 0 || o.device >= ndev) return LENS_EINVAL;
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr)) return LENS_EINVAL;
    auto c = std::make_unique<lens_ctx>();
    c->device = o.device;
    {
        const char *lg = getenv("LENS_LOG");
        c->log = lg && atoi(lg) > 0;
    }
    DeviceGuard dg(c->device);
    c->alloc = o.dev_alloc;
    c->dfree = o.dev_free;
    c->user = o.alloc_user;
    size_t fre = 0, tot = 0;
    if (hipMemGetInfo(&fre, &tot) != hipSuccess) return LENS_EDEVICE;
    c->budget = o.hbm_budget_bytes > 0 ? o.hbm_budget_bytes : (int64_t)(fre * 0.9);
    c->max_inflight = o.max_inflight > 0 ? o.max_inflight : 64;
    c->nonblocking = o.nonblocking_submit != 0;
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return LENS_EDEVICE;
        c->own_stream = true;
    }
    for (int i = 0; i < kServeStreams; ++i)
        if (hipStreamCreateWithFlags(&c->sstreams[i], hipStreamNonBlocking) != hipSuccess) return LENS_EDEVICE;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) return LENS_EDEVICE;
    // the allocation-free entry point's fixed scratch on this device
    if (lensk::noalloc_init(c->device) != hipSuccess) return LENS_EDEVICE;
    c->stats.hbm_budget_bytes = c->budget;
    c->autotune = o.autotune != 0;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->num_cus = cus;
        const char *tf = getenv("LENS_AUTOTUNE_CACHE");
        if (tf && *tf) {
            c->tune_file = tf;
            FILE *f = fopen(tf, "r");
            if (f) {
                char key[256];
                int H = 0, nt = 0;
                while (fscanf(f, "%255s %d %d", key, &H, &nt) == 3) c->tune_cache[key] = {H, nt};
                fclose(f);
            }
        }
    }
    {
        const size_t m = lensk::max_lds_bytes();
        const size_t u = m > 65536 ? lensk::set_lds_limits(m) : 0;
        if (u > 65536) c->lds_max = u;
        (void)hipGetLastError();
        c->lds_cu = lensk::lds_per_cu();
    }
    lens_ctx *raw = c.release();
    log_line(raw, "init: device %d, %d CUs, %zu B of LDS per workgroup, HBM budget %lld B, %s stream", raw->device,
             raw->num_cus, raw->lds_max, (long long)raw->budget, raw->own_stream ? "own" : "caller's");
    raw->sched = std::thread(scheduler_main, raw);
    *out = raw;
    return LENS_OK;
}

extern "C" void lens_shutdown(lens_ctx *c)
{
    if (!c) return;
    log_line(c, "shutdown");
    {
        std::unique_lock<std::mutex> lk(c->smu);
        for (Request *r : c->queue) {
            if (r->tiles_running == 0 && r->state == RState::Queued) {
                r->state = RState::Canceled;
                r->status = LENS_ECANCELED;
            }
            r->cancel = true;
        }
        c->stop = true;
    }
    c->scv.notify_all();
    if (c->sched.joinable()) c->sched.join();
    DeviceGuard dg(c->device);
    // device-buffer calls may still run on callers' streams and read lenses,
    // plans and scratch freed below
    (void)hipDeviceSynchronize();
    for (int i = 0; i < kServeStreams; ++i)
        if (c->sstreams[i]) {
            (void)hipStreamSynchronize(c->sstreams[i]);
            (void)hipStreamDestroy(c->sstreams[i]);
        }
    if (c->cap_stream) {
        (void)hipStreamSynchronize(c->cap_stream);
        (void)hipStreamDestroy(c->cap_stream);
    }
    for (auto &kv : c->plans) {
        Plan *pl = kv.second;
        if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
        if (pl->graph) (void)hipGraphDestroy(pl->graph);
        dev_free(c, pl->dev);
        if (pl->h_params) (void)hipHostFree(pl->h_params);
        if (pl->h_out) (void)hipHostFree(pl->h_out);
        delete pl;
    }
    c->plans.clear();
    for (auto &kv : c->dplans) free_dplan_now(c, kv.second);
    c->dplans.clear();
    for (auto &kv : c->reqs) delete kv.second;
    c->reqs.clear();
    for (auto &kv : c->ensembles) {
        dev_free(c, kv.second->slab);
        delete kv.second;
    }
    c->ensembles.clear();
    for (auto &kv : c->lenses) {
        dev_free(c, kv.second->slab);
        delete kv.second;
    }
    c->lenses.clear();
    for (auto &kv : c->scratch) dev_free(c, kv.second->p);
    c->scratch.clear();
    if (c->d_sync) dev_free(c, c->d_sync);
    if (c->d_serve) dev_free(c, c->d_serve);
    if (c->h_params) (void)hipHostFree(c->h_params);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->h_serve) (void)hipHostFree(c->h_serve);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    t_err.erase(c);
    delete c;
}

extern "C" const char *lens_strerror(lens_status st)
{
    switch (st) {
    case LENS_OK: return "ok";
    case LENS_PENDING: return "pending";
    case LENS_EINVAL: return "invalid argument";
    case LENS_ENOMEM: return "out of device memory or HBM budget";
    case LENS_ENOENT: return "no such lens or request";
    case LENS_EBUSY: return "lens has requests in flight";
    case LENS_EAGAIN: return "no free slot, try again";
    case LENS_EDEVICE: return "HIP device error";
    case LENS_ECANCELED: return "request cancelled";
    case LENS_ETIMEDOUT: return "timed out";
    default: return "unknown status";
    }
}

extern "C" const char *lens_last_error(lens_ctx *c)
{
    auto it = t_err.find(c);
    return it == t_err.end() ? "" : it->second.c_str();
}


// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

std::string shape_key(const LensGeom &g, int64_t needed)
{
    char buf[160];
    // needed pixels in steps of 1/8 of the image: the mask's share of the work
    snprintf(buf, sizeof(buf), "gfx950/m%d/k%d/s%d/y%d/x%d/f%d", g.mode, g.k, g.s, (g.ny + 15) / 16,
             (g.nx + 15) / 16, (int)(8 * needed / std::max<int64_t>(1, (int64_t)g.ny * g.nx)));
    return buf;
}

// Times each candidate (strip height, workgroup size) on synthetic proposals
// of typical shape and keeps the fastest for the lens's shape bucket.
lens_status tune_lens(lens_ctx *c, Lens *L)
{
    const std::string key = shape_key(L->g, L->needed);
    {
        std::lock_guard<std::mutex> lk(c->tune_mu);
        auto it = c->tune_cache.find(key);
        if (it != c->tune_cache.end()) {
            LensGeom g2 = L->g;
            if (set_tiles(g2, it->second.first, it->second.second, c->lds_max)) L->g = g2;
            return LENS_OK;
        }
    }
    // a batch large enough that the last partial wave of workgroups does not decide the ranking
    const int64_t n = std::max<int64_t>(2048, 32LL * c->num_cus);
    std::vector<double> hp((size_t)n * lensk::kStride, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const double j = (double)(i % 97) / 97.0;   // mild spread, all inside the domain
        double *p = &hp[(size_t)i * lensk::kStride];
        p[0] = 0.8 + 0.8 * j; p[1] = 0.6 + 0.3 * j; p[2] = 3.0 * j; p[3] = 0.05 - 0.1 * j; p[4] = 0.02;
        p[5] = 0.03; p[6] = -0.02; p[7] = 0.2; p[8] = 0.4 + 0.4 * j; p[9] = 1.0 + 2.5 * j; p[10] = 0.8;
        p[11] = 1.0; p[12] = 0.3; p[13] = 0.2 + 0.5 * j; p[14] = 0.7 + 2.0 * j; p[15] = 0.7; p[16] = 2.0;
        p[17] = 0.3 - 0.6 * j; p[18] = -0.1;
    }
    std::lock_guard<std::mutex> lk(c->sync_mu);
    void *buf = nullptr;
    const size_t pb = align_up((size_t)n * lensk::kStride * 8, kAlign), cb = align_up((size_t)n * lensk::kPCBytes, kAlign);
    std::unique_lock<std::mutex> hold;
    lens_status rs = stream_scratch(c, c->stream, pb + cb + (size_t)n * 8, &buf, &hold);
    if (rs != LENS_OK) return rs;
    double *dp = (double *)buf;
    lensk::PropBlock *dpc = (lensk::PropBlock *)((char *)buf + pb);
    double *dout = (double *)((char *)buf + pb + cb);
    HIPCHK(c, hipMemcpyAsync(dp, hp.data(), hp.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, lensk::launch_prep(dp, n, dpc, L->prep_code, nullptr, nullptr, 0, c->stream));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    float best = 1e30f;
    int bestH = L->g.strip_h, bestNT = L->g.nt;
    std::vector<std::pair<int, int>> cand = {{L->g.strip_h, L->g.nt}};   // the default shape, then the grid
    for (int nt : {256, 512})
        for (int H : {4, 8, 16, 32})
            if (!(H == L->g.strip_h && nt == L->g.nt)) cand.push_back({H, nt});
    for (const auto &hc : cand) {
        const int H = hc.first, nt = hc.second;
        LensGeom g2 = L->g;
        if (!set_tiles(g2, H, nt, c->lds_max) || g2.strip_h != H) continue;
        float t = 1e30f;
        hipError_t e = lensk::launch_loglike(g2, dpc, n, dout, nullptr, c->stream);  // warm-up
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = lensk::launch_loglike(g2, dpc, n, dout, nullptr, c->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) t = std::min(t, ms);
        }
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return hip_fail(c, e, "autotune launch");
        }
        if (t < best) {
            best = t;
            bestH = H;
            bestNT = nt;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LensGeom g2 = L->g;
    if (set_tiles(g2, bestH, bestNT, c->lds_max)) L->g = g2;
    std::lock_guard<std::mutex> tk(c->tune_mu);
    c->tune_cache[key] = {L->g.strip_h, L->g.nt};
    if (!c->tune_file.empty()) {
        FILE *f = fopen(c->tune_file.c_str(), "a");
        if (f) {
            fprintf(f, "%s %d %d\n", key.c_str(), L->g.strip_h, L->g.nt);
            fclose(f);
        }
    }
    return LENS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// lens registry
// ---------------------------------------------------------------------------
extern "C" lens_status lens_psf_crop(const double *psf, int32_t k, double psf_tail, int32_t *k_used)
{
    if (!psf || !k_used || k < 1 || (k & 1) == 0 || !std::isfinite(psf_tail)) return LENS_EINVAL;
    *k_used = k;
    if (psf_tail < 0.0) return LENS_OK;
    const double tol = psf_tail > 0.0 ? psf_tail : std::ldexp(1.0, -48);
    const int rg = (k - 1) / 2;
    double tot = 0.0;
    for (int i = 0; i < k * k; ++i) tot += std::fabs(psf[i]);
    for (int R = 0; R < rg; ++R) {
        double out = 0.0;   // taps outside the centred (2R+1)^2 square, summed directly
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (std::abs(a - rg) > R || std::abs(b - rg) > R) out += std::fabs(psf[(size_t)a * k + b]);
        if (out <= tol * tot) {
            *k_used = 2 * R + 1;
            break;
        }
    }
    return LENS_OK;
}

extern "C" lens_status lens_load_data(lens_ctx *c, const lens_data_desc *d, lens_id *out_id)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!d || !out_id) return fail(c, LENS_EINVAL, "null descriptor or output");
    DeviceGuard dg(c->device);   // the tile choice queries the device's occupancy
    const int ny = d->ny, nx = d->nx, s = d->supersample, k_given = d->psf_size;
    if (ny < 1 || nx < 1 || ny > 4096 || nx > 4096) return fail(c, LENS_EINVAL, "ny, nx must be in 1..4096");
    if (!(d->pixel_scale > 0.0) || !std::isfinite(d->pixel_scale)) return fail(c, LENS_EINVAL, "pixel_scale must be > 0");
    if (s < 1 || s > 8) return fail(c, LENS_EINVAL, "supersample must be in 1..8");
    if (k_given < 1 || k_given > lensk::kMaxK || (k_given & 1) == 0)
        return fail(c, LENS_EINVAL, "psf_size must be odd, 1..63");
    if (!std::isfinite(d->psf_tail)) return fail(c, LENS_EINVAL, "psf_tail must be finite");
    if (!d->psf || !d->data || !d->sigma || !d->mask) return fail(c, LENS_EINVAL, "null array in descriptor");
    if (d->precision < LENS_PREC_FP32 || d->precision > LENS_PREC_BF16_SPLIT3)
        return fail(c, LENS_EINVAL, "unknown precision mode");
    if (d->amplitudes != LENS_AMP_EXPLICIT && d->amplitudes != LENS_AMP_NNLS)
        return fail(c, LENS_EINVAL, "unknown amplitudes mode");
    if (d->amplitudes == LENS_AMP_NNLS && d->precision != LENS_PREC_FP32)
        return fail(c, LENS_EINVAL, "amplitudes solved by NNLS need the FP32 convolution (LENS_PREC_FP32)");
    if (d->light_model < LENS_LIGHT_BOTH || d->light_model > LENS_LIGHT_DOUBLE)
        return fail(c, LENS_EINVAL, "unknown light model");
    if (d->light_model != LENS_LIGHT_BOTH && d->amplitudes != LENS_AMP_NNLS)
        return fail(c, LENS_EINVAL, "light models other than LENS_LIGHT_BOTH need LENS_AMP_NNLS");
    if (d->mass_model != LENS_MASS_SIE && d->mass_model != LENS_MASS_EPL)
        return fail(c, LENS_EINVAL, "unknown mass model");
    if (d->light_model == LENS_LIGHT_DOUBLE)
        for (int j = 0; j < 4; ++j)
            if (!(d->sersic_n[j] >= lensk::kNMin && d->sersic_n[j] <= lensk::kNMax))
                return fail(c, LENS_EINVAL, "sersic_n must be in [0.1, 20]");
    const int64_t npix = (int64_t)ny * nx;
    for (int i = 0; i < k_given * k_given; ++i)
        if (!std::isfinite(d->psf[i])) return fail(c, LENS_EINVAL, "non-finite PSF value");
    // PSF tail crop (lens_psf_crop)
    int k = k_given;
    (void)lens_psf_crop(d->psf, k_given, d->psf_tail, &k);
    std::vector<double> psf_c;
    const double *psf = d->psf;
    if (k < k_given) {
        const int off = (k_given - k) / 2;
        psf_c.resize((size_t)k * k);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) psf_c[(size_t)a * k + b] = d->psf[(size_t)(a + off) * k_given + (b + off)];
        psf = psf_c.data();
    }
    int64_t masked = 0;
    double norm = 0.0;
    for (int64_t i = 0; i < npix; ++i) {
        if (!d->mask[i]) continue;
        const double sg = d->sigma[i];
        if (!(sg > 0.0) || !std::isfinite(sg) || !std::isfinite(d->data[i]))
            return fail(c, LENS_EINVAL, "sigma must be finite and > 0 and data finite on masked pixels");
        norm += -0.5 * std::log(2.0 * M_PI * sg * sg);
        ++masked;
    }
    const int r = (k - 1) / 2;
    const int kc = lensk::choose_kc(k);
    // LENS_PREC_* equal lensk::MODE_*; solved amplitudes convolve one channel per
    // light component, in the mode of the light model
    static const int solved_mode[4] = {lensk::MODE_FP32N, lensk::MODE_FP32N_LENS, lensk::MODE_FP32N_SRC,
                                       lensk::MODE_FP32N_DBL};
    const int mode = (d->amplitudes == LENS_AMP_NNLS ? solved_mode[d->light_model] : d->precision) |
                     (d->mass_model == LENS_MASS_EPL ? (int)lensk::MODE_EPL : 0);
    const int pitch = (int)align_up((size_t)nx, 16);
    // masked column range of each row
    std::vector<int> mlo(ny, INT_MAX), mhi(ny, INT_MIN);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (d->mask[(int64_t)y * nx + x]) {
                mlo[y] = std::min(mlo[y], x);
                mhi[y] = x + 1;
            }
    // needed range: the masked ranges of rows within r, widened by r, clipped
    std::vector<int2> evr(ny);
    std::vector<uint32_t> evl, cvl;
    std::vector<int> evpre(ny + 1, 0), cvpre(ny + 1, 0);
    for (int y = 0; y < ny; ++y) {
        int lo = INT_MAX, hi = INT_MIN;
        for (int yy = std::max(0, y - r); yy <= std::min(ny - 1, y + r); ++yy)
            if (mhi[yy] > mlo[yy]) {
                lo = std::min(lo, mlo[yy] - r);
                hi = std::max(hi, mhi[yy] + r);
            }
        lo = std::max(lo, 0);
        hi = std::min(hi, nx);
        if (hi <= lo) lo = hi = 0;
        evr[y] = make_int2(lo, hi);
        evpre[y] = (int)evl.size();
        for (int x = lo; x < hi; ++x) evl.push_back(((uint32_t)y << 16) | (uint32_t)x);
        cvpre[y] = (int)cvl.size();
        if (mhi[y] > mlo[y])
            for (int x0 = mlo[y] & ~3; x0 < mhi[y]; x0 += 4) cvl.push_back(((uint32_t)y << 16) | (uint32_t)x0);
    }
    evpre[ny] = (int)evl.size();
    cvpre[ny] = (int)cvl.size();
    LensGeom g{};
    g.ny = ny; g.nx = nx; g.s = s; g.k = k; g.r = r; g.pitch = pitch; g.mode = mode;
    g.conv_scale = 1.0;
    // the ring spans the masked columns [xoff, xoff + span) plus the PSF
    // window: xoff is the leftmost masked column rounded down to 16, where
    // every output group and segment starts at or after it
    int mlo_all = INT_MAX, mhi_all = 0;
    for (int y = 0; y < ny; ++y)
        if (mhi[y] > mlo[y]) {
            mlo_all = std::min(mlo_all, mlo[y]);
            mhi_all = std::max(mhi_all, mhi[y]);
        }
    g.xoff = mlo_all == INT_MAX ? 0 : (mlo_all & ~15);
    g.span = mlo_all == INT_MAX ? 1 : mhi_all - g.xoff;
    g.ring_w = lensk::ring_width(mode, k, g.span);
    if (!set_tiles(g, default_strip(g, c->lds_max, c->lds_cu, &g.nt), g.nt, c->lds_max))
        return fail(c, LENS_EINVAL, "image too wide for the LDS line buffer at this PSF size");
    // MFMA operands: 16-wide output segments covering the mask (row-major, with
    // row prefix) and the banded Toeplitz expansion of the flipped PSF, split
    // into BF16 planes
    std::vector<uint32_t> seg;
    std::vector<int> segpre(ny + 1, 0);
    std::vector<uint16_t> aop;
    if (lensk::mode_base(mode) == lensk::MODE_SPLIT || lensk::mode_base(mode) == lensk::MODE_BF16 ||
        lensk::mode_base(mode) == lensk::MODE_SPLIT3) {
        g.L = lensk::window_len(mode, k);
        g.nchunks = (int)((k * g.L + 31) / 32);
        for (int y = 0; y < ny; ++y) {
            segpre[y] = (int)seg.size();
            if (mhi[y] > mlo[y])
                for (int x0 = mlo[y] & ~15; x0 < mhi[y]; x0 += 16) seg.push_back(((uint32_t)y << 16) | (uint32_t)x0);
        }
        segpre[ny] = (int)seg.size();
        const int npl = lensk::mode_planes(mode);
        // FP16 split: the kernel scaled by 2^j so that its largest tap lies in
        // [2^13, 2^14), well inside the half range, its faint taps normal or
        // finely subnormal; the convolution multiplies by 2^-j again
        const bool f16 = lensk::mode_base(mode) == lensk::MODE_SPLIT;
        double kmax = 0.0;
        for (int t = 0; t < k * k; ++t) kmax = std::max(kmax, std::fabs(psf[t]));
        int kexp = 0;
        (void)std::frexp(kmax, &kexp);   // kmax < 2^kexp
        const double kscale = f16 && kmax > 0.0 ? std::ldexp(1.0, 14 - kexp) : 1.0;
        g.conv_scale = 1.0 / kscale;
        const std::vector<uint16_t> kpl = split_psf_planes(psf, k, npl, f16, kscale);   // [tap][plane]
        aop.assign((size_t)g.nchunks * npl * 64 * 8, 0);
        for (int ch = 0; ch < g.nchunks; ++ch)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int K = 32 * ch + 8 * (lane >> 4) + e, a = K / g.L, i = K % g.L, b = i - (lane & 15);
                    if (!(a < k && b >= 0 && b < k)) continue;
                    for (int q = 0; q < npl; ++q)
                        aop[(((size_t)ch * npl + q) * 64 + lane) * 8 + e] = kpl[((size_t)a * k + b) * npl + q];
                }
    }
    g.sd = d->pixel_scale / s;
    g.cfx = 0.5 * ((double)nx * s - 1.0);
    g.cfy = 0.5 * ((double)ny * s - 1.0);
    g.inv_s2 = (float)(1.0 / ((double)s * s));
    g.norm = norm;
    // two components per galaxy: the fixed indices' 1/(2n) and b_n log2 e (Eqs. 8-9)
    for (int j = 0; j < 4; ++j) {
        const double nj = d->light_model == LENS_LIGHT_DOUBLE ? d->sersic_n[j] : 1.0;
        g.fix_e[j] = 0.5 / nj;
        g.fix_B[j] = lensk::host_sersic_bn(nj) * 1.4426950408889634;
    }
    // host images
    std::vector<float> hd((size_t)ny * pitch, 0.0f), hw((size_t)ny * pitch, 0.0f), hk((size_t)k * k);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t i = (int64_t)y * nx + x;
            if (!d->mask[i]) continue;
            hd[(size_t)y * pitch + x] = (float)d->data[i];
            hw[(size_t)y * pitch + x] = (float)(1.0 / d->sigma[i]);
        }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) hk[(size_t)a * k + b] = (float)psf[(size_t)(k - 1 - a) * k + (k - 1 - b)];
    // D = sum_mask (w d)^2 from the same FP32 values the kernels read (amplitude solve)
    g.dd = 0.0;
    for (size_t i = 0; i < hd.size(); ++i) {
        const double wd = (double)hw[i] * (double)hd[i];
        g.dd += wd * wd;
    }
    // one slab
    size_t off = 0;
    auto place = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 4), kAlign);
        return o;
    };
    const size_t o_psf = place(hk.size() * 4), o_d = place(hd.size() * 4), o_w = place(hw.size() * 4);
    const size_t o_evl = place(evl.size() * 4), o_evpre = place(evpre.size() * 4), o_evr = place(evr.size() * 8);
    const size_t o_cvl = place(cvl.size() * 4), o_cvpre = place(cvpre.size() * 4);
    const size_t o_aop = place(aop.size() * 2), o_seg = place(seg.size() * 4), o_segpre = place(segpre.size() * 4);
    const size_t total = off;
    if (!charge(c, (int64_t)total)) return fail(c, LENS_ENOMEM, "HBM budget exhausted");
    void *slab = dev_alloc(c, total);
    if (!slab) {
        uncharge(c, (int64_t)total);
        return fail(c, LENS_ENOMEM, "device allocation failed");
    }
    char *b = (char *)slab;
    struct {
        size_t o;
        const void *src;
        size_t n;
    } cp[] = {{o_psf, hk.data(), hk.size() * 4},     {o_d, hd.data(), hd.size() * 4},
              {o_w, hw.data(), hw.size() * 4},       {o_evl, evl.data(), evl.size() * 4},
              {o_evpre, evpre.data(), evpre.size() * 4}, {o_evr, evr.data(), evr.size() * 8},
              {o_cvl, cvl.data(), cvl.size() * 4},   {o_cvpre, cvpre.data(), cvpre.size() * 4},
              {o_aop, aop.data(), aop.size() * 2},   {o_seg, seg.data(), seg.size() * 4},
              {o_segpre, segpre.data(), segpre.size() * 4}};
    for (auto &e : cp) {
        if (!e.n) continue;
        hipError_t he = hipMemcpyAsync(b + e.o, e.src, e.n, hipMemcpyHostToDevice, c->stream);
        if (he != hipSuccess) {
            dev_free(c, slab);
            uncharge(c, (int64_t)total);
            return hip_fail(c, he, "hipMemcpyAsync (load)");
        }
    }
    hipError_t he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        dev_free(c, slab);
        uncharge(c, (int64_t)total);
        return hip_fail(c, he, "hipStreamSynchronize (load)");
    }
    g.psf = (const float *)(b + o_psf);
    g.data = (const float *)(b + o_d);
    g.wgt = (const float *)(b + o_w);
    g.evl = (const uint32_t *)(b + o_evl);
    g.evpre = (const int *)(b + o_evpre);
    g.evr = (const int2 *)(b + o_evr);
    g.cvl = (const uint32_t *)(b + o_cvl);
    g.cvpre = (const int *)(b + o_cvpre);
    g.aop = (const uint4 *)(b + o_aop);
    g.seg = (const uint32_t *)(b + o_seg);
    g.segpre = (const int *)(b + o_segpre);
    Lens *L = new Lens();
    L->g = g;
    L->precision = d->precision;
    L->amplitudes = d->amplitudes;
    L->light_model = d->light_model;
    L->mass_model = d->mass_model;
    L->prep_code = d->light_model | (d->mass_model << lensk::kMassShift);
    L->psf_given = k_given;
    L->masked = masked;
    L->needed = (int64_t)evl.size();
    L->slab = slab;
    L->bytes = total;
    if (c->autotune) {
        lens_status ts = tune_lens(c, L);
        if (ts != LENS_OK) {
            dev_free(c, slab);
            uncharge(c, (int64_t)total);
            delete L;
            return ts;
        }
    }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        L->id = c->next_id++;
        c->lenses[L->id] = L;
    }
    log_line(c, "load lens %lld: %dx%d px, s=%d, PSF %d (convolved %d), mode %d, %d-row strips x %d threads, %zu B",
             (long long)L->id, L->g.ny, L->g.nx, L->g.s, d->psf_size, L->g.k, L->g.mode, L->g.strip_h, L->g.nt,
             L->bytes);
    *out_id = L->id;
    return LENS_OK;
}

extern "C" lens_status lens_unload(lens_ctx *c, lens_id id)
{
    if (!c) return LENS_EINVAL;
    Lens *L = nullptr;
    std::lock_guard<std::mutex> plk(c->sync_mu);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->lenses.find(id);
        if (it == c->lenses.end()) return fail(c, LENS_ENOENT, "unknown lens id");
        L = it->second;
        if (L->users > 0) return fail(c, LENS_EBUSY, "lens is in use by a running call or a sampler ensemble");
        {
            std::lock_guard<std::mutex> sl(c->smu);
            if (L->requests > 0) return fail(c, LENS_EBUSY, "lens has serving requests in flight");
        }
        c->lenses.erase(it);
    }
    DeviceGuard dg(c->device);
    // every launch that read the lens has completed: blocking calls synchronise,
    // serving requests are finished; device-buffer calls are ordered on their streams
    (void)hipDeviceSynchronize();
    for (auto it = c->plans.begin(); it != c->plans.end();) {
        if (std::find(it->second->ids.begin(), it->second->ids.end(), id) != it->second->ids.end()) {
            drop_plan(c, it->second);
            it = c->plans.erase(it);
        } else {
            ++it;
        }
    }
    for (auto it = c->dplans.begin(); it != c->dplans.end();) {
        if (dplan_uses(it->second, id)) {
            drop_dplan(c, it->second);
            it = c->dplans.erase(it);
        } else {
            ++it;
        }
    }
    log_line(c, "unload lens %lld", (long long)id);
    dev_free(c, L->slab);
    uncharge(c, (int64_t)L->bytes);
    delete L;
    return LENS_OK;
}

extern "C" lens_status lens_get_info(lens_ctx *c, lens_id id, lens_info *out)
{
    if (!c || !out) return LENS_EINVAL;
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    out->ny = L->g.ny;
    out->nx = L->g.nx;
    out->supersample = L->g.s;
    out->psf_size = L->psf_given;
    out->precision = L->precision;
    out->masked_pixels = L->masked;
    out->needed_pixels = L->needed;
    out->device_bytes = (int64_t)L->bytes;
    out->norm = L->g.norm;
    out->strip_rows = L->g.strip_h;
    out->threads = L->g.nt;
    out->lds_bytes = (int64_t)lensk::ring_bytes(L->g);
    out->psf_used = L->g.k;
    out->amplitudes = L->amplitudes;
    out->light_model = L->light_model;
    out->mass_model = L->mass_model;
    out->n_amplitudes = lensk::mode_solved(L->g.mode) ? lensk::mode_channels(L->g.mode) : 2;
    {
        DeviceGuard dg(c->device);
        out->blocks_per_cu = lensk::loglike_blocks_per_cu(L->g);
    }
    release(c, L);
    return LENS_OK;
}

// ---------------------------------------------------------------------------
// likelihood calls
// ---------------------------------------------------------------------------
namespace {

// pinned staging + device buffers of the blocking calls, for n proposals
lens_status sync_buffers(lens_ctx *c, int64_t n)
{
    if ((size_t)n > c->h_cap) {
        size_t cap = std::max<size_t>((size_t)n, c->h_cap * 3 / 2);
        if (c->h_params) (void)hipHostFree(c->h_params);
        if (c->h_out) (void)hipHostFree(c->h_out);
        c->h_params = c->h_out = nullptr;
        c->h_cap = 0;
        HIPCHK(c, hipHostMalloc((void **)&c->h_params, cap * lensk::kStride * sizeof(double), hipHostMallocDefault));
        HIPCHK(c, hipHostMalloc((void **)&c->h_out, cap * 5 * sizeof(double), hipHostMallocDefault));
        c->h_cap = cap;
    }
    const size_t need = scratch_bytes((int64_t)c->h_cap, true);
    if (need > c->d_sync_bytes) {
        if (c->d_sync) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            dev_free(c, c->d_sync);
            uncharge(c, (int64_t)c->d_sync_bytes);
            c->d_sync = nullptr;
            c->d_sync_bytes = 0;
        }
        if (!charge(c, (int64_t)need)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (staging)");
        c->d_sync = dev_alloc(c, need);
        if (!c->d_sync) {
            uncharge(c, (int64_t)need);
            return fail(c, LENS_ENOMEM, "device allocation failed (staging)");
        }
        c->d_sync_bytes = need;
    }
    return LENS_OK;
}

}  // namespace

extern "C" lens_status lens_loglike_batch(lens_ctx *c, lens_id id, const double *params, int64_t n,
                                          double *out)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || (n > 0 && (!params || !out))) return fail(c, LENS_EINVAL, "bad params/out/n");
    if (n > INT_MAX) return fail(c, LENS_EINVAL, "n too large for one call");
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    if (n == 0) {
        release(c, L);
        return LENS_OK;
    }
    DeviceGuard dg(c->device);
    lens_status rs = LENS_OK;
    {
        std::lock_guard<std::mutex> lk(c->sync_mu);
        rs = sync_buffers(c, n);
        if (rs == LENS_OK) {
            ScratchLayout S = carve(c->d_sync, (int64_t)c->h_cap, true);
            memcpy(c->h_params, params, (size_t)n * lensk::kStride * sizeof(double));
            hipError_t e = hipMemcpyAsync(S.params, c->h_params, (size_t)n * lensk::kStride * sizeof(double),
                                          hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = launch_lens(L, S.params, S.pc, n, S.out, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->h_out, S.out, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_batch");
            else memcpy(out, c->h_out, (size_t)n * sizeof(double));
        }
    }
    release(c, L);
    return rs;
}

extern "C" lens_status lens_loglike_amps(lens_ctx *c, lens_id id, const double *params, int64_t n, double *out,
                                         double *out_amp)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || (n > 0 && (!params || !out || !out_amp))) return fail(c, LENS_EINVAL, "bad params/out/out_amp/n");
    if (n > INT_MAX) return fail(c, LENS_EINVAL, "n too large for one call");
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    if (n == 0) {
        release(c, L);
        return LENS_OK;
    }
    const bool solved = lensk::mode_solved(L->g.mode);
    const int na = solved ? lensk::mode_channels(L->g.mode) : 2;
    DeviceGuard dg(c->device);
    lens_status rs = LENS_OK;
    {
        std::lock_guard<std::mutex> lk(c->sync_mu);
        rs = sync_buffers(c, n);
        if (rs == LENS_OK) {
            ScratchLayout S = carve(c->d_sync, (int64_t)c->h_cap, true);
            memcpy(c->h_params, params, (size_t)n * lensk::kStride * sizeof(double));
            hipError_t e = hipMemcpyAsync(S.params, c->h_params, (size_t)n * lensk::kStride * sizeof(double),
                                          hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = launch_lens(L, S.params, S.pc, n, S.out, c->stream, solved ? S.amp : nullptr);
            // staging: out at [0, n), amplitudes at [h_cap, h_cap + na n) (S.amp = S.out + h_cap)
            double *h_amp = c->h_out + c->h_cap;
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->h_out, S.out, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess && solved)
                e = hipMemcpyAsync(h_amp, S.amp, (size_t)n * na * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                rs = hip_fail(c, e, "lens_loglike_amps");
            } else {
                memcpy(out, c->h_out, (size_t)n * sizeof(double));
                for (int64_t i = 0; i < n; ++i) {
                    const bool ok = out[i] != -INFINITY;
                    if (solved) {
                        for (int a = 0; a < na; ++a) out_amp[na * i + a] = ok ? h_amp[na * i + a] : NAN;
                    } else {
                        out_amp[2 * i] = ok ? params[i * lensk::kStride + 7] : NAN;
                        out_amp[2 * i + 1] = ok ? params[i * lensk::kStride + 12] : NAN;
                    }
                }
            }
        }
    }
    release(c, L);
    return rs;
}

extern "C" lens_status lens_loglike_batch_device(lens_ctx *c, lens_id id, const double *d_params, int64_t n,
                                                 double *d_out, void *stream)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || (n > 0 && (!d_params || !d_out))) return fail(c, LENS_EINVAL, "bad params/out/n");
    if (n > INT_MAX) return fail(c, LENS_EINVAL, "n too large for one call");
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    if (n == 0) {
        release(c, L);
        return LENS_OK;
    }
    DeviceGuard dg(c->device);
    hipStream_t hs = (hipStream_t)stream;  // NULL: the default stream
    void *scr = nullptr;
    std::unique_lock<std::mutex> hold;   // until both launches are enqueued
    lens_status rs = stream_scratch(c, hs, scratch_bytes(n, false), &scr, &hold);
    if (rs == LENS_OK) {
        ScratchLayout S = carve(scr, n, false);
        hipError_t e = launch_lens(L, d_params, S.pc, n, d_out, hs);
        if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_batch_device");
    }
    release(c, L);
    return rs;
}

extern "C" lens_status lens_loglike_batch_device_noalloc(lens_ctx *c, lens_id id, const double *d_params,
                                                         int64_t n, double *d_out, void *stream)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || (n > 0 && (!d_params || !d_out))) return fail(c, LENS_EINVAL, "bad params/out/n");
    if (n > lensk::kNoAllocMax)
        return fail(c, LENS_EINVAL, "n above LENS_NOALLOC_MAX, the fixed scratch of the allocation-free call");
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    lens_status rs = LENS_OK;
    if (n > 0) {
        DeviceGuard dg(c->device);
        lensk::PropBlock *pc = lensk::noalloc_scratch(c->device);   // resolved at lens_init
        if (!pc) {
            rs = fail(c, LENS_EDEVICE, "fixed scratch not set up on this device");
        } else {
            const hipError_t e = launch_lens(L, d_params, pc, n, d_out, (hipStream_t)stream);
            if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_batch_device_noalloc");
        }
    }
    release(c, L);
    return rs;
}

namespace {

void drop_plan(lens_ctx *c, Plan *pl)
{
    // sync_mu held; the plan's launches have completed (every call synchronises)
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    dev_free(c, pl->dev);
    uncharge(c, (int64_t)pl->bytes);
    if (pl->h_params) (void)hipHostFree(pl->h_params);
    if (pl->h_out) (void)hipHostFree(pl->h_out);
    delete pl;
}

std::string plan_key(int32_t nlens, const lens_id *ids, const int64_t *counts)
{
    std::string k;
    k.reserve((size_t)nlens * 24);
    char buf[48];
    for (int i = 0; i < nlens; ++i) {
        snprintf(buf, sizeof(buf), "%lld:%lld,", (long long)ids[i], (long long)counts[i]);
        k += buf;
    }
    return k;
}

// Persistent-launch groups of a multi-lens evaluation.  Entry i of Ls owns
// counts[i] proposals at pooled offset off[i].  Lenses share a launch when
// they share a mode and a workgroup size, and the resident workgroups per CU
// that their own LDS rings allow (the occupancy) are within 25% of the
// group's highest: a persistent launch sizes its grid by its largest ring, so
// a wide lens would hold narrow ones to its occupancy, while every extra
// launch ends in a tail where a few long items keep most CUs idle.  Inside a
// group lenses in descending per-proposal cost, so the longest items start
// first.
struct BatchGroup {
    int mode, nt, nl, nitems, grid;
    size_t lds, o_geom, o_ls, o_lo;
};
struct BatchGroups {
    std::vector<BatchGroup> gs;
    std::vector<LensGeom> geom;   // per entry, group by group
    std::vector<int> lstart;      // per group: entry item starts, then the group's item count
    std::vector<int64_t> lout;    // per entry: pooled offset of its first proposal
};

void group_batch(lens_ctx *c, const std::vector<Lens *> &Ls, const int64_t *counts, const int64_t *off,
                 BatchGroups *out)
{
    const int nl = (int)Ls.size();
    std::map<std::tuple<int, int, int>, std::vector<int>> classes;   // (mode, nt, -occupancy)
    for (int i = 0; i < nl; ++i)
        if (counts[i] > 0) {
            const LensGeom &g = Ls[i]->g;
            const int occ = lensk::batch_blocks_per_cu(g.mode, g.nt, lensk::ring_bytes(g));
            classes[std::make_tuple(g.mode, g.nt, -occ)].push_back(i);
        }
    // classes in descending occupancy within a (mode, nt); a class joins the
    // open group while 4 occ >= 3 occ_top
    std::vector<std::pair<std::pair<int, int>, std::vector<int>>> groups;
    int top = 0;
    for (auto &kv : classes) {
        const int mode = std::get<0>(kv.first), nt = std::get<1>(kv.first), occ = -std::get<2>(kv.first);
        const bool join = !groups.empty() && groups.back().first == std::make_pair(mode, nt) && 4 * occ >= 3 * top;
        if (!join) {
            groups.push_back({{mode, nt}, {}});
            top = occ;
        }
        auto &v = groups.back().second;
        v.insert(v.end(), kv.second.begin(), kv.second.end());
    }
    for (auto &kv : groups) {
        std::vector<int> &v = kv.second;
        auto cost = [&](int i) {
            const LensGeom &g = Ls[i]->g;
            return (double)Ls[i]->needed * g.s * g.s * 200.0 + (double)Ls[i]->masked * g.k * g.k;
        };
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return cost(a) > cost(b); });
        BatchGroup gg{};
        gg.mode = kv.first.first;
        gg.nt = kv.first.second;
        gg.nl = (int)v.size();
        gg.o_geom = out->geom.size();
        gg.o_ls = out->lstart.size();
        gg.o_lo = out->lout.size();
        int items = 0;
        for (int i : v) {
            out->geom.push_back(Ls[i]->g);
            out->lstart.push_back(items);
            out->lout.push_back(off[i]);
            items += (int)counts[i];
            gg.lds = std::max(gg.lds, lensk::ring_bytes(Ls[i]->g));
        }
        out->lstart.push_back(items);
        gg.nitems = items;
        gg.grid = c->num_cus * lensk::batch_blocks_per_cu(gg.mode, gg.nt, gg.lds);
        out->gs.push_back(gg);
    }
}

// Launches the groups of bg in order on stream st.
hipError_t launch_groups(const BatchGroups &bg, hipStream_t st, const LensGeom *d_geom, const int *d_ls,
                         const int64_t *d_lo, const lensk::PropBlock *d_pc, double *d_out, unsigned int *d_cnt)
{
    hipError_t e = hipSuccess;
    for (size_t gi = 0; gi < bg.gs.size() && e == hipSuccess; ++gi) {
        const BatchGroup &gg = bg.gs[gi];
        e = lensk::launch_batch(gg.mode, gg.nt, gg.grid, gg.lds, d_geom + gg.o_geom, d_ls + gg.o_ls, d_lo + gg.o_lo,
                                gg.nl, gg.nitems, d_pc, d_out, d_cnt + gi, st);
    }
    return e;
}

// Build and capture the graph of one call shape (sync_mu held).
lens_status build_plan(lens_ctx *c, int32_t nlens, const lens_id *ids, const int64_t *counts,
                       const std::vector<Lens *> &Ls, int64_t tot, Plan **out)
{
    auto pl = std::make_unique<Plan>();
    pl->ids.assign(ids, ids + nlens);
    pl->counts.assign(counts, counts + nlens);
    pl->tot = tot;
    std::vector<int64_t> off(nlens + 1, 0);
    for (int i = 0; i < nlens; ++i) off[i + 1] = off[i] + counts[i];
    BatchGroups bg;
    group_batch(c, Ls, counts, off.data(), &bg);
    std::vector<BatchGroup> &gs = bg.gs;
    std::vector<LensGeom> &hgeom = bg.geom;
    std::vector<int> &hls = bg.lstart;
    std::vector<int64_t> &hlo = bg.lout;
    // light model of every proposal: one for all, or per lens by proposal offset
    bool one_model = true;
    for (int i = 1; i < nlens; ++i) one_model = one_model && Ls[i]->prep_code == Ls[0]->prep_code;
    std::vector<int> hmodel(nlens);
    for (int i = 0; i < nlens; ++i) hmodel[i] = Ls[i]->prep_code;
    // device layout: params | pc | out | geoms | lstart | lout | counters | pstart | pmodel
    const size_t b_par = align_up((size_t)tot * lensk::kStride * 8, kAlign);
    const size_t b_pc = align_up((size_t)tot * lensk::kPCBytes, kAlign);
    const size_t b_out = align_up((size_t)tot * 8, kAlign);
    const size_t b_geom = align_up(hgeom.size() * sizeof(LensGeom), kAlign);
    const size_t b_ls = align_up(hls.size() * 4, kAlign), b_lo = align_up(hlo.size() * 8, kAlign);
    const size_t b_cnt = align_up(gs.size() * 4 + 4, kAlign);
    const size_t b_ps = align_up((size_t)(nlens + 1) * 8, kAlign), b_pm = align_up((size_t)nlens * 4, kAlign);
    pl->bytes = b_par + b_pc + b_out + b_geom + b_ls + b_lo + b_cnt + b_ps + b_pm;
    if (!charge(c, (int64_t)pl->bytes)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (batch plan)");
    pl->dev = dev_alloc(c, pl->bytes);
    if (!pl->dev) {
        uncharge(c, (int64_t)pl->bytes);
        return fail(c, LENS_ENOMEM, "device allocation failed (batch plan)");
    }
    char *b = (char *)pl->dev;
    double *d_par = (double *)b;
    lensk::PropBlock *d_pc = (lensk::PropBlock *)(b + b_par);
    double *d_out = (double *)(b + b_par + b_pc);
    LensGeom *d_geom = (LensGeom *)(b + b_par + b_pc + b_out);
    int *d_ls = (int *)((char *)d_geom + b_geom);
    int64_t *d_lo = (int64_t *)((char *)d_ls + b_ls);
    unsigned int *d_cnt = (unsigned int *)((char *)d_lo + b_lo);
    int64_t *d_ps = (int64_t *)((char *)d_cnt + b_cnt);
    int *d_pm = (int *)((char *)d_ps + b_ps);
    Plan *raw = pl.get();
    auto bail = [&](hipError_t e, const char *what) {
        raw->used = 0;
        drop_plan(c, pl.release());
        return hip_fail(c, e, what);
    };
    hipError_t e = hipHostMalloc((void **)&pl->h_params, (size_t)tot * lensk::kStride * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&pl->h_out, (size_t)tot * 8, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemcpyAsync(d_geom, hgeom.data(), hgeom.size() * sizeof(LensGeom), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ls, hls.data(), hls.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_lo, hlo.data(), hlo.size() * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !one_model)
        e = hipMemcpyAsync(d_ps, off.data(), (size_t)(nlens + 1) * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !one_model)
        e = hipMemcpyAsync(d_pm, hmodel.data(), (size_t)nlens * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(e, "batch plan set-up");
    // capture: the graph holds only copies and kernels (the work counters are
    // cleared by a kernel node, never by a memset node)
    // captured on a stream of its own (only this thread, under sync_mu, uses it)
    const int64_t ntot = tot;
    double *h_par = pl->h_params, *h_out = pl->h_out;
    const int m0 = hmodel[0];
    // the launch sequence, on stream st: params in, prep, persistent launches, results out
    auto seq = [bg, ntot, one_model, m0, nlens, h_par, h_out, d_par, d_pc, d_out, d_geom, d_ls, d_lo, d_cnt, d_ps,
                d_pm](hipStream_t st) {
        hipError_t ce = hipMemcpyAsync(d_par, h_par, (size_t)ntot * lensk::kStride * 8, hipMemcpyHostToDevice, st);
        if (ce == hipSuccess)
            ce = one_model ? lensk::launch_prep(d_par, ntot, d_pc, m0, nullptr, nullptr, 0, st)
                           : lensk::launch_prep(d_par, ntot, d_pc, 0, d_ps, d_pm, nlens, st);
        if (ce == hipSuccess) ce = launch_groups(bg, st, d_geom, d_ls, d_lo, d_pc, d_out, d_cnt);
        if (ce == hipSuccess) ce = hipMemcpyAsync(h_out, d_out, (size_t)ntot * 8, hipMemcpyDeviceToHost, st);
        return ce;
    };
    pl->eager = seq;
    hipStream_t cs = c->cap_stream;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bail(e, "hipStreamBeginCapture");
    const hipError_t ce = seq(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    pl->graph = graph;
    if (e == hipErrorStreamCaptureInvalidated || ce == hipErrorStreamCaptureInvalidated ||
        ce == hipErrorStreamCaptureImplicit) {
        // another thread's legacy-stream operation broke the capture; nothing
        // ran and the device is fine: this shape runs without a graph
        (void)hipGetLastError();
        if (pl->graph) (void)hipGraphDestroy(pl->graph);
        pl->graph = nullptr;
        log_line(c, "batch plan: capture invalidated by another thread; %d lenses run without a graph", (int)nlens);
        *out = pl.release();
        return LENS_OK;
    }
    if (ce != hipSuccess) return bail(ce, "batch plan capture");
    if (e != hipSuccess) return bail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bail(e, "hipGraphInstantiate");
    log_line(c, "batch plan captured: %d lenses, %lld proposals, %zu persistent launches, %zu B", (int)nlens,
             (long long)tot, gs.size(), pl->bytes);
    *out = pl.release();
    return LENS_OK;
}

}  // namespace

extern "C" lens_status lens_loglike_multi(lens_ctx *c, int32_t nlens, const lens_id *ids, const int64_t *counts,
                                          const double *params, double *out)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (nlens < 0 || (nlens > 0 && (!ids || !counts))) return fail(c, LENS_EINVAL, "bad ids/counts");
    int64_t tot = 0;
    for (int i = 0; i < nlens; ++i) {
        if (counts[i] < 0) return fail(c, LENS_EINVAL, "negative count");
        tot += counts[i];
    }
    if (tot > 0 && (!params || !out)) return fail(c, LENS_EINVAL, "null params/out");
    if (tot > INT_MAX) return fail(c, LENS_EINVAL, "too many proposals for one call");
    if (tot == 0) return LENS_OK;
    DeviceGuard dg(c->device);
    std::lock_guard<std::mutex> lk(c->sync_mu);
    std::vector<Lens *> Ls;
    for (int i = 0; i < nlens; ++i) {
        Lens *L = acquire(c, ids[i]);
        if (!L) {
            for (Lens *x : Ls) release(c, x);
            return fail(c, LENS_ENOENT, "unknown lens id");
        }
        Ls.push_back(L);
    }
    const std::string key = plan_key(nlens, ids, counts);
    Plan *pl = nullptr;
    lens_status rs = LENS_OK;
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        pl = it->second;
    } else {
        if (c->plans.size() >= 8) {  // keep the 8 most recently used shapes
            auto victim = c->plans.begin();
            for (auto j = c->plans.begin(); j != c->plans.end(); ++j)
                if (j->second->used < victim->second->used) victim = j;
            drop_plan(c, victim->second);
            c->plans.erase(victim);
        }
        rs = build_plan(c, nlens, ids, counts, Ls, tot, &pl);
        if (rs == LENS_OK) c->plans[key] = pl;
    }
    if (rs == LENS_OK) {
        pl->used = ++c->plan_clock;
        memcpy(pl->h_params, params, (size_t)tot * lensk::kStride * 8);
        hipError_t e = pl->exec ? hipGraphLaunch(pl->exec, c->stream) : pl->eager(c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_multi");
        else memcpy(out, pl->h_out, (size_t)tot * 8);
    }
    for (Lens *x : Ls) release(c, x);
    return rs;
}

namespace {

struct DPlan {
    std::vector<lens_id> ids;
    std::vector<int64_t> counts;
    int64_t tot = 0;
    BatchGroups bg;
    bool one_model = true;
    int model0 = 0;
    void *dev = nullptr;          // geoms | lstart | lout | pstart | pmodel
    size_t bytes = 0;
    LensGeom *d_geom = nullptr;
    int *d_ls = nullptr, *d_pm = nullptr;
    int64_t *d_lo = nullptr, *d_ps = nullptr;
    uint64_t used = 0;
};

void drop_dplan(lens_ctx *c, DPlan *pl)
{
    // sync_mu held, the device drained
    dev_free(c, pl->dev);
    uncharge(c, (int64_t)pl->bytes);
    delete pl;
}

void free_dplan_now(lens_ctx *c, DPlan *pl)
{
    dev_free(c, pl->dev);
    delete pl;
}

bool dplan_uses(const DPlan *pl, lens_id id)
{
    return std::find(pl->ids.begin(), pl->ids.end(), id) != pl->ids.end();
}

// Build the tables of one call shape (sync_mu held).
lens_status build_dplan(lens_ctx *c, int32_t nlens, const lens_id *ids, const int64_t *counts,
                        const std::vector<Lens *> &Ls, int64_t tot, DPlan **out)
{
    auto pl = std::make_unique<DPlan>();
    pl->ids.assign(ids, ids + nlens);
    pl->counts.assign(counts, counts + nlens);
    pl->tot = tot;
    std::vector<int64_t> off(nlens + 1, 0);
    for (int i = 0; i < nlens; ++i) off[i + 1] = off[i] + counts[i];
    group_batch(c, Ls, counts, off.data(), &pl->bg);
    std::vector<int> hmodel(nlens);
    for (int i = 0; i < nlens; ++i) {
        hmodel[i] = Ls[i]->prep_code;
        pl->one_model = pl->one_model && hmodel[i] == hmodel[0];
    }
    pl->model0 = hmodel[0];
    const BatchGroups &bg = pl->bg;
    const size_t b_geom = align_up(bg.geom.size() * sizeof(LensGeom), kAlign);
    const size_t b_ls = align_up(bg.lstart.size() * 4, kAlign), b_lo = align_up(bg.lout.size() * 8, kAlign);
    const size_t b_ps = align_up((size_t)(nlens + 1) * 8, kAlign), b_pm = align_up((size_t)nlens * 4, kAlign);
    pl->bytes = b_geom + b_ls + b_lo + b_ps + b_pm;
    if (!charge(c, (int64_t)pl->bytes)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (batch tables)");
    pl->dev = dev_alloc(c, pl->bytes);
    if (!pl->dev) {
        uncharge(c, (int64_t)pl->bytes);
        return fail(c, LENS_ENOMEM, "device allocation failed (batch tables)");
    }
    char *b = (char *)pl->dev;
    pl->d_geom = (LensGeom *)b;
    pl->d_ls = (int *)(b + b_geom);
    pl->d_lo = (int64_t *)(b + b_geom + b_ls);
    pl->d_ps = (int64_t *)(b + b_geom + b_ls + b_lo);
    pl->d_pm = (int *)(b + b_geom + b_ls + b_lo + b_ps);
    hipError_t e = hipMemcpyAsync(pl->d_geom, bg.geom.data(), bg.geom.size() * sizeof(LensGeom), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->d_ls, bg.lstart.data(), bg.lstart.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->d_lo, bg.lout.data(), bg.lout.size() * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->d_ps, off.data(), (size_t)(nlens + 1) * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pl->d_pm, hmodel.data(), (size_t)nlens * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        drop_dplan(c, pl.release());
        return hip_fail(c, e, "batch tables set-up");
    }
    log_line(c, "device batch shape: %d lenses, %lld proposals, %zu persistent launches", (int)nlens, (long long)tot,
             bg.gs.size());
    *out = pl.release();
    return LENS_OK;
}

}  // namespace

extern "C" lens_status lens_loglike_multi_device(lens_ctx *c, int32_t nlens, const lens_id *ids,
                                                 const int64_t *counts, const double *d_params, double *d_out,
                                                 void *stream)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (nlens < 0 || (nlens > 0 && (!ids || !counts))) return fail(c, LENS_EINVAL, "bad ids/counts");
    int64_t tot = 0;
    for (int i = 0; i < nlens; ++i) {
        if (counts[i] < 0) return fail(c, LENS_EINVAL, "negative count");
        tot += counts[i];
    }
    if (tot > 0 && (!d_params || !d_out)) return fail(c, LENS_EINVAL, "null params/out");
    if (tot > INT_MAX) return fail(c, LENS_EINVAL, "too many proposals for one call");
    if (tot == 0) return LENS_OK;
    DeviceGuard dg(c->device);
    hipStream_t hs = (hipStream_t)stream;
    // sync_mu keeps the shape's tables alive until the launches are enqueued
    std::lock_guard<std::mutex> lk(c->sync_mu);
    std::vector<Lens *> Ls;
    for (int i = 0; i < nlens; ++i) {
        Lens *L = acquire(c, ids[i]);
        if (!L) {
            for (Lens *x : Ls) release(c, x);
            return fail(c, LENS_ENOENT, "unknown lens id");
        }
        Ls.push_back(L);
    }
    const std::string key = plan_key(nlens, ids, counts);
    DPlan *pl = nullptr;
    lens_status rs = LENS_OK;
    auto it = c->dplans.find(key);
    if (it != c->dplans.end()) {
        pl = it->second;
    } else {
        if (c->dplans.size() >= 8) {  // keep the 8 most recently used shapes
            auto victim = c->dplans.begin();
            for (auto j = c->dplans.begin(); j != c->dplans.end(); ++j)
                if (j->second->used < victim->second->used) victim = j;
            // launches on any stream may still read the victim's tables
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_multi_device");
            else {
                drop_dplan(c, victim->second);
                c->dplans.erase(victim);
            }
        }
        if (rs == LENS_OK) rs = build_dplan(c, nlens, ids, counts, Ls, tot, &pl);
        if (rs == LENS_OK) c->dplans[key] = pl;
    }
    if (rs == LENS_OK) {
        pl->used = ++c->plan_clock;
        const size_t b_pc = align_up((size_t)tot * lensk::kPCBytes, kAlign);
        void *scr = nullptr;
        std::unique_lock<std::mutex> hold;   // until every launch is enqueued
        rs = stream_scratch(c, hs, b_pc + align_up(pl->bg.gs.size() * 4 + 4, kAlign), &scr, &hold);
        if (rs == LENS_OK) {
            lensk::PropBlock *d_pc = (lensk::PropBlock *)scr;
            unsigned int *d_cnt = (unsigned int *)((char *)scr + b_pc);
            hipError_t e = pl->one_model ? lensk::launch_prep(d_params, tot, d_pc, pl->model0, nullptr, nullptr, 0, hs)
                                         : lensk::launch_prep(d_params, tot, d_pc, 0, pl->d_ps, pl->d_pm, nlens, hs);
            if (e == hipSuccess) e = launch_groups(pl->bg, hs, pl->d_geom, pl->d_ls, pl->d_lo, d_pc, d_out, d_cnt);
            if (e != hipSuccess) rs = hip_fail(c, e, "lens_loglike_multi_device");
        }
    }
    for (Lens *x : Ls) release(c, x);
    return rs;
}

extern "C" lens_status lens_model_image(lens_ctx *c, lens_id id, const double *params1, int32_t stage,
                                        double *out_img)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!params1 || !out_img || (stage != 0 && stage != 1)) return fail(c, LENS_EINVAL, "bad arguments");
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    DeviceGuard dg(c->device);
    const int64_t npix = (int64_t)L->g.ny * L->g.nx;
    lens_status rs = LENS_OK;
    {
        std::lock_guard<std::mutex> lk(c->sync_mu);
        // device: params(20 doubles) | pc | img | tmp
        const size_t bytes = 4096 + 2 * align_up((size_t)npix * 4, kAlign);
        void *dbuf = nullptr;
        std::unique_lock<std::mutex> hold;
        rs = stream_scratch(c, c->stream, bytes, &dbuf, &hold);
        if (rs == LENS_OK) {
            char *b = (char *)dbuf;
            double *dp = (double *)b;
            lensk::PropBlock *dpc = (lensk::PropBlock *)(b + 2048);
            float *img = (float *)(b + 4096);
            float *tmp = (float *)(b + 4096 + align_up((size_t)npix * 4, kAlign));
            lensk::PropBlock pc{};
            std::vector<float> hi((size_t)npix);
            hipError_t e = hipMemcpyAsync(dp, params1, lensk::kStride * sizeof(double), hipMemcpyHostToDevice, c->stream);
            const int code = LENS_LIGHT_BOTH | (L->mass_model << lensk::kMassShift);
            if (e == hipSuccess) e = lensk::launch_prep(dp, 1, dpc, code, nullptr, nullptr, 0, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(&pc, dpc, sizeof(pc), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e == hipSuccess && pc.valid != 1.0) {
                rs = fail(c, LENS_EINVAL, "proposal outside the parameter domain (a model image needs finite amplitudes)");
            } else {
                if (e == hipSuccess) e = lensk::launch_model_image(L->g, dpc, stage, img, tmp, c->stream);
                if (e == hipSuccess) e = hipMemcpyAsync(hi.data(), img, (size_t)npix * 4, hipMemcpyDeviceToHost, c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
                if (e != hipSuccess) rs = hip_fail(c, e, "lens_model_image");
                else
                    for (int64_t i = 0; i < npix; ++i) out_img[i] = (double)hi[(size_t)i];
            }
        }
    }
    release(c, L);
    return rs;
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------
namespace {

void finish_request(lens_ctx *c, Request *r)
{
    // called with smu held, when the last tile of r has completed
    if (r->cancel) {
        r->state = RState::Canceled;
        r->status = LENS_ECANCELED;
        c->stats.requests_canceled++;
    } else if (r->status == LENS_PENDING) {
        memcpy(r->out, r->result.data(), (size_t)r->n * sizeof(double));
        r->state = RState::Done;
        r->status = LENS_OK;
        c->stats.requests_done++;
        c->stats.proposals_done += r->n;
        const double us =
            std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - r->t_submit).count();
        if (c->lat_ring.size() < kLatencyWindow) c->lat_ring.push_back(us);
        else c->lat_ring[c->lat_pos] = us;
        c->lat_pos = (c->lat_pos + 1) % kLatencyWindow;
        c->stats.latency_max_us = std::max(c->stats.latency_max_us, us);
    } else {
        r->state = RState::Error;
        c->stats.requests_failed++;
    }
    r->lens->requests--;
    if (r->resident) {
        r->resident = false;
        c->resident--;
    }
    r->result.clear();
    r->result.shrink_to_fit();
    r->params.clear();
    r->params.shrink_to_fit();
}

// Serving slot layout in bytes: tables | params | prep | out on the device,
// tables | params | out in pinned host memory, so that one copy moves a
// batch's lookup tables and parameter rows together.
struct SlotLayout {
    size_t o_geom, o_ls, o_lo, o_cnt, o_ps, o_pm;   // inside the tables
    size_t params, pc, out;                         // device offsets
    size_t h_out;                                   // host offset of out
    size_t dev_bytes, host_bytes;                   // per slot
};

SlotLayout slot_layout()
{
    SlotLayout l{};
    size_t o = 0;
    l.o_geom = o;
    o += align_up((size_t)kBatchPieces * sizeof(LensGeom), kAlign);
    l.o_ls = o;
    o += align_up((size_t)2 * kBatchPieces * 4, kAlign);   // every piece's start, one end per group
    l.o_lo = o;
    o += align_up((size_t)kBatchPieces * 8, kAlign);
    l.o_cnt = o;
    o += align_up((size_t)kBatchPieces * 4, kAlign);
    l.o_ps = o;
    o += align_up((size_t)(kBatchPieces + 1) * 8, kAlign);
    l.o_pm = o;
    o += align_up((size_t)kBatchPieces * 4, kAlign);
    l.params = o;
    const size_t pb = align_up((size_t)kBatchMax * lensk::kStride * 8, kAlign);
    l.pc = l.params + pb;
    l.out = l.pc + align_up((size_t)kBatchMax * lensk::kPCBytes, kAlign);
    l.dev_bytes = l.out + align_up((size_t)kBatchMax * 8, kAlign);
    l.h_out = l.params + pb;
    l.host_bytes = l.h_out + align_up((size_t)kBatchMax * 8, kAlign);
    return l;
}

// The serving buffers: kServeDepth batch slots, charged to the HBM budget at
// the first submit (never allocated on the scheduler thread).
void ensure_serving(lens_ctx *c)
{
    if (c->d_serve) return;
    const SlotLayout l = slot_layout();
    const size_t want = (size_t)kServeDepth * l.dev_bytes;
    if (!charge(c, (int64_t)want)) return;
    c->d_serve = dev_alloc(c, want);
    if (!c->d_serve) {
        uncharge(c, (int64_t)want);
        return;
    }
    if (hipHostMalloc((void **)&c->h_serve, (size_t)kServeDepth * l.host_bytes, hipHostMallocDefault) != hipSuccess) {
        dev_free(c, c->d_serve);
        c->d_serve = nullptr;
        uncharge(c, (int64_t)want);
    }
}

// Gather the next batch (smu held): the queued requests in arrival order, each
// giving its proposals not yet placed, until the batch holds kBatchMax
// proposals, kBatchPieces pieces or kBatchWork sub-pixel evaluations.  A
// request that has no work on the device yet joins only while fewer than
// max_inflight requests do; a request that does not fit is cut, and its rest
// goes to the next batch.
bool form_batch(lens_ctx *c, SBatch *b)
{
    double work = 0.0;
    int64_t n = 0;
    for (size_t qi = 0; qi < c->queue.size(); ++qi) {
        Request *r = c->queue[qi];
        if (r->cancel || r->status != LENS_PENDING) continue;
        if (!r->resident && c->resident >= c->max_inflight) continue;
        const int64_t rem = r->n - r->next_tile;
        if (rem <= 0) continue;
        const Lens *L = r->lens;
        const double per = std::max(1.0, (double)L->needed * L->g.s * L->g.s);
        int64_t take = std::min<int64_t>(rem, kBatchMax - n);
        // the first piece always gets at least one proposal
        take = std::min<int64_t>(take, std::max<int64_t>(n == 0 ? 1 : 0, (int64_t)((kBatchWork - work) / per)));
        if (take <= 0) break;
        b->pieces.push_back(Piece{r, r->next_tile, take, n});
        r->next_tile += take;
        r->tiles_running++;
        r->state = RState::Running;
        if (!r->resident) {
            r->resident = true;
            c->resident++;
        }
        n += take;
        work += per * (double)take;
        if (n >= kBatchMax || (int)b->pieces.size() >= kBatchPieces || work >= kBatchWork) break;
    }
    // fully placed requests leave the queue; cancelled ones with nothing on the device finish
    for (size_t qi = 0; qi < c->queue.size();) {
        Request *r = c->queue[qi];
        if (r->cancel && r->tiles_running == 0) {
            c->queue.erase(c->queue.begin() + (long)qi);
            finish_request(c, r);
            c->dcv.notify_all();
        } else if (r->next_tile >= r->n) {
            c->queue.erase(c->queue.begin() + (long)qi);
        } else {
            ++qi;
        }
    }
    b->n = n;
    return n > 0;
}

// Enqueue one batch on its slot's stream (smu held): the tables and parameter
// rows in one copy, the prep step over the whole batch (per-piece model codes
// when they differ), one persistent launch per lens group, the results back,
// and an event.
hipError_t launch_serving_batch(lens_ctx *c, SBatch &b)
{
    const SlotLayout l = slot_layout();
    char *hb = c->h_serve + (size_t)b.slot * l.host_bytes;
    char *db = (char *)c->d_serve + (size_t)b.slot * l.dev_bytes;
    hipStream_t hs = c->sstreams[b.slot % kServeStreams];
    const int np = (int)b.pieces.size();
    std::vector<Lens *> Ls(np);
    std::vector<int64_t> counts(np), off(np + 1, 0);
    std::vector<int> hmodel(np);
    bool one_model = true;
    for (int i = 0; i < np; ++i) {
        const Piece &pc = b.pieces[i];
        Ls[i] = pc.req->lens;
        counts[i] = pc.n;
        off[i + 1] = off[i] + pc.n;
        hmodel[i] = Ls[i]->prep_code;
        one_model = one_model && hmodel[i] == hmodel[0];
        memcpy(hb + l.params + (size_t)pc.at * lensk::kStride * 8, pc.req->params.data() + pc.off * lensk::kStride,
               (size_t)pc.n * lensk::kStride * 8);
    }
    BatchGroups bg;
    group_batch(c, Ls, counts.data(), off.data(), &bg);
    memcpy(hb + l.o_geom, bg.geom.data(), bg.geom.size() * sizeof(LensGeom));
    memcpy(hb + l.o_ls, bg.lstart.data(), bg.lstart.size() * 4);
    memcpy(hb + l.o_lo, bg.lout.data(), bg.lout.size() * 8);
    memcpy(hb + l.o_ps, off.data(), (size_t)(np + 1) * 8);
    memcpy(hb + l.o_pm, hmodel.data(), (size_t)np * 4);
    double *d_par = (double *)(db + l.params);
    lensk::PropBlock *d_pc = (lensk::PropBlock *)(db + l.pc);
    double *d_out = (double *)(db + l.out);
    hipError_t e = hipMemcpyAsync(db, hb, l.params + (size_t)b.n * lensk::kStride * 8, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = one_model ? lensk::launch_prep(d_par, b.n, d_pc, hmodel[0], nullptr, nullptr, 0, hs)
                      : lensk::launch_prep(d_par, b.n, d_pc, 0, (const int64_t *)(db + l.o_ps),
                                           (const int *)(db + l.o_pm), np, hs);
    if (e == hipSuccess)
        e = launch_groups(bg, hs, (const LensGeom *)(db + l.o_geom), (const int *)(db + l.o_ls),
                          (const int64_t *)(db + l.o_lo), d_pc, d_out, (unsigned int *)(db + l.o_cnt));
    if (e == hipSuccess) e = hipMemcpyAsync(hb + l.h_out, d_out, (size_t)b.n * 8, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b.ev, hs);
    return e;
}

// A batch is done (or failed): results to its requests, finished requests
// answered (smu held).
void settle_batch(lens_ctx *c, SBatch &b, bool ok)
{
    const SlotLayout l = slot_layout();
    const double *ho = (const double *)(c->h_serve + (size_t)b.slot * l.host_bytes + l.h_out);
    for (const Piece &pc : b.pieces) {
        Request *r = pc.req;
        if (!ok) r->status = LENS_EDEVICE;
        else if (!r->cancel && r->status == LENS_PENDING)
            memcpy(r->result.data() + pc.off, ho + pc.at, (size_t)pc.n * 8);
        r->tiles_running--;
        r->done += pc.n;
        if (r->tiles_running == 0 && (r->done >= r->n || r->cancel || r->status != LENS_PENDING)) {
            auto it = std::find(c->queue.begin(), c->queue.end(), r);
            if (it != c->queue.end()) c->queue.erase(it);
            finish_request(c, r);
        }
    }
    if (b.ev) (void)hipEventDestroy(b.ev);
    b.ev = nullptr;
    c->slot_busy[b.slot] = false;
}

// Retire finished batches (smu held).  Returns true if anything finished.
bool retire(lens_ctx *c)
{
    bool any = false;
    for (size_t i = 0; i < c->running.size();) {
        SBatch &b = c->running[i];
        const hipError_t q = hipEventQuery(b.ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        if (q != hipSuccess) c->dev_error.store(1);
        settle_batch(c, b, q == hipSuccess);
        if (i + 1 != c->running.size()) c->running[i] = std::move(c->running.back());
        c->running.pop_back();
        any = true;
    }
    if (c->dev_error.load()) {
        // sticky failure: every request with nothing left on the device fails
        for (size_t qi = 0; qi < c->queue.size();) {
            Request *r = c->queue[qi];
            if (r->tiles_running == 0) {
                c->queue.erase(c->queue.begin() + (long)qi);
                r->status = LENS_EDEVICE;
                finish_request(c, r);
                any = true;
            } else {
                ++qi;
            }
        }
    }
    return any;
}

// Launch batches while a slot is free and work is placeable (smu held).
void admit(lens_ctx *c)
{
    while ((int)c->running.size() < kServeDepth && !c->dev_error.load() && c->d_serve && !c->queue.empty()) {
        int slot = 0;
        while (slot < kServeDepth && c->slot_busy[slot]) ++slot;
        if (slot == kServeDepth) return;
        SBatch b;
        b.slot = slot;
        if (!form_batch(c, &b)) return;
        c->slot_busy[slot] = true;
        const hipError_t e = launch_serving_batch(c, b);
        if (e != hipSuccess) {
            c->dev_error.store(1);
            settle_batch(c, b, false);
            return;
        }
        c->stats.launches++;
        c->stats.batch_pieces += (int64_t)b.pieces.size();
        c->running.push_back(std::move(b));
    }
}

void scheduler_main(lens_ctx *c)
{
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(c->smu);
    while (true) {
        if (retire(c)) c->dcv.notify_all();
        admit(c);
        if (c->dev_error.load() && retire(c)) c->dcv.notify_all();
        if (c->stop && c->running.empty()) break;
        if (c->running.empty()) {
            c->scv.wait(lk, [&] { return c->stop || (!c->queue.empty() && !c->dev_error.load()); });
        } else {
            // batches in flight: poll their events without holding the lock for long
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

}  // namespace

extern "C" lens_status lens_submit(lens_ctx *c, lens_id id, const double *params, int64_t n, double *out,
                                   lens_req *out_req)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || !out_req || (n > 0 && (!params || !out))) return fail(c, LENS_EINVAL, "bad params/out/n");
    Lens *L = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->lenses.find(id);
        if (it == c->lenses.end()) return fail(c, LENS_ENOENT, "unknown lens id");
        L = it->second;
        std::lock_guard<std::mutex> sl(c->smu);
        ensure_serving(c);  // batch buffers are allocated here, never on the scheduler thread
        if (!c->d_serve) return fail(c, LENS_ENOMEM, "HBM budget exhausted (serving buffers)");
        if (c->nonblocking) {
            int waiting = 0;   // queued requests with nothing on the device yet
            for (const Request *q : c->queue) waiting += q->resident ? 0 : 1;
            if (c->resident + waiting >= c->max_inflight) return fail(c, LENS_EAGAIN, "all serving slots busy");
        }
        Request *r = new Request();
        r->id = c->next_req++;
        r->lens = L;
        r->n = n;
        r->params.assign(params, params + n * lensk::kStride);
        r->result.assign((size_t)n, 0.0);
        r->out = out;
        r->t_submit = std::chrono::steady_clock::now();
        L->requests++;
        c->reqs[r->id] = r;
        c->stats.requests_submitted++;
        *out_req = r->id;
        if (n == 0) {
            finish_request(c, r);
        } else {
            c->queue.push_back(r);
        }
    }
    c->scv.notify_all();
    return LENS_OK;
}

namespace {
lens_status final_status(lens_ctx *c, Request *r)
{
    // smu held; returns the request's final answer and forgets it
    lens_status s = r->status;
    c->reqs.erase(r->id);
    delete r;
    return s;
}
bool is_final(const Request *r)
{
    return r->state == RState::Done || r->state == RState::Error || r->state == RState::Canceled;
}
}  // namespace

extern "C" lens_status lens_poll(lens_ctx *c, lens_req req)
{
    if (!c) return LENS_EINVAL;
    std::lock_guard<std::mutex> lk(c->smu);
    auto it = c->reqs.find(req);
    if (it == c->reqs.end()) return fail(c, LENS_ENOENT, "unknown request id");
    if (!is_final(it->second)) return LENS_PENDING;
    return final_status(c, it->second);
}

extern "C" lens_status lens_wait(lens_ctx *c, lens_req req, int64_t timeout_us)
{
    if (!c) return LENS_EINVAL;
    std::unique_lock<std::mutex> lk(c->smu);
    auto it = c->reqs.find(req);
    if (it == c->reqs.end()) return fail(c, LENS_ENOENT, "unknown request id");
    Request *r = it->second;
    auto pred = [&] { return is_final(r); };
    if (timeout_us < 0) c->dcv.wait(lk, pred);
    else if (!c->dcv.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) return LENS_ETIMEDOUT;
    return final_status(c, r);
}

extern "C" lens_status lens_cancel(lens_ctx *c, lens_req req)
{
    if (!c) return LENS_EINVAL;
    std::unique_lock<std::mutex> lk(c->smu);
    auto it = c->reqs.find(req);
    if (it == c->reqs.end()) return fail(c, LENS_ENOENT, "unknown request id");
    Request *r = it->second;
    if (!is_final(r)) {
        r->cancel = true;
        if (r->tiles_running == 0) {
            auto q = std::find(c->queue.begin(), c->queue.end(), r);
            if (q != c->queue.end()) c->queue.erase(q);
            finish_request(c, r);
        } else {
            c->dcv.wait(lk, [&] { return is_final(r); });
        }
    }
    c->reqs.erase(r->id);
    delete r;
    return LENS_OK;
}

extern "C" lens_status lens_reset_stats(lens_ctx *c)
{
    if (!c) return LENS_EINVAL;
    std::lock_guard<std::mutex> lk(c->smu);
    c->stats = lens_stats{};
    c->lat_ring.clear();
    c->lat_pos = 0;
    return LENS_OK;
}

extern "C" lens_status lens_get_stats(lens_ctx *c, lens_stats *out)
{
    if (!c || !out) return LENS_EINVAL;
    std::lock_guard<std::mutex> lk(c->smu);
    *out = c->stats;
    out->queued = (int64_t)c->queue.size();
    out->inflight = (int64_t)c->resident;
    out->hbm_budget_bytes = c->budget;
    out->hbm_used_bytes = c->used.load();
    // nearest-rank quantiles of the latency window
    std::vector<double> w(c->lat_ring);
    out->latency_count = (int64_t)w.size();
    auto rank = [&](double q) {
        const size_t k = (size_t)std::ceil(q * (double)w.size()) - 1;
        std::nth_element(w.begin(), w.begin() + k, w.end());
        return w[k];
    };
    out->latency_p50_us = w.empty() ? 0.0 : rank(0.50);
    out->latency_p99_us = w.empty() ? 0.0 : rank(0.99);
    return LENS_OK;
}

extern "C" lens_status lens_selftest(lens_ctx *c, int32_t which, double *result)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!result || (which != 0 && which != 1)) return fail(c, LENS_EINVAL, "unknown self-test");
    DeviceGuard dg(c->device);
    // D = A B, A 16x32 and B 32x16 with small integers (exact in BF16, FP16 and FP32)
    const bool f16 = which == 1;
    uint16_t (*rn)(float) = f16 ? f16_rn_host : bf16_rn_host;
    float (*val)(uint16_t) = f16 ? f16_to_float : bf16_to_float;
    std::vector<uint16_t> ha(16 * 32), hb(32 * 16);
    std::vector<double> ref(16 * 16, 0.0);
    for (int i = 0; i < 16; ++i)
        for (int kk = 0; kk < 32; ++kk) ha[i * 32 + kk] = rn((float)((i * 7 + kk * 3) % 11 - 5));
    for (int kk = 0; kk < 32; ++kk)
        for (int j = 0; j < 16; ++j) hb[kk * 16 + j] = rn((float)((kk * 5 + j * 2) % 9 - 4));
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j)
            for (int kk = 0; kk < 32; ++kk) ref[i * 16 + j] += (double)val(ha[i * 32 + kk]) * val(hb[kk * 16 + j]);
    std::lock_guard<std::mutex> lk(c->sync_mu);
    void *dbuf = nullptr;
    std::unique_lock<std::mutex> hold;
    lens_status rs = stream_scratch(c, c->stream, 4096, &dbuf, &hold);
    if (rs != LENS_OK) return rs;
    uint16_t *da = (uint16_t *)dbuf, *db = da + 16 * 32;
    float *dd = (float *)((char *)dbuf + 2048);
    std::vector<float> hd(256);
    hipError_t e = hipMemcpyAsync(da, ha.data(), ha.size() * 2, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(db, hb.data(), hb.size() * 2, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = lensk::launch_mfma_probe(f16, da, db, dd, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), dd, 256 * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lens_selftest");
    double err = 0.0;
    for (int i = 0; i < 256; ++i) err = std::max(err, std::fabs((double)hd[i] - ref[i]));
    *result = err;
    return LENS_OK;
}

extern "C" lens_status lens_peak_rate(lens_ctx *c, int32_t op, double *rate)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!rate || op < 0 || op >= LENS_PEAK_COUNT) return fail(c, LENS_EINVAL, "unknown instruction kind");
    DeviceGuard dg(c->device);
    // eight workgroups of four waves per CU: eight waves per SIMD
    const int nt = lensk::peak_threads(), grid = 8 * c->num_cus;
    std::lock_guard<std::mutex> lk(c->sync_mu);
    void *dbuf = nullptr;
    std::unique_lock<std::mutex> hold;
    lens_status rs = stream_scratch(c, c->stream, (size_t)grid * nt * 8, &dbuf, &hold);
    if (rs != LENS_OK) return rs;
    double *out = (double *)dbuf;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // one timed launch of n rounds, in milliseconds
    auto timed = [&](int n, float *ms) {
        hipError_t r = hipEventRecord(e0, c->stream);
        if (r == hipSuccess) r = lensk::launch_peak(op, grid, n, out, c->stream);
        if (r == hipSuccess) r = hipEventRecord(e1, c->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
        return r;
    };
    // a warm-up launch (the first one of a kernel also loads its code), a
    // sizing launch (0.4-2 ms at the expected rates), then three of ~25 ms
    const int n0 = 4096;
    float t0 = 0.f, best = 1e30f;
    if (e == hipSuccess) e = timed(n0, &t0);
    if (e == hipSuccess) e = timed(n0, &t0);
    const int n = (int)std::min(200.0 * n0, std::max(64.0, n0 * 25.0 / std::max(t0, 1e-3f)));
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        float ms = 0.f;
        e = timed(n, &ms);
        if (e == hipSuccess) best = std::min(best, ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(c, e, "lens_peak_rate");
    *rate = (double)grid * nt * n * lensk::peak_ops_per_round(op) / (best * 1e-3);
    return LENS_OK;
}

// ---------------------------------------------------------------------------
// sampler loop on the device: Philox4x32-10 words and stretch-move ensembles
// ---------------------------------------------------------------------------
extern "C" lens_status lens_philox4x32_10(lens_ctx *c, const uint32_t *ctr, const uint32_t *key, int64_t n,
                                          uint32_t *out)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!ctr || !key || n < 0 || (n > 0 && !out)) return fail(c, LENS_EINVAL, "bad ctr/key/out/n");
    if (n > ((int64_t)1 << 32)) return fail(c, LENS_EINVAL, "n above 2^32 (the counter word would repeat)");
    if (n == 0) return LENS_OK;
    DeviceGuard dg(c->device);
    std::lock_guard<std::mutex> lk(c->sync_mu);
    void *dbuf = nullptr;
    std::unique_lock<std::mutex> hold;
    lens_status rs = stream_scratch(c, c->stream, (size_t)n * 16, &dbuf, &hold);
    if (rs != LENS_OK) return rs;
    hipError_t e = lensk::launch_philox_words(ctr, key, n, (uint32_t *)dbuf, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dbuf, (size_t)n * 16, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lens_philox4x32_10");
    return LENS_OK;
}

namespace {

// the ensemble with a call reference taken (drop it with ensemble_done)
Ensemble *ensemble_use(lens_ctx *c, lens_ens id)
{
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->ensembles.find(id);
    if (it == c->ensembles.end()) return nullptr;
    it->second->users++;
    return it->second;
}

void ensemble_done(lens_ctx *c, Ensemble *E)
{
    std::lock_guard<std::mutex> lk(c->mu);
    E->users--;
}

void free_ensemble(lens_ctx *c, Ensemble *E)
{
    if (E->slab) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, E->slab);
        uncharge(c, (int64_t)E->bytes);
    }
    if (E->L) release(c, E->L);
    delete E;
}

}  // namespace

extern "C" lens_status lens_ensemble_create(lens_ctx *c, lens_id id, const lens_ensemble_desc *d, lens_ens *out)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (!d || !out || !d->lo || !d->hi || !d->init) return fail(c, LENS_EINVAL, "null descriptor, array or output");
    const int W = d->walkers;
    if (W < 4 || W > (1 << 24) || (W & 1)) return fail(c, LENS_EINVAL, "walkers must be even, 4..2^24");
    if (!(d->stretch > 1.0) || !std::isfinite(d->stretch)) return fail(c, LENS_EINVAL, "stretch must be finite and > 1");
    int dfree = 0;
    for (int s = 0; s < lensk::kStride; ++s) {
        if (!std::isfinite(d->lo[s]) || !std::isfinite(d->hi[s]) || d->lo[s] > d->hi[s])
            return fail(c, LENS_EINVAL, "box bounds must be finite with lo <= hi");
        dfree += d->hi[s] > d->lo[s];
    }
    if (dfree == 0) return fail(c, LENS_EINVAL, "the box fixes every slot");
    for (int64_t k = 0; k < W; ++k)
        for (int s = 0; s < lensk::kStride; ++s) {
            const double v = d->init[k * lensk::kStride + s];
            if (!(v >= d->lo[s] && v <= d->hi[s])) {
                char msg[96];
                snprintf(msg, sizeof(msg), "initial walker %lld is outside the box (slot %d)", (long long)k, s);
                return fail(c, LENS_EINVAL, msg);
            }
        }
    Lens *L = acquire(c, id);
    if (!L) return fail(c, LENS_ENOENT, "unknown lens id");
    DeviceGuard dg(c->device);
    auto *E = new Ensemble();
    E->L = L;
    E->W = W;
    E->d = dfree;
    E->a = d->stretch;
    E->seed = d->seed;
    const size_t h = (size_t)W / 2, S = lensk::kStride;
    const size_t o_lo = 0, o_hi = align_up(S * 8, kAlign), o_w = o_hi + align_up(S * 8, kAlign);
    const size_t o_lnp = o_w + align_up((size_t)W * S * 8, kAlign), o_acc = o_lnp + align_up((size_t)W * 8, kAlign);
    const size_t o_Y = o_acc + align_up((size_t)W * 8, kAlign), o_aux = o_Y + align_up(h * S * 8, kAlign);
    const size_t o_pc = o_aux + align_up(h * 32, kAlign), o_out = o_pc + align_up((size_t)W * lensk::kPCBytes, kAlign);
    E->bytes = o_out + align_up((size_t)W * 8, kAlign);
    if (!charge(c, (int64_t)E->bytes)) {
        E->bytes = 0;
        free_ensemble(c, E);
        return fail(c, LENS_ENOMEM, "HBM budget exhausted (ensemble)");
    }
    E->slab = dev_alloc(c, E->bytes);
    if (!E->slab) {
        uncharge(c, (int64_t)E->bytes);
        E->bytes = 0;
        free_ensemble(c, E);
        return fail(c, LENS_ENOMEM, "device allocation failed (ensemble)");
    }
    char *b = (char *)E->slab;
    E->lo = (double *)(b + o_lo);
    E->hi = (double *)(b + o_hi);
    E->walkers = (double *)(b + o_w);
    E->lnp = (double *)(b + o_lnp);
    E->accepted = (int64_t *)(b + o_acc);
    E->Y = (double *)(b + o_Y);
    E->aux = (double *)(b + o_aux);
    E->pc = (lensk::PropBlock *)(b + o_pc);
    E->out = (double *)(b + o_out);
    std::vector<double> lnp0((size_t)W);
    hipError_t e = hipMemcpyAsync(E->lo, d->lo, S * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(E->hi, d->hi, S * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(E->walkers, d->init, (size_t)W * S * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(E->accepted, 0, (size_t)W * 8, c->stream);
    // lnP of the initial walkers (all inside the box): their lnL
    if (e == hipSuccess) e = launch_lens(L, E->walkers, E->pc, W, E->lnp, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(lnp0.data(), E->lnp, (size_t)W * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_ensemble(c, E);
        return hip_fail(c, e, "lens_ensemble_create");
    }
    for (int k = 0; k < W; ++k)
        if (!(lnp0[(size_t)k] > -INFINITY)) {
            char msg[96];
            snprintf(msg, sizeof(msg), "initial walker %d has lnL = -inf (outside the model's domain)", k);
            free_ensemble(c, E);
            return fail(c, LENS_EINVAL, msg);
        }
    {
        std::lock_guard<std::mutex> lk(c->mu);
        E->id = c->next_ens++;
        c->ensembles[E->id] = E;
    }
    log_line(c, "ensemble %lld on lens %lld: %d walkers, %d free slots, %zu B", (long long)E->id, (long long)id, W,
             dfree, E->bytes);
    *out = E->id;
    return LENS_OK;
}

namespace {
lens_status ensemble_run(lens_ctx *c, Ensemble *E, int64_t iterations, int32_t thin, double *chain,
                         double *chain_lnp, bool store);
}

extern "C" lens_status lens_ensemble_run(lens_ctx *c, lens_ens id, int64_t iterations, int32_t thin,
                                         double *chain, double *chain_lnp)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (iterations < 0) return fail(c, LENS_EINVAL, "iterations must be >= 0");
    const bool store = chain || chain_lnp;
    if (store && thin < 1) return fail(c, LENS_EINVAL, "thin must be >= 1 when a chain is requested");
    Ensemble *E = ensemble_use(c, id);
    if (!E) return fail(c, LENS_ENOENT, "unknown ensemble id");
    lens_status rs = ensemble_run(c, E, iterations, thin, chain, chain_lnp, store);
    ensemble_done(c, E);
    return rs;
}

namespace {

lens_status ensemble_run(lens_ctx *c, Ensemble *E, int64_t iterations, int32_t thin, double *chain,
                         double *chain_lnp, bool store)
{
    std::lock_guard<std::mutex> elk(E->mu);
    DeviceGuard dg(c->device);
    const int W = E->W, h = W / 2;
    const size_t S = lensk::kStride;
    const int64_t nstore = store ? iterations / thin : 0;
    // device chain: [nstore][W][20] then [nstore][W]
    void *dchain = nullptr;
    size_t cbytes = 0;
    if (nstore > 0) {
        cbytes = (size_t)nstore * W * (S + 1) * 8;
        if (!charge(c, (int64_t)cbytes)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (chain)");
        dchain = dev_alloc(c, cbytes);
        if (!dchain) {
            uncharge(c, (int64_t)cbytes);
            return fail(c, LENS_ENOMEM, "device allocation failed (chain)");
        }
    }
    double *cw = (double *)dchain, *cl = cw ? cw + (size_t)nstore * W * S : nullptr;
    hipError_t e = hipSuccess;
    for (int64_t it = 0; it < iterations && e == hipSuccess; ++it) {
        const uint64_t t = (uint64_t)E->t + (uint64_t)it;
        const bool keep = nstore > 0 && (it + 1) % thin == 0 && (it + 1) / thin <= nstore;
        const int64_t slot = keep ? (it + 1) / thin - 1 : 0;
        for (int half = 0; half < 2 && e == hipSuccess; ++half) {
            e = lensk::launch_stretch_propose(W, half, t, E->seed, E->a, E->L->prep_code, E->walkers, E->lo, E->hi,
                                              E->Y, E->aux, E->pc, c->stream);
            if (e == hipSuccess) e = lensk::launch_loglike(E->L->g, E->pc, h, E->out, nullptr, c->stream);
            if (e == hipSuccess)
                e = lensk::launch_stretch_accept(W, half, E->d, E->walkers, E->lnp, E->Y, E->aux, E->out, E->accepted,
                                                 keep ? cw + (size_t)slot * W * S : nullptr,
                                                 keep ? cl + (size_t)slot * W : nullptr, c->stream);
        }
    }
    if (e == hipSuccess && chain && nstore > 0)
        e = hipMemcpyAsync(chain, cw, (size_t)nstore * W * S * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && chain_lnp && nstore > 0)
        e = hipMemcpyAsync(chain_lnp, cl, (size_t)nstore * W * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (dchain) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, dchain);
        uncharge(c, (int64_t)cbytes);
    }
    if (e != hipSuccess) return hip_fail(c, e, "lens_ensemble_run");
    E->t += iterations;
    return LENS_OK;
}

}  // namespace

namespace {

// Advances every ensemble of Es (their mutexes held) by `iterations`: per
// half-step one proposal launch over all their moving halves, the persistent
// multi-lens likelihood launches over the pooled proposals, one acceptance
// launch.
lens_status ensemble_run_many(lens_ctx *c, const std::vector<Ensemble *> &Es, int64_t iterations, int32_t thin,
                              double *const *chains, double *const *chain_lnps)
{
    const int n = (int)Es.size();
    std::vector<int64_t> hoff(n + 1, 0), cnt(n);
    std::vector<Lens *> Ls(n);
    for (int e = 0; e < n; ++e) {
        cnt[e] = Es[e]->W / 2;
        hoff[e + 1] = hoff[e] + cnt[e];
        Ls[e] = Es[e]->L;
    }
    const int64_t tot = hoff[n];
    if (tot > INT_MAX) return fail(c, LENS_EINVAL, "too many walkers for one call");
    BatchGroups bg;
    group_batch(c, Ls, cnt.data(), hoff.data(), &bg);
    std::vector<lensk::EnsembleDev> hens(n);
    for (int e = 0; e < n; ++e) {
        const Ensemble *E = Es[e];
        lensk::EnsembleDev &D = hens[e];
        D.W = E->W;
        D.d = E->d;
        D.code = E->L->prep_code;
        D.pad = 0;
        D.seed = E->seed;
        D.t0 = E->t;
        D.a = E->a;
        D.walkers = E->walkers;
        D.lnp = E->lnp;
        D.accepted = E->accepted;
        D.lo = E->lo;
        D.hi = E->hi;
        D.off = hoff[e];
    }
    // chain rows kept per ensemble, staged on the device: [nstore][W][20] then [nstore][W]
    const bool store = chains || chain_lnps;
    const int64_t nstore = store ? iterations / thin : 0;
    std::vector<size_t> coff(n + 1, 0);
    for (int e = 0; e < n; ++e)
        coff[e + 1] = coff[e] + (size_t)nstore * Es[e]->W * (lensk::kStride + 1);
    // device: ensembles | hoff | Y | aux | pc | lnL | geoms | lstart | lout | counters | chains
    const size_t S = lensk::kStride;
    const size_t b_ens = align_up((size_t)n * sizeof(lensk::EnsembleDev), kAlign);
    const size_t b_hoff = align_up((size_t)(n + 1) * 8, kAlign);
    const size_t b_Y = align_up((size_t)tot * S * 8, kAlign), b_aux = align_up((size_t)tot * 32, kAlign);
    const size_t b_pc = align_up((size_t)tot * lensk::kPCBytes, kAlign), b_out = align_up((size_t)tot * 8, kAlign);
    const size_t b_geom = align_up(bg.geom.size() * sizeof(LensGeom), kAlign);
    const size_t b_ls = align_up(bg.lstart.size() * 4, kAlign), b_lo = align_up(bg.lout.size() * 8, kAlign);
    const size_t b_cnt = align_up(bg.gs.size() * 4 + 4, kAlign);
    const size_t b_chain = align_up(coff[n] * 8, kAlign);
    const size_t bytes = b_ens + b_hoff + b_Y + b_aux + b_pc + b_out + b_geom + b_ls + b_lo + b_cnt + b_chain;
    if (!charge(c, (int64_t)bytes)) return fail(c, LENS_ENOMEM, "HBM budget exhausted (multi-ensemble step)");
    void *dev = dev_alloc(c, bytes);
    if (!dev) {
        uncharge(c, (int64_t)bytes);
        return fail(c, LENS_ENOMEM, "device allocation failed (multi-ensemble step)");
    }
    char *b = (char *)dev;
    auto *d_ens = (lensk::EnsembleDev *)b;
    auto *d_hoff = (int64_t *)(b += b_ens);
    auto *d_Y = (double *)(b += b_hoff);
    auto *d_aux = (double *)(b += b_Y);
    auto *d_pc = (lensk::PropBlock *)(b += b_aux);
    auto *d_out = (double *)(b += b_pc);
    auto *d_geom = (LensGeom *)(b += b_out);
    auto *d_ls = (int *)(b += b_geom);
    auto *d_lo = (int64_t *)(b += b_ls);
    auto *d_cnt = (unsigned int *)(b += b_lo);
    auto *d_chain = (double *)(b += b_cnt);
    for (int e = 0; e < n; ++e) {
        hens[e].chain_w = nstore > 0 ? d_chain + coff[e] : nullptr;
        hens[e].chain_lnp = nstore > 0 ? d_chain + coff[e] + (size_t)nstore * Es[e]->W * S : nullptr;
    }
    hipError_t e = hipMemcpyAsync(d_ens, hens.data(), (size_t)n * sizeof(lensk::EnsembleDev), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_hoff, hoff.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_geom, bg.geom.data(), bg.geom.size() * sizeof(LensGeom), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_ls, bg.lstart.data(), bg.lstart.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_lo, bg.lout.data(), bg.lout.size() * 8, hipMemcpyHostToDevice, c->stream);
    for (int64_t it = 0; it < iterations && e == hipSuccess; ++it) {
        const bool keep = nstore > 0 && (it + 1) % thin == 0 && (it + 1) / thin <= nstore;
        const int64_t slot = keep ? (it + 1) / thin - 1 : -1;
        for (int half = 0; half < 2 && e == hipSuccess; ++half) {
            e = lensk::launch_stretch_many(half, it, d_ens, d_hoff, n, tot, d_Y, d_aux, d_pc, 0, nullptr, -1,
                                           c->stream);
            if (e == hipSuccess) e = launch_groups(bg, c->stream, d_geom, d_ls, d_lo, d_pc, d_out, d_cnt);
            if (e == hipSuccess)
                e = lensk::launch_stretch_many(half, it, d_ens, d_hoff, n, tot, d_Y, d_aux, d_pc, 1, d_out, slot,
                                               c->stream);
        }
    }
    for (int k = 0; k < n && e == hipSuccess && nstore > 0; ++k) {
        const size_t rows = (size_t)nstore * Es[k]->W;
        if (chains && chains[k])
            e = hipMemcpyAsync(chains[k], d_chain + coff[k], rows * S * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && chain_lnps && chain_lnps[k])
            e = hipMemcpyAsync(chain_lnps[k], d_chain + coff[k] + rows * S, rows * 8, hipMemcpyDeviceToHost, c->stream);
    }
    hipError_t es = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = es;
    dev_free(c, dev);
    uncharge(c, (int64_t)bytes);
    if (e != hipSuccess) return hip_fail(c, e, "lens_ensemble_run_many");
    for (Ensemble *E : Es) E->t += iterations;
    return LENS_OK;
}

}  // namespace

extern "C" lens_status lens_ensemble_run_many(lens_ctx *c, int32_t n, const lens_ens *ids, int64_t iterations,
                                              int32_t thin, double *const *chains, double *const *chain_lnps)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    if (n < 0 || (n > 0 && !ids)) return fail(c, LENS_EINVAL, "bad ensemble list");
    if (iterations < 0) return fail(c, LENS_EINVAL, "iterations must be >= 0");
    if ((chains || chain_lnps) && thin < 1) return fail(c, LENS_EINVAL, "thin must be >= 1 when chains are requested");
    std::vector<lens_ens> sorted(ids, ids + n);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(c, LENS_EINVAL, "an ensemble is listed twice");
    std::vector<Ensemble *> Es;
    for (int i = 0; i < n; ++i) {
        Ensemble *E = ensemble_use(c, ids[i]);
        if (!E) {
            for (Ensemble *x : Es) ensemble_done(c, x);
            return fail(c, LENS_ENOENT, "unknown ensemble id");
        }
        Es.push_back(E);
    }
    lens_status rs = LENS_OK;
    {
        // one call on an ensemble at a time; locks taken in id order
        std::vector<Ensemble *> byid(Es);
        std::sort(byid.begin(), byid.end(), [](const Ensemble *x, const Ensemble *y) { return x->id < y->id; });
        std::vector<std::unique_lock<std::mutex>> locks;
        locks.reserve(byid.size());
        for (Ensemble *E : byid) locks.emplace_back(E->mu);
        if (n > 0 && iterations > 0) {
            DeviceGuard dg(c->device);
            rs = ensemble_run_many(c, Es, iterations, thin, chains, chain_lnps);
        }
    }
    for (Ensemble *E : Es) ensemble_done(c, E);
    return rs;
}

extern "C" lens_status lens_ensemble_get(lens_ctx *c, lens_ens id, double *walkers, double *lnp, int64_t *accepted,
                                         int64_t *iteration)
{
    lens_status st = check_ctx(c);
    if (st != LENS_OK) return st;
    Ensemble *E = ensemble_use(c, id);
    if (!E) return fail(c, LENS_ENOENT, "unknown ensemble id");
    std::unique_lock<std::mutex> elk(E->mu);
    DeviceGuard dg(c->device);
    const int W = E->W;
    hipError_t e = hipSuccess;
    if (walkers)
        e = hipMemcpyAsync(walkers, E->walkers, (size_t)W * lensk::kStride * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && lnp) e = hipMemcpyAsync(lnp, E->lnp, (size_t)W * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && accepted)
        e = hipMemcpyAsync(accepted, E->accepted, (size_t)W * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (iteration) *iteration = E->t;
    elk.unlock();
    ensemble_done(c, E);
    if (e != hipSuccess) return hip_fail(c, e, "lens_ensemble_get");
    return LENS_OK;
}

extern "C" lens_status lens_ensemble_destroy(lens_ctx *c, lens_ens id)
{
    if (!c) return LENS_EINVAL;
    Ensemble *E = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->ensembles.find(id);
        if (it == c->ensembles.end()) return fail(c, LENS_ENOENT, "unknown ensemble id");
        E = it->second;
        if (E->users > 0) return fail(c, LENS_EBUSY, "ensemble is in use by a running call");
        c->ensembles.erase(it);
    }
    DeviceGuard dg(c->device);
    free_ensemble(c, E);
    log_line(c, "ensemble %lld destroyed", (long long)id);
    return LENS_OK;
}
