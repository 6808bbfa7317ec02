// Drives the C-ABI of the library through every entry point on one GPU, for a
// build whose host code (the runtime) carries AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_gpu_runtime_asan.py).  The sanitizers
// report invalid host accesses, use of freed memory and undefined behaviour in
// the runtime's own code: loading, the blocking and multi-lens calls, the
// serving scheduler with cancellations, the sampler ensembles and the error
// paths.  Results are checked only where the library promises bitwise equality
// (the same proposals through different calls) or a sign (-inf outside the
// domain); their accuracy is the parity tests' business.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "lens_api.h"

static int fails = 0;

#define CK(expr)                                                                                       \
    do {                                                                                               \
        const lens_status s_ = (expr);                                                                 \
        if (s_ != LENS_OK) {                                                                           \
            printf("FAIL line %d: %s -> %d (%s)\n", __LINE__, #expr, (int)s_, lens_strerror(s_));     \
            fails++;                                                                                   \
        }                                                                                              \
    } while (0)
#define EXPECT(expr, want)                                                                             \
    do {                                                                                               \
        const lens_status s_ = (expr);                                                                 \
        if (s_ != (want)) {                                                                            \
            printf("FAIL line %d: %s -> %d, expected %d\n", __LINE__, #expr, (int)s_, (int)(want));   \
            fails++;                                                                                   \
        }                                                                                              \
    } while (0)
#define TRUE(cond)                                                                                     \
    do {                                                                                               \
        if (!(cond)) {                                                                                 \
            printf("FAIL line %d: %s\n", __LINE__, #cond);                                             \
            fails++;                                                                                   \
        }                                                                                              \
    } while (0)

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ULL;
double uni()
{
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(g_state >> 11) * 0x1p-53;
}

// the prior box of the survey workloads; slot 19 (gamma) in [1.5, 2.5] for EPL lenses, 0 otherwise
const double kLo[19] = {0.5, 0.5, 0.0, -0.1, -0.1, -0.1, -0.1, 0.05, 0.1, 0.5, 0.5, 0.0, 0.05, 0.1, 0.5, 0.5, 0.0, -1.0, -1.0};
const double kHi[19] = {2.0, 1.0, 3.14159, 0.1, 0.1, 0.1, 0.1, 0.5, 1.0, 4.0, 1.0, 3.14159, 0.5, 1.0, 4.0, 1.0, 3.14159, 1.0, 1.0};

std::vector<double> proposals(int64_t n, bool epl, int every_invalid)
{
    std::vector<double> p((size_t)n * LENS_PARAM_STRIDE);
    for (int64_t i = 0; i < n; ++i) {
        double *v = &p[(size_t)i * LENS_PARAM_STRIDE];
        for (int s = 0; s < 19; ++s) v[s] = kLo[s] + (kHi[s] - kLo[s]) * uni();
        v[19] = epl ? 1.5 + uni() : 0.0;
        if (every_invalid > 0 && i % every_invalid == every_invalid - 1) v[1] = 1.5;   // q_m > 1
    }
    return p;
}

struct Image {
    int ny, nx, s, k;
    double dpix;
    std::vector<double> psf, data, sigma;
    std::vector<uint8_t> mask;
};

Image make_image(int n, int s, int k, double dpix)
{
    Image im{n, n, s, k, dpix, {}, {}, {}, {}};
    double sum = 0.0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            const double r2 = (a - k / 2) * (a - k / 2) + (b - k / 2) * (b - k / 2);
            im.psf.push_back(std::exp(-r2 / (0.18 * k * k)));
            sum += im.psf.back();
        }
    for (double &v : im.psf) v /= sum;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            const double X = (x - 0.5 * (n - 1)) * dpix, Y = (y - 0.5 * (n - 1)) * dpix;
            const double r = std::sqrt(X * X + Y * Y);
            im.data.push_back(0.3 * std::exp(-r * r / 0.2) + 0.1 * std::exp(-(r - 1.0) * (r - 1.0) / 0.02) +
                              0.01 * (uni() - 0.5));
            im.sigma.push_back(0.01);
            im.mask.push_back(r < 0.45 * n * dpix ? 1 : 0);
        }
    return im;
}

lens_data_desc desc_of(const Image &im)
{
    lens_data_desc d;
    memset(&d, 0, sizeof(d));
    d.ny = im.ny;
    d.nx = im.nx;
    d.pixel_scale = im.dpix;
    d.supersample = im.s;
    d.psf_size = im.k;
    d.psf = im.psf.data();
    d.data = im.data.data();
    d.sigma = im.sigma.data();
    d.mask = im.mask.data();
    return d;
}

bool same_bits(const std::vector<double> &a, const double *b, size_t n)
{
    return memcmp(a.data(), b, n * sizeof(double)) == 0;
}

}  // namespace

int main()
{
    lens_ctx *c = nullptr;
    CK(lens_init(nullptr, &c));
    if (!c) return 1;
    const Image small = make_image(40, 2, 7, 0.1), mid = make_image(64, 4, 11, 0.05);

    // lenses: explicit FP32, FP16 split, NNLS, EPL, two components per galaxy
    lens_id A = 0, B = 0, Cn = 0, D = 0, E = 0;
    lens_data_desc d = desc_of(small);
    CK(lens_load_data(c, &d, &A));
    d = desc_of(mid);
    d.precision = LENS_PREC_F16_SPLIT;
    CK(lens_load_data(c, &d, &B));
    d = desc_of(small);
    d.amplitudes = LENS_AMP_NNLS;
    CK(lens_load_data(c, &d, &Cn));
    d = desc_of(mid);
    d.mass_model = LENS_MASS_EPL;
    CK(lens_load_data(c, &d, &D));
    d = desc_of(small);
    d.amplitudes = LENS_AMP_NNLS;
    d.light_model = LENS_LIGHT_DOUBLE;
    const double nfix[4] = {1.0, 4.0, 1.0, 4.0};
    memcpy(d.sersic_n, nfix, sizeof(nfix));
    CK(lens_load_data(c, &d, &E));
    lens_info info;
    for (lens_id id : {A, B, Cn, D, E}) CK(lens_get_info(c, id, &info));
    CK(lens_get_info(c, E, &info));
    TRUE(info.n_amplitudes == 4);

    // blocking calls
    const int64_t n = 300;
    std::vector<double> P = proposals(n, false, 7), PE = proposals(n, true, 7);
    std::vector<double> out(n), out2(n), amp((size_t)n * 4);
    CK(lens_loglike_batch(c, A, P.data(), n, out.data()));
    for (int64_t i = 0; i < n; ++i) TRUE(i % 7 == 6 ? std::isinf(out[i]) && out[i] < 0 : std::isfinite(out[i]));
    CK(lens_loglike_amps(c, Cn, P.data(), n, out2.data(), amp.data()));
    CK(lens_loglike_amps(c, E, P.data(), n, out2.data(), amp.data()));
    CK(lens_loglike_batch(c, D, PE.data(), n, out2.data()));
    CK(lens_loglike_batch(c, A, P.data(), 0, out2.data()));

    // device buffers on the default stream: the same bits as the host call
    double *dp = nullptr, *dout = nullptr;
    TRUE(hipMalloc(&dp, (size_t)n * LENS_PARAM_STRIDE * 8) == hipSuccess);
    TRUE(hipMalloc(&dout, (size_t)n * 8) == hipSuccess);
    TRUE(hipMemcpy(dp, P.data(), (size_t)n * LENS_PARAM_STRIDE * 8, hipMemcpyHostToDevice) == hipSuccess);
    CK(lens_loglike_batch_device(c, A, dp, n, dout, nullptr));
    TRUE(hipDeviceSynchronize() == hipSuccess);
    TRUE(hipMemcpy(out2.data(), dout, (size_t)n * 8, hipMemcpyDeviceToHost) == hipSuccess);
    TRUE(same_bits(out, out2.data(), n));
    // the multi-lens call on device buffers: lens A's n proposals then lens B's
    {
        const lens_id ids2[2] = {A, B};
        const int64_t cnt2[2] = {n, n};
        double *mp = nullptr, *mo = nullptr;
        TRUE(hipMalloc(&mp, (size_t)2 * n * LENS_PARAM_STRIDE * 8) == hipSuccess);
        TRUE(hipMalloc(&mo, (size_t)2 * n * 8) == hipSuccess);
        TRUE(hipMemcpy(mp, P.data(), (size_t)n * LENS_PARAM_STRIDE * 8, hipMemcpyHostToDevice) == hipSuccess);
        TRUE(hipMemcpy(mp + n * LENS_PARAM_STRIDE, P.data(), (size_t)n * LENS_PARAM_STRIDE * 8, hipMemcpyHostToDevice) ==
             hipSuccess);
        CK(lens_loglike_multi_device(c, 2, ids2, cnt2, mp, mo, nullptr));
        TRUE(hipDeviceSynchronize() == hipSuccess);
        std::vector<double> mh((size_t)2 * n), refB(n);
        TRUE(hipMemcpy(mh.data(), mo, (size_t)2 * n * 8, hipMemcpyDeviceToHost) == hipSuccess);
        CK(lens_loglike_batch(c, B, P.data(), n, refB.data()));
        TRUE(same_bits(out, mh.data(), n));
        TRUE(same_bits(refB, mh.data() + n, n));
        EXPECT(lens_loglike_multi_device(c, 2, ids2, cnt2, nullptr, mo, nullptr), LENS_EINVAL);
        (void)hipFree(mp);
        (void)hipFree(mo);
    }
    (void)hipFree(dp);
    (void)hipFree(dout);

    // multi-lens calls: two shapes, each twice (capture, then replay)
    for (int rep = 0; rep < 2; ++rep)
        for (int shape = 0; shape < 2; ++shape) {
            const lens_id ids3[3] = {A, B, D};
            const int64_t cnt3[3] = {shape ? 7 : 50, shape ? 3 : 20, shape ? 9 : 30};
            std::vector<double> mp, mo((size_t)(cnt3[0] + cnt3[1] + cnt3[2]));
            for (int j = 0; j < 3; ++j) {
                std::vector<double> pj = proposals(cnt3[j], ids3[j] == D, 5);
                mp.insert(mp.end(), pj.begin(), pj.end());
            }
            CK(lens_loglike_multi(c, 3, ids3, cnt3, mp.data(), mo.data()));
            int64_t off = 0;
            for (int j = 0; j < 3; ++j) {
                std::vector<double> single((size_t)cnt3[j]);
                CK(lens_loglike_batch(c, ids3[j], mp.data() + off * LENS_PARAM_STRIDE, cnt3[j], single.data()));
                TRUE(same_bits(single, mo.data() + off, (size_t)cnt3[j]));
                off += cnt3[j];
            }
        }

    // serving: mixed requests, some cancelled at once
    {
        const int R = 24;
        std::vector<std::vector<double>> rp(R), ro(R);
        std::vector<lens_req> req(R);
        std::vector<lens_id> rl(R);
        for (int r = 0; r < R; ++r) {
            rl[r] = r % 3 == 0 ? A : r % 3 == 1 ? B : D;
            const int64_t m = 1 + (int64_t)(uni() * (r % 5 == 0 ? 9000 : 1500));
            rp[r] = proposals(m, rl[r] == D, 11);
            ro[r].assign((size_t)m, 0.0);
            CK(lens_submit(c, rl[r], rp[r].data(), m, ro[r].data(), &req[r]));
        }
        for (int r = 0; r < R; r += 7) CK(lens_cancel(c, req[r]));
        for (int r = 0; r < R; ++r) {
            if (r % 7 == 0) continue;
            const lens_status s = lens_poll(c, req[r]);
            TRUE(s == LENS_OK || s == LENS_PENDING);
            if (s == LENS_PENDING) CK(lens_wait(c, req[r], -1));
            std::vector<double> alone(ro[r].size());
            CK(lens_loglike_batch(c, rl[r], rp[r].data(), (int64_t)alone.size(), alone.data()));
            TRUE(same_bits(alone, ro[r].data(), alone.size()));
        }
        EXPECT(lens_poll(c, req[1]), LENS_ENOENT);
        lens_stats st;
        CK(lens_get_stats(c, &st));
        TRUE(st.requests_submitted >= R);
    }

    // sampler ensembles: one alone, two pooled, the chain copied back
    {
        const int W = 16;
        double lo[20], hi[20];
        for (int s = 0; s < 19; ++s) {
            lo[s] = kLo[s];
            hi[s] = kHi[s];
        }
        lo[19] = hi[19] = 0.0;
        std::vector<double> init = proposals(W, false, 0);
        lens_ensemble_desc ed;
        memset(&ed, 0, sizeof(ed));
        ed.walkers = W;
        ed.stretch = 2.0;
        ed.lo = lo;
        ed.hi = hi;
        ed.init = init.data();
        lens_ens e1 = 0, e2 = 0, e3 = 0;
        ed.seed = 1;
        CK(lens_ensemble_create(c, A, &ed, &e1));
        ed.seed = 2;
        CK(lens_ensemble_create(c, B, &ed, &e2));
        CK(lens_ensemble_create(c, A, &ed, &e3));
        std::vector<double> chain((size_t)3 * W * 20), chain_lnp((size_t)3 * W);
        CK(lens_ensemble_run(c, e1, 6, 2, chain.data(), chain_lnp.data()));
        const lens_ens both[2] = {e2, e3};
        std::vector<double> pc2((size_t)W * 20), pc3((size_t)W * 20), pl2(W), pl3(W);
        double *const cws[2] = {pc2.data(), pc3.data()};
        double *const cls[2] = {pl2.data(), nullptr};   // a null entry skips that ensemble
        CK(lens_ensemble_run_many(c, 2, both, 3, 3, cws, cls));
        std::vector<double> w((size_t)W * 20), lnp(W);
        std::vector<int64_t> acc(W);
        int64_t it = 0;
        CK(lens_ensemble_get(c, e2, w.data(), lnp.data(), acc.data(), &it));
        TRUE(it == 3);
        EXPECT(lens_unload(c, A), LENS_EBUSY);
        const lens_ens dup[2] = {e1, e1};
        EXPECT(lens_ensemble_run_many(c, 2, dup, 1, 0, nullptr, nullptr), LENS_EINVAL);
        EXPECT(lens_ensemble_run_many(c, 2, both, 1, 0, cws, nullptr), LENS_EINVAL);   // thin < 1 with a chain
        for (lens_ens e : {e1, e2, e3}) CK(lens_ensemble_destroy(c, e));
        EXPECT(lens_ensemble_destroy(c, e1), LENS_ENOENT);
        uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {1, 2}, words[40];
        CK(lens_philox4x32_10(c, ctr, key, 10, words));
    }

    // debug images, PSF crop, self-test
    {
        std::vector<double> img((size_t)small.ny * small.nx);
        std::vector<double> p1 = proposals(1, false, 0);
        CK(lens_model_image(c, A, p1.data(), 0, img.data()));
        CK(lens_model_image(c, A, p1.data(), 1, img.data()));
        int32_t ku = 0;
        CK(lens_psf_crop(mid.psf.data(), mid.k, 0.0, &ku));
        TRUE(ku >= 1 && ku <= mid.k);
        double r = 0.0;
        CK(lens_selftest(c, 0, &r));
    }

    // error paths
    {
        EXPECT(lens_loglike_batch(c, 12345, P.data(), 1, out2.data()), LENS_ENOENT);
        EXPECT(lens_loglike_batch(c, A, nullptr, 1, out2.data()), LENS_EINVAL);
        lens_data_desc bad = desc_of(small);
        bad.psf_size = 6;
        lens_id x = 0;
        EXPECT(lens_load_data(c, &bad, &x), LENS_EINVAL);
        bad = desc_of(small);
        bad.light_model = LENS_LIGHT_LENS;   // needs LENS_AMP_NNLS
        EXPECT(lens_load_data(c, &bad, &x), LENS_EINVAL);
        EXPECT(lens_wait(c, 987654, 0), LENS_ENOENT);
        TRUE(lens_last_error(c) != nullptr);
    }

    // three threads on the context at once: blocking and multi-lens calls,
    // serving with cancellations, ensembles created, run and destroyed
    {
        std::vector<double> Pa = proposals(700, false, 9), Pd = proposals(500, true, 9);
        std::vector<double> refA(700), refD(500);
        CK(lens_loglike_batch(c, A, Pa.data(), 700, refA.data()));
        CK(lens_loglike_batch(c, D, Pd.data(), 500, refD.data()));
        std::atomic<int> bad{0};
        auto blocking = [&]() {
            std::vector<double> o(700), m(1200);
            const lens_id ids[2] = {A, D};
            const int64_t cnt[2] = {700, 500};
            std::vector<double> pm(Pa);
            pm.insert(pm.end(), Pd.begin(), Pd.end());
            for (int r = 0; r < 8; ++r) {
                if (lens_loglike_batch(c, A, Pa.data(), 700, o.data()) != LENS_OK || !same_bits(refA, o.data(), 700))
                    bad++;
                if (lens_loglike_multi(c, 2, ids, cnt, pm.data(), m.data()) != LENS_OK ||
                    !same_bits(refA, m.data(), 700) || !same_bits(refD, m.data() + 700, 500))
                    bad++;
            }
        };
        auto serving = [&]() {
            for (int r = 0; r < 8; ++r) {
                std::vector<double> o1(700), o2(500);
                lens_req q1 = 0, q2 = 0;
                if (lens_submit(c, A, Pa.data(), 700, o1.data(), &q1) != LENS_OK) bad++;
                if (lens_submit(c, D, Pd.data(), 500, o2.data(), &q2) != LENS_OK) bad++;
                if (r % 3 == 0) {
                    if (lens_cancel(c, q2) != LENS_OK) bad++;
                } else if (lens_wait(c, q2, -1) != LENS_OK || !same_bits(refD, o2.data(), 500)) {
                    bad++;
                }
                if (lens_wait(c, q1, -1) != LENS_OK || !same_bits(refA, o1.data(), 700)) bad++;
            }
        };
        auto sampling = [&]() {
            double lo[20], hi[20];
            for (int s = 0; s < 19; ++s) {
                lo[s] = kLo[s];
                hi[s] = kHi[s];
            }
            lo[19] = hi[19] = 0.0;
            std::vector<double> init = proposals(8, false, 0);
            lens_ensemble_desc ed;
            memset(&ed, 0, sizeof(ed));
            ed.walkers = 8;
            ed.stretch = 2.0;
            ed.seed = 3;
            ed.lo = lo;
            ed.hi = hi;
            ed.init = init.data();
            for (int r = 0; r < 4; ++r) {
                lens_ens e = 0;
                if (lens_ensemble_create(c, B, &ed, &e) != LENS_OK) {
                    bad++;
                    continue;
                }
                if (lens_ensemble_run(c, e, 3, 0, nullptr, nullptr) != LENS_OK) bad++;
                if (lens_ensemble_run_many(c, 1, &e, 2, 0, nullptr, nullptr) != LENS_OK) bad++;
                if (lens_ensemble_destroy(c, e) != LENS_OK) bad++;
            }
        };
        // two more threads enqueue device-buffer calls of different sizes on
        // one shared stream: each result must equal its solo run.  Their
        // buffers are allocated, and the stream's scratch sized, before the
        // threads start; they use only the library and that (non-blocking)
        // stream, never the legacy default stream, while other threads
        // capture graphs.
        hipStream_t shared = nullptr;
        TRUE(hipStreamCreateWithFlags(&shared, hipStreamNonBlocking) == hipSuccess);
        struct DevBuf {
            double *p = nullptr, *o = nullptr;
        } bufA, bufD;
        TRUE(hipMalloc(&bufA.p, (size_t)700 * LENS_PARAM_STRIDE * 8) == hipSuccess);
        TRUE(hipMalloc(&bufA.o, (size_t)700 * 8) == hipSuccess);
        TRUE(hipMalloc(&bufD.p, (size_t)500 * LENS_PARAM_STRIDE * 8) == hipSuccess);
        TRUE(hipMalloc(&bufD.o, (size_t)500 * 8) == hipSuccess);
        TRUE(hipMemcpy(bufA.p, Pa.data(), (size_t)700 * LENS_PARAM_STRIDE * 8, hipMemcpyHostToDevice) == hipSuccess);
        TRUE(hipMemcpy(bufD.p, Pd.data(), (size_t)500 * LENS_PARAM_STRIDE * 8, hipMemcpyHostToDevice) == hipSuccess);
        {
            const int64_t c1[1] = {500};
            CK(lens_loglike_batch_device(c, A, bufA.p, 700, bufA.o, shared));
            CK(lens_loglike_multi_device(c, 1, &D, c1, bufD.p, bufD.o, shared));
            TRUE(hipStreamSynchronize(shared) == hipSuccess);
        }
        auto on_shared = [&](lens_id id, const DevBuf &db, int64_t np, const std::vector<double> &ref, bool multi) {
            std::vector<double> o((size_t)np);
            for (int r = 0; r < 10; ++r) {
                const int64_t cnt1[1] = {np};
                const lens_status s = multi ? lens_loglike_multi_device(c, 1, &id, cnt1, db.p, db.o, shared)
                                            : lens_loglike_batch_device(c, id, db.p, np, db.o, shared);
                if (s != LENS_OK ||
                    hipMemcpyAsync(o.data(), db.o, (size_t)np * 8, hipMemcpyDeviceToHost, shared) != hipSuccess ||
                    hipStreamSynchronize(shared) != hipSuccess || !same_bits(ref, o.data(), (size_t)np))
                    bad++;
            }
        };
        std::thread t1(blocking), t2(serving), t3(sampling);
        std::thread t4([&] { on_shared(A, bufA, 700, refA, false); });
        std::thread t5([&] { on_shared(D, bufD, 500, refD, true); });
        t1.join();
        t2.join();
        t3.join();
        t4.join();
        t5.join();
        (void)hipStreamDestroy(shared);
        for (double *x : {bufA.p, bufA.o, bufD.p, bufD.o}) (void)hipFree(x);
        TRUE(bad.load() == 0);
    }

    for (lens_id id : {A, B, Cn, D, E}) CK(lens_unload(c, id));
    EXPECT(lens_unload(c, A), LENS_ENOENT);
    lens_shutdown(c);

    // a tiny HBM budget and non-blocking submission with one slot
    {
        lens_init_opts o;
        memset(&o, 0, sizeof(o));
        o.hbm_budget_bytes = 4 << 10;
        lens_ctx *c2 = nullptr;
        CK(lens_init(&o, &c2));
        lens_data_desc dd = desc_of(mid);
        lens_id x = 0;
        EXPECT(lens_load_data(c2, &dd, &x), LENS_ENOMEM);
        lens_shutdown(c2);
        memset(&o, 0, sizeof(o));
        o.max_inflight = 1;
        o.nonblocking_submit = 1;
        lens_ctx *c3 = nullptr;
        CK(lens_init(&o, &c3));
        dd = desc_of(small);
        CK(lens_load_data(c3, &dd, &x));
        std::vector<double> pp = proposals(4000, false, 0);
        std::vector<std::vector<double>> oo(6, std::vector<double>(4000));
        std::vector<lens_req> rr;
        for (int r = 0; r < 6; ++r) {
            lens_req q = 0;
            const lens_status s = lens_submit(c3, x, pp.data(), 4000, oo[r].data(), &q);
            TRUE(s == LENS_OK || s == LENS_EAGAIN);
            if (s == LENS_OK) rr.push_back(q);
        }
        for (lens_req q : rr) CK(lens_wait(c3, q, -1));
        // shutdown with a request still queued or running
        lens_req q = 0;
        if (lens_submit(c3, x, pp.data(), 4000, oo[0].data(), &q) == LENS_OK) lens_shutdown(c3);
        else lens_shutdown(c3);
    }

    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
