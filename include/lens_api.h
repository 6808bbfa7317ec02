/*
 * lens_api.h -- C ABI of the MI355X batched lens log-likelihood library.
 *
 * The library evaluates, for many proposed parameter vectors at once, the
 * Gaussian log-likelihood of a galaxy-galaxy strong-lens image under the
 * forward model of Cao et al. (2025), "CSST Strong Lensing Preparation: Fast
 * Modelling of Galaxy-Galaxy Strong Lenses in the Big Data Era":
 *   - lens equation beta = theta - alpha(theta)                 (Sec. 2.1, Eq. 1)
 *   - image = lens light(theta) + source light(beta)             (Sec. 2.1, Eq. 2)
 *   - s x s supersampling, binned by the pixel mean               (Sec. 2.1, after Eq. 2)
 *   - PSF convolution of the binned image                         (Sec. 2.1, Eq. 3)
 *   - lnL = sum over the fitting region of ln N(d_i; I_i, sigma_i)  (Sec. 2.2, Eq. 5)
 *   - SIE mass (the elliptical power law at slope 2) + external shear (Sec. 2.4, Eqs. 12-14),
 *     or the elliptical power law at any slope gamma (LENS_MASS_EPL)
 *   - elliptical Sersic light for lens and source                 (Sec. 2.4, Eqs. 8-10)
 * The light amplitudes are explicit parameters by default, or solved by
 * non-negative least squares per proposal (Sec. 2.3, LENS_AMP_NNLS), which
 * also admits the light models of Sec. 3.1.2 and 3.2 (LENS_LIGHT_*).
 *
 * Conventions (each is a reading of a passage the paper leaves open):
 *   - SIE convergence kappa = theta_E / (2 R_p), R_p = sqrt(q x1^2 + x2^2/q)
 *     the elliptical radius of Eq. 10; alpha = 0 at the mass centre.
 *   - shear potential with the sign printed in Eq. 13:
 *     alpha_shear = -(g1 x + g2 y, g2 x - g1 y), origin at the image centre.
 *   - position angles counter-clockwise from +x; x grows with the column
 *     index, y with the row index; the image centre is pixel ((nx-1)/2, (ny-1)/2).
 *   - sub-pixels are the centres of an s x s split of each pixel; the
 *     binned value is their mean; the lens light is centred on the mass.
 *   - b_n is the exact root of Gamma(2n) = 2 gamma(2n, b_n) (Eq. 9).
 *   - the PSF is a true convolution (kernel flipped), k odd, centred at
 *     (k-1)/2, zero outside the image, output of the image's size.
 *   - lnL = -1/2 chi^2 - 1/2 sum_mask ln(2 pi sigma^2), sums over mask pixels.
 *
 * Parameter vector: LENS_PARAM_STRIDE doubles per proposal, row-major
 * [n][20], arcsec and radians:
 *   0 theta_E  1 q_m  2 phi_m  3 x_m  4 y_m  5 g1  6 g2
 *   7 I_l  8 R_l  9 n_l  10 q_l  11 phi_l
 *   12 I_s 13 R_s 14 n_s 15 q_s 16 phi_s 17 x_s 18 y_s
 *   19 gamma, the power-law slope of a LENS_MASS_EPL lens (ignored by the SIE)
 * A proposal outside the domain is not a call error: its lnL is -INFINITY.
 * The domain is: every slot 0..18 finite, theta_E >= 0, each axis ratio in
 * (0, 1], R_l > 0, R_s > 0, n_l and n_s in [0.1, 20]; for LENS_MASS_EPL also
 * gamma in [1.05, 2.95].
 *
 * Arithmetic: the ray trace and the Sersic exponents in FP64 (FP32 hardware
 * seeds refined by Newton steps; the FP32 hardware log2 and 2^x where their
 * error is not amplified), the binned image rounded to FP32
 * once, the PSF convolution in FP32 on the vector ALU (LENS_PREC_FP32) or as a
 * half-precision matrix-core contraction with FP32 accumulation flushed to FP64
 * (the other precisions), the chi-square reduction and the result in FP64.
 *
 * Threading: every entry point is thread-safe.  Errors: every call returns a
 * lens_status; on a call error nothing is written to the outputs and
 * lens_last_error() holds a message.  A HIP runtime error is sticky: the
 * context then answers LENS_EDEVICE to every call but lens_shutdown.
 */
#ifndef LENS_API_H
#define LENS_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lens_status;
#define LENS_OK 0
#define LENS_PENDING 1         /* lens_poll: the request has not finished */
#define LENS_EINVAL (-1)       /* bad argument */
#define LENS_ENOMEM (-2)       /* device memory or the HBM budget is exhausted */
#define LENS_ENOENT (-3)       /* unknown lens id or request id */
#define LENS_EBUSY (-4)        /* lens has requests in flight */
#define LENS_EAGAIN (-5)       /* non-blocking submit: no room right now */
#define LENS_EDEVICE (-6)      /* HIP runtime error (sticky) */
#define LENS_ECANCELED (-7)    /* request was cancelled */
#define LENS_ETIMEDOUT (-8)    /* lens_wait timed out; the request is still pending */

#define LENS_PARAM_STRIDE 20
#define LENS_NPARAM 19

/* PSF-convolution arithmetic, chosen per lens at load. */
#define LENS_PREC_FP32 0          /* FP32 direct convolution on the vector ALUs (lnL error < 1e-6) */
#define LENS_PREC_F16_SPLIT 1     /* FP16 MFMA, PSF and image split hi+lo, each image row at its own
                                     power-of-two scale, 3 products (22 significand bits; lnL error
                                     < 1e-6); the fastest of the < 1e-6 precisions */
#define LENS_PREC_BF16 2          /* BF16 MFMA, single product (lnL error < 2e-3) */
#define LENS_PREC_BF16_SPLIT3 3   /* BF16 MFMA, hi+mid+lo split, 6 products (lnL error < 1e-6) */

/* Light amplitudes, chosen per lens at load. */
#define LENS_AMP_EXPLICIT 0       /* I_l, I_s are parameters (slots 7 and 12) */
#define LENS_AMP_NNLS 1           /* solved linearly (Sec. 2.3): the amplitudes minimise
                                     sum_mask ((d - s_l a - s_s b)/sigma)^2 over s >= 0, with a, b the
                                     lens-light and source images at unit amplitude, binned and
                                     PSF-convolved; lnL is taken there and slots 7, 12 are ignored.
                                     Needs LENS_PREC_FP32. */

/* Mass models, chosen per lens at load. */
#define LENS_MASS_SIE 0           /* singular isothermal ellipsoid, kappa = theta_E / (2 R_p) (default) */
#define LENS_MASS_EPL 1           /* elliptical power law (Sec. 2.4), kappa = (3 - gamma)/2 (theta_E / R_p)^(gamma - 1)
                                     on the same elliptical radius R_p, gamma from slot 19; gamma = 2 is
                                     the SIE.  Deflection by the hypergeometric series of Tessore &
                                     Metcalf (2015), summed to a 1e-16 tail for axis ratios >= 0.15
                                     (at most 128 terms below that) */

/* Light models, chosen per lens at load; all but LENS_LIGHT_BOTH need
 * LENS_AMP_NNLS.  Each model reads, and validates, only the slots it uses. */
#define LENS_LIGHT_BOTH 0         /* one lens-light and one lensed source Sersic (default) */
#define LENS_LIGHT_LENS 1         /* lens light only, no lensing (the galaxy fits of Sec. 3.1.2):
                                     slots 3, 4 (centre) and 8-11 */
#define LENS_LIGHT_SOURCE 2       /* lensed source only, no lens light: slots 0-6 and 13-18 */
#define LENS_LIGHT_DOUBLE 3       /* two Sersic components per galaxy (Sec. 3.2), each pair sharing
                                     centre, q and phi, with indices fixed per lens (sersic_n):
                                     slot 8 is R_e of the lens's first component and slot 9 that of
                                     its second; slots 13 and 14 likewise for the source.  Four
                                     amplitudes in the order lens a, lens b, source a, source b */

typedef struct lens_ctx lens_ctx;
typedef int64_t lens_id;
typedef int64_t lens_req;
typedef int64_t lens_ens;

/* Device-memory hooks.  alloc returns a device pointer or NULL; both are
 * called with the context's device current. */
typedef void *(*lens_dev_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*lens_dev_free_fn)(void *ptr, void *stream, void *user);

typedef struct lens_init_opts {
    int32_t device;             /* HIP device ordinal */
    int64_t hbm_budget_bytes;   /* cap on library-held device memory; <= 0: 90% of free memory at init */
    int32_t max_inflight;       /* serving: requests with work on the device at once (each batch
                                   mixes pieces of at most this many); <= 0: 64 */
    int32_t nonblocking_submit; /* 1: lens_submit answers LENS_EAGAIN when no slot is free */
    lens_dev_alloc_fn dev_alloc;/* NULL: hipMalloc / hipFree */
    lens_dev_free_fn dev_free;
    void *alloc_user;
    void *stream;               /* hipStream_t for the blocking calls; NULL: a library-owned stream */
    int32_t autotune;           /* 1: time candidate strip heights and workgroup sizes for every new
                                   lens shape at load (cached per shape bucket, and in the file named
                                   by the LENS_AUTOTUNE_CACHE environment variable if set); 0: a
                                   fixed rule from the LDS footprint */
} lens_init_opts;

/* One observed lens image.  All arrays are host memory, row-major, copied by
 * lens_load_data; the caller may free them when it returns. */
typedef struct lens_data_desc {
    int32_t ny, nx;             /* image rows, columns (1..4096) */
    double pixel_scale;         /* arcsec per pixel, > 0 */
    int32_t supersample;        /* s >= 1 (paper: 4), at most 8 */
    int32_t psf_size;           /* k, odd, 1..63 */
    const double *psf;          /* k*k, used as given (not renormalised) */
    const double *data;         /* ny*nx observed image */
    const double *sigma;        /* ny*nx noise; > 0 and finite where mask = 1 */
    const uint8_t *mask;        /* ny*nx; nonzero = pixel enters the likelihood */
    int32_t precision;          /* LENS_PREC_* */
    int32_t amplitudes;         /* LENS_AMP_* (0: explicit) */
    double psf_tail;            /* PSF tail crop: the kernel is cut to the smallest centred odd square
                                   whose discarded taps' total |weight| is <= psf_tail * sum|K|, which
                                   moves any convolved pixel by at most psf_tail * sum|K| * max|binned|.
                                   0: the default 2^-48 (2^-24 below the FP32 resolution of the
                                   brightest pixel); < 0: keep the full k x k kernel */
    int32_t light_model;        /* LENS_LIGHT_* (0: lens and source) */
    double sersic_n[4];         /* LENS_LIGHT_DOUBLE: fixed Sersic indices of lens a, lens b, source a,
                                   source b, each in [0.1, 20] (Sec. 3.2 uses 1, 4, 1, 4); else ignored */
    int32_t mass_model;         /* LENS_MASS_* (0: SIE) */
} lens_data_desc;

typedef struct lens_info {
    int32_t ny, nx, supersample, psf_size, precision;
    int64_t masked_pixels;      /* M */
    int64_t needed_pixels;      /* pixels inside the mask dilated by the PSF footprint */
    int64_t device_bytes;       /* device memory held for this lens */
    double norm;                /* C = -1/2 sum_mask ln(2 pi sigma^2) */
    int32_t strip_rows;         /* tile shape of the likelihood kernel: output rows per strip */
    int32_t threads;            /*   and workgroup size (fixed rule or autotuner) */
    int64_t lds_bytes;          /* dynamic LDS of one workgroup (the binned-row ring) */
    int32_t blocks_per_cu;      /* resident workgroups per compute unit at that shape */
    int32_t psf_used;           /* side of the PSF kernel after the tail crop (psf_tail) */
    int32_t amplitudes;         /* LENS_AMP_* */
    int32_t light_model;        /* LENS_LIGHT_* */
    int32_t n_amplitudes;       /* amplitudes per proposal of lens_loglike_amps: 2, 1, 1 or 4 */
    int32_t mass_model;         /* LENS_MASS_* */
} lens_info;

typedef struct lens_stats {
    int64_t requests_submitted, requests_done, requests_failed, requests_canceled;
    int64_t proposals_done;
    int64_t queued, inflight;
    int64_t hbm_budget_bytes, hbm_used_bytes;
    int64_t launches;
    /* request latency, lens_submit to the result written (lens_poll / lens_wait
     * answer LENS_OK from then on): exact quantiles over the most recent
     * (at most 4,096) completed requests, the maximum over all of them */
    int64_t latency_count;      /* completed requests in the quantile window */
    double latency_p50_us, latency_p99_us, latency_max_us;
    int64_t batch_pieces;       /* request pieces placed in serving batches (launches counts the
                                   batches: batch_pieces / launches requests share a batch on average) */
} lens_stats;

/* Context.  lens_init creates the context on opts->device (NULL opts: all
 * defaults).  With the environment variable LENS_LOG set to 1 at lens_init,
 * the context writes one line to stderr per event: set-up, lens load and
 * unload, batch-plan capture, ensemble create and destroy, and every call
 * error with its message.  lens_shutdown waits for in-flight work, cancels queued
 * requests and frees everything; the pointer is invalid afterwards. */
lens_status lens_init(const lens_init_opts *opts, lens_ctx **out);
void lens_shutdown(lens_ctx *ctx);

/* Copy one lens to the device: the observed image d_i, its noise sigma_i and
 * fitting region (Sec. 2.2, Eq. 5; the region of App. A) as FP32 data and
 * weight mask/sigma, the PSF of Eq. 3 (Sec. 2.1), the supersampling factor of
 * Sec. 2.1, the pixel lists of the mask and of its PSF-dilated footprint, and
 * C = -1/2 sum_mask ln(2 pi sigma^2) in FP64.  Charged to the HBM budget:
 * LENS_ENOMEM if it does not fit.  LENS_EINVAL for a bad descriptor (see the
 * field comments); nothing is loaded then. */
lens_status lens_load_data(lens_ctx *ctx, const lens_data_desc *desc, lens_id *out_id);
/* Free a lens.  LENS_EBUSY while requests on it are queued or running. */
lens_status lens_unload(lens_ctx *ctx, lens_id id);
/* The PSF tail crop lens_load_data applies (Sec. 2.1 convolves the binned image
 * with the PSF; taps that carry a negligible share of its weight are dropped):
 * *k_used = the side of the smallest centred odd square of the k x k row-major
 * kernel `psf` (host memory) whose outside taps' total |weight| is
 * <= psf_tail * sum|K|.  psf_tail = 0 means 2^-48, psf_tail < 0 keeps k.  Host
 * only (no device, no context).  LENS_EINVAL for null pointers, an even or
 * non-positive k or a non-finite psf_tail. */
lens_status lens_psf_crop(const double *psf, int32_t k, double psf_tail, int32_t *k_used);

/* Describe a resident lens: its sizes, M, C and the tile shape its likelihood
 * kernel runs at (strip rows, threads, LDS bytes, resident workgroups per CU).
 * LENS_ENOENT for an unknown id. */
lens_status lens_get_info(lens_ctx *ctx, lens_id id, lens_info *out);

/* ln P(d | xi) of Sec. 2.2, Eq. 5 for n proposals xi (host buffers, params
 * [n][20] read, out [n] written): ray trace (Eq. 1), lens and source light
 * (Eqs. 2, 8-10), supersample and bin (Sec. 2.1), PSF (Eq. 3), masked
 * Gaussian chi^2.  Blocks until the results are in out.  n = 0 is a no-op.
 * LENS_EINVAL for null pointers or n < 0, LENS_ENOENT for an unknown id;
 * out is not written then. */
lens_status lens_loglike_batch(lens_ctx *ctx, lens_id id, const double *params, int64_t n,
                               double *out_loglike);

/* lnL and the amplitudes it was taken at (host buffers, out_amp [n][N] with
 * N = lens_info.n_amplitudes, in component order: lens light, source; lens
 * only; source only; lens a, lens b, source a, source b).  For a
 * LENS_AMP_NNLS lens these are the solved amplitudes; for an
 * explicit-amplitude lens, the proposal's slots 7 and 12.  Proposals outside
 * the domain give lnL = -inf and NaN amplitudes.  Blocks like
 * lens_loglike_batch. */
lens_status lens_loglike_amps(lens_ctx *ctx, lens_id id, const double *params, int64_t n,
                              double *out_loglike, double *out_amp);

/* lnL of Sec. 2.2, Eq. 5 on device buffers: d_params [n][20] and d_out [n]
 * in device memory, enqueued on the hipStream_t `stream` (NULL: the default
 * stream) and not waited for.  The caller keeps both buffers alive until the stream passes
 * the call.  Calls on one stream run in order; the library keeps a separate
 * scratch buffer per stream. */
lens_status lens_loglike_batch_device(lens_ctx *ctx, lens_id id, const double *d_params,
                                      int64_t n, double *d_out, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * call as lens_loglike_batch_device (same kernels, same results bit for bit),
 * except that the prepared constants go to a fixed device array of
 * LENS_NOALLOC_MAX proposals that the library sets up at lens_init, once per
 * device, and holds until the process ends; the call itself allocates
 * nothing.  n > LENS_NOALLOC_MAX answers LENS_EINVAL.  Every call on one GPU
 * shares that array: calls that overlap on the device (two streams, or two
 * contexts on the same GPU) race on it, so issue them on one stream or order
 * them. */
#define LENS_NOALLOC_MAX 32768
lens_status lens_loglike_batch_device_noalloc(lens_ctx *ctx, lens_id id, const double *d_params,
                                              int64_t n, double *d_out, void *stream);

/* Many lenses in one persistent launch (Sec. 2.2, Eq. 5 per proposal; the
 * batched evaluation of Sec. 3.1.4 across lenses).  ids[i] with counts[i] proposals;
 * params holds the proposals of lens 0, then lens 1, ... ([sum counts][20]),
 * out the results in the same order.  Blocking, host buffers.  Workgroups
 * pull (lens, proposal) items, longest first, from a device work counter; the
 * call shape (ids and counts) is captured once as a hipGraph and replayed on
 * later calls of the same shape (the 8 most recent shapes are kept).  Lenses
 * of different precision or workgroup size go to separate persistent launches
 * inside the same graph.  Every result equals the single-lens result bit for
 * bit. */
lens_status lens_loglike_multi(lens_ctx *ctx, int32_t nlens, const lens_id *ids,
                               const int64_t *counts, const double *params, double *out);

/* Many lenses on device buffers (Sec. 2.2, Eq. 5 for every proposal; the
 * batched evaluation of Sec. 3.1.4, extended across lenses): ids[i] with
 * counts[i] proposals (host arrays); d_params [sum counts][20] and d_out
 * [sum counts] in device memory, lens-major in the order of ids.  Enqueued on
 * the hipStream_t `stream` (NULL: the default stream) and not waited for: the
 * prep step over all proposals, then one persistent launch per group of
 * lenses (as lens_loglike_multi, without the graph and the host copies).  The
 * caller keeps both buffers alive until the stream passes the call.  Results
 * equal lens_loglike_multi's and the single-lens results bit for bit.  The
 * lookup tables of the 8 most recent call shapes are kept; the prepared
 * constants and work counters use the stream's scratch buffer.  LENS_EINVAL
 * for null or negative arguments, LENS_ENOENT for an unknown id. */
lens_status lens_loglike_multi_device(lens_ctx *ctx, int32_t nlens, const lens_id *ids,
                                      const int64_t *counts, const double *d_params, double *d_out,
                                      void *stream);

/* Serving (the batched likelihood of Sec. 3.1.4, Eq. 5 per proposal, for many
 * concurrent fits).  lens_submit copies params before it returns; out must
 * stay valid until lens_poll / lens_wait report a final status or lens_cancel
 * returns.  Requests are batched continuously: a scheduler thread packs the
 * waiting proposals of many requests, on any mix of resident lenses, into one
 * batch (one prep launch and one persistent launch per lens group, as in
 * lens_loglike_multi), keeps two batches in flight on two streams, and starts
 * the next batch as soon as one finishes, so requests that arrive while
 * others run join the next batch.  Batch buffers are fixed and charged to the
 * HBM budget at the first submit.  Each result equals the result of the same
 * proposals evaluated alone, bit for bit.  When max_inflight requests already
 * have work on the device a new request queues, or with nonblocking_submit
 * the call answers LENS_EAGAIN. */
lens_status lens_submit(lens_ctx *ctx, lens_id id, const double *params, int64_t n,
                        double *out_loglike, lens_req *out_req);
/* Non-blocking: LENS_PENDING, LENS_OK when out is written (lnL of Sec. 2.2,
 * Eq. 5 per proposal, as lens_loglike_batch), or the request's error.  A
 * request id is forgotten after the first final answer (then LENS_ENOENT). */
lens_status lens_poll(lens_ctx *ctx, lens_req req);
/* Waits up to timeout_us (< 0: forever); LENS_ETIMEDOUT if still pending. */
lens_status lens_wait(lens_ctx *ctx, lens_req req, int64_t timeout_us);
/* Cancels a queued request (LENS_OK) or waits for a running one to finish
 * and discards it; out is then not written.  The id is forgotten. */
lens_status lens_cancel(lens_ctx *ctx, lens_req req);
lens_status lens_get_stats(lens_ctx *ctx, lens_stats *out);
/* Zero the serving counters and empty the latency window (for per-interval
 * figures); requests in flight are not affected, and count in the new
 * interval when they finish. */
lens_status lens_reset_stats(lens_ctx *ctx);

/* ------------------------------------------------------------------------
 * Sampler loop on the device.  The paper's sampler runs on the host and
 * moves every proposal batch across PCIe (Sec. 3.1.4); Sec. 4.2 points to
 * sampling on the GPU.  Here an ensemble of walkers lives in device memory
 * and moves by the stretch move of Goodman & Weare (2010, CAMCoS 5, 65,
 * Sec. 3), in its parallel form: the two halves of the ensemble update in
 * turn.  Proposals are made, evaluated and accepted on the device, and only
 * the final state and the requested chain rows return to the host.
 *
 * Target: lnP = lnL under a uniform box prior (Sec. 2.2): lo[s] <= p[s] <=
 * hi[s] for every slot s.  A slot with lo = hi is fixed; d = the number of
 * free slots enters the acceptance rule.  Fix the slots the lens ignores
 * (slot 19; slots 7 and 12 with LENS_AMP_NNLS; the unused slots of a light
 * model): free slots that do not change lnL only add random-walk directions.
 *
 * Iteration t, walker k of the moving half (half 0: walkers 0..W/2-1, then
 * half 1): the Philox4x32-10 words (Salmon et al., SC'11) of counter
 * (k, t mod 2^32, t div 2^32, 0) under key (seed mod 2^32, seed div 2^32),
 * with u = (word + 1/2) 2^-32, give
 *   partner j = (first walker of the other half) + floor(word0 (W/2) / 2^32),
 *   z = ((a - 1) u1 + 1)^2 / a   (density ~ 1/sqrt(z) on [1/a, a]),
 *   u2 from word 2;
 * the proposal Y = X_j + z (X_k - X_j) replaces X_k when
 *   ln u2 < (d - 1) ln z + lnP(Y) - lnP(X_k).
 * Proposals outside the box get lnP = -inf without being evaluated.  The
 * stream depends only on (seed, k, t): a run split over several calls equals
 * one long run. */
typedef struct lens_ensemble_desc {
    int32_t walkers;            /* W, even, 4..2^24 (each half-step evaluates W/2 proposals) */
    double stretch;             /* a > 1 (Goodman & Weare use 2) */
    uint64_t seed;              /* Philox key */
    const double *lo, *hi;      /* [20] box prior, finite, lo <= hi, at least one free slot */
    const double *init;         /* [W][20] initial walkers, inside the box, each with finite lnL */
} lens_ensemble_desc;

/* Copies the walkers to the device and evaluates their lnP.  The ensemble
 * holds its lens (lens_unload answers LENS_EBUSY) until destroyed.
 * LENS_EINVAL for a bad descriptor, a walker outside the box or one whose
 * lnL is -inf; LENS_ENOMEM past the HBM budget. */
lens_status lens_ensemble_create(lens_ctx *ctx, lens_id id, const lens_ensemble_desc *desc, lens_ens *out);
/* Advances the ensemble by `iterations` iterations (each moves both halves),
 * entirely on the device, blocking until done.  chain (may be NULL): host
 * [iterations/thin][W][20], the walkers after every thin-th iteration of this
 * call; chain_lnp (may be NULL): host [iterations/thin][W], their lnP.  The
 * chain rows are staged in device memory (charged to the HBM budget) and
 * copied back at the end: split long runs into several calls. */
lens_status lens_ensemble_run(lens_ctx *ctx, lens_ens ens, int64_t iterations, int32_t thin,
                              double *chain, double *chain_lnp);
/* Advances the n distinct ensembles ens[0..n-1] by `iterations` iterations
 * each, together: every half-step makes the proposals of all of them in one
 * launch, evaluates the pooled proposals with the multi-lens likelihood
 * (lens_loglike_multi's grouping and kernels) and accepts them in one launch,
 * so that many small ensembles, one per lens of a survey, fill the device
 * where each alone would not.  Each ensemble moves exactly as under
 * lens_ensemble_run from its own iteration count (same stream, same result,
 * bit for bit).  chains (may be NULL): n host pointers, chains[e] receiving
 * [iterations/thin][W_e][20], the walkers of ensemble e after every thin-th
 * iteration of this call; chain_lnps likewise [iterations/thin][W_e]; a NULL
 * entry skips that ensemble.  Blocks until done.  LENS_EINVAL for a repeated
 * id, thin < 1 with a chain requested, or more than INT_MAX pooled proposals
 * (sum of W/2); LENS_ENOENT for an unknown id (nothing moves); LENS_ENOMEM past
 * the HBM budget for the pooled scratch, sum W/2 x 472 bytes plus the
 * per-ensemble descriptors and the staged chain rows. */
lens_status lens_ensemble_run_many(lens_ctx *ctx, int32_t n, const lens_ens *ens, int64_t iterations, int32_t thin,
                                   double *const *chains, double *const *chain_lnps);
/* The current walkers [W][20], their lnP [W], accepted moves per walker [W]
 * and the iterations done so far; any output may be NULL. */
lens_status lens_ensemble_get(lens_ctx *ctx, lens_ens ens, double *walkers, double *lnp,
                              int64_t *accepted, int64_t *iteration);
/* Frees the ensemble and releases its lens.  LENS_EBUSY during a call on it. */
lens_status lens_ensemble_destroy(lens_ctx *ctx, lens_ens ens);
/* The Philox4x32-10 words (Salmon et al., SC'11: ten rounds, multipliers
 * 0xD2511F53 and 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85) of
 * the n counters (ctr[0] + i mod 2^32, ctr[1], ctr[2], ctr[3]), i < n <= 2^32,
 * under key[2], computed on the device into out [n][4] (host).  The stream
 * the sampler draws from, exposed for reproduction and tests. */
lens_status lens_philox4x32_10(lens_ctx *ctx, const uint32_t *ctr, const uint32_t *key, int64_t n,
                               uint32_t *out);

/* Debug/test: the model image of one proposal (params1: 20 doubles) into
 * out_img [ny][nx]: stage 0 binned and unconvolved, stage 1 PSF-convolved.
 * The image is always that of the lens and source model with the explicit
 * amplitudes of slots 7 and 12, whatever the lens's light model and
 * amplitude mode.  A proposal outside that model's domain gives LENS_EINVAL. */
lens_status lens_model_image(lens_ctx *ctx, lens_id id, const double *params1, int32_t stage,
                             double *out_img);

/* Self-test of the device: the matrix-core operand layout the convolution
 * relies on, a 16x32 by 32x16 product of small integers, in BF16 (which = 0)
 * or IEEE half (which = 1, the FP16 split's instruction).  *result = max
 * |device - exact|, 0 when the layout holds; other values of which give
 * LENS_EINVAL. */
lens_status lens_selftest(lens_ctx *ctx, int32_t which, double *result);

/* Instruction kinds for lens_peak_rate. */
#define LENS_PEAK_FMA_F64 0         /* v_fma_f64 */
#define LENS_PEAK_FMA_F32 1         /* v_fma_f32 (not packed) */
#define LENS_PEAK_MUL_F64 2         /* v_mul_f64 */
#define LENS_PEAK_ADD_F64 3         /* v_add_f64 */
#define LENS_PEAK_EXP_F32 4         /* v_exp_f32 (2^x) */
#define LENS_PEAK_LOG_F32 5         /* v_log_f32 (log2 x) */
#define LENS_PEAK_RSQ_F32 6         /* v_rsq_f32 */
#define LENS_PEAK_RCP_F32 7         /* v_rcp_f32 */
#define LENS_PEAK_CVT_F64_F32 8     /* v_cvt_f32_f64 and v_cvt_f64_f32, alternating */
#define LENS_PEAK_LDEXP_F64 9       /* v_ldexp_f64 */
#define LENS_PEAK_FREXP_MANT_F64 10 /* v_frexp_mant_f64 */
#define LENS_PEAK_RNDNE_F64 11      /* v_rndne_f64 */
#define LENS_PEAK_RSQ_F64 12        /* v_rsq_f64 */
#define LENS_PEAK_MFMA_F16 13       /* v_mfma_f32_16x16x32_f16 */
#define LENS_PEAK_MFMA_BF16 14      /* v_mfma_f32_16x16x32_bf16 */
#define LENS_PEAK_FMA_F64_EXP_F32 15 /* v_fma_f64 and v_exp_f32, alternating (both counted) */
#define LENS_PEAK_MFMA_F16_FMA_F64 16 /* four v_fma_f64 after each FP16 product (the FMAs counted) */
#define LENS_PEAK_COUNT 17

/* Measured peak rate of one instruction kind on this context's device, for
 * the roofline the likelihood kernels are held against (the operation
 * counts behind it: ray trace and Sersic profiles of Sec. 2.1 and 2.4, the
 * PSF contraction of Eq. 4).  A launch of eight waves per SIMD, every lane
 * running eight independent chains of the instruction, timed with HIP events
 * on the context's stream, best of three launches of ~25 ms each after a
 * warm-up and a sizing launch.  *rate = lane operations per second for the vector ALU
 * kinds (an FMA counts once, so FMA FLOP/s = 2 *rate), FLOP/s for the
 * matrix-core products (2 x 16 x 16 x 32 per instruction).  An op outside
 * [0, LENS_PEAK_COUNT) gives LENS_EINVAL.  Holds the context's blocking-call
 * lock while it runs; meant for characterisation, not for the hot path. */
lens_status lens_peak_rate(lens_ctx *ctx, int32_t op, double *rate);

const char *lens_strerror(lens_status st);
/* Last error message of the calling thread on this context ("" if none). */
const char *lens_last_error(lens_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LENS_API_H */
