// lens_internal.h -- structures shared by the host runtime and the HIP kernels.
// Private to the library; the public interface is include/lens_api.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lensk {

constexpr int kStride = 20;   // doubles per proposal vector
constexpr int kBlock = 256;   // threads per workgroup of the likelihood kernels
constexpr int kMaxK = 63;     // largest PSF side
constexpr double kNMin = 0.1, kNMax = 20.0;

// Derived constants of one Sersic component (Sec. 2.4, Eqs. 8, 10).
struct LightK {
    double P, Q, S;   // (R_p/R_e)^2 = P dx^2 + Q dy^2 + S dx dy, the rotation of Eq. 10 folded in
    double e;         // 1 / (2n): t = ((R_p/R_e)^2)^e = (R_p/R_e)^(1/n)
    double B;         // b_n log2(e): I = I_e 2^(B (1 - t))
    double I;         // I_e
};

// Derived constants of one proposal, written by the prep kernel and read
// (uniformly, through the scalar cache) by every workgroup of that proposal.
struct alignas(16) PropBlock {
    double valid;                              // 1 inside the domain; 2 inside except for non-finite
                                               // amplitudes (usable when they are solved); 0 outside
    double xm, ym, cm, sm, q2m, ce;            // SIE: centre, cos/sin phi, q^2, c = sqrt(1 - q^2)
    double bsie, bsc;                          // theta_E sqrt(q), theta_E sqrt(q) / c (0 if c = 0)
    // u = R(-phi_m) (theta - alpha_shear - source centre) at the mass centre's
    // abscissa (dx = 0), affine in the ordinate y: u1 = au1 + bu1 y, u2 = au2 + bu2 y
    double au1, bu1, au2, bu2;
    // lens light: (R_p/R_e)^2 in image-plane offsets from the centre; source:
    // in source-plane offsets from its centre taken in the frame of the mass
    // ellipse, w = R(-phi_m) (beta - source centre), so that the ray trace
    // never rotates its deflection back
    LightK lens, src;
    double ku1, ku2;                           // d/dx of u = R(-phi_m) (theta - alpha_shear - source centre)
    double dlg_l, dlg_s;                       // two-component light: 2 log2(R_a / R_b) of the lens, of the source
    // elliptical power law (slope gamma = t + 1): q, 2 b^t / (1 + q) with b = theta_E sqrt(q),
    // (1 - t) / 2, and -f = -(1 - q) / (1 + q) (the series ratio's sign and scale)
    double epl_q, epl_pref, epl_h, epl_mf;
};
static_assert(sizeof(PropBlock) == 272, "PropBlock layout");
constexpr int kPCBytes = (int)sizeof(PropBlock);

// PSF-convolution modes: the public LENS_PREC_* values (0-3), then the FP32
// convolution of unit-amplitude channels whose amplitudes are solved by
// non-negative least squares (Sec. 2.3), one mode per light model: lens light
// and source (4), lens light only, no lensing (5), lensed source only (6), and
// two components per galaxy sharing centre and ellipticity with fixed Sersic
// indices (7).
// The flag MODE_EPL (added to any of them) selects the elliptical power-law
// mass in place of the SIE.
enum : int {
    MODE_FP32 = 0,
    MODE_SPLIT = 1,
    MODE_BF16 = 2,
    MODE_SPLIT3 = 3,
    MODE_FP32N = 4,
    MODE_FP32N_LENS = 5,
    MODE_FP32N_SRC = 6,
    MODE_FP32N_DBL = 7,
    MODE_EPL = 8
};
__host__ __device__ constexpr int mode_base(int mode) { return mode & 7; }
__host__ __device__ constexpr bool mode_epl(int mode) { return (mode & MODE_EPL) != 0; }
__host__ __device__ constexpr int mode_planes(int mode)
{
    return mode_base(mode) == MODE_SPLIT ? 2 : mode_base(mode) == MODE_SPLIT3 ? 3 : 1;
}
__host__ __device__ constexpr bool mode_solved(int mode) { return mode_base(mode) >= MODE_FP32N; }
// Matrix-core window of a 16-wide output segment along one PSF row: 16 + k - 1
// ring columns, rounded up to 8 (BF16 modes: K-chunks of 32 run on across PSF
// rows) or to 32 (the FP16 split: every K-chunk within one ring row, whose
// scale it carries).
__host__ __device__ constexpr int window_len(int mode, int k)
{
    return mode_base(mode) == MODE_SPLIT ? (k + 15 + 31) / 32 * 32 : (k + 15 + 7) / 8 * 8;
}
// ring rows the FP16 split's per-row scales are kept for (strip + PSF halo)
constexpr int kRingRowsMax = 128;
// binned channels (components at unit amplitude) of a solved-amplitude mode
__host__ __device__ constexpr int mode_channels(int mode)
{
    return mode_base(mode) == MODE_FP32N                                             ? 2
           : mode_base(mode) == MODE_FP32N_LENS || mode_base(mode) == MODE_FP32N_SRC ? 1
           : mode_base(mode) == MODE_FP32N_DBL                                      ? 4
                                                                                    : 0;
}

// Light models (the public LENS_LIGHT_* values); they fix what the prep kernel
// reads from the parameter slots.
enum : int { LIGHT_BOTH = 0, LIGHT_LENS = 1, LIGHT_SRC = 2, LIGHT_DOUBLE = 3 };
__host__ __device__ constexpr int mode_light(int mode)
{
    return mode_base(mode) == MODE_FP32N_LENS  ? LIGHT_LENS
           : mode_base(mode) == MODE_FP32N_SRC ? LIGHT_SRC
           : mode_base(mode) == MODE_FP32N_DBL ? LIGHT_DOUBLE
                                               : LIGHT_BOTH;
}
// The prep step's model code: light model | (mass model << 8), mass 1 = EPL.
constexpr int kMassShift = 8;
constexpr int kEplMaxTerms = 128;   // terms of the power-law deflection series
constexpr double kGammaMin = 1.05, kGammaMax = 2.95;
// per-proposal SIE deflection table in LDS: intervals of u = q |x1| / psi and
// doubles per interval (centre, two sets of 6 coefficients, padding to 16 bytes)
constexpr int kSieIntervals = 32, kSieEntry = 14;

// Everything a likelihood launch needs to know about one resident lens.
struct LensGeom {
    int ny, nx, s, k, r;   // rows, columns, supersampling, PSF side, (k-1)/2
    int pitch;             // row pitch (floats) of data and weight, multiple of 4
    int mode;              // MODE_*
    int nt;                // threads per workgroup (256 or 512)
    int strip_h;           // output rows per strip
    int ring_rows;         // strip_h + 2r binned rows kept in LDS
    int ring_w;            // elements per LDS row (FP32 ring: floats; MFMA ring: bf16 per plane)
    int plane;             // MFMA ring: elements per bf16 plane (ring_rows * ring_w)
    int L;                 // MFMA: window length per segment (window_len)
    int nchunks;           // MFMA: K-chunks of 32, ceil(k L / 32)
    int nstrips;           // ceil(ny / strip_h)
    int xoff;              // ring column of image column x is x + r - xoff (a multiple of 16 at or left of
                           // every masked column: the ring spans only the columns the convolution reads)
    int span;              // columns from xoff to the right edge of the mask (ring width less the PSF window)
    double sd;             // pixel_scale / s: sub-pixel pitch
    double cfx, cfy;       // (nx*s - 1)/2, (ny*s - 1)/2: fine-grid centre
    float inv_s2;          // 1/s^2
    double norm;           // C = -1/2 sum_mask ln(2 pi sigma^2)
    double dd;             // solved amplitudes: sum_mask (w d)^2 in FP64 of the FP32 w and d
    double conv_scale;     // FP16 split: 2^-j, undoing the power of two the PSF planes were scaled by
    double fix_e[4];       // MODE_FP32N_DBL: 1/(2n) of the fixed indices (lens a, lens b, source a, source b)
    double fix_B[4];       //   and b_n log2 e
    const float *psf;      // flipped kernel Kf[a][b] = K[k-1-a][k-1-b], [k][k]
    const float *data;     // [ny][pitch], 0 outside the mask and the image
    const float *wgt;      // [ny][pitch], mask/sigma, 0 outside the mask and the image
    const uint32_t *evl;   // pixels whose binned value is needed, (y << 16) | x, row-major
    const int *evpre;      // [ny + 1] prefix of evl by row
    const int2 *evr;       // [ny] needed column range [lo, hi) of each row
    const uint32_t *cvl;   // FP32 mode: groups of 4 output pixels covering the mask, (y << 16) | x0
    const int *cvpre;      // FP32 mode: [ny + 1] prefix of cvl by row
    const uint4 *aop;      // MFMA: Toeplitz A operand, [nchunks][planes][64 lanes] x 8 bf16
    const uint32_t *seg;   // MFMA: 16-wide output segments (y << 16) | x0 covering the mask, row-major
    const int *segpre;     // MFMA: [ny + 1] prefix of seg by row
};

size_t ring_bytes(const LensGeom &g);
double host_sersic_bn(double n);   // b_n of Eq. 9 by FP64 Newton iteration, on the host
int choose_kc(int k);
// LDS row width (elements) and bytes per ring row for a mode, PSF side and
// span (LensGeom::span: the masked columns from xoff on)
int ring_width(int mode, int k, int span);
size_t ring_row_bytes(int mode, int k, int span);
// largest dynamic LDS one workgroup may use on this device
size_t max_lds_bytes();
size_t set_lds_limits(size_t bytes);   // dynamic LDS now accepted by every ring kernel; 0 on refusal
size_t lds_per_cu();

// Derived constants of n proposals.  Each proposal is read under a model code
// (light model | mass << kMassShift): `model` for all of them, or, with
// d_pstart (nl + 1 proposal offsets) and d_pmodel (nl codes) in device memory,
// that of the lens owning it.
hipError_t launch_prep(const double *d_params, int64_t n, PropBlock *d_pc, int model, const int64_t *d_pstart,
                       const int *d_pmodel, int nl, hipStream_t st);
// the fused likelihood of n proposals of one lens (FP32 or MFMA convolution per g.mode)
// d_amp (solved-amplitude modes, may be null): the solved amplitudes, [n][mode_channels(g.mode)]
hipError_t launch_loglike(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, double *d_amp,
                          hipStream_t st);
// persistent multi-lens launch (counter reset + kernel) and its occupancy
int batch_blocks_per_cu(int mode, int nt, size_t lds);
// static LDS (deflection table, reduction slots) of the multi-lens kernel of a
// mode and workgroup size; the single-lens kernels hold no more
size_t batch_static_lds(int mode, int nt);
int loglike_blocks_per_cu(const LensGeom &g);    // resident single-lens workgroups per CU; 0 if unknown
hipError_t launch_batch(int mode, int nt, int grid, size_t lds, const LensGeom *d_geoms, const int *d_lstart,
                        const int64_t *d_lout, int nl, int nitems, const PropBlock *d_pc, double *d_out,
                        unsigned int *d_counter, hipStream_t st);
// sampler loop (lens_sampler.hip): Philox4x32-10 words of counters
// (ctr[0] + i, ctr[1], ctr[2], ctr[3]), i < n, into d_out [n][4]; the two
// halves of a stretch-move step (d_aux: [W/2][4] doubles)
hipError_t launch_philox_words(const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t *d_out,
                               hipStream_t st);
// One ensemble of a multi-ensemble step, in device memory.  Its walkers of the
// moving half occupy pooled slots [off, off + W/2).
struct EnsembleDev {
    int W, d, code, pad;        // walkers, free slots, prep model code
    uint64_t seed;
    int64_t t0;                 // the ensemble's iteration at the start of the call
    double a;                   // stretch scale
    double *walkers, *lnp;
    int64_t *accepted;
    const double *lo, *hi;
    int64_t off;
    double *chain_w, *chain_lnp;   // device chain staging of this call, [rows][W][20] and [rows][W]; may be null
};
// stage 0: proposals of half `half` of every ensemble at iteration t0 + it into
// the pooled d_Y [total][20], d_aux [total][4], d_pc [total]; stage 1: their
// acceptance from the pooled lnL d_lnl [total], and with slot >= 0 the walkers
// after the move written to chain row `slot` of every ensemble that has a
// chain.  d_hoff: [n + 1] prefix of W/2.
hipError_t launch_stretch_many(int half, int64_t it, const EnsembleDev *d_ens, const int64_t *d_hoff, int n,
                               int64_t total, double *d_Y, double *d_aux, PropBlock *d_pc, int stage, const double *d_lnl,
                               int64_t slot, hipStream_t st);
hipError_t launch_stretch_propose(int W, int half, uint64_t t, uint64_t seed, double a, int model_code,
                                  const double *d_walkers, const double *d_lo, const double *d_hi, double *d_Y,
                                  double *d_aux, PropBlock *d_pc, hipStream_t st);
hipError_t launch_stretch_accept(int W, int half, int d, double *d_walkers, double *d_lnp, const double *d_Y,
                                 const double *d_aux, const double *d_lnl, int64_t *d_accepted, double *d_chain_w,
                                 double *d_chain_lnp, hipStream_t st);
// The allocation-free entry point's prepared-constant scratch: a fixed device
// array of kNoAllocMax PropBlocks (lens_kernels.hip).  noalloc_init resolves its
// address on `device` (which must be current) once; noalloc_scratch returns it,
// or null before that.
constexpr int kNoAllocMax = 32768;
constexpr int kNoAllocDevices = 64;
hipError_t noalloc_init(int device);
PropBlock *noalloc_scratch(int device);
// self-test of the matrix-core operand layout: D = A B for a 16x32 by 32x16 BF16 product
hipError_t launch_mfma_probe(bool f16, const uint16_t *d_a, const uint16_t *d_b, float *d_d, hipStream_t st);
// issue-rate probes (lens_peak_rate): `grid` workgroups of peak_threads()
// threads, n rounds each, one double per thread into out; each lane does
// peak_ops_per_round(op) operations per round
int peak_threads();
double peak_ops_per_round(int op);
hipError_t launch_peak(int op, int grid, int n, double *out, hipStream_t st);
// stage 0: binned image of one proposal into d_img [ny][nx]; stage 1: convolved,
// using d_tmp [ny][nx] for the binned image.
hipError_t launch_model_image(const LensGeom &g, const PropBlock *d_pc, int stage, float *d_img,
                              float *d_tmp, hipStream_t st);

}  // namespace lensk
