// lens_kernels.hip -- HIP kernels of the batched lens log-likelihood (gfx950).
//
// k_prep          one thread per proposal: domain check, FP64 b_n, derived constants.
// k_loglike_fp32  one workgroup per proposal: the whole forward model and the
//                 chi-square in one pass, the binned image never leaving LDS;
//                 PSF convolution on the vector ALU in FP32.
// k_loglike_mfma  the same with the PSF convolution as a BF16 matrix-core
//                 contraction (plain, hi+lo split or hi+mid+lo split operands).
// k_model_*       debug: full model images of one proposal.
//
// Forward model: Cao et al. (2025), Sec. 2.1 (Eqs. 1-3), Sec. 2.2 (Eq. 5), Sec. 2.4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "lens_device.h"
#include "lens_internal.h"
#include "lens_prep.h"

namespace lensk {

// ---------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------
// One thread per proposal; the light model of proposal i is `model`, or, with
// a per-lens table, that of the lens owning i.
__global__ void __launch_bounds__(256) k_prep(const double *__restrict__ params, int64_t n, PropBlock *__restrict__ pc,
                                              int model, const int64_t *__restrict__ pstart,
                                              const int *__restrict__ pmodel, int nl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lm = model;
    if (pstart) {
        int lo = 0, hi = nl;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pstart[mid] <= i) lo = mid; else hi = mid;
        }
        lm = pmodel[lo];
    }
    const double *p = params + i * kStride;
    double v[kStride];
#pragma unroll
    for (int j = 0; j < kStride; ++j) v[j] = p[j];
    pc[i] = prep_proposal(v, lm);
}

// ---------------------------------------------------------------------------
// fused likelihood: shared pieces
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
// the matrix-core A operands in the global address space: their loads then
// count on vmcnt alone, and an LDS wait does not also wait for them
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 *gptr4;
// and the B operands' LDS ring, kept in the LDS address space through arrays
typedef const __attribute__((address_space(3))) uint16_t *lptr16;
typedef const __attribute__((address_space(3))) u32x4 *lptr4;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __forceinline__ uint16_t bf16_rn(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// How a binned value is kept in the LDS ring: FP32, or NPL BF16 planes whose
// sum is the value (hi, hi + lo, hi + mid + lo).  The FP16 split first keeps
// the FP32 value's upper and lower 16 bits in its two planes; once the row is
// complete, convert_rows_f16 turns them into half planes at the row's scale.
template <int MODE>
struct RingStore {
    static constexpr int NPL = mode_planes(MODE);
    __device__ static void put(void *ring, int plane, int idx, float v)
    {
        if (MODE == MODE_FP32) {
            static_cast<float *>(ring)[idx] = v;
        } else if (MODE == MODE_SPLIT) {
            uint16_t *b = static_cast<uint16_t *>(ring);
            const uint32_t u = __float_as_uint(v);
            b[idx] = (uint16_t)(u >> 16);
            b[plane + idx] = (uint16_t)u;
        } else {
            uint16_t *b = static_cast<uint16_t *>(ring);
            const uint16_t h = bf16_rn(v);
            b[idx] = h;
            if (NPL >= 2) {
                const float r1 = v - bf16_f(h);
                const uint16_t m = bf16_rn(r1);
                b[plane + idx] = m;
                if (NPL >= 3) b[2 * plane + idx] = bf16_rn(r1 - bf16_f(m));
            }
        }
    }
    __device__ static void zero(void *ring, int plane, int idx)
    {
        if (MODE == MODE_FP32) {
            static_cast<float *>(ring)[idx] = 0.0f;
        } else {
            uint16_t *b = static_cast<uint16_t *>(ring);
#pragma unroll
            for (int p = 0; p < NPL; ++p) b[p * plane + idx] = 0;
        }
    }
};

// Solved amplitudes: the NCH unit-amplitude channels of a pixel form one ring
// element (float, float2 or float4).
template <int NCH> struct FVec;
template <> struct FVec<1> {
    typedef float T;
    __device__ static T make(const float (&c)[1]) { return c[0]; }
    __device__ static float at(const T &v, int) { return v; }
};
template <> struct FVec<2> {
    typedef float2 T;
    __device__ static T make(const float (&c)[2]) { return make_float2(c[0], c[1]); }
    __device__ static float at(const T &v, int i) { return i == 0 ? v.x : v.y; }
};
template <> struct FVec<4> {
    typedef float4 T;
    __device__ static T make(const float (&c)[4]) { return make_float4(c[0], c[1], c[2], c[3]); }
    __device__ static float at(const T &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
};

template <int NCH>
struct RingStoreN {
    typedef typename FVec<NCH>::T T;
    __device__ static void put(void *ring, int, int idx, T v) { static_cast<T *>(ring)[idx] = v; }
    __device__ static void zero(void *ring, int, int idx)
    {
        const float z[NCH] = {};
        static_cast<T *>(ring)[idx] = FVec<NCH>::make(z);
    }
};
template <> struct RingStore<MODE_FP32N> : RingStoreN<2> {};
template <> struct RingStore<MODE_FP32N_LENS> : RingStoreN<1> {};
template <> struct RingStore<MODE_FP32N_SRC> : RingStoreN<1> {};
template <> struct RingStore<MODE_FP32N_DBL> : RingStoreN<4> {};
// the mass model does not change the ring
template <int MODE> struct RingStoreM : RingStore<mode_base(MODE)> {};

// FP16 split: per ring slot, the largest |value| of the row being filled (FP32
// bits, by atomic max) and, once converted, the factor 2^-j that undoes the
// row's scale.
__device__ __forceinline__ uint32_t *f16_rowmax()
{
    __shared__ uint32_t m[kRingRowsMax];
    return m;
}
__device__ __forceinline__ float *f16_rowscale()
{
    __shared__ float sc[kRingRowsMax];
    return sc;
}

// Binned rows [ya, yb) of the FP16 split, complete in the ring as FP32 bits:
// each row scaled by the power of two 2^j that brings its largest |value|
// into [2^13, 2^14), and split into the nearest half h and the nearest half to
// the remainder.  The pair keeps 22 significant bits of every value from
// 2^-3 of the row's largest up; below, the remainder is subnormal and the
// absolute error stays under 2^-39 of the row's largest value.  One wave per
// row; the row's maximum is cleared for the slot's next row after the next
// barrier (clear_rowmax_f16).
template <int NT>
__device__ __forceinline__ void convert_rows_f16(const LensGeom &g, uint16_t *ring, int ya, int yb)
{
    const int W = g.ring_w, RB = g.ring_rows, lane = threadIdx.x & 63;
    for (int y = ya + (int)(threadIdx.x >> 6); y < yb; y += NT / 64) {
        const int slot = (y + g.r) % RB;
        const float m = __uint_as_float(f16_rowmax()[slot]);
        int e = 0;
        (void)frexpf(m, &e);                       // m < 2^e
        e = m > 0.0f ? max(e, -100) : 14;          // tiny rows: the scale stays finite
        const float sc = ldexpf(1.0f, 14 - e), inv = ldexpf(1.0f, e - 14);
        if (lane == 0) f16_rowscale()[slot] = inv;
        uint16_t *hi = ring + slot * W, *lo = hi + g.plane;
        for (int x = lane; x < W; x += 64) {
            const float v = __uint_as_float(((uint32_t)hi[x] << 16) | lo[x]) * sc;
            const _Float16 h = (_Float16)v;
            const _Float16 l = (_Float16)(v - (float)h);
            hi[x] = __builtin_bit_cast(uint16_t, h);
            lo[x] = __builtin_bit_cast(uint16_t, l);
        }
    }
}

template <int NT>
__device__ __forceinline__ void clear_rowmax_f16(const LensGeom &g, int ya, int yb)
{
    for (int y = ya + (int)threadIdx.x; y < yb; y += NT) f16_rowmax()[(y + g.r) % g.ring_rows] = 0u;
}

// Modes whose ray trace may take the SIE deflection table: the SIE mass with a
// lensed source, one light component per galaxy (with four channels the
// table's operands cost the multi-lens kernel a wave per SIMD: 0.66x of one
// lens at a time, against 1.03x without the table).
template <int MODE>
__host__ __device__ constexpr bool sie_tab()
{
    return !mode_epl(MODE) && mode_light(MODE) != LIGHT_LENS && mode_light(MODE) != LIGHT_DOUBLE;
}

// Binned rows [ya, yb) (all < ny) into their ring slots: every pixel in the
// row's needed range is evaluated; the rest of the row is cleared when the
// slot is being reused (clear = true).  Ring column of image column x is
// x + r - xoff; columns outside the image are never written and stay zero.
template <int MODE, int NT>
__device__ __forceinline__ void fill_rows(const LensGeom &g, const PropBlock &P, void *ring,
                                          const uint32_t *__restrict__ evl, const int *__restrict__ evpre,
                                          const int2 *__restrict__ evr, int ya, int yb, bool clear)
{
    const int W = g.ring_w, RB = g.ring_rows, r = g.r, c0 = r - g.xoff;
    const int slot_a = (ya + r) % RB;  // rows [ya, yb) occupy consecutive slots modulo RB
    if (clear) {
        const int xa = max(0, -c0), xb = min(g.nx, W - c0);   // image columns that have ring columns
        for (int y = ya; y < yb; ++y) {
            int slot = slot_a + (y - ya);
            if (slot >= RB) slot -= RB;
            const int2 lr = evr[y];
            for (int x = xa + threadIdx.x; x < xb; x += NT)
                if (x < lr.x || x >= lr.y) RingStoreM<MODE>::zero(ring, g.plane, slot * W + c0 + x);
        }
    }
    const int fb = evpre[yb];
    // TAB: the SIE deflection from the proposal's table (a uniform branch)
    auto pixels = [&](auto tab) {
        constexpr bool TAB = decltype(tab)::value;
        for (int f = evpre[ya] + threadIdx.x; f < fb; f += NT) {
            const uint32_t e = evl[f];
            const int y = (int)(e >> 16), x = (int)(e & 0xffffu);
            int slot = slot_a + (y - ya);
            if (slot >= RB) slot -= RB;
            if constexpr (mode_solved(MODE)) {
                constexpr int NCH = mode_channels(MODE);
                float ch[NCH];
                binned_pixel_channels<mode_light(MODE), mode_epl(MODE), TAB>(g, P, y, x, ch);
                RingStoreM<MODE>::put(ring, g.plane, slot * W + c0 + x, FVec<NCH>::make(ch));
            } else {
                const float v = binned_pixel<mode_epl(MODE), TAB>(g, P, y, x);
                RingStoreM<MODE>::put(ring, g.plane, slot * W + c0 + x, v);
                if constexpr (mode_base(MODE) == MODE_SPLIT) atomicMax(&f16_rowmax()[slot], __float_as_uint(fabsf(v)));
            }
        }
    };
    if (sie_tab<MODE>() && sie_use_table(P)) pixels(std::true_type{});
    else pixels(std::false_type{});
}

// The strip sweep shared by every kernel: binned rows enter the ring strip by
// strip, each binned row is computed once, and conv(y0, y1, strip) returns this
// thread's contribution (chi-square, or the NNLS moments) of output rows [y0, y1).
template <int MODE, int NT, typename Acc, typename Conv>
__device__ __forceinline__ Acc strip_sweep(const LensGeom &g, const PropBlock &P, void *ring,
                                           const uint32_t *__restrict__ evl, const int *__restrict__ evpre,
                                           const int2 *__restrict__ evr, Conv conv)
{
    const int ny = g.ny, r = g.r, H = g.strip_h, RB = g.ring_rows;
    const int nwords = (mode_base(MODE) == MODE_FP32 ? RB * g.ring_w
                        : mode_solved(MODE)            ? mode_channels(MODE) * RB * g.ring_w
                                                       : RB * g.ring_w * mode_planes(MODE) / 2) / 4;
    constexpr bool F16 = mode_base(MODE) == MODE_SPLIT;
    float4 *r4 = static_cast<float4 *>(ring);
    for (int i = threadIdx.x; i < nwords; i += NT) r4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (F16) {
        for (int i = threadIdx.x; i < RB; i += NT) {
            f16_rowmax()[i] = 0u;
            f16_rowscale()[i] = 1.0f;   // rows above the image stay zero at scale 1
        }
    }
    __syncthreads();
    // binned rows [0, r) precede the first strip
    fill_rows<MODE, NT>(g, P, ring, evl, evpre, evr, 0, min(r, ny), false);
    Acc acc{};
    int strip = 0;
    for (int y0 = 0; y0 < ny; y0 += H, ++strip) {
        __syncthreads();  // the previous strip is done reading the slots reused below
        const int ya = y0 + r, yb = y0 + H + r;  // new binned rows
        if (y0 > 0) {
            const int c0 = r - g.xoff, xa = max(0, -c0), xb = min(g.nx, g.ring_w - c0);
            for (int y = max(ya, ny); y < yb; ++y) {  // rows past the image: clear reused slots
                const int slot = (y + r) % RB;
                for (int x = xa + threadIdx.x; x < xb; x += NT)
                    RingStoreM<MODE>::zero(ring, g.plane, slot * g.ring_w + c0 + x);
            }
        }
        if (ya < ny) fill_rows<MODE, NT>(g, P, ring, evl, evpre, evr, ya, min(yb, ny), y0 > 0);
        __syncthreads();
        if constexpr (F16) {
            // the rows that entered the ring since the last conversion, as halves
            const int ca = y0 == 0 ? 0 : ya;
            convert_rows_f16<NT>(g, static_cast<uint16_t *>(ring), ca, yb);
            __syncthreads();
            clear_rowmax_f16<NT>(g, ca, yb);   // read for the last time above
        }
        acc += conv(y0, min(y0 + H, ny), strip);
    }
    return acc;
}

// Explicit amplitudes: lnL = C - chi^2 / 2, the per-thread chi-square sums
// reduced through a wave64 shuffle tree and a fixed-order sum over the waves.
template <int MODE, int NT, typename Conv>
__device__ __forceinline__ void strip_loop(const LensGeom &g, const PropBlock &P, void *ring,
                                           const uint32_t *__restrict__ evl, const int *__restrict__ evpre,
                                           const int2 *__restrict__ evr, double *__restrict__ out,
                                           int64_t p, Conv conv)
{
    __shared__ double red[NT / 64];
    if constexpr (mode_epl(MODE)) epl_setup(P);   // published by strip_sweep's first barrier
    if constexpr (sie_tab<MODE>()) sie_setup(P);  // likewise
    double acc = strip_sweep<MODE, NT, double>(g, P, ring, evl, evpre, evr, conv);
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        out[p] = g.norm - 0.5 * s;
    }
}

// Moments of the amplitude solve (Sec. 2.3) over the masked pixels, with the
// columns c_a of M (each light component at unit amplitude), the data d and
// the weights w = mask/sigma: F_ab = sum (w c_a)(w c_b) (upper triangle, row by
// row) and g_a = sum (w c_a)(w d).  FP64 sums of products of FP32 values.
template <int NCH>
struct MomN {
    static constexpr int NF = NCH * (NCH + 1) / 2, NM = NF + NCH;
    double m[NM];
    __device__ MomN &operator+=(const MomN &o)
    {
#pragma unroll
        for (int i = 0; i < NM; ++i) m[i] += o.m[i];
        return *this;
    }
    __device__ void add(const double (&c)[NCH], float d, float w)
    {
        double wc[NCH];
        const double wd = (double)w * (double)d;
#pragma unroll
        for (int a = 0; a < NCH; ++a) wc[a] = (double)w * c[a];
        int i = 0;
#pragma unroll
        for (int a = 0; a < NCH; ++a)
#pragma unroll
            for (int b = a; b < NCH; ++b, ++i) m[i] = fma(wc[a], wc[b], m[i]);
#pragma unroll
        for (int a = 0; a < NCH; ++a) m[NF + a] = fma(wc[a], wd, m[NF + a]);
    }
};

// Non-negative least squares in NCH <= 4 variables (Sec. 2.3): the minimiser of
// chi^2(s) = D - 2 s.g + s.F s over s >= 0 is the least-squares solution on one
// of the 2^NCH supports that is feasible and has the smallest chi^2; on a
// support S the optimum has F_S s_S = g_S, so chi^2 = D - s_S.g_S.  Each
// support's system is solved by Gaussian elimination with partial pivoting
// and skipped when singular (a pivot below 1e-13 of the largest diagonal
// entry).  D = sum (wd)^2.  Returns chi^2 (>= 0) and the amplitudes.
template <int NCH>
__device__ inline double nnls_small(const MomN<NCH> &mo, double D, double (&best_s)[NCH])
{
    constexpr int NF = MomN<NCH>::NF;
    double F[NCH][NCH];
    int i = 0;
    for (int a = 0; a < NCH; ++a)
        for (int b = a; b < NCH; ++b) F[a][b] = F[b][a] = mo.m[i++];
    double dmax = 0.0;
    for (int a = 0; a < NCH; ++a) dmax = fmax(dmax, fabs(F[a][a]));
    double best = D;
    for (int a = 0; a < NCH; ++a) best_s[a] = 0.0;
    for (int S = 1; S < (1 << NCH); ++S) {
        int idx[NCH], m = 0;
        for (int a = 0; a < NCH; ++a)
            if (S & (1 << a)) idx[m++] = a;
        double A[NCH][NCH], b[NCH], x[NCH];
        for (int r = 0; r < m; ++r) {
            b[r] = mo.m[NF + idx[r]];
            for (int c = 0; c < m; ++c) A[r][c] = F[idx[r]][idx[c]];
        }
        bool ok = dmax > 0.0;
        for (int col = 0; col < m && ok; ++col) {
            int piv = col;
            for (int r = col + 1; r < m; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            if (!(fabs(A[piv][col]) > 1e-13 * dmax)) {
                ok = false;
                break;
            }
            if (piv != col) {
                for (int c = 0; c < m; ++c) {
                    const double t = A[col][c];
                    A[col][c] = A[piv][c];
                    A[piv][c] = t;
                }
                const double t = b[col];
                b[col] = b[piv];
                b[piv] = t;
            }
            for (int r = col + 1; r < m; ++r) {
                const double f = A[r][col] / A[col][col];
                for (int c = col; c < m; ++c) A[r][c] -= f * A[col][c];
                b[r] -= f * b[col];
            }
        }
        if (!ok) continue;
        for (int r = m - 1; r >= 0; --r) {
            double acc = b[r];
            for (int c = r + 1; c < m; ++c) acc -= A[r][c] * x[c];
            x[r] = acc / A[r][r];
        }
        bool feasible = true;
        double sg = 0.0;
        for (int r = 0; r < m; ++r) {
            feasible = feasible && x[r] >= 0.0;
            sg += x[r] * mo.m[NF + idx[r]];
        }
        const double c2 = D - sg;
        if (feasible && c2 < best) {
            best = c2;
            for (int a = 0; a < NCH; ++a) best_s[a] = 0.0;
            for (int r = 0; r < m; ++r) best_s[idx[r]] = x[r];
        }
    }
    return fmax(best, 0.0);
}

// Solved amplitudes: the moments reduced like the chi-square, then one thread
// solves and writes lnL = C - chi^2 / 2 (and, if amp is not null, the NCH
// amplitudes of proposal p at amp[NCH p ...]).
template <int MODE, int NT, typename Conv>
__device__ __forceinline__ void strip_loop_solved(const LensGeom &g, const PropBlock &P, void *ring,
                                                  const uint32_t *__restrict__ evl, const int *__restrict__ evpre,
                                                  const int2 *__restrict__ evr, double *__restrict__ out,
                                                  double *__restrict__ amp, int64_t p, Conv conv)
{
    constexpr int NCH = mode_channels(MODE), NM = MomN<NCH>::NM;
    __shared__ double red[NM][NT / 64];
    if constexpr (mode_epl(MODE)) epl_setup(P);   // published by strip_sweep's first barrier
    if constexpr (sie_tab<MODE>()) sie_setup(P);  // likewise
    if constexpr (NCH >= 2) {
        // each strip's moments are reduced over the wave and added to the
        // wave's LDS slots at once, so that no FP64 accumulators stay live
        // through the next strip's ray trace
        for (int i = threadIdx.x; i < NM * (NT / 64); i += NT) (&red[0][0])[i] = 0.0;
        (void)strip_sweep<MODE, NT, MomN<NCH>>(g, P, ring, evl, evpre, evr, [&](int y0, int y1, int st) {
            MomN<NCH> mo = conv(y0, y1, st);
#pragma unroll
            for (int i = 0; i < NM; ++i) mo.m[i] = wave_sum(mo.m[i]);
            if ((threadIdx.x & 63) == 0)
                for (int i = 0; i < NM; ++i) red[i][threadIdx.x >> 6] += mo.m[i];
            return MomN<NCH>{};
        });
    } else {
        // one channel: few moments, a single reduction at the end
        MomN<NCH> mo = strip_sweep<MODE, NT, MomN<NCH>>(g, P, ring, evl, evpre, evr, conv);
#pragma unroll
        for (int i = 0; i < NM; ++i) mo.m[i] = wave_sum(mo.m[i]);
        if ((threadIdx.x & 63) == 0)
            for (int i = 0; i < NM; ++i) red[i][threadIdx.x >> 6] = mo.m[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        MomN<NCH> t{};
        for (int w = 0; w < NT / 64; ++w)
            for (int i = 0; i < NM; ++i) t.m[i] += red[i][w];
        double s[NCH];
        const double chi2 = nnls_small<NCH>(t, g.dd, s);
        out[p] = g.norm - 0.5 * chi2;
        if (amp)
            for (int a = 0; a < NCH; ++a) amp[NCH * p + a] = s[a];
    }
}

// ---------------------------------------------------------------------------
// FP32 PSF convolution on the vector ALU
// ---------------------------------------------------------------------------
// chi-square contribution of output rows [ya, yb): four horizontally adjacent
// outputs per thread, the window of each PSF row held in registers, PSF
// weights read through the scalar cache.  Row partial sums are accumulated
// separately (blocked summation).
template <int K, int NT>
__device__ __forceinline__ double conv_rows(const LensGeom &g, const float *ring, const float *__restrict__ psf,
                                            const uint32_t *__restrict__ cvl, const int *__restrict__ cvpre,
                                            const float *__restrict__ data, const float *__restrict__ wgt,
                                            int ya, int yb)
{
    constexpr int KC = (K + 6) / 4;
    const int W = g.ring_w, RB = g.ring_rows;
    double acc = 0.0;
    const int gb = cvpre[yb];
    for (int gi = cvpre[ya] + threadIdx.x; gi < gb; gi += NT) {
        const uint32_t e = cvl[gi];
        const int y = (int)(e >> 16), x0 = (int)(e & 0xffffu);
        double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;   // sum over PSF rows in FP64
        int slot = y % RB;  // ring slot of binned row y - r
#pragma unroll 1
        for (int a = 0; a < K; ++a) {
            const float4 *rowp = reinterpret_cast<const float4 *>(ring + slot * W + x0 - g.xoff);
            float win[4 * KC];
#pragma unroll
            for (int i = 0; i < KC; ++i) {
                const float4 t = rowp[i];
                win[4 * i + 0] = t.x;
                win[4 * i + 1] = t.y;
                win[4 * i + 2] = t.z;
                win[4 * i + 3] = t.w;
            }
            const float *kr = psf + a * K;
            float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
            for (int b = 0; b < K; ++b) {
                const float w = kr[b];
                p0 = fmaf(w, win[b + 0], p0);
                p1 = fmaf(w, win[b + 1], p1);
                p2 = fmaf(w, win[b + 2], p2);
                p3 = fmaf(w, win[b + 3], p3);
            }
            o0 += (double)p0;
            o1 += (double)p1;
            o2 += (double)p2;
            o3 += (double)p3;
            slot = (slot + 1 == RB) ? 0 : slot + 1;
        }
        const float4 d = *reinterpret_cast<const float4 *>(data + (size_t)y * g.pitch + x0);
        const float4 w = *reinterpret_cast<const float4 *>(wgt + (size_t)y * g.pitch + x0);
        const double r0 = ((double)d.x - o0) * (double)w.x;
        const double r1 = ((double)d.y - o1) * (double)w.y;
        const double r2 = ((double)d.z - o2) * (double)w.z;
        const double r3 = ((double)d.w - o3) * (double)w.w;
        acc = fma(r0, r0, acc);
        acc = fma(r1, r1, acc);
        acc = fma(r2, r2, acc);
        acc = fma(r3, r3, acc);
    }
    return acc;
}

template <int K, int NT>
__global__ void __launch_bounds__(NT)
k_loglike_fp32(const LensGeom g, const PropBlock *__restrict__ pc, const float *__restrict__ psf,
               const uint32_t *__restrict__ evl, const int *__restrict__ evpre, const int2 *__restrict__ evr,
               const uint32_t *__restrict__ cvl, const int *__restrict__ cvpre,
               const float *__restrict__ data, const float *__restrict__ wgt, double *__restrict__ out)
{
    extern __shared__ float4 lds4[];
    float *ring = reinterpret_cast<float *>(lds4);
    const int64_t p = blockIdx.x;
    const PropBlock *c = pc + p;
    if (c->valid != 1.0) {
        if (threadIdx.x == 0) out[p] = -INFINITY;
        return;
    }
    const PropBlock P = *c;
    strip_loop<MODE_FP32, NT>(g, P, ring, evl, evpre, evr, out, p, [&](int y0, int y1, int) {
        return conv_rows<K, NT>(g, ring, psf, cvl, cvpre, data, wgt, y0, y1);
    });
}

// ---------------------------------------------------------------------------
// PSF convolution as a matrix-core contraction
// ---------------------------------------------------------------------------
// For a segment of 16 outputs x0..x0+15 of row y,
//   out[x0 + j] = sum_{a, i} T_a[j, i] w_a[i],  T_a[j, i] = Kf[a][i - j] (0 <= i - j < k),
//   w_a[i] = binned[y - r + a][x0 - r + i],  i < L (window_len: 16 + k - 1 rounded up),
// i.e. C = A B with A the banded Toeplitz expansion of the flipped PSF
// (16 x kL, built once per lens) and the B column of a segment its stacked
// PSF-row windows.  One v_mfma_f32_16x16x32_{bf16,f16} takes 32 of the kL
// products for 16 segments at once.  Operand layout (wave64): lane l holds A
// row l%16, B column l%16, K elements 8(l/16)..8(l/16)+7 of the 32; D rows
// 4(l/16)..+3 of column l%16.  The BF16 split3 forms the six products of three
// planes that reach 2^-24; the FP16 split is conv_tiles_f16.
template <int MODE>
__device__ __forceinline__ f32x4 mfma_products(const bf16x8 (&a)[3], const bf16x8 (&b)[3], f32x4 c)
{
    if (mode_base(MODE) == MODE_SPLIT3) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], c, 0, 0, 0);
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], c, 0, 0, 0);
}

// The FP32 accumulator of the contraction is added into FP64 sums every
// kFlushChunks K-chunks: summed over all k L products in FP32, an output
// collects a rounding error at every accumulate step relative to its whole
// running sum, which reached ~5e-7 of the lnL error metric on the 200x200 /
// 41x41 workload; flushed, each FP32 partial is a short sum.
constexpr int kFlushChunks = 2;

// NTL tiles of 16 segments starting at segment t (tile j: t + 16 j ..), with
// one load of each A chunk shared by the tiles: per output the same products
// in the same order as a tile alone.  Lanes past the strip's last segment s1
// compute a discarded column.  Returns this lane's chi-square contribution.
template <int MODE, int NTL>
__device__ __forceinline__ double conv_tiles(const LensGeom &g, const uint16_t *ring, const uint4 *__restrict__ aop,
                                             const uint32_t *__restrict__ seg, const float *__restrict__ data,
                                             const float *__restrict__ wgt, int t, int s0, int s1)
{
    constexpr int NPL = mode_planes(MODE);
    const int lane = threadIdx.x & 63, n = lane & 15, kb = lane >> 4;
    const int W = g.ring_w, RB = g.ring_rows, L = g.L, nch = g.nchunks, plane = g.plane;
    int i = 8 * kb, adv = 0;     // window offset of this lane's K elements (K = 8 kb), and the rows it skips
    while (i >= L) {             // (only for L < 32)
        i -= L;
        ++adv;
    }
    bool dummy[NTL];
    int y[NTL], x0[NTL], slot[NTL];
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
        dummy[j] = t + 16 * j + n >= s1;
        const uint32_t e = dummy[j] ? seg[s0] : seg[t + 16 * j + n];
        y[j] = (int)(e >> 16);
        x0[j] = (int)(e & 0xffffu);
        slot[j] = (y[j] % RB + adv) % RB;   // ring slot of binned row y - r + a
    }
    double o[NTL][4] = {};       // outputs 4 kb .. 4 kb + 3 of column n, FP64
    gptr4 ap = (gptr4)aop + lane;
    for (int ch0 = 0; ch0 < nch; ch0 += kFlushChunks) {
        f32x4 c[NTL];
#pragma unroll
        for (int j = 0; j < NTL; ++j) c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int ch1 = min(ch0 + kFlushChunks, nch);
        for (int ch = ch0; ch < ch1; ++ch) {
            bf16x8 av[3];
#pragma unroll
            for (int q = 0; q < NPL; ++q) av[q] = __builtin_bit_cast(bf16x8, ap[q * 64]);
#pragma unroll
            for (int j = 0; j < NTL; ++j) {
                bf16x8 bv[3];
                const uint16_t *bp = ring + (x0[j] - g.xoff) + slot[j] * W + i;
#pragma unroll
                for (int q = 0; q < NPL; ++q)
                    bv[q] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(bp + q * plane));
                c[j] = mfma_products<MODE>(av, bv, c[j]);
            }
            ap += NPL * 64;
            i += 32;
            while (i >= L) {
                i -= L;
#pragma unroll
                for (int j = 0; j < NTL; ++j) slot[j] = slot[j] + 1 == RB ? 0 : slot[j] + 1;
            }
        }
#pragma unroll
        for (int j = 0; j < NTL; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) o[j][v] += (double)c[j][v];
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
        if (dummy[j]) continue;
        const int xo = x0[j] + 4 * kb;
        const float4 d = *reinterpret_cast<const float4 *>(data + (size_t)y[j] * g.pitch + xo);
        const float4 w = *reinterpret_cast<const float4 *>(wgt + (size_t)y[j] * g.pitch + xo);
        const double r0 = ((double)d.x - o[j][0]) * (double)w.x;
        const double r1 = ((double)d.y - o[j][1]) * (double)w.y;
        const double r2 = ((double)d.z - o[j][2]) * (double)w.z;
        const double r3 = ((double)d.w - o[j][3]) * (double)w.w;
        acc = fma(r0, r0, acc);
        acc = fma(r1, r1, acc);
        acc = fma(r2, r2, acc);
        acc = fma(r3, r3, acc);
    }
    return acc;
}

// The FP16 split: the PSF (scaled by 2^j, conv_scale = 2^-j) and each ring row
// (at its own scale) as hi + lo halves, three products a_hi b_hi + a_lo b_hi +
// a_hi b_lo per tap (the dropped a_lo b_lo and both truncations are each below
// 2^-22 of the tap's product).  A PSF row's window is CPR = L / 32 whole
// K-chunks of one ring row, so the FP32 partial of each PSF row is flushed to
// the FP64 output times the two scales, exactly (powers of two).  A PSF
// row's A operands are loaded from L2 and its B operands from LDS at the start
// of the row (loading the next row's A during this row's products measured
// slower: a wave per SIMD of registers with two tiles, or without the tiles'
// shared A loads with one).  Same operand layout and output mapping as
// conv_tiles.
template <int NTL, int CPR>
__device__ __forceinline__ double conv_tiles_f16(const LensGeom &g, const uint16_t *ring,
                                                 const uint4 *__restrict__ aop, const uint32_t *__restrict__ seg,
                                                 const float *__restrict__ data, const float *__restrict__ wgt, int t,
                                                 int s0, int s1)
{
    const int lane = threadIdx.x & 63, n = lane & 15, kb = lane >> 4;
    const int W = g.ring_w, RB = g.ring_rows, plane = g.plane, k = g.k;
    const float *rs = f16_rowscale();
    bool dummy[NTL];
    int y[NTL], x0[NTL], slot[NTL];
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
        dummy[j] = t + 16 * j + n >= s1;
        const uint32_t e = dummy[j] ? seg[s0] : seg[t + 16 * j + n];
        y[j] = (int)(e >> 16);
        x0[j] = (int)(e & 0xffffu);
        slot[j] = y[j] % RB;   // ring slot of binned row y - r + a at a = 0
    }
    double o[NTL][4] = {};     // outputs 4 kb .. 4 kb + 3 of column n, FP64
    gptr4 ap = (gptr4)aop + lane;
    for (int a = 0; a < k; ++a) {
        f32x4 c[NTL];
        lptr16 bp[NTL];
#pragma unroll
        for (int j = 0; j < NTL; ++j) {
            c[j] = f32x4{0.f, 0.f, 0.f, 0.f};
            bp[j] = (lptr16)ring + slot[j] * W + (x0[j] - g.xoff) + 8 * kb;
        }
#pragma unroll
        for (int h = 0; h < CPR; ++h) {
            const f16x8 a0 = __builtin_bit_cast(f16x8, ap[0]), a1 = __builtin_bit_cast(f16x8, ap[64]);
            ap += 2 * 64;
#pragma unroll
            for (int j = 0; j < NTL; ++j) {
                const f16x8 b0 = __builtin_bit_cast(f16x8, *(lptr4)(bp[j] + 32 * h));
                const f16x8 b1 = __builtin_bit_cast(f16x8, *(lptr4)(bp[j] + 32 * h + plane));
                c[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b1, c[j], 0, 0, 0);
                c[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, b0, c[j], 0, 0, 0);
                c[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, b0, c[j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < NTL; ++j) {
            const double sc = (double)rs[slot[j]] * g.conv_scale;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[j][v] = fma((double)c[j][v], sc, o[j][v]);
            slot[j] = slot[j] + 1 == RB ? 0 : slot[j] + 1;
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
        if (dummy[j]) continue;
        const int xo = x0[j] + 4 * kb;
        const float4 d = *reinterpret_cast<const float4 *>(data + (size_t)y[j] * g.pitch + xo);
        const float4 w = *reinterpret_cast<const float4 *>(wgt + (size_t)y[j] * g.pitch + xo);
        const double r0 = ((double)d.x - o[j][0]) * (double)w.x;
        const double r1 = ((double)d.y - o[j][1]) * (double)w.y;
        const double r2 = ((double)d.z - o[j][2]) * (double)w.z;
        const double r3 = ((double)d.w - o[j][3]) * (double)w.w;
        acc = fma(r0, r0, acc);
        acc = fma(r1, r1, acc);
        acc = fma(r2, r2, acc);
        acc = fma(r3, r3, acc);
    }
    return acc;
}

// Two tiles at a time where two are left (PSF rows of three K-chunks, k > 49:
// one at a time, which keeps the registers of the prefetched operands at the
// two-chunk level).
template <int CPR>
__device__ __forceinline__ double conv_pair_f16(const LensGeom &g, const uint16_t *ring, const uint4 *__restrict__ aop,
                                                const uint32_t *__restrict__ seg, const float *__restrict__ data,
                                                const float *__restrict__ wgt, int t, int s0, int s1)
{
    if (CPR <= 2 && t + 16 < s1) return conv_tiles_f16<2, CPR>(g, ring, aop, seg, data, wgt, t, s0, s1);
    double acc = conv_tiles_f16<1, CPR>(g, ring, aop, seg, data, wgt, t, s0, s1);
    if (CPR > 2 && t + 16 < s1) acc += conv_tiles_f16<1, CPR>(g, ring, aop, seg, data, wgt, t + 16, s0, s1);
    return acc;
}

// Chi-square contribution of output rows [ya, yb): each wave takes two tiles
// of 16 segments at a time (one where only one is left), so that every A
// chunk loaded from L2 feeds two matrix-core products.
template <int MODE, int NT>
__device__ __forceinline__ double conv_mfma(const LensGeom &g, const uint16_t *ring,
                                            const uint4 *__restrict__ aop, const uint32_t *__restrict__ seg,
                                            const int *__restrict__ segpre, const float *__restrict__ data,
                                            const float *__restrict__ wgt, int ya, int yb)
{
    const int wave = threadIdx.x >> 6;
    double acc = 0.0;
    const int s0 = segpre[ya], s1 = segpre[yb];
    for (int t = s0 + 32 * wave; t < s1; t += 32 * (NT / 64)) {
        if constexpr (mode_base(MODE) == MODE_SPLIT) {
            // K-chunks per PSF row: window_len(k) / 32, at most 3 (k <= 63)
            const int cpr = g.L >> 5;
            if (cpr == 2) acc += conv_pair_f16<2>(g, ring, aop, seg, data, wgt, t, s0, s1);
            else if (cpr == 1) acc += conv_pair_f16<1>(g, ring, aop, seg, data, wgt, t, s0, s1);
            else acc += conv_pair_f16<3>(g, ring, aop, seg, data, wgt, t, s0, s1);
        } else {
            if (t + 16 < s1) acc += conv_tiles<MODE, 2>(g, ring, aop, seg, data, wgt, t, s0, s1);
            else acc += conv_tiles<MODE, 1>(g, ring, aop, seg, data, wgt, t, s0, s1);
        }
    }
    return acc;
}

template <int MODE, int NT>
__global__ void __launch_bounds__(NT)
k_loglike_mfma(const LensGeom g, const PropBlock *__restrict__ pc, const uint32_t *__restrict__ evl,
               const int *__restrict__ evpre, const int2 *__restrict__ evr, const uint4 *__restrict__ aop,
               const uint32_t *__restrict__ seg, const int *__restrict__ segpre, const float *__restrict__ data,
               const float *__restrict__ wgt, double *__restrict__ out)
{
    extern __shared__ float4 lds4[];
    uint16_t *ring = reinterpret_cast<uint16_t *>(lds4);
    const int64_t p = blockIdx.x;
    const PropBlock *c = pc + p;
    if (c->valid != 1.0) {
        if (threadIdx.x == 0) out[p] = -INFINITY;
        return;
    }
    const PropBlock P = *c;
    strip_loop<MODE, NT>(g, P, ring, evl, evpre, evr, out, p, [&](int y0, int y1, int) {
        return conv_mfma<MODE, NT>(g, ring, aop, seg, segpre, data, wgt, y0, y1);
    });
}

// ---------------------------------------------------------------------------
// persistent multi-lens kernel
// ---------------------------------------------------------------------------
// FP32 convolution with the PSF side chosen at run time (each lens of a batch
// has its own).  It issues, for every output, the same fmaf sequence as
// conv_rows<K> (weights in ascending order within a PSF row, row partials added
// in ascending row order), so batch and single-lens results agree bit for
// bit; the window slides through four registers instead of a K-sized array,
// which keeps the batch kernel's register count at the single-lens level.
template <int NT>
__device__ __forceinline__ double conv_rows_rt(const LensGeom &g, const float *ring, int ya, int yb)
{
    const int W = g.ring_w, RB = g.ring_rows, k = g.k;
    const float *__restrict__ psf = g.psf;
    double acc = 0.0;
    const int gb = g.cvpre[yb];
    for (int gi = g.cvpre[ya] + threadIdx.x; gi < gb; gi += NT) {
        const uint32_t e = g.cvl[gi];
        const int y = (int)(e >> 16), x0 = (int)(e & 0xffffu);
        double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;   // sum over PSF rows in FP64
        int slot = y % RB;
        for (int a = 0; a < k; ++a) {
            const float *row = ring + slot * W + x0 - g.xoff;
            const float *kr = psf + a * k;
            float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
            float v0 = row[0], v1 = row[1], v2 = row[2];
            int b = 0;
            for (; b + 4 <= k; b += 4) {
                const float w0 = kr[b], w1 = kr[b + 1], w2 = kr[b + 2], w3 = kr[b + 3];
                const float v3 = row[b + 3], v4 = row[b + 4], v5 = row[b + 5], v6 = row[b + 6];
                p0 = fmaf(w0, v0, p0); p1 = fmaf(w0, v1, p1); p2 = fmaf(w0, v2, p2); p3 = fmaf(w0, v3, p3);
                p0 = fmaf(w1, v1, p0); p1 = fmaf(w1, v2, p1); p2 = fmaf(w1, v3, p2); p3 = fmaf(w1, v4, p3);
                p0 = fmaf(w2, v2, p0); p1 = fmaf(w2, v3, p1); p2 = fmaf(w2, v4, p2); p3 = fmaf(w2, v5, p3);
                p0 = fmaf(w3, v3, p0); p1 = fmaf(w3, v4, p1); p2 = fmaf(w3, v5, p2); p3 = fmaf(w3, v6, p3);
                v0 = v4; v1 = v5; v2 = v6;
            }
            for (; b < k; ++b) {
                const float w = kr[b], v3 = row[b + 3];
                p0 = fmaf(w, v0, p0); p1 = fmaf(w, v1, p1); p2 = fmaf(w, v2, p2); p3 = fmaf(w, v3, p3);
                v0 = v1; v1 = v2; v2 = v3;
            }
            o0 += (double)p0;
            o1 += (double)p1;
            o2 += (double)p2;
            o3 += (double)p3;
            slot = (slot + 1 == RB) ? 0 : slot + 1;
        }
        const float4 d = *reinterpret_cast<const float4 *>(g.data + (size_t)y * g.pitch + x0);
        const float4 w = *reinterpret_cast<const float4 *>(g.wgt + (size_t)y * g.pitch + x0);
        const double r0 = ((double)d.x - o0) * (double)w.x;
        const double r1 = ((double)d.y - o1) * (double)w.y;
        const double r2 = ((double)d.z - o2) * (double)w.z;
        const double r3 = ((double)d.w - o3) * (double)w.w;
        acc = fma(r0, r0, acc);
        acc = fma(r1, r1, acc);
        acc = fma(r2, r2, acc);
        acc = fma(r3, r3, acc);
    }
    return acc;
}

// Solved amplitudes: the NCH unit-amplitude channels convolved with the
// runtime-k sliding window of conv_rows_rt (the same fmaf order per channel),
// and the moments of the amplitude solve accumulated in FP64 from the FP32
// columns, data and weights.
template <int MODE, int NT>
__device__ __forceinline__ MomN<mode_channels(MODE)> conv_rows_solved(const LensGeom &g,
                                                                      const typename FVec<mode_channels(MODE)>::T *ring,
                                                                      int ya, int yb)
{
    constexpr int NCH = mode_channels(MODE);
    // channels convolved in passes of at most two, so that four channels keep
    // the register footprint of two
    constexpr int CP = NCH < 2 ? NCH : 2, NPASS = NCH / CP;
    typedef FVec<CP> V;
    const typename V::T *ringp = reinterpret_cast<const typename V::T *>(ring);
    const int W = g.ring_w, RB = g.ring_rows, k = g.k;
    const float *__restrict__ psf = g.psf;
    MomN<NCH> mo{};
    const int gb = g.cvpre[yb];
    for (int gi = g.cvpre[ya] + threadIdx.x; gi < gb; gi += NT) {
        const uint32_t e = g.cvl[gi];
        const int y = (int)(e >> 16), x0 = (int)(e & 0xffffu);
        double o[4][NCH] = {};   // sums over PSF rows in FP64
#pragma unroll
        for (int pass = 0; pass < NPASS; ++pass) {
            int slot = y % RB;
            for (int a = 0; a < k; ++a) {
                const typename V::T *row = ringp + (size_t)(slot * W + x0 - g.xoff) * NPASS + pass;
                const float *kr = psf + a * k;
                float pp[4][CP] = {};
                typename V::T v0 = row[0], v1 = row[NPASS], v2 = row[2 * NPASS];
                // one channel: four taps per step (their weights fetched
                // together), then the tail; more channels: one tap per step
                // (fewer live registers: one more resident workgroup per CU for
                // two channels, 8.8e5 against 7.8e5 evals/s).  Per output and
                // channel the fmaf order is ascending in b either way.
                int b = 0;
                for (; NCH == 1 && b + 4 <= k; b += 4) {
                    const float w0 = kr[b], w1 = kr[b + 1], w2 = kr[b + 2], w3 = kr[b + 3];
                    const typename V::T v3 = row[(b + 3) * NPASS], v4 = row[(b + 4) * NPASS];
                    const typename V::T v5 = row[(b + 5) * NPASS], v6 = row[(b + 6) * NPASS];
#pragma unroll
                    for (int c = 0; c < CP; ++c) {
                        pp[0][c] = fmaf(w0, V::at(v0, c), pp[0][c]);
                        pp[1][c] = fmaf(w0, V::at(v1, c), pp[1][c]);
                        pp[2][c] = fmaf(w0, V::at(v2, c), pp[2][c]);
                        pp[3][c] = fmaf(w0, V::at(v3, c), pp[3][c]);
                        pp[0][c] = fmaf(w1, V::at(v1, c), pp[0][c]);
                        pp[1][c] = fmaf(w1, V::at(v2, c), pp[1][c]);
                        pp[2][c] = fmaf(w1, V::at(v3, c), pp[2][c]);
                        pp[3][c] = fmaf(w1, V::at(v4, c), pp[3][c]);
                        pp[0][c] = fmaf(w2, V::at(v2, c), pp[0][c]);
                        pp[1][c] = fmaf(w2, V::at(v3, c), pp[1][c]);
                        pp[2][c] = fmaf(w2, V::at(v4, c), pp[2][c]);
                        pp[3][c] = fmaf(w2, V::at(v5, c), pp[3][c]);
                        pp[0][c] = fmaf(w3, V::at(v3, c), pp[0][c]);
                        pp[1][c] = fmaf(w3, V::at(v4, c), pp[1][c]);
                        pp[2][c] = fmaf(w3, V::at(v5, c), pp[2][c]);
                        pp[3][c] = fmaf(w3, V::at(v6, c), pp[3][c]);
                    }
                    v0 = v4;
                    v1 = v5;
                    v2 = v6;
                }
                for (; b < k; ++b) {
                    const float w = kr[b];
                    const typename V::T v3 = row[(b + 3) * NPASS];
#pragma unroll
                    for (int c = 0; c < CP; ++c) {
                        pp[0][c] = fmaf(w, V::at(v0, c), pp[0][c]);
                        pp[1][c] = fmaf(w, V::at(v1, c), pp[1][c]);
                        pp[2][c] = fmaf(w, V::at(v2, c), pp[2][c]);
                        pp[3][c] = fmaf(w, V::at(v3, c), pp[3][c]);
                    }
                    v0 = v1;
                    v1 = v2;
                    v2 = v3;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int c = 0; c < CP; ++c) o[j][CP * pass + c] += (double)pp[j][c];
                slot = (slot + 1 == RB) ? 0 : slot + 1;
            }
        }
        const float4 d = *reinterpret_cast<const float4 *>(g.data + (size_t)y * g.pitch + x0);
        const float4 w = *reinterpret_cast<const float4 *>(g.wgt + (size_t)y * g.pitch + x0);
        mo.add(o[0], d.x, w.x);
        mo.add(o[1], d.y, w.y);
        mo.add(o[2], d.z, w.z);
        mo.add(o[3], d.w, w.w);
    }
    return mo;
}

// Light amplitudes solved by NNLS (Sec. 2.3), for the light model of MODE: one
// workgroup per proposal, the NCH channels through the LDS ring and the FP32
// convolution, the moments reduced and the problem solved in the workgroup.
// amp (may be null): [n][NCH].
template <int MODE, int NT>
__global__ void __launch_bounds__(NT)
k_loglike_nnls(const LensGeom g, const PropBlock *__restrict__ pc, double *__restrict__ out,
               double *__restrict__ amp)
{
    constexpr int NCH = mode_channels(MODE);
    extern __shared__ float4 lds4[];
    auto *ring = reinterpret_cast<typename FVec<NCH>::T *>(lds4);
    const int64_t p = blockIdx.x;
    const PropBlock *c = pc + p;
    if (c->valid == 0.0) {
        if (threadIdx.x == 0) {
            out[p] = -INFINITY;
            if (amp)
                for (int a = 0; a < NCH; ++a) amp[NCH * p + a] = NAN;
        }
        return;
    }
    const PropBlock P = *c;
    strip_loop_solved<MODE, NT>(g, P, ring, g.evl, g.evpre, g.evr, out, amp, p, [&](int y0, int y1, int) {
        return conv_rows_solved<MODE, NT>(g, ring, y0, y1);
    });
}

// Explicit amplitudes with the PSF side chosen at run time (conv_rows_rt): the
// elliptical power-law lenses, whose ray trace is too long for the PSF-size
// templates of k_loglike_fp32 to pay.
template <int MODE, int NT>
__global__ void __launch_bounds__(NT) k_loglike_rt(const LensGeom g, const PropBlock *__restrict__ pc,
                                                   double *__restrict__ out)
{
    extern __shared__ float4 lds4[];
    float *ring = reinterpret_cast<float *>(lds4);
    const int64_t p = blockIdx.x;
    const PropBlock *c = pc + p;
    if (c->valid != 1.0) {
        if (threadIdx.x == 0) out[p] = -INFINITY;
        return;
    }
    const PropBlock P = *c;
    strip_loop<MODE, NT>(g, P, ring, g.evl, g.evpre, g.evr, out, p,
                         [&](int y0, int y1, int) { return conv_rows_rt<NT>(g, ring, y0, y1); });
}

__global__ void k_reset_counter(unsigned int *counter) { *counter = 0u; }

// Work items are (lens, proposal) pairs numbered lens-major in the batch's
// order (longest per-proposal cost first); item i belongs to the lens j with
// lstart[j] <= i < lstart[j + 1], and its result goes to out[lout[j] + i - lstart[j]].
// Each workgroup takes the next item from a global counter until none is left:
// every wave leaves the loop on the same item index, so the grid drains.
template <int MODE, int NT>
__global__ void __launch_bounds__(NT)
k_loglike_batch(const LensGeom *__restrict__ geoms, const int *__restrict__ lstart,
                const int64_t *__restrict__ lout, int nl, int nitems, const PropBlock *__restrict__ pc,
                double *__restrict__ out, unsigned int *__restrict__ counter)
{
    extern __shared__ float4 lds4[];
    __shared__ int s_item;
    // a workgroup never takes more than nitems items: the cap bounds the loop
    // even if the counter protocol were broken
    for (int iter = 0; iter <= nitems; ++iter) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // uniform across the workgroup: readfirstlane lets the compiler keep the
        // lens descriptor and the proposal constants in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= nitems) break;
        int lo = 0, hi = nl;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (lstart[mid] <= item) lo = mid; else hi = mid;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const LensGeom g = geoms[lo];
        const int64_t p = lout[lo] + (item - lstart[lo]);
        const PropBlock *c = pc + p;
        if (mode_solved(MODE) ? c->valid == 0.0 : c->valid != 1.0) {
            if (threadIdx.x == 0) out[p] = -INFINITY;
        } else {
            const PropBlock P = *c;
            if constexpr (mode_solved(MODE)) {
                auto *ring = reinterpret_cast<typename FVec<mode_channels(MODE)>::T *>(lds4);
                strip_loop_solved<MODE, NT>(g, P, ring, g.evl, g.evpre, g.evr, out, nullptr, p,
                                            [&](int y0, int y1, int) { return conv_rows_solved<MODE, NT>(g, ring, y0, y1); });
            } else if (mode_base(MODE) == MODE_FP32) {
                float *ring = reinterpret_cast<float *>(lds4);
                strip_loop<MODE, NT>(g, P, ring, g.evl, g.evpre, g.evr, out, p, [&](int y0, int y1, int) {
                    return conv_rows_rt<NT>(g, ring, y0, y1);
                });
            } else {
                uint16_t *ring = reinterpret_cast<uint16_t *>(lds4);
                strip_loop<MODE, NT>(g, P, ring, g.evl, g.evpre, g.evr, out, p, [&](int y0, int y1, int) {
                    return conv_mfma<MODE, NT>(g, ring, g.aop, g.seg, g.segpre, g.data, g.wgt, y0, y1);
                });
            }
        }
        // Reconverge before thread 0 takes the next item.  Without this barrier
        // the thread-0 result store above and the thread-0 atomic at the top of
        // the loop can be merged into one divergent region spanning the back
        // edge, and the other lanes would pass the next barrier before the new
        // item has been published.
        __syncthreads();
    }
}

template <bool F16>
__global__ void k_mfma_probe(const uint16_t *__restrict__ a, const uint16_t *__restrict__ b, float *__restrict__ d)
{
    // a: 16 x 32 row-major, b: 32 x 16 row-major, d: 16 x 16 row-major; one wave;
    // BF16 or (F16) IEEE-half operands
    const int l = threadIdx.x, n = l & 15, kb = l >> 4;
    uint16_t ta[8], tb[8];
    for (int e = 0; e < 8; ++e) {
        ta[e] = a[n * 32 + 8 * kb + e];
        tb[e] = b[(8 * kb + e) * 16 + n];
    }
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    if constexpr (F16)
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, *reinterpret_cast<const uint4 *>(ta)),
                                                   __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4 *>(tb)), c,
                                                   0, 0, 0);
    else
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(ta)),
                                                    __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(tb)),
                                                    c, 0, 0, 0);
    for (int v = 0; v < 4; ++v) d[(4 * kb + v) * 16 + n] = c[v];
}

// ---------------------------------------------------------------------------
// debug model images
// ---------------------------------------------------------------------------
template <bool EPL>
__global__ void k_model_binned(const LensGeom g, const PropBlock *__restrict__ pc, float *__restrict__ img)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const PropBlock P = *pc;
    if constexpr (EPL) {
        epl_setup(P);
        __syncthreads();
    }
    if (i >= g.ny * g.nx) return;
    img[i] = binned_pixel<EPL>(g, P, i / g.nx, i % g.nx);
}

__global__ void k_model_conv(const LensGeom g, const float *__restrict__ img, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.ny * g.nx) return;
    const int y = i / g.nx, x = i % g.nx, k = g.k, r = g.r;
    double o = 0.0;
    for (int a = 0; a < k; ++a) {
        const int yy = y - r + a;
        float pr = 0.0f;
        for (int b = 0; b < k; ++b) {
            const int xx = x - r + b;
            const float v = (yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx) ? img[yy * g.nx + xx] : 0.0f;
            pr = fmaf(g.psf[a * k + b], v, pr);
        }
        o += (double)pr;
    }
    out[i] = (float)o;
}

// ---------------------------------------------------------------------------
// fixed scratch of the allocation-free entry point
// ---------------------------------------------------------------------------
// Prepared constants of up to kNoAllocMax proposals: one array per device,
// held until the process ends.  In host code the name `scratch` is a host-side
// stand-in, not a device address; noalloc_init resolves the device address
// once per device and every launch takes that pointer.
static __device__ __align__(256) PropBlock scratch[kNoAllocMax];
static void *g_scratch_dev[kNoAllocDevices];
static std::mutex g_scratch_mu;

hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
    return hipSuccess;
}

PropBlock *noalloc_scratch(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return static_cast<PropBlock *>(g_scratch_dev[device]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int choose_kc(int k) { return (k + 6) / 4; }

double host_sersic_bn(double n) { return sersic_bn(n); }

// Output groups (4 wide, FP32) and segments (16 wide, matrix cores) start at
// multiples of 4 and 16 at or right of xoff, below xoff + span, and each reads
// a window of 4 KC or L ring columns from its start.
int ring_width(int mode, int k, int span)
{
    if (mode_base(mode) == MODE_FP32 || mode_solved(mode)) return (span + 3) / 4 * 4 + 4 * choose_kc(k);
    return (span + 15) / 16 * 16 + window_len(mode, k);
}

size_t ring_row_bytes(int mode, int k, int span)
{
    const size_t elem = mode_base(mode) == MODE_FP32 ? 4
                        : mode_solved(mode)          ? 4 * mode_channels(mode)
                                                     : 2 * mode_planes(mode);
    return (size_t)ring_width(mode, k, span) * elem;
}

size_t ring_bytes(const LensGeom &g) { return (size_t)g.ring_rows * ring_row_bytes(g.mode, g.k, g.span); }

// Dynamic LDS one workgroup may use: the opt-in limit when the device reports
// one above the default per-block limit (gfx950 addresses all 160 KB of a CU
// from one workgroup), never more than a CU holds.
size_t max_lds_bytes()
{
    int dev = 0, v = 0, optin = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        per_cu = 0;
    (void)hipGetLastError();
    size_t m = (size_t)std::max(v, optin);
    if (per_cu > 0) m = std::min(m, (size_t)per_cu);
    return m;
}

hipError_t launch_prep(const double *d_params, int64_t n, PropBlock *d_pc, int model, const int64_t *d_pstart,
                       const int *d_pmodel, int nl, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)nb), dim3(bs), 0, st, d_params, n, d_pc, model, d_pstart, d_pmodel, nl);
    return hipGetLastError();
}

template <int K, int NT>
static hipError_t launch_k(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, hipStream_t st)
{
    hipLaunchKernelGGL((k_loglike_fp32<K, NT>), dim3((unsigned)n), dim3(NT), ring_bytes(g), st, g, d_pc,
                       g.psf, g.evl, g.evpre, g.evr, g.cvl, g.cvpre, g.data, g.wgt, d_out);
    return hipGetLastError();
}

template <int NT>
static hipError_t launch_fp32_nt(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, hipStream_t st)
{
    switch (g.k) {
#define LENS_K(KK) \
    case KK: return launch_k<KK, NT>(g, d_pc, n, d_out, st);
        LENS_K(1) LENS_K(3) LENS_K(5) LENS_K(7) LENS_K(9) LENS_K(11) LENS_K(13) LENS_K(15)
        LENS_K(17) LENS_K(19) LENS_K(21) LENS_K(23) LENS_K(25) LENS_K(27) LENS_K(29) LENS_K(31)
        LENS_K(33) LENS_K(35) LENS_K(37) LENS_K(39) LENS_K(41) LENS_K(43) LENS_K(45) LENS_K(47)
        LENS_K(49) LENS_K(51) LENS_K(53) LENS_K(55) LENS_K(57) LENS_K(59) LENS_K(61) LENS_K(63)
#undef LENS_K
    default: return hipErrorInvalidValue;
    }
}

// Every mode, with the SIE and with the elliptical power law (MODE_EPL).
#define LENS_FOR_MODES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

// The single-lens likelihood kernel of a mode other than the SIE's FP32 one
// (which has one kernel per PSF side): runtime-k FP32, MFMA, or solved amplitudes.
template <int MODE, int NT>
static const void *mode_kernel_ptr()
{
    if constexpr (mode_solved(MODE)) return reinterpret_cast<const void *>(&k_loglike_nnls<MODE, NT>);
    else if constexpr (mode_base(MODE) == MODE_FP32) return reinterpret_cast<const void *>(&k_loglike_rt<MODE, NT>);
    else return reinterpret_cast<const void *>(&k_loglike_mfma<MODE, NT>);
}

template <int MODE, int NT>
static hipError_t launch_mode(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, double *d_amp,
                              hipStream_t st)
{
    if constexpr (mode_solved(MODE))
        hipLaunchKernelGGL((k_loglike_nnls<MODE, NT>), dim3((unsigned)n), dim3(NT), ring_bytes(g), st, g, d_pc, d_out,
                           d_amp);
    else if constexpr (mode_base(MODE) == MODE_FP32)
        hipLaunchKernelGGL((k_loglike_rt<MODE, NT>), dim3((unsigned)n), dim3(NT), ring_bytes(g), st, g, d_pc, d_out);
    else
        hipLaunchKernelGGL((k_loglike_mfma<MODE, NT>), dim3((unsigned)n), dim3(NT), ring_bytes(g), st, g, d_pc,
                           g.evl, g.evpre, g.evr, g.aop, g.seg, g.segpre, g.data, g.wgt, d_out);
    return hipGetLastError();
}

template <int NT>
static hipError_t launch_nt(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, double *d_amp,
                            hipStream_t st)
{
    if (g.mode == MODE_FP32) return launch_fp32_nt<NT>(g, d_pc, n, d_out, st);
    switch (g.mode) {
#define LENS_M(M) \
    case M: return launch_mode<M, NT>(g, d_pc, n, d_out, d_amp, st);
        LENS_FOR_MODES(LENS_M)
#undef LENS_M
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_loglike(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, double *d_amp,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (g.nt == 512) return launch_nt<512>(g, d_pc, n, d_out, d_amp, st);
    if (g.nt == 256) return launch_nt<256>(g, d_pc, n, d_out, d_amp, st);
    return hipErrorInvalidValue;
}

static const void *batch_kernel(int mode, int nt);

template <int NT>
static const void *loglike_kernel_nt(const LensGeom &g)
{
    if (g.mode != MODE_FP32) {
        switch (g.mode) {
#define LENS_M(M) \
    case M: return mode_kernel_ptr<M, NT>();
            LENS_FOR_MODES(LENS_M)
#undef LENS_M
        default: return nullptr;
        }
    }
    switch (g.k) {
#define LENS_K(KK) \
    case KK: return reinterpret_cast<const void *>(&k_loglike_fp32<KK, NT>);
        LENS_K(1) LENS_K(3) LENS_K(5) LENS_K(7) LENS_K(9) LENS_K(11) LENS_K(13) LENS_K(15)
        LENS_K(17) LENS_K(19) LENS_K(21) LENS_K(23) LENS_K(25) LENS_K(27) LENS_K(29) LENS_K(31)
        LENS_K(33) LENS_K(35) LENS_K(37) LENS_K(39) LENS_K(41) LENS_K(43) LENS_K(45) LENS_K(47)
        LENS_K(49) LENS_K(51) LENS_K(53) LENS_K(55) LENS_K(57) LENS_K(59) LENS_K(61) LENS_K(63)
#undef LENS_K
    default: return nullptr;
    }
}

int loglike_blocks_per_cu(const LensGeom &g)
{
    const void *k = g.nt == 512 ? loglike_kernel_nt<512>(g) : g.nt == 256 ? loglike_kernel_nt<256>(g) : nullptr;
    int nb = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, g.nt, ring_bytes(g)) != hipSuccess) return 0;
    return nb;
}

template <int NT>
static void likelihood_kernels_nt(std::vector<const void *> &v)
{
#define LENS_K(KK) v.push_back(reinterpret_cast<const void *>(&k_loglike_fp32<KK, NT>));
    LENS_K(1) LENS_K(3) LENS_K(5) LENS_K(7) LENS_K(9) LENS_K(11) LENS_K(13) LENS_K(15)
    LENS_K(17) LENS_K(19) LENS_K(21) LENS_K(23) LENS_K(25) LENS_K(27) LENS_K(29) LENS_K(31)
    LENS_K(33) LENS_K(35) LENS_K(37) LENS_K(39) LENS_K(41) LENS_K(43) LENS_K(45) LENS_K(47)
    LENS_K(49) LENS_K(51) LENS_K(53) LENS_K(55) LENS_K(57) LENS_K(59) LENS_K(61) LENS_K(63)
#undef LENS_K
#define LENS_M(M)                                 \
    if (M != MODE_FP32) v.push_back(mode_kernel_ptr<M, NT>()); \
    v.push_back(batch_kernel(M, NT));
    LENS_FOR_MODES(LENS_M)
#undef LENS_M
}

// Raise every ring-using kernel's dynamic-LDS limit so that dynamic plus
// static LDS reaches `bytes`.  Returns the dynamic bytes all of them accept
// (0 if the runtime refused any, leaving the default limit in force).
size_t set_lds_limits(size_t bytes)
{
    std::vector<const void *> ks;
    likelihood_kernels_nt<256>(ks);
    likelihood_kernels_nt<512>(ks);
    size_t usable = bytes;
    for (const void *k : ks) {
        hipFuncAttributes a{};
        if (!k || hipFuncGetAttributes(&a, k) != hipSuccess) return 0;
        const size_t dyn = bytes > a.sharedSizeBytes ? bytes - a.sharedSizeBytes : 0;
        if (dyn == 0 || hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess)
            return 0;
        usable = std::min(usable, dyn);
    }
    return usable;
}

size_t lds_per_cu()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || v <= 0) {
        (void)hipGetLastError();
        return 65536;
    }
    return (size_t)v;
}

static const void *batch_kernel(int mode, int nt)
{
    switch (mode) {
#define LENS_M(M)                                                                                    \
    case M:                                                                                          \
        return nt == 256 ? reinterpret_cast<const void *>(&k_loglike_batch<M, 256>)                  \
               : nt == 512 ? reinterpret_cast<const void *>(&k_loglike_batch<M, 512>) : nullptr;
        LENS_FOR_MODES(LENS_M)
#undef LENS_M
    default: return nullptr;
    }
}

size_t batch_static_lds(int mode, int nt)
{
    const void *k = batch_kernel(mode, nt);
    hipFuncAttributes a{};
    if (!k || hipFuncGetAttributes(&a, k) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return (size_t)a.sharedSizeBytes;
}

int batch_blocks_per_cu(int mode, int nt, size_t lds)
{
    const void *k = batch_kernel(mode, nt);
    int nb = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, nt, lds) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_batch(int mode, int nt, int grid, size_t lds, const LensGeom *d_geoms, const int *d_lstart,
                        const int64_t *d_lout, int nl, int nitems, const PropBlock *d_pc, double *d_out,
                        unsigned int *d_counter, hipStream_t st)
{
    const void *k = batch_kernel(mode, nt);
    if (!k || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&d_geoms, (void *)&d_lstart, (void *)&d_lout, (void *)&nl, (void *)&nitems,
                    (void *)&d_pc, (void *)&d_out, (void *)&d_counter};
    return hipLaunchKernel(k, dim3(grid), dim3(nt), args, lds, st);
}

hipError_t launch_mfma_probe(bool f16, const uint16_t *d_a, const uint16_t *d_b, float *d_d, hipStream_t st)
{
    if (f16) hipLaunchKernelGGL(k_mfma_probe<true>, dim3(1), dim3(64), 0, st, d_a, d_b, d_d);
    else hipLaunchKernelGGL(k_mfma_probe<false>, dim3(1), dim3(64), 0, st, d_a, d_b, d_d);
    return hipGetLastError();
}

hipError_t launch_model_image(const LensGeom &g, const PropBlock *d_pc, int stage, float *d_img, float *d_tmp,
                              hipStream_t st)
{
    const int npix = g.ny * g.nx;
    const int bs = 256, nb = (npix + bs - 1) / bs;
    float *dst = stage == 0 ? d_img : d_tmp;
    if (mode_epl(g.mode)) hipLaunchKernelGGL((k_model_binned<true>), dim3(nb), dim3(bs), 0, st, g, d_pc, dst);
    else hipLaunchKernelGGL((k_model_binned<false>), dim3(nb), dim3(bs), 0, st, g, d_pc, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || stage == 0) return e;
    hipLaunchKernelGGL(k_model_conv, dim3(nb), dim3(bs), 0, st, g, d_tmp, d_img);
    return hipGetLastError();
}

}  // namespace lensk
