// lens_kernels.hip -- HIP kernels of the batched lens log-likelihood (gfx950).
//
// k_prep          one thread per proposal: domain check, FP64 b_n, derived FP32 constants.
// k_loglike_fp32  one workgroup per proposal: the whole forward model and the
//                 chi-square in one pass, the binned image never leaving LDS.
// k_model_*       debug: full model images of one proposal.
//
// Forward model: Cao et al. (2025), Sec. 2.1 (Eqs. 1-3), Sec. 2.2 (Eq. 5), Sec. 2.4.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lens_device.h"
#include "lens_internal.h"

namespace lensk {

// ---------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------
__device__ LightK light_constants(double I, double R, double n, double q, double phi)
{
    // x1 = c dx + s dy, x2 = -s dx + c dy, (R_p/R_e)^2 = (q x1^2 + x2^2/q) / R_e^2
    const double c = cos(phi), s = sin(phi), A = q / (R * R), Bq = 1.0 / (q * R * R);
    LightK L;
    L.P = A * c * c + Bq * s * s;
    L.Q = A * s * s + Bq * c * c;
    L.S = 2.0 * (A - Bq) * c * s;
    L.e = 0.5 / n;
    L.B = bn_device(n) * 1.4426950408889634;
    L.I = I;
    return L;
}

__global__ void __launch_bounds__(256) k_prep(const double *__restrict__ params, int64_t n,
                                              PropBlock *__restrict__ pc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *p = params + i * kStride;
    PropBlock b{};
    double v[19];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 19; ++j) {
        v[j] = p[j];
        ok = ok && isfinite(v[j]);
    }
    ok = ok && v[0] >= 0.0;
    ok = ok && v[1] > 0.0 && v[1] <= 1.0 && v[10] > 0.0 && v[10] <= 1.0 && v[15] > 0.0 && v[15] <= 1.0;
    ok = ok && v[8] > 0.0 && v[13] > 0.0;
    ok = ok && v[9] >= kNMin && v[9] <= kNMax && v[14] >= kNMin && v[14] <= kNMax;
    if (ok) {
        const double q = v[1];
        b.valid = 1.0;
        b.xm = v[3];
        b.ym = v[4];
        b.cm = cos(v[2]);
        b.sm = sin(v[2]);
        b.q2m = q * q;
        b.ce = sqrt((1.0 - q) * (1.0 + q));
        b.bsie = v[0] * sqrt(q);
        b.bsc = b.ce > 0.0 ? b.bsie / b.ce : 0.0;
        b.g1 = v[5];
        b.g2 = v[6];
        b.xs = v[17];
        b.ys = v[18];
        b.lens = light_constants(v[7], v[8], v[9], v[10], v[11]);
        b.src = light_constants(v[12], v[13], v[14], v[15], v[16]);
    }
    pc[i] = b;
}

// ---------------------------------------------------------------------------
// fused FP32 likelihood
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Binned rows [ya, yb) (all < ny) into their ring slots: every pixel in the
// row's needed range is evaluated; the rest of the row is cleared when the
// slot is being reused (clear = true).
__device__ __forceinline__ void fill_rows(const LensGeom &g, const PropBlock &P, float *ring,
                                          const uint32_t *__restrict__ evl, const int *__restrict__ evpre,
                                          const int2 *__restrict__ evr, int ya, int yb, bool clear)
{
    const int W = g.ring_w, RB = g.ring_rows, r = g.r, nx = g.nx;
    const int slot_a = (ya + r) % RB;  // rows [ya, yb) occupy consecutive slots modulo RB
    if (clear) {
        for (int y = ya; y < yb; ++y) {
            int slot = slot_a + (y - ya);
            if (slot >= RB) slot -= RB;
            const int2 lr = evr[y];
            for (int x = threadIdx.x; x < nx; x += blockDim.x)
                if (x < lr.x || x >= lr.y) ring[slot * W + r + x] = 0.0f;
        }
    }
    const int fb = evpre[yb];
    for (int f = evpre[ya] + threadIdx.x; f < fb; f += blockDim.x) {
        const uint32_t e = evl[f];
        const int y = (int)(e >> 16), x = (int)(e & 0xffffu);
        int slot = slot_a + (y - ya);
        if (slot >= RB) slot -= RB;
        ring[slot * W + r + x] = binned_pixel(g, P, y, x);
    }
}

// chi-square contribution of output rows [ya, yb): four horizontally adjacent
// outputs per thread, the window of each PSF row held in registers, PSF
// weights read through the scalar cache.  Row partial sums are accumulated
// separately (blocked summation).
template <int K>
__device__ __forceinline__ double conv_rows(const LensGeom &g, const float *ring, const float *__restrict__ psf,
                                            const uint32_t *__restrict__ cvl, const int *__restrict__ cvpre,
                                            const float *__restrict__ data, const float *__restrict__ wgt,
                                            int ya, int yb)
{
    constexpr int KC = (K + 6) / 4;
    const int W = g.ring_w, RB = g.ring_rows;
    double acc = 0.0;
    const int gb = cvpre[yb];
    for (int gi = cvpre[ya] + threadIdx.x; gi < gb; gi += blockDim.x) {
        const uint32_t e = cvl[gi];
        const int y = (int)(e >> 16), x0 = (int)(e & 0xffffu);
        float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f;
        int slot = y % RB;  // ring slot of binned row y - r
#pragma unroll 1
        for (int a = 0; a < K; ++a) {
            const float4 *rowp = reinterpret_cast<const float4 *>(ring + slot * W + x0);
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
            o0 += p0;
            o1 += p1;
            o2 += p2;
            o3 += p3;
            slot = (slot + 1 == RB) ? 0 : slot + 1;
        }
        const float4 d = *reinterpret_cast<const float4 *>(data + (size_t)y * g.pitch + x0);
        const float4 w = *reinterpret_cast<const float4 *>(wgt + (size_t)y * g.pitch + x0);
        const double r0 = (double)((d.x - o0) * w.x);
        const double r1 = (double)((d.y - o1) * w.y);
        const double r2 = (double)((d.z - o2) * w.z);
        const double r3 = (double)((d.w - o3) * w.w);
        acc = fma(r0, r0, acc);
        acc = fma(r1, r1, acc);
        acc = fma(r2, r2, acc);
        acc = fma(r3, r3, acc);
    }
    return acc;
}

template <int K>
__global__ void __launch_bounds__(kBlock)
k_loglike_fp32(const LensGeom g, const PropBlock *__restrict__ pc, const float *__restrict__ psf,
               const uint32_t *__restrict__ evl, const int *__restrict__ evpre, const int2 *__restrict__ evr,
               const uint32_t *__restrict__ cvl, const int *__restrict__ cvpre,
               const float *__restrict__ data, const float *__restrict__ wgt, double *__restrict__ out)
{
    extern __shared__ float4 lds4[];
    float *ring = reinterpret_cast<float *>(lds4);
    __shared__ double red[kBlock / 64];
    const int64_t p = blockIdx.x;
    const PropBlock *c = pc + p;
    if (c->valid == 0.0) {
        if (threadIdx.x == 0) out[p] = -INFINITY;
        return;
    }
    const PropBlock P = *c;
    const int ny = g.ny, r = g.r, H = g.strip_h;
    const int n4 = g.ring_rows * g.ring_w / 4;
    for (int i = threadIdx.x; i < n4; i += blockDim.x) lds4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // binned rows [0, r) precede the first strip
    fill_rows(g, P, ring, evl, evpre, evr, 0, min(r, ny), false);
    double acc = 0.0;
    for (int y0 = 0; y0 < ny; y0 += H) {
        __syncthreads();  // the previous strip is done reading the slots reused below
        // new binned rows [y0 + r, y0 + H + r); rows past the image stay zero
        const int ya = y0 + r, yb = y0 + H + r;
        if (y0 > 0) {
            // rows beyond the image: clear their reused slots
            for (int y = max(ya, ny); y < yb; ++y) {
                const int slot = (y + r) % g.ring_rows;
                for (int x = threadIdx.x; x < g.nx; x += blockDim.x) ring[slot * g.ring_w + r + x] = 0.0f;
            }
        }
        if (ya < ny) fill_rows(g, P, ring, evl, evpre, evr, ya, min(yb, ny), y0 > 0);
        __syncthreads();
        acc += conv_rows<K>(g, ring, psf, cvl, cvpre, data, wgt, y0, min(y0 + H, ny));
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w];
        out[p] = g.norm - 0.5 * s;
    }
}

// ---------------------------------------------------------------------------
// debug model images
// ---------------------------------------------------------------------------
__global__ void k_model_binned(const LensGeom g, const PropBlock *__restrict__ pc, float *__restrict__ img)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.ny * g.nx) return;
    const PropBlock P = *pc;
    img[i] = binned_pixel(g, P, i / g.nx, i % g.nx);
}

__global__ void k_model_conv(const LensGeom g, const float *__restrict__ img, float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.ny * g.nx) return;
    const int y = i / g.nx, x = i % g.nx, k = g.k, r = g.r;
    float o = 0.0f;
    for (int a = 0; a < k; ++a) {
        const int yy = y - r + a;
        float pr = 0.0f;
        for (int b = 0; b < k; ++b) {
            const int xx = x - r + b;
            const float v = (yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx) ? img[yy * g.nx + xx] : 0.0f;
            pr = fmaf(g.psf[a * k + b], v, pr);
        }
        o += pr;
    }
    out[i] = o;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int choose_kc(int k) { return (k + 6) / 4; }

size_t ring_bytes(const LensGeom &g) { return (size_t)g.ring_rows * g.ring_w * sizeof(float); }

hipError_t launch_prep(const double *d_params, int64_t n, PropBlock *d_pc, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t nb = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)nb), dim3(bs), 0, st, d_params, n, d_pc);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_k(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_loglike_fp32<K>, dim3((unsigned)n), dim3(kBlock), ring_bytes(g), st, g, d_pc,
                       g.psf, g.evl, g.evpre, g.evr, g.cvl, g.cvpre, g.data, g.wgt, d_out);
    return hipGetLastError();
}

hipError_t launch_loglike_fp32(const LensGeom &g, const PropBlock *d_pc, int64_t n, double *d_out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    switch (g.k) {
#define LENS_K(KK) \
    case KK: return launch_k<KK>(g, d_pc, n, d_out, st);
        LENS_K(1) LENS_K(3) LENS_K(5) LENS_K(7) LENS_K(9) LENS_K(11) LENS_K(13) LENS_K(15)
        LENS_K(17) LENS_K(19) LENS_K(21) LENS_K(23) LENS_K(25) LENS_K(27) LENS_K(29) LENS_K(31)
        LENS_K(33) LENS_K(35) LENS_K(37) LENS_K(39) LENS_K(41) LENS_K(43) LENS_K(45) LENS_K(47)
        LENS_K(49) LENS_K(51) LENS_K(53) LENS_K(55) LENS_K(57) LENS_K(59) LENS_K(61) LENS_K(63)
#undef LENS_K
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_model_image(const LensGeom &g, const PropBlock *d_pc, int stage, float *d_img, float *d_tmp,
                              hipStream_t st)
{
    const int npix = g.ny * g.nx;
    const int bs = 256, nb = (npix + bs - 1) / bs;
    if (stage == 0) {
        hipLaunchKernelGGL(k_model_binned, dim3(nb), dim3(bs), 0, st, g, d_pc, d_img);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_model_binned, dim3(nb), dim3(bs), 0, st, g, d_pc, d_tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_model_conv, dim3(nb), dim3(bs), 0, st, g, d_tmp, d_img);
    return hipGetLastError();
}

}  // namespace lensk
