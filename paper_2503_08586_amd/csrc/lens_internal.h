// lens_internal.h -- structures shared by the host runtime and the HIP kernels.
// Private to the library; the public interface is include/lens_api.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lensk {

constexpr int kStride = 20;   // doubles per proposal vector
constexpr int kPC = 32;       // floats of derived per-proposal constants
constexpr int kBlock = 256;   // threads per workgroup of the likelihood kernels
constexpr int kMaxK = 63;     // largest PSF side
constexpr float kNMin = 0.1f, kNMax = 20.0f;

// Layout of the derived per-proposal constants (written by the prep kernel).
enum : int {
    PC_VALID = 0,
    // SIE + shear
    PC_XM, PC_YM, PC_CM, PC_SM, PC_Q2M, PC_CE, PC_BSIE, PC_G1, PC_G2,
    // lens light: amplitude, rotation, q/R^2, 1/(q R^2), 1/(2n), b_n log2(e) as hi + lo
    PC_IL, PC_CL, PC_SL, PC_AL, PC_BL, PC_EL, PC_BLH, PC_BLL,
    // source light: the same plus its centre
    PC_IS, PC_XS, PC_YS, PC_CS, PC_SS, PC_AS, PC_BS, PC_ES, PC_BSH, PC_BSL,
    PC_COUNT
};
static_assert(PC_COUNT <= kPC, "per-proposal constant block too small");

// Everything a likelihood launch needs to know about one resident lens.
struct LensGeom {
    int ny, nx, s, k, r;   // rows, columns, supersampling, PSF side, (k-1)/2
    int pitch;             // row pitch (floats) of data and weight, multiple of 4
    int strip_h;           // output rows per strip
    int ring_rows;         // strip_h + 2r binned rows kept in LDS
    int ring_w;            // floats per LDS row
    int kc;                // float4 chunks of the conv window (4*kc >= k + 3)
    float sd;              // pixel_scale / s: sub-pixel pitch
    float cfx, cfy;        // (nx*s - 1)/2, (ny*s - 1)/2: fine-grid centre
    float inv_s2;          // 1/s^2
    double norm;           // C = -1/2 sum_mask ln(2 pi sigma^2)
    const float *psf;      // flipped kernel Kf[a][b] = K[k-1-a][k-1-b], [k][k]
    const float *data;     // [ny][pitch], 0 outside the mask and the image
    const float *wgt;      // [ny][pitch], mask/sigma, 0 outside the mask and the image
    const uint32_t *evl;   // pixels whose binned value is needed, (y << 16) | x, row-major
    const int *evpre;      // [ny + 1] prefix of evl by row
    const int2 *evr;       // [ny] needed column range [lo, hi) of each row
    const uint32_t *cvl;   // groups of 4 output pixels covering the mask, (y << 16) | x0
    const int *cvpre;      // [ny + 1] prefix of cvl by row
};

size_t ring_bytes(const LensGeom &g);
int choose_kc(int k);

hipError_t launch_prep(const double *d_params, int64_t n, float *d_pc, hipStream_t st);
hipError_t launch_loglike_fp32(const LensGeom &g, const float *d_pc, int64_t n, double *d_out,
                               hipStream_t st);
// stage 0: binned image of one proposal into d_img [ny][nx]; stage 1: convolved,
// using d_tmp [ny][nx] for the binned image.
hipError_t launch_model_image(const LensGeom &g, const float *d_pc, int stage, float *d_img,
                              float *d_tmp, hipStream_t st);

}  // namespace lensk
