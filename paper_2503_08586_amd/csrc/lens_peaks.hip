// lens_peaks.hip -- issue-rate probes of the instruction kinds the likelihood
// kernels are built from (the vector ALU's FP64/FP32 arithmetic, conversions
// and transcendentals, and the FP16/BF16 matrix-core products), behind
// lens_peak_rate.  They give the roofline's peaks as measured on the device
// rather than taken from unit counts and the nominal clock.
//
// Each lane runs kPeakChains independent chains of one instruction for n
// rounds; chain c's next instruction reads its own previous result, so the
// compiler can neither drop nor hoist the work, and the chains are far enough
// apart that no instruction waits on its predecessor's latency.  The vector
// ops are written as inline asm so that each round is exactly one instruction
// of the named kind (no loads: every operand is a register or an inline
// constant); values stay finite and normal (x <- x/2 + 1/2 has its fixed
// point at 1, FP64 rsq alternates between x and 1/sqrt(x) towards 1, ...).
#include <hip/hip_runtime.h>

#include "lens_api.h"
#include "lens_internal.h"

namespace lensk {

namespace {

constexpr int kPeakChains = 8;
constexpr int kPeakThreads = 256;

typedef float f32x4p __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4p __attribute__((ext_vector_type(4)));

#define LENS_PEAK_ROUND(stmt)                           \
    _Pragma("unroll") for (int c = 0; c < kPeakChains; ++c) { stmt; }

template <int OP>
__global__ void __launch_bounds__(kPeakThreads) k_peak_valu(int n, double seed, double *__restrict__ out)
{
    const int gid = blockIdx.x * kPeakThreads + threadIdx.x;
    double x[kPeakChains];
    float y[kPeakChains], z[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) {
        x[c] = seed + 0.01 * c;
        y[c] = (float)x[c];
        z[c] = y[c];
    }
    // Constants are inline operands (no second register read, so no register
    // bank conflicts between sources).  The FP32 transcendentals are issued
    // independently (each reads its chain's fixed input z and overwrites y).
    for (int r = 0; r < n; ++r) {
        if constexpr (OP == LENS_PEAK_FMA_F64) {
            LENS_PEAK_ROUND(asm volatile("v_fma_f64 %0, %0, 0.5, 0.5" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_FMA_F32) {
            LENS_PEAK_ROUND(asm volatile("v_fma_f32 %0, %0, 0.5, 0.5" : "+v"(y[c])))
        } else if constexpr (OP == LENS_PEAK_MUL_F64) {
            LENS_PEAK_ROUND(asm volatile("v_mul_f64 %0, %0, 1.0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_ADD_F64) {
            LENS_PEAK_ROUND(asm volatile("v_add_f64 %0, %0, 0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_EXP_F32) {
            LENS_PEAK_ROUND(asm volatile("v_exp_f32 %0, %1" : "=v"(y[c]) : "v"(z[c])))
        } else if constexpr (OP == LENS_PEAK_LOG_F32) {
            LENS_PEAK_ROUND(asm volatile("v_log_f32 %0, %1" : "=v"(y[c]) : "v"(z[c])))
        } else if constexpr (OP == LENS_PEAK_RSQ_F32) {
            LENS_PEAK_ROUND(asm volatile("v_rsq_f32 %0, %1" : "=v"(y[c]) : "v"(z[c])))
        } else if constexpr (OP == LENS_PEAK_RCP_F32) {
            LENS_PEAK_ROUND(asm volatile("v_rcp_f32 %0, %1" : "=v"(y[c]) : "v"(z[c])))
        } else if constexpr (OP == LENS_PEAK_CVT_F64_F32) {
            // two conversions per round: FP64 -> FP32 -> FP64
            LENS_PEAK_ROUND(asm volatile("v_cvt_f32_f64 %1, %0\n\tv_cvt_f64_f32 %0, %1" : "+v"(x[c]), "=&v"(y[c])))
        } else if constexpr (OP == LENS_PEAK_LDEXP_F64) {
            LENS_PEAK_ROUND(asm volatile("v_ldexp_f64 %0, %0, 0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_FREXP_MANT_F64) {
            LENS_PEAK_ROUND(asm volatile("v_frexp_mant_f64 %0, %0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_RNDNE_F64) {
            LENS_PEAK_ROUND(asm volatile("v_rndne_f64 %0, %0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_RSQ_F64) {
            LENS_PEAK_ROUND(asm volatile("v_rsq_f64 %0, %0" : "+v"(x[c])))
        } else if constexpr (OP == LENS_PEAK_FMA_F64_EXP_F32) {
            // one FP64 FMA and one FP32 2^x per chain and round: whether the
            // transcendental issues beside the FMAs or takes their slots
            LENS_PEAK_ROUND(asm volatile("v_fma_f64 %0, %0, 0.5, 0.5\n\tv_exp_f32 %1, %2"
                                         : "+v"(x[c]), "=v"(y[c]) : "v"(z[c])))
        }
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) s += x[c] + (double)y[c];
    out[gid] = s;
}

// Matrix-core products: kPeakChains independent accumulators per wave, each
// D = A B + D with A = B = 2^-6 everywhere (exact in FP16 and BF16), so each
// product adds 32 * 2^-12 to every accumulator element.  Written as inline
// asm with the accumulator updated in place: with the builtins the compiler
// rotates the accumulators through other registers every round, which adds
// moves the count would include.  The chains are kPeakChains products apart,
// far beyond the dependent-product latency; the wait before the results are
// read (the compiler does not see the asm as a matrix-core op) is explicit.
// MIX: four independent FP64 FMAs after each FP16 product (the FMAs are what
// is counted): whether the vector ALU keeps issuing while the matrix core
// works on the wave's product.
template <bool F16, bool MIX = false>
__global__ void __launch_bounds__(kPeakThreads) k_peak_mfma(int n, double seed, double *__restrict__ out)
{
    const int gid = blockIdx.x * kPeakThreads + threadIdx.x;
    f32x4p acc[kPeakChains];
    double x[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) {
        acc[c] = f32x4p{(float)seed, 0.f, 0.f, 0.f};
        x[c] = seed + 0.01 * c;
    }
    // 2^-6 in both formats, twice per 32-bit word
    const unsigned int w = F16 ? 0x24002400u : 0x3c803c80u;
    const u32x4p a = {w, w, w, w};
    for (int r = 0; r < n; ++r) {
        if constexpr (MIX) {
            LENS_PEAK_ROUND(asm volatile("v_mfma_f32_16x16x32_f16 %0, %2, %2, %0\n\t"
                                         "v_fma_f64 %1, %1, 0.5, 0.5\n\tv_fma_f64 %1, %1, 0.5, 0.5\n\t"
                                         "v_fma_f64 %1, %1, 0.5, 0.5\n\tv_fma_f64 %1, %1, 0.5, 0.5"
                                         : "+v"(acc[c]), "+v"(x[c]) : "v"(a)))
        } else if constexpr (F16) {
            LENS_PEAK_ROUND(asm volatile("v_mfma_f32_16x16x32_f16 %0, %1, %1, %0" : "+v"(acc[c]) : "v"(a)))
        } else {
            LENS_PEAK_ROUND(asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(acc[c]) : "v"(a)))
        }
    }
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) s += (double)acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3] + x[c];
    out[gid] = s;
}

#undef LENS_PEAK_ROUND

template <int OP>
hipError_t launch_valu(int grid, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_peak_valu<OP>, dim3(grid), dim3(kPeakThreads), 0, st, n, 0.5, out);
    return hipGetLastError();
}

}  // namespace

int peak_threads() { return kPeakThreads; }

double peak_ops_per_round(int op)
{
    // per lane and round, over all chains: lane instructions (vector ops) or,
    // for the matrix-core products, FLOPs per lane (16x16x32 products per wave / 64 lanes)
    if (op == LENS_PEAK_MFMA_F16 || op == LENS_PEAK_MFMA_BF16) return kPeakChains * (2.0 * 16 * 16 * 32 / 64.0);
    if (op == LENS_PEAK_CVT_F64_F32 || op == LENS_PEAK_FMA_F64_EXP_F32) return 2.0 * kPeakChains;
    if (op == LENS_PEAK_MFMA_F16_FMA_F64) return 4.0 * kPeakChains;
    return kPeakChains;
}

hipError_t launch_peak(int op, int grid, int n, double *out, hipStream_t st)
{
    switch (op) {
    case LENS_PEAK_FMA_F64: return launch_valu<LENS_PEAK_FMA_F64>(grid, n, out, st);
    case LENS_PEAK_FMA_F32: return launch_valu<LENS_PEAK_FMA_F32>(grid, n, out, st);
    case LENS_PEAK_MUL_F64: return launch_valu<LENS_PEAK_MUL_F64>(grid, n, out, st);
    case LENS_PEAK_ADD_F64: return launch_valu<LENS_PEAK_ADD_F64>(grid, n, out, st);
    case LENS_PEAK_EXP_F32: return launch_valu<LENS_PEAK_EXP_F32>(grid, n, out, st);
    case LENS_PEAK_LOG_F32: return launch_valu<LENS_PEAK_LOG_F32>(grid, n, out, st);
    case LENS_PEAK_RSQ_F32: return launch_valu<LENS_PEAK_RSQ_F32>(grid, n, out, st);
    case LENS_PEAK_RCP_F32: return launch_valu<LENS_PEAK_RCP_F32>(grid, n, out, st);
    case LENS_PEAK_CVT_F64_F32: return launch_valu<LENS_PEAK_CVT_F64_F32>(grid, n, out, st);
    case LENS_PEAK_LDEXP_F64: return launch_valu<LENS_PEAK_LDEXP_F64>(grid, n, out, st);
    case LENS_PEAK_FREXP_MANT_F64: return launch_valu<LENS_PEAK_FREXP_MANT_F64>(grid, n, out, st);
    case LENS_PEAK_RNDNE_F64: return launch_valu<LENS_PEAK_RNDNE_F64>(grid, n, out, st);
    case LENS_PEAK_RSQ_F64: return launch_valu<LENS_PEAK_RSQ_F64>(grid, n, out, st);
    case LENS_PEAK_FMA_F64_EXP_F32: return launch_valu<LENS_PEAK_FMA_F64_EXP_F32>(grid, n, out, st);
    case LENS_PEAK_MFMA_F16_FMA_F64:
        hipLaunchKernelGGL((k_peak_mfma<true, true>), dim3(grid), dim3(kPeakThreads), 0, st, n, 0.0, out);
        return hipGetLastError();
    case LENS_PEAK_MFMA_F16:
        hipLaunchKernelGGL(k_peak_mfma<true>, dim3(grid), dim3(kPeakThreads), 0, st, n, 0.0, out);
        return hipGetLastError();
    case LENS_PEAK_MFMA_BF16:
        hipLaunchKernelGGL(k_peak_mfma<false>, dim3(grid), dim3(kPeakThreads), 0, st, n, 0.0, out);
        return hipGetLastError();
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lensk
