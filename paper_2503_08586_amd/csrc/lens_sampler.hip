// lens_sampler.hip -- the sampler loop on the device (gfx950).
//
// An ensemble of W walkers moves by the stretch move of Goodman & Weare
// (2010, CAMCoS 5, 65, Sec. 3) in its parallel form: the two halves of the
// ensemble update in turn, each walker of the moving half against a partner
// drawn from the other half.  Proposals are made, prepared, evaluated and
// accepted on the device, so no parameter vector crosses PCIe inside the loop
// (the transfer overhead Cao et al. 2025 note in Sec. 3.1.4, on the way to
// the device-side sampling of their Sec. 4.2).  The target is the posterior
// of Sec. 2.2 under a uniform box prior.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, Sec. 3),
// one counter per (walker, iteration), so a run is reproducible and can be
// split into any number of calls.
//
// k_philox_words      Philox words of consecutive counters (for callers and tests).
// k_stretch_propose   one thread per walker of the moving half: partner, stretch
//                     factor, acceptance draw, proposal, box check and the
//                     proposal's derived constants (the prep step, fused).
// k_stretch_accept    one thread per walker of the moving half: the acceptance
//                     rule, the walker update, the chain row.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lens_internal.h"
#include "lens_prep.h"

namespace lensk {

// Philox4x32-10: ten rounds of the Philox S-box on four 32-bit words, the
// key advancing by the Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;   // round multipliers
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;   // key increments
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k.x += kW0;
            k.y += kW1;
        }
        const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
        const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

__global__ void __launch_bounds__(256) k_philox_words(uint4 base, uint2 key, int64_t n, uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 r = philox4x32_10(make_uint4(base.x + (uint32_t)i, base.y, base.z, base.w), key);
    reinterpret_cast<uint4 *>(out)[i] = r;
}

// Walker k (of W; half h = k / (W/2)) in iteration t draws the words of
// counter (k, t mod 2^32, t div 2^32, 0) under key (seed mod 2^32, seed div
// 2^32): word 0 picks the partner j in the other half, word 1 the stretch
// factor z = ((a - 1) u1 + 1)^2 / a (density ~ 1/sqrt(z) on [1/a, a]), word 2
// the acceptance draw u2; u = (word + 1/2) 2^-32.  The proposal is
// Y = X_j + z (X_k - X_j).  aux = (z, ln u2, inside the box ? 1 : 0, -).
// A proposal outside the box is not evaluated: its prepared constants are
// marked outside the domain, so the likelihood kernel returns -inf at once.
__device__ __forceinline__ void stretch_propose_one(int W, int half, int i, uint64_t t, uint64_t seed, double a,
                                                    int model_code, const double *__restrict__ walkers,
                                                    const double *__restrict__ lo, const double *__restrict__ hi,
                                                    double *__restrict__ Y, double4 *__restrict__ aux,
                                                    PropBlock *__restrict__ pc)
{
    const int h = W / 2;
    const int k = half * h + i;
    const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)t, (uint32_t)(t >> 32), 0u),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const int j = (1 - half) * h + (int)(((uint64_t)r.x * (uint64_t)h) >> 32);
    const double u1 = ((double)r.y + 0.5) * 0x1p-32, u2 = ((double)r.z + 0.5) * 0x1p-32;
    const double w = (a - 1.0) * u1 + 1.0;
    const double z = w * w / a;
    const double *xk = walkers + (size_t)k * kStride, *xj = walkers + (size_t)j * kStride;
    double v[kStride];
    bool inside = true;
#pragma unroll
    for (int s = 0; s < kStride; ++s) {
        v[s] = xj[s] + z * (xk[s] - xj[s]);
        inside = inside && v[s] >= lo[s] && v[s] <= hi[s];
        Y[s] = v[s];
    }
    *aux = make_double4(z, log(u2), inside ? 1.0 : 0.0, 0.0);
    *pc = inside ? prep_proposal(v, model_code) : PropBlock{};
}

// Walker k takes its proposal when ln u2 < (d - 1) ln z + lnP(Y) - lnP(X_k),
// lnP(Y) = lnL(Y) inside the box and -inf outside; d = free slots.  With
// chain_w non-null the walker's state after the move (taken or not) is
// written to chain_w[k], its lnP to chain_lnp[k].
__device__ __forceinline__ void stretch_accept_one(int W, int half, int i, int d, double *__restrict__ walkers,
                                                   double *__restrict__ lnp, const double *__restrict__ Y,
                                                   double4 x, double lnl, int64_t *__restrict__ accepted,
                                                   double *__restrict__ chain_w, double *__restrict__ chain_lnp)
{
    const int k = half * (W / 2) + i;
    const double lnpY = x.z != 0.0 ? lnl : -INFINITY;
    const double rhs = (double)(d - 1) * log(x.x) + lnpY - lnp[k];
    double *wk = walkers + (size_t)k * kStride;
    if (lnpY > -INFINITY && x.y < rhs) {
#pragma unroll
        for (int s = 0; s < kStride; ++s) wk[s] = Y[s];
        lnp[k] = lnpY;
        accepted[k] += 1;
    }
    if (chain_w) {
#pragma unroll
        for (int s = 0; s < kStride; ++s) chain_w[(size_t)k * kStride + s] = wk[s];
        chain_lnp[k] = lnp[k];
    }
}

__global__ void __launch_bounds__(64)
k_stretch_propose(int W, int half, uint64_t t, uint64_t seed, double a, int model_code,
                  const double *__restrict__ walkers, const double *__restrict__ lo,
                  const double *__restrict__ hi, double *__restrict__ Y, double4 *__restrict__ aux,
                  PropBlock *__restrict__ pc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W / 2) return;
    stretch_propose_one(W, half, i, t, seed, a, model_code, walkers, lo, hi, Y + (size_t)i * kStride, aux + i, pc + i);
}

__global__ void __launch_bounds__(256)
k_stretch_accept(int W, int half, int d, double *__restrict__ walkers, double *__restrict__ lnp,
                 const double *__restrict__ Y, const double4 *__restrict__ aux, const double *__restrict__ lnl,
                 int64_t *__restrict__ accepted, double *__restrict__ chain_w, double *__restrict__ chain_lnp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W / 2) return;
    stretch_accept_one(W, half, i, d, walkers, lnp, Y + (size_t)i * kStride, aux[i], lnl[i], accepted, chain_w,
                       chain_lnp);
}

// Many ensembles in one launch: the moving halves of all of them, walker i of
// the pooled half belonging to ensemble e with hoff[e] <= i < hoff[e + 1]
// (hoff: prefix of W/2 over the ensembles).  Each walker runs exactly the
// single-ensemble arithmetic, at its ensemble's own iteration t0 + it.
__device__ __forceinline__ int ensemble_of(const int64_t *__restrict__ hoff, int n, int64_t i)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (hoff[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(64)
k_stretch_propose_many(const EnsembleDev *__restrict__ ens, const int64_t *__restrict__ hoff, int n, int half,
                       int64_t it, double *__restrict__ Y, double4 *__restrict__ aux, PropBlock *__restrict__ pc)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= hoff[n]) return;
    const EnsembleDev &E = ens[ensemble_of(hoff, n, g)];
    const int i = (int)(g - E.off);
    stretch_propose_one(E.W, half, i, (uint64_t)(E.t0 + it), E.seed, E.a, E.code, E.walkers, E.lo, E.hi,
                        Y + (size_t)g * kStride, aux + g, pc + g);
}

__global__ void __launch_bounds__(256)
k_stretch_accept_many(const EnsembleDev *__restrict__ ens, const int64_t *__restrict__ hoff, int n, int half,
                      const double *__restrict__ Y, const double4 *__restrict__ aux, const double *__restrict__ lnl,
                      int64_t slot)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= hoff[n]) return;
    const EnsembleDev &E = ens[ensemble_of(hoff, n, g)];
    const int i = (int)(g - E.off);
    const bool keep = slot >= 0 && E.chain_w;
    stretch_accept_one(E.W, half, i, E.d, E.walkers, E.lnp, Y + (size_t)g * kStride, aux[g], lnl[g], E.accepted,
                       keep ? E.chain_w + (size_t)slot * E.W * kStride : nullptr,
                       keep ? E.chain_lnp + (size_t)slot * E.W : nullptr);
}

hipError_t launch_philox_words(const uint32_t ctr[4], const uint32_t key[2], int64_t n, uint32_t *d_out,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st,
                       make_uint4(ctr[0], ctr[1], ctr[2], ctr[3]), make_uint2(key[0], key[1]), n, d_out);
    return hipGetLastError();
}

hipError_t launch_stretch_propose(int W, int half, uint64_t t, uint64_t seed, double a, int model_code,
                                  const double *d_walkers, const double *d_lo, const double *d_hi, double *d_Y,
                                  double *d_aux, PropBlock *d_pc, hipStream_t st)
{
    // one wave per workgroup: the prep step is latency-bound (two b_n roots per
    // walker), so the half's walkers are spread over as many CUs as possible
    const int h = W / 2, bs = 64;
    hipLaunchKernelGGL(k_stretch_propose, dim3((unsigned)((h + bs - 1) / bs)), dim3(bs), 0, st, W, half, t, seed,
                       a, model_code, d_walkers, d_lo, d_hi, d_Y, reinterpret_cast<double4 *>(d_aux), d_pc);
    return hipGetLastError();
}

hipError_t launch_stretch_many(int half, int64_t it, const EnsembleDev *d_ens, const int64_t *d_hoff, int n,
                               int64_t total, double *d_Y, double *d_aux, PropBlock *d_pc, int stage, const double *d_lnl,
                               int64_t slot, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    if (stage == 0) {
        const int bs = 64;
        hipLaunchKernelGGL(k_stretch_propose_many, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, d_ens,
                           d_hoff, n, half, it, d_Y, reinterpret_cast<double4 *>(d_aux), d_pc);
    } else {
        const int bs = 256;
        hipLaunchKernelGGL(k_stretch_accept_many, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, d_ens,
                           d_hoff, n, half, d_Y, reinterpret_cast<const double4 *>(d_aux), d_lnl, slot);
    }
    return hipGetLastError();
}

hipError_t launch_stretch_accept(int W, int half, int d, double *d_walkers, double *d_lnp, const double *d_Y,
                                 const double *d_aux, const double *d_lnl, int64_t *d_accepted, double *d_chain_w,
                                 double *d_chain_lnp, hipStream_t st)
{
    const int h = W / 2, bs = 256;
    hipLaunchKernelGGL(k_stretch_accept, dim3((unsigned)((h + bs - 1) / bs)), dim3(bs), 0, st, W, half, d, d_walkers,
                       d_lnp, d_Y, reinterpret_cast<const double4 *>(d_aux), d_lnl, d_accepted, d_chain_w,
                       d_chain_lnp);
    return hipGetLastError();
}

}  // namespace lensk
