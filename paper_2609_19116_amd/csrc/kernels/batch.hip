// End of a batch: per-weight bins and batch statistics (Section 4.1,
// Eq. (reweight)), written straight into host-mapped memory so that the
// host reads them after one stream synchronisation, without a copy.
//
// Besides the sums of P_acc and P_acc * fail (and of their squares, for the
// standard errors), each bin gets the counts that
// the likelihood of the error analysis works with (Appendix "Error analysis
// of the subset-sampling estimator", Eq. (loglik-split)): a shot counts as
// accepted iff u < P_acc for one uniform u of its own, and as wrong iff it
// is accepted and its accepted branch fails.  u is the first output of the
// SplitMix64 stream (Steele, Lea, Flood 2014) keyed as the fault draws but
// with the seed XOR'ed by a fixed constant (the first 64 fraction bits of
// pi), converted as (x >> 11) 2^-53; screened shots have P_acc = 0.
//
// One 256-thread workgroup.  Counts use LDS integer atomics (exact); the
// FP64 sums are reduced in a fixed order (per bin, each thread walks a
// fixed strided subset of the survivors, then a fixed tree), so the bins
// are bit-reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

constexpr int RT = 256;
constexpr uint64_t kAcceptKey = 0x243F6A8885A308D3ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double acceptance_uniform(uint64_t seed, uint64_t shot) {
    const uint64_t st = mix64((seed ^ kAcceptKey) ^ mix64(shot)) + 0x9E3779B97F4A7C15ull;
    return static_cast<double>(mix64(st) >> 11) * (1.0 / 9007199254740992.0);
}

__device__ double block_sum_fixed(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < RT / 64; ++j) s += red[j];
    return s;
}

__global__ __launch_bounds__(RT) void batch_reduce_kernel(int64_t n, uint64_t seed, uint64_t first,
                                                          const int64_t* __restrict__ off,
                                                          const int64_t* __restrict__ idx,
                                                          const int64_t* __restrict__ n_surv,
                                                          const msc_shot_result* __restrict__ res,
                                                          int nb, const int64_t* __restrict__ nnz,
                                                          double* __restrict__ bins,
                                                          BatchTotals* __restrict__ tot,
                                                          const double* __restrict__ surv,
                                                          int n_seg, double* __restrict__ sbins) {
    __shared__ int s_cnt[kMaxBins];
    __shared__ int s_scnt[kMaxBins];
    __shared__ int s_kacc[kMaxBins];
    __shared__ int s_kerr[kMaxBins];
    __shared__ double s_red[RT / 64];
    __shared__ unsigned long long s_n2q, s_sweeps;
    __shared__ int s_acc, s_chi, s_status;
    const int tid = threadIdx.x;
    for (int b = tid; b < nb; b += RT) {
        s_cnt[b] = 0;
        s_scnt[b] = 0;
        s_kacc[b] = 0;
        s_kerr[b] = 0;
    }
    if (tid == 0) {
        s_n2q = 0;
        s_sweeps = 0;
        s_acc = 0;
        s_chi = 0;
        s_status = 0;
    }
    __syncthreads();
    auto weight = [&](int64_t s) {
        const int64_t w = off[s + 1] - off[s];
        return static_cast<int>(w < nb - 1 ? w : nb - 1);
    };
    for (int64_t i = tid; i < n; i += RT) atomicAdd(&s_cnt[weight(i)], 1);
    const int64_t ns = *n_surv;
    double fl = 0.0;
    for (int64_t s = tid; s < ns; s += RT) {
        const int64_t i = idx[s];
        const int wb = weight(i);
        atomicAdd(&s_scnt[wb], 1);
        const msc_shot_result& r = res[s];
        if (acceptance_uniform(seed, first + static_cast<uint64_t>(i)) < r.p_acc) {
            atomicAdd(&s_kacc[wb], 1);
            if (r.fail) atomicAdd(&s_kerr[wb], 1);
        }
        atomicAdd(&s_n2q, static_cast<unsigned long long>(r.n2q));
        atomicAdd(&s_sweeps, static_cast<unsigned long long>(r.sweeps));
        if (r.p_acc > 0.0) atomicAdd(&s_acc, 1);
        atomicMax(&s_chi, r.chi_peak);
        atomicOr(&s_status, r.status);
        fl += r.flops;
    }
    fl = block_sum_fixed(fl, s_red);
    for (int b = 0; b < nb; ++b) {
        if (s_scnt[b] == 0) {            // block-uniform
            if (tid == 0) {
                bins[nb + b] = 0.0;
                bins[2 * nb + b] = 0.0;
                bins[5 * nb + b] = 0.0;
                bins[6 * nb + b] = 0.0;
                for (int g = 0; g < n_seg; ++g) sbins[b * n_seg + g] = 0.0;
            }
            continue;
        }
        // reach probabilities of the segments (space-time mode)
        for (int g = 0; g < n_seg; ++g) {
            double r = 0.0;
            for (int64_t s = tid; s < ns; s += RT)
                if (weight(idx[s]) == b) r += surv[s * n_seg + g];
            r = block_sum_fixed(r, s_red);
            if (tid == 0) sbins[b * n_seg + g] = r;
        }
        double a = 0.0, e = 0.0, a2 = 0.0, e2 = 0.0;
        for (int64_t s = tid; s < ns; s += RT) {
            if (weight(idx[s]) != b) continue;
            const double x = res[s].p_acc, y = x * res[s].fail;
            a += x;
            e += y;
            a2 += x * x;
            e2 += y * y;
        }
        a = block_sum_fixed(a, s_red);
        e = block_sum_fixed(e, s_red);
        a2 = block_sum_fixed(a2, s_red);
        e2 = block_sum_fixed(e2, s_red);
        if (tid == 0) {
            bins[nb + b] = a;
            bins[2 * nb + b] = e;
            bins[5 * nb + b] = a2;
            bins[6 * nb + b] = e2;
        }
    }
    __syncthreads();
    for (int b = tid; b < nb; b += RT) {
        bins[b] = s_cnt[b];
        bins[3 * nb + b] = s_kacc[b];
        bins[4 * nb + b] = s_kerr[b];
    }
    if (tid == 0) {
        tot->nnz = *nnz;
        tot->n_survivors = ns;
        tot->n_accepted = s_acc;
        tot->n2q = static_cast<int64_t>(s_n2q);
        tot->sweeps = static_cast<int64_t>(s_sweeps);
        tot->flops = fl;
        tot->chi_peak = s_chi;
        tot->status_or = s_status;
    }
}

__global__ __launch_bounds__(RT) void identity_kernel(int64_t n, int64_t* idx, int64_t* count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
    if (i < n) idx[i] = i;
    if (i == 0) *count = n;
}

// zero records (rejected_at -1) for every shot of a shot-indexed output
__global__ __launch_bounds__(RT) void fill_results_kernel(int64_t n, msc_shot_result* out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
    if (i >= n) return;
    msc_shot_result z{};
    z.rejected_at = -1;
    out[i] = z;
}

// survivor-indexed results to shot-indexed ones
__global__ __launch_bounds__(RT) void scatter_results_kernel(int64_t n, const int64_t* n_surv,
                                                             const int64_t* idx,
                                                             const msc_shot_result* res,
                                                             msc_shot_result* out) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * RT + threadIdx.x;
    if (s >= *n_surv || s >= n) return;
    const int64_t i = idx[s];
    if (i >= 0 && i < n) out[i] = res[s];
}

}  // namespace

hipError_t launch_batch_reduce(int64_t n, uint64_t seed, uint64_t first, const int64_t* off,
                               const int64_t* idx, const int64_t* n_surv,
                               const msc_shot_result* res, int nb, const int64_t* nnz,
                               double* bins, BatchTotals* tot, const double* surv, int n_seg,
                               double* sbins, hipStream_t s) {
    if (nb < 1 || nb > kMaxBins || n_seg < 0 || (n_seg > 0 && (!surv || !sbins)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(1), dim3(RT), 0, s, n, seed, first, off, idx,
                       n_surv, res, nb, nnz, bins, tot, surv, n_seg, sbins);
    return hipGetLastError();
}

hipError_t launch_identity(int64_t n, int64_t* idx, int64_t* count, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(n > 0 ? (n + RT - 1) / RT : 1));
    hipLaunchKernelGGL(identity_kernel, grid, dim3(RT), 0, s, n, idx, count);
    return hipGetLastError();
}

hipError_t launch_scatter_results(int64_t n, const int64_t* n_surv, const int64_t* idx,
                                  const msc_shot_result* res, msc_shot_result* out,
                                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + RT - 1) / RT));
    hipLaunchKernelGGL(fill_results_kernel, grid, dim3(RT), 0, s, n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scatter_results_kernel, grid, dim3(RT), 0, s, n, n_surv, idx, res, out);
    return hipGetLastError();
}

}  // namespace msc
