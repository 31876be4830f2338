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
// Two launches: workgroups over fixed chunks of the shots (chunk size set
// by the batch size alone) count with LDS integer atomics (exact) and sum
// the FP64 quantities per bin in a fixed order (each thread a fixed strided
// subset of the chunk's survivors, then a fixed tree); one workgroup then
// adds the chunks' sums in chunk order.  The bins are bit-reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// Per-chunk partial results of the batch reduction: integer counts per bin
// (exact), FP64 sums per bin in a fixed order, the chunk's totals.
struct ChunkTot {
    unsigned long long n2q, sweeps;
    int acc, chi, status, pad;
    double flops;
};

// Chunk c of the shots [c * chunk, (c + 1) * chunk) and of the survivors at
// the same positions: weight counts of all its shots; for its survivors the
// per-bin counts, acceptance and error counts, and per bin (every bin, zero
// when the chunk has none) the sums of P_acc, P_acc * fail, their squares
// and the segment reaches, each a fixed-order workgroup sum.
__global__ __launch_bounds__(RT) void batch_chunk_kernel(int64_t n, int64_t chunk, uint64_t seed,
                                                         uint64_t first,
                                                         const int64_t* __restrict__ off,
                                                         const int64_t* __restrict__ idx,
                                                         const int64_t* __restrict__ n_surv,
                                                         const msc_shot_result* __restrict__ res,
                                                         int nb, const double* __restrict__ surv,
                                                         int n_seg, int32_t* __restrict__ pint,
                                                         double* __restrict__ pdbl,
                                                         ChunkTot* __restrict__ ptot) {
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
    auto weight = [&](int64_t i) {
        const int64_t w = off[i + 1] - off[i];
        return static_cast<int>(w < nb - 1 ? w : nb - 1);
    };
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t i1 = min(n, c0 + chunk);
    for (int64_t i = c0 + tid; i < i1; i += RT) atomicAdd(&s_cnt[weight(i)], 1);
    const int64_t ns = min(*n_surv, n);
    const int64_t s1 = min(ns, c0 + chunk);
    double fl = 0.0;
    for (int64_t s = c0 + tid; s < s1; s += RT) {
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
    const int nd = 4 + n_seg;
    double* pd = pdbl + static_cast<size_t>(blockIdx.x) * nb * nd;
    for (int b = 0; b < nb; ++b) {
        if (s_scnt[b] == 0) {            // block-uniform
            for (int q = tid; q < nd; q += RT) pd[b * nd + q] = 0.0;
            continue;
        }
        for (int g = 0; g < n_seg; ++g) {
            double r = 0.0;
            for (int64_t s = c0 + tid; s < s1; s += RT)
                if (weight(idx[s]) == b) r += surv[s * n_seg + g];
            r = block_sum_fixed(r, s_red);
            if (tid == 0) pd[b * nd + 4 + g] = r;
        }
        double x4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t s = c0 + tid; s < s1; s += RT) {
            if (weight(idx[s]) != b) continue;
            const double x = res[s].p_acc, y = x * res[s].fail;
            x4[0] += x;
            x4[1] += y;
            x4[2] += x * x;
            x4[3] += y * y;
        }
        for (int q = 0; q < 4; ++q) {
            const double v = block_sum_fixed(x4[q], s_red);
            if (tid == 0) pd[b * nd + q] = v;
        }
    }
    __syncthreads();
    int32_t* pi = pint + static_cast<size_t>(blockIdx.x) * nb * 4;
    for (int b = tid; b < nb; b += RT) {
        pi[4 * b] = s_cnt[b];
        pi[4 * b + 1] = s_scnt[b];
        pi[4 * b + 2] = s_kacc[b];
        pi[4 * b + 3] = s_kerr[b];
    }
    if (tid == 0) {
        ChunkTot t;
        t.n2q = s_n2q;
        t.sweeps = s_sweeps;
        t.acc = s_acc;
        t.chi = s_chi;
        t.status = s_status;
        t.pad = 0;
        t.flops = fl;
        ptot[blockIdx.x] = t;
    }
}

// The chunks' partials summed in chunk order (each bin by one thread) into
// the bins, the segment sums and the totals.
__global__ __launch_bounds__(RT) void batch_final_kernel(int nchunk, int nb, int n_seg,
                                                         const int64_t* __restrict__ n_surv,
                                                         int64_t n,
                                                         const int64_t* __restrict__ nnz,
                                                         const int32_t* __restrict__ pint,
                                                         const double* __restrict__ pdbl,
                                                         const ChunkTot* __restrict__ ptot,
                                                         double* __restrict__ bins,
                                                         BatchTotals* __restrict__ tot,
                                                         double* __restrict__ sbins) {
    const int tid = threadIdx.x;
    const int nd = 4 + n_seg;
    for (int b = tid; b < nb; b += RT) {
        int64_t ci[4] = {0, 0, 0, 0};
        double x4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < nchunk; ++c) {
            const int32_t* pi = pint + (static_cast<size_t>(c) * nb + b) * 4;
            const double* pd = pdbl + (static_cast<size_t>(c) * nb + b) * nd;
            for (int q = 0; q < 4; ++q) {
                ci[q] += pi[q];
                x4[q] += pd[q];
            }
        }
        bins[b] = static_cast<double>(ci[0]);
        bins[nb + b] = x4[0];
        bins[2 * nb + b] = x4[1];
        bins[3 * nb + b] = static_cast<double>(ci[2]);
        bins[4 * nb + b] = static_cast<double>(ci[3]);
        bins[5 * nb + b] = x4[2];
        bins[6 * nb + b] = x4[3];
    }
    for (int e = tid; e < nb * n_seg; e += RT) {
        const int b = e / n_seg, g = e - b * n_seg;
        double r = 0.0;
        for (int c = 0; c < nchunk; ++c) r += pdbl[(static_cast<size_t>(c) * nb + b) * nd + 4 + g];
        sbins[e] = r;
    }
    if (tid == 0) {
        unsigned long long n2q = 0, sweeps = 0;
        int64_t acc = 0;
        int chi = 0, status = 0;
        double fl = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            const ChunkTot& t = ptot[c];
            n2q += t.n2q;
            sweeps += t.sweeps;
            acc += t.acc;
            chi = max(chi, t.chi);
            status |= t.status;
            fl += t.flops;
        }
        tot->nnz = *nnz;
        tot->n_survivors = min(*n_surv, n);
        tot->n_accepted = acc;
        tot->n2q = static_cast<int64_t>(n2q);
        tot->sweeps = static_cast<int64_t>(sweeps);
        tot->flops = fl;
        tot->chi_peak = chi;
        tot->status_or = status;
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

// Chunks of at least 4096 shots, at most 256 of them: fixed by n, so the
// summation order (and every bit of the sums) depends on the batch only.
static int64_t reduce_chunk(int64_t n) {
    const int64_t c = (std::max<int64_t>(n, 1) + 255) / 256;
    return std::max<int64_t>(4096, (c + RT - 1) / RT * RT);
}

int64_t batch_reduce_tmp_bytes(int64_t n, int nb, int n_seg) {
    const int64_t nchunk = (std::max<int64_t>(n, 1) + reduce_chunk(n) - 1) / reduce_chunk(n);
    return nchunk * (static_cast<int64_t>(nb) * (4 * sizeof(int32_t) + (4 + n_seg) * sizeof(double)) +
                     static_cast<int64_t>(sizeof(ChunkTot)));
}

hipError_t launch_batch_reduce(int64_t n, uint64_t seed, uint64_t first, const int64_t* off,
                               const int64_t* idx, const int64_t* n_surv,
                               const msc_shot_result* res, int nb, const int64_t* nnz,
                               double* bins, BatchTotals* tot, const double* surv, int n_seg,
                               double* sbins, void* tmp, hipStream_t s) {
    if (nb < 1 || nb > kMaxBins || n_seg < 0 || (n_seg > 0 && (!surv || !sbins)) || !tmp)
        return hipErrorInvalidValue;
    const int64_t chunk = reduce_chunk(n);
    const int64_t nchunk = (std::max<int64_t>(n, 1) + chunk - 1) / chunk;
    ChunkTot* ptot = static_cast<ChunkTot*>(tmp);
    double* pdbl = reinterpret_cast<double*>(ptot + nchunk);
    int32_t* pint = reinterpret_cast<int32_t*>(pdbl + nchunk * nb * (4 + n_seg));
    const int nc = static_cast<int>(nchunk);
    hipLaunchKernelGGL(batch_chunk_kernel, dim3(nc), dim3(RT), 0, s, n, chunk, seed, first, off,
                       idx, n_surv, res, nb, surv, n_seg, pint, pdbl, ptot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_final_kernel, dim3(1), dim3(RT), 0, s, nc, nb, n_seg, n_surv, n, nnz,
                       pint, pdbl, ptot, bins, tot, sbins);
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
