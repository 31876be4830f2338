// Subset-sampling fault draws on the device (Section 4.1), one shot per
// lane.
//
// The draws are the same pure function of (seed, shot index) as the host
// sampler: SplitMix64 (Steele, Lea, Flood 2014) seeded with
// mix(seed ^ mix(shot)); a weight w either given per shot or found by
// inverting the FP64 cumulative Bin(M, p) table against u = (x >> 11) 2^-53;
// Floyd's uniform w-subset of the M channels with Lemire's bounded integers;
// the subset in ascending order; one uniform non-identity Pauli per chosen
// channel (3, 15 or 63 choices for a one-, two- or three-qubit depolarising
// channel, X for an X flip).  Only integer and IEEE basic operations are
// used, so every bit of the CSR matches the host's.
//
// Three launches: (1) every lane draws its shot's weight and the block
// writes block-local inclusive prefixes of the weights to shot_off[i+1]
// plus the block total; (2) one block scans the block totals; (3) every
// lane adds its block's base to shot_off[i+1], replays its generator and
// writes its channels and Paulis at that offset (only when the slice ends
// within the caller's capacity, so an undersized output is never written
// past its end).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

// the one-workgroup scans use 256 threads: small enough to find room beside
// resident shot kernels of other streams
constexpr int kScanT = 256;

constexpr int ST = 256;   // shots per block
constexpr int kSup = 256; // blocks per superblock of the offset scan
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct DevRng {
    uint64_t s;
    __device__ DevRng(uint64_t seed, uint64_t shot) : s(mix64(seed ^ mix64(shot))) {}
    __device__ uint64_t next() {
        s += kGolden;
        return mix64(s);
    }
    // uniform integer in [0, n): Lemire's multiply-and-reject
    __device__ uint64_t bounded(uint64_t n) {
        uint64_t x = next();
        uint64_t lo = x * n;
        uint64_t hi = __umul64hi(x, n);
        if (lo < n) {
            const uint64_t t = (0ull - n) % n;
            while (lo < t) {
                x = next();
                lo = x * n;
                hi = __umul64hi(x, n);
            }
        }
        return hi;
    }
    __device__ double uniform01() {
        return static_cast<double>(next() >> 11) * (1.0 / 9007199254740992.0);
    }
};

// weight of one shot; advances rng exactly as the host does
__device__ __forceinline__ int64_t draw_weight(DevRng& rng, int64_t i, const int32_t* weights,
                                               const double* cdf, int32_t n_cdf, int64_t M) {
    int64_t w;
    if (weights) {
        w = weights[i];
        if (w < 0) w = 0;
    } else {
        const double u = rng.uniform01();
        w = n_cdf - 1;
        for (int32_t k = 0; k < n_cdf; ++k) {
            if (u < cdf[k]) {
                w = k;
                break;
            }
        }
    }
    return w < M ? w : M;
}

__global__ __launch_bounds__(ST) void weight_kernel(int64_t n, uint64_t seed, uint64_t first,
                                                    const int32_t* __restrict__ weights,
                                                    const double* __restrict__ cdf, int32_t n_cdf,
                                                    int64_t M, int64_t* __restrict__ shot_off,
                                                    int64_t* __restrict__ block_tot) {
    __shared__ int64_t s[ST];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x;
    int64_t w = 0;
    if (i < n) {
        DevRng rng(seed, first + static_cast<uint64_t>(i));
        w = draw_weight(rng, i, weights, cdf, n_cdf, M);
    }
    s[threadIdx.x] = w;
    __syncthreads();
    // Hillis-Steele inclusive scan over the block
    for (int d = 1; d < ST; d <<= 1) {
        const int64_t v = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    if (i < n) shot_off[i + 1] = s[threadIdx.x];
    if (threadIdx.x == ST - 1) block_tot[blockIdx.x] = s[ST - 1];
}

// exclusive scan of the block totals within each superblock of kSup blocks,
// in place (one workgroup per superblock, coalesced), the superblock's
// total into sup[superblock]
__global__ __launch_bounds__(kSup) void local_scan_kernel(int64_t* cnt, int64_t nb,
                                                          int64_t* sup) {
    __shared__ int64_t sh[kSup];
    const int t = threadIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kSup + t;
    const int64_t v = j < nb ? cnt[j] : 0;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kSup; d <<= 1) {
        const int64_t a = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    if (j < nb) cnt[j] = sh[t] - v;
    if (t == kSup - 1) sup[blockIdx.x] = sh[t];
}

// exclusive scan of the superblock totals in place (one block), grand total
// at [nb]
__global__ __launch_bounds__(kScanT) void total_scan_kernel(int64_t* cnt, int64_t nb) {
    __shared__ int64_t part[kScanT];
    const int tid = threadIdx.x;
    const int64_t per = (nb + kScanT - 1) / kScanT;
    const int64_t lo = tid * per, hi = (lo + per < nb) ? lo + per : nb;
    int64_t acc = 0;
    for (int64_t j = lo; j < hi; ++j) acc += cnt[j];
    part[tid] = acc;
    __syncthreads();
    for (int d = 1; d < kScanT; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = tid ? part[tid - 1] : 0;
    if (tid == kScanT - 1) cnt[nb] = part[kScanT - 1];
    for (int64_t j = lo; j < hi; ++j) {
        const int64_t v = cnt[j];
        cnt[j] = run;
        run += v;
    }
}

__global__ __launch_bounds__(ST) void draw_kernel(int64_t n, uint64_t seed, uint64_t first,
                                                  const int32_t* __restrict__ weights,
                                                  const double* __restrict__ cdf, int32_t n_cdf,
                                                  int64_t M, const uint8_t* __restrict__ kind,
                                                  const int64_t* __restrict__ block_base,
                                                  const int64_t* __restrict__ sup_base,
                                                  int64_t nnz_cap, int64_t* __restrict__ shot_off,
                                                  int32_t* __restrict__ chan,
                                                  uint8_t* __restrict__ pauli) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x;
    if (i == 0) shot_off[0] = 0;
    if (i >= n) return;
    DevRng rng(seed, first + static_cast<uint64_t>(i));
    const int64_t w = draw_weight(rng, i, weights, cdf, n_cdf, M);
    const int64_t end = shot_off[i + 1] + block_base[blockIdx.x] + sup_base[blockIdx.x / kSup];
    shot_off[i + 1] = end;
    const int64_t o = end - w;
    if (w == 0 || end > nnz_cap) return;
    int32_t* c = chan + o;
    // Floyd: for j in [M-w, M) take t uniform in [0, j], or j if t is taken
    int64_t k = 0;
    for (int64_t j = M - w; j < M; ++j) {
        const int32_t t = static_cast<int32_t>(rng.bounded(static_cast<uint64_t>(j + 1)));
        bool have = false;
        for (int64_t q = 0; q < k; ++q) have |= c[q] == t;
        c[k++] = have ? static_cast<int32_t>(j) : t;
    }
    // ascending order (insertion sort: w is small on the hot path)
    for (int64_t a = 1; a < w; ++a) {
        const int32_t v = c[a];
        int64_t b = a - 1;
        while (b >= 0 && c[b] > v) {
            c[b + 1] = c[b];
            --b;
        }
        c[b + 1] = v;
    }
    for (int64_t a = 0; a < w; ++a) {
        const int kd = kind[c[a]];
        uint8_t code;
        if (kd == CH_XERR) code = 1;
        else if (kd == CH_DEP1) code = static_cast<uint8_t>(1 + rng.bounded(3));
        else if (kd == CH_DEP2) code = static_cast<uint8_t>(1 + rng.bounded(15));
        else code = static_cast<uint8_t>(1 + rng.bounded(63));
        pauli[o + a] = code;
    }
}

}  // namespace

// the block totals, the superblock totals, the grand total
int64_t sampler_tmp_words(int64_t n) {
    const int64_t nb = (n + ST - 1) / ST;
    return nb + (nb + kSup - 1) / kSup + 1;
}

hipError_t launch_sampler(int64_t n, uint64_t seed, uint64_t first, const int32_t* weights,
                          const double* cdf, int32_t n_cdf, int64_t M, const uint8_t* kind,
                          int64_t nnz_cap, int64_t* shot_off, int32_t* chan, uint8_t* pauli,
                          int64_t* tmp, int64_t n_tmp, hipStream_t s) {
    const int64_t nb = (n + ST - 1) / ST;
    if (nb == 0) return hipSuccess;
    const int64_t ns = (nb + kSup - 1) / kSup;
    if (n_tmp < nb + ns + 1 || nb > 0x7fffffff) return hipErrorInvalidValue;
    int64_t* sup = tmp + nb;
    if (!weights && (!cdf || n_cdf < 1)) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(nb));
    hipLaunchKernelGGL(weight_kernel, grid, dim3(ST), 0, s, n, seed, first, weights, cdf, n_cdf, M,
                       shot_off, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(local_scan_kernel, dim3(static_cast<unsigned>(ns)), dim3(kSup), 0, s, tmp,
                       nb, sup);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(total_scan_kernel, dim3(1), dim3(kScanT), 0, s, sup, ns);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(draw_kernel, grid, dim3(ST), 0, s, n, seed, first, weights, cdf, n_cdf, M,
                       kind, tmp, sup, nnz_cap, shot_off, chan, pauli);
    return hipGetLastError();
}

}  // namespace msc
