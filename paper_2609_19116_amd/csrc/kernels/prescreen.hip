// Offline-screening kernel (Section 4.2): one shot per lane.
//
// A shot's signature over the decided measurements is the XOR of its
// faults' signatures; the shot must be simulated iff that signature is
// zero.  A fault's signature (the XOR of its basis components, X and Z on
// each of the channel's up to three qubits) is precombined per (channel,
// Pauli code) on the host, so each fault costs one W-word lookup.  Each lane
// streams its shot's CSR slice from HBM, XORs <= W-word signatures from the
// L2-resident table in registers, and the wavefront's verdicts are packed
// with a 64-lane ballot into one uint64 of the survivor bitmap (lane j of
// wave w <-> shot 64 w + j).  A second pass turns the bitmap into an
// ascending survivor index list: per-block popcounts, one scan block, and a
// scatter with a per-wave prefix from the ballot mask.  Integer only.
//
// The CSR is checked on the way: a channel index outside [0, M), channels
// not strictly ascending within a shot, a Pauli code that is zero or names
// a qubit the channel does not have, or decreasing offsets set bits of a
// device flag word (CsrFlag), and the host turns a nonzero flag into
// MSC_E_INVALID.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.h"

namespace msc {
namespace {

// the one-workgroup scans use 256 threads: small enough to find room beside
// resident shot kernels of other streams
constexpr int kScanT = 256;

constexpr int PT = 256;   // threads per block (4 waves, 256 shots)
constexpr int kSup = 256; // blocks per superblock of the survivor scan

// tmp words of a screen of n shots: the per-block survivor counts (their
// scan in place), the superblock totals (their scan in place, plus one),
// the survivor total and the CSR flag word
constexpr int64_t screen_tmp_words(int64_t n) {
    return (n + PT - 1) / PT + ((n + PT - 1) / PT + kSup - 1) / kSup + 1 + 2;
}

// Largest Pauli code + 1 of each channel kind (ChanKind order): one qubit
// (x, z bits), two, the X flip (x of qubit 0 only), three.
__device__ __forceinline__ int code_limit(int kind) {
    return kind == CH_DEP1 ? 4 : kind == CH_DEP2 ? 16 : kind == CH_XERR ? 2 : 64;
}

// Checks of one fault against the previous one of its shot (CsrFlag bits).
__device__ __forceinline__ int fault_check(int64_t c, int64_t prev, int p, int32_t nch,
                                           const uint8_t* __restrict__ kind) {
    if (c < 0 || c >= nch) return CSR_BAD_CHANNEL;
    int bad = c <= prev ? CSR_NOT_ASCENDING : 0;
    if (p == 0 || p >= code_limit(kind[c])) bad |= CSR_BAD_PAULI;
    return bad;
}

template <int W>
__global__ __launch_bounds__(PT) void screen_kernel(int32_t nch, int64_t n,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ chan,
                                                    const uint8_t* __restrict__ pauli,
                                                    const uint64_t* __restrict__ sig,
                                                    const int32_t* __restrict__ sig_off,
                                                    const uint8_t* __restrict__ /*kind*/,
                                                    uint64_t* __restrict__ bits,
                                                    int64_t* __restrict__ block_cnt,
                                                    int* __restrict__ flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * PT + threadIdx.x;
    bool alive = false;
    int bad = 0;
    if (i < n) {
        uint64_t acc[W];
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] = 0;
        const int64_t f0 = off[i], f1 = off[i + 1];
        if (f1 < f0 || f0 < 0) bad |= CSR_BAD_OFFSETS;
        int64_t prev = -1;
        for (int64_t f = f0; f < f1; ++f) {
            const int64_t c = chan[f];
            const int p = pauli[f];
            // the channel's first table entry and its kind, one load
            const int32_t ek = c >= 0 && c < nch ? sig_off[c] : 0;
            int fb = 0;
            if (c < 0 || c >= nch) {
                fb = CSR_BAD_CHANNEL;
            } else {
                fb = c <= prev ? CSR_NOT_ASCENDING : 0;
                if (p == 0 || p >= code_limit(ek & 3)) fb |= CSR_BAD_PAULI;
            }
            bad |= fb;
            prev = c;
            // an invalid channel or code has no entry (the call fails anyway)
            if (fb & (CSR_BAD_CHANNEL | CSR_BAD_PAULI)) continue;
            const uint64_t* s = sig + (static_cast<int64_t>(ek >> 2) + p) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) acc[w] ^= s[w];
        }
        uint64_t any = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) any |= acc[w];
        alive = any == 0;
    }
    if (bad) atomicOr(flag, bad);
    const uint64_t mask = __ballot(alive);
    const int lane = threadIdx.x & 63;
    const int64_t word = (static_cast<int64_t>(blockIdx.x) * PT + (threadIdx.x & ~63)) >> 6;
    __shared__ int s_cnt[PT / 64];
    if (lane == 0) {
        if (word * 64 < n) bits[word] = mask;
        s_cnt[threadIdx.x >> 6] = __popcll(mask);
    }
    __syncthreads();
    if (threadIdx.x == 0 && block_cnt) {
        int64_t t = 0;
        for (int w = 0; w < PT / 64; ++w) t += s_cnt[w];
        block_cnt[blockIdx.x] = t;
    }
}

// The same checks alone, one shot per lane (for the entry points that
// take a caller's CSR without screening it).
__global__ __launch_bounds__(PT) void validate_kernel(int32_t nch, int64_t n,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ chan,
                                                      const uint8_t* __restrict__ pauli,
                                                      const uint8_t* __restrict__ kind,
                                                      int* __restrict__ flag) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * PT + threadIdx.x;
    if (i >= n) return;
    const int64_t f0 = off[i], f1 = off[i + 1];
    int bad = (f1 < f0 || f0 < 0) ? CSR_BAD_OFFSETS : 0;
    int64_t prev = -1;
    for (int64_t f = f0; f < f1; ++f) {
        const int64_t c = chan[f];
        bad |= fault_check(c, prev, pauli[f], nch, kind);
        prev = c;
    }
    if (bad) atomicOr(flag, bad);
}

// one word set to zero by a kernel (a fill node, not a memset, if captured)
__global__ void clear_flag_kernel(int* flag) { *flag = 0; }

// exclusive scan of the block counts within each superblock of kSup blocks,
// in place (one workgroup per superblock, coalesced), the superblock's total
// into sup[superblock]
__global__ __launch_bounds__(kSup) void scan_local_kernel(int64_t* cnt, int64_t nb,
                                                          int64_t* sup) {
    __shared__ int64_t s[kSup];
    const int t = threadIdx.x;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kSup + t;
    const int64_t v = j < nb ? cnt[j] : 0;
    s[t] = v;
    __syncthreads();
    // inclusive scan in LDS, log2(kSup) steps
    for (int d = 1; d < kSup; d <<= 1) {
        const int64_t a = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    if (j < nb) cnt[j] = s[t] - v;
    if (t == kSup - 1) sup[blockIdx.x] = s[t];
}

// exclusive scan of the superblock totals in place (one block), the total
// at *total
__global__ __launch_bounds__(kScanT) void scan_kernel(int64_t* cnt, int64_t nb, int64_t* total) {
    __shared__ int64_t part[kScanT];
    const int tid = threadIdx.x;
    const int64_t per = (nb + kScanT - 1) / kScanT;
    const int64_t lo = tid * per, hi = (lo + per < nb) ? lo + per : nb;
    int64_t s = 0;
    for (int64_t j = lo; j < hi; ++j) s += cnt[j];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int j = 0; j < kScanT; ++j) {
            int64_t v = part[j];
            part[j] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int64_t run = part[tid];
    for (int64_t j = lo; j < hi; ++j) {
        int64_t v = cnt[j];
        cnt[j] = run;
        run += v;
    }
}

__global__ __launch_bounds__(PT) void scatter_kernel(int64_t n, const uint64_t* __restrict__ bits,
                                                     const int64_t* __restrict__ block_off,
                                                     const int64_t* __restrict__ sup_off,
                                                     int64_t* __restrict__ idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * PT + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t word = (static_cast<int64_t>(blockIdx.x) * PT + (threadIdx.x & ~63)) >> 6;
    const uint64_t mask = (word * 64 < n) ? bits[word] : 0ull;
    __shared__ int s_pre[PT / 64];
    if (lane == 0) s_pre[wv] = __popcll(mask);
    __syncthreads();
    int64_t base = sup_off[blockIdx.x / kSup] + block_off[blockIdx.x];
    for (int w = 0; w < wv; ++w) base += s_pre[w];
    if (i < n && ((mask >> lane) & 1)) {
        const uint64_t below = lane ? (mask & ((1ull << lane) - 1)) : 0ull;
        idx[base + __popcll(below)] = i;
    }
}

}  // namespace

int64_t prescreen_tmp_words(int64_t n) { return screen_tmp_words(n); }

hipError_t launch_prescreen(int words, int32_t n_channels, int64_t n, const int64_t* off, const int32_t* chan,
                            const uint8_t* pauli, const uint64_t* sig, const int32_t* sig_off,
                            const uint8_t* kind,
                            uint64_t* bits, int64_t* survivor_idx, int64_t* block_tmp,
                            int64_t n_blocks_tmp, int* flag, hipStream_t s) {
    const int64_t nb = (n + PT - 1) / PT;
    if (nb == 0) return hipSuccess;
    const int64_t ns = (nb + kSup - 1) / kSup;
    if (n_blocks_tmp < screen_tmp_words(n) || !flag) return hipErrorInvalidValue;
    int64_t* sup = block_tmp + nb;                    // ns + 1 words
    int64_t* total = block_tmp + n_blocks_tmp - 2;    // then the flag word
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    dim3 grid(static_cast<unsigned>(nb));
    switch (words) {
#define MSC_SCREEN_CASE(WW)                                                                   \
    case WW:                                                                                  \
        hipLaunchKernelGGL(screen_kernel<WW>, grid, dim3(PT), 0, s, n_channels, n, off, chan,  \
                           pauli, sig, sig_off, kind, bits, block_tmp, flag);                 \
        break;
        MSC_SCREEN_CASE(1)
        MSC_SCREEN_CASE(2)
        MSC_SCREEN_CASE(3)
        MSC_SCREEN_CASE(4)
        MSC_SCREEN_CASE(5)
        MSC_SCREEN_CASE(6)
        MSC_SCREEN_CASE(7)
        MSC_SCREEN_CASE(8)
#undef MSC_SCREEN_CASE
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_local_kernel, dim3(static_cast<unsigned>(ns)), dim3(kSup), 0, s,
                       block_tmp, nb, sup);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanT), 0, s, sup, ns, total);
    e = hipGetLastError();
    if (e != hipSuccess || !survivor_idx) return e;
    hipLaunchKernelGGL(scatter_kernel, grid, dim3(PT), 0, s, n, bits, block_tmp, sup,
                       survivor_idx);
    return hipGetLastError();
}

hipError_t launch_validate_csr(int32_t n_channels, int64_t n, const int64_t* off,
                               const int32_t* chan, const uint8_t* pauli, const uint8_t* kind,
                               int* flag, hipStream_t s) {
    if (!flag) return hipErrorInvalidValue;
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    const dim3 grid(static_cast<unsigned>((n + PT - 1) / PT));
    hipLaunchKernelGGL(validate_kernel, grid, dim3(PT), 0, s, n_channels, n, off, chan, pauli,
                       kind, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed scratch of msc_prescreen_noalloc: the block counts and their scan
// (one word per 256 shots), the superblock totals, the survivor total and
// the CSR flag, for at most kNoAllocShots shots.  Each device holds its own copy until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host it
// is only a stand-in symbol): the device address is resolved once per device
// with hipGetSymbolAddress and that pointer is used everywhere.
namespace {
constexpr int64_t kNoAllocWords = screen_tmp_words(kNoAllocShots);
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) int64_t scratch[kNoAllocWords];

static std::mutex g_scratch_mu;
static int64_t* g_scratch_ptr[kMaxDevices] = {};

hipError_t prescreen_noalloc_scratch(int device, int64_t** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<int64_t*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace msc
