// Batched two-site contraction + gate on MFMA (Section 3.1): FP32 split
// complex with FP32 accumulation, or BF16x3 split precision.
//
// theta[(a,i),(j,b)] = sum_{i'j'} G[ij][i'j'] sum_c A[(a,i'),c] B[c,(j',b)]
//
// The complex product is four real GEMMs on v_mfma_f32_16x16x4f32:
// Re += Ar Br + (-Ai) Bi, Im += Ar Bi + Ai Br.  A workgroup (4 waves) owns a
// 128-row x (64 b, both j') tile of one batch element; K = chi is streamed
// through double-buffered LDS in steps of 16.  Each wave keeps a 64 x (32 b,
// both j') accumulator block, so the four (i', j') partial products of an
// output (a, b) sit in the same lane and the 4x4 gate is applied in
// registers before the single store of theta.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128;   // rows (a,i) per workgroup
constexpr int TB = 64;    // b columns per workgroup (times 2 for j')
constexpr int TK = 16;    // k per LDS stage
constexpr int NTH = 256;

// Workgroups are dispatched to the 8 XCDs in turn (block h runs on XCD
// h mod 8).  Block h takes the logical block that makes each XCD work
// through one contiguous run of logical blocks, so the tiles of one batch
// element share that XCD's L2 instead of being spread over all eight.
__device__ __forceinline__ int xcd_block(int h, int nb) {
    return (nb & 7) ? h : (h & 7) * (nb >> 3) + (h >> 3);
}

__global__ __launch_bounds__(NTH) void twosite_kernel(int chi, int tiles, const float* __restrict__ Ag,
                                                      const float* __restrict__ Bg,
                                                      const float* __restrict__ gate,
                                                      float* __restrict__ Tg) {
    // LDS: [stage][plane][k][col]
    __shared__ float As[2][2][TK][TM];
    __shared__ float Bs[2][2][TK][2 * TB];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m = 2 * chi;                    // rows of A and theta
    const int n = 2 * chi;                    // columns of B and theta
    const int rows_tiles = m / TM;
    const int lg = xcd_block(blockIdx.x, gridDim.x);
    const int tile = lg % tiles;
    const int R0 = (tile % rows_tiles) * TM;
    const int B0 = (tile / rows_tiles) * TB;
    const size_t bidx = lg / tiles;
    const float* A = Ag + bidx * 2 * (size_t)m * chi;
    const float* Bm = Bg + bidx * 2 * (size_t)chi * n;
    float* T = Tg + bidx * 2 * (size_t)m * n;

    float g[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) g[j] = gate[j];

    floatx4 acc[4][2][2][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int d = 0; d < 2; ++d) acc[a][b][c][d] = floatx4{0.f, 0.f, 0.f, 0.f};

    float4 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int idx = tid + NTH * s;
            const int plane = idx >> 9, rem = idx & 511;
            const int row = rem >> 2, kq = rem & 3;
            ra[s] = *reinterpret_cast<const float4*>(A + (size_t)plane * m * chi +
                                                     (size_t)(R0 + row) * chi + k0 + 4 * kq);
            const int kr = rem >> 5, cq = rem & 31;
            const int cl = 4 * cq;
            const int col = (cl >> 6) * chi + B0 + (cl & 63);
            rb[s] = *reinterpret_cast<const float4*>(Bm + (size_t)plane * chi * n +
                                                     (size_t)(k0 + kr) * n + col);
        }
    };
    auto lstore = [&](int st) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int idx = tid + NTH * s;
            const int plane = idx >> 9, rem = idx & 511;
            const int row = rem >> 2, kq = rem & 3;
            As[st][plane][4 * kq + 0][row] = ra[s].x;
            As[st][plane][4 * kq + 1][row] = ra[s].y;
            As[st][plane][4 * kq + 2][row] = ra[s].z;
            As[st][plane][4 * kq + 3][row] = ra[s].w;
            const int kr = rem >> 5, cq = rem & 31;
            *reinterpret_cast<float4*>(&Bs[st][plane][kr][4 * cq]) = rb[s];
        }
    };

    const int nk = chi / TK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int st = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * TK);
#pragma unroll
        for (int ks = 0; ks < TK / 4; ++ks) {
            const int kk = 4 * ks + (lane >> 4);
            float ar[4], ai[4], br[2][2], bi[2][2];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int r = wm * 64 + mt * 16 + (lane & 15);
                ar[mt] = As[st][0][kk][r];
                ai[mt] = As[st][1][kk][r];
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int jp = 0; jp < 2; ++jp) {
                    const int c = jp * TB + wn * 32 + nt * 16 + (lane & 15);
                    br[nt][jp] = Bs[st][0][kk][c];
                    bi[nt][jp] = Bs[st][1][kk][c];
                }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int jp = 0; jp < 2; ++jp) {
                        floatx4& re = acc[mt][nt][jp][0];
                        floatx4& im = acc[mt][nt][jp][1];
                        re = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], br[nt][jp], re, 0, 0, 0);
                        re = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[mt], bi[nt][jp], re, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[mt], bi[nt][jp], im, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mt], br[nt][jp], im, 0, 0, 0);
                    }
        }
        if (kt + 1 < nk) lstore(st ^ 1);
        __syncthreads();
    }

    // epilogue: gate on the physical legs, then store theta
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int rp = 0; rp < 2; ++rp) {
                // rows 4*(lane/16) + 2 rp + i' of this 16x16 tile
                const int row0 = R0 + wm * 64 + mt * 16 + 4 * (lane >> 4) + 2 * rp;
                const int b = B0 + wn * 32 + nt * 16 + (lane & 15);
                float sr[4], si[4];   // S[i'j'] at index 2 i' + j'
#pragma unroll
                for (int ip = 0; ip < 2; ++ip)
#pragma unroll
                    for (int jp = 0; jp < 2; ++jp) {
                        sr[2 * ip + jp] = acc[mt][nt][jp][0][2 * rp + ip];
                        si[2 * ip + jp] = acc[mt][nt][jp][1][2 * rp + ip];
                    }
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    float xr = 0.f, xi = 0.f;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float gr = g[2 * (4 * o + j)], gi = g[2 * (4 * o + j) + 1];
                        xr += gr * sr[j] - gi * si[j];
                        xi += gr * si[j] + gi * sr[j];
                    }
                    const int i = o >> 1, j = o & 1;
                    const size_t at = (size_t)(row0 + i) * n + (size_t)j * chi + b;
                    T[at] = xr;
                    T[(size_t)m * n + at] = xi;
                }
            }
}

// ---------------------------------------------------------------------------
// BF16x3 split precision: every FP32 operand x is split into x_hi = bf16(x)
// and x_lo = bf16(x - x_hi) (round to nearest even, v_cvt_pk_bf16_f32), and
// a real product is x_hi y_hi + x_hi y_lo + x_lo y_hi with FP32
// accumulation on v_mfma_f32_16x16x32_bf16 (the x_lo y_lo term, ~2^-16
// relative, is dropped).  Workgroup tile: 64 rows x (64 b, both j'); each of
// the 4 waves keeps a 32 x (32 b, both j') block; K = chi is streamed in
// steps of 32 through LDS with the next step prefetched into registers.
// Every thread splits runs of 8 consecutive k of one row of A or one column
// of B, so each hi or lo run is one 16-byte LDS store in the k-contiguous
// layout the MFMA operands are read in.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int BM = 64;    // rows per workgroup
constexpr int BB = 64;    // b columns per workgroup (times 2 for j')
constexpr int BK = 32;    // k per step (one MFMA)
constexpr int BKP = 40;   // padded k stride in LDS (bf16 elements)

// hi/lo split of 8 consecutive values: hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split8(const float (&x)[8], uint4& hi, uint4& lo) {
    unsigned h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const f32x2 v = {x[2 * p], x[2 * p + 1]};
        const unsigned hu = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
        const f32x2 r = {v.x - __uint_as_float(hu << 16), v.y - __uint_as_float(hu & 0xffff0000u)};
        h[p] = hu;
        l[p] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
    }
    hi = make_uint4(h[0], h[1], h[2], h[3]);
    lo = make_uint4(l[0], l[1], l[2], l[3]);
}

__global__ __launch_bounds__(NTH, 2) void twosite_bf16x3_kernel(int chi, int tiles,
                                                                const float* __restrict__ Ag,
                                                                const float* __restrict__ Bg,
                                                                const float* __restrict__ gate,
                                                                float* __restrict__ Tg) {
    // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo; A as [row][k], B as [col][k]
    __shared__ __attribute__((aligned(16))) unsigned short As[4][BM][BKP];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[4][2 * BB][BKP];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m = 2 * chi, n = 2 * chi;
    const int rows_tiles = m / BM;
    const int lg = xcd_block(blockIdx.x, gridDim.x);
    const int tile = lg % tiles;
    const int R0 = (tile % rows_tiles) * BM;
    const int B0 = (tile / rows_tiles) * BB;
    const size_t bidx = lg / tiles;
    const float* A = Ag + bidx * 2 * (size_t)m * chi;
    const float* Bm = Bg + bidx * 2 * (size_t)chi * n;
    float* T = Tg + bidx * 2 * (size_t)m * n;

    float g[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) g[j] = gate[j];

    floatx4 acc[2][2][2][2];   // [mt][nt][jp][re/im]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int d = 0; d < 2; ++d) acc[a][b][c][d] = floatx4{0.f, 0.f, 0.f, 0.f};

    // A: 64 rows x 4 runs of 8 k, one (row, run) of both planes per thread
    // (run index fastest across lanes); B: 2 planes x 32 column quads x 4 runs of 8 k,
    // one (quad, run) per thread, loaded as 8 rows of 4 columns
    const int a_row = (tid >> 2) & 63, a_kc = tid & 3;
    const int b_plane = tid >> 7, b_cq = (tid >> 2) & 31, b_kc = tid & 3;
    const int b_col = ((4 * b_cq) >> 6) * chi + B0 + ((4 * b_cq) & 63);
    float4 ra[2][2], rb[8];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {          // s = plane
            const float* src = A + (size_t)s * m * chi + (size_t)(R0 + a_row) * chi + k0 + 8 * a_kc;
            ra[s][0] = *reinterpret_cast<const float4*>(src);
            ra[s][1] = *reinterpret_cast<const float4*>(src + 4);
        }
        const float* src = Bm + (size_t)b_plane * chi * n + (size_t)(k0 + 8 * b_kc) * n + b_col;
#pragma unroll
        for (int e = 0; e < 8; ++e) rb[e] = *reinterpret_cast<const float4*>(src + (size_t)e * n);
    };
    auto lstore = [&]() {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float x[8] = {ra[s][0].x, ra[s][0].y, ra[s][0].z, ra[s][0].w,
                                ra[s][1].x, ra[s][1].y, ra[s][1].z, ra[s][1].w};
            uint4 hi, lo;
            split8(x, hi, lo);
            *reinterpret_cast<uint4*>(&As[2 * s][a_row][8 * a_kc]) = hi;
            *reinterpret_cast<uint4*>(&As[2 * s + 1][a_row][8 * a_kc]) = lo;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = c == 0 ? rb[e].x : c == 1 ? rb[e].y : c == 2 ? rb[e].z : rb[e].w;
            uint4 hi, lo;
            split8(x, hi, lo);
            *reinterpret_cast<uint4*>(&Bs[2 * b_plane][4 * b_cq + c][8 * b_kc]) = hi;
            *reinterpret_cast<uint4*>(&Bs[2 * b_plane + 1][4 * b_cq + c][8 * b_kc]) = lo;
        }
    };
    auto frag = [&](const unsigned short* p) { return *reinterpret_cast<const bf16x8*>(p); };
    auto neg = [&](bf16x8 x) {   // both sign bits of each dword at once
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        u32x4 u = __builtin_bit_cast(u32x4, x);
        u ^= 0x80008000u;
        return __builtin_bit_cast(bf16x8, u);
    };

    const int nk = chi / BK;
    gload(0);
    for (int kt = 0; kt < nk; ++kt) {
        lstore();
        __syncthreads();
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const int kk = 8 * (lane >> 4);
        bf16x8 a[2][6];   // re_hi re_lo im_hi im_lo -im_hi -im_lo
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const int r = wm * 32 + mt * 16 + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) a[mt][pl] = frag(&As[pl][r][kk]);
            a[mt][4] = neg(a[mt][2]);
            a[mt][5] = neg(a[mt][3]);
        }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int jp = 0; jp < 2; ++jp) {
                const int c = jp * BB + wn * 32 + nt * 16 + (lane & 15);
                bf16x8 b[4];
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) b[pl] = frag(&Bs[pl][c][kk]);
                // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br   (each x3); the
                // four accumulators of (mt, re/im) advance in turn
                const int ta[6] = {0, 0, 1, 4, 4, 5}, tb[6] = {0, 1, 0, 2, 3, 2};
                const int ua[6] = {0, 0, 1, 2, 2, 3}, ub[6] = {2, 3, 2, 0, 1, 0};
#pragma unroll
                for (int t = 0; t < 6; ++t)
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        floatx4& re = acc[mt][nt][jp][0];
                        floatx4& im = acc[mt][nt][jp][1];
                        re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][ta[t]], b[tb[t]], re, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][ua[t]], b[ub[t]], im, 0, 0, 0);
                    }
            }
        __syncthreads();
    }

#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int rp = 0; rp < 2; ++rp) {
                const int row0 = R0 + wm * 32 + mt * 16 + 4 * (lane >> 4) + 2 * rp;
                const int b = B0 + wn * 32 + nt * 16 + (lane & 15);
                float sr[4], si[4];
#pragma unroll
                for (int ip = 0; ip < 2; ++ip)
#pragma unroll
                    for (int jp = 0; jp < 2; ++jp) {
                        sr[2 * ip + jp] = acc[mt][nt][jp][0][2 * rp + ip];
                        si[2 * ip + jp] = acc[mt][nt][jp][1][2 * rp + ip];
                    }
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    float xr = 0.f, xi = 0.f;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float gr = g[2 * (4 * o + j)], gi = g[2 * (4 * o + j) + 1];
                        xr += gr * sr[j] - gi * si[j];
                        xi += gr * si[j] + gi * sr[j];
                    }
                    const int i = o >> 1, j = o & 1;
                    const size_t at = (size_t)(row0 + i) * n + (size_t)j * chi + b;
                    T[at] = xr;
                    T[(size_t)m * n + at] = xi;
                }
            }
}

}  // namespace

hipError_t launch_twosite(int precision, int chi, int batch, const float* A, const float* B,
                          const float* gate, float* theta, hipStream_t s) {
    if (chi % 64 != 0 || chi < 64) return hipErrorInvalidValue;
    if (precision == MSC_BF16X3) {
        const int tiles = (2 * chi / BM) * (chi / BB);
        hipLaunchKernelGGL(twosite_bf16x3_kernel, dim3(tiles * batch), dim3(NTH), 0, s, chi, tiles,
                           A, B, gate, theta);
    } else {
        const int tiles = (2 * chi / TM) * (chi / TB);
        hipLaunchKernelGGL(twosite_kernel, dim3(tiles * batch), dim3(NTH), 0, s, chi, tiles, A, B,
                           gate, theta);
    }
    return hipGetLastError();
}

}  // namespace msc
