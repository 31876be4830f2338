// Batched large two-site updates on MFMA (Section 3.1): the contraction
// theta = G (A[k] A[k+1]) and the FP64 Gram matrix of theta's vectors for
// every shot the shot kernel parked, ragged shapes in one tile list.
//
// A parked shot i has bonds cl, cm, cr around sites k, k+1 (its saved
// state).  Its theta is m x n = 2cl x 2cr (rows (a,i), columns (j,b)), stored
// planar in the slot's theta buffer.  The contraction is a complex GEMM over
// c < cm split into real MFMA products (Re += Ar Br - Ai Bi, Im += Ar Bi +
// Ai Br); a workgroup (2 x 2 waves) owns a tile of rows x (b values, both j')
// so the four (i', j') partial products of an output (a, b) end in the same
// lane and the 4x4 gate is applied in registers before the one store.
// Operands outside the shot's shape are read as zero and outputs outside it
// are not written, so one kernel serves every shape.
//
// The Gram matrix G = V^H V of the vectors the factorisation orthogonalises
// (theta's columns when the centre moves right, its rows when it moves left)
// is formed in FP64 on v_mfma_f64_16x16x4f64 from theta converted on load,
// for the tiles on and above the block diagonal.
//
// All kernels loop over the tile list with a fixed grid and read the list
// sizes from the plan in device memory.  Workgroup h runs on XCD h mod 8; the
// tile order is remapped so that each XCD walks a contiguous run of tiles
// (mostly one shot's), which keeps a shot's operands in one L2.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int NTH = 256;
constexpr int PLAN_T = 256;

// ---------------------------------------------------------------------------
// plan: shapes and tile counts of the parked shots, prefix sums

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

struct Tiles4 {
    LxTiles t[kLxBuckets];
};

// shapes of parked shot `slot`: theta's sides, vector count, bucket
__device__ __forceinline__ void parked_shape(const ShotState& st, int& cl, int& cr, int& nv,
                                             int& bk) {
    cl = st.chi[st.k];
    cr = st.chi[st.k + 2];
    nv = st.dir ? 2 * cr : 2 * cl;
    bk = lx_bucket(max(2 * cl, 2 * cr));
}

// One workgroup: the park list in park order, then per bucket its shots
// (in park order), their tile counts and the prefix sums.  The counts are
// exact integers, so the plan does not depend on thread timing.
__global__ __launch_bounds__(PLAN_T) void lx_plan_kernel(LxArgs a, Tiles4 tt) {
    __shared__ int s_c[PLAN_T], s_g[PLAN_T], s_n[PLAN_T];
    __shared__ double s_f[2][PLAN_T];
    LxPlan* pl = a.plan;
    const int tid = threadIdx.x;
    int cnt = *a.park_count;
    if (cnt > kLxMaxParked) cnt = kLxMaxParked;
    const int per = ceil_div(cnt, PLAN_T);
    const int lo = tid * per, hi = min(cnt, lo + per);
    // the round's algorithmic flops (integers, exact in FP64 in any order)
    double fc = 0.0, fg = 0.0;
    for (int i = lo; i < hi; ++i) {
        const ShotState& st = a.state[a.park_list[i]];
        pl->slot[i] = a.park_list[i];
        const double cl = st.chi[st.k], cm = st.chi[st.k + 1], cr = st.chi[st.k + 2];
        const double nv = st.dir ? 2 * cr : 2 * cl, len = st.dir ? 2 * cl : 2 * cr;
        fc += 32.0 * cl * cm * cr;
        fg += 4.0 * nv * (nv + 1.0) * len;
    }
    s_f[0][tid] = fc;
    s_f[1][tid] = fg;
    __syncthreads();
    if (tid == 0) {
        pl->count = cnt;
        double tc = 0.0, tg = 0.0;
        for (int j = 0; j < PLAN_T; ++j) {
            tc += s_f[0][j];
            tg += s_f[1][j];
        }
        a.flops[0] += tc;
        a.flops[1] += tg;
    }
    for (int b = 0; b < kLxBuckets; ++b) {
        const LxTiles t = tt.t[b];
        int sc = 0, sg = 0, sn = 0;
        for (int i = lo; i < hi; ++i) {
            int cl, cr, nv, bk;
            parked_shape(a.state[a.park_list[i]], cl, cr, nv, bk);
            if (bk != b) continue;
            const int nb = ceil_div(nv, t.gram);
            sc += ceil_div(2 * cl, t.cm_rows) * ceil_div(cr, t.cm_b);
            sg += nb * (nb + 1) / 2;
            ++sn;
        }
        __syncthreads();
        s_c[tid] = sc;
        s_g[tid] = sg;
        s_n[tid] = sn;
        __syncthreads();
        if (tid == 0) {
            int rc = 0, rg = 0, rn = 0;
            for (int j = 0; j < PLAN_T; ++j) {
                const int vc = s_c[j], vg = s_g[j], vn = s_n[j];
                s_c[j] = rc;
                s_g[j] = rg;
                s_n[j] = rn;
                rc += vc;
                rg += vg;
                rn += vn;
            }
            LxBucket& B = pl->b[b];
            B.count = rn;
            B.ctiles = rc;
            B.gtiles = rg;
            B.coff[rn] = rc;
            B.goff[rn] = rg;
        }
        __syncthreads();
        int rc = s_c[tid], rg = s_g[tid], rn = s_n[tid];
        LxBucket& B = pl->b[b];
        for (int i = lo; i < hi; ++i) {
            const int slot = a.park_list[i];
            int cl, cr, nv, bk;
            parked_shape(a.state[slot], cl, cr, nv, bk);
            if (bk != b) continue;
            const int nb = ceil_div(nv, t.gram);
            B.slot[rn] = slot;
            B.coff[rn] = rc;
            B.goff[rn] = rg;
            rc += ceil_div(2 * cl, t.cm_rows) * ceil_div(cr, t.cm_b);
            rg += nb * (nb + 1) / 2;
            ++rn;
        }
    }
}

__global__ void lx_reset_kernel(ShotState* state, int n_slots, int32_t* park_count,
                                double* flops, unsigned long long* counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_slots) state[i].status = kSlotRun;
    if (i == 0) {
        *park_count = 0;
        flops[0] = 0.0;
        flops[1] = 0.0;
        for (int q = 0; q < 4; ++q) counts[q] = 0;
    }
}

__global__ void lx_clear_kernel(int32_t* park_count) { *park_count = 0; }

// parked shot owning tile t: the last i with off[i] <= t (binary search)
__device__ __forceinline__ int owner(const int32_t* off, int cnt, int t) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// workgroup h -> logical tile h' so that XCD (h mod 8) walks a contiguous
// range of the tile list
__device__ __forceinline__ int xcd_tile(int h, int grid) {
    if (grid & 7) return h;
    return (h & 7) * (grid >> 3) + (h >> 3);
}

// ---------------------------------------------------------------------------
// contraction: T = float (v_mfma_f32_16x16x4f32) or double
// (v_mfma_f64_16x16x4f64); WM rows x WN b values per wave, 2 x 2 waves

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef floatx4 acc_t;
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    typedef doublex4 acc_t;
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Row of a 16 x 16 MFMA block that lane l feeds through the A operand,
// chosen so that lane l's four outputs are rows 4 (l / 16) + r, r = 0..3,
// for both instructions: v_mfma_f32_16x16x4f32 returns rows 4 (l / 16) + r
// of its A rows, v_mfma_f64_16x16x4f64 rows l / 16 + 4 r (checked on the
// device), so for FP64 A row rho = l mod 16 carries block row
// 4 (rho mod 4) + rho / 4.
template <typename T>
__device__ __forceinline__ int a_row(int lane) {
    if constexpr (sizeof(T) == sizeof(double)) return 4 * (lane & 3) + ((lane & 15) >> 2);
    return lane & 15;
}

constexpr int CK = 16;   // k per LDS stage

template <typename T, int WM, int WN>
__global__ __launch_bounds__(NTH) void lx_contract_kernel(LxArgs a, int bucket) {
    constexpr int BM = 2 * WM;          // rows (a,i) per workgroup
    constexpr int BN = 2 * WN;          // b values per workgroup
    constexpr int MT = WM / 16, NT2 = WN / 16;
    __shared__ T As[2][CK][BM];         // [plane][k][row]
    __shared__ T Bs[2][CK][2 * BN];     // [plane][k][(j', b)]
    typedef typename Mfma<T>::acc_t acc_t;

    const LxBucket* pl = &a.plan->b[bucket];
    const int total = pl->ctiles, cnt = pl->count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    for (int t0 = xcd_tile(blockIdx.x, gridDim.x); t0 < total; t0 += gridDim.x) {
        const int i = owner(pl->coff, cnt, t0);
        const int slot = pl->slot[i];
        const ShotState& st = a.state[slot];
        const int k = st.k;
        const int cl = st.chi[k], cm = st.chi[k + 1], cr = st.chi[k + 2];
        const int m = 2 * cl, n = 2 * cr;
        const int rtiles = (m + BM - 1) / BM;
        const int tl = t0 - pl->coff[i];
        const int R0 = (tl % rtiles) * BM;
        const int B0 = (tl / rtiles) * BN;
        const T* base = static_cast<const T*>(a.arena) + (size_t)slot * a.slot_stride;
        const T* Ar = base + a.site_off[k];
        const T* Ai = Ar + a.site_half[k];
        const T* Br = base + a.site_off[k + 1];
        const T* Bi = Br + a.site_half[k + 1];
        T* Th = static_cast<T*>(a.theta) + (size_t)slot * a.theta_stride;
        const double* g = a.g4 + st.gate_id * 32;

        acc_t acc[MT][NT2][2][2];
#pragma unroll
        for (int x = 0; x < MT; ++x)
#pragma unroll
            for (int y = 0; y < NT2; ++y)
#pragma unroll
                for (int z = 0; z < 2; ++z) {
                    acc[x][y][z][0] = acc_t{0, 0, 0, 0};
                    acc[x][y][z][1] = acc_t{0, 0, 0, 0};
                }
        for (int k0 = 0; k0 < cm; k0 += CK) {
            __syncthreads();
            // A: rows R0.., k0..: consecutive threads read consecutive k of a row
            for (int e = tid; e < 2 * CK * BM; e += NTH) {
                const int plane = e / (CK * BM), rem = e - plane * CK * BM;
                const int row = rem / CK, kk = rem - row * CK;
                const int r = R0 + row, c = k0 + kk;
                T v = T(0);
                if (r < m && c < cm) v = (plane ? Ai : Ar)[(size_t)r * cm + c];
                As[plane][kk][row] = v;
            }
            // B: rows c = k0.., columns (j', b) with b fastest
            for (int e = tid; e < 2 * CK * 2 * BN; e += NTH) {
                const int plane = e / (CK * 2 * BN), rem = e - plane * CK * 2 * BN;
                const int kk = rem / (2 * BN), col = rem - kk * (2 * BN);
                const int jp = col / BN, b = B0 + (col - jp * BN);
                const int c = k0 + kk;
                T v = T(0);
                if (c < cm && b < cr) v = (plane ? Bi : Br)[(size_t)c * n + jp * cr + b];
                Bs[plane][kk][col] = v;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < CK / 4; ++ks) {
                const int kk = 4 * ks + (lane >> 4);
                T ar[MT], ai[MT], br[NT2][2], bi[NT2][2];
#pragma unroll
                for (int x = 0; x < MT; ++x) {
                    const int r = wm * WM + x * 16 + a_row<T>(lane);
                    ar[x] = As[0][kk][r];
                    ai[x] = As[1][kk][r];
                }
#pragma unroll
                for (int y = 0; y < NT2; ++y)
#pragma unroll
                    for (int jp = 0; jp < 2; ++jp) {
                        const int c = jp * BN + wn * WN + y * 16 + (lane & 15);
                        br[y][jp] = Bs[0][kk][c];
                        bi[y][jp] = Bs[1][kk][c];
                    }
#pragma unroll
                for (int x = 0; x < MT; ++x)
#pragma unroll
                    for (int y = 0; y < NT2; ++y)
#pragma unroll
                        for (int jp = 0; jp < 2; ++jp) {
                            acc_t& re = acc[x][y][jp][0];
                            acc_t& im = acc[x][y][jp][1];
                            re = Mfma<T>::mac(ar[x], br[y][jp], re);
                            re = Mfma<T>::mac(-ai[x], bi[y][jp], re);
                            im = Mfma<T>::mac(ar[x], bi[y][jp], im);
                            im = Mfma<T>::mac(ai[x], br[y][jp], im);
                        }
            }
        }
        // epilogue: the 4x4 gate on the physical legs, then theta
        T gg[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) gg[q] = static_cast<T>(g[q]);
#pragma unroll
        for (int x = 0; x < MT; ++x)
#pragma unroll
            for (int y = 0; y < NT2; ++y)
#pragma unroll
                for (int rp = 0; rp < 2; ++rp) {
                    // rows 4 (lane / 16) + 2 rp + i' of this 16 x 16 tile
                    const int row0 = R0 + wm * WM + x * 16 + 4 * (lane >> 4) + 2 * rp;
                    const int b = B0 + wn * WN + y * 16 + (lane & 15);
                    if (row0 >= m || b >= cr) continue;
                    T sr[4], si[4];   // S[i'j'] at 2 i' + j'
#pragma unroll
                    for (int ip = 0; ip < 2; ++ip)
#pragma unroll
                        for (int jp = 0; jp < 2; ++jp) {
                            sr[2 * ip + jp] = acc[x][y][jp][0][2 * rp + ip];
                            si[2 * ip + jp] = acc[x][y][jp][1][2 * rp + ip];
                        }
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        T xr = T(0), xi = T(0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const T gr = gg[2 * (4 * o + q)], gi = gg[2 * (4 * o + q) + 1];
                            xr += gr * sr[q] - gi * si[q];
                            xi += gr * si[q] + gi * sr[q];
                        }
                        const int ii = o >> 1, jj = o & 1;
                        const size_t at = (size_t)(row0 + ii) * n + (size_t)jj * cr + b;
                        Th[at] = xr;
                        Th[(size_t)m * n + at] = xi;
                    }
                }
    }
}

// ---------------------------------------------------------------------------
// contraction in BF16x3 split precision (FP32 tensors): each FP32 operand x
// is split into hi = bf16(x) and lo = bf16(x - hi), both rounded to nearest
// even, and a real product is hi hi' + hi lo' + lo hi' with FP32
// accumulation on v_mfma_f32_16x16x32_bf16 (the lo lo' term, ~2^-16
// relative, is dropped).  Operands are staged in LDS k-contiguous ([row][k]
// for A, [column][k] for B) in runs of 8 k that the MFMA reads as one
// 16-byte fragment; the output layout and the gate epilogue are those of the
// FP32 kernel.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int XK = 32;    // k per step (one MFMA)
constexpr int XKP = 40;   // padded k stride in LDS (bf16 elements)

// hi/lo split of 8 consecutive values: hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split8x(const float (&x)[8], uint4& hi, uint4& lo) {
    unsigned h[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x2 v = {x[2 * q], x[2 * q + 1]};
        const unsigned hu = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
        const f32x2 r = {v.x - __uint_as_float(hu << 16), v.y - __uint_as_float(hu & 0xffff0000u)};
        h[q] = hu;
        l[q] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
    }
    hi = make_uint4(h[0], h[1], h[2], h[3]);
    lo = make_uint4(l[0], l[1], l[2], l[3]);
}

template <int WM, int WN>
__global__ __launch_bounds__(NTH) void lx_contract_bf16x3_kernel(LxArgs a, int bucket) {
    constexpr int BM = 2 * WM, BN = 2 * WN;
    constexpr int MT = WM / 16, NT2 = WN / 16;
    // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
    __shared__ __attribute__((aligned(16))) unsigned short As[4][BM][XKP];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[4][2 * BN][XKP];
    const LxBucket* pl = &a.plan->b[bucket];
    const int total = pl->ctiles, cnt = pl->count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    auto frag = [&](const unsigned short* p) { return *reinterpret_cast<const bf16x8*>(p); };
    auto neg = [&](bf16x8 x) {   // both sign bits of each dword at once
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        u32x4 u = __builtin_bit_cast(u32x4, x);
        u ^= 0x80008000u;
        return __builtin_bit_cast(bf16x8, u);
    };
    for (int t0 = xcd_tile(blockIdx.x, gridDim.x); t0 < total; t0 += gridDim.x) {
        const int i = owner(pl->coff, cnt, t0);
        const int slot = pl->slot[i];
        const ShotState& st = a.state[slot];
        const int k = st.k;
        const int cl = st.chi[k], cm = st.chi[k + 1], cr = st.chi[k + 2];
        const int m = 2 * cl, n = 2 * cr;
        const int rtiles = (m + BM - 1) / BM;
        const int tl = t0 - pl->coff[i];
        const int R0 = (tl % rtiles) * BM;
        const int B0 = (tl / rtiles) * BN;
        const float* base = static_cast<const float*>(a.arena) + (size_t)slot * a.slot_stride;
        const float* Ar = base + a.site_off[k];
        const float* Ai = Ar + a.site_half[k];
        const float* Br = base + a.site_off[k + 1];
        const float* Bi = Br + a.site_half[k + 1];
        float* Th = static_cast<float*>(a.theta) + (size_t)slot * a.theta_stride;
        const double* g = a.g4 + st.gate_id * 32;

        floatx4 acc[MT][NT2][2][2];
#pragma unroll
        for (int x = 0; x < MT; ++x)
#pragma unroll
            for (int y = 0; y < NT2; ++y)
#pragma unroll
                for (int z = 0; z < 2; ++z) {
                    acc[x][y][z][0] = floatx4{0.f, 0.f, 0.f, 0.f};
                    acc[x][y][z][1] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
        for (int k0 = 0; k0 < cm; k0 += XK) {
            __syncthreads();
            // A: units (plane, row, run of 8 k)
            for (int u = tid; u < 2 * BM * (XK / 8); u += NTH) {
                const int plane = u / (BM * (XK / 8)), rem = u - plane * BM * (XK / 8);
                const int row = rem / (XK / 8), run = rem - row * (XK / 8);
                const int r = R0 + row;
                const float* src = (plane ? Ai : Ar) + (size_t)r * cm;
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int c = k0 + 8 * run + e;
                    x[e] = (r < m && c < cm) ? src[c] : 0.f;
                }
                uint4 hi, lo;
                split8x(x, hi, lo);
                *reinterpret_cast<uint4*>(&As[2 * plane][row][8 * run]) = hi;
                *reinterpret_cast<uint4*>(&As[2 * plane + 1][row][8 * run]) = lo;
            }
            // B: units (plane, column (j', b), run of 8 k), b fastest
            for (int u = tid; u < 2 * 2 * BN * (XK / 8); u += NTH) {
                const int plane = u / (2 * BN * (XK / 8)), rem = u - plane * 2 * BN * (XK / 8);
                const int run = rem / (2 * BN), col = rem - run * (2 * BN);
                const int jp = col / BN, b = B0 + (col - jp * BN);
                const float* src = (plane ? Bi : Br) + jp * cr + b;
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int c = k0 + 8 * run + e;
                    x[e] = (b < cr && c < cm) ? src[(size_t)c * n] : 0.f;
                }
                uint4 hi, lo;
                split8x(x, hi, lo);
                *reinterpret_cast<uint4*>(&Bs[2 * plane][col][8 * run]) = hi;
                *reinterpret_cast<uint4*>(&Bs[2 * plane + 1][col][8 * run]) = lo;
            }
            __syncthreads();
            const int kk = 8 * (lane >> 4);
            bf16x8 af[MT][6];   // re_hi re_lo im_hi im_lo -im_hi -im_lo
#pragma unroll
            for (int x = 0; x < MT; ++x) {
                const int r = wm * WM + x * 16 + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; ++q) af[x][q] = frag(&As[q][r][kk]);
                af[x][4] = neg(af[x][2]);
                af[x][5] = neg(af[x][3]);
            }
#pragma unroll
            for (int y = 0; y < NT2; ++y)
#pragma unroll
                for (int jp = 0; jp < 2; ++jp) {
                    const int c = jp * BN + wn * WN + y * 16 + (lane & 15);
                    bf16x8 bf[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) bf[q] = frag(&Bs[q][c][kk]);
                    // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br   (each x3)
                    const int ta[6] = {0, 0, 1, 4, 4, 5}, tb[6] = {0, 1, 0, 2, 3, 2};
                    const int ua[6] = {0, 0, 1, 2, 2, 3}, ub[6] = {2, 3, 2, 0, 1, 0};
#pragma unroll
                    for (int q = 0; q < 6; ++q)
#pragma unroll
                        for (int x = 0; x < MT; ++x) {
                            floatx4& re = acc[x][y][jp][0];
                            floatx4& im = acc[x][y][jp][1];
                            re = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[x][ta[q]], bf[tb[q]], re, 0, 0, 0);
                            im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[x][ua[q]], bf[ub[q]], im, 0, 0, 0);
                        }
                }
        }
        float gg[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) gg[q] = static_cast<float>(g[q]);
#pragma unroll
        for (int x = 0; x < MT; ++x)
#pragma unroll
            for (int y = 0; y < NT2; ++y)
#pragma unroll
                for (int rp = 0; rp < 2; ++rp) {
                    const int row0 = R0 + wm * WM + x * 16 + 4 * (lane >> 4) + 2 * rp;
                    const int b = B0 + wn * WN + y * 16 + (lane & 15);
                    if (row0 >= m || b >= cr) continue;
                    float sr[4], si[4];
#pragma unroll
                    for (int ip = 0; ip < 2; ++ip)
#pragma unroll
                        for (int jp = 0; jp < 2; ++jp) {
                            sr[2 * ip + jp] = acc[x][y][jp][0][2 * rp + ip];
                            si[2 * ip + jp] = acc[x][y][jp][1][2 * rp + ip];
                        }
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        float xr = 0.f, xi = 0.f;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float gr = gg[2 * (4 * o + q)], gi = gg[2 * (4 * o + q) + 1];
                            xr += gr * sr[q] - gi * si[q];
                            xi += gr * si[q] + gi * sr[q];
                        }
                        const int ii = o >> 1, jj = o & 1;
                        const size_t at = (size_t)(row0 + ii) * n + (size_t)jj * cr + b;
                        Th[at] = xr;
                        Th[(size_t)m * n + at] = xi;
                    }
                }
    }
}

// ---------------------------------------------------------------------------
// Gram: G[p][q] = sum_e conj(V[e][p]) V[e][q] in FP64, tiles (bp <= bq) of
// BG x BG, 2 x 2 waves of BG/2 x BG/2; V[e][v] = theta[e][v] (columns,
// centre moving right) or theta[v][e] (rows, centre moving left)

constexpr int GK = 16;

template <typename T, int BG>
__global__ __launch_bounds__(NTH) void lx_gram_kernel(LxArgs a, int bucket) {
    constexpr int WG = BG / 2, GT = WG / 16;
    __shared__ double Ps[2][GK][BG];   // [plane][e][p]
    __shared__ double Qs[2][GK][BG];   // [plane][e][q]
    const LxBucket* pl = &a.plan->b[bucket];
    const int total = pl->gtiles, cnt = pl->count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wp = w >> 1, wq = w & 1;
    for (int t0 = xcd_tile(blockIdx.x, gridDim.x); t0 < total; t0 += gridDim.x) {
        const int i = owner(pl->goff, cnt, t0);
        const int slot = pl->slot[i];
        const ShotState& st = a.state[slot];
        const int k = st.k, dir = st.dir;
        const int m = 2 * st.chi[k], n = 2 * st.chi[k + 2];
        const int nv = dir ? n : m, len = dir ? m : n;
        const int nb = (nv + BG - 1) / BG;
        // tile index -> (bp, bq), bp <= bq, row by row of the upper triangle
        int tl = t0 - pl->goff[i], bp = 0, rowlen = nb;
        while (tl >= rowlen) {
            tl -= rowlen;
            ++bp;
            --rowlen;
        }
        const int bq = bp + tl;
        const int P0 = bp * BG, Q0 = bq * BG;
        const T* Tr = static_cast<const T*>(a.theta) + (size_t)slot * a.theta_stride;
        const T* Ti = Tr + (size_t)m * n;
        double* Gr = a.gram + (size_t)slot * a.gram_stride;
        double* Gi = Gr + (size_t)nv * nv;

        doublex4 acc[GT][GT][2];
#pragma unroll
        for (int x = 0; x < GT; ++x)
#pragma unroll
            for (int y = 0; y < GT; ++y) {
                acc[x][y][0] = doublex4{0, 0, 0, 0};
                acc[x][y][1] = doublex4{0, 0, 0, 0};
            }
        for (int e0 = 0; e0 < len; e0 += GK) {
            __syncthreads();
            for (int idx = tid; idx < 2 * 2 * GK * BG; idx += NTH) {
                const int side = idx / (2 * GK * BG), rem0 = idx - side * 2 * GK * BG;
                const int plane = rem0 / (GK * BG), rem = rem0 - plane * GK * BG;
                int e, v;
                if (dir) {   // columns: v fastest (contiguous in a row of theta)
                    e = rem / BG;
                    v = rem - e * BG;
                } else {     // rows: e fastest (contiguous in a row of theta)
                    v = rem / GK;
                    e = rem - v * GK;
                }
                const int vv = (side ? Q0 : P0) + v, ee = e0 + e;
                double x = 0.0;
                if (vv < nv && ee < len) {
                    const size_t at = dir ? (size_t)ee * n + vv : (size_t)vv * n + ee;
                    x = static_cast<double>((plane ? Ti : Tr)[at]);
                }
                (side ? Qs : Ps)[plane][e][v] = x;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < GK / 4; ++ks) {
                const int e = 4 * ks + (lane >> 4);
                double pr[GT], pi[GT], qr[GT], qi[GT];
#pragma unroll
                for (int x = 0; x < GT; ++x) {
                    const int p = wp * WG + x * 16 + a_row<double>(lane);
                    pr[x] = Ps[0][e][p];
                    pi[x] = Ps[1][e][p];
                    const int q = wq * WG + x * 16 + (lane & 15);
                    qr[x] = Qs[0][e][q];
                    qi[x] = Qs[1][e][q];
                }
                // Re += pr qr + pi qi ; Im += pr qi - pi qr   (conj on p)
#pragma unroll
                for (int x = 0; x < GT; ++x)
#pragma unroll
                    for (int y = 0; y < GT; ++y) {
                        doublex4& re = acc[x][y][0];
                        doublex4& im = acc[x][y][1];
                        re = __builtin_amdgcn_mfma_f64_16x16x4f64(pr[x], qr[y], re, 0, 0, 0);
                        re = __builtin_amdgcn_mfma_f64_16x16x4f64(pi[x], qi[y], re, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f64_16x16x4f64(pr[x], qi[y], im, 0, 0, 0);
                        im = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi[x], qr[y], im, 0, 0, 0);
                    }
            }
        }
#pragma unroll
        for (int x = 0; x < GT; ++x)
#pragma unroll
            for (int y = 0; y < GT; ++y) {
                const int q = Q0 + wq * WG + y * 16 + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int p = P0 + wp * WG + x * 16 + 4 * (lane >> 4) + r;
                    if (p < nv && q < nv) {
                        Gr[(size_t)p * nv + q] = acc[x][y][0][r];
                        Gi[(size_t)p * nv + q] = acc[x][y][1][r];
                    }
                }
            }
    }
}

template <typename T>
hipError_t launch_contract_t(const LxArgs& a, int bucket, const LxTiles& t, int grid,
                             hipStream_t s) {
#define MSC_LX_CASE(WM, WN)                                                                 \
    if (t.cm_rows == 2 * (WM) && t.cm_b == 2 * (WN)) {                                      \
        hipLaunchKernelGGL((lx_contract_kernel<T, WM, WN>), dim3(grid), dim3(NTH), 0, s, a,  \
                           bucket);                                                         \
        return hipGetLastError();                                                           \
    }
    MSC_LX_CASE(16, 16)
    MSC_LX_CASE(32, 16)
    MSC_LX_CASE(32, 32)
    if constexpr (sizeof(T) == sizeof(float)) {
        MSC_LX_CASE(64, 32)
    }
#undef MSC_LX_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_gram_t(const LxArgs& a, int bucket, const LxTiles& t, int grid,
                         hipStream_t s) {
    if (t.gram == 32) {
        hipLaunchKernelGGL((lx_gram_kernel<T, 32>), dim3(grid), dim3(NTH), 0, s, a, bucket);
    } else if (t.gram == 64) {
        hipLaunchKernelGGL((lx_gram_kernel<T, 64>), dim3(grid), dim3(NTH), 0, s, a, bucket);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lx_plan(const LxArgs& a, const LxTiles* t, hipStream_t s) {
    Tiles4 tt;
    for (int b = 0; b < kLxBuckets; ++b) {
        if (t[b].cm_rows <= 0 || t[b].cm_b <= 0 || t[b].gram <= 0) return hipErrorInvalidValue;
        tt.t[b] = t[b];
    }
    hipLaunchKernelGGL(lx_plan_kernel, dim3(1), dim3(PLAN_T), 0, s, a, tt);
    return hipGetLastError();
}

hipError_t launch_lx_contract(int precision, const LxArgs& a, int bucket, const LxTiles& t,
                              int grid, hipStream_t s) {
    if (bucket < 0 || bucket >= kLxBuckets) return hipErrorInvalidValue;
    if (precision == MSC_FP64) return launch_contract_t<double>(a, bucket, t, grid, s);
    if (precision == MSC_BF16X3) {
#define MSC_LX_BF(WM, WN)                                                                  \
        if (t.cm_rows == 2 * (WM) && t.cm_b == 2 * (WN)) {                                  \
            hipLaunchKernelGGL((lx_contract_bf16x3_kernel<WM, WN>), dim3(grid), dim3(NTH), 0, \
                               s, a, bucket);                                              \
            return hipGetLastError();                                                      \
        }
        MSC_LX_BF(16, 16)
        MSC_LX_BF(32, 16)
        MSC_LX_BF(32, 32)
#undef MSC_LX_BF
        return hipErrorInvalidValue;
    }
    return launch_contract_t<float>(a, bucket, t, grid, s);
}

hipError_t launch_lx_gram(int precision, const LxArgs& a, int bucket, const LxTiles& t,
                          int grid, hipStream_t s) {
    if (bucket < 0 || bucket >= kLxBuckets) return hipErrorInvalidValue;
    if (precision == MSC_FP64) return launch_gram_t<double>(a, bucket, t, grid, s);
    return launch_gram_t<float>(a, bucket, t, grid, s);
}

hipError_t launch_lx_reset(ShotState* state, int n_slots, int32_t* park_count, double* flops,
                           unsigned long long* counts, hipStream_t s) {
    const int g = (n_slots + 255) / 256;
    hipLaunchKernelGGL(lx_reset_kernel, dim3(g > 0 ? g : 1), dim3(256), 0, s, state, n_slots,
                       park_count, flops, counts);
    return hipGetLastError();
}

hipError_t launch_lx_clear(int32_t* park_count, hipStream_t s) {
    hipLaunchKernelGGL(lx_clear_kernel, dim3(1), dim3(1), 0, s, park_count);
    return hipGetLastError();
}

int lx_tile_variants(int precision, LxTiles* out, int cap) {
    static const LxTiles f32[] = {{64, 32, 64}, {32, 32, 64}, {64, 64, 64}, {128, 64, 64},
                                  {64, 32, 32}, {32, 32, 32}};
    static const LxTiles f64[] = {{32, 32, 32}, {64, 32, 64}, {64, 64, 64}, {32, 32, 64}};
    static const LxTiles bf[] = {{64, 64, 64}, {64, 32, 64}, {32, 32, 64}, {64, 64, 32}};
    const LxTiles* v = precision == MSC_FP64 ? f64 : precision == MSC_BF16X3 ? bf : f32;
    const int nv = precision == MSC_FP64 ? 4 : precision == MSC_BF16X3 ? 4 : 6;
    for (int i = 0; i < nv && i < cap; ++i) out[i] = v[i];
    return nv;
}

}  // namespace msc
