// CAMPS shots (section "Clifford augmented MPS"): the state is C|m> with C a
// Clifford frame and |m> the magic residual, an MPS in FP64.
//
// The frame is held as the images of the single-qubit Paulis, C^dag X_q C
// and C^dag Z_q C for every qubit q: Pauli strings over the residual's
// sites, each i^ph X^x Z^z with bit vectors x, z and ph mod 4.  A Clifford
// gate G (C <- G C) rewrites the images of the qubits it acts on from the
// old ones; a Pauli fault or a reset's X only flips signs.  A T^(+-1) on q
// applies exp(-+ i pi/8 R) = cos(pi/8) I -+ i sin(pi/8) R to |m> with
// R = C^dag Z_q C; a measurement of q with expected outcome e projects |m>
// with (I + (-1)^e R)/2 after p(e) = (1 + (-1)^e <R>)/2.  Applying
// a I + b R to the MPS: over the sites lo..hi where R acts, the MPS of the
// sum has block tensors [a A | b' O A], diag(A, O A), [A ; O A] (O the
// per-site Pauli, b' = b i^ph); it is compressed by one left-to-right SVD
// sweep and one right-to-left sweep that keeps singular values above
// tau * sigma_max (the exact regime).  Then one greedy disentangling sweep
// over the bonds max(lo-1, 0) .. min(hi, n-2): for each bond, the purity
// tr(rho^2) of D theta across it for every candidate two-qubit Clifford D
// (one per class modulo local Cliffords); the best one, if it beats the
// current purity by more than a relative 1e-9 (earlier candidates win
// ties), is applied to the residual and its inverse to the frame; the bond
// is then split by SVD.  One-site operators change no bond and get no
// sweep.  The seed's Bloch vector gives the fidelity.
//
// One 256-thread workgroup per shot, persistent over the shot list.  The
// frame lives in LDS; site tensors (capacity kCampsK per bond, dense in
// their actual dims) and work matrices in the slot's global memory.  SVDs
// are one-sided Jacobi with the pairs of a round processed in parallel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

constexpr int CT = 256;
constexpr int K = kCampsK;
constexpr int NR = 2 * kMaxSites;
constexpr int kMaxSweeps = 60;

// scratch layout (doubles) of one slot
constexpr int64_t oW = 0;                     // 2 x (2K x K), column-major, ld 2K
constexpr int64_t oV = oW + 4LL * K * K;      // 2 x (K x K), column-major, ld K
constexpr int64_t oC = oV + 2LL * K * K;      // carry, 2 x (K x K) row-major, ld K
constexpr int64_t oF = oC + 2LL * K * K;      // 2 x 2K^2
constexpr int64_t oE = oF + 4LL * K * K;      // 2 x K^2
constexpr int64_t oE2 = oE + 2LL * K * K;     // 2 x K^2
constexpr int64_t oTH = oE2 + 2LL * K * K;    // 2 x 2K^2
constexpr int64_t oTC = oTH + 4LL * K * K;    // 2 x K^2
static_assert(oTC + 2LL * K * K <= kCampsScratch, "scratch layout");

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < CT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < CT / 64; ++w) s = fmax(s, red[w]);
    __syncthreads();
    return s;
}

struct Frame {
    uint64_t* x;   // [NR][2]
    uint64_t* z;   // [NR][2]
    uint8_t* ph;   // [NR]
};

__device__ __forceinline__ int getbit(const uint64_t* w, int s) { return (w[s >> 6] >> (s & 63)) & 1; }

// row r <- i^add (row a)(row b)  (single thread)
__device__ void row_prod(Frame F, int r, int a, int b, int add) {
    const uint64_t xa0 = F.x[2 * a], xa1 = F.x[2 * a + 1], za0 = F.z[2 * a], za1 = F.z[2 * a + 1];
    const uint64_t xb0 = F.x[2 * b], xb1 = F.x[2 * b + 1], zb0 = F.z[2 * b], zb1 = F.z[2 * b + 1];
    const int ph = F.ph[a] + F.ph[b] + add + 2 * (__popcll(za0 & xb0) + __popcll(za1 & xb1));
    F.x[2 * r] = xa0 ^ xb0;
    F.x[2 * r + 1] = xa1 ^ xb1;
    F.z[2 * r] = za0 ^ zb0;
    F.z[2 * r + 1] = za1 ^ zb1;
    F.ph[r] = static_cast<uint8_t>(ph & 3);
}

__device__ void row_copy(Frame F, int r, int a) {
    F.x[2 * r] = F.x[2 * a];
    F.x[2 * r + 1] = F.x[2 * a + 1];
    F.z[2 * r] = F.z[2 * a];
    F.z[2 * r + 1] = F.z[2 * a + 1];
    F.ph[r] = F.ph[a];
}

// Per-slot view: residual sites and scratch, bond dims in LDS.
struct Res {
    double* arena;        // n sites x kCampsSiteDoubles
    double* scr;
    int* chi;             // LDS [n + 1]
    int n;
    __device__ double* re(int k) const { return arena + static_cast<int64_t>(k) * kCampsSiteDoubles; }
    __device__ double* im(int k) const { return re(k) + 2LL * K * K; }
};

// Pauli O = X^x Z^z on the physical index: (O A)[a, i, b] = (-1)^(z (i^x)) A[a, i^x, b]
__device__ __forceinline__ void pauli_elem(int x, int z, int i, int& src, double& sg) {
    src = i ^ x;
    sg = (z && src) ? -1.0 : 1.0;
}

// Work matrices of one SVD: W (len x nv, column-major, leading dimension
// ldw) and V (nv x nv, column-major, ldv), in LDS when they fit (len <=
// kWaveLen, nv <= kWaveCols: one wavefront factorises them without
// workgroup barriers) and otherwise in the slot's global scratch.
constexpr int kWaveLen = 64, kWaveCols = 32;
struct WV {
    double *wr, *wi, *vr, *vi;
    int ldw, ldv;
    bool wave;
};

// a fence that makes this wavefront's LDS and global writes visible to all
// of its lanes, without a workgroup barrier
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// one Jacobi rotation of the pair (p, q) by a group of G lanes (lane l):
// returns whether it rotated
__device__ __forceinline__ bool jacobi_pair(const WV& w, int len, int nv, int p, int q, int G,
                                            int l) {
    const bool live = p < nv && q < nv;
    double a = 0, b = 0, gr = 0, gi = 0;
    if (live) {
        const double *xr = w.wr + p * w.ldw, *xi = w.wi + p * w.ldw;
        const double *yr = w.wr + q * w.ldw, *yi = w.wi + q * w.ldw;
        for (int r = l; r < len; r += G) {
            a += xr[r] * xr[r] + xi[r] * xi[r];
            b += yr[r] * yr[r] + yi[r] * yi[r];
            // gamma = x^H y
            gr += xr[r] * yr[r] + xi[r] * yi[r];
            gi += xr[r] * yi[r] - xi[r] * yr[r];
        }
    }
    for (int o = G / 2; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
        gr += __shfl_xor(gr, o);
        gi += __shfl_xor(gi, o);
    }
    const double gm = sqrt(gr * gr + gi * gi);
    if (!(live && a > 1e-300 && b > 1e-300 && gm > 1e-15 * sqrt(a * b))) return false;
    const double d = b - a;
    const double D = fabs(d) + sqrt(d * d + 4.0 * gm * gm);
    const double rq = 1.0 / sqrt(D * D + 4.0 * gm * gm);
    const double c = D * rq;
    const double sg = 2.0 * (d >= 0.0 ? 1.0 : -1.0) * rq;
    // x <- c x - sg conj(gamma) y ; y <- c y + sg gamma x
    const double ur = sg * gr, ui = sg * gi;
    auto rot = [&](double* xr, double* xi, double* yr, double* yi, int r) {
        const double x0r = xr[r], x0i = xi[r], y0r = yr[r], y0i = yi[r];
        xr[r] = c * x0r - (ur * y0r + ui * y0i);
        xi[r] = c * x0i - (ur * y0i - ui * y0r);
        yr[r] = c * y0r + (ur * x0r - ui * x0i);
        yi[r] = c * y0i + (ur * x0i + ui * x0r);
    };
    for (int r = l; r < len; r += G)
        rot(w.wr + p * w.ldw, w.wi + p * w.ldw, w.wr + q * w.ldw, w.wi + q * w.ldw, r);
    for (int r = l; r < nv; r += G) rot(w.vr + p * w.ldv, w.vi + p * w.ldv, w.vr + q * w.ldv, w.vi + q * w.ldv, r);
    return true;
}

// pair i of round t of the round-robin over m (even) columns
__device__ __forceinline__ void rr_pair(int i, int t, int m, int& p, int& q) {
    const int i1 = m - 1 - i;
    p = i == 0 ? 0 : 1 + (i - 1 + t) % (m - 1);
    q = i1 == 0 ? 0 : 1 + (i1 - 1 + t) % (m - 1);
}

// One-sided Jacobi on the columns of W: W <- W V with V unitary and the
// columns of the result mutually orthogonal.  Whole workgroup; the LDS
// variant runs on wavefront 0 alone.  Returns the sweeps used (-1: no
// convergence).
__device__ int jacobi_cols(const WV& w, int len, int nv, int* s_flag) {
    const int tid = threadIdx.x;
    if (w.wave) {
        __shared__ int s_sw;
        if (tid < 64) {
            for (int e = tid; e < nv * nv; e += 64) {
                const int col = e / nv, row = e - col * nv;
                w.vr[col * w.ldv + row] = row == col ? 1.0 : 0.0;
                w.vi[col * w.ldv + row] = 0.0;
            }
            wave_sync();
            int used = 0;
            if (nv >= 2) {
                const int m = nv + (nv & 1), np = m / 2;
                int G = 64;
                while (G > 1 && G * np > 64) G >>= 1;
                const int g = tid / G, l = tid - g * G;
                used = -1;
                for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
                    int rotated = 0;
                    for (int t = 0; t < m - 1; ++t) {
                        if (g < np) {
                            int p, q;
                            rr_pair(g, t, m, p, q);
                            if (jacobi_pair(w, len, nv, p, q, G, l)) rotated = 1;
                        }
                        wave_sync();
                    }
                    if (__ballot(rotated) == 0ull) {
                        used = sweep + 1;
                        break;
                    }
                }
            }
            if (tid == 0) s_sw = used;
        }
        __syncthreads();
        const int used = s_sw;
        __syncthreads();
        return used;
    }
    for (int e = tid; e < nv * nv; e += CT) {
        const int col = e / nv, row = e - col * nv;
        w.vr[col * w.ldv + row] = row == col ? 1.0 : 0.0;
        w.vi[col * w.ldv + row] = 0.0;
    }
    __syncthreads();
    if (nv < 2) return 0;
    const int m = nv + (nv & 1);
    const int np = m / 2;
    int G = 64;
    while (G > 1 && G * np > CT) G >>= 1;
    const int g = tid / G, l = tid - g * G;
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) *s_flag = 0;
        __syncthreads();
        for (int t = 0; t < m - 1; ++t) {
            if (g < np) {
                int p, q;
                rr_pair(g, t, m, p, q);
                if (jacobi_pair(w, len, nv, p, q, G, l) && l == 0) *s_flag = 1;
            }
            __syncthreads();
        }
        const int changed = *s_flag;
        __syncthreads();
        if (!changed) return sweep + 1;
    }
    return -1;
}

// column norms of W (nv columns) into sg[], kept columns (sigma > tau *
// sigma_max, in order) into keep[]; returns how many
__device__ int select_cols(const WV& w, int len, int nv, double tau, double* sg, int* keep,
                           double* red) {
    const int tid = threadIdx.x;
    for (int col = tid; col < nv; col += CT) {
        double s = 0;
        for (int r = 0; r < len; ++r) {
            const double a = w.wr[col * w.ldw + r];
            const double b = w.wi[col * w.ldw + r];
            s += a * a + b * b;
        }
        sg[col] = sqrt(s);
    }
    __syncthreads();
    double mx = 0;
    for (int col = tid; col < nv; col += CT) mx = fmax(mx, sg[col]);
    mx = block_max(mx, red);
    __shared__ int s_cnt;
    if (tid == 0) {
        int r = 0;
        for (int col = 0; col < nv; ++col)
            if (sg[col] > tau * mx && sg[col] > 0.0) keep[r++] = col;
        s_cnt = r;
    }
    __syncthreads();
    const int r = s_cnt;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// centre moves: the centre site's matrix split by SVD, truncated at tau
struct Ctl {
    double* red;      // LDS reductions
    int* flag;        // LDS
    double* sg;       // LDS [K]
    int* keep;        // LDS [K]
    int* center;      // LDS
    int* status;      // LDS: shot status bits
    int* sweeps;      // LDS: Jacobi sweeps
    int* chi_peak;    // LDS
    int* old;         // LDS [kMaxSites + 1]: bonds before apply_sum
    double *lwr, *lwi, *lvr, *lvi;   // LDS work matrices of the wave SVDs
};

__device__ __forceinline__ WV work_mats(const Res& R, const Ctl& c, int len, int nv) {
    WV w;
    if (len <= kWaveLen && nv <= kWaveCols) {
        w.wr = c.lwr;
        w.wi = c.lwi;
        w.vr = c.lvr;
        w.vi = c.lvi;
        w.ldw = kWaveLen;
        w.ldv = kWaveCols;
        w.wave = true;
    } else {
        w.wr = R.scr + oW;
        w.wi = w.wr + 2LL * K * K;
        w.vr = R.scr + oV;
        w.vi = w.vr + K * K;
        w.ldw = 2 * K;
        w.ldv = K;
        w.wave = false;
    }
    return w;
}

__device__ void note_sweeps(const Ctl& c, int sw) {
    if (threadIdx.x == 0) {
        if (sw < 0) *c.status |= MSC_SHOT_NOCONV;
        else *c.sweeps += sw;
    }
}

// centre k -> k+1
__device__ void move_right(const Res& R, const Ctl& c, int k, double tau) {
    const int tid = threadIdx.x;
    const int cl = R.chi[k], cr = R.chi[k + 1], cn = R.chi[k + 2];
    const double *ar = R.re(k), *ai = R.im(k);
    const int len = 2 * cl;
    const WV w = work_mats(R, c, len, cr);
    double *wr = w.wr, *wi = w.wi, *vr = w.vr, *vi = w.vi;
    const int ldw = w.ldw, ldv = w.ldv;
    for (int e = tid; e < len * cr; e += CT) {
        const int row = e / cr, b = e - row * cr;
        wr[b * ldw + row] = ar[row * cr + b];
        wi[b * ldw + row] = ai[row * cr + b];
    }
    __syncthreads();
    note_sweeps(c, jacobi_cols(w, len, cr, c.flag));
    const int r = select_cols(w, len, cr, tau, c.sg, c.keep, c.red);
    double *Ar = R.re(k), *Ai = R.im(k);
    for (int e = tid; e < len * r; e += CT) {
        const int row = e / r, j = e - row * r;
        const int col = c.keep[j];
        const double s = 1.0 / c.sg[col];
        Ar[row * r + j] = wr[col * ldw + row] * s;
        Ai[row * r + j] = wi[col * ldw + row] * s;
    }
    // next site: (S V^dag) A_{k+1}, via TH
    double *tr = R.scr + oTH, *ti = tr + 2LL * K * K;
    const double *br = R.re(k + 1), *bi = R.im(k + 1);
    const int nb = 2 * cn;
    for (int e = tid; e < r * nb; e += CT) {
        const int j = e / nb, col2 = e - j * nb;
        const int col = c.keep[j];
        const double s = c.sg[col];
        double xr = 0, xi = 0;
        for (int b = 0; b < cr; ++b) {
            // conj(V[b][col]) * A[b][col2]
            const double v_r = vr[col * ldv + b], v_i = -vi[col * ldv + b];
            const double a_r = br[b * nb + col2], a_i = bi[b * nb + col2];
            xr += v_r * a_r - v_i * a_i;
            xi += v_r * a_i + v_i * a_r;
        }
        tr[e] = s * xr;
        ti[e] = s * xi;
    }
    __syncthreads();
    double *Br = R.re(k + 1), *Bi = R.im(k + 1);
    for (int e = tid; e < r * nb; e += CT) {
        Br[e] = tr[e];
        Bi[e] = ti[e];
    }
    if (tid == 0) {
        R.chi[k + 1] = r;
        *c.center = k + 1;
        if (r > *c.chi_peak) *c.chi_peak = r;
    }
    __syncthreads();
}

// centre k -> k-1
__device__ void move_left(const Res& R, const Ctl& c, int k, double tau) {
    const int tid = threadIdx.x;
    const int cp = R.chi[k - 1], cl = R.chi[k], cr = R.chi[k + 1];
    const double *ar = R.re(k), *ai = R.im(k);
    const int len = 2 * cr;
    const WV w = work_mats(R, c, len, cl);
    double *wr = w.wr, *wi = w.wi, *vr = w.vr, *vi = w.vi;
    const int ldw = w.ldw, ldv = w.ldv;
    // W = A^dag: column a holds conj(A[a, :])
    for (int e = tid; e < cl * len; e += CT) {
        const int a = e / len, x = e - a * len;
        wr[a * ldw + x] = ar[a * len + x];
        wi[a * ldw + x] = -ai[a * len + x];
    }
    __syncthreads();
    note_sweeps(c, jacobi_cols(w, len, cl, c.flag));
    const int r = select_cols(w, len, cl, tau, c.sg, c.keep, c.red);
    double *Ar = R.re(k), *Ai = R.im(k);
    for (int e = tid; e < r * len; e += CT) {
        const int j = e / len, x = e - j * len;
        const int col = c.keep[j];
        const double s = 1.0 / c.sg[col];
        Ar[j * len + x] = wr[col * ldw + x] * s;
        Ai[j * len + x] = -wi[col * ldw + x] * s;
    }
    // previous site: A_{k-1} (V S)
    double *tr = R.scr + oTH, *ti = tr + 2LL * K * K;
    const double *pr = R.re(k - 1), *pi = R.im(k - 1);
    const int rows = 2 * cp;
    for (int e = tid; e < rows * r; e += CT) {
        const int row = e / r, j = e - row * r;
        const int col = c.keep[j];
        const double s = c.sg[col];
        double xr = 0, xi = 0;
        for (int a = 0; a < cl; ++a) {
            const double p_r = pr[row * cl + a], p_i = pi[row * cl + a];
            const double v_r = vr[col * ldv + a], v_i = vi[col * ldv + a];
            xr += p_r * v_r - p_i * v_i;
            xi += p_r * v_i + p_i * v_r;
        }
        tr[e] = s * xr;
        ti[e] = s * xi;
    }
    __syncthreads();
    double *Pr = R.re(k - 1), *Pi = R.im(k - 1);
    for (int e = tid; e < rows * r; e += CT) {
        Pr[e] = tr[e];
        Pi[e] = ti[e];
    }
    if (tid == 0) {
        R.chi[k] = r;
        *c.center = k - 1;
        if (r > *c.chi_peak) *c.chi_peak = r;
    }
    __syncthreads();
}

__device__ void move_center(const Res& R, const Ctl& c, int to, double tau) {
    while (*c.center < to) move_right(R, c, *c.center, tau);
    while (*c.center > to) move_left(R, c, *c.center, tau);
}

// support of row r: first and last site (lo = -1 if empty)
__device__ void support(Frame F, int r, int n, int& lo, int& hi) {
    lo = -1;
    hi = -1;
    for (int w = 0; w < 2; ++w) {
        const uint64_t m = F.x[2 * r + w] | F.z[2 * r + w];
        if (!m) continue;
        const int a = w * 64 + __ffsll(static_cast<long long>(m)) - 1;
        const int b = w * 64 + 63 - __clzll(static_cast<long long>(m));
        if (lo < 0) lo = a;
        hi = b;
    }
    if (hi >= n) hi = n - 1;
}

// <m| R |m> for the row r (real part; R Hermitian)
__device__ double expect(const Res& R, const Ctl& c, Frame F, int r, double tau) {
    int lo, hi;
    support(F, r, R.n, lo, hi);
    const int tid = threadIdx.x;
    if (lo < 0) {
        const int ph = F.ph[r];
        return ph == 0 ? 1.0 : (ph == 2 ? -1.0 : 0.0);
    }
    move_center(R, c, lo, tau);
    double *er = R.scr + oE, *ei = er + K * K;
    double *e2r = R.scr + oE2, *e2i = e2r + K * K;
    double *fr = R.scr + oF, *fi = fr + 2LL * K * K;
    const int c0 = R.chi[lo];
    for (int e = tid; e < c0 * c0; e += CT) {
        er[e] = (e / c0 == e % c0) ? 1.0 : 0.0;
        ei[e] = 0.0;
    }
    __syncthreads();
    for (int k = lo; k <= hi; ++k) {
        const int cl = R.chi[k], cr = R.chi[k + 1];
        const int x = getbit(F.x + 2 * r, k), z = getbit(F.z + 2 * r, k);
        const double *ar = R.re(k), *ai = R.im(k);
        // F[a][i][b'] = sum_a' E[a][a'] (O A)[a'][i][b']
        for (int e = tid; e < cl * 2 * cr; e += CT) {
            const int a = e / (2 * cr), rem = e - a * 2 * cr, i = rem / cr, b = rem - i * cr;
            int src;
            double s;
            pauli_elem(x, z, i, src, s);
            double xr = 0, xi = 0;
            for (int a2 = 0; a2 < cl; ++a2) {
                const double Er = er[a * cl + a2], Ei = ei[a * cl + a2];
                const double Or = s * ar[(a2 * 2 + src) * cr + b], Oi = s * ai[(a2 * 2 + src) * cr + b];
                xr += Er * Or - Ei * Oi;
                xi += Er * Oi + Ei * Or;
            }
            fr[e] = xr;
            fi[e] = xi;
        }
        __syncthreads();
        // E'[b][b'] = sum_{a,i} conj(A[a][i][b]) F[a][i][b']
        for (int e = tid; e < cr * cr; e += CT) {
            const int b = e / cr, b2 = e - b * cr;
            double xr = 0, xi = 0;
            for (int a = 0; a < cl; ++a)
                for (int i = 0; i < 2; ++i) {
                    const double Ar = ar[(a * 2 + i) * cr + b], Ai = -ai[(a * 2 + i) * cr + b];
                    const double Fr = fr[(a * 2 + i) * cr + b2], Fi = fi[(a * 2 + i) * cr + b2];
                    xr += Ar * Fr - Ai * Fi;
                    xi += Ar * Fi + Ai * Fr;
                }
            e2r[e] = xr;
            e2i[e] = xi;
        }
        __syncthreads();
        for (int e = tid; e < cr * cr; e += CT) {
            er[e] = e2r[e];
            ei[e] = e2i[e];
        }
        __syncthreads();
    }
    const int cn = R.chi[hi + 1];
    double tr = 0, ti = 0;
    for (int b = tid; b < cn; b += CT) {
        tr += er[b * cn + b];
        ti += ei[b * cn + b];
    }
    tr = block_sum(tr, c.red);
    ti = block_sum(ti, c.red);
    // times i^ph
    const int ph = F.ph[r];
    return ph == 0 ? tr : ph == 1 ? -ti : ph == 2 ? -tr : ti;
}

// |m> <- al |m> + be i^ph O |m> for row r; returns false if a bond would
// exceed the cap (the shot is then flagged)
__device__ bool apply_sum(const Res& R, const Ctl& c, Frame F, int r, double alr, double ali,
                          double ber, double bei, double tau, int cap, int& lo_out, int& hi_out) {
    int lo, hi;
    support(F, r, R.n, lo, hi);
    lo_out = lo;
    hi_out = hi;
    const int tid = threadIdx.x;
    const int ph = F.ph[r];
    // b' = be i^ph
    double bpr = ber, bpi = bei;
    for (int t = 0; t < ph; ++t) {
        const double nr = -bpi, ni = bpr;
        bpr = nr;
        bpi = ni;
    }
    if (lo < 0) {
        // R = i^ph I: a global factor (al + b') on the centre site
        const int k = *c.center;
        const int ne = R.chi[k] * 2 * R.chi[k + 1];
        const double fr = alr + bpr, fi = ali + bpi;
        double *Ar = R.re(k), *Ai = R.im(k);
        for (int e = tid; e < ne; e += CT) {
            const double a = Ar[e], b = Ai[e];
            Ar[e] = fr * a - fi * b;
            Ai[e] = fr * b + fi * a;
        }
        __syncthreads();
        return true;
    }
    move_center(R, c, lo, tau);
    for (int k = lo + tid; k <= hi + 1; k += CT) c.old[k] = R.chi[k];
    __syncthreads();
    double *cr_ = R.scr + oC, *ci_ = cr_ + K * K;
    double *tr = R.scr + oTH, *ti = tr + 2LL * K * K;
    if (lo == hi) {
        const int k = lo, cl = R.chi[k], cr = R.chi[k + 1];
        const int x = getbit(F.x + 2 * r, k), z = getbit(F.z + 2 * r, k);
        const double *ar = R.re(k), *ai = R.im(k);
        for (int e = tid; e < cl * 2 * cr; e += CT) {
            const int a = e / (2 * cr), rem = e - a * 2 * cr, i = rem / cr, b = rem - i * cr;
            int src;
            double s;
            pauli_elem(x, z, i, src, s);
            const double Or = s * ar[(a * 2 + src) * cr + b], Oi = s * ai[(a * 2 + src) * cr + b];
            tr[e] = alr * ar[e] - ali * ai[e] + bpr * Or - bpi * Oi;
            ti[e] = alr * ai[e] + ali * ar[e] + bpr * Oi + bpi * Or;
        }
        __syncthreads();
        double *Ar = R.re(k), *Ai = R.im(k);
        for (int e = tid; e < cl * 2 * cr; e += CT) {
            Ar[e] = tr[e];
            Ai[e] = ti[e];
        }
        __syncthreads();
        return true;
    }
    // left-to-right over lo..hi with the carry matrix (rows = kept left
    // rank, columns = the sum MPS's left bond at the next site)
    int rows = R.chi[lo];              // left rank (unchanged left of lo)
    for (int k = lo; k <= hi; ++k) {
        const int cl = c.old[k], cr = c.old[k + 1];   // dims of the original tensor
        const int x = getbit(F.x + 2 * r, k), z = getbit(F.z + 2 * r, k);
        const double *ar = R.re(k), *ai = R.im(k);
        const int D = k == hi ? cr : 2 * cr;          // right bond of the sum tensor
        const int len = 2 * rows;
        const WV w = work_mats(R, c, len, D);
        double *wr = w.wr, *wi = w.wi, *vr = w.vr, *vi = w.vi;
        const int ldw = w.ldw, ldv = w.ldv;
        // M[(j,i)][col] into W (column-major) or, at the last site, TH
        for (int e = tid; e < len * D; e += CT) {
            const int row = e / D, col = e - row * D;
            const int j = row >> 1, i = row & 1;
            const bool second = k != hi && col >= cr;
            const int b = second ? col - cr : col;
            int src;
            double s;
            pauli_elem(x, z, i, src, s);
            double xr = 0, xi = 0;
            if (k == lo) {
                // S_lo = [al A | b' O A]; the carry is the identity
                if (!second) {
                    const double a_r = ar[(j * 2 + i) * cr + b], a_i = ai[(j * 2 + i) * cr + b];
                    xr = alr * a_r - ali * a_i;
                    xi = alr * a_i + ali * a_r;
                    if (k == hi) {
                        const double o_r = s * ar[(j * 2 + src) * cr + b], o_i = s * ai[(j * 2 + src) * cr + b];
                        xr += bpr * o_r - bpi * o_i;
                        xi += bpr * o_i + bpi * o_r;
                    }
                } else {
                    const double o_r = s * ar[(j * 2 + src) * cr + b], o_i = s * ai[(j * 2 + src) * cr + b];
                    xr = bpr * o_r - bpi * o_i;
                    xi = bpr * o_i + bpi * o_r;
                }
            } else {
                // carry (rows x 2 cl): first cl columns meet A, last cl meet O A
                const bool lower = k == hi;     // S_hi = [A ; O A]
                for (int u = 0; u < cl; ++u) {
                    if (lower || !second) {
                        const double c_r = cr_[j * K + u], c_i = ci_[j * K + u];
                        const double a_r = ar[(u * 2 + i) * cr + b], a_i = ai[(u * 2 + i) * cr + b];
                        xr += c_r * a_r - c_i * a_i;
                        xi += c_r * a_i + c_i * a_r;
                    }
                    if (lower || second) {
                        const double c_r = cr_[j * K + cl + u], c_i = ci_[j * K + cl + u];
                        const double o_r = s * ar[(u * 2 + src) * cr + b], o_i = s * ai[(u * 2 + src) * cr + b];
                        xr += c_r * o_r - c_i * o_i;
                        xi += c_r * o_i + c_i * o_r;
                    }
                }
            }
            if (k == hi) {
                tr[e] = xr;
                ti[e] = xi;
            } else {
                wr[col * ldw + row] = xr;
                wi[col * ldw + row] = xi;
            }
        }
        __syncthreads();
        if (k == hi) {
            double *Ar = R.re(k), *Ai = R.im(k);
            for (int e = tid; e < len * D; e += CT) {
                Ar[e] = tr[e];
                Ai[e] = ti[e];
            }
            if (tid == 0) {
                R.chi[k] = rows;
                *c.center = hi;
            }
            __syncthreads();
            break;
        }
        note_sweeps(c, jacobi_cols(w, len, D, c.flag));
        const int rn = select_cols(w, len, D, 1e-14, c.sg, c.keep, c.red);
        if (rn > K) return false;     // cannot happen: rn <= D <= K
        double *Ar = R.re(k), *Ai = R.im(k);
        for (int e = tid; e < len * rn; e += CT) {
            const int row = e / rn, jj = e - row * rn;
            const int col = c.keep[jj];
            const double s = 1.0 / c.sg[col];
            Ar[row * rn + jj] = wr[col * ldw + row] * s;
            Ai[row * rn + jj] = wi[col * ldw + row] * s;
        }
        // new carry: S V^dag (rn x D)
        for (int e = tid; e < rn * D; e += CT) {
            const int jj = e / D, col2 = e - jj * D;
            const int col = c.keep[jj];
            cr_[jj * K + col2] = c.sg[col] * vr[col * ldv + col2];
            ci_[jj * K + col2] = -c.sg[col] * vi[col * ldv + col2];
        }
        if (tid == 0) {
            R.chi[k] = rows;
            R.chi[k + 1] = rn;
        }
        __syncthreads();
        rows = rn;
    }
    // right-to-left: true Schmidt values now, truncate at tau
    for (int k = hi; k > lo; --k) move_left(R, c, k, tau);
    for (int k = lo + 1; k <= hi; ++k)
        if (R.chi[k] > cap) return false;
    return true;
}

}  // namespace

__global__ __launch_bounds__(CT) void camps_kernel(CampsArgs P) {
    __shared__ uint64_t s_x[NR * 2], s_z[NR * 2];
    __shared__ uint8_t s_ph[NR];
    __shared__ uint8_t s_laste[kMaxSites];
    __shared__ int s_chi[kMaxSites + 1];
    __shared__ int s_old[kMaxSites + 1];
    __shared__ double s_red[CT / 64];
    __shared__ double s_sg[K];
    __shared__ int s_keep[K];
    __shared__ int s_flag, s_center, s_status, s_sweeps, s_peak, s_best;
    __shared__ double s_pur[kCampsCand + 1];
    __shared__ double s_dm[(kCampsCand + 1) * 32];   // identity, then the candidates
    __shared__ double s_part[CT];
    __shared__ double s_lwr[kWaveLen * kWaveCols], s_lwi[kWaveLen * kWaveCols];
    __shared__ double s_lvr[kWaveCols * kWaveCols], s_lvi[kWaveCols * kWaveCols];
    const int tid = threadIdx.x;
    const int n = P.n;
    Frame F;
    F.x = s_x;
    F.z = s_z;
    F.ph = s_ph;
    Res R{P.arena + static_cast<int64_t>(blockIdx.x) * n * kCampsSiteDoubles,
          P.scratch + static_cast<int64_t>(blockIdx.x) * kCampsScratch, s_chi, n};
    Ctl C;
    C.red = s_red;
    C.flag = &s_flag;
    C.sg = s_sg;
    C.keep = s_keep;
    C.center = &s_center;
    C.status = &s_status;
    C.sweeps = &s_sweeps;
    C.chi_peak = &s_peak;
    C.old = s_old;
    C.lwr = s_lwr;
    C.lwi = s_lwi;
    C.lvr = s_lvr;
    C.lvi = s_lvi;
    const double c8 = 0.92387953251128675613, s8 = 0.38268343236508977173;   // cos, sin of pi/8
    for (int e = tid; e < (kCampsCand + 1) * 32; e += CT) {
        const int c = e / 32, w = e - c * 32;
        s_dm[e] = c == 0 ? ((w % 2 == 0 && (w / 2) % 5 == 0) ? 1.0 : 0.0) : P.dmat[(c - 1) * 32 + w];
    }
    __syncthreads();

    for (int64_t it = blockIdx.x; it < P.n_shots; it += gridDim.x) {
        const int64_t shot = P.shot_idx ? P.shot_idx[it] : it;
        if (shot < 0 || shot >= P.n_csr) {
            if (tid == 0) {
                msc_shot_result bad{};
                bad.rejected_at = -1;
                P.out[it] = bad;
            }
            continue;
        }
        // ---- initial frame (identity) and residual |0...0>
        for (int q = tid; q < n; q += CT) {
            const int s = P.site_of[q];
            const int rx = 2 * q, rz = 2 * q + 1;
            s_x[2 * rx] = s < 64 ? 1ull << s : 0;
            s_x[2 * rx + 1] = s >= 64 ? 1ull << (s - 64) : 0;
            s_z[2 * rx] = 0;
            s_z[2 * rx + 1] = 0;
            s_x[2 * rz] = 0;
            s_x[2 * rz + 1] = 0;
            s_z[2 * rz] = s < 64 ? 1ull << s : 0;
            s_z[2 * rz + 1] = s >= 64 ? 1ull << (s - 64) : 0;
            s_ph[rx] = 0;
            s_ph[rz] = 0;
            s_laste[q] = 0;
        }
        for (int k = tid; k <= n; k += CT) s_chi[k] = 1;
        for (int k = tid; k < n; k += CT) {
            R.re(k)[0] = 1.0;
            R.re(k)[1] = 0.0;
            R.im(k)[0] = 0.0;
            R.im(k)[1] = 0.0;
        }
        if (tid == 0) {
            s_center = 0;
            s_status = 0;
            s_sweeps = 0;
            s_peak = 1;
        }
        __syncthreads();
        double p_acc = 1.0, infid = 0.0;
        int rej_at = -1;
        bool alive = true;
        int64_t fcur = P.shot_off[shot];
        const int64_t fend = P.shot_off[shot + 1];
        int64_t n_dis = 0;
        const double tau = P.tau;
        int start = 0;
        if (P.ck_mode == 2) {
            // fork from the last checkpoint of the noiseless run before the
            // shot's first fault (the ops before it are fault-free here)
            const int navail = *P.ck_avail;
            const int jj = fcur < fend ? P.chan[fcur] / P.ck_k : P.n_ck - 1;
            const int jck = jj < navail ? jj : navail - 1;
            if (jck >= 0) {
                const CampsCk& h = P.ck_hdr[jck];
                for (int k = tid; k <= n; k += CT) s_chi[k] = h.chi[k];
                for (int q = tid; q < n; q += CT) s_laste[q] = h.laste[q];
                const uint64_t* fw = P.ck_frame + static_cast<int64_t>(jck) * 4 * NR;
                for (int w = tid; w < 4 * n; w += CT) {
                    s_x[w] = fw[w];
                    s_z[w] = fw[2 * NR + w];
                }
                for (int r = tid; r < 2 * n; r += CT)
                    s_ph[r] = P.ck_ph[static_cast<int64_t>(jck) * 2 * kMaxSites + r];
                __syncthreads();
                const double* src = P.ck_data + P.ck_off[jck];
                int64_t o = 0;
                for (int k = 0; k < n; ++k) {
                    const int ne = s_chi[k] * 2 * s_chi[k + 1];
                    double *dr = R.re(k), *di = R.im(k);
                    for (int e = tid; e < ne; e += CT) {
                        dr[e] = src[o + e];
                        di[e] = src[o + ne + e];
                    }
                    o += 2 * ne;
                }
                if (tid == 0) {
                    s_center = h.center;
                    s_status = h.status;
                    s_sweeps = h.sweeps;
                    s_peak = h.peak;
                }
                p_acc = h.p_acc;
                n_dis = h.n_dis;
                start = P.ck_op[jck];
                __syncthreads();
            }
        }
        int next_ck = 0;              // record mode: next checkpoint to take
        int64_t ck_pos = 0;           // record mode: doubles written so far
        bool ck_full = false;

        // greedy disentangling sweep over bonds k0..k1.  Per bond, theta
        // (sites k, k+1) and the Gram matrix of its smaller side give the
        // reduced density matrix of D theta for every candidate D without
        // forming D theta: rho_D = sum D G D^dag over the bond's own legs.
        auto disentangle = [&](int k0, int k1) {
            move_center(R, C, k0, tau);
            for (int k = k0; k <= k1; ++k) {
                if (s_status & MSC_SHOT_CHI_CAP) break;     // bonds may exceed the buffers
                const int cl = s_chi[k], cm = s_chi[k + 1], cr = s_chi[k + 2];
                const int m = 2 * cl, nn = 2 * cr;
                double *thr = R.scr + oTC, *thi = thr + K * K;
                double *gr = R.scr + oF, *gi = R.scr + oTH;
                const double *ar = R.re(k), *ai = R.im(k), *br = R.re(k + 1), *bi = R.im(k + 1);
                // theta[(a,i)][(j,b)] = sum_u A[a,i,u] B[u,j,b]
                for (int e = tid; e < m * nn; e += CT) {
                    const int row = e / nn, col = e - row * nn;
                    double xr = 0, xi = 0;
                    for (int u = 0; u < cm; ++u) {
                        const double a_r = ar[row * cm + u], a_i = ai[row * cm + u];
                        const double b_r = br[u * nn + col], b_i = bi[u * nn + col];
                        xr += a_r * b_r - a_i * b_i;
                        xi += a_r * b_i + a_i * b_r;
                    }
                    thr[e] = xr;
                    thi[e] = xi;
                }
                __syncthreads();
                // Gram of the smaller side: left G[(a,i,j)][(a2,i2,j2)] =
                // sum_b th[(a,i),(j,b)] conj(th[(a2,i2),(j2,b)]); right
                // G[(i,j,b)][(i2,j2,b2)] = sum_a conj(th[(a,i),(j,b)]) th[(a,i2),(j2,b2)]
                const bool left = cl <= cr;
                const int sd = left ? cl : cr, gd = 4 * sd;
                for (int e = tid; e < gd * gd; e += CT) {
                    const int u = e / gd, v = e - u * gd;
                    double xr = 0, xi = 0;
                    if (left) {
                        const int a = u >> 2, i = (u >> 1) & 1, j = u & 1;
                        const int a2 = v >> 2, i2 = (v >> 1) & 1, j2 = v & 1;
                        const double *p_r = thr + (a * 2 + i) * nn + j * cr, *p_i = thi + (a * 2 + i) * nn + j * cr;
                        const double *q_r = thr + (a2 * 2 + i2) * nn + j2 * cr, *q_i = thi + (a2 * 2 + i2) * nn + j2 * cr;
                        for (int b = 0; b < cr; ++b) {
                            xr += p_r[b] * q_r[b] + p_i[b] * q_i[b];
                            xi += p_i[b] * q_r[b] - p_r[b] * q_i[b];
                        }
                    } else {
                        const int ij = u / cr, b = u - ij * cr, ij2 = v / cr, b2 = v - ij2 * cr;
                        const int i = ij >> 1, j = ij & 1, i2 = ij2 >> 1, j2 = ij2 & 1;
                        for (int a = 0; a < cl; ++a) {
                            const int s1 = (a * 2 + i) * nn + j * cr + b, s2 = (a * 2 + i2) * nn + j2 * cr + b2;
                            xr += thr[s1] * thr[s2] + thi[s1] * thi[s2];
                            xi += thr[s1] * thi[s2] - thi[s1] * thr[s2];
                        }
                    }
                    gr[e] = xr;
                    gi[e] = xi;
                }
                __syncthreads();
                // purity of every candidate (0 = no gate), kCampsCand + 1 teams
                // of 12 threads, each summing |rho|^2 over a fixed stride
                constexpr int TPC = CT / (kCampsCand + 1);
                const int cand = tid / TPC, lane = tid - cand * TPC;
                double part = 0.0;
                if (cand <= kCampsCand) {
                    const double* d = s_dm + cand * 32;
                    const int rd = left ? m : nn;           // rho is rd x rd
                    for (int e = lane; e < rd * rd; e += TPC) {
                        const int x1 = e / rd, x2 = e - x1 * rd;
                        double rr = 0, ri = 0;
                        if (left) {
                            const int a = x1 >> 1, ip = x1 & 1, a2 = x2 >> 1, i2p = x2 & 1;
                            for (int jp = 0; jp < 2; ++jp)
                                for (int in = 0; in < 4; ++in) {
                                    const int o1 = (2 * ip + jp) * 4 + in;
                                    const double d1r = d[2 * o1], d1i = d[2 * o1 + 1];
                                    if (d1r == 0.0 && d1i == 0.0) continue;
                                    for (int in2 = 0; in2 < 4; ++in2) {
                                        const int o2 = (2 * i2p + jp) * 4 + in2;
                                        const double d2r = d[2 * o2], d2i = -d[2 * o2 + 1];
                                        if (d2r == 0.0 && d2i == 0.0) continue;
                                        const int g = (a * 4 + in) * gd + (a2 * 4 + in2);
                                        // d1 * conj(d2') * G
                                        const double pr_ = d1r * d2r - d1i * d2i, pi_ = d1r * d2i + d1i * d2r;
                                        rr += pr_ * gr[g] - pi_ * gi[g];
                                        ri += pr_ * gi[g] + pi_ * gr[g];
                                    }
                                }
                        } else {
                            const int jp = x1 / cr, b = x1 - jp * cr, j2p = x2 / cr, b2 = x2 - j2p * cr;
                            for (int ip = 0; ip < 2; ++ip)
                                for (int in = 0; in < 4; ++in) {
                                    const int o1 = (2 * ip + jp) * 4 + in;
                                    const double d1r = d[2 * o1], d1i = -d[2 * o1 + 1];   // conj
                                    if (d1r == 0.0 && d1i == 0.0) continue;
                                    for (int in2 = 0; in2 < 4; ++in2) {
                                        const int o2 = (2 * ip + j2p) * 4 + in2;
                                        const double d2r = d[2 * o2], d2i = d[2 * o2 + 1];
                                        if (d2r == 0.0 && d2i == 0.0) continue;
                                        const int g = (in * cr + b) * gd + (in2 * cr + b2);
                                        const double pr_ = d1r * d2r - d1i * d2i, pi_ = d1r * d2i + d1i * d2r;
                                        rr += pr_ * gr[g] - pi_ * gi[g];
                                        ri += pr_ * gi[g] + pi_ * gr[g];
                                    }
                                }
                        }
                        part += rr * rr + ri * ri;
                    }
                    s_part[tid] = part;
                }
                __syncthreads();
                if (tid <= kCampsCand) {
                    double acc = 0.0;
                    for (int l = 0; l < TPC; ++l) acc += s_part[tid * TPC + l];
                    s_pur[tid] = acc;
                }
                __syncthreads();
                if (tid == 0) {
                    double best = s_pur[0];
                    int choice = -1;
                    for (int cc = 0; cc < kCampsCand; ++cc)
                        if (s_pur[cc + 1] > best * (1.0 + 1e-9)) {
                            best = s_pur[cc + 1];
                            choice = cc;
                        }
                    s_best = choice;
                }
                __syncthreads();
                const int choice = s_best;
                if (choice < 0) {
                    // nothing gains: just move the centre on
                    move_right(R, C, k, tau);
                    continue;
                }
                ++n_dis;
                const WV w = work_mats(R, C, m, nn);
                double *wr = w.wr, *wi = w.wi, *vr = w.vr, *vi = w.vi;
                const int ldw = w.ldw, ldv = w.ldv;
                const double* d = s_dm + (choice + 1) * 32;
                // W <- (D theta) column-major
                for (int e = tid; e < m * nn; e += CT) {
                    const int row = e / nn, col = e - row * nn;
                    const int a = row >> 1, i2 = row & 1, j2 = col / cr, b = col - j2 * cr;
                    const int o = 2 * i2 + j2;
                    double xr = 0, xi = 0;
                    for (int in = 0; in < 4; ++in) {
                        const int i1 = in >> 1, j1 = in & 1;
                        const double g_r = d[2 * (o * 4 + in)], g_i = d[2 * (o * 4 + in) + 1];
                        const int src = (a * 2 + i1) * nn + j1 * cr + b;
                        xr += g_r * thr[src] - g_i * thi[src];
                        xi += g_r * thi[src] + g_i * thr[src];
                    }
                    wr[col * ldw + row] = xr;
                    wi[col * ldw + row] = xi;
                }
                // frame: every row's part on sites k, k+1 conjugated by D
                const uint8_t* tab = P.dtab + choice * 16;
                for (int r = tid; r < 2 * n; r += CT) {
                    const int x1 = getbit(s_x + 2 * r, k), z1 = getbit(s_z + 2 * r, k);
                    const int x2 = getbit(s_x + 2 * r, k + 1), z2 = getbit(s_z + 2 * r, k + 1);
                    const int t = tab[x1 | (z1 << 1) | (x2 << 2) | (z2 << 3)];
                    const int w0 = k >> 6, w1 = (k + 1) >> 6;
                    const uint64_t m0 = 1ull << (k & 63), m1 = 1ull << ((k + 1) & 63);
                    s_x[2 * r + w0] = (s_x[2 * r + w0] & ~m0) | ((t & 1) ? m0 : 0);
                    s_z[2 * r + w0] = (s_z[2 * r + w0] & ~m0) | ((t & 2) ? m0 : 0);
                    s_x[2 * r + w1] = (s_x[2 * r + w1] & ~m1) | ((t & 4) ? m1 : 0);
                    s_z[2 * r + w1] = (s_z[2 * r + w1] & ~m1) | ((t & 8) ? m1 : 0);
                    s_ph[r] = static_cast<uint8_t>((s_ph[r] + (t >> 4)) & 3);
                }
                __syncthreads();
                // split D theta: A_k = U, A_{k+1} = S V^dag
                note_sweeps(C, jacobi_cols(w, m, nn, &s_flag));
                const int rr = select_cols(w, m, nn, tau, s_sg, s_keep, s_red);
                double *Ar = R.re(k), *Ai = R.im(k), *Br = R.re(k + 1), *Bi = R.im(k + 1);
                for (int e = tid; e < m * rr; e += CT) {
                    const int row = e / rr, jj = e - row * rr;
                    const int col = s_keep[jj];
                    const double s = 1.0 / s_sg[col];
                    Ar[row * rr + jj] = wr[col * ldw + row] * s;
                    Ai[row * rr + jj] = wi[col * ldw + row] * s;
                }
                for (int e = tid; e < rr * nn; e += CT) {
                    const int jj = e / nn, col2 = e - jj * nn;
                    const int col = s_keep[jj];
                    Br[e] = s_sg[col] * vr[col * ldv + col2];
                    Bi[e] = -s_sg[col] * vi[col * ldv + col2];
                }
                if (tid == 0) {
                    s_chi[k + 1] = rr;
                    s_center = k + 1;
                    if (rr > s_peak) s_peak = rr;
                    if (rr > P.chi_cap) s_status |= MSC_SHOT_CHI_CAP;
                }
                __syncthreads();
            }
        };

        for (int oi = start; oi < P.n_ops && alive; ++oi) {
            if (P.ck_mode == 1 && !ck_full && next_ck < P.n_ck && P.ck_op[next_ck] == oi) {
                // ---- record: the frame and the residual before op oi
                int64_t sz = 0;
                for (int k = 0; k < n; ++k) sz += 4LL * s_chi[k] * s_chi[k + 1];
                if (ck_pos + sz <= P.ck_cap) {
                    double* dst = P.ck_data + ck_pos;
                    int64_t o = 0;
                    for (int k = 0; k < n; ++k) {
                        const int ne = s_chi[k] * 2 * s_chi[k + 1];
                        const double *sr = R.re(k), *si = R.im(k);
                        for (int e = tid; e < ne; e += CT) {
                            dst[o + e] = sr[e];
                            dst[o + ne + e] = si[e];
                        }
                        o += 2 * ne;
                    }
                    uint64_t* fw = P.ck_frame + static_cast<int64_t>(next_ck) * 4 * NR;
                    for (int w = tid; w < 4 * n; w += CT) {
                        fw[w] = s_x[w];
                        fw[2 * NR + w] = s_z[w];
                    }
                    for (int r = tid; r < 2 * n; r += CT)
                        P.ck_ph[static_cast<int64_t>(next_ck) * 2 * kMaxSites + r] = s_ph[r];
                    CampsCk& h = P.ck_hdr[next_ck];
                    for (int k = tid; k <= n; k += CT) h.chi[k] = s_chi[k];
                    for (int q = tid; q < n; q += CT) h.laste[q] = s_laste[q];
                    if (tid == 0) {
                        h.p_acc = p_acc;
                        h.n_dis = n_dis;
                        h.center = s_center;
                        h.status = s_status;
                        h.sweeps = s_sweeps;
                        h.peak = s_peak;
                        P.ck_off[next_ck] = ck_pos;
                    }
                    ck_pos += sz;
                    __syncthreads();
                    if (tid == 0) *P.ck_avail = next_ck + 1;
                    ++next_ck;
                } else {
                    ck_full = true;
                }
            }
            const DevOp op = P.ops[oi];
            if (op.kind == CO_G1) {
                if (tid == 0) {
                    const int rx = 2 * op.a, rz = 2 * op.a + 1;
                    switch (op.aux) {
                    case G_H: {   // X <-> Z
                        const uint64_t a0 = s_x[2 * rx], a1 = s_x[2 * rx + 1], b0 = s_z[2 * rx],
                                       b1 = s_z[2 * rx + 1];
                        const uint8_t pa = s_ph[rx];
                        row_copy(F, rx, rz);
                        s_x[2 * rz] = a0;
                        s_x[2 * rz + 1] = a1;
                        s_z[2 * rz] = b0;
                        s_z[2 * rz + 1] = b1;
                        s_ph[rz] = pa;
                        break;
                    }
                    case G_S: row_prod(F, rx, rx, rz, 3); break;     // S^dag X S = -i X Z
                    case G_SDG: row_prod(F, rx, rx, rz, 1); break;   // S X S^dag = i X Z
                    case G_X: s_ph[rz] = (s_ph[rz] + 2) & 3; break;
                    case G_Z: s_ph[rx] = (s_ph[rx] + 2) & 3; break;
                    case G_Y:
                        s_ph[rx] = (s_ph[rx] + 2) & 3;
                        s_ph[rz] = (s_ph[rz] + 2) & 3;
                        break;
                    default: break;
                    }
                }
                __syncthreads();
            } else if (op.kind == CO_CX) {
                if (tid == 0) {
                    // X_a -> X_a X_b, Z_b -> Z_a Z_b
                    row_prod(F, 2 * op.a, 2 * op.a, 2 * op.b, 0);
                    row_prod(F, 2 * op.b + 1, 2 * op.a + 1, 2 * op.b + 1, 0);
                }
                __syncthreads();
            } else if (op.kind == CO_CZ) {
                if (tid == 0) {
                    // X_a -> X_a Z_b, X_b -> Z_a X_b (from the old rows)
                    const int xa = 2 * op.a, xb = 2 * op.b;
                    row_prod(F, xa, xa, 2 * op.b + 1, 0);
                    row_prod(F, xb, 2 * op.a + 1, xb, 0);
                }
                __syncthreads();
            } else if (op.kind == CO_FAULT) {
                if (tid == 0) {
                    while (fcur < fend && P.chan[fcur] == op.a) {
                        const int code = P.pauli[fcur];
                        for (int j = 0; j < 3; ++j) {
                            const int q = P.chan_q[3 * op.a + j];
                            if (q < 0) continue;
                            const int fx = (code >> (2 * j)) & 1, fz = (code >> (2 * j + 1)) & 1;
                            if (fz) s_ph[2 * q] = (s_ph[2 * q] + 2) & 3;
                            if (fx) s_ph[2 * q + 1] = (s_ph[2 * q + 1] + 2) & 3;
                        }
                        ++fcur;
                    }
                }
                // every thread follows the same cursor
                while (fcur < fend && P.chan[fcur] == op.a) ++fcur;
                __syncthreads();
            } else if (op.kind == CO_RESET) {
                if (tid == 0 && s_laste[op.a]) {
                    s_ph[2 * op.a + 1] = (s_ph[2 * op.a + 1] + 2) & 3;
                    s_laste[op.a] = 0;
                }
                __syncthreads();
            } else if (op.kind == CO_ROT || op.kind == CO_MEAS) {
                const int row = 2 * op.a + 1;
                double alr, ali, ber, bei;
                if (op.kind == CO_ROT) {
                    alr = c8;
                    ali = 0.0;
                    ber = 0.0;
                    bei = op.aux > 0 ? -s8 : s8;
                } else {
                    const int e = P.expected[op.aux];
                    const double ev = expect(R, C, F, row, tau);
                    const double sgn = e ? -1.0 : 1.0;
                    const double pe = 0.5 * (1.0 + sgn * ev);
                    if (!(pe >= P.tau_rej)) {
                        alive = false;
                        rej_at = op.aux;
                        p_acc = 0.0;
                        if (tid == 0) s_status |= MSC_SHOT_REJECTED;
                        __syncthreads();
                        break;
                    }
                    p_acc *= pe;
                    if (tid == 0) s_laste[op.a] = static_cast<uint8_t>(e);
                    __syncthreads();
                    if (fabs(pe - 1.0) <= 1e-12) continue;   // already an eigenstate
                    alr = 0.5 / sqrt(pe);
                    ali = 0.0;
                    ber = sgn * alr;
                    bei = 0.0;
                }
                int lo, hi;
                const bool ok = apply_sum(R, C, F, row, alr, ali, ber, bei, tau, P.chi_cap, lo, hi);
                if (!ok) {
                    if (tid == 0) s_status |= MSC_SHOT_CHI_CAP;
                    __syncthreads();
                    alive = false;
                    p_acc = 0.0;
                    break;
                }
                if (hi > lo && n > 1) disentangle(max(lo - 1, 0), min(hi, n - 2));
                if (s_status & MSC_SHOT_CHI_CAP) {
                    alive = false;
                    p_acc = 0.0;
                    break;
                }
            } else if (op.kind == CO_FINAL) {
                const int rx = 2 * op.a, rz = 2 * op.a + 1;
                const double ex = expect(R, C, F, rx, tau);
                const double ez = expect(R, C, F, rz, tau);
                // Y = i X Z: a scratch row (index 2n) from the two images
                if (tid == 0) row_prod(F, 2 * n, rx, rz, 1);
                __syncthreads();
                const double ey = expect(R, C, F, 2 * n, tau);
                const double f = 0.5 * (1.0 + ex * P.rt[0] + ey * P.rt[1] + ez * P.rt[2]);
                infid = fmax(0.0, 1.0 - f);
            }
        }
        if (tid == 0) {
            msc_shot_result res{};
            res.p_acc = p_acc;
            res.infid = alive ? infid : 0.0;
            res.disc_weight = 0.0;
            res.chi_peak = s_peak;
            res.status = s_status | (alive ? MSC_SHOT_DONE : 0);
            res.rejected_at = rej_at;
            res.fail = (alive && p_acc > 0.0 && infid > P.tau_fail) ? 1 : 0;
            res.n2q = n_dis;
            res.flops = 0.0;
            res.sweeps = s_sweeps;
            P.out[it] = res;
        }
        __syncthreads();
    }
}

hipError_t launch_camps(const CampsArgs& a, int grid, hipStream_t s) {
    if (a.n < 1 || a.n > kMaxSites - 1 || grid < 1 || a.chi_cap < 1 || a.chi_cap > kCampsCap)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(camps_kernel, dim3(grid), dim3(CT), 0, s, a);
    return hipGetLastError();
}

int camps_blocks_per_cu() {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, camps_kernel, CT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return b > 0 ? b : 1;
}

}  // namespace msc
