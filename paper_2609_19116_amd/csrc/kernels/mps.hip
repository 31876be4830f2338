// Persistent batched MPS shot kernel for gfx950.
//
// One workgroup (4 wavefronts, one per SIMD) owns one MPS slot in HBM and runs whole shots
// through the compiled op stream, taking shots blockIdx.x, blockIdx.x +
// gridDim.x, ...  Each shot has its own ragged bond dimensions, kept in LDS,
// and stops at the first measurement whose expected outcome has probability
// below tau_rej (online screening, Section 4.3), so a rejected shot frees
// its workgroup for the next one at once.
//
// Per op (Section 3.1 for the MPS, Section 4 for the shot semantics):
//  * 1q gates and Pauli faults act on one site tensor (chi_l x 2 x chi_r);
//  * a two-site update contracts A[k] A[k+1] (complex, in the tensor
//    precision T), applies the 4x4 gate, and factorises the result exactly:
//    one-sided Jacobi (Hestenes) SVD in FP64 on the columns (centre moves
//    right) or rows (centre moves left) of theta, held in LDS when both
//    sides are at most SMAX, else in the slot's HBM scratch; singular values
//    sigma_i <= tau * sigma_0 are dropped (numerical zeros), the bond becomes
//    the number kept, the isometric factor is the normalised orthogonal
//    vectors and the centre factor is the projection of theta on them,
//    renormalised in FP64 (Section 3.1, "exact regime" of Section 5.1);
//  * a measurement, taken with the centre on the site, computes
//    p_e = ||A[:, e, :]||^2 / ||A||^2 in FP64, rejects if p_e < tau_rej,
//    otherwise projects, renormalises and multiplies P_acc by p_e;
//  * the final op reads the seed qubit's reduced density matrix and the
//    fidelity with the target (Appendix "Post-selection and logical error").
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "kernels.h"

namespace msc {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int MAXV = 2 * kMaxChiKernel;   // vectors in a two-site SVD
constexpr int kStage = 2048;               // doubles of LDS staging per workgroup

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NW; ++j) s += red[j * K + k];
        v[k] = s;
    }
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int j = 1; j < NW; ++j) m = fmax(m, red[j]);
    return m;
}

// Round-robin ("circle") pairing: slot 0 fixed, the others rotate each step.
__device__ __forceinline__ int player(int slot, int t, int nv) {
    return slot == 0 ? 0 : 1 + (slot - 1 + t) % (nv - 1);
}

// One sweep of one-sided Jacobi (Hestenes) over the nv vectors list[0..nv)
// of length len (planar FP64 at vre/vim, vector v at v*ld, ld >= len padded
// against LDS bank conflicts): every pair (p, q) once, in round-robin order
// so that the pairs of a step are disjoint and rotate in parallel (an odd
// count gets a dummy slot).  The 2x2 rotation
// makes the pair orthogonal: with gamma = x^H y, zeta = (|y|^2 - |x|^2) /
// (2|gamma|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1+t^2),
// s = c t and y~ = y conj(gamma)/|gamma|: x <- c x - s y~, y <- s x + c y~.
__device__ void jacobi_sweep(double* vre, double* vim, const int* list, int nv, int len, int ld,
                             double floor2, double tol) {
    const int tid = threadIdx.x;
    if (nv < 2) return;
    const int nve = nv + (nv & 1);   // the slot nv (if odd) is a dummy
    const int npairs = nve / 2;
    int tpp = NT / npairs;
    if (tpp > 64) tpp = 64;
    if (tpp < 1) tpp = 1;
    int t2 = 1;
    while (t2 * 2 <= tpp) t2 *= 2;
    tpp = t2;
    const int groups = NT / tpp;
    const int gl = tid % tpp;
    const int gi = tid / tpp;
    for (int t = 0; t < nve - 1; ++t) {
        for (int pb = 0; pb < npairs; pb += groups) {
            const int pi = pb + gi;
            const int sp = pi < npairs ? player(pi, t, nve) : 0;
            const int sq = pi < npairs ? player(nve - 1 - pi, t, nve) : 0;
            const bool active = pi < npairs && sp < nv && sq < nv;
            int p = 0, q = 0;
            double a = 0.0, b = 0.0, gr = 0.0, gim = 0.0;
            if (active) {
                p = list[sp];
                q = list[sq];
                const double* xr = vre + (size_t)p * ld;
                const double* xi = vim + (size_t)p * ld;
                const double* yr = vre + (size_t)q * ld;
                const double* yi = vim + (size_t)q * ld;
                for (int e = gl; e < len; e += tpp) {
                    double x0 = xr[e], x1 = xi[e], y0 = yr[e], y1 = yi[e];
                    a += x0 * x0 + x1 * x1;
                    b += y0 * y0 + y1 * y1;
                    gr += x0 * y0 + x1 * y1;
                    gim += x0 * y1 - x1 * y0;
                }
            }
            for (int o = tpp >> 1; o > 0; o >>= 1) {
                a += __shfl_xor(a, o);
                b += __shfl_xor(b, o);
                gr += __shfl_xor(gr, o);
                gim += __shfl_xor(gim, o);
            }
            if (active) {
                const double g = sqrt(gr * gr + gim * gim);
                if (a > floor2 && b > floor2 && g > tol * sqrt(a * b)) {
                    const double ig = 1.0 / g;
                    const double zeta = 0.5 * (b - a) * ig;
                    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) /
                                      (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + tt * tt);
                    const double s = c * tt;
                    const double pr = gr * ig, pim = gim * ig;
                    double* xr = vre + (size_t)p * ld;
                    double* xi = vim + (size_t)p * ld;
                    double* yr = vre + (size_t)q * ld;
                    double* yi = vim + (size_t)q * ld;
                    for (int e = gl; e < len; e += tpp) {
                        double x0 = xr[e], x1 = xi[e];
                        double y0 = yr[e] * pr + yi[e] * pim;
                        double y1 = yi[e] * pr - yr[e] * pim;
                        xr[e] = c * x0 - s * y0;
                        xi[e] = c * x1 - s * y1;
                        yr[e] = s * x0 + c * y0;
                        yi[e] = s * x1 + c * y1;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Squared norms of nv vectors (stride ld) into nrm.
__device__ void vector_norms(const double* vre, const double* vim, int nv, int len, int ld,
                             double* nrm) {
    for (int v = threadIdx.x; v < nv; v += NT) {
        double s = 0.0;
        const double* xr = vre + (size_t)v * ld;
        const double* xi = vim + (size_t)v * ld;
        for (int e = 0; e < len; ++e) s += xr[e] * xr[e] + xi[e] * xi[e];
        nrm[v] = s;
    }
    __syncthreads();
}

// One parallel pass over every pair of vectors whose squared norms exceed
// floor2 (only pairs with a vector flagged in `only`, if given): marks in
// `bad` every vector of a pair that overlaps by more than tol and returns
// true (block-uniform) if there is one.
__device__ bool not_orthogonal(const double* vre, const double* vim, int nv, int len, int ld,
                               const double* nrm, double floor2, double tol, int* bad,
                               const int* only) {
    for (int v = threadIdx.x; v < nv; v += NT) bad[v] = 0;
    __syncthreads();
    int any = 0;
    for (int t = threadIdx.x; t < nv * nv; t += NT) {
        const int p = t / nv, q = t - p * nv;
        if (q <= p) continue;
        if (only && !(only[p] | only[q])) continue;
        const double a = nrm[p], b = nrm[q];
        if (!(a > floor2 && b > floor2)) continue;
        const double* xr = vre + (size_t)p * ld;
        const double* xi = vim + (size_t)p * ld;
        const double* yr = vre + (size_t)q * ld;
        const double* yi = vim + (size_t)q * ld;
        double gr = 0.0, gim = 0.0;
        for (int e = 0; e < len; ++e) {
            gr += xr[e] * yr[e] + xi[e] * yi[e];
            gim += xr[e] * yi[e] - xi[e] * yr[e];
        }
        if (gr * gr + gim * gim > tol * tol * a * b) {
            any = 1;
            bad[p] = 1;   // benign race: every writer stores 1
            bad[q] = 1;
        }
    }
    return __syncthreads_or(any) != 0;
}

// Compacts the flagged vectors into list (ascending); returns their count.
__device__ int flagged_list(const int* flag, int nv, int* list, int* red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int base = 0;
    for (int b0 = 0; b0 < nv; b0 += NT) {
        const int v = b0 + tid;
        const bool f = v < nv && flag[v];
        const uint64_t m = __ballot(f);
        __syncthreads();
        if (lane == 0) red[w] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int q = 0; q < w; ++q) off += red[q];
        if (f) list[off + __popcll(m & ((1ull << lane) - 1ull))] = v;
        for (int q = 0; q < NW; ++q) base += red[q];
    }
    __syncthreads();
    return base;
}

struct Kept {
    int r;
    double kept, dropped;
};

// Keep the vectors with sigma^2 > tau2 * sigma_0^2 (at most capb), ordered by
// decreasing norm: sel[0..r) are their indices.
__device__ Kept select_kept(const double* nrm, int nv, double tau2, int capb, int* sel,
                            double* red) {
    double mx = 0.0;
    for (int v = threadIdx.x; v < nv; v += NT) mx = fmax(mx, nrm[v]);
    mx = block_max(mx, red);
    double kd[3] = {0.0, 0.0, 0.0};
    for (int v = threadIdx.x; v < nv; v += NT) {
        const double x = nrm[v];
        int rank = 0;
        for (int u = 0; u < nv; ++u) {
            const double y = nrm[u];
            rank += (y > x) || (y == x && u < v);
        }
        const bool keep = (x > tau2 * mx || rank == 0) && rank < capb;
        if (keep) {
            sel[rank] = v;
            kd[0] += 1.0;
            kd[1] += x;
        } else {
            kd[2] += x;
        }
    }
    block_sum<3>(kd, red);
    Kept k;
    k.r = static_cast<int>(kd[0] + 0.5);
    k.kept = kd[1];
    k.dropped = kd[2];
    return k;
}

template <typename T>
struct SiteView {
    T* re;
    T* im;
};

template <typename T, int SMAX>
__global__ __launch_bounds__(NT) void mps_kernel(MpsArgs P) {
    __shared__ int s_chi[kMaxSites + 1];
    __shared__ int s_laste[kMaxSites];
    __shared__ double s_vre[SMAX * (SMAX + 1)];
    __shared__ double s_vim[SMAX * (SMAX + 1)];
    __shared__ double s_nrm[SMAX];
    __shared__ int s_sel[SMAX];
    __shared__ int s_bad[SMAX];
    __shared__ int s_list[SMAX];
    __shared__ int s_ired[NW];
    __shared__ double s_red[NW * 4];
    __shared__ double s_gph[8];
    __shared__ int s_gsrc[4];
    // per-site layout of the slot and bond caps, read once per launch
    __shared__ int64_t s_soff[kMaxSites];
    __shared__ int64_t s_shalf[kMaxSites];
    __shared__ int s_cap[kMaxSites + 1];
    // staging: the two site tensors of an update (tensor type), then the
    // copy of theta kept for the projection (FP64)
    __shared__ double s_u[kStage];

    const int tid = threadIdx.x;
    const int N = P.n_sites;
    T* slot_base = static_cast<T*>(P.arena) + (size_t)blockIdx.x * P.slot_stride;
    double* scr = P.scratch + (size_t)blockIdx.x * P.scratch_stride;
    // per-vector arrays of SVDs too large for LDS, at the end of the slot's scratch
    double* g_nrm = scr + P.scratch_stride - 4 * MAXV;
    int* g_sel = reinterpret_cast<int*>(g_nrm + MAXV);
    int* g_bad = g_sel + MAXV;
    int* g_list = g_bad + MAXV;

    for (int k = tid; k < N; k += NT) {
        s_soff[k] = P.site_off[k];
        s_shalf[k] = P.site_half[k];
    }
    for (int k = tid; k <= N; k += NT) s_cap[k] = P.cap[k];
    __syncthreads();

    auto site = [&](int k) {
        SiteView<T> v;
        v.re = slot_base + s_soff[k];
        v.im = v.re + s_shalf[k];
        return v;
    };

    for (int64_t j = blockIdx.x; j < P.n_shots; j += gridDim.x) {
        const int64_t it = P.perm ? P.perm[j] : j;
        const int64_t shot = P.shot_idx ? P.shot_idx[it] : it;
        if (shot < 0 || shot >= P.n_csr) {
            if (tid == 0) {
                msc_shot_result bad{};
                bad.rejected_at = -1;
                P.out[it] = bad;
            }
            continue;
        }
        double p_acc = 1.0, disc = 0.0, infid = 0.0;
        int chi_peak = 1, status = 0, rej_at = -1;
        int64_t n2q = 0;
        double flops = 0.0;
        int64_t sweeps_total = 0;
        int64_t fcur = P.shot_off[shot];
        const int64_t fend = P.shot_off[shot + 1];
        int fcode = 0;     // code of the last channel read (three-qubit faults)
        bool alive = true;
        int start = 0;
        int jck = -1;
        if (P.ck_mode == 2) {
            // fork from the last checkpoint of the noiseless run before the
            // shot's first fault (the ops before it are fault-free here)
            const int navail = *P.ck_avail;
            int j = fcur < fend ? P.chan[fcur] / P.ck_k : P.n_ck - 1;
            jck = j < navail ? j : navail - 1;
        }
        if (jck >= 0) {
            const CkHdr& h = P.ck_hdr[jck];
            for (int k = tid; k <= N; k += NT) s_chi[k] = h.chi[k];
            for (int k = tid; k < N; k += NT) s_laste[k] = h.laste[k];
            __syncthreads();
            const T* src = static_cast<const T*>(P.ck_data) + P.ck_off[jck];
            int64_t o = 0;
            for (int k = 0; k < N; ++k) {
                const int ne = s_chi[k] * 2 * s_chi[k + 1];
                SiteView<T> v = site(k);
                for (int idx = tid; idx < ne; idx += NT) {
                    v.re[idx] = src[o + idx];
                    v.im[idx] = src[o + ne + idx];
                }
                o += 2 * ne;
            }
            p_acc = h.p_acc;
            disc = h.disc;
            chi_peak = h.chi_peak;
            status = h.status;
            start = P.ck_op[jck];
        } else {
            // ---- initial product state |0...0>
            for (int k = tid; k <= N; k += NT) s_chi[k] = 1;
            for (int k = tid; k < N; k += NT) {
                s_laste[k] = 0;
                SiteView<T> v = site(k);
                v.re[0] = T(1);
                v.re[1] = T(0);
                v.im[0] = T(0);
                v.im[1] = T(0);
            }
        }
        __syncthreads();
        int next_ck = 0;           // record mode: next checkpoint to take
        int64_t ck_pos = 0;        // record mode: elements written so far
        bool ck_full = false;

        DevOp next_op = start < P.n_ops ? P.ops[start] : DevOp{};
        for (int oi = start; oi < P.n_ops && alive; ++oi) {
            if (P.ck_mode == 1 && !ck_full && next_ck < P.n_ck && P.ck_op[next_ck] == oi) {
                // ---- record: the state before op oi, densely, site by site
                int64_t sz = 0;
                for (int k = 0; k < N; ++k) sz += 4 * (int64_t)s_chi[k] * s_chi[k + 1];
                if (ck_pos + sz <= P.ck_cap) {
                    T* dst = static_cast<T*>(P.ck_data) + ck_pos;
                    int64_t o = 0;
                    for (int k = 0; k < N; ++k) {
                        const int ne = s_chi[k] * 2 * s_chi[k + 1];
                        SiteView<T> v = site(k);
                        for (int idx = tid; idx < ne; idx += NT) {
                            dst[o + idx] = v.re[idx];
                            dst[o + ne + idx] = v.im[idx];
                        }
                        o += 2 * ne;
                    }
                    CkHdr& h = P.ck_hdr[next_ck];
                    for (int k = tid; k <= N; k += NT) h.chi[k] = s_chi[k];
                    for (int k = tid; k < N; k += NT) h.laste[k] = s_laste[k];
                    if (tid == 0) {
                        h.p_acc = p_acc;
                        h.disc = disc;
                        h.chi_peak = chi_peak;
                        h.status = status;
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
            const DevOp op = next_op;
            if (oi + 1 < P.n_ops) next_op = P.ops[oi + 1];   // in flight during this op
            bool twosite = op.kind == OP_G2;
            int gate_id = op.aux;
            if (op.kind == OP_MOVE) {
                // ---- move the centre by one site with a one-site split; when
                // the site's vectors are already orthogonal (they are after a
                // split that left the centre there) this is a selection and a
                // rescaling, else fall back to the two-site identity update
                const int k = op.a, dir = op.b;
                const int cl = s_chi[k], cm = s_chi[k + 1], cr = s_chi[k + 2];
                SiteView<T> A = site(k), B = site(k + 1);
                const int nv = cm, len = dir ? 2 * cl : 2 * cr, ld = len + 1;
                bool fast = false;
                if (nv <= SMAX && len <= SMAX) {
                    for (int idx = tid; idx < nv * len; idx += NT) {
                        const int v = idx / len, e = idx - v * len;
                        const int at = dir ? e * cm + v : v * len + e;
                        const SiteView<T>& S = dir ? A : B;
                        s_vre[v * ld + e] = static_cast<double>(S.re[at]);
                        s_vim[v * ld + e] = static_cast<double>(S.im[at]);
                    }
                    __syncthreads();
                    vector_norms(s_vre, s_vim, nv, len, ld, s_nrm);
                    double tsum[1] = {0.0};
                    for (int v = tid; v < nv; v += NT) tsum[0] += s_nrm[v];
                    block_sum<1>(tsum, s_red);
                    const double tau2 = P.tau * P.tau;
                    const double tol = sizeof(T) == sizeof(double)
                                           ? static_cast<double>(len) * DBL_EPSILON
                                           : 8.0 * static_cast<double>(FLT_EPSILON);
                    if (!not_orthogonal(s_vre, s_vim, nv, len, ld, s_nrm, 1e-4 * tau2 * tsum[0], tol,
                                        s_bad, nullptr)) {
                        const int capb = min(P.chi_max, s_cap[k + 1]);
                        const Kept kp = select_kept(s_nrm, nv, tau2, capb, s_sel, s_red);
                        const int r = kp.r;
                        disc += kp.dropped;
                        if (kp.dropped > 1e-12 * tsum[0] && r == capb) status |= MSC_SHOT_CHI_CAP;
                        const double renorm = 1.0 / sqrt(kp.kept);
                        // staging for the rescaled neighbour: LDS (free once the
                        // normalised vectors are written) when it fits
                        const int tmp_n = dir ? r * 2 * cr : 2 * cl * r;
                        const bool tlds = tmp_n <= SMAX * (SMAX + 1);
                        double* tr_ = tlds ? s_vre : scr;
                        double* ti_ = tlds ? s_vim : scr + (size_t)2 * cl * cm + (size_t)2 * cm * cr;
                        if (dir) {
                            // A[k] <- normalised columns; A[k+1] <- its selected rows
                            for (int idx = tid; idx < 2 * cl * r; idx += NT) {
                                const int e = idx / r, c = idx - e * r;
                                const int v = s_sel[c];
                                const double is = 1.0 / sqrt(s_nrm[v]);
                                A.re[idx] = T(s_vre[v * ld + e] * is);
                                A.im[idx] = T(s_vim[v * ld + e] * is);
                            }
                            __syncthreads();
                            const int w = 2 * cr;
                            for (int idx = tid; idx < r * w; idx += NT) {
                                const int c = idx / w, x = idx - c * w;
                                const int v = s_sel[c];
                                const double sc = sqrt(s_nrm[v]) * renorm;
                                tr_[idx] = static_cast<double>(B.re[v * w + x]) * sc;
                                ti_[idx] = static_cast<double>(B.im[v * w + x]) * sc;
                            }
                            __syncthreads();
                            for (int idx = tid; idx < r * w; idx += NT) {
                                B.re[idx] = T(tr_[idx]);
                                B.im[idx] = T(ti_[idx]);
                            }
                        } else {
                            // A[k+1] <- normalised rows; A[k] <- its selected columns
                            const int w = 2 * cr;
                            for (int idx = tid; idx < r * w; idx += NT) {
                                const int c = idx / w, e = idx - c * w;
                                const int v = s_sel[c];
                                const double is = 1.0 / sqrt(s_nrm[v]);
                                B.re[idx] = T(s_vre[v * ld + e] * is);
                                B.im[idx] = T(s_vim[v * ld + e] * is);
                            }
                            __syncthreads();
                            for (int idx = tid; idx < 2 * cl * r; idx += NT) {
                                const int row = idx / r, c = idx - row * r;
                                const int v = s_sel[c];
                                const double sc = sqrt(s_nrm[v]) * renorm;
                                tr_[idx] = static_cast<double>(A.re[row * cm + v]) * sc;
                                ti_[idx] = static_cast<double>(A.im[row * cm + v]) * sc;
                            }
                            __syncthreads();
                            for (int idx = tid; idx < 2 * cl * r; idx += NT) {
                                A.re[idx] = T(tr_[idx]);
                                A.im[idx] = T(ti_[idx]);
                            }
                        }
                        __syncthreads();
                        if (tid == 0) s_chi[k + 1] = r;
                        __syncthreads();
                        fast = true;
                    }
                }
                if (!fast) {
                    twosite = true;
                    gate_id = G4_I;
                }
            }
            if (op.kind == OP_G1 || op.kind == OP_FAULT || op.kind == OP_FAULT3 ||
                op.kind == OP_RESET) {
                // ---- local 2x2 on one site (two for a two-qubit fault)
                int g0 = -1, g1 = -1;
                if (op.kind == OP_G1) {
                    g0 = op.aux;
                } else if (op.kind == OP_RESET) {
                    if (s_laste[op.a] == 1) g0 = G_X;
                } else if (op.kind == OP_FAULT3) {
                    const int x2 = (fcode >> 4) & 1, z2 = (fcode >> 5) & 1;
                    if (x2 | z2) g0 = (x2 && z2) ? G_Y : (x2 ? G_X : G_Z);
                } else {
                    int code = 0;
                    if (fcur < fend && P.chan[fcur] == op.aux) {
                        code = P.pauli[fcur];
                        ++fcur;
                    }
                    fcode = code;
                    const int x0 = code & 1, z0 = (code >> 1) & 1;
                    const int x1 = (code >> 2) & 1, z1 = (code >> 3) & 1;
                    if (x0 | z0) g0 = (x0 && z0) ? G_Y : (x0 ? G_X : G_Z);
                    if ((x1 | z1) && op.b >= 0) g1 = (x1 && z1) ? G_Y : (x1 ? G_X : G_Z);
                }
                for (int h = 0; h < 2; ++h) {
                    const int gid = h == 0 ? g0 : g1;
                    if (gid < 0) continue;
                    const int k = h == 0 ? op.a : op.b;
                    const double* m = P.g1 + gid * 8;
                    const double m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
                    const double m4 = m[4], m5 = m[5], m6 = m[6], m7 = m[7];
                    SiteView<T> v = site(k);
                    const int cl = s_chi[k], cr = s_chi[k + 1];
                    for (int idx = tid; idx < cl * cr; idx += NT) {
                        const int a = idx / cr, b = idx - a * cr;
                        const int i0 = (a * 2) * cr + b, i1 = i0 + cr;
                        const double x0r = v.re[i0], x0i = v.im[i0], x1r = v.re[i1], x1i = v.im[i1];
                        v.re[i0] = T(m0 * x0r - m1 * x0i + m2 * x1r - m3 * x1i);
                        v.im[i0] = T(m0 * x0i + m1 * x0r + m2 * x1i + m3 * x1r);
                        v.re[i1] = T(m4 * x0r - m5 * x0i + m6 * x1r - m7 * x1i);
                        v.im[i1] = T(m4 * x0i + m5 * x0r + m6 * x1i + m7 * x1r);
                    }
                    __syncthreads();
                }
            } else if (op.kind == OP_SWAPP) {
                // ---- SWAP with a qubit that is unentangled in every shot:
                // its tensor is psi (x) M, so the swap moves psi to the other
                // site as psi (x) I and folds M into the neighbour (no SVD;
                // canonical form is kept because psi is normalised)
                const int k = op.a, side = op.b;
                const int ps = k + side, os = k + 1 - side;
                SiteView<T> Pv = site(ps), Ov = site(os);
                const int pl = s_chi[ps], pr = s_chi[ps + 1];
                double r4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int idx = tid; idx < pl * pr; idx += NT) {
                    const int a = idx / pr, b = idx - a * pr;
                    const int i0 = (a * 2) * pr + b, i1 = i0 + pr;
                    const double x0r = Pv.re[i0], x0i = Pv.im[i0], x1r = Pv.re[i1], x1i = Pv.im[i1];
                    r4[0] += x0r * x0r + x0i * x0i;
                    r4[1] += x1r * x1r + x1i * x1i;
                    r4[2] += x0r * x1r + x0i * x1i;     // rho01 = x0 conj(x1)
                    r4[3] += x0i * x1r - x0r * x1i;
                }
                block_sum<4>(r4, s_red);
                const double tr = r4[0] + r4[1];
                double p0r, p0i, p1r, p1i;               // psi, unit norm
                if (r4[1] > r4[0]) {
                    const double d = 1.0 / sqrt(r4[1] * tr);
                    p0r = r4[2] * d;
                    p0i = r4[3] * d;
                    p1r = r4[1] * d;
                    p1i = 0.0;
                } else {
                    const double d = 1.0 / sqrt(r4[0] * tr);
                    p0r = r4[0] * d;
                    p0i = 0.0;
                    p1r = r4[2] * d;                     // rho10 = conj(rho01)
                    p1i = -r4[3] * d;
                }
                // M = sum_i conj(psi_i) P[:, i, :]   (pl x pr, FP64)
                const bool mlds = pl * pr <= SMAX * (SMAX + 1);
                double* mr = mlds ? s_vre : scr;
                double* mi = mlds ? s_vim : scr + (size_t)pl * pr;
                for (int idx = tid; idx < pl * pr; idx += NT) {
                    const int a = idx / pr, b = idx - a * pr;
                    const int i0 = (a * 2) * pr + b, i1 = i0 + pr;
                    const double x0r = Pv.re[i0], x0i = Pv.im[i0], x1r = Pv.re[i1], x1i = Pv.im[i1];
                    mr[idx] = p0r * x0r + p0i * x0i + p1r * x1r + p1i * x1i;
                    mi[idx] = p0r * x0i - p0i * x0r + p1r * x1i - p1i * x1r;
                }
                __syncthreads();
                int newb;
                if (side) {
                    // product on k+1: new A[k+1] = A[k] M  (ol, 2, pr)
                    const int ol = s_chi[k];
                    for (int idx = tid; idx < ol * 2 * pr; idx += NT) {
                        const int row = idx / pr, c = idx - row * pr;
                        double xr = 0.0, xi = 0.0;
                        for (int b = 0; b < pl; ++b) {
                            const double ar = Ov.re[row * pl + b], ai = Ov.im[row * pl + b];
                            const double br = mr[b * pr + c], bi = mi[b * pr + c];
                            xr += ar * br - ai * bi;
                            xi += ar * bi + ai * br;
                        }
                        Pv.re[idx] = T(xr);
                        Pv.im[idx] = T(xi);
                    }
                    newb = ol;
                } else {
                    // product on k: new A[k] = M A[k+1]  (pl, 2, ocr)
                    const int ocr = s_chi[k + 2];
                    const int w = 2 * ocr;
                    for (int idx = tid; idx < pl * w; idx += NT) {
                        const int a = idx / w, rem = idx - a * w;
                        double xr = 0.0, xi = 0.0;
                        for (int b = 0; b < pr; ++b) {
                            const double ar = mr[a * pr + b], ai = mi[a * pr + b];
                            const double br = Ov.re[b * w + rem], bi = Ov.im[b * w + rem];
                            xr += ar * br - ai * bi;
                            xi += ar * bi + ai * br;
                        }
                        Pv.re[idx] = T(xr);
                        Pv.im[idx] = T(xi);
                    }
                    newb = ocr;
                }
                __syncthreads();
                // the unentangled qubit on the other site: psi (x) identity
                for (int idx = tid; idx < newb * 2 * newb; idx += NT) {
                    const int a = idx / (2 * newb), rem = idx - a * 2 * newb;
                    const int i = rem / newb, a2 = rem - i * newb;
                    const bool on = a == a2;
                    Ov.re[idx] = T(on ? (i ? p1r : p0r) : 0.0);
                    Ov.im[idx] = T(on ? (i ? p1i : p0i) : 0.0);
                }
                if (tid == 0) s_chi[k + 1] = newb;
                __syncthreads();
            } else if (op.kind == OP_MEAS) {
                const int k = op.a;
                SiteView<T> v = site(k);
                const int cl = s_chi[k], cr = s_chi[k + 1];
                double pp[2] = {0.0, 0.0};
                for (int idx = tid; idx < cl * cr; idx += NT) {
                    const int a = idx / cr, b = idx - a * cr;
                    const int i0 = (a * 2) * cr + b, i1 = i0 + cr;
                    const double x0r = v.re[i0], x0i = v.im[i0], x1r = v.re[i1], x1i = v.im[i1];
                    pp[0] += x0r * x0r + x0i * x0i;
                    pp[1] += x1r * x1r + x1i * x1i;
                }
                block_sum<2>(pp, s_red);
                const double tot = pp[0] + pp[1];
                int e;
                if (P.calibrate) e = pp[1] > pp[0] ? 1 : 0;
                else e = P.expected[op.aux];
                const double raw = pp[e];
                const double pe = tot > 0.0 ? raw / tot : 0.0;
                if (P.calibrate && tid == 0) {
                    P.cal_p[op.aux] = pe;
                    P.cal_e[op.aux] = static_cast<uint8_t>(e);
                }
                if (!(pe >= P.tau_rej)) {
                    alive = false;
                    status |= MSC_SHOT_REJECTED;
                    rej_at = op.aux;
                    p_acc = 0.0;
                    break;
                }
                p_acc *= pe;
                const double sc = 1.0 / sqrt(raw);
                for (int idx = tid; idx < cl * cr; idx += NT) {
                    const int a = idx / cr, b = idx - a * cr;
                    const int ie = (a * 2 + e) * cr + b, io = (a * 2 + 1 - e) * cr + b;
                    v.re[ie] = T(static_cast<double>(v.re[ie]) * sc);
                    v.im[ie] = T(static_cast<double>(v.im[ie]) * sc);
                    v.re[io] = T(0);
                    v.im[io] = T(0);
                }
                if (tid == 0) s_laste[k] = e;
                __syncthreads();
            } else if (op.kind == OP_FINAL) {
                const int k = op.a;
                SiteView<T> v = site(k);
                const int cl = s_chi[k], cr = s_chi[k + 1];
                double r[4] = {0.0, 0.0, 0.0, 0.0};   // r00, r11, Re r01, Im r01
                for (int idx = tid; idx < cl * cr; idx += NT) {
                    const int a = idx / cr, b = idx - a * cr;
                    const int i0 = (a * 2) * cr + b, i1 = i0 + cr;
                    const double x0r = v.re[i0], x0i = v.im[i0], x1r = v.re[i1], x1i = v.im[i1];
                    r[0] += x0r * x0r + x0i * x0i;
                    r[1] += x1r * x1r + x1i * x1i;
                    // rho01 = x0 * conj(x1)
                    r[2] += x0r * x1r + x0i * x1i;
                    r[3] += x0i * x1r - x0r * x1i;
                }
                block_sum<4>(r, s_red);
                const double tr = r[0] + r[1];
                // f = |t0|^2 rho00 + |t1|^2 rho11 + 2 Re(conj(t0) t1 rho01)
                const double ctr = P.t0r * P.t1r + P.t0i * P.t1i;   // conj(t0) t1
                const double cti = P.t0r * P.t1i - P.t0i * P.t1r;
                const double f = ((P.t0r * P.t0r + P.t0i * P.t0i) * r[0] +
                                  (P.t1r * P.t1r + P.t1i * P.t1i) * r[1] +
                                  2.0 * (ctr * r[2] - cti * r[3])) / tr;
                infid = fmax(0.0, 1.0 - f);
            }
            if (twosite) {
                // ---- two-site update on sites k, k+1
                const int k = op.a, dir = op.b;
                const int cl = s_chi[k], cm = s_chi[k + 1], cr = s_chi[k + 2];
                const int m = 2 * cl, n = 2 * cr;
                SiteView<T> A = site(k), B = site(k + 1);
                // theta's copy for the projection: LDS staging when it fits
                double* thr = 2 * (size_t)m * n <= (size_t)kStage ? s_u : scr;
                double* thi = thr + (size_t)m * n;
                const int nv = dir ? n : m, len = dir ? m : n;
                const int ld = len + 1;
                const bool lds = nv <= SMAX && len <= SMAX;
                double* vre = lds ? s_vre : scr + 2 * (size_t)m * n;
                double* vim = lds ? s_vim : vre + (size_t)nv * ld;
                double* nrm = lds ? s_nrm : g_nrm;
                int* sel = lds ? s_sel : g_sel;
                int* bad = lds ? s_bad : g_bad;
                int* list = lds ? s_list : g_list;
                if (tid < 4) {
                    // the 4x4 gates of the op stream are monomial: one
                    // nonzero per row, found here once per update
                    const double* g = P.g4 + gate_id * 32 + tid * 8;
                    int src = 0;
                    for (int j = 1; j < 4; ++j)
                        if (fabs(g[2 * j]) + fabs(g[2 * j + 1]) > fabs(g[2 * src]) + fabs(g[2 * src + 1]))
                            src = j;
                    s_gsrc[tid] = src;
                    s_gph[2 * tid] = g[2 * src];
                    s_gph[2 * tid + 1] = g[2 * src + 1];
                }
                // both site tensors into LDS with one coalesced pass when they
                // fit: the contraction then reads each element from LDS
                const int na = cl * 2 * cm, nb = cm * 2 * cr;
                const T* Ar = A.re;
                const T* Ai = A.im;
                const T* Br = B.re;
                const T* Bi = B.im;
                if ((size_t)2 * (na + nb) * sizeof(T) <= kStage * sizeof(double)) {
                    T* st = reinterpret_cast<T*>(s_u);
                    for (int i = tid; i < na; i += NT) {
                        st[i] = A.re[i];
                        st[na + i] = A.im[i];
                    }
                    for (int i = tid; i < nb; i += NT) {
                        st[2 * na + i] = B.re[i];
                        st[2 * na + nb + i] = B.im[i];
                    }
                    Ar = st;
                    Ai = st + na;
                    Br = st + 2 * na;
                    Bi = Br + nb;
                }
                __syncthreads();
                double nsum[1] = {0.0};
                for (int idx = tid; idx < cl * cr; idx += NT) {
                    const int a = idx / cr, b = idx - a * cr;
                    T sr[4] = {T(0), T(0), T(0), T(0)}, si[4] = {T(0), T(0), T(0), T(0)};
                    const T* a0r = Ar + (a * 2) * cm;
                    const T* a0i = Ai + (a * 2) * cm;
                    for (int c = 0; c < cm; ++c) {
                        const T x0r = a0r[c], x0i = a0i[c], x1r = a0r[cm + c], x1i = a0i[cm + c];
                        const int b0 = (c * 2) * cr + b, b1 = b0 + cr;
                        const T y0r = Br[b0], y0i = Bi[b0], y1r = Br[b1], y1i = Bi[b1];
                        // S[i'j'] += A[a,i',c] B[c,j',b]
                        sr[0] += x0r * y0r - x0i * y0i; si[0] += x0r * y0i + x0i * y0r;
                        sr[1] += x0r * y1r - x0i * y1i; si[1] += x0r * y1i + x0i * y1r;
                        sr[2] += x1r * y0r - x1i * y0i; si[2] += x1r * y0i + x1i * y0r;
                        sr[3] += x1r * y1r - x1i * y1i; si[3] += x1r * y1i + x1i * y1r;
                    }
                    // monomial gate: output o = phase[o] * S[src[o]]
                    double tr_[4], ti_[4];
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int j = s_gsrc[o];
                        const double xr = static_cast<double>(sr[j]), xi = static_cast<double>(si[j]);
                        const double pr = s_gph[2 * o], pim = s_gph[2 * o + 1];
                        tr_[o] = pr * xr - pim * xi;
                        ti_[o] = pr * xi + pim * xr;
                    }
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int i = o >> 1, j = o & 1;
                        const int row = a * 2 + i, col = j * cr + b;
                        const size_t vi = dir ? (size_t)col * ld + row : (size_t)row * ld + col;
                        vre[vi] = tr_[o];
                        vim[vi] = ti_[o];
                        nsum[0] += tr_[o] * tr_[o] + ti_[o] * ti_[o];
                    }
                }
                block_sum<1>(nsum, s_red);
                const double total = nsum[0];
                const double tau2 = P.tau * P.tau;
                const double floor2 = 1e-4 * tau2 * total;
                // orthogonality tolerance: a few ulps of the tensor precision
                const double tol = sizeof(T) == sizeof(double)
                                       ? static_cast<double>(len) * DBL_EPSILON
                                       : 8.0 * static_cast<double>(FLT_EPSILON);
                // squared norms, then one parallel pass over every pair: if
                // all vectors are already orthogonal (the common case) no
                // Jacobi sweep is needed at all
                vector_norms(vre, vim, nv, len, ld, nrm);
                const bool rotated =
                    not_orthogonal(vre, vim, nv, len, ld, nrm, floor2, tol, bad, nullptr);
                if (rotated) {
                    // keep theta for the projection (the vectors still hold it)
                    for (int idx = tid; idx < m * n; idx += NT) {
                        const int row = idx / n, col = idx - row * n;
                        const size_t vi = dir ? (size_t)col * ld + row : (size_t)row * ld + col;
                        thr[idx] = vre[vi];
                        thi[idx] = vim[vi];
                    }
                    // sweep until the parallel check finds every pair orthogonal
                    // only vectors of an overlapping pair need rotating: the
                    // others stay orthogonal to every combination of them
                    int sweeps = 0;
                    bool again = true;
                    while (again && sweeps < 40) {
                        const int nb = flagged_list(bad, nv, list, s_ired);
                        jacobi_sweep(vre, vim, list, nb, len, ld, floor2, tol);
                        ++sweeps;
                        vector_norms(vre, vim, nv, len, ld, nrm);
                        for (int v = tid; v < nv; v += NT) sel[v] = bad[v];
                        __syncthreads();
                        again = not_orthogonal(vre, vim, nv, len, ld, nrm, floor2, tol, bad, sel);
                    }
                    if (again) status |= MSC_SHOT_NOCONV;
                    sweeps_total += sweeps;
                }
                const int capb = min(P.chi_max, s_cap[k + 1]);
                const Kept kp = select_kept(nrm, nv, tau2, capb, sel, s_red);
                const int r = kp.r;
                const double kept = kp.kept;
                disc += kp.dropped;
                if (kp.dropped > 1e-12 * total && r == capb) status |= MSC_SHOT_CHI_CAP;
                const double renorm = 1.0 / sqrt(kept);
                // isometric factor: normalised vectors; centre factor: the
                // projection of theta on them.  When no rotation was needed the
                // vectors are theta's own columns (rows), so the projection is
                // sigma_c on the selected column (row) and zero elsewhere, up
                // to overlaps below the orthogonality tolerance.
                if (!rotated) {
                    if (dir) {
                        for (int idx = tid; idx < m * r; idx += NT) {
                            const int row = idx / r, c = idx - row * r;
                            const int v = sel[c];
                            const double is = 1.0 / sqrt(nrm[v]);
                            A.re[idx] = T(vre[(size_t)v * ld + row] * is);
                            A.im[idx] = T(vim[(size_t)v * ld + row] * is);
                        }
                        for (int idx = tid; idx < r * n; idx += NT) {
                            const int c = idx / n, col = idx - c * n;
                            const int v = sel[c];
                            B.re[idx] = T(col == v ? sqrt(nrm[v]) * renorm : 0.0);
                            B.im[idx] = T(0);
                        }
                    } else {
                        for (int idx = tid; idx < r * n; idx += NT) {
                            const int c = idx / n, col = idx - c * n;
                            const int v = sel[c];
                            const double is = 1.0 / sqrt(nrm[v]);
                            B.re[idx] = T(vre[(size_t)v * ld + col] * is);
                            B.im[idx] = T(vim[(size_t)v * ld + col] * is);
                        }
                        for (int idx = tid; idx < m * r; idx += NT) {
                            const int row = idx / r, c = idx - row * r;
                            const int v = sel[c];
                            A.re[idx] = T(row == v ? sqrt(nrm[v]) * renorm : 0.0);
                            A.im[idx] = T(0);
                        }
                    }
                } else if (dir) {
                    // A[k] (cl,2,r): U[row][c] = w_sel[c][row] / |w|
                    for (int idx = tid; idx < m * r; idx += NT) {
                        const int row = idx / r, c = idx - row * r;
                        const int v = sel[c];
                        const double is = 1.0 / sqrt(nrm[v]);
                        A.re[idx] = T(vre[(size_t)v * ld + row] * is);
                        A.im[idx] = T(vim[(size_t)v * ld + row] * is);
                    }
                    // A[k+1] (r,2,cr): R[c][col] = sum_row conj(U[row][c]) theta[row][col]
                    for (int idx = tid; idx < r * n; idx += NT) {
                        const int c = idx / n, col = idx - c * n;
                        const int v = sel[c];
                        const double is = renorm / sqrt(nrm[v]);
                        const double* ur = vre + (size_t)v * ld;
                        const double* ui = vim + (size_t)v * ld;
                        double xr = 0.0, xi = 0.0;
                        for (int row = 0; row < m; ++row) {
                            const double a0 = ur[row], a1 = ui[row];
                            const double t0 = thr[(size_t)row * n + col], t1 = thi[(size_t)row * n + col];
                            xr += a0 * t0 + a1 * t1;
                            xi += a0 * t1 - a1 * t0;
                        }
                        B.re[idx] = T(xr * is);
                        B.im[idx] = T(xi * is);
                    }
                } else {
                    // A[k+1] (r,2,cr): V[c][col] = w_sel[c][col] / |w|
                    for (int idx = tid; idx < r * n; idx += NT) {
                        const int c = idx / n, col = idx - c * n;
                        const int v = sel[c];
                        const double is = 1.0 / sqrt(nrm[v]);
                        B.re[idx] = T(vre[(size_t)v * ld + col] * is);
                        B.im[idx] = T(vim[(size_t)v * ld + col] * is);
                    }
                    // A[k] (cl,2,r): L[row][c] = sum_col theta[row][col] conj(V[c][col])
                    for (int idx = tid; idx < m * r; idx += NT) {
                        const int row = idx / r, c = idx - row * r;
                        const int v = sel[c];
                        const double is = renorm / sqrt(nrm[v]);
                        const double* wr = vre + (size_t)v * ld;
                        const double* wi = vim + (size_t)v * ld;
                        double xr = 0.0, xi = 0.0;
                        for (int col = 0; col < n; ++col) {
                            const double t0 = thr[(size_t)row * n + col], t1 = thi[(size_t)row * n + col];
                            const double b0 = wr[col], b1 = wi[col];
                            xr += t0 * b0 + t1 * b1;
                            xi += t1 * b0 - t0 * b1;
                        }
                        A.re[idx] = T(xr * is);
                        A.im[idx] = T(xi * is);
                    }
                }
                __syncthreads();
                if (tid == 0) s_chi[k + 1] = r;
                chi_peak = max(chi_peak, r);
                ++n2q;
                {
                    const double dl = cl, dm = cm, dr = cr, dk = r;
                    flops += 32.0 * dl * dm * dr + 32.0 * dl * dl * dr + 32.0 * dk * dl * dr +
                             104.0 * dl * dl * dl;
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            msc_shot_result res;
            res.p_acc = p_acc;
            res.infid = alive ? infid : 0.0;
            res.disc_weight = disc;
            res.chi_peak = chi_peak;
            res.status = status | (alive ? MSC_SHOT_DONE : 0);
            res.rejected_at = rej_at;
            res.fail = (alive && p_acc > 0.0 && infid > P.tau_fail) ? 1 : 0;
            res.n2q = n2q;
            res.flops = flops;
            res.sweeps = sweeps_total;
            P.out[it] = res;
        }
        __syncthreads();
    }
}

// Processing order of the shots: a stable counting sort into 16 buckets,
// the longest-running shots first so that the tail of the persistent grid
// stays short.  Without checkpoints the key is the fault count (capped at
// 15): low-weight shots are the ones that run to the end of the circuit,
// online screening stops the others early.  With checkpoints a shot starts
// at its first fault, so the key is the position of that channel in the
// circuit (fault-free shots, which only read out, last).
__global__ __launch_bounds__(1024) void order_kernel(int64_t n, const int64_t* shot_off,
                                                     const int64_t* shot_idx, int64_t n_csr,
                                                     const int32_t* chan, int32_t n_channels,
                                                     int64_t* perm) {
    __shared__ int64_t s_base;
    __shared__ int s_wcnt[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_base = 0;
    __syncthreads();
    for (int key = 0; key < 16; ++key) {
        for (int64_t base = 0; base < n; base += 1024) {
            const int64_t j = base + tid;
            bool hit = false;
            if (j < n) {
                const int64_t sh = shot_idx ? shot_idx[j] : j;
                int c = 15;
                if (sh >= 0 && sh < n_csr) {
                    const int64_t f0 = shot_off[sh], f = shot_off[sh + 1] - f0;
                    if (n_channels > 0) {
                        const int64_t ch = f > 0 ? chan[f0] : n_channels;
                        c = ch < 0 ? 0 : ch >= n_channels ? 15
                                                          : static_cast<int>(ch * 15 / n_channels);
                    } else {
                        c = f < 15 ? static_cast<int>(f) : 15;
                    }
                }
                hit = c == key;
            }
            const uint64_t m = __ballot(hit);
            if (lane == 0) s_wcnt[w] = __popcll(m);
            __syncthreads();
            int64_t off = s_base;
            for (int q = 0; q < w; ++q) off += s_wcnt[q];
            if (hit) perm[off + __popcll(m & ((1ull << lane) - 1ull))] = j;
            __syncthreads();
            if (tid == 0) {
                int64_t t = 0;
                for (int q = 0; q < 16; ++q) t += s_wcnt[q];
                s_base += t;
            }
            __syncthreads();
        }
    }
}

}  // namespace

int mps_blocks_per_cu(int precision, bool small) {
    int b = 0;
    hipError_t e;
    if (precision == MSC_FP64)
        e = small ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mps_kernel<double, 32>, NT, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mps_kernel<double, 64>, NT, 0);
    else
        e = small ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mps_kernel<float, 32>, NT, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, mps_kernel<float, 64>, NT, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return b < 1 ? 1 : b;
}

hipError_t launch_order(int64_t n, const int64_t* shot_off, const int64_t* shot_idx, int64_t n_csr,
                        const int32_t* chan, int32_t n_channels, int64_t* perm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, s, n, shot_off, shot_idx, n_csr, chan,
                       n_channels, perm);
    return hipGetLastError();
}

hipError_t launch_mps(int precision, bool small, const MpsArgs& a, int grid, hipStream_t s) {
    if (precision == MSC_FP64) {
        if (small) hipLaunchKernelGGL((mps_kernel<double, 32>), dim3(grid), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((mps_kernel<double, 64>), dim3(grid), dim3(NT), 0, s, a);
    } else {
        if (small) hipLaunchKernelGGL((mps_kernel<float, 32>), dim3(grid), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((mps_kernel<float, 64>), dim3(grid), dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace msc
