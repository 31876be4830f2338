// Launch interfaces of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../msc_internal.h"

namespace msc {

constexpr int kMaxSites = 128;     // MPS sites per circuit
constexpr int kMaxChiKernel = 256; // bond cap handled by the shot kernel

// Header of one noiseless-prefix checkpoint: the shot state right before a
// given op of the noiseless run (the tensors themselves are stored densely,
// site after site, real plane then imaginary plane, at ck_off[j]).
struct CkHdr {
    double p_acc, disc;
    int32_t chi_peak, status;
    int32_t meas_done, pad;    // measurements before the checkpoint's op
    int32_t chi[kMaxSites + 1];
    int32_t laste[kMaxSites];
};

struct MpsArgs {
    const DevOp* ops;
    int32_t n_ops;
    int32_t n_sites;
    const double* g1;          // 2x2 complex gates, 8 doubles each
    const double* g4;          // 4x4 complex gates, 32 doubles each
    const int64_t* shot_off;   // fault CSR
    const int32_t* chan;
    const uint8_t* pauli;
    const int64_t* shot_idx;   // optional subset
    const int64_t* perm;       // processing order of the n_shots entries
    int64_t n_shots;           // shots to simulate (entries of shot_idx)
    const int64_t* n_dev;      // if set: the count on the device (<= n_shots)
    int64_t n_csr;             // shots held by the CSR
    const uint8_t* expected;   // e_m per measurement
    msc_shot_result* out;
    void* arena;               // n_slots * slot_stride elements of T
    int64_t slot_stride;
    const int64_t* site_off;   // per-site offset (elements of T) of Re part
    const int64_t* site_half;  // per-site offset of Im part from Re part
    const int32_t* cap;        // bond capacities [n_sites + 1]
    double* scratch;           // n_slots * scratch_stride doubles
    int64_t scratch_stride;
    int32_t chi_max;
    double tau;                // keep sigma > tau * sigma_0
    double tau_rej;
    double tau_fail;
    double t0r, t0i, t1r, t1i; // target state amplitudes
    int32_t calibrate;         // 1: choose the likelier outcome and record it
    double* cal_p;             // [n_meas] probability of the chosen outcome
    uint8_t* cal_e;            // [n_meas] chosen outcome
    // noiseless-prefix checkpoints: ck_mode 0 off, 1 record them from the
    // (single, fault-free) shot, 2 start every shot from one of them
    int32_t ck_mode;
    int32_t n_ck;              // checkpoint j < n_ck - 1 sits before the fault
                               // op of channel j * ck_k, the last before OP_FINAL
    int32_t ck_k;
    const int32_t* ck_op;      // [n_ck] op index of each checkpoint
    int32_t* ck_avail;         // checkpoints written (record) / usable (fork)
    int64_t* ck_off;           // [n_ck] element offset of each checkpoint's tensors
    CkHdr* ck_hdr;             // [n_ck]
    void* ck_data;             // ck_cap elements of T
    int64_t ck_cap;
    double* ck_pm;             // [n_meas] noiseless running P_acc before each
                               // measurement (written when recording)
    // optional reach probabilities: surv[out index * n_seg + s] = P_acc
    // before measurement seg_meas[s] (0 after a rejection)
    double* surv;
    const int32_t* seg_meas;
    int32_t n_seg;
};

// precision: MSC_FP64 or MSC_FP32; small: use the 32-wide LDS variant
hipError_t launch_mps(int precision, bool small, const MpsArgs& a, int grid, hipStream_t s);
// perm[0..n): stable order of the shots, by fault count (fewest first) or,
// with n_channels > 0, by first faulty channel (earliest first, fault-free
// shots last): the order in which their remaining work shrinks
hipError_t launch_order(int64_t n, const int64_t* n_dev, const int64_t* shot_off,
                        const int64_t* shot_idx, int64_t n_csr, const int32_t* chan,
                        int32_t n_channels, int64_t* perm, hipStream_t s);
// resident workgroups per CU of the chosen variant (sizes the persistent grid)
int mps_blocks_per_cu(int precision, bool small);

hipError_t launch_prescreen(int words, int32_t n_channels, int64_t n, const int64_t* off, const int32_t* chan,
                            const uint8_t* pauli, const uint64_t* sig, uint64_t* survive_bits,
                            int64_t* survivor_idx, int64_t* block_tmp, int64_t n_blocks_tmp,
                            hipStream_t s);
int64_t prescreen_tmp_words(int64_t n);

// device fault sampler: CSR of shots first .. first+n-1 (see sampler.hip);
// tmp holds sampler_tmp_words(n) int64, its last used entry the nnz total
hipError_t launch_sampler(int64_t n, uint64_t seed, uint64_t first, const int32_t* weights,
                          const double* cdf, int32_t n_cdf, int64_t M, const uint8_t* kind,
                          int64_t nnz_cap, int64_t* shot_off, int32_t* chan, uint8_t* pauli,
                          int64_t* tmp, int64_t n_tmp, hipStream_t s);
int64_t sampler_tmp_words(int64_t n);

// batch reduction into host-mapped memory (batch.hip)
constexpr int kMaxBins = 1024;
struct BatchTotals {
    int64_t nnz, n_survivors, n_accepted, n2q, sweeps;
    double flops;
    int32_t chi_peak, status_or;
};
constexpr int kBinRows = 5;   // shots, sum P_acc, sum P_acc*fail, accepted, wrong
// surv (optional): per survivor n_seg reach probabilities, summed per bin
// into sbins[b * n_seg + s]
hipError_t launch_batch_reduce(int64_t n, uint64_t seed, uint64_t first, const int64_t* off,
                               const int64_t* idx, const int64_t* n_surv,
                               const msc_shot_result* res, int nb, const int64_t* nnz,
                               double* bins, BatchTotals* tot, const double* surv, int n_seg,
                               double* sbins, hipStream_t s);
// idx[i] = i for i < n and *count = n (every shot a survivor)
hipError_t launch_identity(int64_t n, int64_t* idx, int64_t* count, hipStream_t s);
hipError_t launch_scatter_results(int64_t n, const int64_t* n_surv, const int64_t* idx,
                                  const msc_shot_result* res, msc_shot_result* out,
                                  hipStream_t s);

hipError_t launch_twosite(int precision, int chi, int batch, const float* A, const float* B,
                          const float* gate, float* theta, hipStream_t s);

// ---------------------------------------------------------------------------
// CAMPS shots (camps.hip): Clifford frame + magic-residual MPS in FP64
constexpr int kCampsK = 64;        // stored bond capacity of the residual
constexpr int kCampsCap = 32;      // bond cap after every recompression
constexpr int kCampsCand = 19;     // two-qubit Clifford classes tried per bond
constexpr int64_t kCampsSiteDoubles = 4LL * kCampsK * kCampsK;   // re + im
constexpr int64_t kCampsScratch = 98304;                         // doubles per slot

// Header of one checkpoint of the noiseless CAMPS run (the frame and the
// residual right before a given op; tensors densely at ck_off[j], site by
// site, real plane then imaginary plane)
struct CampsCk {
    double p_acc;
    int64_t n_dis;
    int32_t center, status, sweeps, peak;
    int32_t chi[kMaxSites + 1];
    uint8_t laste[kMaxSites];
};

struct CampsArgs {
    const DevOp* ops;          // CAMPS op stream (CampsKind)
    int32_t n_ops;
    int32_t n;                 // qubits = residual sites
    const int32_t* site_of;    // [n] residual site of each qubit
    const int32_t* chan_q;     // [3 M] qubits of each channel (-1 unused)
    const int64_t* shot_off;
    const int32_t* chan;
    const uint8_t* pauli;
    const int64_t* shot_idx;   // optional subset
    int64_t n_shots;
    int64_t n_csr;
    const uint8_t* expected;
    msc_shot_result* out;
    double* arena;             // n_slots * n * kCampsSiteDoubles
    double* scratch;           // n_slots * kCampsScratch
    const double* dmat;        // [kCampsCand][32] candidate unitaries (re,im) row-major
    const uint8_t* dtab;       // [kCampsCand][16] Pauli map: bits x1 z1 x2 z2 | phase << 4
    int32_t chi_cap;           // <= kCampsCap
    double tau, tau_rej, tau_fail;
    double rt[3];              // Bloch vector of the target state
    // checkpoints of the noiseless run: ck_mode 0 off, 1 record them from
    // the single fault-free shot, 2 start every shot from one of them
    int32_t ck_mode, n_ck, ck_k;
    const int32_t* ck_op;      // [n_ck] op index (before channel j * ck_k's
                               // fault op, the last before CO_FINAL)
    int32_t* ck_avail;
    int64_t* ck_off;
    CampsCk* ck_hdr;
    uint64_t* ck_frame;        // [n_ck][8 * kMaxSites]: x words, then z words
                               // (2 words for each of the 2 kMaxSites rows)
    uint8_t* ck_ph;            // [n_ck][2 * kMaxSites]
    double* ck_data;
    int64_t ck_cap;
};
hipError_t launch_camps(const CampsArgs& a, int grid, hipStream_t s);
int camps_blocks_per_cu();

}  // namespace msc
