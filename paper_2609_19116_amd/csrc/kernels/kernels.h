// Launch interfaces of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../msc_internal.h"

namespace msc {

constexpr int kMaxSites = 128;     // MPS sites per circuit
constexpr int kMaxChiKernel = 1024; // bond cap handled by the shot kernels

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

// Slot states of the shot kernel when large updates are handed to the
// batched engine (ShotState.status)
enum SlotStatus : int32_t {
    kSlotRun = 0,      // start the slot's next shot (first launch)
    kSlotParked = 1,   // waiting at a large two-site update
    kSlotResume = 2,   // the update is done: continue after it
    kSlotDone = 3      // no shots left for this slot
};

// Everything a shot carries between ops, saved when it parks at a large
// two-site update (one record per slot, device memory) and restored when it
// resumes after the batched engine has done that update.
struct ShotState {
    int64_t j;                 // position in the slot's sequence of shots
    int64_t fcur, fend;        // fault cursor in the CSR
    int64_t ck_pos;            // record mode: checkpoint elements written
    int64_t n2q, sweeps;       // per-shot counters
    double p_acc, infid, disc, flops;
    int32_t status;            // SlotStatus
    int32_t oi;                // op to resume at
    int32_t next_ch, fcode;
    int32_t meas_done, next_seg, rej_at, alive;
    int32_t next_ck, ck_full;
    int32_t shot_status, chi_peak;
    // the parked update: sites k, k+1, centre direction, 4x4 gate id
    int32_t k, dir, gate_id, pad;
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
    // batched large updates: a two-site update whose theta has a side above
    // park_side (0: never) parks the shot (state[slot], slot appended to
    // park_list, park_count incremented) and its workgroup exits; a later
    // launch with the same arguments resumes every slot marked kSlotResume.
    // state == nullptr: no parking, every slot starts at its first shot.
    int32_t park_side;
    ShotState* state;
    int32_t* park_count;
    int32_t* park_list;
    // the wavefront kernel: shots taken from the shared counter next (zero
    // at the launch); a shot that outgrows its slot's bond cap (below
    // chi_max) appends its index in the run to retry_list and yields no
    // result there.  Both nullptr for the workgroup kernel.
    unsigned long long* next;
    int32_t* retry_count;
    int64_t* retry_list;
};

// precision: MSC_FP64 or MSC_FP32; small: use the 32-wide LDS variant
hipError_t launch_mps(int precision, bool small, const MpsArgs& a, int grid, hipStream_t s);
// perm[0..n): stable order of the shots, by fault count (fewest first) or,
// with n_channels > 0, by first faulty channel (earliest first, fault-free
// shots last): the order in which their remaining work shrinks
hipError_t launch_order(int64_t n, const int64_t* n_dev, const int64_t* shot_off,
                        const int64_t* shot_idx, int64_t n_csr, const int32_t* chan,
                        int32_t n_channels, int64_t* perm, void* tmp, hipStream_t s);
// bytes of launch_order's tmp for n entries (per-chunk key counts and offsets)
int64_t order_tmp_bytes(int64_t n);
// resident workgroups per CU of the chosen variant (sizes the persistent grid)
int mps_blocks_per_cu(int precision, bool small);
// One shot per wavefront (four per workgroup of 256 threads): grid
// workgroups serve 4 * grid slots.  Needs next (zeroed), retry_count and
// retry_list; ck_mode 0, 1 or 2; no calibration and no parking.
hipError_t launch_mps_wave(int precision, const MpsArgs& a, int grid, hipStream_t s);
int mps_wave_blocks_per_cu(int precision);
constexpr int kWaveTeams = 4;      // shots per workgroup of the wavefront kernel

// Bits of the CSR check flag written by the screen and validation kernels
enum CsrFlag : int {
    CSR_BAD_CHANNEL = 1,     // channel index outside [0, M)
    CSR_NOT_ASCENDING = 2,   // channels of a shot not strictly ascending
    CSR_BAD_PAULI = 4,       // Pauli code zero or beyond the channel's qubits
    CSR_BAD_OFFSETS = 8      // shot_off decreasing or negative
};
// sig: per (channel, Pauli code) the fault's W-word signature; sig_off[c]
// holds the index of channel c's first entry shifted left by two with the
// channel's ChanKind in the low two bits (code_limit(kind) entries); kind:
// ChanKind per channel (uint8); flag: one device int, cleared first
hipError_t launch_prescreen(int words, int32_t n_channels, int64_t n, const int64_t* off, const int32_t* chan,
                            const uint8_t* pauli, const uint64_t* sig, const int32_t* sig_off,
                            const uint8_t* kind,
                            uint64_t* survive_bits, int64_t* survivor_idx, int64_t* block_tmp,
                            int64_t n_blocks_tmp, int* flag, hipStream_t s);
int64_t prescreen_tmp_words(int64_t n);
hipError_t launch_validate_csr(int32_t n_channels, int64_t n, const int64_t* off,
                               const int32_t* chan, const uint8_t* pauli, const uint8_t* kind,
                               int* flag, hipStream_t s);
// Fixed device scratch of msc_prescreen_noalloc (prescreen.hip): at most
// kNoAllocShots shots per call; the words hold the block counts and their
// scan, the superblock totals, the survivor total and the CSR flag.  prescreen_noalloc_scratch(device) resolves the array's
// address on `device` (which must be current) once and caches it.
constexpr int64_t kNoAllocShots = int64_t(1) << 26;
hipError_t prescreen_noalloc_scratch(int device, int64_t** out);

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
// shots, sum P_acc, sum P_acc*fail, accepted, wrong, sum P_acc^2, sum (P_acc*fail)^2
constexpr int kBinRows = 7;
// surv (optional): per survivor n_seg reach probabilities, summed per bin
// into sbins[b * n_seg + s]
hipError_t launch_batch_reduce(int64_t n, uint64_t seed, uint64_t first, const int64_t* off,
                               const int64_t* idx, const int64_t* n_surv,
                               const msc_shot_result* res, int nb, const int64_t* nnz,
                               double* bins, BatchTotals* tot, const double* surv, int n_seg,
                               double* sbins, void* tmp, hipStream_t s);
// bytes of launch_batch_reduce's tmp (per-chunk partial sums)
int64_t batch_reduce_tmp_bytes(int64_t n, int nb, int n_seg);
// idx[i] = i for i < n and *count = n (every shot a survivor)
hipError_t launch_identity(int64_t n, int64_t* idx, int64_t* count, hipStream_t s);
hipError_t launch_scatter_results(int64_t n, const int64_t* n_surv, const int64_t* idx,
                                  const msc_shot_result* res, msc_shot_result* out,
                                  hipStream_t s);

hipError_t launch_twosite(int precision, int chi, int batch, const float* A, const float* B,
                          const float* gate, float* theta, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched engine for large two-site updates (lx.hip, mps.hip): the shots
// parked by the shot kernel (MpsArgs.park_*) are updated together.
//   plan:     per parked shot its shapes and tile counts, prefix sums
//   contract: theta = G (A[k] A[k+1]) on MFMA, ragged shapes, one tile list
//   gram:     G = V^H V of theta's vectors (columns if the centre moves
//             right, rows if left) in FP64 on MFMA, upper block triangle
//   factor:   (mps.hip) eigen-decomposition of the overlapping vectors'
//             block, rotation, selection, new site tensors, slot resumed
// Every kernel takes its counts from device memory (LxPlan), so a launch
// sequence does not depend on what the shot kernel parked (graph capture).
constexpr int kLxMaxParked = 8192;
// buckets of parked shots by theta's larger side: <= 128, <= 256, <= 512, more
constexpr int kLxBuckets = 4;
__host__ __device__ inline int lx_bucket(int side) {
    return side <= 128 ? 0 : side <= 256 ? 1 : side <= 512 ? 2 : 3;
}
struct LxBucket {
    int32_t count;                     // parked shots in the bucket
    int32_t ctiles, gtiles;            // total contraction / Gram tiles
    int32_t pad;
    int32_t slot[kLxMaxParked];        // slot of the bucket's shot i
    int32_t coff[kLxMaxParked + 1];    // first contraction tile of shot i
    int32_t goff[kLxMaxParked + 1];    // first Gram tile of shot i
};
struct LxPlan {
    int32_t count;                     // parked shots
    int32_t pad[3];
    int32_t slot[kLxMaxParked];        // slot of parked shot i (park order)
    LxBucket b[kLxBuckets];
};
struct LxArgs {
    const ShotState* state;            // per slot
    const int32_t* park_count;
    const int32_t* park_list;
    LxPlan* plan;
    void* arena;                       // slot tensors (element type T)
    int64_t slot_stride;
    const int64_t* site_off;           // per site offset of the Re plane
    const int64_t* site_half;          // Im plane offset from the Re plane
    const double* g4;                  // 4x4 gates, 32 doubles each
    void* theta;                       // per slot theta (T), theta_stride elements
    int64_t theta_stride;
    double* gram;                      // per slot Gram (FP64 planar), gram_stride doubles
    int64_t gram_stride;
    int32_t n_slots;
    double* flops;                     // [2] running algorithmic flops: contractions
                                       // (32 cl cm cr each), Gram matrices (4 nv (nv+1) len)
    unsigned long long* counts;        // [4] factor steps in LDS, in the workspace
                                       // (many overlapping vectors), overlapping vectors
                                       // summed, Jacobi sweeps summed
};
// contraction tile (rows of (a, i) x b columns of both j') and Gram tile sizes
struct LxTiles {
    int32_t cm_rows, cm_b;             // contraction tile: rows (a,i) and b values
    int32_t gram;                      // Gram tile side
};
// precision: MSC_FP32 (FP32 MFMA), MSC_BF16X3 (bf16 hi/lo split), MSC_FP64;
// t[kLxBuckets]: the tiles of each bucket
hipError_t launch_lx_plan(const LxArgs& a, const LxTiles* t, hipStream_t s);
hipError_t launch_lx_contract(int precision, const LxArgs& a, int bucket, const LxTiles& t,
                              int grid, hipStream_t s);
hipError_t launch_lx_gram(int precision, const LxArgs& a, int bucket, const LxTiles& t,
                          int grid, hipStream_t s);
// slot states to kSlotRun, the park count and the flop counters to 0 (a
// kernel, not a memset)
hipError_t launch_lx_reset(ShotState* state, int n_slots, int32_t* park_count, double* flops,
                           unsigned long long* counts, hipStream_t s);
// the park count to 0
hipError_t launch_lx_clear(int32_t* park_count, hipStream_t s);
// the tile shapes compiled for a precision (autotuner candidates)
int lx_tile_variants(int precision, LxTiles* out, int cap);
// factor step of the engine (mps.hip); the slot's Gram buffer doubles as
// its FP64 workspace once the Gram matrix has been read
struct LxFactor {
    const int32_t* cap;                // bond capacities [n_sites + 1]
    int32_t chi_max;
    double tau;                        // keep sigma_i > tau * sigma_0
};
constexpr int kLxFactorMax = 64;       // overlapping vectors diagonalised in LDS
hipError_t launch_lx_factor(int precision, const LxArgs& a, const LxFactor& f, int grid,
                            hipStream_t s);
// doubles of one slot's Gram buffer for theta sides up to S: the Gram
// matrix (2 S^2), or the workspace of rotated vectors (2 S (S + 1)), then
// the per-vector arrays (7 S)
inline int64_t lx_gram_doubles(int64_t S) { return 2 * S * (S + 1) + 7 * S + 64; }

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
