/*
 * msc.h -- C ABI of the batched exact-MPS magic-state-cultivation shot
 * simulator for MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *  - Every function that can fail returns int: MSC_OK (0) or a negative
 *    msc_status.  msc_last_error() returns a thread-local message for the
 *    most recent failure.  No C++ exception crosses this boundary.
 *  - Handles (msc_ctx, msc_circuit) are created and freed by the library.
 *    Every array is owned by the caller.  Arguments documented as "device"
 *    must be device pointers on the context's GPU (for example the data of a
 *    torch tensor); arguments documented as "host" must be host pointers.
 *  - Device entry points run on the context's stream and return after the
 *    stream has finished the call (results are ready on return).
 *
 * Circuit text format (one op per line, '#' comments):
 *   QUBITS n | ORDER q0 q1 ... (qubit held by MPS site i) | SEED q |
 *   TARGET T|S | H S SDG T TDG X Y Z q | CX CZ CS CSDG a b | CCZ a b c |
 *   M q | R q | DEP1 q | DEP2 a b | DEP3 a b c | XERR q | TICK | SEGMENT
 * CS/CSDG are controlled-S and controlled-S^dagger, CCZ the doubly
 * controlled Z: with T and T^dagger the diagonal non-Clifford gates of the
 * method (Sections 2 and 4.2).  Channels (DEP1, DEP2, DEP3, XERR) and
 * measurements are numbered in text order.
 * R is legal only as the first op on a qubit or when the last op on that
 * qubit was M.  SEGMENT starts a new segment of the circuit for the
 * space-time accounting (no action on the state; see msc_segment).
 */
#ifndef MSC_H
#define MSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum msc_status {
    MSC_OK = 0,
    MSC_E_PARSE = -1,            /* malformed circuit text                    */
    MSC_E_INVALID = -2,          /* bad argument, size or pointer             */
    MSC_E_NONDETERMINISTIC = -3, /* noiseless run: some p(e_m) != 1 or f != 1 */
    MSC_E_CAPACITY = -4,         /* caller-provided capacity too small        */
    MSC_E_DEVICE = -5,           /* HIP error (message has the HIP text)      */
    MSC_E_OOM = -6,              /* device allocation failed                  */
    MSC_E_STATE = -7             /* call not valid in the current state       */
};

enum msc_precision {
    MSC_FP64 = 0,   /* complex128 tensors and contractions                    */
    MSC_FP32 = 1,   /* complex64 tensors, FP32 contractions, FP64 truncation,
                       norms and probabilities                                */
    MSC_BF16X3 = 2  /* as MSC_FP32, but the batched engine's contractions
                       split FP32 inputs into bf16 hi + lo and take three
                       bf16 products per real product with FP32
                       accumulation (relative error ~1e-5)                   */
};

/* bits of msc_shot_result.status */
enum msc_shot_status {
    MSC_SHOT_DONE = 1,          /* reached the end of the circuit             */
    MSC_SHOT_REJECTED = 2,      /* an expected outcome had p < tau_rej        */
    MSC_SHOT_CHI_CAP = 4,       /* chi_max bound with weight > 1e-12 dropped  */
    MSC_SHOT_NOCONV = 8,        /* an SVD hit its sweep limit                 */
    MSC_SHOT_MPS_RERUN = 16     /* CAMPS only: the residual outgrew its bond
                                   cap and the shot was run again by the FP64
                                   MPS path, whose record this is            */
};

typedef struct msc_ctx msc_ctx;
typedef struct msc_circuit msc_circuit;

/* One segment of a circuit (the ops between SEGMENT lines), for the
   space-time accounting of Appendix "Space-time overhead": its volume is
   n_qubits x depth.  n_qubits counts the qubits its gates, measurements and
   resets act on; depth is the layer count of an as-soon-as-possible
   schedule of those ops (noise channels are not layers).  A shot reaches
   the segment with the product of its expected-outcome probabilities over
   measurements 0 .. first_meas - 1 (0 once one has rejected it).         */
typedef struct {
    int32_t first_meas;   /* measurements before the segment                 */
    int32_t n_qubits;
    int32_t depth;
    int32_t noisy;        /* 1 iff the segment holds a noise channel         */
} msc_segment;

typedef struct {
    int32_t n_qubits;
    int32_t n_meas;
    int32_t n_channels;   /* M of Eq. (reweight)                             */
    int32_t n_decided;    /* measurements decided by the offline screen      */
    int32_t seed_qubit;
    int32_t target;       /* 'T' or 'S'                                      */
    int32_t words;        /* uint64 words per pre-screen signature           */
    int32_t calibrated;   /* expected outcomes known (msc_circuit_calibrate) */
    int64_t n_ops;        /* compiled MPS op stream length                   */
    int64_t n_twosite;    /* two-site SVD updates in one full shot           */
    int64_t n_swaps;      /* of which routing SWAPs                          */
    int64_t n_product_swaps; /* routing SWAPs of a qubit that is unentangled
                             in every shot (a reset or measured ancilla):
                             applied without an SVD                        */
    int64_t n_moves;      /* one-site moves of the orthogonality centre      */
} msc_circuit_info;

typedef struct {
    int32_t precision;    /* msc_precision                                   */
    int32_t chi_max;      /* bond cap (must not bind in the exact regime)    */
    double tau_trunc;     /* keep sigma_i > tau_trunc * sigma_0; <= 0: auto
                             (1e-12 for MSC_FP64, 1e-5 for MSC_FP32, 1e-4
                             for MSC_BF16X3, above its ~2^-16 product error) */
    double tau_rej;       /* reject when p(e_m) < tau_rej (default 1e-6)     */
    double tau_fail;      /* logical failure iff 1 - f > tau_fail (1e-4)     */
    int32_t n_slots;      /* persistent workgroups; 0 = auto                 */
    int32_t lds_width;    /* largest two-site SVD side kept in LDS: 32 or 64;
                             larger sides use the slot's HBM scratch; 0 = 32 */
    int32_t prefix;       /* 1: fork every shot from a checkpoint of the
                             noiseless run taken before its first fault (w = 0
                             shots from the one before the read-out); the
                             checkpoints are built once per circuit and option
                             set (first call) and results are bit-identical
                             to prefix = 0.  0: every shot from |0...0>.     */
    int32_t large_side;   /* two-site updates whose theta has a side above
                             this go to the batched engine: the shot parks,
                             and the updates of all parked shots run together
                             as ragged MFMA contractions (tensor precision;
                             BF16x3 splits for MSC_BF16X3), FP64 Gram
                             matrices on MFMA and FP64 eigen-decompositions of
                             their overlapping blocks, then the shots resume.
                             0: 256; -1: off (the shot kernel factorises
                             every update itself, in HBM scratch when wide);
                             any other value must be at least 2.            */
    int32_t use_graphs;   /* 1: one engine round (its ~10 launches) is
                             captured once as a HIP graph and replayed      */
    int32_t wave_chi;     /* one shot per wavefront (four per workgroup, no
                             workgroup barriers, three times the resident
                             shots of the workgroup kernel) in slots whose
                             bonds are capped at wave_chi; a shot that would
                             need a larger bond (above the cap and below
                             chi_max) is run again from its start by the
                             workgroup kernel, so results follow chi_max.
                             0: 16 when lds_width is 0 and the circuit's
                             calibrated noiseless run stays within bond 16,
                             else off; -1: off; else 2..64.               */
    const char* autotune_cache; /* path of an msc_autotune JSON file giving
                             the engine's tile shapes per precision and bucket
                             of theta sides; NULL: built-in shapes          */
} msc_sim_opts;

typedef struct {
    double p_acc;         /* prod_m p(e_m): post-selection probability       */
    double infid;         /* 1 - |<target|rho_seed|target>| (0 if rejected)  */
    double disc_weight;   /* sum of dropped sigma^2 over the shot            */
    int32_t chi_peak;     /* largest bond dimension reached                  */
    int32_t status;       /* msc_shot_status bits                            */
    int32_t rejected_at;  /* measurement index that rejected, or -1          */
    int32_t fail;         /* 1 iff accepted (p_acc > 0) and infid > tau_fail */
    int64_t n2q;          /* two-site updates executed                       */
    double flops;         /* algorithmic flops of those updates: per update
                             32 cl cm cr (contraction) + 32 cl^2 cr (Gram)
                             + 32 r cl cr (projection) + 104 cl^3 (eigen-
                             solve) with cl, cm, cr the bonds around the two
                             sites and r the new bond                      */
    int64_t sweeps;       /* Jacobi sweeps summed over the shot's SVDs       */
} msc_shot_result;

typedef struct {
    double p_acc;         /* Eq. (reweight), first line                      */
    double p_acc_le;      /* Eq. (reweight), second line                     */
    double p_le;          /* p_acc_le / p_acc                                */
    double trunc_bound;   /* B = sum_{w > w_max} Bin_w(p)                     */
    double sem_p_acc;     /* standard error of p_acc (see msc_reweight)      */
    double sem_p_acc_le;  /* standard error of p_acc_le                      */
} msc_estimate;

typedef struct {
    int64_t n_shots;      /* shots drawn                                     */
    int64_t nnz;          /* faults drawn                                    */
    int64_t n_survivors;  /* shots left by the offline screen                */
    int64_t n_accepted;   /* survivors with P_acc > 0                        */
    int64_t n2q;          /* two-site updates executed                       */
    int64_t sweeps;       /* Jacobi sweeps                                   */
    double flops;         /* algorithmic flops of the two-site updates       */
    int32_t chi_peak;     /* largest bond dimension over the batch           */
    int32_t status_or;    /* OR of the survivors' msc_shot_status bits       */
    double ms_sample;     /* kernel time of the sampling (ms, context stream) */
    double ms_screen;     /* kernel time of the offline screen               */
    double ms_simulate;   /* kernel time of the shots                        */
} msc_batch_stats;

/* Message of the last failure on this thread (never NULL). */
const char* msc_last_error(void);

/* Library version string. */
const char* msc_version(void);

/* ---------------------------------------------------------------------- */
/* Context: one GPU, one stream, grow-only device scratch.                 */

/* Create a context on HIP device `device`.  `stream` is the hipStream_t
   every device entry point of the context runs on: NULL gives the context
   a non-blocking stream of its own (default priority, destroyed with the
   context); a caller's stream is used as is and stays the caller's (it
   must belong to `device` and outlive the context).  The context also
   readies the device's fixed scratch of msc_prescreen_noalloc.  Fails with
   MSC_E_DEVICE when no GPU is usable.                                     */
int msc_ctx_create(int device, void* stream, msc_ctx** out);
void msc_ctx_destroy(msc_ctx* ctx);
/* Duration in ms of the last kernel work of the named kind, measured with
   HIP events on the context's stream: "sample" (device fault draws),
   "prescreen", "simulate" (shot kernel), "prefix" (checkpoint recording of
   the noiseless run), "camps", "camps_prefix", "twosite".  msc_run_batch
   sets "sample", "prescreen" and "simulate".  Returns a negative value if
   none was timed.                                                         */
double msc_ctx_last_kernel_ms(msc_ctx* ctx, const char* which);

/* What the kernels did in the context's last msc_simulate or msc_run_batch
   call: the batched engine for large two-site updates (zero if nothing
   parked) and the wavefront kernel (msc_sim_opts.wave_chi).               */
typedef struct {
    int64_t rounds;         /* engine rounds (each: all parked updates)      */
    int64_t updates;        /* two-site updates done by the engine           */
    double contract_flops;  /* algorithmic: 32 cl cm cr per update          */
    double gram_flops;      /* algorithmic: 4 nv (nv + 1) len per update     */
    double contract_ms;     /* kernel time of the contractions (HIP events;
                               0 when the rounds ran as graph replays)      */
    double gram_ms;         /* kernel time of the Gram matrices             */
    double factor_ms;       /* kernel time of the factor steps              */
    double shot_ms;         /* kernel time of the shot kernel's launches     */
    double total_ms;        /* all of the call's shot work                   */
    int64_t factor_lds;     /* factor steps whose overlapping vectors were
                               diagonalised in LDS (at most 64 of them)      */
    int64_t factor_wide;    /* factor steps with more: one-sided Jacobi in
                               the slot's workspace                          */
    int64_t overlapping;    /* overlapping vectors, summed over the updates  */
    int64_t sweeps;         /* Jacobi sweeps, summed                         */
    int64_t wave_slots;     /* shots in flight in the wavefront kernel (0:
                               the workgroup kernel ran every shot)         */
    int64_t wave_retries;   /* shots it handed to the workgroup kernel       */
} msc_engine_stats;

int msc_ctx_engine_stats(msc_ctx* ctx, msc_engine_stats* out);

/* ---------------------------------------------------------------------- */
/* Circuit: parse + compile on the host (no GPU needed).                  */

/* Parse `len` bytes of circuit text and compile it: MPS layout (site order
   from `order` if non-NULL (host, n_qubits entries: order[site] = qubit),
   else the text's ORDER line, else identity), SWAP routing of non-adjacent
   two-qubit gates (Section 3.1: long-range gates touch every bond in
   between), the channel table (Section 4) and the offline-screening
   tables (Section 4.2).  Errors: MSC_E_PARSE, MSC_E_INVALID.             */
int msc_circuit_load(const char* text, size_t len, const int32_t* order,
                     msc_circuit** out);
int msc_circuit_get_info(const msc_circuit* c, msc_circuit_info* out);
/* Expected outcome e_m of every measurement (host, n_meas bytes).  Before
   calibration these are all 0 (the paper's rule: kept iff all outcomes are
   0, Section 4).                                                          */
int msc_circuit_expected(const msc_circuit* c, uint8_t* out);
/* Noiseless FP64 run on the GPU: records e_m and checks that every
   measurement is deterministic (p(e_m) = 1 +- 1e-10) and the final
   fidelity is 1 (Appendix "Post-selection and logical error").  Returns
   MSC_E_NONDETERMINISTIC otherwise.  Required before msc_simulate.       */
int msc_circuit_calibrate(msc_ctx* ctx, msc_circuit* c);
/* Record of the calibration's noiseless run (host out): its bond peak,
   two-site updates and algorithmic flops.  MSC_E_STATE before
   calibration.                                                           */
int msc_circuit_noiseless(const msc_circuit* c, msc_shot_result* out);
/* The circuit's segments (host out, up to cap entries; *n_out = their
   number, at least 1: a circuit without SEGMENT lines is one segment).
   MSC_E_CAPACITY if cap is smaller.                                       */
int msc_circuit_segments(const msc_circuit* c, int32_t cap, msc_segment* out,
                         int32_t* n_out);
void msc_circuit_free(msc_circuit* c);

/* ---------------------------------------------------------------------- */
/* Fault sampling (Section 4.1, subset sampling), host.                    */

/* Draw faults for shots first_shot .. first_shot+n_shots-1 with seed
   `seed`.  Per shot: weight w = weights[i] if `weights` (host, n_shots) is
   non-NULL, else w ~ Bin(M, p); a uniform w-subset of the M channels
   (Floyd); a uniform non-identity Pauli per chosen channel (3 for DEP1, 15
   for DEP2, 63 for DEP3, X for XERR).  Output CSR (host):
   shot_off[n_shots+1] (int64), chan[nnz] (int32, ascending within a shot),
   pauli[nnz] (uint8, bits 2j and 2j+1 = x and z bit of the channel's j-th
   qubit, j < 3).  MSC_E_CAPACITY if more than nnz_cap
   faults are needed (nnz_out then holds the required count).            */
int msc_sample_faults(const msc_circuit* c, uint64_t seed, uint64_t first_shot,
                      int64_t n_shots, const int32_t* weights, double p,
                      int64_t* shot_off, int32_t* chan, uint8_t* pauli,
                      int64_t nnz_cap, int64_t* nnz_out);

/* The same draws on the context's GPU, one shot per lane: the CSR is
   bit-identical to msc_sample_faults for the same arguments.  weights
   (device, n_shots int32) or NULL for w ~ Bin(M, p); shot_off (device,
   n_shots+1 int64), chan and pauli (device, nnz_cap entries; may be NULL
   only if nnz_cap is 0).  nnz_out (host) receives the total fault count.
   MSC_E_CAPACITY if it exceeds nnz_cap: shot_off is then complete, chan
   and pauli hold only the shots that fit (never written past nnz_cap).   */
int msc_sample_faults_device(msc_ctx* ctx, const msc_circuit* c, uint64_t seed,
                             uint64_t first_shot, int64_t n_shots,
                             const int32_t* weights, double p, int64_t* shot_off,
                             int32_t* chan, uint8_t* pauli, int64_t nnz_cap,
                             int64_t* nnz_out);

/* ---------------------------------------------------------------------- */
/* Offline screening (Section 4.2).                                        */

/* Copy the pre-screen tables to host arrays (either may be NULL):
   sig[(6*channel + k)*words + j] (k = 2j' + z: X or Z on the channel's
   j'-th qubit, zero rows for qubits a channel does not have) is the bitmask
   of decided measurements flipped by that basis fault; decided[i] is the
   measurement index of decided measurement i (n_decided entries).        */
int msc_prescreen_tables(const msc_circuit* c, uint64_t* sig, int32_t* decided);

/* Bit-exact screen of n_shots shots given as a device CSR.  Writes
   survive_bits (device, ceil(n_shots/64) words; bit set = must be
   simulated), and, if survivor_idx (device, n_shots capacity) is non-NULL,
   the indices of surviving shots in ascending order; n_survivors (host)
   receives their count.                                                   */
int msc_prescreen(msc_ctx* ctx, const msc_circuit* c, int64_t n_shots,
                  const int64_t* shot_off, const int32_t* chan,
                  const uint8_t* pauli, uint64_t* survive_bits,
                  int64_t* survivor_idx, int64_t* n_survivors);

/* msc_prescreen for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same screen, bit for bit, with its block counts, their scan and the
   CSR check word in a fixed per-device array of the library (2 MiB and
   8 KiB, held until the process ends) instead of context scratch.  At most 2^26 shots per call (else
   MSC_E_INVALID, nothing launched).  The circuit's tables must already be
   on the context's device (msc_circuit_calibrate or an earlier
   msc_prescreen put them there), else MSC_E_STATE.  Every call on one GPU
   uses the same array, so calls that overlap on a GPU race; each call
   overwrites what it reads before reading it.  No allocation, no free.   */
int msc_prescreen_noalloc(msc_ctx* ctx, const msc_circuit* c, int64_t n_shots,
                          const int64_t* shot_off, const int32_t* chan,
                          const uint8_t* pauli, uint64_t* survive_bits,
                          int64_t* survivor_idx, int64_t* n_survivors);

/* ---------------------------------------------------------------------- */
/* Batched exact MPS simulation (Sections 3.1, 4, 4.3).                    */

/* Simulate shots of a device CSR holding n_shots shots (as produced by
   msc_sample_faults and copied to the device).  If shot_idx (device, n_sel
   entries) is non-NULL only those shots are simulated and out[i] belongs to
   shot shot_idx[i] (entries outside [0, n_shots) are not simulated: their
   record has status 0); otherwise n_sel is ignored and out[i] belongs to
   shot i.  out: device array of msc_shot_result, one per simulated shot.
   Every shot runs the compiled op stream on its own ragged MPS, stops at
   the first expected outcome with p < tau_rej (online screening), and
   reports P_acc = prod_m p(e_m) and the seed qubit's infidelity against
   the target.  Requires a calibrated circuit.                             */
int msc_simulate(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                 int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                 const uint8_t* pauli, const int64_t* shot_idx, int64_t n_sel,
                 msc_shot_result* out);

/* One batch of the whole path on the context's stream with a single
   synchronisation at the end (no host round trip between the stages, so
   calls on different contexts overlap on the GPU): shots first_shot ..
   first_shot+n_shots-1 drawn as by msc_sample_faults with w ~ Bin(M, p)
   (Section 4.1), screened as by msc_prescreen (Section 4.2), the survivors
   simulated as by msc_simulate with `opts` (Sections 3.1, 4, 4.3), and the
   results reduced per fault weight for Eq. (reweight): bins (host,
   7 * n_bins doubles, 1 <= n_bins <= 1024) receives bins[w] = number of
   shots of weight w, bins[n_bins + w] = sum of their P_acc,
   bins[2 n_bins + w] = sum of P_acc * fail (both summed in a fixed
   order), and the counts of the error analysis's likelihood (Eq.
   (loglik-split)): bins[3 n_bins + w] = shots counted as accepted, i.e.
   with u < P_acc for the shot's acceptance uniform u, bins[4 n_bins + w] =
   those of them whose accepted branch fails; bins[5 n_bins + w] and
   bins[6 n_bins + w] are the sums of P_acc^2 and (P_acc * fail)^2 (fixed
   order) for the standard errors of msc_reweight.  u = (x >> 11) 2^-53 with x
   the first output of the SplitMix64 stream keyed as the fault draws but
   with seed ^ 0x243F6A8885A308D3.  Weights >= n_bins - 1 share the last
   bin; screened shots count with P_acc = 0.  stats (host) is optional.  out (device, n_shots records) is
   optional: out[i] is the result of shot i (screened shots: all zero,
   rejected_at -1).  The fault buffer is sized for the largest weight the
   Bin(M, p) table can draw; MSC_E_CAPACITY if that exceeds 2^28 faults.
   surv_bins (host, n_bins * n_seg doubles with n_seg from
   msc_circuit_segments) is optional; if given, the batch runs in
   space-time mode: the offline screen is skipped (every shot is simulated
   and stops at its first rejecting measurement, as a physical shot would)
   and surv_bins[w * n_seg + s] receives the sum over the shots of weight w
   of their probability of reaching segment s (fixed-order FP64 sums);
   stats->n_survivors is then n_shots.                                      */
int msc_run_batch(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                  uint64_t seed, uint64_t first_shot, int64_t n_shots, double p,
                  int32_t n_bins, double* bins, msc_batch_stats* stats,
                  msc_shot_result* out, double* surv_bins);

/* ---------------------------------------------------------------------- */
/* CAMPS (section "Clifford augmented MPS").                               */

/* Simulate shots as msc_simulate does (same arguments, shot selection and
   result records) with the Clifford-augmented MPS: the state is C|m>, C a
   Clifford frame held as the images C^dag X_q C, C^dag Z_q C of the
   single-qubit Paulis, |m> the magic residual, an FP64 MPS.  Clifford
   gates and Pauli faults act on the frame only; T and T^dagger (CS,
   CS^dagger and CCZ written over T, T^dagger and CX) become rotations
   exp(-+i pi/8 C^dag Z C) of the residual and measurements projections
   (I +- C^dag Z C)/2, applied to the MPS and recompressed in the exact
   regime (sigma > tau_trunc sigma_max, default 1e-12); after each one that
   acts on two sites or more, a greedy sweep over its bonds moves the
   entanglement-lowering two-qubit Clifford of highest purity gain (19
   classes modulo local Cliffords) into the frame.  opts: precision
   MSC_FP64, chi_max in [1, 32] (the residual's bond cap: a shot that needs
   more is run again, after the CAMPS launch, by the plain FP64 MPS path of
   msc_simulate with bond cap 256 and the same tau's and prefix option; its
   record is that path's, with MSC_SHOT_MPS_RERUN set), lds_width 0 and
   wave_chi 0 or -1;
   prefix 1 forks every shot from a checkpoint of the noiseless CAMPS run
   taken before its first fault (built on first use, <= 2 GiB; results are
   bit-identical to prefix 0; MSC_E_NONDETERMINISTIC if the noiseless run's
   residual outgrows the cap).  out[i].chi_peak is the residual's peak bond dimension,
   out[i].n2q the disentangling Cliffords applied; disc_weight and flops
   are 0.  Requires a calibrated circuit with at most 127 qubits.         */
int msc_simulate_camps(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                       int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                       const uint8_t* pauli, const int64_t* shot_idx, int64_t n_sel,
                       msc_shot_result* out);

/* The disentangler's candidates (host out): *n_out = 19; dmat (optional,
   32 doubles each) their unitaries as (re, im) pairs, row-major over
   |s_k s_k+1> with the left site the high bit; dtab (optional, 16 bytes
   each) their Pauli maps: entry x1 | z1 << 1 | x2 << 2 | z2 << 3 gives the
   image of X1^x1 Z1^z1 X2^x2 Z2^z2 in the same bits plus its phase
   exponent of i in bits 4-5.                                              */
int msc_camps_candidates(double* dmat, uint8_t* dtab, int32_t* n_out);

/* ---------------------------------------------------------------------- */
/* Autotuning of the batched engine's tile shapes.                         */

/* One bucket's choice: theta sides of the bucket's representative update,
   the contraction tile (rows of (a, i) x b values) and Gram tile chosen,
   and their timings per launch (microseconds, best of `reps`).          */
typedef struct {
    int32_t bucket, side, batch, rows, b, gram;
    double contract_us, gram_us;
} msc_tune_entry;

/* Times every tile shape the library has for `precision` (MSC_FP32 or
   MSC_FP64; MSC_BF16X3 tunes the FP32 contraction's shapes with the
   bf16 split) on a synthetic batch of parked updates per bucket of theta
   sides (<= 128, <= 256, <= 512, larger; chi_l = chi_m = chi_r = 64, 128,
   256, 512, random normalised tensors, CX gate), `reps` launches each,
   and keeps the fastest contraction and Gram tiles per bucket.  out (host,
   4 entries, optional) receives the choices.  If `cache_path` is non-NULL
   the choices are written there as JSON: {"device": ..., "entries":
   [{"precision", "bucket", "side", "rows", "b", "gram", "contract_us",
   "gram_us"}, ...]}, replacing the file's entries of this precision and
   keeping the others; msc_sim_opts.autotune_cache reads it back.         */
int msc_autotune(msc_ctx* ctx, int32_t precision, int32_t reps, const char* cache_path,
                 msc_tune_entry* out);

/* ---------------------------------------------------------------------- */
/* Two-site contraction on MFMA (Section 3.1), standalone.                 */

/* theta_b = G * (A_b . B_b) for `batch` independent two-site updates with
   chi_l = chi_m = chi_r = chi on MFMA, FP32 split complex with FP32
   accumulation (precision MSC_FP32) or BF16x3 split precision
   (MSC_BF16X3).  Layouts (device, float): A and B are [batch][2 (re,im)]
   [chi*2][chi] and [batch][2][chi][2*chi] (row-major, rows (a,i) resp. c,
   columns c resp. (j,b)); gate (device, 32 floats) is the 4x4 complex gate
   in row-major (re,im) pairs over |i j>; theta is [batch][2][2*chi][2*chi]
   with rows (a,i) and columns (j,b).  chi must be a multiple of 64 in
   [64, 1024].                                                             */
int msc_twosite_contract(msc_ctx* ctx, int32_t precision, int32_t chi,
                         int32_t batch, const float* A, const float* B,
                         const float* gate, float* theta);

/* One two-site update through the batched large-update engine (Section
   3.1; the exact regime of Section 5.1), on caller tensors.  For each of
   `batch` independent pairs A_b (chi_l x 2 x chi_m) and B_b (chi_m x 2 x
   chi_r): theta = G (A_b B_b) with the 4x4 gate `gate` (ids: 0 identity,
   1 SWAP, 2 CX with control on A's qubit, 3 CX with control on B's, 4 CZ,
   5 CS, 6 CS^dagger), contracted on MFMA in `precision` (MSC_FP32,
   MSC_FP64, MSC_BF16X3); the FP64 Gram matrix of theta's vectors (columns
   for dir 1, rows for dir 0) on MFMA; the FP64 Jacobi eigen-decomposition
   of its overlapping block; then the split theta / |theta_kept| = A' B'
   keeping the singular values sigma_i > tau sigma_0, at most chi_max of
   them.  dir 1 leaves A' isometric (its (a,i) x c matrix has orthonormal
   columns) and B' = Sigma V^H; dir 0 leaves B' isometric (orthonormal rows
   c x (j,b)) and A' = U Sigma.
   Layouts (host, FP64, planar per tensor): A is [batch][2 (re, im)]
   [chi_l * 2 * chi_m] with element (a, i, c) at (a * 2 + i) * chi_m + c;
   B is [batch][2][chi_m * 2 * chi_r] with (c, j, b) at (c * 2 + j) * chi_r
   + b.  With rmax = min(chi_max, 2 min(chi_l, chi_r)): A_out is
   [batch][2][chi_l * 2 * rmax] and B_out [batch][2][rmax * 2 * chi_r],
   holding A' (chi_l x 2 x r) and B' (r x 2 x chi_r) densely with their
   actual r = r_out[b] (host, batch) at the start of each plane, zeros after.
   Bonds and chi_max in [1, 1024], batch in [1, 8192], tau in (0, 1);
   synchronous; MSC_E_INVALID for bad arguments, MSC_E_OOM, MSC_E_DEVICE. */
int msc_engine_update(msc_ctx* ctx, int32_t precision, int32_t chi_l,
                      int32_t chi_m, int32_t chi_r, int32_t batch, int32_t dir,
                      int32_t gate, int32_t chi_max, double tau, const double* A,
                      const double* B, double* A_out, double* B_out,
                      int32_t* r_out);

/* ---------------------------------------------------------------------- */
/* Re-weighting (Section 4.1, Eq. (reweight); Appendix "Systematics").     */

/* Per-bin sums (host, n_bins each): bin_n[w] shots, bin_acc[w] = sum of
   P_acc, bin_fail[w] = sum of P_acc * fail, and optionally (host or NULL)
   bin_acc2[w], bin_fail2[w] the sums of their squares (msc_run_batch's
   rows 5 and 6).  For each p in p_grid (host, n_p) writes out[k] (host):
   p_acc, p_acc * p_le, p_le, the truncation bound
   B = sum_{w >= n_bins} Bin_w(p), and the standard errors of the first two:
   the bins are independent samples, so sem^2 = sum_w Bin_w(p)^2 var_w / n_w
   with var_w the unbiased sample variance of the bin's per-shot values
   when the sums of squares are given and n_w >= 2, else the Bhatia-Davis
   bound mu_w (1 - mu_w) of a variable in [0, 1] with mean mu_w.  Bins with
   bin_n[w] == 0 are skipped.                                              */
int msc_reweight(const double* bin_n, const double* bin_acc,
                 const double* bin_fail, const double* bin_acc2,
                 const double* bin_fail2, int32_t n_bins, int64_t M,
                 const double* p_grid, int32_t n_p, msc_estimate* out);

/* ---------------------------------------------------------------------- */
/* Qubit-order search (Section 3.1: the linear order drives the routing    */
/* and the bond dimension; an automatic search is the paper's future work).*/

/* Fixed cost of one op of the shot kernel, in flop equivalents, in the
   order-search cost below: the kernel is latency-bound, so an op costs a
   number of cycles beyond its flops (measured per op kind on the 49-qubit
   workload: about 7e3 cycles per product swap, 1.2e4 per centre move,
   2.5e4 per two-site update at the smallest bonds), priced at 100 flops
   per cycle, the rate of a two-site update at chi = 32.                    */
#define MSC_ORDER_COST_PSWAP   7.0e5
#define MSC_ORDER_COST_MOVE    1.2e6
#define MSC_ORDER_COST_TWOSITE 2.5e6

/* Local search for the qubit -> site order of the circuit `text` (len
   bytes) from `start` (host, n_qubits entries, order[site] = qubit; NULL:
   the text's ORDER line, else identity).  Cost of an order = algorithmic
   flops of its noiseless run (msc_circuit_noiseless after calibration on
   ctx's GPU) + MSC_ORDER_COST_PSWAP * n_product_swaps + MSC_ORDER_COST_MOVE
   * n_moves + MSC_ORDER_COST_TWOSITE * n_twosite of the circuit compiled
   with that order (msc_circuit_info); +inf if the noiseless run exceeds
   the bond cap.  Each of the `budget` evaluations after the first tries
   one move drawn from a SplitMix64 stream keyed by `seed` between sites i
   and j at distance 1 + floor(-4 ln u): exchange them, reverse the run
   between them, or move site i to position j (probability 1/3 each); a
   move is kept iff the cost falls.
   order_out (host, n_qubits): the best order; cost_out (host, 2 doubles):
   the start order's cost and the best cost.  Calibration errors other than
   the bond cap are returned.                                              */
int msc_order_search(msc_ctx* ctx, const char* text, size_t len,
                     const int32_t* start, uint64_t seed, int32_t budget,
                     int32_t* order_out, double* cost_out);

/* The search's cost of a calibrated circuit's own order (host out): the
   algorithmic flops of its noiseless run + MSC_ORDER_COST_PSWAP *
   n_product_swaps + MSC_ORDER_COST_MOVE * n_moves + MSC_ORDER_COST_TWOSITE *
   n_twosite.  MSC_E_STATE before calibration.                            */
int msc_order_cost(const msc_circuit* c, double* out);

/* ---------------------------------------------------------------------- */
/* Likelihood statistics (Appendix "Error analysis of the subset-sampling  */
/* estimator"; Appendix "Credible intervals for rate ratios"; Appendix     */
/* "Losses").  Host only, no device work.                                   */

/* Per-bin counts (host, n_bins each, integer-valued doubles): bin_n[w]
   shots of weight w, bin_acc[w] = k_w of them accepted, bin_err[w] = m_w of
   those accepted with a logical failure (0 <= m_w <= k_w <= n_w);
   msc_run_batch's rows 0, 3 and 4.  Bins with n_w = 0 are unsampled and
   left out of the likelihood.  p_le^(w) = 0 is imposed for w < d_e (such a
   bin must have m_w = 0).  Bin_w = C(M, w) p^w (1-p)^(M-w).  The joint
   log-likelihood is the sum over bins of Eq. (loglik-split).            */
enum msc_functional {
    MSC_STAT_PACC = 0,    /* p_acc = sum_w Bin_w p_acc^(w)                     */
    MSC_STAT_PLE = 1      /* p_le = sum_w Bin_w p_acc^(w) p_le^(w) / p_acc     */
};

typedef struct {
    double estimate;      /* the functional at the maximum-likelihood rates  */
    double lo, hi;        /* Eq. (profile) endpoints at threshold log R       */
    double hi_trunc;      /* hi + B: the truncation bound added upward only   */
    double trunc_bound;   /* B = sum_{w >= n_bins} Bin_w(p)                   */
    double unaccepted;    /* sum over sampled bins with k_w = 0 of
                             Bin_w (1 - R^(-1/n_w)): their worst case       */
    double unsampled_mass;/* sum of Bin_w over the bins with n_w = 0          */
    int32_t n_unsampled;  /* number of those bins                             */
    int32_t n_bins_used;  /* bins with n_w > 0                                */
} msc_interval;

/* Eq. (profile) at one value: *out = max over all bin rates with
   functional = theta of the joint log-likelihood, minus its unconstrained
   maximum (<= 0; -inf when theta is not attainable).                     */
int msc_profile_loglik(const double* bin_n, const double* bin_acc,
                       const double* bin_err, int32_t n_bins, int64_t M,
                       double p, int32_t d_e, int32_t functional,
                       double theta, double* out);

/* Likelihood-ratio interval of Eq. (profile): every theta whose profile is
   at least -log R (R > 1; the paper uses R = 100), endpoints by bisection
   to 2^-60 of the range.  out (host) as described above.  MSC_E_INVALID if
   no bin is sampled or the counts are inconsistent.                      */
int msc_lr_interval(const double* bin_n, const double* bin_acc,
                    const double* bin_err, int32_t n_bins, int64_t M,
                    double p, int32_t d_e, int32_t functional, double R,
                    msc_interval* out);

/* Central credible interval (probability `level`) of the ratio T / S of
   two logical error rates: T is p_le of the counts given (posterior = the
   normalised profile likelihood with a prior flat in log theta), S has the
   Jeffreys posterior Beta(s_err + 1/2, s_acc - s_err + 1/2) from s_acc
   accepted shots of which s_err failed.  The densities of log T and log S
   are sampled on the lattice j h (natural log; h in (0, 0.1]) until they
   are 18 log-units below their maxima on both sides, log T - log S is
   their discrete convolution, its CDF is read at cell edges (j + 1/2) h
   and interpolated linearly.  Needs at least one failure in the counts.  */
int msc_ratio_credible(const double* bin_n, const double* bin_acc,
                       const double* bin_err, int32_t n_bins, int64_t M,
                       double p, int32_t d_e, double s_acc, double s_err,
                       double level, double h, double* lo, double* hi);

/* Expected space-time volume (Appendix "Space-time overhead") at physical
   error rate p from msc_run_batch's space-time mode: bin_n (host, n_bins)
   shots per weight, surv_bins (host, n_bins * n_seg) their summed reach
   probabilities, segs (host, n_seg) the circuit's segments.  reach (host,
   n_seg) receives sum_w Bin_w(p) surv_bins[w][s] / n_w over the sampled
   bins; volume (host, 2 doubles) the expected volume summed over the noisy
   segments, n_qubits x depth x reach, and the same plus B times their
   total volume (B = sum_{w >= n_bins} Bin_w(p), the truncation bound).    */
int msc_expected_volume(const double* bin_n, const double* surv_bins,
                        int32_t n_bins, const msc_segment* segs, int32_t n_seg,
                        int64_t M, double p, double* reach, double* volume);

/* Multiplicative factor on the expected number of attempts when each of M
   channels carries an independent, detected loss of probability p_loss:
   (1 - p_loss)^(-M) (Appendix "Losses").                                  */
int msc_loss_factor(int64_t M, double p_loss, double* out);

#ifdef __cplusplus
}
#endif

#endif /* MSC_H */
