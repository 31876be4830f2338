// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msc.h"

namespace msc {

// ---------------------------------------------------------------------------
// Compiled MPS op stream (device).  Sites are MPS positions, not qubits.
enum OpKind : int32_t {
    OP_G1 = 0,     // a = site, aux = 1q gate id (gate2 table)
    OP_G2 = 1,     // a = k (sites k, k+1), b = dir (1: centre -> k+1,
                   // 0: centre -> k), aux = 4x4 gate id (gate4 table)
    OP_FAULT = 2,  // a = site of the channel's first qubit, b = second or -1,
                   // aux = channel index (reads the shot's code for it)
    OP_MEAS = 3,   // a = site, aux = measurement index
    OP_RESET = 4,  // a = site: X^e with e the outcome last projected there
    OP_FINAL = 5,  // a = site of the seed qubit
    OP_SWAPP = 6,  // a = k: SWAP of sites k, k+1 where the qubit on site
                   // k + b (b = 0 or 1) is in a product state with the rest
    OP_MOVE = 7,   // a = k: move the orthogonality centre from k to k+1
                   // (b = 1) or from k+1 to k (b = 0)
    OP_FAULT3 = 8  // a = site of a three-qubit channel's third qubit; uses
                   // bits 4, 5 of the code read by the OP_FAULT right before
};

struct DevOp {
    int32_t kind, a, b, aux;
};

// CAMPS op stream (kind of DevOp): qubits are physical qubits
enum CampsKind : int32_t {
    CO_G1 = 0,      // a = qubit, aux = Gate1 (Clifford: H S SDG X Y Z)
    CO_CX = 1,      // a = control, b = target
    CO_CZ = 2,      // a, b
    CO_ROT = 3,     // a = qubit, aux = +1 (T) or -1 (T^dagger)
    CO_FAULT = 4,   // a = channel index
    CO_MEAS = 5,    // a = qubit, aux = measurement index
    CO_RESET = 6,   // a = qubit: X^e with e the outcome last projected
    CO_FINAL = 7    // a = seed qubit
};

// 1q gate ids (rows of the 2x2 complex table)
enum Gate1 : int32_t { G_H = 0, G_S, G_SDG, G_T, G_TDG, G_X, G_Y, G_Z, G1_COUNT };
// 4x4 gate ids in site order |s_k s_{k+1}>
enum Gate4 : int32_t { G4_I = 0, G4_SWAP, G4_CX01, G4_CX10, G4_CZ, G4_CS, G4_CSDG, G4_COUNT };

// Parsed circuit op (qubit level)
enum IrKind : int32_t { IR_G1 = 0, IR_G2, IR_M, IR_R, IR_CH, IR_G3 };
enum ChanKind : int32_t { CH_DEP1 = 0, CH_DEP2 = 1, CH_XERR = 2, CH_DEP3 = 3 };
// IR_G2 gate codes
enum Gate2 : int32_t { G2_CX = 0, G2_CZ = 1, G2_CS = 2, G2_CSDG = 3 };
// basis faults per channel in the screening signatures: X and Z on each of
// up to three qubits
constexpr int kFaultComponents = 6;
struct IrOp {
    int32_t kind;
    int32_t g;        // IR_G1: Gate1; IR_G2: Gate2; IR_G3: 0 (CCZ); IR_CH: ChanKind
    int32_t a, b, c;  // qubits (-1 if unused)
    int32_t idx;      // measurement or channel index
};

void gate1_matrix(int g, double out[8]);    // (re,im) row-major 2x2
void gate4_matrix(int g, double out[32]);   // (re,im) row-major 4x4

// FP64 cumulative Bin(M, p) table of the sampler (sampler.cpp)
std::vector<double> binomial_cdf(int64_t M, double p);

// log Bin_w(p) = log C(M, w) + w log p + (M - w) log(1 - p) (sampler.cpp)
double log_bin(int64_t M, int64_t w, double p);

// Error helpers (capi.cpp)
int set_error(int code, const std::string& msg);

}  // namespace msc

// Device checkpoints of the noiseless run for one option set (see the
// shot kernel): built on first use by msc_simulate with prefix = 1.
struct PrefixCk {
    bool valid = false;
    int dev = -1, precision = -1, chi_max = 0, lds_width = 0, park_side = 0, wave_chi = 0;
    double tau = 0.0, tau_rej = 0.0;
    int n_ck = 0, ck_k = 1, avail = 0;
    int64_t cap = 0;           // elements of the tensor type
    float build_ms = 0.f;
    void* d_op = nullptr;      // int32[n_ck]
    void* d_avail = nullptr;   // int32
    void* d_off = nullptr;     // int64[n_ck]
    void* d_hdr = nullptr;     // CkHdr[n_ck]
    void* d_data = nullptr;
    void* d_pm = nullptr;     // [n_meas] running P_acc before each measurement
};

// Device checkpoints of the noiseless CAMPS run (msc_simulate_camps with
// prefix = 1), built on first use for one (chi cap, tau, tau_rej) set.
struct CampsPrefix {
    bool valid = false;
    int dev = -1, chi_cap = 0;
    double tau = 0.0, tau_rej = 0.0;
    int n_ck = 0, ck_k = 1, avail = 0;
    int64_t cap = 0;           // doubles of tensor storage
    float build_ms = 0.f;
    void *d_op = nullptr, *d_avail = nullptr, *d_off = nullptr, *d_hdr = nullptr;
    void *d_frame = nullptr, *d_ph = nullptr, *d_data = nullptr;
};

struct msc_circuit {
    int n = 0;
    int seed = 0;
    int target = 'T';
    std::vector<int32_t> order;          // site -> qubit
    std::vector<msc::IrOp> ir;
    int n_meas = 0, n_channels = 0;
    std::vector<int32_t> chan_kind;
    // compiled MPS op stream
    std::vector<msc::DevOp> ops;
    int64_t n_twosite = 0, n_swaps = 0, n_product_swaps = 0, n_moves = 0;
    int final_site = 0;
    std::vector<int32_t> chan_op;        // op index of each channel's OP_FAULT
    // expected outcomes
    std::vector<uint8_t> expected;
    bool calibrated = false;
    msc_shot_result noiseless{};         // the calibration run's record
    // segments (SEGMENT lines): first IR op of each, and their table
    std::vector<int32_t> seg_ir;
    std::vector<msc_segment> segs;
    void* d_segm = nullptr;              // int32 first_meas per segment
    // CAMPS op stream (built on first use) and its device copies
    std::vector<msc::DevOp> camps_ops;
    std::vector<int32_t> chan_q;         // [3 n_channels]
    void* d_camps_ops = nullptr;
    void* d_chan_q = nullptr;
    void* d_site_of = nullptr;
    void* d_dmat = nullptr;              // candidate tables (camps_candidates)
    void* d_dtab = nullptr;
    CampsPrefix camps_prefix;
    // offline screening tables
    int words = 0;
    std::vector<int32_t> decided;        // measurement index per decided slot
    std::vector<uint64_t> sig;           // [6*n_channels][words]
    // device copies (owned), on device `dev`
    int dev = -1;
    void* d_ops = nullptr;
    void* d_g1 = nullptr;
    void* d_g4 = nullptr;
    void* d_sig = nullptr;               // uint64 [codes of all channels][words]
    void* d_sig_off = nullptr;           // int32 first code entry per channel
    void* d_expected = nullptr;
    void* d_kind = nullptr;              // uint8 ChanKind per channel
    PrefixCk prefix;
};

namespace msc {
int compile_circuit(msc_circuit* c);        // ops from ir + layout
int prescreen_compile(msc_circuit* c);      // decided set + signatures
int parse_circuit(const char* text, size_t len, msc_circuit* c);
void segment_table(msc_circuit* c);         // segs from seg_ir and ir
void camps_compile(msc_circuit* c);         // camps_ops and chan_q from ir
// candidate two-qubit Cliffords of the disentangler: unitaries (32 doubles
// each, (re, im) row-major over |s_k s_k+1>) and Pauli maps (16 bytes each)
void camps_candidates(std::vector<double>& dmat, std::vector<uint8_t>& dtab);
}  // namespace msc
