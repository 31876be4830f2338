// C ABI: context, circuit lifetime, device dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../kernels/kernels.h"
#include "../msc_internal.h"

namespace msc {

static thread_local std::string g_err = "no error";

int set_error(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

}  // namespace msc

using namespace msc;

#define MSC_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_error(MSC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct msc_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;     // created here (destroyed with the context)
    int n_cu = 0;
    std::map<std::string, DevBuf> bufs;       // grow-only scratch
    std::map<std::string, double> last_ms;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
    // what the slot-layout and Bin(M, p) buffers currently hold
    int layout_n = -1, layout_chi = -1;
    int wlayout_n = -1, wlayout_chi = -1;     // the wavefront kernel's slots
    int64_t cdf_m = -1;
    double cdf_p = -1.0;
    int32_t cdf_len = 0;
    // host-mapped pinned block the batch reduction writes into
    void* hmap = nullptr;
    void* hmap_dev = nullptr;
    size_t hmap_bytes = 0;
    // one round of the large-update engine captured as a graph, and the
    // bytes of the arguments it was captured with
    hipGraphExec_t lx_exec = nullptr;
    std::string lx_key;
    msc_engine_stats lx_stats{}; // the engine in the last shot run
    hipEvent_t lxev[6] = {};     // phase boundaries of an engine round
};

static int ctx_buf(msc_ctx* ctx, const std::string& name, size_t bytes, void** out) {
    DevBuf& b = ctx->bufs[name];
    if (b.bytes < bytes) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        hipError_t e = hipMalloc(&b.p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(MSC_E_OOM, "hipMalloc(" + std::to_string(bytes) + ") for " + name +
                                            ": " + hipGetErrorString(e));
        }
        b.bytes = std::max<size_t>(bytes, 256);
    }
    *out = b.p;
    return MSC_OK;
}

// MSC_E_INVALID with the CSR check bits spelled out
static int csr_error(int bad) {
    std::string m = "invalid fault CSR:";
    if (bad & CSR_BAD_CHANNEL) m += " channel index outside [0, M);";
    if (bad & CSR_NOT_ASCENDING) m += " channels of a shot not strictly ascending;";
    if (bad & CSR_BAD_PAULI) m += " Pauli code zero or beyond the channel's qubits;";
    if (bad & CSR_BAD_OFFSETS) m += " shot offsets decreasing or negative;";
    return set_error(MSC_E_INVALID, m);
}

extern "C" const char* msc_last_error(void) { return g_err.c_str(); }

extern "C" const char* msc_version(void) { return "msc-mps 0.1 (gfx950)"; }

extern "C" int msc_ctx_create(int device, void* stream, msc_ctx** out) {
    if (!out) return set_error(MSC_E_INVALID, "null out");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return set_error(MSC_E_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) return set_error(MSC_E_INVALID, "device index out of range");
    std::unique_ptr<msc_ctx> ctx(new msc_ctx());
    ctx->device = device;
    MSC_HIP(hipSetDevice(device));
    if (stream) {
        ctx->stream = static_cast<hipStream_t>(stream);
    } else {
        MSC_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    int64_t* fixed = nullptr;   // the device's msc_prescreen_noalloc scratch
    MSC_HIP(prescreen_noalloc_scratch(device, &fixed));
    MSC_HIP(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device));
    MSC_HIP(hipEventCreate(&ctx->ev0));
    MSC_HIP(hipEventCreate(&ctx->ev1));
    MSC_HIP(hipEventCreate(&ctx->ev2));
    MSC_HIP(hipEventCreate(&ctx->ev3));
    for (hipEvent_t& ev : ctx->lxev) MSC_HIP(hipEventCreate(&ev));
    *out = ctx.release();
    return MSC_OK;
}

extern "C" void msc_ctx_destroy(msc_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    for (hipEvent_t ev : {ctx->ev0, ctx->ev1, ctx->ev2, ctx->ev3})
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : ctx->lxev)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->hmap) (void)hipHostFree(ctx->hmap);
    if (ctx->lx_exec) (void)hipGraphExecDestroy(ctx->lx_exec);
    if (ctx->stream && ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

extern "C" int msc_ctx_engine_stats(msc_ctx* ctx, msc_engine_stats* out) {
    if (!ctx || !out) return set_error(MSC_E_INVALID, "null argument");
    *out = ctx->lx_stats;
    return MSC_OK;
}

extern "C" double msc_ctx_last_kernel_ms(msc_ctx* ctx, const char* which) {
    if (!ctx || !which) return -1.0;
    auto it = ctx->last_ms.find(which);
    return it == ctx->last_ms.end() ? -1.0 : it->second;
}

// ---------------------------------------------------------------------------
// circuits

extern "C" int msc_circuit_load(const char* text, size_t len, const int32_t* order,
                                msc_circuit** out) {
    if (!text || !out) return set_error(MSC_E_INVALID, "null argument");
    *out = nullptr;
    std::unique_ptr<msc_circuit> c(new msc_circuit());
    int rc = parse_circuit(text, len, c.get());
    if (rc) return rc;
    if (c->n > kMaxSites) return set_error(MSC_E_INVALID, "more than 128 qubits");
    if (order) c->order.assign(order, order + c->n);
    rc = compile_circuit(c.get());
    if (rc) return rc;
    rc = prescreen_compile(c.get());
    if (rc) return rc;
    *out = c.release();
    return MSC_OK;
}

extern "C" int msc_circuit_get_info(const msc_circuit* c, msc_circuit_info* o) {
    if (!c || !o) return set_error(MSC_E_INVALID, "null argument");
    o->n_qubits = c->n;
    o->n_meas = c->n_meas;
    o->n_channels = c->n_channels;
    o->n_decided = static_cast<int32_t>(c->decided.size());
    o->seed_qubit = c->seed;
    o->target = c->target;
    o->words = c->words;
    o->calibrated = c->calibrated ? 1 : 0;
    o->n_ops = static_cast<int64_t>(c->ops.size());
    o->n_twosite = c->n_twosite;
    o->n_swaps = c->n_swaps;
    o->n_product_swaps = c->n_product_swaps;
    o->n_moves = c->n_moves;
    return MSC_OK;
}

extern "C" int msc_circuit_segments(const msc_circuit* c, int32_t cap, msc_segment* out,
                                    int32_t* n_out) {
    if (!c || !n_out || (cap > 0 && !out)) return set_error(MSC_E_INVALID, "null argument");
    const int32_t n = static_cast<int32_t>(c->segs.size());
    *n_out = n;
    if (cap < n) return set_error(MSC_E_CAPACITY, "cap below the number of segments");
    std::copy(c->segs.begin(), c->segs.end(), out);
    return MSC_OK;
}

extern "C" int msc_circuit_expected(const msc_circuit* c, uint8_t* out) {
    if (!c || !out) return set_error(MSC_E_INVALID, "null argument");
    std::copy(c->expected.begin(), c->expected.end(), out);
    return MSC_OK;
}

static void free_prefix(PrefixCk& pk) {
    if (pk.dev >= 0) {
        (void)hipSetDevice(pk.dev);
        for (void** p : {&pk.d_op, &pk.d_avail, &pk.d_off, &pk.d_hdr, &pk.d_data, &pk.d_pm}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
    }
    pk = PrefixCk();
}

static void free_camps_prefix(CampsPrefix& pk) {
    if (pk.dev >= 0) {
        (void)hipSetDevice(pk.dev);
        for (void** p : {&pk.d_op, &pk.d_avail, &pk.d_off, &pk.d_hdr, &pk.d_frame, &pk.d_ph,
                         &pk.d_data}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
    }
    pk = CampsPrefix();
}

static void free_device(msc_circuit* c) {
    free_prefix(c->prefix);
    free_camps_prefix(c->camps_prefix);
    if (c->dev < 0) return;
    (void)hipSetDevice(c->dev);
    for (void** p : {&c->d_ops, &c->d_g1, &c->d_g4, &c->d_sig, &c->d_sig_off, &c->d_expected, &c->d_kind,
                     &c->d_segm, &c->d_camps_ops, &c->d_chan_q, &c->d_site_of, &c->d_dmat,
                     &c->d_dtab}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    c->dev = -1;
}

extern "C" void msc_circuit_free(msc_circuit* c) {
    if (!c) return;
    free_device(c);
    delete c;
}

static int upload(msc_ctx* ctx, msc_circuit* c) {
    if (c->dev == ctx->device && c->d_ops) return MSC_OK;
    free_device(c);
    MSC_HIP(hipSetDevice(ctx->device));
    std::vector<double> g1(G1_COUNT * 8), g4(G4_COUNT * 32);
    for (int g = 0; g < G1_COUNT; ++g) gate1_matrix(g, &g1[g * 8]);
    for (int g = 0; g < G4_COUNT; ++g) gate4_matrix(g, &g4[g * 32]);
    auto put = [&](void** dst, const void* src, size_t bytes) -> int {
        MSC_HIP(hipMalloc(dst, std::max<size_t>(bytes, 64)));
        if (bytes) MSC_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return MSC_OK;
    };
    c->dev = ctx->device;
    int rc;
    if ((rc = put(&c->d_ops, c->ops.data(), c->ops.size() * sizeof(DevOp)))) return rc;
    if ((rc = put(&c->d_g1, g1.data(), g1.size() * sizeof(double)))) return rc;
    if ((rc = put(&c->d_g4, g4.data(), g4.size() * sizeof(double)))) return rc;
    // the screen's table: per channel and Pauli code the XOR of the code's
    // basis-component signatures (one lookup per fault)
    {
        const int W = c->words;
        std::vector<int32_t> soff(std::max(1, c->n_channels));
        std::vector<uint64_t> comb;
        for (int ch = 0; ch < c->n_channels; ++ch) {
            const int k = c->chan_kind[ch];
            const int codes = k == CH_DEP1 ? 4 : k == CH_DEP2 ? 16 : k == CH_XERR ? 2 : 64;
            // entry index of the channel's code 0, shifted, with its kind
            // in the low two bits: the screen reads both with one load
            const size_t entry = comb.size() / std::max(1, W);
            if (entry >= (size_t(1) << 29))
                return set_error(MSC_E_INVALID, "screen table above 2^29 entries");
            soff[ch] = static_cast<int32_t>(entry << 2) | k;
            for (int p = 0; p < codes; ++p)
                for (int w = 0; w < W; ++w) {
                    uint64_t x = 0;
                    for (int b = 0; b < kFaultComponents; ++b)
                        if ((p >> b) & 1)
                            x ^= c->sig[(static_cast<size_t>(ch) * kFaultComponents + b) * W + w];
                    comb.push_back(x);
                }
        }
        if ((rc = put(&c->d_sig, comb.data(), comb.size() * sizeof(uint64_t)))) return rc;
        if ((rc = put(&c->d_sig_off, soff.data(), soff.size() * sizeof(int32_t)))) return rc;
    }
    if ((rc = put(&c->d_expected, c->expected.data(), c->expected.size()))) return rc;
    std::vector<uint8_t> kind(c->chan_kind.begin(), c->chan_kind.end());
    if ((rc = put(&c->d_kind, kind.data(), kind.size()))) return rc;
    std::vector<int32_t> segm;
    for (const msc_segment& g : c->segs) segm.push_back(g.first_meas);
    if ((rc = put(&c->d_segm, segm.data(), segm.size() * sizeof(int32_t)))) return rc;
    return MSC_OK;
}

extern "C" int msc_prescreen_tables(const msc_circuit* c, uint64_t* sig, int32_t* decided) {
    if (!c) return set_error(MSC_E_INVALID, "null circuit");
    if (sig) std::copy(c->sig.begin(), c->sig.end(), sig);
    if (decided) std::copy(c->decided.begin(), c->decided.end(), decided);
    return MSC_OK;
}

// ---------------------------------------------------------------------------
// simulation

namespace {

struct Layout {
    std::vector<int32_t> cap;
    std::vector<int64_t> off, half;
    int64_t slot_elems = 0;     // elements of T per slot
    int64_t scratch = 0;        // doubles per slot
};

// side_in: the widest theta the shot kernel factorises itself (in its HBM
// scratch when wider than its LDS vectors); wider ones go to the engine
Layout make_layout(int n, int chi_max, int side_in) {
    Layout L;
    L.cap.resize(n + 1);
    // every inner bond may reach chi_max: swapping an unentangled qubit
    // moves a bond dimension to a neighbouring bond unchanged
    for (int k = 0; k <= n; ++k) L.cap[k] = (k == 0 || k == n) ? 1 : chi_max;
    L.off.resize(n);
    L.half.resize(n);
    int64_t pos = 0;
    for (int k = 0; k < n; ++k) {
        int64_t elems = static_cast<int64_t>(L.cap[k]) * 2 * L.cap[k + 1];
        elems = (elems + 31) / 32 * 32;   // 128-byte aligned planes for FP32
        L.off[k] = pos;
        L.half[k] = elems;
        pos += 2 * elems;
    }
    L.slot_elems = (pos + 63) / 64 * 64;
    const int64_t s = std::min<int64_t>(2ll * chi_max, side_in);
    const int64_t cm = chi_max;
    // the shot kernel's FP64 scratch: theta copy + padded vectors of an
    // in-kernel factorisation, the staged neighbour of a centre move (at
    // most 64 kept vectors of 2 chi_max), or a product swap's bond matrix,
    // then the per-vector arrays (6 x 2 kMaxChiKernel doubles)
    const int64_t work = std::max({4 * s * s + 4 * s, 4 * 64 * cm, 2 * cm * cm});
    L.scratch = work + 64 + 6 * 2 * kMaxChiKernel;
    return L;
}

// Bond cap of the wavefront kernel's slots: the automatic choice, and the
// largest a caller may ask for.
constexpr int kAutoWaveChi = 16;
constexpr int kMaxWaveChi = 64;

// Options of one shot-kernel run.
struct RunCfg {
    int precision = MSC_FP64;
    int chi_max = 256;
    double tau = 1e-12, tau_rej = 1e-6, tau_fail = 1e-4;
    int n_slots = 0;
    int lds_width = 32;
    int park_side = 0;           // 0: the shot kernel does every update
    int wave_chi = 0;            // > 0: one shot per wavefront in slots of this bond cap
    bool graphs = false;
    LxTiles tiles[kLxBuckets];
};

}  // namespace

// The engine's tile shapes when no autotune cache names them: per bucket of
// theta sides (<= 128, <= 256, <= 512, larger).
static void default_tiles(int precision, LxTiles* t) {
    for (int b = 0; b < kLxBuckets; ++b) {
        if (precision == MSC_FP64) t[b] = b == 0 ? LxTiles{32, 32, 32} : LxTiles{64, 32, 64};
        else if (precision == MSC_BF16X3) t[b] = b == 0 ? LxTiles{64, 32, 64} : LxTiles{64, 64, 64};
        else t[b] = b == 0 ? LxTiles{64, 32, 64} : LxTiles{128, 64, 64};
    }
}

// One round of the engine on the context's stream: plan, contraction and
// Gram per bucket, factor, park count cleared, shot kernel resumed.
// With `timed`, events at the phase boundaries (lxev[0..4]; not in a graph).
static int enqueue_lx_round(msc_ctx* ctx, const RunCfg& cfg, bool small, const MpsArgs& a,
                            const LxArgs& lx, const LxFactor& fac, int n_slots, bool timed) {
    const int grid = ctx->n_cu * 4;
    hipStream_t s = ctx->stream;
    if (timed) MSC_HIP(hipEventRecord(ctx->lxev[0], s));
    MSC_HIP(launch_lx_plan(lx, cfg.tiles, s));
    for (int b = 0; b < kLxBuckets; ++b)
        MSC_HIP(launch_lx_contract(cfg.precision, lx, b, cfg.tiles[b], grid, s));
    if (timed) MSC_HIP(hipEventRecord(ctx->lxev[1], s));
    for (int b = 0; b < kLxBuckets; ++b)
        MSC_HIP(launch_lx_gram(cfg.precision, lx, b, cfg.tiles[b], grid, s));
    if (timed) MSC_HIP(hipEventRecord(ctx->lxev[2], s));
    MSC_HIP(launch_lx_factor(cfg.precision, lx, fac, n_slots, s));
    MSC_HIP(launch_lx_clear(a.park_count, s));
    if (timed) MSC_HIP(hipEventRecord(ctx->lxev[3], s));
    MSC_HIP(launch_mps(cfg.precision, small, a, n_slots, s));
    if (timed) MSC_HIP(hipEventRecord(ctx->lxev[4], s));
    return MSC_OK;
}

// The shot kernels' arguments that do not depend on the slot layout.
static MpsArgs shot_args(const msc_circuit* c, const RunCfg& cfg, int64_t n, int64_t n_csr,
                         const int64_t* off, const int32_t* chan, const uint8_t* pauli,
                         const int64_t* shot_idx, msc_shot_result* out, int calibrate,
                         double* cal_p, uint8_t* cal_e, int ck_mode, const PrefixCk* pk,
                         const int64_t* n_dev, double* surv) {
    MpsArgs a{};
    a.ops = static_cast<const DevOp*>(c->d_ops);
    a.n_ops = static_cast<int32_t>(c->ops.size());
    a.n_sites = c->n;
    a.g1 = static_cast<const double*>(c->d_g1);
    a.g4 = static_cast<const double*>(c->d_g4);
    a.shot_off = off;
    a.chan = chan;
    a.pauli = pauli;
    a.shot_idx = shot_idx;
    a.n_shots = n;
    a.n_dev = n_dev;
    a.n_csr = n_csr;
    a.expected = static_cast<const uint8_t*>(c->d_expected);
    a.out = out;
    a.chi_max = cfg.chi_max;
    a.tau = cfg.tau;
    a.tau_rej = cfg.tau_rej;
    a.tau_fail = cfg.tau_fail;
    const double r = 1.0 / std::sqrt(2.0);
    a.t0r = r;
    a.t0i = 0.0;
    if (c->target == 'T') {
        a.t1r = 0.5;
        a.t1i = 0.5;
    } else {
        a.t1r = 0.0;
        a.t1i = r;
    }
    a.calibrate = calibrate;
    a.cal_p = cal_p;
    a.cal_e = cal_e;
    a.ck_mode = pk ? ck_mode : 0;
    if (a.ck_mode) {
        a.n_ck = pk->n_ck;
        a.ck_k = pk->ck_k;
        a.ck_op = static_cast<const int32_t*>(pk->d_op);
        a.ck_avail = static_cast<int32_t*>(pk->d_avail);
        a.ck_off = static_cast<int64_t*>(pk->d_off);
        a.ck_hdr = static_cast<CkHdr*>(pk->d_hdr);
        a.ck_data = pk->d_data;
        a.ck_cap = pk->cap;
        a.ck_pm = static_cast<double*>(pk->d_pm);
    }
    if (surv) {
        a.surv = surv;
        a.seg_meas = static_cast<const int32_t*>(c->d_segm);
        a.n_seg = static_cast<int32_t>(c->segs.size());
    }
    return a;
}

static int enqueue_shots(msc_ctx* ctx, const msc_circuit* c, const RunCfg& cfg, int64_t n,
                         int64_t n_csr, const int64_t* off, const int32_t* chan,
                         const uint8_t* pauli, const int64_t* shot_idx, msc_shot_result* out,
                         int calibrate, double* cal_p, uint8_t* cal_e, int ck_mode,
                         const PrefixCk* pk, const int64_t* n_dev, double* surv,
                         const int64_t* perm_in);

// The wavefront kernel's pass over the shots (slots of bond cap wave_chi,
// one shot per wavefront, shots taken from a shared counter), then the shots
// that outgrew their slots, from their start (no fork) in the workgroup
// kernel with the caller's other options.  One stream synchronisation reads
// how many there are.
static int enqueue_wave(msc_ctx* ctx, const msc_circuit* c, const RunCfg& cfg, int64_t n,
                        int64_t n_csr, const int64_t* off, const int32_t* chan,
                        const uint8_t* pauli, const int64_t* shot_idx, msc_shot_result* out,
                        int ck_mode, const PrefixCk* pk, const int64_t* n_dev, double* surv) {
    const int precision = cfg.precision, cw = cfg.wave_chi;
    Layout L = make_layout(c->n, cw, 2 * cw);
    if (L.slot_elems >= (int64_t(1) << 31)) return set_error(MSC_E_INVALID, "slot above 2^31 elements");
    int64_t teams = cfg.n_slots > 0 ? cfg.n_slots
                                    : static_cast<int64_t>(ctx->n_cu) *
                                          mps_wave_blocks_per_cu(precision) * kWaveTeams;
    teams = std::max<int64_t>(1, std::min<int64_t>(teams, n));
    const int grid = static_cast<int>((teams + kWaveTeams - 1) / kWaveTeams);
    const int64_t slots = static_cast<int64_t>(grid) * kWaveTeams;
    const size_t tsize = precision == MSC_FP64 ? sizeof(double) : sizeof(float);
    void *arena, *scratch, *dcap, *doff, *dhalf, *dperm, *dctr, *dlist;
    int rc;
    if ((rc = ctx_buf(ctx, "w_arena", static_cast<size_t>(slots) * L.slot_elems * tsize, &arena))) return rc;
    if ((rc = ctx_buf(ctx, "w_scratch", static_cast<size_t>(slots) * L.scratch * sizeof(double), &scratch))) return rc;
    if ((rc = ctx_buf(ctx, "w_cap", L.cap.size() * sizeof(int32_t), &dcap))) return rc;
    if ((rc = ctx_buf(ctx, "w_off", L.off.size() * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "w_half", L.half.size() * sizeof(int64_t), &dhalf))) return rc;
    if ((rc = ctx_buf(ctx, "w_perm", static_cast<size_t>(n) * sizeof(int64_t), &dperm))) return rc;
    // the shared shot counter (8 bytes) and the retry count (4 bytes)
    if ((rc = ctx_buf(ctx, "w_ctr", 16, &dctr))) return rc;
    if ((rc = ctx_buf(ctx, "w_retry", static_cast<size_t>(n) * sizeof(int64_t), &dlist))) return rc;
    if (ctx->wlayout_n != c->n || ctx->wlayout_chi != cw) {
        MSC_HIP(hipMemcpyAsync(dcap, L.cap.data(), L.cap.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipMemcpyAsync(doff, L.off.data(), L.off.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipMemcpyAsync(dhalf, L.half.data(), L.half.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipStreamSynchronize(ctx->stream));
        ctx->wlayout_n = c->n;
        ctx->wlayout_chi = cw;
    }
    MpsArgs a = shot_args(c, cfg, n, n_csr, off, chan, pauli, shot_idx, out, 0, nullptr, nullptr,
                          ck_mode, pk, n_dev, surv);
    a.perm = static_cast<const int64_t*>(dperm);
    a.arena = arena;
    a.slot_stride = L.slot_elems;
    a.site_off = static_cast<const int64_t*>(doff);
    a.site_half = static_cast<const int64_t*>(dhalf);
    a.cap = static_cast<const int32_t*>(dcap);
    a.scratch = static_cast<double*>(scratch);
    a.scratch_stride = L.scratch;
    a.next = static_cast<unsigned long long*>(dctr);
    a.retry_count = reinterpret_cast<int32_t*>(static_cast<char*>(dctr) + 8);
    a.retry_list = static_cast<int64_t*>(dlist);
    ctx->lx_stats = msc_engine_stats{};
    MSC_HIP(hipMemsetAsync(dctr, 0, 16, ctx->stream));
    void* otmp;
    if ((rc = ctx_buf(ctx, "order_tmp", order_tmp_bytes(n), &otmp))) return rc;
    MSC_HIP(launch_order(n, n_dev, off, shot_idx, n_csr, chan,
                         a.ck_mode == 2 ? c->n_channels : 0, static_cast<int64_t*>(dperm), otmp,
                         ctx->stream));
    MSC_HIP(launch_mps_wave(precision, a, grid, ctx->stream));
    int32_t n_retry = 0;
    MSC_HIP(hipMemcpyAsync(&n_retry, a.retry_count, sizeof(n_retry), hipMemcpyDeviceToHost,
                           ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    if (n_retry > 0) {
        RunCfg wg = cfg;
        wg.wave_chi = 0;
        rc = enqueue_shots(ctx, c, wg, n_retry, n_csr, off, chan, pauli, shot_idx, out, 0, nullptr,
                           nullptr, 0, nullptr, nullptr, surv, a.retry_list);
        if (rc) return rc;
    }
    ctx->lx_stats.wave_slots = slots;
    ctx->lx_stats.wave_retries = n_retry;
    return MSC_OK;
}

// Enqueues the order and shot kernels on the context's stream.  n bounds the
// shots (a device count n_dev, if given, may be smaller).  With the engine
// on (cfg.park_side > 0) the shot kernel parks every shot at a two-site
// update wider than park_side; the host then runs engine rounds (each does
// every parked update and resumes the shot kernel) until a launch parks
// nothing, reading the park count after each round (one stream
// synchronisation per round).  Otherwise nothing waits here.
static int enqueue_shots(msc_ctx* ctx, const msc_circuit* c, const RunCfg& cfg, int64_t n,
                         int64_t n_csr, const int64_t* off, const int32_t* chan,
                         const uint8_t* pauli, const int64_t* shot_idx, msc_shot_result* out,
                         int calibrate, double* cal_p, uint8_t* cal_e, int ck_mode,
                         const PrefixCk* pk, const int64_t* n_dev, double* surv,
                         const int64_t* perm_in) {
    if (cfg.wave_chi > 0 && !calibrate)
        return enqueue_wave(ctx, c, cfg, n, n_csr, off, chan, pauli, shot_idx, out, ck_mode, pk,
                            n_dev, surv);
    const int precision = cfg.precision, chi_max = cfg.chi_max;
    const bool engine = cfg.park_side > 0;
    Layout L = make_layout(c->n, chi_max, engine ? cfg.park_side : 2 * chi_max);
    // the shot kernel keeps the site offsets within a slot as 32-bit values
    if (L.slot_elems >= (int64_t(1) << 31)) return set_error(MSC_E_INVALID, "slot above 2^31 elements");
    const bool small = cfg.lds_width == 32;
    int n_slots = cfg.n_slots;
    if (n_slots <= 0) n_slots = ctx->n_cu * mps_blocks_per_cu(precision, small);
    n_slots = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_slots, n)));
    if (engine) n_slots = std::min(n_slots, kLxMaxParked);
    const size_t tsize = precision == MSC_FP64 ? sizeof(double) : sizeof(float);
    void *arena, *scratch, *dcap, *doff, *dhalf, *dperm;
    int rc;
    if ((rc = ctx_buf(ctx, "arena", static_cast<size_t>(n_slots) * L.slot_elems * tsize, &arena))) return rc;
    if ((rc = ctx_buf(ctx, "scratch", static_cast<size_t>(n_slots) * L.scratch * sizeof(double), &scratch))) return rc;
    if ((rc = ctx_buf(ctx, "cap", L.cap.size() * sizeof(int32_t), &dcap))) return rc;
    if ((rc = ctx_buf(ctx, "off", L.off.size() * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "half", L.half.size() * sizeof(int64_t), &dhalf))) return rc;
    if ((rc = ctx_buf(ctx, "perm", static_cast<size_t>(n) * sizeof(int64_t), &dperm))) return rc;
    if (ctx->layout_n != c->n || ctx->layout_chi != chi_max) {
        // the layout depends on (n, chi_max) only: uploaded when it changes
        MSC_HIP(hipMemcpyAsync(dcap, L.cap.data(), L.cap.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipMemcpyAsync(doff, L.off.data(), L.off.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipMemcpyAsync(dhalf, L.half.data(), L.half.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        MSC_HIP(hipStreamSynchronize(ctx->stream));
        ctx->layout_n = c->n;
        ctx->layout_chi = chi_max;
    }
    MpsArgs a = shot_args(c, cfg, n, n_csr, off, chan, pauli, shot_idx, out, calibrate, cal_p,
                          cal_e, ck_mode, pk, n_dev, surv);
    a.perm = perm_in ? perm_in : static_cast<const int64_t*>(dperm);
    a.arena = arena;
    a.slot_stride = L.slot_elems;
    a.site_off = static_cast<const int64_t*>(doff);
    a.site_half = static_cast<const int64_t*>(dhalf);
    a.cap = static_cast<const int32_t*>(dcap);
    a.scratch = static_cast<double*>(scratch);
    a.scratch_stride = L.scratch;
    ctx->lx_stats = msc_engine_stats{};
    void *dstate = nullptr, *dcount = nullptr, *dlist = nullptr, *dflops = nullptr;
    if (engine) {
        if ((rc = ctx_buf(ctx, "lx_state", static_cast<size_t>(n_slots) * sizeof(ShotState), &dstate))) return rc;
        if ((rc = ctx_buf(ctx, "lx_count", sizeof(int32_t), &dcount))) return rc;
        if ((rc = ctx_buf(ctx, "lx_list", static_cast<size_t>(n_slots) * sizeof(int32_t), &dlist))) return rc;
        if ((rc = ctx_buf(ctx, "lx_flops", 2 * sizeof(double) + 4 * sizeof(uint64_t), &dflops))) return rc;
        a.park_side = cfg.park_side;
        a.state = static_cast<ShotState*>(dstate);
        a.park_count = static_cast<int32_t*>(dcount);
        a.park_list = static_cast<int32_t*>(dlist);
        MSC_HIP(launch_lx_reset(a.state, n_slots, a.park_count, static_cast<double*>(dflops),
                                reinterpret_cast<unsigned long long*>(static_cast<double*>(dflops) + 2),
                                ctx->stream));
    }
    if (!perm_in) {
        void* otmp;
        if ((rc = ctx_buf(ctx, "order_tmp", order_tmp_bytes(n), &otmp))) return rc;
        MSC_HIP(launch_order(n, n_dev, off, shot_idx, n_csr, chan,
                             a.ck_mode == 2 ? c->n_channels : 0, static_cast<int64_t*>(dperm),
                             otmp, ctx->stream));
    }
    if (engine) MSC_HIP(hipEventRecord(ctx->lxev[4], ctx->stream));
    MSC_HIP(launch_mps(precision, small, a, n_slots, ctx->stream));
    if (engine) MSC_HIP(hipEventRecord(ctx->lxev[5], ctx->stream));
    if (!engine) return MSC_OK;
    msc_engine_stats& es = ctx->lx_stats;
    bool first = true;

    // ---- engine rounds until a shot-kernel launch parks nothing
    LxArgs lx{};
    LxFactor fac{};
    bool have_bufs = false;
    for (;;) {
        int32_t parked = 0;
        MSC_HIP(hipMemcpyAsync(&parked, a.park_count, sizeof(parked), hipMemcpyDeviceToHost,
                               ctx->stream));
        MSC_HIP(hipStreamSynchronize(ctx->stream));
        float t = 0.f;
        if (first) {
            MSC_HIP(hipEventElapsedTime(&t, ctx->lxev[4], ctx->lxev[5]));
            es.shot_ms += t;
            first = false;
        } else if (!cfg.graphs) {
            double* acc[4] = {&es.contract_ms, &es.gram_ms, &es.factor_ms, &es.shot_ms};
            for (int q = 0; q < 4; ++q) {
                MSC_HIP(hipEventElapsedTime(&t, ctx->lxev[q], ctx->lxev[q + 1]));
                *acc[q] += t;
            }
        }
        if (parked == 0) break;
        es.updates += parked;
        ++es.rounds;
        if (!have_bufs) {
            // theta and Gram buffers per slot, sized for sides up to 2 chi_max
            const int64_t S = 2ll * chi_max;
            void *dplan, *dtheta, *dgram;
            if ((rc = ctx_buf(ctx, "lx_plan", sizeof(LxPlan), &dplan))) return rc;
            if ((rc = ctx_buf(ctx, "lx_theta", static_cast<size_t>(n_slots) * 2 * S * S * tsize, &dtheta))) return rc;
            if ((rc = ctx_buf(ctx, "lx_gram", static_cast<size_t>(n_slots) * lx_gram_doubles(S) * sizeof(double), &dgram))) return rc;
            lx.state = a.state;
            lx.park_count = a.park_count;
            lx.park_list = a.park_list;
            lx.plan = static_cast<LxPlan*>(dplan);
            lx.arena = arena;
            lx.slot_stride = L.slot_elems;
            lx.site_off = a.site_off;
            lx.site_half = a.site_half;
            lx.g4 = a.g4;
            lx.theta = dtheta;
            lx.theta_stride = 2 * S * S;
            lx.gram = static_cast<double*>(dgram);
            lx.gram_stride = lx_gram_doubles(S);
            lx.n_slots = n_slots;
            lx.flops = static_cast<double*>(dflops);
            lx.counts = reinterpret_cast<unsigned long long*>(lx.flops + 2);
            fac.cap = a.cap;
            fac.chi_max = chi_max;
            fac.tau = cfg.tau;
            have_bufs = true;
        }
        if (cfg.graphs) {
            // the round's launches depend only on these argument bytes
            std::string key(reinterpret_cast<const char*>(&a), sizeof(a));
            key.append(reinterpret_cast<const char*>(&lx), sizeof(lx));
            key.append(reinterpret_cast<const char*>(&fac), sizeof(fac));
            key.append(reinterpret_cast<const char*>(cfg.tiles), sizeof(cfg.tiles));
            key.append(reinterpret_cast<const char*>(&precision), sizeof(precision));
            key.append(reinterpret_cast<const char*>(&n_slots), sizeof(n_slots));
            key.append(small ? "s" : "w");
            if (!ctx->lx_exec || ctx->lx_key != key) {
                if (ctx->lx_exec) (void)hipGraphExecDestroy(ctx->lx_exec);
                ctx->lx_exec = nullptr;
                hipGraph_t g = nullptr;
                MSC_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                const int rc2 = enqueue_lx_round(ctx, cfg, small, a, lx, fac, n_slots, false);
                hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
                if (rc2) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc2;
                }
                if (e2 != hipSuccess) return set_error(MSC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e2));
                e2 = hipGraphInstantiate(&ctx->lx_exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e2 != hipSuccess) {
                    ctx->lx_exec = nullptr;
                    return set_error(MSC_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
                }
                ctx->lx_key = key;
            }
            MSC_HIP(hipGraphLaunch(ctx->lx_exec, ctx->stream));
        } else {
            if ((rc = enqueue_lx_round(ctx, cfg, small, a, lx, fac, n_slots, true))) return rc;
        }
    }
    if (have_bufs) {
        double fl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // 2 flop sums, 4 counts
        MSC_HIP(hipMemcpy(fl, lx.flops, sizeof(fl), hipMemcpyDeviceToHost));
        es.contract_flops = fl[0];
        es.gram_flops = fl[1];
        uint64_t cnt[4];
        std::memcpy(cnt, fl + 2, sizeof(cnt));
        es.factor_lds = static_cast<int64_t>(cnt[0]);
        es.factor_wide = static_cast<int64_t>(cnt[1]);
        es.overlapping = static_cast<int64_t>(cnt[2]);
        es.sweeps = static_cast<int64_t>(cnt[3]);
    }
    return MSC_OK;
}

static int run_shots(msc_ctx* ctx, const msc_circuit* c, const RunCfg& cfg, int64_t n,
                     int64_t n_csr, const int64_t* off, const int32_t* chan, const uint8_t* pauli,
                     const int64_t* shot_idx, msc_shot_result* out, int calibrate,
                     double* cal_p, uint8_t* cal_e, const char* timer, int ck_mode = 0,
                     const PrefixCk* pk = nullptr) {
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    int rc = enqueue_shots(ctx, c, cfg, n, n_csr, off, chan, pauli, shot_idx, out, calibrate,
                           cal_p, cal_e, ck_mode, pk, nullptr, nullptr, nullptr);
    if (rc) return rc;
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (timer) ctx->last_ms[timer] = ms;
    ctx->lx_stats.total_ms = ms;
    return MSC_OK;
}

extern "C" int msc_circuit_calibrate(msc_ctx* ctx, msc_circuit* c) {
    if (!ctx || !c) return set_error(MSC_E_INVALID, "null argument");
    MSC_HIP(hipSetDevice(ctx->device));
    int rc = upload(ctx, c);
    if (rc) return rc;
    void *doff, *dchan, *dpa, *dout, *dp, *de;
    const int nm = std::max(1, c->n_meas);
    if ((rc = ctx_buf(ctx, "cal_off", 2 * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "cal_chan", 64, &dchan))) return rc;
    if ((rc = ctx_buf(ctx, "cal_pa", 64, &dpa))) return rc;
    if ((rc = ctx_buf(ctx, "cal_out", sizeof(msc_shot_result), &dout))) return rc;
    if ((rc = ctx_buf(ctx, "cal_p", nm * sizeof(double), &dp))) return rc;
    if ((rc = ctx_buf(ctx, "cal_e", nm, &de))) return rc;
    int64_t zero[2] = {0, 0};
    MSC_HIP(hipMemcpy(doff, zero, sizeof(zero), hipMemcpyHostToDevice));
    // the noiseless FP64 run, likelier outcome recorded at every
    // measurement; bond cap 256 first (small slot), the full cap if it binds
    msc_shot_result res;
    for (int chi_max : {256, kMaxChiKernel}) {
        RunCfg cfg;
        cfg.precision = MSC_FP64;
        cfg.chi_max = chi_max;
        cfg.tau = 1e-12;
        cfg.tau_rej = 0.0;
        cfg.n_slots = 1;
        cfg.lds_width = 64;
        default_tiles(cfg.precision, cfg.tiles);
        rc = run_shots(ctx, c, cfg, 1, 1, static_cast<int64_t*>(doff),
                       static_cast<int32_t*>(dchan), static_cast<uint8_t*>(dpa), nullptr,
                       static_cast<msc_shot_result*>(dout), 1, static_cast<double*>(dp),
                       static_cast<uint8_t*>(de), "calibrate");
        if (rc) return rc;
        MSC_HIP(hipMemcpy(&res, dout, sizeof(res), hipMemcpyDeviceToHost));
        if (!(res.status & MSC_SHOT_CHI_CAP)) break;
    }
    std::vector<double> p(nm);
    std::vector<uint8_t> e(nm);
    MSC_HIP(hipMemcpy(p.data(), dp, nm * sizeof(double), hipMemcpyDeviceToHost));
    MSC_HIP(hipMemcpy(e.data(), de, nm, hipMemcpyDeviceToHost));
    c->noiseless = res;
    for (int m = 0; m < c->n_meas; ++m) {
        if (!(std::fabs(p[m] - 1.0) <= 1e-10))
            return set_error(MSC_E_NONDETERMINISTIC, "measurement " + std::to_string(m) +
                                                         " has p(e) = " + std::to_string(p[m]));
    }
    if (!(res.infid <= 1e-10))
        return set_error(MSC_E_NONDETERMINISTIC,
                         "noiseless infidelity " + std::to_string(res.infid));
    if (res.status & MSC_SHOT_CHI_CAP)
        return set_error(MSC_E_NONDETERMINISTIC, "noiseless run exceeded the bond cap");
    for (int m = 0; m < c->n_meas; ++m) c->expected[m] = e[m];
    MSC_HIP(hipMemcpy(c->d_expected, c->expected.data(), c->n_meas, hipMemcpyHostToDevice));
    c->calibrated = true;
    free_prefix(c->prefix);   // checkpoints follow the expected outcomes
    free_camps_prefix(c->camps_prefix);
    return MSC_OK;
}

// Checkpoints of the noiseless run (the shot with no fault) in the batch's
// precision and kernel variant: one before the fault op of every ck_k-th
// channel (ck_k chosen for at most 256 of them) and one before the final
// read-out, written densely while they fit in kPrefixBytes.  A shot whose
// first fault is on channel c forks from checkpoint c / ck_k; the ops it
// skips are exactly the fault-free ops it would have run, in the same
// kernel with the same arithmetic, so its result does not change.
static constexpr int64_t kPrefixBytes = int64_t(2) << 30;

static int ensure_prefix(msc_ctx* ctx, msc_circuit* c, const RunCfg& cfg) {
    PrefixCk& pk = c->prefix;
    const int precision = cfg.precision, chi_max = cfg.chi_max, lds_width = cfg.lds_width;
    const double tau = cfg.tau, tau_rej = cfg.tau_rej;
    if (pk.valid && pk.dev == ctx->device && pk.precision == precision &&
        pk.chi_max == chi_max && pk.lds_width == lds_width && pk.tau == tau &&
        pk.tau_rej == tau_rej && pk.park_side == cfg.park_side && pk.wave_chi == cfg.wave_chi)
        return MSC_OK;
    free_prefix(pk);
    pk.dev = ctx->device;
    const int M = c->n_channels;
    pk.ck_k = std::max(1, (M + 255) / 256);
    const int n_reg = (M + pk.ck_k - 1) / pk.ck_k;
    pk.n_ck = n_reg + 1;
    std::vector<int32_t> ck_op(pk.n_ck);
    for (int j = 0; j < n_reg; ++j) ck_op[j] = c->chan_op[static_cast<size_t>(j) * pk.ck_k];
    ck_op[n_reg] = static_cast<int32_t>(c->ops.size()) - 1;   // OP_FINAL
    for (int j = 0; j + 1 < pk.n_ck; ++j)
        if (!(ck_op[j] >= 0 && ck_op[j] < ck_op[j + 1]))
            return set_error(MSC_E_INVALID, "checkpoint ops not increasing");
    const size_t tsize = precision == MSC_FP64 ? sizeof(double) : sizeof(float);
    pk.cap = kPrefixBytes / static_cast<int64_t>(tsize);
    auto dmalloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 64));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return set_error(MSC_E_OOM, std::string("checkpoints: ") + hipGetErrorString(e));
        }
        return MSC_OK;
    };
    int rc;
    if ((rc = dmalloc(&pk.d_op, pk.n_ck * sizeof(int32_t)))) return rc;
    if ((rc = dmalloc(&pk.d_avail, sizeof(int32_t)))) return rc;
    if ((rc = dmalloc(&pk.d_off, pk.n_ck * sizeof(int64_t)))) return rc;
    if ((rc = dmalloc(&pk.d_hdr, pk.n_ck * sizeof(CkHdr)))) return rc;
    if ((rc = dmalloc(&pk.d_data, static_cast<size_t>(pk.cap) * tsize))) return rc;
    if ((rc = dmalloc(&pk.d_pm, static_cast<size_t>(std::max(1, c->n_meas)) * sizeof(double))))
        return rc;
    const int32_t zero = 0;
    MSC_HIP(hipMemcpy(pk.d_op, ck_op.data(), pk.n_ck * sizeof(int32_t), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(pk.d_avail, &zero, sizeof(zero), hipMemcpyHostToDevice));
    void *doff, *dchan, *dpa, *dout;
    if ((rc = ctx_buf(ctx, "cal_off", 2 * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "cal_chan", 64, &dchan))) return rc;
    if ((rc = ctx_buf(ctx, "cal_pa", 64, &dpa))) return rc;
    if ((rc = ctx_buf(ctx, "cal_out", sizeof(msc_shot_result), &dout))) return rc;
    int64_t zz[2] = {0, 0};
    MSC_HIP(hipMemcpy(doff, zz, sizeof(zz), hipMemcpyHostToDevice));
    RunCfg one = cfg;
    one.n_slots = 1;
    rc = run_shots(ctx, c, one, 1, 1, static_cast<int64_t*>(doff), static_cast<int32_t*>(dchan),
                   static_cast<uint8_t*>(dpa), nullptr, static_cast<msc_shot_result*>(dout), 0,
                   nullptr, nullptr, "prefix", 1, &pk);
    if (rc) {
        free_prefix(pk);
        return rc;
    }
    MSC_HIP(hipMemcpy(&pk.avail, pk.d_avail, sizeof(int32_t), hipMemcpyDeviceToHost));
    msc_shot_result res;
    MSC_HIP(hipMemcpy(&res, dout, sizeof(res), hipMemcpyDeviceToHost));
    if (!(res.status & MSC_SHOT_DONE)) {
        free_prefix(pk);
        return set_error(MSC_E_NONDETERMINISTIC, "noiseless run rejected in the batch precision");
    }
    pk.precision = precision;
    pk.chi_max = chi_max;
    pk.lds_width = lds_width;
    pk.park_side = cfg.park_side;
    pk.wave_chi = cfg.wave_chi;
    pk.tau = tau;
    pk.tau_rej = tau_rej;
    pk.build_ms = static_cast<float>(ctx->last_ms["prefix"]);
    pk.valid = true;
    return MSC_OK;
}

// Tile shapes for `precision` from an msc_autotune cache file: a JSON object
// whose "entries" array holds objects with integer fields "precision",
// "bucket", "rows", "b" and "gram" (other fields are ignored).  Entries of
// other precisions are skipped; a bucket without an entry keeps its shapes.
static int read_tune_cache(const char* path, int precision, LxTiles* tiles) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(MSC_E_INVALID, std::string("cannot open autotune cache ") + path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    const size_t at = text.find("\"entries\"");
    if (at == std::string::npos) return set_error(MSC_E_PARSE, "autotune cache without entries");
    size_t pos = text.find('[', at);
    const size_t end = text.find(']', pos == std::string::npos ? at : pos);
    if (pos == std::string::npos || end == std::string::npos)
        return set_error(MSC_E_PARSE, "autotune cache: entries is not an array");
    while (true) {
        const size_t o = text.find('{', pos);
        if (o == std::string::npos || o > end) break;
        const size_t cl = text.find('}', o);
        if (cl == std::string::npos || cl > end) return set_error(MSC_E_PARSE, "autotune cache: open entry");
        const std::string obj = text.substr(o, cl - o);
        auto field = [&](const char* name, long* out) {
            const std::string key = std::string("\"") + name + "\"";
            const size_t kp = obj.find(key);
            if (kp == std::string::npos) return false;
            const size_t colon = obj.find(':', kp + key.size());
            if (colon == std::string::npos) return false;
            char* e = nullptr;
            *out = std::strtol(obj.c_str() + colon + 1, &e, 10);
            return e != obj.c_str() + colon + 1;
        };
        long pr, bk, rows, b, gram;
        if (!(field("precision", &pr) && field("bucket", &bk) && field("rows", &rows) &&
              field("b", &b) && field("gram", &gram)))
            return set_error(MSC_E_PARSE, "autotune cache: entry without precision, bucket, "
                                          "rows, b or gram");
        if (pr == precision && bk >= 0 && bk < kLxBuckets) {
            LxTiles v[16];
            const int nvar = lx_tile_variants(precision, v, 16);
            bool known_c = false, known_g = false;
            for (int i = 0; i < nvar; ++i) {
                known_c |= v[i].cm_rows == rows && v[i].cm_b == b;
                known_g |= v[i].gram == gram;
            }
            if (!(known_c && known_g))
                return set_error(MSC_E_INVALID, "autotune cache names a tile shape the library "
                                                "does not have");
            tiles[bk] = LxTiles{static_cast<int32_t>(rows), static_cast<int32_t>(b),
                                static_cast<int32_t>(gram)};
        }
        pos = cl + 1;
    }
    return MSC_OK;
}

// The run options of msc_sim_opts (validated), with the engine's tile shapes
// from the autotune cache when one is named.  With wave_chi 0 and lds_width
// 0 the wavefront kernel (slots of bond cap 16) takes the shots of circuits
// whose calibrated noiseless run stays within bond 16.
static int sim_cfg(const msc_sim_opts* o, const msc_circuit* c, RunCfg* cfg) {
    if (o->precision != MSC_FP64 && o->precision != MSC_FP32 && o->precision != MSC_BF16X3)
        return set_error(MSC_E_INVALID, "unknown precision");
    if (o->chi_max < 1 || o->chi_max > kMaxChiKernel)
        return set_error(MSC_E_INVALID, "chi_max must be in [1, 1024]");
    if (o->lds_width != 0 && o->lds_width != 32 && o->lds_width != 64)
        return set_error(MSC_E_INVALID, "lds_width must be 0, 32 or 64");
    if (o->prefix != 0 && o->prefix != 1) return set_error(MSC_E_INVALID, "prefix must be 0 or 1");
    if (o->use_graphs != 0 && o->use_graphs != 1)
        return set_error(MSC_E_INVALID, "use_graphs must be 0 or 1");
    if (o->large_side < -1 || o->large_side == 1)
        return set_error(MSC_E_INVALID, "large_side must be -1, 0 or at least 2");
    if (o->wave_chi < -1 || o->wave_chi == 1 || o->wave_chi > kMaxWaveChi)
        return set_error(MSC_E_INVALID, "wave_chi must be -1, 0 or in [2, 64]");
    cfg->precision = o->precision;
    cfg->chi_max = o->chi_max;
    cfg->tau = o->tau_trunc > 0 ? o->tau_trunc
                                : (o->precision == MSC_FP64 ? 1e-12
                                   : o->precision == MSC_FP32 ? 1e-5 : 1e-4);
    cfg->tau_rej = o->tau_rej > 0 ? o->tau_rej : 1e-6;
    cfg->tau_fail = o->tau_fail > 0 ? o->tau_fail : 1e-4;
    cfg->n_slots = o->n_slots;
    cfg->lds_width = o->lds_width == 64 ? 64 : 32;
    cfg->park_side = o->large_side == -1 ? 0 : o->large_side == 0 ? 256 : o->large_side;
    cfg->graphs = o->use_graphs == 1;
    int wc = 0;
    if (o->wave_chi > 0)
        wc = o->wave_chi;
    else if (o->wave_chi == 0 && o->lds_width == 0 && c && c->calibrated &&
             c->noiseless.chi_peak <= kAutoWaveChi)
        wc = kAutoWaveChi;
    cfg->wave_chi = std::min(wc, cfg->chi_max);
    default_tiles(cfg->precision, cfg->tiles);
    if (o->autotune_cache) {
        int rc = read_tune_cache(o->autotune_cache, cfg->precision, cfg->tiles);
        if (rc) return rc;
    }
    return MSC_OK;
}

// Checks a caller's fault CSR on the device (channel range and order, Pauli
// codes, offsets) before any kernel relies on it; MSC_E_INVALID if not.
static int validate_csr(msc_ctx* ctx, const msc_circuit* c, int64_t n, const int64_t* off,
                        const int32_t* chan, const uint8_t* pauli) {
    void* dflag;
    int rc;
    if ((rc = ctx_buf(ctx, "csr_flag", sizeof(int), &dflag))) return rc;
    MSC_HIP(launch_validate_csr(c->n_channels, n, off, chan, pauli,
                                static_cast<const uint8_t*>(c->d_kind), static_cast<int*>(dflag),
                                ctx->stream));
    int bad = 0;
    MSC_HIP(hipMemcpyAsync(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    return bad ? csr_error(bad) : MSC_OK;
}

extern "C" int msc_simulate(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                            int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                            const uint8_t* pauli, const int64_t* shot_idx, int64_t n_sel,
                            msc_shot_result* out) {
    if (!ctx || !c || !opts || n_shots < 0 || !shot_off || (shot_idx && n_sel < 0))
        return set_error(MSC_E_INVALID, "null argument");
    const int64_t n = shot_idx ? n_sel : n_shots;
    if (n > 0 && !out) return set_error(MSC_E_INVALID, "null out");
    if (!c->calibrated) return set_error(MSC_E_STATE, "circuit not calibrated");
    RunCfg cfg;
    int rc = sim_cfg(opts, c, &cfg);
    if (rc) return rc;
    if (n == 0) return MSC_OK;
    MSC_HIP(hipSetDevice(ctx->device));
    // the library only uploads into circuits it owns; const is logical here
    if ((rc = upload(ctx, const_cast<msc_circuit*>(c)))) return rc;
    if ((rc = validate_csr(ctx, c, n_shots, shot_off, chan, pauli))) return rc;
    if (opts->prefix && (rc = ensure_prefix(ctx, const_cast<msc_circuit*>(c), cfg))) return rc;
    return run_shots(ctx, c, cfg, n, n_shots, shot_off, chan, pauli, shot_idx, out, 0, nullptr,
                     nullptr, "simulate", opts->prefix ? 2 : 0,
                     opts->prefix ? &c->prefix : nullptr);
}

// The screen of a device CSR on the context's stream into caller buffers and
// the tmp words (prescreen_tmp_words(n) of them: block counts, the survivor
// total, the CSR flag); waits for the stream, reads the total and the flag.
static int screen_into(msc_ctx* ctx, const msc_circuit* c, int64_t n_shots,
                       const int64_t* shot_off, const int32_t* chan, const uint8_t* pauli,
                       uint64_t* survive_bits, int64_t* survivor_idx, int64_t* tmp, int64_t nt,
                       int64_t* n_survivors) {
    int* flag = reinterpret_cast<int*>(tmp + (nt - 1));
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    MSC_HIP(launch_prescreen(c->words, c->n_channels, n_shots, shot_off, chan, pauli,
                             static_cast<const uint64_t*>(c->d_sig),
                             static_cast<const int32_t*>(c->d_sig_off),
                             static_cast<const uint8_t*>(c->d_kind), survive_bits, survivor_idx,
                             tmp, nt, flag, ctx->stream));
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    int64_t tail[2] = {0, 0};   // survivor total, flag word
    MSC_HIP(hipMemcpyAsync(tail, tmp + (nt - 2), sizeof(tail), hipMemcpyDeviceToHost,
                           ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms["prescreen"] = ms;
    const int bad = static_cast<int>(tail[1] & 0xffffffff);
    if (bad) return csr_error(bad);
    *n_survivors = tail[0];
    return MSC_OK;
}

extern "C" int msc_prescreen(msc_ctx* ctx, const msc_circuit* c, int64_t n_shots,
                             const int64_t* shot_off, const int32_t* chan, const uint8_t* pauli,
                             uint64_t* survive_bits, int64_t* survivor_idx,
                             int64_t* n_survivors) {
    if (!ctx || !c || n_shots < 0 || !shot_off || !survive_bits || !n_survivors)
        return set_error(MSC_E_INVALID, "null argument");
    if (c->words > 8) return set_error(MSC_E_INVALID, "more than 512 decided measurements");
    *n_survivors = 0;
    if (n_shots == 0) return MSC_OK;
    MSC_HIP(hipSetDevice(ctx->device));
    int rc = upload(ctx, const_cast<msc_circuit*>(c));
    if (rc) return rc;
    const int64_t nt = prescreen_tmp_words(n_shots);
    void* tmp;
    if ((rc = ctx_buf(ctx, "screen_tmp", nt * sizeof(int64_t), &tmp))) return rc;
    return screen_into(ctx, c, n_shots, shot_off, chan, pauli, survive_bits, survivor_idx,
                       static_cast<int64_t*>(tmp), nt, n_survivors);
}

// msc_prescreen without device allocations: the block counts and the flag
// live in the library's fixed per-device scratch (prescreen.hip), so calls on
// one GPU share it (overlapping calls race) and each call starts by
// overwriting what it needs (the flag is cleared by a kernel, every block
// count is written before the scan reads it).
extern "C" int msc_prescreen_noalloc(msc_ctx* ctx, const msc_circuit* c, int64_t n_shots,
                                     const int64_t* shot_off, const int32_t* chan,
                                     const uint8_t* pauli, uint64_t* survive_bits,
                                     int64_t* survivor_idx, int64_t* n_survivors) {
    if (!ctx || !c || n_shots < 0 || !shot_off || !survive_bits || !n_survivors)
        return set_error(MSC_E_INVALID, "null argument");
    if (n_shots > kNoAllocShots)
        return set_error(MSC_E_INVALID, "msc_prescreen_noalloc takes at most 2^26 shots per call");
    if (c->words > 8) return set_error(MSC_E_INVALID, "more than 512 decided measurements");
    *n_survivors = 0;
    if (n_shots == 0) return MSC_OK;
    if (c->dev != ctx->device || !c->d_sig || !c->d_kind)
        return set_error(MSC_E_STATE, "the circuit's tables are not on this device yet "
                                      "(msc_circuit_calibrate or msc_prescreen uploads them)");
    MSC_HIP(hipSetDevice(ctx->device));
    int64_t* fixed = nullptr;
    MSC_HIP(prescreen_noalloc_scratch(ctx->device, &fixed));
    return screen_into(ctx, c, n_shots, shot_off, chan, pauli, survive_bits, survivor_idx,
                       fixed, prescreen_tmp_words(n_shots), n_survivors);
}

// The Bin(M, p) cumulative table on the device, uploaded when (M, p) changes.
static int device_cdf(msc_ctx* ctx, int64_t M, double p, void** out, int32_t* len) {
    int rc;
    if (ctx->cdf_m != M || !(ctx->cdf_p == p)) {
        std::vector<double> cdf = binomial_cdf(M, p);
        void* d;
        if ((rc = ctx_buf(ctx, "cdf", cdf.size() * sizeof(double), &d))) return rc;
        MSC_HIP(hipMemcpyAsync(d, cdf.data(), cdf.size() * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
        MSC_HIP(hipStreamSynchronize(ctx->stream));
        ctx->cdf_m = M;
        ctx->cdf_p = p;
        ctx->cdf_len = static_cast<int32_t>(cdf.size());
    }
    if ((rc = ctx_buf(ctx, "cdf", ctx->cdf_len * sizeof(double), out))) return rc;
    *len = ctx->cdf_len;
    return MSC_OK;
}

extern "C" int msc_sample_faults_device(msc_ctx* ctx, const msc_circuit* c, uint64_t seed,
                                        uint64_t first_shot, int64_t n_shots,
                                        const int32_t* weights, double p, int64_t* shot_off,
                                        int32_t* chan, uint8_t* pauli, int64_t nnz_cap,
                                        int64_t* nnz_out) {
    if (!ctx || !c || n_shots < 0 || !shot_off || !nnz_out || nnz_cap < 0)
        return set_error(MSC_E_INVALID, "null argument");
    if ((!chan || !pauli) && nnz_cap > 0) return set_error(MSC_E_INVALID, "null chan/pauli");
    if (!weights && !(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
    *nnz_out = 0;
    MSC_HIP(hipSetDevice(ctx->device));
    int rc = upload(ctx, const_cast<msc_circuit*>(c));
    if (rc) return rc;
    if (n_shots == 0) {
        const int64_t zero = 0;
        MSC_HIP(hipMemcpy(shot_off, &zero, sizeof(zero), hipMemcpyHostToDevice));
        return MSC_OK;
    }
    void* dcdf = nullptr;
    int32_t ncdf = 0;
    if (!weights && (rc = device_cdf(ctx, c->n_channels, p, &dcdf, &ncdf))) return rc;
    const int64_t nt = sampler_tmp_words(n_shots);
    void* tmp;
    if ((rc = ctx_buf(ctx, "sample_tmp", nt * sizeof(int64_t), &tmp))) return rc;
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    MSC_HIP(launch_sampler(n_shots, seed, first_shot, weights, static_cast<const double*>(dcdf),
                           ncdf, c->n_channels,
                           static_cast<const uint8_t*>(c->d_kind), nnz_cap, shot_off, chan, pauli,
                           static_cast<int64_t*>(tmp), nt, ctx->stream));
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    int64_t total = 0;
    MSC_HIP(hipMemcpyAsync(&total, static_cast<int64_t*>(tmp) + (nt - 1), sizeof(int64_t),
                           hipMemcpyDeviceToHost, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms["sample"] = ms;
    *nnz_out = total;
    if (total > nnz_cap) return set_error(MSC_E_CAPACITY, "nnz_cap too small");
    return MSC_OK;
}

extern "C" int msc_run_batch(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                             uint64_t seed, uint64_t first_shot, int64_t n_shots, double p,
                             int32_t n_bins, double* bins, msc_batch_stats* stats,
                             msc_shot_result* out, double* surv_bins) {
    if (!ctx || !c || !opts || !bins || n_shots < 0) return set_error(MSC_E_INVALID, "null argument");
    if (n_bins < 1 || n_bins > kMaxBins) return set_error(MSC_E_INVALID, "n_bins must be in [1, 1024]");
    if (!(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
    if (!c->calibrated) return set_error(MSC_E_STATE, "circuit not calibrated");
    RunCfg cfg;
    int rc = sim_cfg(opts, c, &cfg);
    if (rc) return rc;
    if (c->words > 8) return set_error(MSC_E_INVALID, "more than 512 decided measurements");
    MSC_HIP(hipSetDevice(ctx->device));
    if ((rc = upload(ctx, const_cast<msc_circuit*>(c)))) return rc;
    if (opts->prefix && (rc = ensure_prefix(ctx, const_cast<msc_circuit*>(c), cfg))) return rc;
    // host-mapped block for the reduction: bins, then the totals
    const bool space_time = surv_bins != nullptr;
    const int n_seg = space_time ? static_cast<int>(c->segs.size()) : 0;
    const size_t hbytes = (kBinRows * static_cast<size_t>(n_bins) +
                           static_cast<size_t>(n_bins) * n_seg) * sizeof(double) +
                          sizeof(BatchTotals);
    if (ctx->hmap_bytes < hbytes) {
        if (ctx->hmap) (void)hipHostFree(ctx->hmap);
        ctx->hmap = nullptr;
        ctx->hmap_bytes = 0;
        MSC_HIP(hipHostMalloc(&ctx->hmap, hbytes, hipHostMallocMapped | hipHostMallocCoherent));
        MSC_HIP(hipHostGetDevicePointer(&ctx->hmap_dev, ctx->hmap, 0));
        ctx->hmap_bytes = hbytes;
    }
    void* dcdf;
    int32_t ncdf;
    if ((rc = device_cdf(ctx, c->n_channels, p, &dcdf, &ncdf))) return rc;
    // every shot draws at most the table's largest weight (and at most M)
    const int64_t wmax = std::min<int64_t>(c->n_channels, std::max<int32_t>(0, ncdf - 1));
    const int64_t cap = std::max<int64_t>(1, n_shots * wmax);
    if (cap > (int64_t(1) << 28)) return set_error(MSC_E_CAPACITY, "fault buffer above 2^28 entries");
    const int64_t nts = sampler_tmp_words(n_shots), ntp = prescreen_tmp_words(n_shots);
    void *doff, *dchan, *dpa, *dbits, *didx, *dres, *dts, *dtp;
    if ((rc = ctx_buf(ctx, "b_off", (n_shots + 1) * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "b_chan", cap * sizeof(int32_t), &dchan))) return rc;
    if ((rc = ctx_buf(ctx, "b_pauli", cap, &dpa))) return rc;
    if ((rc = ctx_buf(ctx, "b_bits", ((n_shots + 63) / 64 + 1) * sizeof(uint64_t), &dbits))) return rc;
    if ((rc = ctx_buf(ctx, "b_idx", std::max<int64_t>(1, n_shots) * sizeof(int64_t), &didx))) return rc;
    if ((rc = ctx_buf(ctx, "b_res", std::max<int64_t>(1, n_shots) * sizeof(msc_shot_result), &dres))) return rc;
    if ((rc = ctx_buf(ctx, "b_tmp_s", nts * sizeof(int64_t), &dts))) return rc;
    if ((rc = ctx_buf(ctx, "b_tmp_p", std::max<int64_t>(3, ntp) * sizeof(int64_t), &dtp))) return rc;
    void* dsurv = nullptr;
    if (space_time &&
        (rc = ctx_buf(ctx, "b_surv", std::max<int64_t>(1, n_shots * n_seg) * sizeof(double), &dsurv)))
        return rc;
    int64_t* offp = static_cast<int64_t*>(doff);
    int64_t* idxp = static_cast<int64_t*>(didx);
    int64_t* nsurv = static_cast<int64_t*>(dtp) + (ntp - 2);   // the screen's total
    // the CSR check word (this batch's faults come from the library's own
    // sampler, so it is never set)
    int* csr_flag = reinterpret_cast<int*>(static_cast<int64_t*>(dtp) + (ntp - 1));
    int64_t* nnz = static_cast<int64_t*>(dts) + (nts - 1);     // the sampler's total
    double* hbins = static_cast<double*>(ctx->hmap_dev);
    BatchTotals* htot = reinterpret_cast<BatchTotals*>(hbins + kBinRows * static_cast<size_t>(n_bins));
    double* hsurv = reinterpret_cast<double*>(htot + 1);
    msc_shot_result* res = static_cast<msc_shot_result*>(dres);
    if (n_shots == 0) {
        for (int32_t b = 0; b < kBinRows * n_bins; ++b) bins[b] = 0.0;
        for (int32_t b = 0; b < n_bins * n_seg; ++b) surv_bins[b] = 0.0;
        if (stats) *stats = msc_batch_stats{};
        return MSC_OK;
    }
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    MSC_HIP(launch_sampler(n_shots, seed, first_shot, nullptr, static_cast<const double*>(dcdf),
                           ncdf, c->n_channels, static_cast<const uint8_t*>(c->d_kind), cap, offp,
                           static_cast<int32_t*>(dchan), static_cast<uint8_t*>(dpa),
                           static_cast<int64_t*>(dts), nts, ctx->stream));
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    if (space_time) {
        // every shot runs to its first rejecting measurement
        MSC_HIP(launch_identity(n_shots, idxp, nsurv, ctx->stream));
    } else {
        MSC_HIP(launch_prescreen(c->words, c->n_channels, n_shots, offp,
                                 static_cast<int32_t*>(dchan), static_cast<uint8_t*>(dpa),
                                 static_cast<const uint64_t*>(c->d_sig),
                             static_cast<const int32_t*>(c->d_sig_off),
                                 static_cast<const uint8_t*>(c->d_kind),
                                 static_cast<uint64_t*>(dbits), idxp, static_cast<int64_t*>(dtp),
                                 ntp, csr_flag, ctx->stream));
    }
    MSC_HIP(hipEventRecord(ctx->ev2, ctx->stream));
    rc = enqueue_shots(ctx, c, cfg, n_shots, n_shots, offp, static_cast<int32_t*>(dchan),
                       static_cast<uint8_t*>(dpa), idxp, res, 0, nullptr, nullptr,
                       opts->prefix ? 2 : 0, opts->prefix ? &c->prefix : nullptr, nsurv,
                       static_cast<double*>(dsurv), nullptr);
    if (rc) return rc;
    MSC_HIP(hipEventRecord(ctx->ev3, ctx->stream));
    void* dred;
    if ((rc = ctx_buf(ctx, "b_reduce", batch_reduce_tmp_bytes(n_shots, n_bins, n_seg), &dred))) return rc;
    MSC_HIP(launch_batch_reduce(n_shots, seed, first_shot, offp, idxp, nsurv, res, n_bins, nnz,
                                hbins, htot, static_cast<const double*>(dsurv), n_seg, hsurv,
                                dred, ctx->stream));
    if (out) MSC_HIP(launch_scatter_results(n_shots, nsurv, idxp, res, out, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    const double* hb = static_cast<const double*>(ctx->hmap);
    for (int32_t b = 0; b < kBinRows * n_bins; ++b) bins[b] = hb[b];
    const BatchTotals* ht = reinterpret_cast<const BatchTotals*>(hb + kBinRows * static_cast<size_t>(n_bins));
    const double* hs = reinterpret_cast<const double*>(ht + 1);
    for (int32_t b = 0; b < n_bins * n_seg; ++b) surv_bins[b] = hs[b];
    float t01 = 0.f, t12 = 0.f, t23 = 0.f;
    MSC_HIP(hipEventElapsedTime(&t01, ctx->ev0, ctx->ev1));
    MSC_HIP(hipEventElapsedTime(&t12, ctx->ev1, ctx->ev2));
    MSC_HIP(hipEventElapsedTime(&t23, ctx->ev2, ctx->ev3));
    ctx->last_ms["sample"] = t01;
    ctx->last_ms["prescreen"] = t12;
    ctx->last_ms["simulate"] = t23;
    ctx->lx_stats.total_ms = t23;
    if (stats) {
        stats->n_shots = n_shots;
        stats->nnz = ht->nnz;
        stats->n_survivors = ht->n_survivors;
        stats->n_accepted = ht->n_accepted;
        stats->n2q = ht->n2q;
        stats->sweeps = ht->sweeps;
        stats->flops = ht->flops;
        stats->chi_peak = ht->chi_peak;
        stats->status_or = ht->status_or;
        stats->ms_sample = t01;
        stats->ms_screen = t12;
        stats->ms_simulate = t23;
    }
    return MSC_OK;
}

// CAMPS op stream, channel qubits, layout and candidate tables on the device
static int camps_upload(msc_ctx* ctx, msc_circuit* c) {
    int rc = upload(ctx, c);
    if (rc) return rc;
    if (c->d_camps_ops) return MSC_OK;
    camps_compile(c);
    std::vector<double> dmat;
    std::vector<uint8_t> dtab;
    camps_candidates(dmat, dtab);
    if (static_cast<int>(dtab.size()) != 16 * kCampsCand)
        return set_error(MSC_E_INVALID, "candidate table size");
    std::vector<int32_t> site_of(c->n);
    for (int s = 0; s < c->n; ++s) site_of[c->order[s]] = s;
    auto put = [&](void** dst, const void* src, size_t bytes) -> int {
        MSC_HIP(hipMalloc(dst, std::max<size_t>(bytes, 64)));
        if (bytes) MSC_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return MSC_OK;
    };
    if ((rc = put(&c->d_camps_ops, c->camps_ops.data(), c->camps_ops.size() * sizeof(DevOp)))) return rc;
    if ((rc = put(&c->d_chan_q, c->chan_q.data(), c->chan_q.size() * sizeof(int32_t)))) return rc;
    if ((rc = put(&c->d_site_of, site_of.data(), site_of.size() * sizeof(int32_t)))) return rc;
    if ((rc = put(&c->d_dmat, dmat.data(), dmat.size() * sizeof(double)))) return rc;
    if ((rc = put(&c->d_dtab, dtab.data(), dtab.size()))) return rc;
    return MSC_OK;
}

static int run_camps(msc_ctx* ctx, msc_circuit* c, int chi_cap, double tau, double tau_rej,
                     double tau_fail, int n_slots, int64_t n, int64_t n_csr,
                     const int64_t* shot_off, const int32_t* chan, const uint8_t* pauli,
                     const int64_t* shot_idx, msc_shot_result* out, int ck_mode,
                     CampsPrefix* pk, const char* timer);
static int camps_rerun(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts, int64_t n,
                       int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                       const uint8_t* pauli, const int64_t* shot_idx, msc_shot_result* out);

// Checkpoints of the noiseless CAMPS run: before the fault op of every
// ck_k-th channel (at most 256 of them) and before the read-out, densely
// while they fit in kPrefixBytes.  A shot whose first fault is on channel
// ch forks from checkpoint ch / ck_k: the ops it skips are exactly the
// fault-free ops it would have run, in the same kernel, so its result does
// not change.
static int ensure_camps_prefix(msc_ctx* ctx, msc_circuit* c, int chi_cap, double tau,
                               double tau_rej, double tau_fail) {
    CampsPrefix& pk = c->camps_prefix;
    if (pk.valid && pk.dev == ctx->device && pk.chi_cap == chi_cap && pk.tau == tau &&
        pk.tau_rej == tau_rej)
        return MSC_OK;
    free_camps_prefix(pk);
    pk.dev = ctx->device;
    const int M = c->n_channels;
    std::vector<int32_t> chan_op(M, -1);
    for (size_t i = 0; i < c->camps_ops.size(); ++i)
        if (c->camps_ops[i].kind == CO_FAULT) chan_op[c->camps_ops[i].a] = static_cast<int32_t>(i);
    pk.ck_k = std::max(1, (M + 255) / 256);
    const int n_reg = (M + pk.ck_k - 1) / pk.ck_k;
    pk.n_ck = n_reg + 1;
    std::vector<int32_t> ck_op(pk.n_ck);
    for (int j = 0; j < n_reg; ++j) ck_op[j] = chan_op[static_cast<size_t>(j) * pk.ck_k];
    ck_op[n_reg] = static_cast<int32_t>(c->camps_ops.size()) - 1;   // CO_FINAL
    for (int j = 0; j + 1 < pk.n_ck; ++j)
        if (!(ck_op[j] >= 0 && ck_op[j] < ck_op[j + 1]))
            return set_error(MSC_E_INVALID, "CAMPS checkpoint ops not increasing");
    pk.cap = kPrefixBytes / static_cast<int64_t>(sizeof(double));
    auto dmalloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 64));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return set_error(MSC_E_OOM, std::string("CAMPS checkpoints: ") + hipGetErrorString(e));
        }
        return MSC_OK;
    };
    int rc;
    if ((rc = dmalloc(&pk.d_op, pk.n_ck * sizeof(int32_t)))) return rc;
    if ((rc = dmalloc(&pk.d_avail, sizeof(int32_t)))) return rc;
    if ((rc = dmalloc(&pk.d_off, pk.n_ck * sizeof(int64_t)))) return rc;
    if ((rc = dmalloc(&pk.d_hdr, pk.n_ck * sizeof(CampsCk)))) return rc;
    if ((rc = dmalloc(&pk.d_frame, static_cast<size_t>(pk.n_ck) * 8 * kMaxSites * sizeof(uint64_t)))) return rc;
    if ((rc = dmalloc(&pk.d_ph, static_cast<size_t>(pk.n_ck) * 2 * kMaxSites))) return rc;
    if ((rc = dmalloc(&pk.d_data, static_cast<size_t>(pk.cap) * sizeof(double)))) return rc;
    const int32_t zero = 0;
    MSC_HIP(hipMemcpy(pk.d_op, ck_op.data(), pk.n_ck * sizeof(int32_t), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(pk.d_avail, &zero, sizeof(zero), hipMemcpyHostToDevice));
    void *doff, *dchan, *dpa, *dout;
    if ((rc = ctx_buf(ctx, "cal_off", 2 * sizeof(int64_t), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "cal_chan", 64, &dchan))) return rc;
    if ((rc = ctx_buf(ctx, "cal_pa", 64, &dpa))) return rc;
    if ((rc = ctx_buf(ctx, "cal_out", sizeof(msc_shot_result), &dout))) return rc;
    int64_t zz[2] = {0, 0};
    MSC_HIP(hipMemcpy(doff, zz, sizeof(zz), hipMemcpyHostToDevice));
    rc = run_camps(ctx, c, chi_cap, tau, tau_rej, tau_fail, 1, 1, 1, static_cast<int64_t*>(doff),
                   static_cast<int32_t*>(dchan), static_cast<uint8_t*>(dpa), nullptr,
                   static_cast<msc_shot_result*>(dout), 1, &pk, "camps_prefix");
    if (rc) {
        free_camps_prefix(pk);
        return rc;
    }
    MSC_HIP(hipMemcpy(&pk.avail, pk.d_avail, sizeof(int32_t), hipMemcpyDeviceToHost));
    msc_shot_result res;
    MSC_HIP(hipMemcpy(&res, dout, sizeof(res), hipMemcpyDeviceToHost));
    if (!(res.status & MSC_SHOT_DONE)) {
        free_camps_prefix(pk);
        return set_error(MSC_E_NONDETERMINISTIC, "noiseless CAMPS run did not complete");
    }
    pk.chi_cap = chi_cap;
    pk.tau = tau;
    pk.tau_rej = tau_rej;
    pk.build_ms = static_cast<float>(ctx->last_ms["camps_prefix"]);
    pk.valid = true;
    return MSC_OK;
}

extern "C" int msc_simulate_camps(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts,
                                  int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                                  const uint8_t* pauli, const int64_t* shot_idx, int64_t n_sel,
                                  msc_shot_result* out) {
    if (!ctx || !c || !opts || n_shots < 0 || !shot_off || (shot_idx && n_sel < 0))
        return set_error(MSC_E_INVALID, "null argument");
    const int64_t n = shot_idx ? n_sel : n_shots;
    if (n > 0 && !out) return set_error(MSC_E_INVALID, "null out");
    if (!c->calibrated) return set_error(MSC_E_STATE, "circuit not calibrated");
    if (opts->precision != MSC_FP64) return set_error(MSC_E_INVALID, "CAMPS runs in MSC_FP64");
    if (opts->chi_max < 1 || opts->chi_max > kCampsCap)
        return set_error(MSC_E_INVALID, "CAMPS chi_max must be in [1, 32]");
    if (c->n > kMaxSites - 1) return set_error(MSC_E_INVALID, "CAMPS takes at most 127 qubits");
    if ((opts->prefix != 0 && opts->prefix != 1) || opts->wave_chi > 0 || opts->lds_width != 0)
        return set_error(MSC_E_INVALID, "CAMPS takes prefix 0 or 1, no lds_width or wave_chi option");
    if (n == 0) return MSC_OK;
    MSC_HIP(hipSetDevice(ctx->device));
    msc_circuit* cc = const_cast<msc_circuit*>(c);
    int rc = camps_upload(ctx, cc);
    if (rc) return rc;
    if ((rc = validate_csr(ctx, cc, n_shots, shot_off, chan, pauli))) return rc;
    const double tau = opts->tau_trunc > 0 ? opts->tau_trunc : 1e-12;
    const double tau_rej = opts->tau_rej > 0 ? opts->tau_rej : 1e-6;
    const double tau_fail = opts->tau_fail > 0 ? opts->tau_fail : 1e-4;
    if (opts->prefix && (rc = ensure_camps_prefix(ctx, cc, opts->chi_max, tau, tau_rej, tau_fail)))
        return rc;
    if ((rc = run_camps(ctx, cc, opts->chi_max, tau, tau_rej, tau_fail, opts->n_slots, n, n_shots,
                        shot_off, chan, pauli, shot_idx, out, opts->prefix ? 2 : 0,
                        opts->prefix ? &cc->camps_prefix : nullptr, "camps")))
        return rc;
    // shots whose residual outgrew the cap: run again by the FP64 MPS path
    try {
        return camps_rerun(ctx, c, opts, n, n_shots, shot_off, chan, pauli, shot_idx, out);
    } catch (const std::bad_alloc&) {
        return set_error(MSC_E_OOM, "host memory for the CAMPS rerun");
    }
}

// The records of a CAMPS launch whose residual outgrew the cap (status
// MSC_SHOT_CHI_CAP) replaced by the FP64 MPS path's, flagged
// MSC_SHOT_MPS_RERUN (out and shot_idx on the device).
static int camps_rerun(msc_ctx* ctx, const msc_circuit* c, const msc_sim_opts* opts, int64_t n,
                       int64_t n_shots, const int64_t* shot_off, const int32_t* chan,
                       const uint8_t* pauli, const int64_t* shot_idx, msc_shot_result* out) {
    int rc;
    std::vector<msc_shot_result> h(n);
    MSC_HIP(hipMemcpy(h.data(), out, n * sizeof(msc_shot_result), hipMemcpyDeviceToHost));
    std::vector<int64_t> pos, ids;
    std::vector<int64_t> hsel;
    if (shot_idx) {
        hsel.resize(n);
        MSC_HIP(hipMemcpy(hsel.data(), shot_idx, n * sizeof(int64_t), hipMemcpyDeviceToHost));
    }
    for (int64_t i = 0; i < n; ++i) {
        if (h[i].status & MSC_SHOT_CHI_CAP) {
            pos.push_back(i);
            ids.push_back(shot_idx ? hsel[i] : i);
        }
    }
    if (pos.empty()) return MSC_OK;
    const int64_t k = static_cast<int64_t>(pos.size());
    void *didx, *dres;
    if ((rc = ctx_buf(ctx, "camps_rerun_idx", k * sizeof(int64_t), &didx))) return rc;
    if ((rc = ctx_buf(ctx, "camps_rerun_out", k * sizeof(msc_shot_result), &dres))) return rc;
    MSC_HIP(hipMemcpy(didx, ids.data(), k * sizeof(int64_t), hipMemcpyHostToDevice));
    msc_sim_opts mo{};
    mo.precision = MSC_FP64;
    mo.chi_max = 256;
    mo.tau_trunc = opts->tau_trunc;
    mo.tau_rej = opts->tau_rej;
    mo.tau_fail = opts->tau_fail;
    mo.prefix = opts->prefix;
    mo.wave_chi = -1;
    if ((rc = msc_simulate(ctx, c, &mo, n_shots, shot_off, chan, pauli,
                           static_cast<const int64_t*>(didx), k,
                           static_cast<msc_shot_result*>(dres))))
        return rc;
    MSC_HIP(hipStreamSynchronize(ctx->stream));   // the rerun may still be in flight
    std::vector<msc_shot_result> r(k);
    MSC_HIP(hipMemcpy(r.data(), dres, k * sizeof(msc_shot_result), hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < k; ++j) {
        r[j].status |= MSC_SHOT_MPS_RERUN;
        h[pos[j]] = r[j];
    }
    MSC_HIP(hipMemcpy(out, h.data(), n * sizeof(msc_shot_result), hipMemcpyHostToDevice));
    return MSC_OK;
}

static int run_camps(msc_ctx* ctx, msc_circuit* c, int chi_cap, double tau, double tau_rej,
                     double tau_fail, int n_slots, int64_t n, int64_t n_csr,
                     const int64_t* shot_off, const int32_t* chan, const uint8_t* pauli,
                     const int64_t* shot_idx, msc_shot_result* out, int ck_mode,
                     CampsPrefix* pk, const char* timer) {
    int rc;
    if (n_slots <= 0) n_slots = ctx->n_cu * camps_blocks_per_cu();
    n_slots = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_slots, n)));
    void *arena, *scratch;
    if ((rc = ctx_buf(ctx, "camps_arena",
                      static_cast<size_t>(n_slots) * c->n * kCampsSiteDoubles * sizeof(double), &arena)))
        return rc;
    if ((rc = ctx_buf(ctx, "camps_scratch", static_cast<size_t>(n_slots) * kCampsScratch * sizeof(double),
                      &scratch)))
        return rc;
    CampsArgs a{};
    a.ops = static_cast<const DevOp*>(c->d_camps_ops);
    a.n_ops = static_cast<int32_t>(c->camps_ops.size());
    a.n = c->n;
    a.site_of = static_cast<const int32_t*>(c->d_site_of);
    a.chan_q = static_cast<const int32_t*>(c->d_chan_q);
    a.shot_off = shot_off;
    a.chan = chan;
    a.pauli = pauli;
    a.shot_idx = shot_idx;
    a.n_shots = n;
    a.n_csr = n_csr;
    a.expected = static_cast<const uint8_t*>(c->d_expected);
    a.out = out;
    a.arena = static_cast<double*>(arena);
    a.scratch = static_cast<double*>(scratch);
    a.dmat = static_cast<const double*>(c->d_dmat);
    a.dtab = static_cast<const uint8_t*>(c->d_dtab);
    a.chi_cap = chi_cap;
    a.tau = tau;
    a.tau_rej = tau_rej;
    a.tau_fail = tau_fail;
    a.ck_mode = pk ? ck_mode : 0;
    if (a.ck_mode) {
        a.n_ck = pk->n_ck;
        a.ck_k = pk->ck_k;
        a.ck_op = static_cast<const int32_t*>(pk->d_op);
        a.ck_avail = static_cast<int32_t*>(pk->d_avail);
        a.ck_off = static_cast<int64_t*>(pk->d_off);
        a.ck_hdr = static_cast<CampsCk*>(pk->d_hdr);
        a.ck_frame = static_cast<uint64_t*>(pk->d_frame);
        a.ck_ph = static_cast<uint8_t*>(pk->d_ph);
        a.ck_data = static_cast<double*>(pk->d_data);
        a.ck_cap = pk->cap;
    }
    const double r = 1.0 / std::sqrt(2.0);
    if (c->target == 'T') {
        a.rt[0] = r;
        a.rt[1] = r;
    } else {
        a.rt[0] = 0.0;
        a.rt[1] = 1.0;
    }
    a.rt[2] = 0.0;
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    MSC_HIP(launch_camps(a, n_slots, ctx->stream));
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms[timer] = ms;
    return MSC_OK;
}

extern "C" int msc_camps_candidates(double* dmat, uint8_t* dtab, int32_t* n_out) {
    if (!n_out) return set_error(MSC_E_INVALID, "null argument");
    std::vector<double> m;
    std::vector<uint8_t> t;
    camps_candidates(m, t);
    *n_out = static_cast<int32_t>(t.size() / 16);
    if (dmat) std::copy(m.begin(), m.end(), dmat);
    if (dtab) std::copy(t.begin(), t.end(), dtab);
    return MSC_OK;
}

// ---------------------------------------------------------------------------
// autotuning of the engine's tile shapes

// The raw text of each object in a JSON file's "entries" array with its
// "precision" field (the cache format msc_autotune writes).
static std::vector<std::pair<long, std::string>> cache_entries(const char* path) {
    std::vector<std::pair<long, std::string>> out;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    const size_t at = text.find("\"entries\"");
    if (at == std::string::npos) return out;
    size_t pos = text.find('[', at);
    const size_t end = pos == std::string::npos ? pos : text.find(']', pos);
    while (pos != std::string::npos && end != std::string::npos) {
        const size_t o = text.find('{', pos);
        if (o == std::string::npos || o > end) break;
        const size_t cl = text.find('}', o);
        if (cl == std::string::npos || cl > end) break;
        const std::string obj = text.substr(o, cl - o + 1);
        long pr = -1;
        const size_t kp = obj.find("\"precision\"");
        if (kp != std::string::npos) {
            const size_t colon = obj.find(':', kp);
            if (colon != std::string::npos) pr = std::strtol(obj.c_str() + colon + 1, nullptr, 10);
        }
        out.emplace_back(pr, obj);
        pos = cl + 1;
    }
    return out;
}

extern "C" int msc_autotune(msc_ctx* ctx, int32_t precision, int32_t reps, const char* cache_path,
                            msc_tune_entry* out) {
    if (!ctx) return set_error(MSC_E_INVALID, "null context");
    if (precision != MSC_FP32 && precision != MSC_FP64 && precision != MSC_BF16X3)
        return set_error(MSC_E_INVALID, "unknown precision");
    if (reps < 1 || reps > 1000) return set_error(MSC_E_INVALID, "reps must be in [1, 1000]");
    MSC_HIP(hipSetDevice(ctx->device));
    const size_t tsize = precision == MSC_FP64 ? sizeof(double) : sizeof(float);
    LxTiles var[16];
    const int nvar = lx_tile_variants(precision, var, 16);
    const int sides[kLxBuckets] = {128, 256, 512, 1024};
    const int batches[kLxBuckets] = {256, 96, 24, 6};
    std::vector<double> g4(G4_COUNT * 32);
    for (int g = 0; g < G4_COUNT; ++g) gate4_matrix(g, &g4[g * 32]);
    msc_tune_entry res[kLxBuckets];
    const int grid = ctx->n_cu * 4;
    int rc;
    for (int bk = 0; bk < kLxBuckets; ++bk) {
        const int chi = sides[bk] / 2, N = batches[bk];
        const int64_t site = 2ll * chi * chi;          // elements of one plane
        const int64_t stride = 4 * site;               // two sites, two planes
        std::vector<ShotState> st(N);
        std::vector<int32_t> list(N);
        for (int i = 0; i < N; ++i) {
            st[i] = ShotState{};
            st[i].status = kSlotParked;
            st[i].k = 0;
            st[i].dir = i & 1;
            st[i].gate_id = G4_CX01;
            st[i].chi[0] = st[i].chi[1] = st[i].chi[2] = chi;
            list[i] = i;
        }
        // random tensors of unit scale from a fixed 64-bit LCG
        std::vector<double> hd(static_cast<size_t>(N) * stride);
        uint64_t x = 0x5EED0107ull;
        for (double& v : hd) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            v = static_cast<double>(static_cast<int64_t>(x >> 11) - (int64_t(1) << 52)) /
                static_cast<double>(int64_t(1) << 52) / chi;
        }
        std::vector<float> hf;
        if (precision != MSC_FP64) hf.assign(hd.begin(), hd.end());
        const int64_t S = 2ll * chi;
        void *dstate, *dcount, *dlist, *dplan, *darena, *dtheta, *dgram, *doff, *dhalf, *dg4, *dfl;
        if ((rc = ctx_buf(ctx, "tune_state", N * sizeof(ShotState), &dstate))) return rc;
        if ((rc = ctx_buf(ctx, "tune_count", sizeof(int32_t), &dcount))) return rc;
        if ((rc = ctx_buf(ctx, "tune_list", N * sizeof(int32_t), &dlist))) return rc;
        if ((rc = ctx_buf(ctx, "tune_plan", sizeof(LxPlan), &dplan))) return rc;
        if ((rc = ctx_buf(ctx, "tune_arena", N * stride * tsize, &darena))) return rc;
        if ((rc = ctx_buf(ctx, "tune_theta", N * 2 * S * S * tsize, &dtheta))) return rc;
        if ((rc = ctx_buf(ctx, "tune_gram", N * lx_gram_doubles(S) * sizeof(double), &dgram))) return rc;
        if ((rc = ctx_buf(ctx, "tune_off", 2 * sizeof(int64_t), &doff))) return rc;
        if ((rc = ctx_buf(ctx, "tune_half", 2 * sizeof(int64_t), &dhalf))) return rc;
        if ((rc = ctx_buf(ctx, "tune_g4", g4.size() * sizeof(double), &dg4))) return rc;
        if ((rc = ctx_buf(ctx, "tune_flops", 6 * sizeof(double), &dfl))) return rc;
        const int64_t off[2] = {0, 2 * site}, half[2] = {site, site};
        const int32_t count = N;
        MSC_HIP(hipMemcpy(dstate, st.data(), N * sizeof(ShotState), hipMemcpyHostToDevice));
        MSC_HIP(hipMemcpy(dcount, &count, sizeof(count), hipMemcpyHostToDevice));
        MSC_HIP(hipMemcpy(dlist, list.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
        if (precision == MSC_FP64)
            MSC_HIP(hipMemcpy(darena, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice));
        else
            MSC_HIP(hipMemcpy(darena, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice));
        MSC_HIP(hipMemcpy(doff, off, sizeof(off), hipMemcpyHostToDevice));
        MSC_HIP(hipMemcpy(dhalf, half, sizeof(half), hipMemcpyHostToDevice));
        MSC_HIP(hipMemcpy(dg4, g4.data(), g4.size() * sizeof(double), hipMemcpyHostToDevice));
        LxArgs la{};
        la.state = static_cast<const ShotState*>(dstate);
        la.park_count = static_cast<const int32_t*>(dcount);
        la.park_list = static_cast<const int32_t*>(dlist);
        la.plan = static_cast<LxPlan*>(dplan);
        la.arena = darena;
        la.slot_stride = stride;
        la.site_off = static_cast<const int64_t*>(doff);
        la.site_half = static_cast<const int64_t*>(dhalf);
        la.g4 = static_cast<const double*>(dg4);
        la.theta = dtheta;
        la.theta_stride = 2 * S * S;
        la.gram = static_cast<double*>(dgram);
        la.gram_stride = lx_gram_doubles(S);
        la.n_slots = N;
        la.flops = static_cast<double*>(dfl);
        la.counts = reinterpret_cast<unsigned long long*>(la.flops + 2);
        double best_c = 1e300, best_g = 1e300;
        LxTiles pick{0, 0, 0};
        for (int v = 0; v < nvar; ++v) {
            LxTiles t4[kLxBuckets];
            for (int q = 0; q < kLxBuckets; ++q) t4[q] = var[v];
            MSC_HIP(launch_lx_plan(la, t4, ctx->stream));
            double tc = 1e300, tg = 1e300;
            for (int r = 0; r <= reps; ++r) {   // the first launch warms up
                float ms = 0.f;
                MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
                MSC_HIP(launch_lx_contract(precision, la, bk, var[v], grid, ctx->stream));
                MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
                MSC_HIP(launch_lx_gram(precision, la, bk, var[v], grid, ctx->stream));
                MSC_HIP(hipEventRecord(ctx->ev2, ctx->stream));
                MSC_HIP(hipStreamSynchronize(ctx->stream));
                if (r == 0) continue;
                MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                tc = std::min(tc, static_cast<double>(ms));
                MSC_HIP(hipEventElapsedTime(&ms, ctx->ev1, ctx->ev2));
                tg = std::min(tg, static_cast<double>(ms));
            }
            if (tc < best_c) {
                best_c = tc;
                pick.cm_rows = var[v].cm_rows;
                pick.cm_b = var[v].cm_b;
            }
            if (tg < best_g) {
                best_g = tg;
                pick.gram = var[v].gram;
            }
        }
        res[bk] = msc_tune_entry{bk, sides[bk], N, pick.cm_rows, pick.cm_b, pick.gram,
                                 best_c * 1e3, best_g * 1e3};
    }
    if (out) std::copy(res, res + kLxBuckets, out);
    if (cache_path) {
        std::vector<std::pair<long, std::string>> keep;
        for (auto& e : cache_entries(cache_path))
            if (e.first != precision) keep.push_back(e);
        hipDeviceProp_t prop;
        MSC_HIP(hipGetDeviceProperties(&prop, ctx->device));
        FILE* f = std::fopen(cache_path, "wb");
        if (!f) return set_error(MSC_E_INVALID, std::string("cannot write ") + cache_path);
        std::fprintf(f, "{\"device\": \"%s\", \"entries\": [\n", prop.gcnArchName);
        bool first = true;
        for (auto& e : keep) {
            std::fprintf(f, "%s  %s", first ? "" : ",\n", e.second.c_str());
            first = false;
        }
        for (const msc_tune_entry& e : res) {
            std::fprintf(f,
                         "%s  {\"precision\": %d, \"bucket\": %d, \"side\": %d, \"batch\": %d, "
                         "\"rows\": %d, \"b\": %d, \"gram\": %d, \"contract_us\": %.3f, "
                         "\"gram_us\": %.3f}",
                         first ? "" : ",\n", precision, e.bucket, e.side, e.batch, e.rows, e.b,
                         e.gram, e.contract_us, e.gram_us);
            first = false;
        }
        std::fprintf(f, "\n]}\n");
        std::fclose(f);
    }
    return MSC_OK;
}

static int engine_update(msc_ctx* ctx, int32_t precision, int32_t chi_l, int32_t chi_m,
                         int32_t chi_r, int32_t batch, int32_t dir, int32_t gate, int32_t chi_max,
                         double tau, const double* A, const double* B, double* A_out,
                         double* B_out, int32_t* r_out) {
    if (!ctx || !A || !B || !A_out || !B_out || !r_out) return set_error(MSC_E_INVALID, "null argument");
    if (precision != MSC_FP32 && precision != MSC_FP64 && precision != MSC_BF16X3)
        return set_error(MSC_E_INVALID, "unknown precision");
    if (chi_l < 1 || chi_m < 1 || chi_r < 1 || chi_l > kMaxChiKernel || chi_m > kMaxChiKernel ||
        chi_r > kMaxChiKernel || chi_max < 1 || chi_max > kMaxChiKernel)
        return set_error(MSC_E_INVALID, "bonds and chi_max must be in [1, " +
                                            std::to_string(kMaxChiKernel) + "]");
    if (batch < 1 || batch > kLxMaxParked)
        return set_error(MSC_E_INVALID, "batch must be in [1, " + std::to_string(kLxMaxParked) + "]");
    if ((dir != 0 && dir != 1) || gate < 0 || gate >= G4_COUNT || !(tau > 0.0 && tau < 1.0))
        return set_error(MSC_E_INVALID, "dir must be 0 or 1, gate a 4x4 gate id, tau in (0, 1)");
    MSC_HIP(hipSetDevice(ctx->device));
    const size_t tsize = precision == MSC_FP64 ? sizeof(double) : sizeof(float);
    // the factor's vector arrays hold theta sides up to 2 cf
    const int cf = std::max(chi_max, std::max(chi_l, chi_r));
    const int rmax = std::min(chi_max, 2 * std::min(chi_l, chi_r));
    const int cb = std::max(chi_m, rmax);                       // capacity of the middle bond
    const int64_t pa = 2ll * chi_l * cb, pb = 2ll * cb * chi_r;  // plane capacities
    const int64_t stride = (2 * pa + 2 * pb + 15) / 16 * 16;
    const int64_t S = 2ll * cf;
    std::vector<ShotState> st(batch);
    std::vector<int32_t> list(batch);
    for (int i = 0; i < batch; ++i) {
        st[i] = ShotState{};
        st[i].status = kSlotParked;
        st[i].k = 0;
        st[i].dir = dir;
        st[i].gate_id = gate;
        st[i].chi[0] = chi_l;
        st[i].chi[1] = chi_m;
        st[i].chi[2] = chi_r;
        list[i] = i;
    }
    // inputs into the slots' layout, in the tensor type
    const int64_t na = 2ll * chi_l * chi_m, nb = 2ll * chi_m * chi_r;
    std::vector<double> hd(static_cast<size_t>(batch) * stride, 0.0);
    for (int i = 0; i < batch; ++i) {
        double* slot = hd.data() + static_cast<size_t>(i) * stride;
        const double* a = A + static_cast<size_t>(i) * 2 * na;
        const double* b = B + static_cast<size_t>(i) * 2 * nb;
        std::copy(a, a + na, slot);
        std::copy(a + na, a + 2 * na, slot + pa);
        std::copy(b, b + nb, slot + 2 * pa);
        std::copy(b + nb, b + 2 * nb, slot + 2 * pa + pb);
    }
    std::vector<double> g4(G4_COUNT * 32);
    for (int g = 0; g < G4_COUNT; ++g) gate4_matrix(g, &g4[g * 32]);
    const int32_t cap[3] = {chi_l, chi_max, chi_r};
    const int64_t off[2] = {0, 2 * pa}, half[2] = {pa, pb};
    const int32_t count = batch;
    int rc;
    void *dstate, *dcount, *dlist, *dplan, *darena, *dtheta, *dgram, *doff, *dhalf, *dg4, *dfl, *dcap;
    if ((rc = ctx_buf(ctx, "eu_state", batch * sizeof(ShotState), &dstate))) return rc;
    if ((rc = ctx_buf(ctx, "eu_count", sizeof(int32_t), &dcount))) return rc;
    if ((rc = ctx_buf(ctx, "eu_list", batch * sizeof(int32_t), &dlist))) return rc;
    if ((rc = ctx_buf(ctx, "eu_plan", sizeof(LxPlan), &dplan))) return rc;
    if ((rc = ctx_buf(ctx, "eu_arena", batch * stride * tsize, &darena))) return rc;
    if ((rc = ctx_buf(ctx, "eu_theta", batch * 2 * S * S * tsize, &dtheta))) return rc;
    if ((rc = ctx_buf(ctx, "eu_gram", batch * lx_gram_doubles(S) * sizeof(double), &dgram))) return rc;
    if ((rc = ctx_buf(ctx, "eu_off", sizeof(off), &doff))) return rc;
    if ((rc = ctx_buf(ctx, "eu_half", sizeof(half), &dhalf))) return rc;
    if ((rc = ctx_buf(ctx, "eu_g4", g4.size() * sizeof(double), &dg4))) return rc;
    if ((rc = ctx_buf(ctx, "eu_flops", 6 * sizeof(double), &dfl))) return rc;
    if ((rc = ctx_buf(ctx, "eu_cap", sizeof(cap), &dcap))) return rc;
    MSC_HIP(hipMemcpy(dstate, st.data(), batch * sizeof(ShotState), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(dcount, &count, sizeof(count), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(dlist, list.data(), batch * sizeof(int32_t), hipMemcpyHostToDevice));
    if (precision == MSC_FP64) {
        MSC_HIP(hipMemcpy(darena, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> hf(hd.begin(), hd.end());
        MSC_HIP(hipMemcpy(darena, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    MSC_HIP(hipMemcpy(doff, off, sizeof(off), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(dhalf, half, sizeof(half), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(dg4, g4.data(), g4.size() * sizeof(double), hipMemcpyHostToDevice));
    MSC_HIP(hipMemcpy(dcap, cap, sizeof(cap), hipMemcpyHostToDevice));
    LxArgs la{};
    la.state = static_cast<const ShotState*>(dstate);
    la.park_count = static_cast<const int32_t*>(dcount);
    la.park_list = static_cast<const int32_t*>(dlist);
    la.plan = static_cast<LxPlan*>(dplan);
    la.arena = darena;
    la.slot_stride = stride;
    la.site_off = static_cast<const int64_t*>(doff);
    la.site_half = static_cast<const int64_t*>(dhalf);
    la.g4 = static_cast<const double*>(dg4);
    la.theta = dtheta;
    la.theta_stride = 2 * S * S;
    la.gram = static_cast<double*>(dgram);
    la.gram_stride = lx_gram_doubles(S);
    la.n_slots = batch;
    la.flops = static_cast<double*>(dfl);
    la.counts = reinterpret_cast<unsigned long long*>(la.flops + 2);
    LxFactor fac{};
    fac.cap = static_cast<const int32_t*>(dcap);
    fac.chi_max = cf;
    fac.tau = tau;
    LxTiles tiles[kLxBuckets];
    default_tiles(precision, tiles);
    const int grid = ctx->n_cu * 4;
    hipStream_t s = ctx->stream;
    MSC_HIP(hipEventRecord(ctx->ev0, s));
    MSC_HIP(launch_lx_plan(la, tiles, s));
    for (int b = 0; b < kLxBuckets; ++b) MSC_HIP(launch_lx_contract(precision, la, b, tiles[b], grid, s));
    for (int b = 0; b < kLxBuckets; ++b) MSC_HIP(launch_lx_gram(precision, la, b, tiles[b], grid, s));
    MSC_HIP(launch_lx_factor(precision, la, fac, batch, s));
    MSC_HIP(hipEventRecord(ctx->ev1, s));
    MSC_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms["engine_update"] = ms;
    MSC_HIP(hipMemcpy(st.data(), dstate, batch * sizeof(ShotState), hipMemcpyDeviceToHost));
    if (precision == MSC_FP64) {
        MSC_HIP(hipMemcpy(hd.data(), darena, hd.size() * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> hf(hd.size());
        MSC_HIP(hipMemcpy(hf.data(), darena, hf.size() * sizeof(float), hipMemcpyDeviceToHost));
        std::copy(hf.begin(), hf.end(), hd.begin());
    }
    const int64_t oa = 2ll * chi_l * rmax, ob = 2ll * rmax * chi_r;   // output planes
    for (int i = 0; i < batch; ++i) {
        const int r = st[i].chi[1];
        if (r < 1 || r > rmax)
            return set_error(MSC_E_DEVICE, "engine update " + std::to_string(i) +
                                               " returned bond " + std::to_string(r));
        r_out[i] = r;
        const double* slot = hd.data() + static_cast<size_t>(i) * stride;
        double* ao = A_out + static_cast<size_t>(i) * 2 * oa;
        double* bo = B_out + static_cast<size_t>(i) * 2 * ob;
        std::fill(ao, ao + 2 * oa, 0.0);
        std::fill(bo, bo + 2 * ob, 0.0);
        const int64_t ua = 2ll * chi_l * r, ub = 2ll * r * chi_r;
        std::copy(slot, slot + ua, ao);
        std::copy(slot + pa, slot + pa + ua, ao + oa);
        std::copy(slot + 2 * pa, slot + 2 * pa + ub, bo);
        std::copy(slot + 2 * pa + pb, slot + 2 * pa + pb + ub, bo + ob);
    }
    return MSC_OK;
}

// (host staging of a large batch can exceed host memory: no C++ exception
// crosses the ABI)
extern "C" int msc_engine_update(msc_ctx* ctx, int32_t precision, int32_t chi_l,
                                 int32_t chi_m, int32_t chi_r, int32_t batch, int32_t dir,
                                 int32_t gate, int32_t chi_max, double tau, const double* A,
                                 const double* B, double* A_out, double* B_out, int32_t* r_out) {
    try {
        return engine_update(ctx, precision, chi_l, chi_m, chi_r, batch, dir, gate, chi_max, tau,
                             A, B, A_out, B_out, r_out);
    } catch (const std::bad_alloc&) {
        return set_error(MSC_E_OOM, "host memory for the engine update's staging");
    }
}

extern "C" int msc_twosite_contract(msc_ctx* ctx, int32_t precision, int32_t chi, int32_t batch,
                                    const float* A, const float* B, const float* gate, float* theta) {
    if (!ctx || !A || !B || !gate || !theta) return set_error(MSC_E_INVALID, "null argument");
    if (chi < 64 || chi > 1024 || chi % 64 != 0 || batch < 1 || batch > 65535)
        return set_error(MSC_E_INVALID, "chi must be a multiple of 64 in [64, 1024], batch in [1, 65535]");
    MSC_HIP(hipSetDevice(ctx->device));
    MSC_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    if (precision != MSC_FP32 && precision != MSC_BF16X3)
        return set_error(MSC_E_INVALID, "twosite precision must be MSC_FP32 or MSC_BF16X3");
    MSC_HIP(launch_twosite(precision, chi, batch, A, B, gate, theta, ctx->stream));
    MSC_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    MSC_HIP(hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    MSC_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->last_ms["twosite"] = ms;
    return MSC_OK;
}
