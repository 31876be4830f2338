// Circuit text parser and MPS op-stream compiler.
//
// Layout and routing follow Section 3.1: the MPS needs a linear order of the
// qubits, and a two-qubit gate between qubits that are not neighbours in
// that order has to touch every bond in between.  Here such gates are routed
// with SWAP updates: the qubit shared with the neighbouring gates walks next
// to its partner, the gate is applied, and the walker goes home lazily (only
// when another qubit needs to move), with back-to-back SWAPs on the same
// bond cancelled.  The orthogonality centre is scheduled at compile time: a
// two-site update requires the centre on one of its sites, a measurement or
// the final read-out requires it on the site itself, and each update leaves
// the centre on the side of the next op that needs it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>
#include <string>

#include "../msc_internal.h"

namespace msc {

void gate1_matrix(int g, double o[8]) {
    const double r = 1.0 / std::sqrt(2.0);
    for (int i = 0; i < 8; ++i) o[i] = 0.0;
    auto set = [&](int i, int j, double re, double im) {
        o[2 * (2 * i + j)] = re;
        o[2 * (2 * i + j) + 1] = im;
    };
    switch (g) {
        case G_H: set(0, 0, r, 0); set(0, 1, r, 0); set(1, 0, r, 0); set(1, 1, -r, 0); break;
        case G_S: set(0, 0, 1, 0); set(1, 1, 0, 1); break;
        case G_SDG: set(0, 0, 1, 0); set(1, 1, 0, -1); break;
        case G_T: set(0, 0, 1, 0); set(1, 1, r, r); break;
        case G_TDG: set(0, 0, 1, 0); set(1, 1, r, -r); break;
        case G_X: set(0, 1, 1, 0); set(1, 0, 1, 0); break;
        case G_Y: set(0, 1, 0, -1); set(1, 0, 0, 1); break;
        case G_Z: set(0, 0, 1, 0); set(1, 1, -1, 0); break;
        default: break;
    }
}

void gate4_matrix(int g, double o[32]) {
    for (int i = 0; i < 32; ++i) o[i] = 0.0;
    auto one = [&](int row, int col) { o[2 * (4 * row + col)] = 1.0; };
    switch (g) {
        case G4_I: for (int i = 0; i < 4; ++i) one(i, i); break;
        case G4_SWAP: one(0, 0); one(1, 2); one(2, 1); one(3, 3); break;
        case G4_CX01: one(0, 0); one(1, 1); one(2, 3); one(3, 2); break;   // control s_k
        case G4_CX10: one(0, 0); one(1, 3); one(2, 2); one(3, 1); break;   // control s_{k+1}
        case G4_CZ: one(0, 0); one(1, 1); one(2, 2); o[2 * 15] = -1.0; break;
        case G4_CS: one(0, 0); one(1, 1); one(2, 2); o[2 * 15 + 1] = 1.0; break;
        case G4_CSDG: one(0, 0); one(1, 1); one(2, 2); o[2 * 15 + 1] = -1.0; break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// parser

static bool parse_int(const std::string& s, int& out) {
    if (s.empty()) return false;
    char* end = nullptr;
    long v = std::strtol(s.c_str(), &end, 10);
    if (*end != '\0' || v < 0 || v > (1 << 20)) return false;
    out = static_cast<int>(v);
    return true;
}

int parse_circuit(const char* text, size_t len, msc_circuit* c) {
    std::string src(text, len);
    std::istringstream in(src);
    std::string line;
    int lineno = 0;
    bool have_n = false;
    std::vector<int> order;
    c->n_meas = 0;
    c->n_channels = 0;
    c->seg_ir.assign(1, 0);
    auto perr = [&](const std::string& msg) {
        return set_error(MSC_E_PARSE, "line " + std::to_string(lineno) + ": " + msg);
    };
    while (std::getline(in, line)) {
        ++lineno;
        auto hash = line.find('#');
        if (hash != std::string::npos) line.resize(hash);
        std::istringstream ls(line);
        std::vector<std::string> tok;
        std::string t;
        while (ls >> t) tok.push_back(t);
        if (tok.empty()) continue;
        std::string op = tok[0];
        for (auto& ch : op) ch = static_cast<char>(std::toupper(static_cast<unsigned char>(ch)));
        std::vector<int> args;
        if (op != "TARGET") {
            for (size_t i = 1; i < tok.size(); ++i) {
                int v;
                if (!parse_int(tok[i], v)) return perr("bad integer '" + tok[i] + "'");
                args.push_back(v);
            }
        }
        auto need = [&](size_t k) { return args.size() == k; };
        auto qok = [&](int q) { return have_n && q >= 0 && q < c->n; };
        if (op != "QUBITS" && !have_n) return perr("QUBITS must come first");
        if (op == "QUBITS") {
            if (have_n) return perr("QUBITS given twice");
            if (!need(1) || args[0] < 1 || args[0] > 1024) return perr("QUBITS needs 1..1024");
            c->n = args[0];
            have_n = true;
        } else if (op == "ORDER") {
            order = args;
        } else if (op == "SEED") {
            if (!need(1) || !qok(args[0])) return perr("bad SEED");
            c->seed = args[0];
        } else if (op == "TARGET") {
            if (tok.size() != 2 || (tok[1] != "T" && tok[1] != "S")) return perr("TARGET T|S");
            c->target = tok[1][0];
        } else if (op == "TICK") {
            continue;
        } else if (op == "SEGMENT") {
            if (!need(0)) return perr("SEGMENT takes no operand");
            if (c->seg_ir.back() != static_cast<int32_t>(c->ir.size()))
                c->seg_ir.push_back(static_cast<int32_t>(c->ir.size()));
        } else {
            IrOp o{};
            o.b = -1;
            o.c = -1;
            o.idx = -1;
            static const char* g1n[] = {"H", "S", "SDG", "T", "TDG", "X", "Y", "Z"};
            int g1 = -1;
            for (int i = 0; i < G1_COUNT; ++i)
                if (op == g1n[i]) g1 = i;
            if (g1 >= 0) {
                if (!need(1) || !qok(args[0])) return perr("bad 1q gate operand");
                o.kind = IR_G1;
                o.g = g1;
                o.a = args[0];
            } else if (op == "CX" || op == "CZ" || op == "CS" || op == "CSDG") {
                if (!need(2) || !qok(args[0]) || !qok(args[1]) || args[0] == args[1])
                    return perr("bad 2q gate operands");
                o.kind = IR_G2;
                o.g = op == "CX" ? G2_CX : op == "CZ" ? G2_CZ : op == "CS" ? G2_CS : G2_CSDG;
                o.a = args[0];
                o.b = args[1];
            } else if (op == "CCZ") {
                if (!need(3) || !qok(args[0]) || !qok(args[1]) || !qok(args[2]) ||
                    args[0] == args[1] || args[0] == args[2] || args[1] == args[2])
                    return perr("bad CCZ operands");
                o.kind = IR_G3;
                o.g = 0;
                o.a = args[0];
                o.b = args[1];
                o.c = args[2];
            } else if (op == "M") {
                if (!need(1) || !qok(args[0])) return perr("bad M operand");
                o.kind = IR_M;
                o.a = args[0];
                o.idx = c->n_meas++;
            } else if (op == "R") {
                if (!need(1) || !qok(args[0])) return perr("bad R operand");
                o.kind = IR_R;
                o.a = args[0];
            } else if (op == "DEP1" || op == "XERR") {
                if (!need(1) || !qok(args[0])) return perr("bad channel operand");
                o.kind = IR_CH;
                o.g = op == "DEP1" ? CH_DEP1 : CH_XERR;
                o.a = args[0];
                o.idx = c->n_channels++;
            } else if (op == "DEP2") {
                if (!need(2) || !qok(args[0]) || !qok(args[1]) || args[0] == args[1])
                    return perr("bad DEP2 operands");
                o.kind = IR_CH;
                o.g = CH_DEP2;
                o.a = args[0];
                o.b = args[1];
                o.idx = c->n_channels++;
            } else if (op == "DEP3") {
                if (!need(3) || !qok(args[0]) || !qok(args[1]) || !qok(args[2]) ||
                    args[0] == args[1] || args[0] == args[2] || args[1] == args[2])
                    return perr("bad DEP3 operands");
                o.kind = IR_CH;
                o.g = CH_DEP3;
                o.a = args[0];
                o.b = args[1];
                o.c = args[2];
                o.idx = c->n_channels++;
            } else {
                return perr("unknown op '" + tok[0] + "'");
            }
            c->ir.push_back(o);
        }
    }
    if (!have_n) return set_error(MSC_E_PARSE, "missing QUBITS");
    if (!order.empty()) {
        if (static_cast<int>(order.size()) != c->n) return set_error(MSC_E_PARSE, "ORDER length");
        c->order = order;
    }
    // R legality: first op on the qubit, or the last op on it was M
    std::vector<int> last(c->n, -1);   // -1 none, else IrKind
    for (const auto& o : c->ir) {
        if (o.kind == IR_R && !(last[o.a] == -1 || last[o.a] == IR_M))
            return set_error(MSC_E_PARSE, "R on qubit " + std::to_string(o.a) +
                                              " not at start or right after M");
        if (o.kind == IR_CH) continue;   // noise does not change legality
        last[o.a] = o.kind;
        if (o.b >= 0) last[o.b] = o.kind;
        if (o.c >= 0) last[o.c] = o.kind;
    }
    for (const auto& o : c->ir) {
        if (o.kind != IR_CH) continue;
        c->chan_kind.push_back(o.g);
    }
    c->expected.assign(c->n_meas, 0);
    segment_table(c);
    return MSC_OK;
}

// Segments for the space-time accounting (Appendix "Space-time overhead"):
// a segment's volume is the qubits its gates, measurements and resets use
// times its depth, the layer count of an as-soon-as-possible schedule of
// those ops (noise channels are not layers); a shot reaches the segment
// with the product of its outcome probabilities over the first_meas
// measurements before it.
void segment_table(msc_circuit* c) {
    c->segs.clear();
    const int ns = static_cast<int>(c->seg_ir.size());
    int meas = 0;
    for (int s = 0; s < ns; ++s) {
        const size_t lo = static_cast<size_t>(c->seg_ir[s]);
        const size_t hi = s + 1 < ns ? static_cast<size_t>(c->seg_ir[s + 1]) : c->ir.size();
        msc_segment g{};
        g.first_meas = meas;
        std::vector<int> layer(c->n, 0);
        std::vector<char> used(c->n, 0);
        for (size_t i = lo; i < hi; ++i) {
            const IrOp& o = c->ir[i];
            if (o.kind == IR_CH) {
                g.noisy = 1;
                continue;
            }
            const int qs[3] = {o.a, o.b, o.c};
            int t = 0;
            for (int q : qs)
                if (q >= 0) t = std::max(t, layer[q]);
            ++t;
            for (int q : qs)
                if (q >= 0) {
                    layer[q] = t;
                    used[q] = 1;
                }
            g.depth = std::max(g.depth, t);
            if (o.kind == IR_M) ++meas;
        }
        for (char u : used) g.n_qubits += u;
        c->segs.push_back(g);
    }
}

// ---------------------------------------------------------------------------
// compiler

namespace {

struct LOp {          // logical op before centre scheduling
    int32_t kind, a, b, aux;
};

struct Router {
    std::vector<int> site_of, qubit_at, home;
    std::vector<char> product;   // qubit known to be unentangled in every shot
    std::vector<LOp> out;
    int64_t swaps = 0, pswaps = 0;

    static bool is_swap(const LOp& o) {
        return (o.kind == OP_G2 && o.aux == G4_SWAP) || o.kind == OP_SWAPP;
    }
    void swap_bond(int k) {
        if (!out.empty() && is_swap(out.back()) && out.back().a == k) {
            (out.back().kind == OP_SWAPP ? pswaps : swaps) -= 1;
            out.pop_back();          // SWAP . SWAP = identity
        } else if (product[qubit_at[k + 1]] || product[qubit_at[k]]) {
            // a product qubit swaps without an SVD
            out.push_back({OP_SWAPP, k, product[qubit_at[k + 1]] ? 1 : 0, -1});
            ++pswaps;
        } else {
            out.push_back({OP_G2, k, -1, G4_SWAP});
            ++swaps;
        }
        int qa = qubit_at[k], qb = qubit_at[k + 1];
        qubit_at[k] = qb;
        qubit_at[k + 1] = qa;
        site_of[qa] = k + 1;
        site_of[qb] = k;
    }
    void walk_to(int q, int target_site) {
        while (site_of[q] < target_site) swap_bond(site_of[q]);
        while (site_of[q] > target_site) swap_bond(site_of[q] - 1);
    }
    void go_home(int q) { walk_to(q, home[q]); }
    bool displaced() const {
        for (size_t s = 0; s < qubit_at.size(); ++s)
            if (home[qubit_at[s]] != static_cast<int>(s)) return true;
        return false;
    }
};

}  // namespace

// CCZ(a, b, c) = diag(1, ..., 1, -1) as CNOT + T gates: the textbook
// Toffoli network with the target's Hadamards dropped (seven T-type gates,
// six CNOTs); the MPS applies it gate by gate.
static void expand_ccz(const IrOp& o, std::vector<IrOp>& out) {
    auto g1 = [&](int g, int q) { out.push_back({IR_G1, g, q, -1, -1, -1}); };
    auto cx = [&](int a, int b) { out.push_back({IR_G2, G2_CX, a, b, -1, -1}); };
    const int a = o.a, b = o.b, t = o.c;
    cx(b, t); g1(G_TDG, t); cx(a, t); g1(G_T, t); cx(b, t); g1(G_TDG, t); cx(a, t);
    g1(G_T, b); g1(G_T, t); cx(a, b); g1(G_T, a); g1(G_TDG, b); cx(a, b);
}

int compile_circuit(msc_circuit* c) {
    const int n = c->n;
    if (c->order.empty()) {
        c->order.resize(n);
        for (int i = 0; i < n; ++i) c->order[i] = i;
    }
    {
        std::vector<int> seen(n, 0);
        for (int q : c->order) {
            if (q < 0 || q >= n || seen[q]) return set_error(MSC_E_INVALID, "order is not a permutation");
            seen[q] = 1;
        }
    }
    // the router and the scheduler see CCZ as its one- and two-qubit gates
    std::vector<IrOp> ir;
    ir.reserve(c->ir.size());
    for (const auto& o : c->ir) {
        if (o.kind == IR_G3) expand_ccz(o, ir);
        else ir.push_back(o);
    }
    Router R;
    R.site_of.assign(n, 0);
    R.qubit_at = c->order;
    for (int s = 0; s < n; ++s) R.site_of[c->order[s]] = s;
    R.home = R.site_of;
    R.product.assign(n, 1);      // |0...0>: every qubit starts unentangled

    // index of 2q gates for the mover choice
    std::vector<int> g2pos;
    for (size_t i = 0; i < ir.size(); ++i)
        if (ir[i].kind == IR_G2) g2pos.push_back(static_cast<int>(i));
    auto shares = [&](int i, int j) {
        const IrOp &x = ir[i], &y = ir[j];
        if (x.a == y.a || x.a == y.b) return x.a;
        if (x.b == y.a || x.b == y.b) return x.b;
        return -1;
    };
    int walker = -1;   // qubit currently away from home (lazy return)
    std::vector<int> last_meas_site_op(n, -1);
    int g2i = 0;
    for (size_t i = 0; i < ir.size(); ++i) {
        const IrOp& o = ir[i];
        switch (o.kind) {
            case IR_G1:
                R.out.push_back({OP_G1, R.site_of[o.a], -1, o.g});
                break;
            case IR_CH:
                R.out.push_back({OP_FAULT, R.site_of[o.a], o.b >= 0 ? R.site_of[o.b] : -1, o.idx});
                if (o.c >= 0) R.out.push_back({OP_FAULT3, R.site_of[o.c], -1, o.idx});
                break;
            case IR_M:
                R.out.push_back({OP_MEAS, R.site_of[o.a], -1, o.idx});
                break;
            case IR_R:
                // legal only at start (no-op: the qubit is |0>) or after M
                if (last_meas_site_op[o.a] >= 0) R.out.push_back({OP_RESET, R.site_of[o.a], -1, -1});
                break;
            case IR_G2: {
                int self = g2pos[g2i];
                int mover = -1;
                if (g2i + 1 < static_cast<int>(g2pos.size())) mover = shares(self, g2pos[g2i + 1]);
                if (mover < 0 && g2i > 0) mover = shares(self, g2pos[g2i - 1]);
                if (mover < 0) mover = o.a;
                int other = mover == o.a ? o.b : o.a;
                ++g2i;
                if (walker >= 0 && walker != mover) {
                    R.go_home(walker);
                    walker = -1;
                }
                if (std::abs(R.site_of[mover] - R.site_of[other]) > 1) {
                    int t = R.site_of[other] + (R.site_of[mover] < R.site_of[other] ? -1 : 1);
                    R.walk_to(mover, t);
                }
                walker = R.site_of[mover] == R.home[mover] ? -1 : mover;
                if (walker < 0 && R.displaced()) {
                    // the mover is home but others were shifted: impossible
                    // with a single walker; keep the invariant explicit
                    return set_error(MSC_E_INVALID, "router invariant broken");
                }
                int k = std::min(R.site_of[o.a], R.site_of[o.b]);
                int g;
                if (o.g == G2_CX) g = (R.site_of[o.a] == k) ? G4_CX01 : G4_CX10;
                else if (o.g == G2_CZ) g = G4_CZ;
                else if (o.g == G2_CS) g = G4_CS;      // diagonal and symmetric
                else g = G4_CSDG;
                R.out.push_back({OP_G2, k, -1, g});
                break;
            }
            default:
                break;
        }
        // product status: a projective measurement or a reset leaves the
        // qubit unentangled; a two-qubit gate may entangle both operands;
        // one-qubit gates and Pauli faults keep the status
        if (o.kind == IR_M || o.kind == IR_R) R.product[o.a] = 1;
        if (o.kind == IR_G2) R.product[o.a] = R.product[o.b] = 0;
        if (o.kind == IR_M) last_meas_site_op[o.a] = 1;
        else if (o.kind == IR_G1 || o.kind == IR_G2) {
            last_meas_site_op[o.a] = -1;
            if (o.b >= 0) last_meas_site_op[o.b] = -1;
        }
    }
    c->final_site = R.site_of[c->seed];
    R.out.push_back({OP_FINAL, c->final_site, -1, -1});

    // centre scheduling
    auto need_lo = [](const LOp& o) { return o.kind == OP_G2 ? o.a : o.a; };
    auto need_hi = [](const LOp& o) { return o.kind == OP_G2 ? o.a + 1 : o.a; };
    auto needs = [](const LOp& o) { return o.kind == OP_G2 || o.kind == OP_MEAS || o.kind == OP_FINAL; };
    std::vector<int> next_need(R.out.size() + 1, -1);
    for (int i = static_cast<int>(R.out.size()) - 1; i >= 0; --i)
        next_need[i] = needs(R.out[i]) ? i : next_need[i + 1];
    c->ops.clear();
    c->chan_op.assign(c->n_channels, -1);
    c->n_twosite = 0;
    c->n_moves = 0;
    int centre = 0;
    auto move_to = [&](int lo, int hi) {
        while (centre < lo) {
            c->ops.push_back({OP_MOVE, centre, 1, G4_I});
            ++centre;
            ++c->n_moves;
        }
        while (centre > hi) {
            c->ops.push_back({OP_MOVE, centre - 1, 0, G4_I});
            --centre;
            ++c->n_moves;
        }
    };
    for (size_t i = 0; i < R.out.size(); ++i) {
        LOp o = R.out[i];
        if (!needs(o)) {
            if (o.kind == OP_FAULT) c->chan_op[o.aux] = static_cast<int32_t>(c->ops.size());
            c->ops.push_back({o.kind, o.a, o.b, o.aux});
            // the unentangled qubit's partner takes over the centre
            if (o.kind == OP_SWAPP && (centre == o.a || centre == o.a + 1)) centre = o.a + o.b;
            continue;
        }
        move_to(need_lo(o), need_hi(o));
        if (o.kind == OP_G2) {
            int j = (i + 1 < R.out.size()) ? next_need[i + 1] : -1;
            int dir = 1;
            if (j >= 0) {
                const LOp& nx = R.out[j];
                if (need_hi(nx) <= o.a) dir = 0;
                else if (need_lo(nx) >= o.a + 1) dir = 1;
                else dir = (need_lo(nx) <= o.a) ? 0 : 1;
            }
            c->ops.push_back({OP_G2, o.a, dir, o.aux});
            centre = o.a + dir;
            ++c->n_twosite;
        } else {
            c->ops.push_back({o.kind, o.a, o.b, o.aux});
        }
    }
    c->n_swaps = R.swaps;
    c->n_product_swaps = R.pswaps;
    return MSC_OK;
}

}  // namespace msc
