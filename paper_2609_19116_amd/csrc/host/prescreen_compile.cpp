// Offline-screening precompilation (Section 4.2).
//
// Pass 1 walks a sign-free stabiliser tableau of the noiseless circuit:
// Clifford gates conjugate the tracked generators, each diagonal
// non-Clifford gate (T, T^dagger, CS, CS^dagger, CCZ) keeps the largest
// subgroup without X/Y on its support, and each Z measurement is either decided (Z_q is in the tracked
// group) or undecided; an undecided measurement adds +Z_q (only the expected
// outcome is ever accepted) and gets a destabiliser: a Pauli that
// anticommutes with Z_q and commutes with every other tracked generator.
//
// Pass 2 propagates every basis fault (channel c, component X or Z on each
// of the channel's up to three qubits) as a Pauli frame, 64 faults per machine word (bit-sliced frames):
// Cliffords conjugate the frame, diagonal non-Cliffords leave it alone,
// a decided measurement records whether the frame anticommutes with Z_q
// (the outcome flips), an undecided one multiplies in the destabiliser where
// the frame anticommutes with Z_q (the accepted branch pins that sign), and
// a reset clears the qubit.  The result is the GF(2) signature of every
// basis fault over the decided measurements; a shot's signature is the XOR
// of its faults' signatures (SymFT-style precompilation, Section 4.2).
#include <algorithm>
#include <cstring>

#include "../msc_internal.h"

namespace msc {
namespace {

struct Pauli {
    std::vector<uint64_t> x, z;
};

struct Bits {
    int nw;
    explicit Bits(int n) : nw((n + 63) / 64) {}
};

inline bool getb(const std::vector<uint64_t>& v, int i) { return (v[i >> 6] >> (i & 63)) & 1; }
inline void flipb(std::vector<uint64_t>& v, int i) { v[i >> 6] ^= 1ull << (i & 63); }
inline void xorv(std::vector<uint64_t>& a, const std::vector<uint64_t>& b) {
    for (size_t i = 0; i < a.size(); ++i) a[i] ^= b[i];
}

struct Tab {
    int n, nw;
    std::vector<Pauli> g;
    explicit Tab(int n_) : n(n_), nw((n_ + 63) / 64) {
        for (int q = 0; q < n; ++q) {
            Pauli p;
            p.x.assign(nw, 0);
            p.z.assign(nw, 0);
            flipb(p.z, q);
            g.push_back(p);
        }
    }
    void h(int q) {
        for (auto& p : g) {
            bool xb = getb(p.x, q), zb = getb(p.z, q);
            if (xb != zb) { flipb(p.x, q); flipb(p.z, q); }
        }
    }
    void s(int q) {
        for (auto& p : g) if (getb(p.x, q)) flipb(p.z, q);
    }
    void cx(int c, int t) {
        for (auto& p : g) {
            if (getb(p.x, c)) flipb(p.x, t);
            if (getb(p.z, t)) flipb(p.z, c);
        }
    }
    void cz(int a, int b) {
        for (auto& p : g) {
            bool xa = getb(p.x, a), xb = getb(p.x, b);
            if (xb) flipb(p.z, a);
            if (xa) flipb(p.z, b);
        }
    }
    // keep the subgroup without X on q
    void drop_x(int q) {
        int piv = -1;
        for (size_t i = 0; i < g.size(); ++i)
            if (getb(g[i].x, q)) { piv = static_cast<int>(i); break; }
        if (piv < 0) return;
        for (size_t i = 0; i < g.size(); ++i) {
            if (static_cast<int>(i) != piv && getb(g[i].x, q)) {
                xorv(g[i].x, g[piv].x);
                xorv(g[i].z, g[piv].z);
            }
        }
        g.erase(g.begin() + piv);
    }
    // is the Pauli (x, z) in the span of the generators?
    bool in_span(const Pauli& t) const {
        // Gaussian elimination on concatenated (x|z) rows
        int L = 2 * n;
        std::vector<std::vector<uint64_t>> rows;
        auto cat = [&](const Pauli& p) {
            std::vector<uint64_t> r((L + 63) / 64, 0);
            for (int i = 0; i < n; ++i) {
                if (getb(p.x, i)) flipb(r, i);
                if (getb(p.z, i)) flipb(r, n + i);
            }
            return r;
        };
        for (const auto& p : g) rows.push_back(cat(p));
        std::vector<uint64_t> tv = cat(t);
        std::vector<int> pivcol;
        int rank = 0;
        for (int col = 0; col < L && rank < static_cast<int>(rows.size()); ++col) {
            int pr = -1;
            for (int r = rank; r < static_cast<int>(rows.size()); ++r)
                if (getb(rows[r], col)) { pr = r; break; }
            if (pr < 0) continue;
            std::swap(rows[rank], rows[pr]);
            for (int r = 0; r < static_cast<int>(rows.size()); ++r)
                if (r != rank && getb(rows[r], col)) xorv(rows[r], rows[rank]);
            pivcol.push_back(col);
            ++rank;
        }
        for (int r = 0; r < rank; ++r)
            if (getb(tv, pivcol[r])) xorv(tv, rows[r]);
        for (auto w : tv) if (w) return false;
        return true;
    }
    // Pauli D with D.x_q = 1 commuting with every generator except index gi
    bool destabiliser(int gi, int q, Pauli& D) const {
        // unknown vector u = (dx | dz) of length 2n; constraint per generator
        // j != gi: dx . z_j + dz . x_j = 0; plus dx_q = 1.
        int L = 2 * n;
        int W = (L + 1 + 63) / 64;   // last column = right-hand side
        std::vector<std::vector<uint64_t>> rows;
        for (size_t j = 0; j < g.size(); ++j) {
            if (static_cast<int>(j) == gi) continue;
            std::vector<uint64_t> r(W, 0);
            for (int i = 0; i < n; ++i) {
                if (getb(g[j].z, i)) flipb(r, i);
                if (getb(g[j].x, i)) flipb(r, n + i);
            }
            rows.push_back(r);
        }
        {
            std::vector<uint64_t> r(W, 0);
            flipb(r, q);
            flipb(r, L);
            rows.push_back(r);
        }
        std::vector<int> pivcol;
        int rank = 0;
        for (int col = 0; col < L && rank < static_cast<int>(rows.size()); ++col) {
            int pr = -1;
            for (int r = rank; r < static_cast<int>(rows.size()); ++r)
                if (getb(rows[r], col)) { pr = r; break; }
            if (pr < 0) continue;
            std::swap(rows[rank], rows[pr]);
            for (int r = 0; r < static_cast<int>(rows.size()); ++r)
                if (r != rank && getb(rows[r], col)) xorv(rows[r], rows[rank]);
            pivcol.push_back(col);
            ++rank;
        }
        for (int r = rank; r < static_cast<int>(rows.size()); ++r)
            if (getb(rows[r], L)) return false;   // inconsistent
        D.x.assign(nw, 0);
        D.z.assign(nw, 0);
        for (int r = 0; r < rank; ++r) {
            if (!getb(rows[r], L)) continue;     // free variables = 0
            int col = pivcol[r];
            if (col < n) flipb(D.x, col);
            else flipb(D.z, col - n);
        }
        return true;
    }
};

enum MeasClass { M_DECIDED = 0, M_UNDECIDED = 1 };

}  // namespace

int prescreen_compile(msc_circuit* c) {
    const int n = c->n;
    Tab tab(n);
    std::vector<int> mclass(c->n_meas, M_UNDECIDED);
    std::vector<int> dslot(c->n_meas, -1);
    std::vector<Pauli> destab(c->n_meas);
    c->decided.clear();
    for (const auto& o : c->ir) {
        switch (o.kind) {
            case IR_G1:
                if (o.g == G_H) tab.h(o.a);
                else if (o.g == G_S || o.g == G_SDG) tab.s(o.a);
                else if (o.g == G_T || o.g == G_TDG) tab.drop_x(o.a);
                break;
            case IR_G2:
                if (o.g == G2_CX) tab.cx(o.a, o.b);
                else if (o.g == G2_CZ) tab.cz(o.a, o.b);
                else {                         // CS, CS^dagger: diagonal
                    tab.drop_x(o.a);
                    tab.drop_x(o.b);
                }
                break;
            case IR_G3:                        // CCZ: diagonal
                tab.drop_x(o.a);
                tab.drop_x(o.b);
                tab.drop_x(o.c);
                break;
            case IR_M: {
                Pauli zq;
                zq.x.assign(tab.nw, 0);
                zq.z.assign(tab.nw, 0);
                flipb(zq.z, o.a);
                if (tab.in_span(zq)) {
                    mclass[o.idx] = M_DECIDED;
                    dslot[o.idx] = static_cast<int>(c->decided.size());
                    c->decided.push_back(o.idx);
                } else {
                    // standard update: remove generators anticommuting with Z_q
                    tab.drop_x(o.a);
                    tab.g.push_back(zq);
                    if (!tab.destabiliser(static_cast<int>(tab.g.size()) - 1, o.a, destab[o.idx]))
                        return set_error(MSC_E_INVALID, "no destabiliser for an undecided measurement");
                }
                break;
            }
            default:
                break;
        }
    }
    const int nd = static_cast<int>(c->decided.size());
    const int W = std::max(1, (nd + 63) / 64);
    c->words = W;
    constexpr int NC = kFaultComponents;
    const int nb = NC * c->n_channels;
    c->sig.assign(static_cast<size_t>(nb) * W, 0);
    // channel -> ir position
    std::vector<int> chan_pos(c->n_channels, -1);
    for (size_t i = 0; i < c->ir.size(); ++i)
        if (c->ir[i].kind == IR_CH) chan_pos[c->ir[i].idx] = static_cast<int>(i);
    std::vector<uint64_t> fx(n), fz(n);
    for (int base = 0; base < nb; base += 64) {
        std::fill(fx.begin(), fx.end(), 0);
        std::fill(fz.begin(), fz.end(), 0);
        int first_chan = base / NC;
        int last_chan = std::min(c->n_channels - 1, (base + 63) / NC);
        for (size_t i = chan_pos[first_chan]; i < c->ir.size(); ++i) {
            const IrOp& o = c->ir[i];
            switch (o.kind) {
                case IR_CH: {
                    if (o.idx < first_chan || o.idx > last_chan) break;
                    for (int k = 0; k < NC; ++k) {
                        int b = NC * o.idx + k - base;
                        if (b < 0 || b >= 64) continue;
                        int q = k < 2 ? o.a : k < 4 ? o.b : o.c;
                        if (q < 0) continue;
                        if (k % 2 == 0) fx[q] ^= 1ull << b;
                        else fz[q] ^= 1ull << b;
                    }
                    break;
                }
                case IR_G1:
                    if (o.g == G_H) std::swap(fx[o.a], fz[o.a]);
                    else if (o.g == G_S || o.g == G_SDG) fz[o.a] ^= fx[o.a];
                    break;   // Paulis and diagonal non-Cliffords: frame unchanged
                case IR_G2:
                    if (o.g == G2_CX) {
                        fx[o.b] ^= fx[o.a];
                        fz[o.a] ^= fz[o.b];
                    } else if (o.g == G2_CZ) {
                        fz[o.a] ^= fx[o.b];
                        fz[o.b] ^= fx[o.a];
                    }
                    break;   // CS, CS^dagger (and CCZ, IR_G3): frame unchanged
                case IR_M: {
                    uint64_t m = fx[o.a];
                    if (mclass[o.idx] == M_DECIDED) {
                        int d = dslot[o.idx];
                        while (m) {
                            int b = __builtin_ctzll(m);
                            m &= m - 1;
                            c->sig[static_cast<size_t>(base + b) * W + (d >> 6)] |= 1ull << (d & 63);
                        }
                    } else if (m) {
                        const Pauli& D = destab[o.idx];
                        for (int q = 0; q < n; ++q) {
                            if (getb(D.x, q)) fx[q] ^= m;
                            if (getb(D.z, q)) fz[q] ^= m;
                        }
                    }
                    break;
                }
                case IR_R:
                    fx[o.a] = 0;
                    fz[o.a] = 0;
                    break;
                default:
                    break;
            }
        }
    }
    return MSC_OK;
}

}  // namespace msc
