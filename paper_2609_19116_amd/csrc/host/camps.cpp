// Host side of the CAMPS shots (section "Clifford augmented MPS"): the op
// stream of the frame and the residual, and the disentangler's candidate
// two-qubit Cliffords.
//
// Op stream.  Clifford gates (H S SDG X Y Z CX CZ) act on the frame only;
// T and T^dagger become Pauli rotations of the residual; CS, CS^dagger and
// CCZ are first written over T, T^dagger and CX (CS = T_a T_b CX T^dag_b CX,
// CCZ by the textbook seven-T network); faults, measurements, resets and
// the final read-out keep their order.
//
// Candidates.  Two-qubit Cliffords modulo Paulis are the 720 symplectic
// matrices S over GF(2) acting on (x1, z1, x2, z2).  The entanglement of
// D|m> across the bond is the same for every member of a class
// {(L1 + L2) S : L1, L2 in SL(2, 2)} (local Cliffords after D), so one
// member per class is tried: the one with the smallest code
// sum_{r,c} S[r][c] 2^(4r+c), classes in increasing code, the class of the
// identity left out (19).  The unitary D of S satisfies
// D P D^dag = Q(S v_P) for P = X1, Z1, X2, Z2 with Q(v) the Hermitian Pauli
// i^(x1 z1 + x2 z2) X^x1 Z^z1 (x) X^x2 Z^z2; its phase is fixed by
// D|00> = normalised (I + Q_Z1)(I + Q_Z2)|w> (w the first basis state that
// gives a nonzero vector, first nonzero amplitude real positive) and
// D|ab> = Q_X1^a Q_X2^b D|00>, qubit 1 being the left site.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <vector>

#include "../msc_internal.h"

namespace msc {

void camps_compile(msc_circuit* c) {
    c->camps_ops.clear();
    c->chan_q.assign(static_cast<size_t>(3) * c->n_channels, -1);
    auto& o = c->camps_ops;
    auto g1 = [&](int g, int q) { o.push_back({CO_G1, q, -1, g}); };
    auto rot = [&](int q, int sgn) { o.push_back({CO_ROT, q, -1, sgn}); };
    auto cx = [&](int a, int b) { o.push_back({CO_CX, a, b, 0}); };
    for (const IrOp& op : c->ir) {
        switch (op.kind) {
        case IR_G1:
            if (op.g == G_T) rot(op.a, 1);
            else if (op.g == G_TDG) rot(op.a, -1);
            else g1(op.g, op.a);
            break;
        case IR_G2:
            if (op.g == G2_CX) {
                cx(op.a, op.b);
            } else if (op.g == G2_CZ) {
                o.push_back({CO_CZ, op.a, op.b, 0});
            } else {
                const int s = op.g == G2_CS ? 1 : -1;
                rot(op.a, s);
                rot(op.b, s);
                cx(op.a, op.b);
                rot(op.b, -s);
                cx(op.a, op.b);
            }
            break;
        case IR_G3: {
            const int a = op.a, b = op.b, t = op.c;
            cx(b, t); rot(t, -1); cx(a, t); rot(t, 1); cx(b, t); rot(t, -1); cx(a, t);
            rot(b, 1); rot(t, 1); cx(a, b); rot(a, 1); rot(b, -1); cx(a, b);
            break;
        }
        case IR_M:
            o.push_back({CO_MEAS, op.a, -1, op.idx});
            break;
        case IR_R:
            o.push_back({CO_RESET, op.a, -1, 0});
            break;
        case IR_CH:
            o.push_back({CO_FAULT, op.idx, -1, 0});
            c->chan_q[3 * op.idx] = op.a;
            c->chan_q[3 * op.idx + 1] = op.b;
            c->chan_q[3 * op.idx + 2] = op.c;
            break;
        default:
            break;
        }
    }
    o.push_back({CO_FINAL, c->seed, -1, 0});
}

namespace {

typedef std::complex<double> cd;
typedef std::array<std::array<int, 4>, 4> Mat2;   // GF(2) 4x4

Mat2 from_code(int code) {
    Mat2 S{};
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) S[r][c] = (code >> (4 * r + c)) & 1;
    return S;
}

int to_code(const Mat2& S) {
    int k = 0;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) k |= S[r][c] << (4 * r + c);
    return k;
}

Mat2 mul(const Mat2& A, const Mat2& B) {
    Mat2 C{};
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            int v = 0;
            for (int k = 0; k < 4; ++k) v ^= A[r][k] & B[k][c];
            C[r][c] = v;
        }
    return C;
}

bool symplectic(const Mat2& S) {
    // S^T Omega S = Omega with Omega pairing (x1, z1) and (x2, z2)
    auto omega = [](int i, int j) { return (i ^ 1) == j ? 1 : 0; };
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            int v = 0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) v ^= S[a][i] & omega(a, b) & S[b][j];
            if (v != omega(i, j)) return false;
        }
    return true;
}

// 4x4 matrix of the Hermitian Pauli Q(v), v = (x1, z1, x2, z2)
std::array<cd, 16> pauli_matrix(int x1, int z1, int x2, int z2) {
    auto one = [](int x, int z) {
        // X^x Z^z as a 2x2 matrix
        std::array<cd, 4> m{cd(1), cd(0), cd(0), cd(1)};
        if (z) m = {cd(1), cd(0), cd(0), cd(-1)};
        if (x) m = {m[2], m[3], m[0], m[1]};
        return m;
    };
    const auto a = one(x1, z1), b = one(x2, z2);
    cd ph(1, 0);
    for (int k = 0; k < x1 * z1 + x2 * z2; ++k) ph *= cd(0, 1);
    std::array<cd, 16> m{};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l)
                    m[(2 * i + k) * 4 + (2 * j + l)] = ph * a[2 * i + j] * b[2 * k + l];
    return m;
}

std::array<cd, 4> matvec(const std::array<cd, 16>& m, const std::array<cd, 4>& v) {
    std::array<cd, 4> r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r[i] += m[i * 4 + j] * v[j];
    return r;
}

}  // namespace

void camps_candidates(std::vector<double>& dmat, std::vector<uint8_t>& dtab) {
    std::vector<Mat2> locals;
    for (int a = 0; a < 16; ++a)
        for (int b = 0; b < 16; ++b) {
            const int a00 = a & 1, a01 = (a >> 1) & 1, a10 = (a >> 2) & 1, a11 = (a >> 3) & 1;
            const int b00 = b & 1, b01 = (b >> 1) & 1, b10 = (b >> 2) & 1, b11 = (b >> 3) & 1;
            if (((a00 & a11) ^ (a01 & a10)) == 0 || ((b00 & b11) ^ (b01 & b10)) == 0) continue;
            Mat2 L{};
            L[0][0] = a00; L[0][1] = a01; L[1][0] = a10; L[1][1] = a11;
            L[2][2] = b00; L[2][3] = b01; L[3][2] = b10; L[3][3] = b11;
            locals.push_back(L);
        }
    auto rep = [&](const Mat2& S) {
        int best = 1 << 16;
        for (const Mat2& L : locals) best = std::min(best, to_code(mul(L, S)));
        return best;
    };
    std::vector<int> reps;
    for (int code = 0; code < (1 << 16); ++code) {
        const Mat2 S = from_code(code);
        if (symplectic(S)) reps.push_back(rep(S));
    }
    std::sort(reps.begin(), reps.end());
    reps.erase(std::unique(reps.begin(), reps.end()), reps.end());
    Mat2 I{};
    for (int i = 0; i < 4; ++i) I[i][i] = 1;
    const int ident = rep(I);
    reps.erase(std::remove(reps.begin(), reps.end(), ident), reps.end());
    dmat.assign(static_cast<size_t>(reps.size()) * 32, 0.0);
    dtab.assign(static_cast<size_t>(reps.size()) * 16, 0);
    for (size_t ci = 0; ci < reps.size(); ++ci) {
        const Mat2 S = from_code(reps[ci]);
        std::array<std::array<cd, 16>, 4> Q;   // images of X1, Z1, X2, Z2
        for (int c = 0; c < 4; ++c) Q[c] = pauli_matrix(S[0][c], S[1][c], S[2][c], S[3][c]);
        // projector (I + Q_Z1)(I + Q_Z2)
        std::array<cd, 16> P{};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cd v = 0;
                for (int k = 0; k < 4; ++k) {
                    const cd a = (i == k ? cd(1) : cd(0)) + Q[1][i * 4 + k];
                    const cd b = (k == j ? cd(1) : cd(0)) + Q[3][k * 4 + j];
                    v += a * b;
                }
                P[i * 4 + j] = v;
            }
        std::array<cd, 4> v00{};
        for (int w = 0; w < 4; ++w) {
            double nr = 0;
            for (int i = 0; i < 4; ++i) nr += std::norm(P[i * 4 + w]);
            if (std::sqrt(nr) > 1e-9) {
                for (int i = 0; i < 4; ++i) v00[i] = P[i * 4 + w] / std::sqrt(nr);
                break;
            }
        }
        for (int i = 0; i < 4; ++i)
            if (std::abs(v00[i]) > 1e-9) {
                const cd ph = std::abs(v00[i]) / v00[i];
                for (auto& x : v00) x *= ph;
                break;
            }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                std::array<cd, 4> v = v00;
                if (a) v = matvec(Q[0], v);
                if (b) v = matvec(Q[2], v);
                for (int i = 0; i < 4; ++i) {
                    dmat[ci * 32 + 2 * (i * 4 + 2 * a + b)] = v[i].real();
                    dmat[ci * 32 + 2 * (i * 4 + 2 * a + b) + 1] = v[i].imag();
                }
            }
        // Pauli map: X1^x1 Z1^z1 X2^x2 Z2^z2 -> Q_X1^x1 Q_Z1^z1 Q_X2^x2 Q_Z2^z2,
        // each factor i^h X^a Z^b with a, b bit pairs (qubit 1 in bit 0)
        for (int loc = 0; loc < 16; ++loc) {
            int h = 0, ax = 0, bz = 0;
            for (int f = 0; f < 4; ++f) {
                if (!((loc >> f) & 1)) continue;
                const int x1 = S[0][f], z1 = S[1][f], x2 = S[2][f], z2 = S[3][f];
                const int a2 = x1 | (x2 << 1), b2 = z1 | (z2 << 1);
                const int h2 = x1 * z1 + x2 * z2;
                h += h2 + 2 * __builtin_popcount(bz & a2);
                ax ^= a2;
                bz ^= b2;
            }
            const int bits = (ax & 1) | ((bz & 1) << 1) | (((ax >> 1) & 1) << 2) | (((bz >> 1) & 1) << 3);
            dtab[ci * 16 + loc] = static_cast<uint8_t>(bits | ((h & 3) << 4));
        }
    }
}

}  // namespace msc
