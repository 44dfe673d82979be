// Host planner of the effective block algorithm (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>

namespace bbc {

namespace {

const double kR6 = 1.0 / std::sqrt(6.0), kR2 = 1.0 / std::sqrt(2.0);
const double kR3 = 1.0 / std::sqrt(3.0), kR23 = std::sqrt(2.0 / 3.0);

// Baryon fields of Sec. 2, Eqs. (FieldOperator_N), (FieldOperator_SLXi),
// (FieldOperator_xxx).  Lambda and Sigma0 keep the fixed field order
// (d, s, u) used in Sec. 3, Eq. (LN.pLLp.ududsu): X_d = eps (s C g5 u) d and
// X_s = eps (u C g5 d) s are cyclic rotations of that order (an even
// permutation of three Grassmann fields), so only their tensor roles move.
// Further fields of the general form of Sec. 2, Eq. (FieldOperator_B): the
// nucleon with {C, gamma_5} (same flavour terms as p, n) and the decuplet fields
// with {C gamma_l, 1} (Sec. 4 footnote), l = 1, 2, 3.  The decuplet members of
// mixed flavour are the symmetric flavour combinations (a reading), e.g.
// Delta+ = (2 eps (u G d) u + eps (u G u) d) / sqrt3 in the field order (u, d, u):
// the string u u d is the order's transposition (0 2 1), so that term's weight
// carries -1; the three terms of Sigma*0 are cyclic rotations of (u, d, s).
enum { B_P, B_N, B_SP, B_SM, B_X0, B_XM, B_L, B_S0, B_P2, B_N2, B_DPP1, B_DM1 = B_DPP1 + 3, B_OM1 = B_DM1 + 3,
       B_DP1 = B_OM1 + 3, B_D01 = B_DP1 + 3, B_SSP1 = B_D01 + 3, B_SS01 = B_SSP1 + 3, B_SSM1 = B_SS01 + 3,
       B_XS01 = B_SSM1 + 3, B_XSM1 = B_XS01 + 3, B_COUNT = B_XSM1 + 3 };
static_assert(B_COUNT == kNumBaryons && B_P2 == kNumOctet, "baryon table");

const Baryon kBaryons[B_COUNT] = {
    {"p",  {FU, FD, FU}, 1, {{+1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"n",  {FU, FD, FD}, 1, {{-1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"S+", {FU, FS, FU}, 1, {{-1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"S-", {FD, FS, FD}, 1, {{-1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"X0", {FU, FS, FS}, 1, {{+1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"X-", {FD, FS, FS}, 1, {{-1.0, {0, 1, 2}, "-"}}, SP_OCTET},
    {"L",  {FD, FS, FU}, 3, {{kR6, {0, 1, 2}, "Xu"}, {kR6, {1, 2, 0}, "Xd"}, {-2.0 * kR6, {2, 0, 1}, "Xs"}}, SP_OCTET},
    {"S0", {FD, FS, FU}, 2, {{kR2, {0, 1, 2}, "Xu"}, {-kR2, {1, 2, 0}, "Xd"}}, SP_OCTET},
    {"p2", {FU, FD, FU}, 1, {{+1.0, {0, 1, 2}, "-"}}, SP_CHI2},
    {"n2", {FU, FD, FD}, 1, {{-1.0, {0, 1, 2}, "-"}}, SP_CHI2},
    {"D++(1)", {FU, FU, FU}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1},
    {"D++(2)", {FU, FU, FU}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 1},
    {"D++(3)", {FU, FU, FU}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 2},
    {"D-(1)", {FD, FD, FD}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1},
    {"D-(2)", {FD, FD, FD}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 1},
    {"D-(3)", {FD, FD, FD}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 2},
    {"O-(1)", {FS, FS, FS}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1},
    {"O-(2)", {FS, FS, FS}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 1},
    {"O-(3)", {FS, FS, FS}, 1, {{1.0, {0, 1, 2}, "-"}}, SP_DEC1 + 2},
#define BBC_DEC2(NAME, F0, F1, L)                                                                               \
    {NAME "(" #L ")", {F0, F1, F0}, 2, {{2.0 * kR3, {0, 1, 2}, "-"}, {-kR3, {0, 2, 1}, "-"}}, SP_DEC1 + L - 1}
    BBC_DEC2("D+", FU, FD, 1), BBC_DEC2("D+", FU, FD, 2), BBC_DEC2("D+", FU, FD, 3),
    BBC_DEC2("D0", FD, FU, 1), BBC_DEC2("D0", FD, FU, 2), BBC_DEC2("D0", FD, FU, 3),
    BBC_DEC2("S*+", FU, FS, 1), BBC_DEC2("S*+", FU, FS, 2), BBC_DEC2("S*+", FU, FS, 3),
#define BBC_DECS0(L)                                                                                            \
    {"S*0(" #L ")", {FU, FD, FS}, 3, {{kR23, {0, 1, 2}, "-"}, {kR23, {1, 2, 0}, "-"}, {kR23, {2, 0, 1}, "-"}},  \
     SP_DEC1 + L - 1}
    BBC_DECS0(1), BBC_DECS0(2), BBC_DECS0(3),
    BBC_DEC2("S*-", FD, FS, 1), BBC_DEC2("S*-", FD, FS, 2), BBC_DEC2("S*-", FD, FS, 3),
    BBC_DEC2("X*0", FS, FU, 1), BBC_DEC2("X*0", FS, FU, 2), BBC_DEC2("X*0", FS, FU, 3),
    BBC_DEC2("X*-", FS, FD, 1), BBC_DEC2("X*-", FS, FD, 2), BBC_DEC2("X*-", FS, FD, 3),
#undef BBC_DEC2
#undef BBC_DECS0
};

// Complex 4x4 matrices with Gaussian-integer entries, enough for products of
// Dirac matrices in the Dirac representation.
struct GI { int re, im; };
using M4 = std::array<std::array<GI, 4>, 4>;
M4 mmul(const M4 &A, const M4 &B) {
    M4 C{};
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) {
        int re = 0, im = 0;
        for (int k = 0; k < 4; ++k) {
            re += A[i][k].re * B[k][j].re - A[i][k].im * B[k][j].im;
            im += A[i][k].re * B[k][j].im + A[i][k].im * B[k][j].re;
        }
        C[i][j] = GI{re, im};
    }
    return C;
}
// Dirac representation: gamma_4 = diag(1, 1, -1, -1); gamma_k has -i sigma_k in the
// upper right and i sigma_k in the lower left 2x2 block; gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
M4 dirac_gamma(int mu) {
    M4 G{};
    if (mu == 4) {
        for (int i = 0; i < 4; ++i) G[i][i] = GI{i < 2 ? 1 : -1, 0};
        return G;
    }
    if (mu == 5) return mmul(mmul(dirac_gamma(1), dirac_gamma(2)), mmul(dirac_gamma(3), dirac_gamma(4)));
    // Pauli matrix sigma_mu
    GI sg[2][2];
    if (mu == 1) { sg[0][0] = {0, 0}; sg[0][1] = {1, 0}; sg[1][0] = {1, 0}; sg[1][1] = {0, 0}; }
    else if (mu == 2) { sg[0][0] = {0, 0}; sg[0][1] = {0, -1}; sg[1][0] = {0, 1}; sg[1][1] = {0, 0}; }
    else { sg[0][0] = {1, 0}; sg[0][1] = {0, 0}; sg[1][0] = {0, 0}; sg[1][1] = {-1, 0}; }
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
        G[i][2 + j] = GI{sg[i][j].im, -sg[i][j].re};       // -i sigma
        G[2 + i][j] = GI{-sg[i][j].im, sg[i][j].re};       //  i sigma
    }
    return G;
}
M4 identity4() {
    M4 I{};
    for (int i = 0; i < 4; ++i) I[i][i] = GI{1, 0};
    return I;
}
// Monomial form of M: per row the column and the power of i of its single nonzero entry.
void monomial(const M4 &M, int p[4], int k[4]) {
    for (int i = 0; i < 4; ++i) {
        int n = 0;
        for (int j = 0; j < 4; ++j) {
            const GI v = M[i][j];
            if (v.re == 0 && v.im == 0) continue;
            ++n;
            p[i] = j;
            if (v.re == 1 && v.im == 0) k[i] = 0;
            else if (v.re == 0 && v.im == 1) k[i] = 1;
            else if (v.re == -1 && v.im == 0) k[i] = 2;
            else if (v.re == 0 && v.im == -1) k[i] = 3;
            else throw std::logic_error("spin matrix entry is not a power of i");
        }
        if (n != 1) throw std::logic_error("spin matrix is not monomial");
    }
}
SpinStruct make_spin(const M4 &G1, const M4 &G2) {
    SpinStruct S{};
    monomial(G1, S.p1, S.k1);
    monomial(G2, S.p2, S.k2);
    bool sym = true, anti = true;
    for (int m = 0; m < 4; ++m) {
        const int n = S.p1[m];
        sym = sym && S.p1[n] == m && S.k1[n] == S.k1[m];
        anti = anti && S.p1[n] == m && S.k1[n] == (S.k1[m] + 2) % 4;
    }
    if (sym == anti) throw std::logic_error("Gamma_1 neither symmetric nor antisymmetric");
    S.x = sym ? -1 : +1;
    return S;
}

// Channel list of Sec. 4 (printed order), then the four omitted isospin-zero ones.
const int kChannels[kNumChannelsAll][4] = {
    {B_P, B_N, B_P, B_N},
    {B_P, B_L, B_P, B_L}, {B_P, B_L, B_SP, B_N}, {B_P, B_L, B_S0, B_P},
    {B_SP, B_N, B_P, B_L}, {B_SP, B_N, B_SP, B_N}, {B_SP, B_N, B_S0, B_P},
    {B_S0, B_P, B_P, B_L}, {B_S0, B_P, B_SP, B_N}, {B_S0, B_P, B_S0, B_P},
    {B_L, B_L, B_L, B_L}, {B_L, B_L, B_P, B_XM}, {B_L, B_L, B_N, B_X0}, {B_L, B_L, B_SP, B_SM},
    {B_L, B_L, B_S0, B_S0},
    {B_P, B_XM, B_L, B_L}, {B_P, B_XM, B_P, B_XM}, {B_P, B_XM, B_N, B_X0}, {B_P, B_XM, B_SP, B_SM},
    {B_P, B_XM, B_S0, B_S0}, {B_P, B_XM, B_S0, B_L},
    {B_N, B_X0, B_L, B_L}, {B_N, B_X0, B_P, B_XM}, {B_N, B_X0, B_N, B_X0}, {B_N, B_X0, B_SP, B_SM},
    {B_N, B_X0, B_S0, B_S0}, {B_N, B_X0, B_S0, B_L},
    {B_SP, B_SM, B_L, B_L}, {B_SP, B_SM, B_P, B_XM}, {B_SP, B_SM, B_N, B_X0},
    {B_SP, B_SM, B_SP, B_SM}, {B_SP, B_SM, B_S0, B_S0}, {B_SP, B_SM, B_S0, B_L},
    {B_S0, B_S0, B_L, B_L}, {B_S0, B_S0, B_P, B_XM}, {B_S0, B_S0, B_N, B_X0},
    {B_S0, B_S0, B_SP, B_SM}, {B_S0, B_S0, B_S0, B_S0},
    {B_S0, B_L, B_P, B_XM}, {B_S0, B_L, B_N, B_X0}, {B_S0, B_L, B_SP, B_SM}, {B_S0, B_L, B_S0, B_L},
    {B_XM, B_L, B_XM, B_L}, {B_XM, B_L, B_SM, B_X0}, {B_XM, B_L, B_S0, B_XM},
    {B_SM, B_X0, B_XM, B_L}, {B_SM, B_X0, B_SM, B_X0}, {B_SM, B_X0, B_S0, B_XM},
    {B_S0, B_XM, B_XM, B_L}, {B_S0, B_XM, B_SM, B_X0}, {B_S0, B_XM, B_S0, B_XM},
    {B_XM, B_X0, B_XM, B_X0},
    // omitted in Sec. 4: identically zero in the isospin limit
    {B_L, B_L, B_S0, B_L}, {B_S0, B_S0, B_S0, B_L}, {B_S0, B_L, B_L, B_L}, {B_S0, B_L, B_S0, B_S0},
};

int perm_sign(const int *p, int n) {
    int q[8];
    for (int i = 0; i < n; ++i) q[i] = p[i];
    int s = 1;
    for (int i = 0; i < n; ++i)
        while (q[i] != i) { std::swap(q[i], q[q[i]]); s = -s; }
    return s;
}

// The spin structure an intermediate needs to know of a source baryon with n
// diquark legs and ncp delta legs at its site: a lone diquark leg carries no
// tensor factor, a lone delta leg only a row of Gamma_2, two diquark legs only
// Gamma_1; structures that agree on what is used share the smallest id.
int effective_spin(int s, int n, int ncp) {
    if (n == 1 && ncp == 0) return 0;
    const SpinStruct &S = spin_struct(s);
    for (int t = 0; t < s; ++t) {
        const SpinStruct &U = spin_struct(t);
        bool same = true;
        for (int m = 0; m < 4; ++m) {
            if (ncp) same = same && U.p2[m] == S.p2[m] && U.k2[m] == S.k2[m];
            if (n) same = same && U.p1[m] == S.p1[m] && U.k1[m] == S.k1[m];
        }
        if (same) return t;
    }
    return s;
}

// Canonical key of an intermediate from per-role (light/strange, source baryon
// X, source role a'/b'/c') and the spin structures involved.  Exchanging sink
// roles a and b together with their propagators multiplies the sink tensor by
// its exchange sign x (+1 for C gamma_5 and C, -1 for the symmetric C gamma_l),
// and which source baryon is "first" is a label; the canonical form relabels
// source baryons by first appearance and takes the smaller of the two role
// orders.  The source legs a' and b' are relabelled too: in the canonical form
// the diquark leg at the lower role (or the only local one, next to a local c')
// is a' and both read 0; where that exchanges a' and b' the intermediate picks
// up the source field's exchange sign x.  A lone diquark leg without c' carries
// no tensor factor, so its label is free.  *sign receives the product of these
// factors for the chosen form, ymap X -> canonical Y, csrc the spin structure
// of each canonical Y (-1 if absent).
uint32_t canonical(const int pf[3], const int X[3], const int T[3], int sink_spin, const int src_spin[2],
                   int ymap[2], int cpf[3], int cy[3], int ct[3], int csrc[2], int *sign) {
    uint32_t best = 0xffffffffu;
    const int orders[2][3] = {{0, 1, 2}, {1, 0, 2}};
    for (int o = 0; o < 2; ++o) {
        const int *ord = orders[o];
        int m[2] = {-1, -1}, nx = 0;
        int lpf[3], ly[3], lt[3];
        int sg = o ? spin_struct(sink_spin).x : 1;
        for (int i = 0; i < 3; ++i) {
            int r = ord[i];
            if (m[X[r]] < 0) m[X[r]] = nx++;
            lpf[i] = pf[r]; ly[i] = m[X[r]];
            lt[i] = T[r] == 2 ? 2 : 0;
        }
        int ls[2] = {-1, -1};
        for (int x = 0; x < 2; ++x) {
            if (m[x] < 0) continue;
            int tp[3], n = 0, ncp = 0;
            for (int i = 0; i < 3; ++i)
                if (X[ord[i]] == x) { if (T[ord[i]] == 2) ++ncp; else tp[n++] = T[ord[i]]; }
            const bool relabel = (n == 2 || (n == 1 && ncp == 1)) && tp[0] == 1;
            if (relabel) sg *= spin_struct(src_spin[x]).x;
            ls[m[x]] = effective_spin(src_spin[x], n, ncp);
        }
        uint32_t key = 0;
        for (int i = 0; i < 3; ++i) key = key * 16 + (uint32_t)((lpf[i] * 2 + ly[i]) * 4 + lt[i]);
        key = (key << 12) | ((uint32_t)sink_spin << 8) | ((uint32_t)(ls[0] < 0 ? 15 : ls[0]) << 4) |
              (uint32_t)(ls[1] < 0 ? 15 : ls[1]);
        if (key < best) {
            best = key;
            *sign = sg;
            ymap[0] = m[0]; ymap[1] = m[1];
            csrc[0] = ls[0]; csrc[1] = ls[1];
            for (int i = 0; i < 3; ++i) { cpf[i] = lpf[i]; cy[i] = ly[i]; ct[i] = lt[i]; }
        }
    }
    return best;
}

Intermediate make_intermediate(uint32_t key, const int pf[3], const int y[3], const int t[3], int sink_spin,
                               const int src_spin[2]) {
    Intermediate I{};
    I.key = key;
    for (int i = 0; i < 3; ++i) { I.pflav[i] = pf[i]; I.role_y[i] = y[i]; I.role_t[i] = t[i]; }
    I.sink_spin = sink_spin;
    I.src_spin[0] = src_spin[0]; I.src_spin[1] = src_spin[1];
    I.ny = (y[0] == 1 || y[1] == 1 || y[2] == 1) ? 2 : 1;
    for (int Y = 0; Y < 2; ++Y) {
        int nD = 0, nd = 0;
        for (int i = 0; i < 3; ++i)
            if (y[i] == Y) (t[i] == 2 ? nd : nD)++;
        int kind = -1;
        if (nD == 2 && nd == 1) kind = Y_FULL;
        else if (nD == 2 && nd == 0) kind = Y_DD;
        else if (nD == 1 && nd == 1) kind = Y_DDELTA;
        else if (nD == 1 && nd == 0) kind = Y_DIN;
        else if (nD == 0 && nd == 1) kind = Y_DELTAIN;
        else if (nD == 0 && nd == 0) kind = -1;
        else throw std::logic_error("impossible source-baryon arrangement");
        I.kind[Y] = kind;
        static const int NO[5] = {2, 1, 2, 1, 2}, NK[5] = {1, 3, 12, 12, 3};
        I.no[Y] = kind < 0 ? 1 : NO[kind];
        I.nk[Y] = kind < 0 ? 1 : NK[kind];
    }
    int d1 = I.no[1] * I.nk[1];
    I.stride_o[0] = I.nk[0] * d1; I.stride_k[0] = d1;
    I.stride_o[1] = I.nk[1];      I.stride_k[1] = 1;
    I.ncomp = I.no[0] * I.nk[0] * d1;
    return I;
}

}  // namespace

const SpinStruct &spin_struct(int s) {
    static const std::array<SpinStruct, kNumSpinStructsAll> t = [] {
        std::array<SpinStruct, kNumSpinStructsAll> v{};
        const M4 C = mmul(dirac_gamma(4), dirac_gamma(2));
        v[SP_OCTET] = make_spin(mmul(C, dirac_gamma(5)), identity4());
        v[SP_CHI2] = make_spin(C, dirac_gamma(5));
        for (int l = 1; l <= 3; ++l) v[SP_DEC1 + l - 1] = make_spin(mmul(C, dirac_gamma(l)), identity4());
        for (int s = 0; s < kNumSpinStructs; ++s) {
            SpinStruct &u = v[kNumSpinStructs + s];
            u = v[s];
            for (int g = 0; g < 4; ++g) {
                u.p2[g] = v[s].p2[(g + 2) & 3];
                u.k2[g] = v[s].k2[(g + 2) & 3];
            }
        }
        return v;
    }();
    return t[s];
}

const Baryon &baryon(int id) { return kBaryons[id]; }

// Baryon quadruple of a channel id: the listed channels, the octet quadruples,
// then the quadruples of all fields.
std::array<int, 4> channel_baryons(int ch) {
    if (ch < kChannelExtBase) return {kChannels[ch][0], kChannels[ch][1], kChannels[ch][2], kChannels[ch][3]};
    if (ch < kChannelGenBase) {
        const int e = ch - kChannelExtBase;
        return {e / 512, (e / 64) % 8, (e / 8) % 8, e % 8};
    }
    const int e = ch - kChannelGenBase, n = kNumBaryons;
    return {e / (n * n * n), (e / (n * n)) % n, (e / n) % n, e % n};
}

bool channel_valid(int ch) {
    if (ch < 0 || ch >= kNumChannelIds) return false;
    const auto b = channel_baryons(ch);
    if (ch >= kChannelGenBase && b[0] < kNumOctet && b[1] < kNumOctet && b[2] < kNumOctet && b[3] < kNumOctet)
        return false;                               // octet quadruples have their id below kChannelGenBase
    int n[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        n[kBaryons[b[0]].flav[i]]++; n[kBaryons[b[1]].flav[i]]++;
        n[kBaryons[b[2]].flav[i]]--; n[kBaryons[b[3]].flav[i]]--;
    }
    return n[0] == 0 && n[1] == 0 && n[2] == 0;
}

int channel_id(const int b[4]) {
    for (int c = 0; c < kNumChannelsAll; ++c)
        if (kChannels[c][0] == b[0] && kChannels[c][1] == b[1] && kChannels[c][2] == b[2] && kChannels[c][3] == b[3])
            return c;
    if (b[0] < kNumOctet && b[1] < kNumOctet && b[2] < kNumOctet && b[3] < kNumOctet)
        return kChannelExtBase + ((b[0] * 8 + b[1]) * 8 + b[2]) * 8 + b[3];
    const int n = kNumBaryons;
    return kChannelGenBase + ((b[0] * n + b[1]) * n + b[2]) * n + b[3];
}

std::string channel_name(int ch) {
    const auto b = channel_baryons(ch);
    return std::string(kBaryons[b[0]].name) + " " + kBaryons[b[1]].name + " > " + kBaryons[b[2]].name + " " +
           kBaryons[b[3]].name;
}

std::vector<Diagram> classify(int ch, int t3, int t4, std::map<uint32_t, int> *index,
                              std::vector<Intermediate> *inters, const int *lower) {
    const auto bb = channel_baryons(ch);
    const Baryon &B1 = kBaryons[bb[0]], &B2 = kBaryons[bb[1]], &B3 = kBaryons[bb[2]], &B4 = kBaryons[bb[3]];
    // spin structure of each baryon, its shifted form where its lower pair is asked for
    int spn[4];
    for (int i = 0; i < 4; ++i) spn[i] = kBaryons[bb[i]].spin + (lower && lower[i] ? kNumSpinStructs : 0);
    int fs[6], fsrc[6], rsrc[6];
    for (int i = 0; i < 3; ++i) {
        fs[i] = B1.flav[i]; fs[3 + i] = B2.flav[i];
        fsrc[i] = B3.flav[i]; fsrc[3 + i] = B4.flav[i];
    }
    // role of each source field in the chosen source terms
    for (int r = 0; r < 3; ++r) {
        rsrc[B3.term[t3].role[r]] = r;
        rsrc[3 + B4.term[t4].role[r]] = r;
    }
    const double w34 = B3.term[t3].w * B4.term[t4].w;
    const int srcspin[2] = {spn[2], spn[3]};
    std::vector<Diagram> out;
    // A diagram is the set of source fields contracted with the quarks of B1
    // (site X+r); Wick maps differing only by exchanges of identical quarks
    // inside one sink baryon belong to the same diagram (Sec. 3).
    for (int a0 = 0; a0 < 6; ++a0)
        for (int a1 = a0 + 1; a1 < 6; ++a1)
            for (int a2 = a1 + 1; a2 < 6; ++a2) {
                int inA[6] = {0, 0, 0, 0, 0, 0};
                inA[a0] = inA[a1] = inA[a2] = 1;
                int cnt[3] = {0, 0, 0};
                for (int i = 0; i < 3; ++i) cnt[fs[i]]++;
                for (int q = 0; q < 6; ++q)
                    if (inA[q]) cnt[fsrc[q]]--;
                if (cnt[0] || cnt[1] || cnt[2]) continue;
                // representative: each flavour's quarks of a site go to that
                // site's source fields of the flavour in increasing order
                int sig[6];
                for (int s = 0; s < 2; ++s)
                    for (int f = 0; f < 3; ++f) {
                        int qs[6], nq = 0;
                        for (int q = 0; q < 6; ++q)
                            if (inA[q] == (s == 0) && fsrc[q] == f) qs[nq++] = q;
                        int k = 0;
                        for (int i = 3 * s; i < 3 * s + 3; ++i)
                            if (fs[i] == f) sig[i] = qs[k++];
                    }
                Diagram d;
                d.sign = perm_sign(sig, 6);
                d.coef = d.sign * w34;
                d.K = 1;
                for (int X = 0; X < 2; ++X) {
                    int n1 = inA[3 * X] + inA[3 * X + 1] + inA[3 * X + 2];
                    const Baryon &BX = X ? B4 : B3;
                    int cfield = 3 * X + BX.term[X ? t4 : t3].role[2];
                    d.carry[X] = inA[cfield] ? 0 : 1;
                    d.kdim[X] = 1;
                    if (n1 == 1 || n1 == 2) {
                        int lone = -1;
                        for (int q = 3 * X; q < 3 * X + 3; ++q)
                            if (inA[q] == (n1 == 1)) lone = q;
                        d.kdim[X] = rsrc[lone] == 2 ? 3 : 12;
                    }
                    d.K *= d.kdim[X];
                }
                if (index) {
                    for (int s = 0; s < 2; ++s) {
                        const Baryon &Bs = s ? B2 : B1;
                        // flavour-preserving permutations of the site's three fields
                        static const int P3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
                        for (int t = 0; t < Bs.nterm; ++t)
                            for (const auto &pi : P3) {
                                if (Bs.flav[pi[0]] != Bs.flav[0] || Bs.flav[pi[1]] != Bs.flav[1] ||
                                    Bs.flav[pi[2]] != Bs.flav[2])
                                    continue;
                                int pf[3], X[3], T[3];
                                for (int r = 0; r < 3; ++r) {
                                    int p = Bs.term[t].role[r];
                                    int q = sig[3 * s + pi[p]];
                                    pf[r] = Bs.flav[p] == FS ? 1 : 0;
                                    X[r] = q / 3;
                                    T[r] = rsrc[q];
                                }
                                BlockRef br;
                                int cpf[3], cy[3], ct[3], csrc[2], csign = 1;
                                uint32_t key = canonical(pf, X, T, spn[s], srcspin, br.ymap, cpf, cy, ct, csrc,
                                                         &csign);
                                auto it = index->find(key);
                                if (it == index->end()) {
                                    int id = (int)inters->size();
                                    inters->push_back(make_intermediate(key, cpf, cy, ct, spn[s], csrc));
                                    it = index->emplace(key, id).first;
                                }
                                br.inter = it->second;
                                br.coef = Bs.term[t].w * perm_sign(pi, 3) * csign;
                                d.blk[s].push_back(br);
                            }
                    }
                    // consistency of the open indices between the two sites: a split
                    // source baryon leaves the same open index at both sites, a full one
                    // sits at one site only, and its outer spin is carried by one site
                    for (int X = 0; X < 2; ++X)
                        for (int s = 0; s < 2; ++s)
                            for (const BlockRef &r : d.blk[s]) {
                                const Intermediate &I = (*inters)[r.inter];
                                int y = r.ymap[X];
                                int nk = y >= 0 ? I.nk[y] : 0, no = y >= 0 ? I.no[y] : 1;
                                bool ok = d.kdim[X] > 1 ? (nk == d.kdim[X]) : (nk == 0 || nk == 1);
                                ok = ok && (no == (d.carry[X] == s ? 2 : 1));
                                if (!ok) throw std::logic_error("inconsistent open indices in " + channel_name(ch));
                            }
                }
                out.push_back(std::move(d));
            }
    return out;
}

namespace {

// eps(c0, c1, c2)
int eps3(int a, int b, int c) {
    if (a == b || b == c || a == c) return 0;
    return ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) ? 1 : -1;
}

struct Part { int e[3]; int set[3]; int ph; };     // partial assignment of source indices; ph: power of i

// Source-tensor pieces of one canonical source baryon Y at the site, for fixed (o, k).
// Source tensor (Sec. 3, with the general field of Sec. 2): eps(c'_a c'_b c'_c)
// Gamma_1(mu'_a, mu'_b) Gamma_2(so + o, mu'_c); the outer spin o selects the row of Gamma_2.
std::vector<Part> y_parts(const Intermediate &I, int Y, int o, int k, int so) {
    // canonical labelling: a' is the diquark leg at the lower role, or the only one
    int ra = -1, rb = -1, rd = -1;
    for (int r = 0; r < 3; ++r) {
        if (I.role_y[r] != Y) continue;
        if (I.role_t[r] == 2) rd = r;
        else if (ra < 0) ra = r;
        else rb = r;
    }
    std::vector<Part> out;
    auto base = []() { Part p{}; p.ph = 0; for (int i = 0; i < 3; ++i) { p.e[i] = 0; p.set[i] = 0; } return p; };
    auto put = [](Part &p, int r, int e) { p.e[r] = e; p.set[r] = 1; };
    if (I.kind[Y] < 0) { out.push_back(base()); return out; }
    const SpinStruct &S = spin_struct(I.src_spin[Y]);
    int inv1[4];
    for (int m = 0; m < 4; ++m) inv1[S.p1[m]] = m;
    const int g = so + o, mc = S.p2[g], kc = S.k2[g];     // Gamma_2(g, mc) = i^kc
    switch (I.kind[Y]) {
    case Y_FULL:
        for (int c1 = 0; c1 < 3; ++c1) for (int c2 = 0; c2 < 3; ++c2) for (int c3 = 0; c3 < 3; ++c3) {
            int e = eps3(c1, c2, c3);
            if (!e) continue;
            for (int m1 = 0; m1 < 4; ++m1) {
                Part p = base();
                p.ph = (e < 0 ? 2 : 0) + S.k1[m1] + kc;
                put(p, ra, 3 * m1 + c1);
                put(p, rb, 3 * S.p1[m1] + c2);
                put(p, rd, 3 * mc + c3);
                out.push_back(p);
            }
        }
        break;
    case Y_DD:   // k = colour of the delta quark, which sits at the other site
        for (int c1 = 0; c1 < 3; ++c1) for (int c2 = 0; c2 < 3; ++c2) {
            int e = eps3(c1, c2, k);
            if (!e) continue;
            for (int m1 = 0; m1 < 4; ++m1) {
                Part p = base();
                p.ph = (e < 0 ? 2 : 0) + S.k1[m1];
                put(p, ra, 3 * m1 + c1);
                put(p, rb, 3 * S.p1[m1] + c2);
                out.push_back(p);
            }
        }
        break;
    case Y_DDELTA: {  // k = (mu_L, c_L) of the diquark partner at the other site
        const int muL = k / 3, cL = k % 3;
        for (int cD = 0; cD < 3; ++cD) for (int cd = 0; cd < 3; ++cd) {
            Part p = base();
            int e;
            if (ra >= 0) {           // local quark is a': Gamma_1(mD, mu_L)
                const int mD = inv1[muL];
                e = eps3(cD, cL, cd);
                p.ph = S.k1[mD];
                put(p, ra, 3 * mD + cD);
            } else {                 // local quark is b': Gamma_1(mu_L, mD)
                const int mD = S.p1[muL];
                e = eps3(cL, cD, cd);
                p.ph = S.k1[muL];
                put(p, rb, 3 * mD + cD);
            }
            if (!e) continue;
            p.ph += (e < 0 ? 2 : 0) + kc;
            put(p, rd, 3 * mc + cd);
            out.push_back(p);
        }
        break;
    }
    case Y_DIN: {
        Part p = base();
        put(p, ra >= 0 ? ra : rb, k);
        out.push_back(p);
        break;
    }
    case Y_DELTAIN: {
        Part p = base();
        p.ph = kc;
        put(p, rd, 3 * mc + k);
        out.push_back(p);
        break;
    }
    default:
        out.push_back(base());
    }
    return out;
}

}  // namespace

Plan build_plan(const std::vector<int> &channels, int spin_offset, const int *lower) {
    Plan P;
    P.channels = channels;
    P.spin_offset = spin_offset;
    std::map<uint32_t, int> index;
    for (int ch : channels) {
        if (!channel_valid(ch)) throw std::invalid_argument("channel index out of range or flavour not conserved");
        P.ch_begin.push_back((int)P.diags.size());
        const auto bb = channel_baryons(ch);
        for (int t3 = 0; t3 < kBaryons[bb[2]].nterm; ++t3)
            for (int t4 = 0; t4 < kBaryons[bb[3]].nterm; ++t4)
                for (auto &d : classify(ch, t3, t4, &index, &P.inters, lower)) {
                    P.iterations += d.K;
                    P.diags.push_back(std::move(d));
                }
    }
    P.ch_begin.push_back((int)P.diags.size());
    // component layout: intermediates grouped by pattern (so the block kernel
    // builds each diquark tensor once), then in registration order
    std::vector<int> order(P.inters.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return pattern_id(P.inters[a]) < pattern_id(P.inters[b]);
    });
    int off = 0;
    for (int id : order) {
        P.inters[id].offset = off;
        off += P.inters[id].ncomp;
    }
    P.ncomp = off;
    // block-kernel term lists, per component (sink spin is applied by the kernel)
    P.term_begin.assign(P.ncomp + 1, 0);
    P.comp_pat.assign(P.ncomp, 0);
    std::vector<std::vector<uint32_t>> per(P.ncomp);
    for (const auto &I : P.inters) {
        for (int o0 = 0; o0 < I.no[0]; ++o0) for (int k0 = 0; k0 < I.nk[0]; ++k0)
        for (int o1 = 0; o1 < I.no[1]; ++o1) for (int k1 = 0; k1 < I.nk[1]; ++k1) {
            int c = I.offset + o0 * I.stride_o[0] + k0 * I.stride_k[0] + o1 * I.stride_o[1] + k1 * I.stride_k[1];
            P.comp_pat[c] = pattern_id(I);
            auto p0 = y_parts(I, 0, o0, k0, spin_offset);
            auto p1 = y_parts(I, 1, o1, k1, spin_offset);
            for (const auto &a : p0) for (const auto &b : p1) {
                int e[3];
                for (int r = 0; r < 3; ++r) {
                    if (a.set[r] + b.set[r] != 1) throw std::logic_error("role not covered exactly once");
                    e[r] = a.set[r] ? a.e[r] : b.e[r];
                }
                const int ph = (a.ph + b.ph) & 3;       // coefficient i^ph: bit 13 = factor i, bit 12 = factor -1
                per[c].push_back((uint32_t)e[0] | ((uint32_t)e[1] << 4) | ((uint32_t)e[2] << 8) |
                                 ((uint32_t)(ph >> 1) << 12) | ((uint32_t)(ph & 1) << 13));
            }
        }
    }
    for (int c = 0; c < P.ncomp; ++c) {
        P.term_begin[c] = (int)P.terms.size();
        P.terms.insert(P.terms.end(), per[c].begin(), per[c].end());
    }
    P.term_begin[P.ncomp] = (int)P.terms.size();
    return P;
}

}  // namespace bbc
