// Host planner of the effective block algorithm: baryon operators, diagram
// classification, block intermediates and the tables the GPU kernels read.
//
// Paper: H. Nemura, arXiv:1510.00903.  Sec. 2 (interpolating fields),
// Sec. 3 (Wick contraction, effective blocks, FFT correlation), Sec. 4 (the 52
// channels, Tables 1-4), Appendix A (reusable blocks).
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace bbc {

enum : int { FU = 0, FD = 1, FS = 2 };

// Spin structure {Gamma_1, Gamma_2} of a field B = eps((q1 Gamma_1 q2) Gamma_2 q3)
// (Sec. 2, Eq. (FieldOperator_B)).  Every structure used is monomial in the Dirac
// representation: Gamma_1(mu, p1[mu]) = i^k1[mu] and Gamma_2(g, p2[g]) = i^k2[g], all
// other entries zero.  x is the sign of the tensor eps Gamma_1 under exchanging its
// first two legs (-1 times the transpose symmetry of Gamma_1).
struct SpinStruct {
    int p1[4], k1[4], p2[4], k2[4];
    int x;
};
enum : int {
    SP_OCTET = 0,    // {C gamma_5, 1}: the octet fields of Sec. 2
    SP_CHI2 = 1,     // {C, gamma_5}: the other nucleon field
    SP_DEC1 = 2,     // {C gamma_l, 1}, l = 1, 2, 3: decuplet fields (Sec. 4 footnote)
    kNumSpinStructs = 5,
    // structure s + kNumSpinStructs is s with the rows of Gamma_2 moved up by two
    // (Gamma_2'(g, .) = Gamma_2(g + 2 mod 4, .)): its spin components 0, 1 are the
    // components 2, 3 of s, so one baryon of a channel can take its lower pair
    // while the others take the upper one (all 256 spin components, Sec. 6 uses
    // the lower pair backward in time)
    kNumSpinStructsAll = 2 * kNumSpinStructs
};
const SpinStruct &spin_struct(int s);

// One term of a baryon field: weight and, for each tensor role r in {a, b, c}
// (eps(c_a c_b c_c) Gamma_1(mu_a, mu_b) Gamma_2(gamma, mu_c)), the position of
// the quark field that plays it in the baryon's fixed field order.
struct BaryonTerm {
    double w;
    int role[3];
    const char *name;
};

struct Baryon {
    const char *name;
    int flav[3];      // flavour of the quark fields in Grassmann order
    int nterm;
    BaryonTerm term[3];
    int spin;         // spin structure (SP_*)
};

constexpr int kNumChannels = 52;
constexpr int kNumChannelsAll = 56;
// Other charge states: ids from kChannelExtBase name any quadruple of the 8
// octet fields, id = kChannelExtBase + ((b1 * 8 + b2) * 8 + b3) * 8 + b4.
// Fields with other spin structures (ids 8..39: p2, n2 with {C, gamma_5}; the
// decuplet Delta++, Delta-, Omega-, Delta+, Delta0, Sigma*+, Sigma*0, Sigma*-,
// Xi*0, Xi*- with {C gamma_l, 1}, l = 1..3) enter through ids from kChannelGenBase:
// id = kChannelGenBase + ((b1 * 40 + b2) * 40 + b3) * 40 + b4 for quadruples holding
// at least one of them.
constexpr int kNumOctet = 8;
constexpr int kNumBaryons = 40;
constexpr int kChannelExtBase = kNumChannelsAll;
constexpr int kChannelGenBase = kChannelExtBase + kNumOctet * kNumOctet * kNumOctet * kNumOctet;
constexpr int kNumChannelIds = kChannelGenBase + kNumBaryons * kNumBaryons * kNumBaryons * kNumBaryons;

const Baryon &baryon(int id);
std::array<int, 4> channel_baryons(int ch);  // 4 baryon ids: sink B1, B2, source B3, B4
std::string channel_name(int ch);
// In range, and the sink and source hold the same number of u, d and s quarks.
bool channel_valid(int ch);
// Id of a baryon quadruple: its index in the channel list if listed, else the extended id.
int channel_id(const int b[4]);

// Kinds of what one source baryon leaves at one sink site.
enum YKind : int { Y_FULL = 0, Y_DD = 1, Y_DDELTA = 2, Y_DIN = 3, Y_DELTAIN = 4 };

// A block intermediate: the sink tensor of one baryon term contracted with three
// propagators and with the parts of the source tensors that close on that site.
// Indices: sink spin g (2), then per source baryon Y present (canonical order):
// outer spin o_Y (no = 1 or 2) and open index k_Y (nk = 1, 3 or 12).
struct Intermediate {
    uint32_t key;
    int pflav[3];     // per role a, b, c: 0 light, 1 strange
    int role_y[3];    // per role: canonical source baryon 0/1
    int role_t[3];    // per role: 0 = source diquark leg, 2 = delta quark c'; of two diquark legs
                      // the one at the lower role is a' (canonical labelling, see canonical())
    int sink_spin;    // spin structure of the sink field
    int src_spin[2];  // spin structure of canonical source baryon Y (-1 if absent)
    int ny;
    int kind[2], no[2], nk[2];
    int ncomp;        // components per sink spin
    int offset;       // offset of component 0 in the per-spin component space
    int stride_o[2], stride_k[2];
};

struct BlockRef {
    int inter;
    double coef;      // sink-term weight times sign of the in-site exchange
    int ymap[2];      // canonical Y of source baryon B3 / B4 at this site, -1 if absent
};

struct Diagram {
    int K;            // open-index iterations (kdim3 * kdim4)
    int sign;         // parity of the representative permutation
    int kdim[2];      // open-index dimension contributed by B3 / B4 (1, 3, 12)
    int carry[2];     // site (0: B1 at X+r, 1: B2 at X) holding the outer spin of B3 / B4
    double coef;      // sign * w3 * w4
    std::vector<BlockRef> blk[2];
};

struct Plan {
    std::vector<int> channels;               // requested channel list
    int spin_offset = 0;                     // 0 upper, 2 lower components
    std::vector<Intermediate> inters;
    int ncomp = 0;                           // components per sink spin, all intermediates
    std::vector<Diagram> diags;
    std::vector<int> ch_begin;               // per requested channel: first diagram (size n+1)
    // block-kernel tables
    std::vector<uint32_t> terms;             // packed (e_a, e_b, e_c, sign)
    std::vector<int32_t> term_begin;         // per component (size ncomp+1)
    std::vector<int32_t> comp_pat;           // per component: pattern id (pattern_id)
    int64_t iterations = 0;                  // sum of K over diagrams
};

// Diagrams of one channel and source-term pair; intermediates are registered in
// `index`/`inters` (pass nullptrs to only classify).
// `lower` (optional, per baryon B1..B4): 1 takes that baryon's lower spin pair
// through its shifted structure (see kNumSpinStructsAll).
std::vector<Diagram> classify(int ch, int t3, int t4, std::map<uint32_t, int> *index,
                              std::vector<Intermediate> *inters, const int *lower = nullptr);

// spin_offset 0 (upper pair of every baryon) or 2 (lower pair of every baryon);
// with `lower`, spin_offset is 0 and each baryon's pair is chosen on its own.
Plan build_plan(const std::vector<int> &channels, int spin_offset, const int *lower = nullptr);

// Pattern of an intermediate: what the block kernel builds once for all its
// components -- the sink spin structure, the flavours of the two diquark roles
// (the diquark tensor) and of the third role.
constexpr int kNumPatterns = kNumSpinStructsAll * 8;
inline int pattern_id(const Intermediate &I) {
    return ((I.sink_spin * 2 + I.pflav[0]) * 2 + I.pflav[1]) * 2 + I.pflav[2];
}

}  // namespace bbc
