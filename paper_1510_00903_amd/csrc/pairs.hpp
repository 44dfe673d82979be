// Pair form of the momentum-space contraction (Sec. 3, Eq. (LN.pLLp.FFT)).
//
// A diagram's blocks are weighted sums of block intermediates, so by
// linearity every channel is a weighted sum of products of two intermediate
// *views* (an intermediate with the assignment of the source baryons B3, B4
// to its canonical source slots), one at each sink site:
//
//   C~_ch(q)_{a b a' b'} = sum_t w_t P_{p(t)}(q)_{a b a' b'},
//   P_p(q)_{a b a' b'}   = sum_k X_p(q; a, ., k) Y_p(-q; b, ., k),
//
// k = (k3, k4) the open source indices and the outer spins a', b' carried by
// the view at the site of each source baryon's delta quark.  A pair product
// is the same for every diagram and channel that uses it, so it is computed
// once per momentum and the channels are formed from the pair products with
// the weights w = (diagram sign x source weights) x (the two sink-term
// weights); the planner's diagrams and intermediates (the blocks of Sec. 3 and
// Appendix A) fix the pairs and the weights.
//
// Host side only (no HIP types): the tables are uploaded as they are.
#pragma once

#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace bbc {

constexpr int kMaxPartners = 8;
constexpr int kMaxTileRows = 3;

// One intermediate view at one site: component offset and strides of the
// outer spins and open indices (0 where the view does not hold them).
struct PView {
    int32_t base;
    int32_t so3, so4;     // a' (source baryon B3), b' (B4)
    int32_t sk3, sk4;     // open index of B3, of B4
};

// A task: one row view and up to kMaxPartners column views sharing it, all
// of one open-index shape.  Shapes of the per-momentum product:
//   shape 0: 4 rows (sink spin, one outer spin) x 4 cols (sink spin, the other)
//   shape 1: 8 rows (sink spin, a', b') x 2 cols (sink spin), done as two
//            halves (b' = 0, 1) of 4 rows x 4 cols with two zero columns.
// row_site: 0 if the row view is at site 0 (B1, momentum q), 1 if at site 1
// (B2, momentum -q); the column views are at the other site.
struct PTask {
    int32_t K, kd4, inv;  // open-index items, extent of k4, ceil(65536 / kd4)
    int32_t shape;
    int32_t row_site;
    int32_t row_a;        // shape 0: the row view carries a' (1) or b' (0)
    int32_t np;           // partners
    int32_t cost;         // loads + products, for ordering
    PView row;
    PView col[kMaxPartners];
    int32_t pair[kMaxPartners];
    // row tiles (PairTables::tiles): up to kMaxTileRows row views of the same
    // class, each with its own products against the same columns: row 0 is `row`
    // with pair[], row r >= 1 is rowx[r - 1] with pairx[r - 1][]; a pair id is -1
    // where that row does not pair with column i.  nrow = 1 in PairTables::tasks.
    int32_t nrow;
    PView rowx[kMaxTileRows - 1];
    int32_t pairx[kMaxTileRows - 1][kMaxPartners];
};

// One channel term in pair-major order: channel ch (within its chunk) gains
// w times pair product `pair`.
struct CombEntry {
    int32_t pair;
    int32_t ch;
    double w;
};
constexpr int kCombChunk = 64;        // channels per pass of the channel sums
constexpr int kCombSubs = 8;          // channel classes (ch mod 8) per pass

struct PairTables {
    std::vector<PTask> tasks;         // most expensive first
    // the same products as tiles of up to kMaxTileRows row views sharing up to
    // kMaxPartners (shape 1: kMaxPartners / 2) column views, rows of a class
    // grouped greedily by common partners, so that a column view is loaded once
    // for all rows of its tile
    std::vector<PTask> tiles;
    int npair = 0;
    std::vector<int32_t> term_begin;  // per requested channel, n_ch + 1 entries
    std::vector<int32_t> term_pair;
    std::vector<double> term_w;
    // the same terms per chunk of kCombChunk channels and per class ch mod kCombSubs,
    // each class sorted by pair: entries [comb_begin[c * kCombSubs + k], comb_begin[... + 1])
    std::vector<CombEntry> comb;
    std::vector<int32_t> comb_begin;
    int64_t pair_items = 0;           // sum over pairs of K
};

// Pairs, tasks and channel terms of a plan (throws std::logic_error on a
// shape the kernels do not take); row tiles of at most tile_rows rows and
// tile_cols columns (shape 1: half as many, rounded down).
PairTables build_pair_tables(const Plan &P, int tile_rows = kMaxTileRows, int tile_cols = kMaxPartners);

}  // namespace bbc
