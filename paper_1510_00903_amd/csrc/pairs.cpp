// Pair tables of the momentum-space contraction (see pairs.hpp).
// Paper: arXiv:1510.00903, Sec. 3 (effective blocks, Eq. (LN.pLLp.FFT)),
// Tables 1-4 (the diagrams and their open-index sums).
#include "pairs.hpp"

#include <algorithm>
#include <map>
#include <stdexcept>
#include <tuple>

namespace bbc {

namespace {

// View of intermediate `inter` with source baryons B3, B4 in canonical slots
// ymap[0], ymap[1] (-1: not at this site).
PView make_view(const Plan &P, const BlockRef &r) {
    const Intermediate &I = P.inters[r.inter];
    PView v{};
    v.base = I.offset;
    int so[2] = {0, 0}, sk[2] = {0, 0};
    for (int X = 0; X < 2; ++X) {
        const int y = r.ymap[X];
        if (y < 0) continue;
        if (I.no[y] == 2) so[X] = I.stride_o[y];
        if (I.nk[y] > 1) sk[X] = I.stride_k[y];
    }
    v.so3 = so[0]; v.so4 = so[1]; v.sk3 = sk[0]; v.sk4 = sk[1];
    return v;
}

using ViewKey = std::tuple<int, int, int>;                    // intermediate, ymap of B3, of B4
using PairKey = std::tuple<ViewKey, ViewKey, int, int, int, int>;   // views at sites 0, 1; kdims; carries

struct PairInfo {
    ViewKey v[2];
    PView pv[2];
    int kd3, kd4, carry3, carry4;
};

}  // namespace

PairTables build_pair_tables(const Plan &P, int tile_rows, int tile_cols) {
    if (tile_rows < 1 || tile_rows > kMaxTileRows) throw std::logic_error("tile rows");
    if (tile_cols < 2 || tile_cols > kMaxPartners) throw std::logic_error("tile columns");
    PairTables T;
    const int n = (int)P.channels.size();
    std::map<PairKey, int> pair_index;
    std::vector<PairInfo> pairs;
    std::vector<std::map<int, double>> ch_terms(n);
    for (int m = 0; m < n; ++m) {
        for (int d = P.ch_begin[m]; d < P.ch_begin[m + 1]; ++d) {
            const Diagram &D = P.diags[d];
            if (D.K > 255 || D.kdim[1] > 15) throw std::logic_error("open-index range");
            for (const BlockRef &r0 : D.blk[0])
                for (const BlockRef &r1 : D.blk[1]) {
                    const ViewKey k0{r0.inter, r0.ymap[0], r0.ymap[1]}, k1{r1.inter, r1.ymap[0], r1.ymap[1]};
                    const PairKey key{k0, k1, D.kdim[0], D.kdim[1], D.carry[0], D.carry[1]};
                    auto it = pair_index.find(key);
                    int p;
                    if (it == pair_index.end()) {
                        p = (int)pairs.size();
                        pair_index.emplace(key, p);
                        PairInfo pi;
                        pi.v[0] = k0; pi.v[1] = k1;
                        pi.pv[0] = make_view(P, r0); pi.pv[1] = make_view(P, r1);
                        pi.kd3 = D.kdim[0]; pi.kd4 = D.kdim[1];
                        pi.carry3 = D.carry[0]; pi.carry4 = D.carry[1];
                        pairs.push_back(pi);
                        T.pair_items += D.K;
                    } else {
                        p = it->second;
                    }
                    ch_terms[m][p] += D.coef * r0.coef * r1.coef;
                }
        }
    }
    // every component a kernel reads lies inside the component space
    for (const PairInfo &pi : pairs)
        for (int s = 0; s < 2; ++s) {
            const PView &v = pi.pv[s];
            const long top = (long)v.base + v.so3 + v.so4 + (long)(pi.kd3 - 1) * v.sk3 + (long)(pi.kd4 - 1) * v.sk4;
            if (v.base < 0 || top >= P.ncomp) throw std::logic_error("pair view outside the component space");
        }
    T.npair = (int)pairs.size();
    T.term_begin.assign(n + 1, 0);
    for (int m = 0; m < n; ++m) {
        T.term_begin[m] = (int)T.term_pair.size();
        for (const auto &kv : ch_terms[m]) {
            if (kv.second == 0.0) continue;
            T.term_pair.push_back(kv.first);
            T.term_w.push_back(kv.second);
        }
    }
    T.term_begin[n] = (int)T.term_pair.size();
    // pair-major form: per chunk of channels and class ch mod kCombSubs, by pair
    // (within a channel the terms keep their ascending pair order)
    const int nchunk = (n + kCombChunk - 1) / kCombChunk;
    T.comb_begin.assign((size_t)nchunk * kCombSubs + 1, 0);
    for (int c = 0; c < nchunk; ++c)
        for (int k = 0; k < kCombSubs; ++k) {
            std::vector<CombEntry> e;
            for (int m = c * kCombChunk + k; m < std::min(n, (c + 1) * kCombChunk); m += kCombSubs)
                for (int t = T.term_begin[m]; t < T.term_begin[m + 1]; ++t)
                    e.push_back(CombEntry{T.term_pair[t], m - c * kCombChunk, T.term_w[t]});
            std::stable_sort(e.begin(), e.end(), [](const CombEntry &a, const CombEntry &b) { return a.pair < b.pair; });
            T.comb_begin[(size_t)c * kCombSubs + k] = (int)T.comb.size();
            T.comb.insert(T.comb.end(), e.begin(), e.end());
        }
    T.comb_begin[(size_t)nchunk * kCombSubs] = (int)T.comb.size();

    // Tasks.  The row view is the one holding both outer spins (shape 1), else
    // (shape 0) the side whose views are fewer within the pair's class, so that
    // a row view has more partners to share its loads with.
    using ClassKey = std::tuple<int, int, int, int>;             // kd3, kd4, carry3, carry4
    std::map<ClassKey, std::pair<std::map<ViewKey, int>, std::map<ViewKey, int>>> views_of_class;
    for (const PairInfo &pi : pairs) {
        auto &vc = views_of_class[ClassKey{pi.kd3, pi.kd4, pi.carry3, pi.carry4}];
        vc.first[pi.v[0]]++;
        vc.second[pi.v[1]]++;
    }
    // (row site, class, row view) -> pairs
    std::map<std::tuple<int, ClassKey, ViewKey>, std::vector<int>> rows;
    for (int p = 0; p < T.npair; ++p) {
        const PairInfo &pi = pairs[p];
        const ClassKey ck{pi.kd3, pi.kd4, pi.carry3, pi.carry4};
        int rs;
        if (pi.carry3 == pi.carry4) {
            rs = pi.carry3;                                   // the site holding both outer spins
        } else {
            const auto &vc = views_of_class[ck];
            rs = vc.second.size() < vc.first.size() ? 1 : 0;
        }
        rows[std::make_tuple(rs, ck, pi.v[rs])].push_back(p);
    }
    for (const auto &kv : rows) {
        const int rs = std::get<0>(kv.first);
        const std::vector<int> &ps = kv.second;
        const PairInfo &p0 = pairs[ps[0]];
        const int shape = p0.carry3 == p0.carry4 ? 1 : 0;
        const int maxp = shape == 0 ? kMaxPartners : kMaxPartners / 2;
        for (size_t b = 0; b < ps.size(); b += maxp) {
            PTask t{};
            t.K = p0.kd3 * p0.kd4;
            t.kd4 = p0.kd4;
            t.inv = (65536 + p0.kd4 - 1) / p0.kd4;
            for (int kk = 0; kk < t.K; ++kk)
                if (((kk * t.inv) >> 16) != kk / t.kd4) throw std::logic_error("open-index reciprocal");
            t.shape = shape;
            t.row_site = rs;
            // shape 0: which outer spin the row view carries (a' sits at site carry3)
            t.row_a = shape == 0 ? (p0.carry3 == rs ? 1 : 0) : 0;
            t.row = p0.pv[rs];
            t.np = (int)std::min<size_t>(maxp, ps.size() - b);
            for (int i = 0; i < t.np; ++i) {
                const PairInfo &pi = pairs[ps[b + i]];
                t.col[i] = pi.pv[1 - rs];
                t.pair[i] = ps[b + i];
            }
            const int steps = (t.K + 3) / 4;
            const int halves = shape == 1 ? 2 : 1;
            t.cost = steps * (2 * halves + t.np * (2 + 8 * halves));
            t.nrow = 1;
            for (int r = 0; r < kMaxTileRows - 1; ++r)
                for (int i = 0; i < kMaxPartners; ++i) t.pairx[r][i] = -1;
            T.tasks.push_back(t);
        }
    }
    std::stable_sort(T.tasks.begin(), T.tasks.end(), [](const PTask &a, const PTask &b) { return a.cost > b.cost; });

    // Row tiles.  Per (row site, class): each row view in turn (in key order)
    // starts a tile, and the not yet taken row view sharing most column views
    // with the tile's columns so far (at least two) joins it, up to kMaxTileRows
    // rows; the union of their columns, in key order, is cut into tiles of maxp
    // columns.
    std::map<std::pair<int, ClassKey>, std::vector<ViewKey>> rows_of_class;
    for (const auto &kv : rows) rows_of_class[{std::get<0>(kv.first), std::get<1>(kv.first)}].push_back(std::get<2>(kv.first));
    for (const auto &rc : rows_of_class) {
        const int rs = rc.first.first;
        const ClassKey &ck = rc.first.second;
        const std::vector<ViewKey> &rv = rc.second;
        // column view -> pair, per row view
        std::vector<std::map<ViewKey, int>> nb(rv.size());
        for (size_t i = 0; i < rv.size(); ++i)
            for (int p : rows.at(std::make_tuple(rs, ck, rv[i]))) nb[i][pairs[p].v[1 - rs]] = p;
        std::vector<bool> taken(rv.size(), false);
        for (size_t i = 0; i < rv.size(); ++i) {
            if (taken[i]) continue;
            taken[i] = true;
            std::vector<int> members{(int)i};
            std::map<ViewKey, std::vector<int>> cols;              // column -> pair per member row
            for (const auto &kv : nb[i]) cols[kv.first] = {kv.second};
            while ((int)members.size() < tile_rows) {
                int best = -1;
                size_t bc = 0;
                for (size_t j = i + 1; j < rv.size(); ++j) {
                    if (taken[j]) continue;
                    size_t c = 0;
                    for (const auto &kv : nb[j]) c += cols.count(kv.first);
                    if (c > bc) { best = (int)j; bc = c; }
                }
                if (best < 0 || bc < 2) break;
                taken[best] = true;
                const int m = (int)members.size();
                members.push_back(best);
                for (auto &kv : cols) kv.second.resize(m + 1, -1);
                for (const auto &kv : nb[best]) {
                    auto it = cols.find(kv.first);
                    if (it == cols.end()) { cols[kv.first] = std::vector<int>(m + 1, -1); it = cols.find(kv.first); }
                    it->second[m] = kv.second;
                }
            }
            const int nr = (int)members.size();
            for (auto &kv : cols) kv.second.resize(nr, -1);
            const PairInfo &p0 = pairs[nb[i].begin()->second];
            const int shape = p0.carry3 == p0.carry4 ? 1 : 0;
            const int maxp = shape == 0 ? tile_cols : tile_cols / 2;
            std::vector<std::vector<int>> cl;
            for (const auto &kv : cols) cl.push_back(kv.second);
            for (size_t b = 0; b < cl.size(); b += maxp) {
                PTask t{};
                t.K = p0.kd3 * p0.kd4;
                t.kd4 = p0.kd4;
                t.inv = (65536 + p0.kd4 - 1) / p0.kd4;
                t.shape = shape;
                t.row_site = rs;
                t.row_a = shape == 0 ? (p0.carry3 == rs ? 1 : 0) : 0;
                t.row = p0.pv[rs];
                t.nrow = nr;
                for (int r = 1; r < nr; ++r) t.rowx[r - 1] = pairs[nb[members[r]].begin()->second].pv[rs];
                t.np = (int)std::min<size_t>(maxp, cl.size() - b);
                for (int k = 0; k < kMaxPartners; ++k) {
                    t.pair[k] = -1;
                    for (int r = 0; r < kMaxTileRows - 1; ++r) t.pairx[r][k] = -1;
                }
                int nprod = 0;
                for (int k = 0; k < t.np; ++k) {
                    const std::vector<int> &pc = cl[b + k];
                    int any = -1;
                    for (int r = 0; r < nr; ++r) {
                        if (pc[r] >= 0) { any = pc[r]; ++nprod; }
                        if (r == 0) t.pair[k] = pc[0];
                        else t.pairx[r - 1][k] = pc[r];
                    }
                    t.col[k] = pairs[any].pv[1 - rs];
                }
                const int steps = (t.K + 3) / 4;
                const int halves = shape == 1 ? 2 : 1;
                t.cost = steps * (2 * halves * t.nrow + t.np * 2 + nprod * 8 * halves);
                T.tiles.push_back(t);
            }
        }
    }
    std::stable_sort(T.tiles.begin(), T.tiles.end(), [](const PTask &a, const PTask &b) { return a.cost > b.cost; });
    // every pair exactly once in the tiles
    std::vector<int> seen(T.npair, 0);
    for (const PTask &t : T.tiles)
        for (int k = 0; k < t.np; ++k) {
            if (t.pair[k] >= 0) seen[t.pair[k]]++;
            for (int r = 0; r + 1 < t.nrow; ++r)
                if (t.pairx[r][k] >= 0) seen[t.pairx[r][k]]++;
        }
    for (int p = 0; p < T.npair; ++p)
        if (seen[p] != 1) throw std::logic_error("row tiles do not cover every pair once");
    return T;
}

}  // namespace bbc
