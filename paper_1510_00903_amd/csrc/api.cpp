// C ABI of the MI355X effective-block correlator (include/bbcorr.h).
//
// The driver owns a plan cache (per channel list and spin selection), the
// device copies of the planner tables and a workspace that grows on demand
// within the context's HBM budget.  Each time slice runs the kernel sequence
// of kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <thread>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bbcorr.h"
#include "kernels.hpp"
#include "pairs.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

bbc_status fail(bbc_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                                       \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) return fail(BBC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DevPlan {
    bbc::Plan plan;
    bbc::BlockPatterns pats;
    int ntask = 0, npair = 0, ntile = 0;
    // every table the kernels read, as one image (byte offsets below): block-kernel
    // component records and terms (kernels.hpp, BlockComp), pair tasks and channel
    // terms (pairs.hpp), per-channel quark content
    std::vector<unsigned char> image;
    size_t off_terms = 0, off_comps = 0, off_tasks = 0, off_tiles = 0, off_comb = 0, off_comb_begin = 0,
           off_content = 0;
    void *d_image = nullptr;        // device copy, made by the entry points that allocate
    size_t table_bytes = 0;
    // request key: channel list, spin offset, precision, and a hash of the list
    std::vector<int> chans;
    int spin_offset = 0, prec = 0;
    uint64_t chash = 0;
    // all-components request: which of the 16 upper/lower choices (bit i: baryon
    // B(i+1) takes its lower pair) this plan evaluates, else -1
    int full_sub = -1;
    ~DevPlan() { (void)hipFree(d_image); }
};

// FNV-1a over the channel list (identifies a channel set in the tuning table).
uint64_t channel_hash(const std::vector<int> &chans) {
    uint64_t h = 1469598103934665603ull;
    for (int c : chans)
        for (int b = 0; b < 4; ++b) {
            h ^= (uint64_t)((c >> (8 * b)) & 255);
            h *= 1099511628211ull;
        }
    return h;
}

// Device pointers of one plan's tables, for an image copied to `base`.
struct PlanDev {
    const DevPlan *dp;
    const uint32_t *terms;
    const bbc::BlockComp *comps;
    const bbc::PTask *tasks;
    const bbc::PTask *tiles;
    const bbc::CombEntry *comb;
    const int32_t *comb_begin;
    const int2 *content;
};
PlanDev plan_dev(const DevPlan *dp, const void *base) {
    const char *b = (const char *)base;
    return PlanDev{dp, (const uint32_t *)(b + dp->off_terms), (const bbc::BlockComp *)(b + dp->off_comps),
                   (const bbc::PTask *)(b + dp->off_tasks), (const bbc::PTask *)(b + dp->off_tiles),
                   (const bbc::CombEntry *)(b + dp->off_comb), (const int32_t *)(b + dp->off_comb_begin),
                   (const int2 *)(b + dp->off_content)};
}

// Number of self-conjugate momenta (q = -q mod L): 0 and L/2 along each even axis.
long self_conjugate(const int L[3]) {
    long s = 1;
    for (int d = 0; d < 3; ++d) s *= (L[d] % 2 == 0) ? 2 : 1;
    return s;
}

// Positions of the momentum-grouped copy: V momenta, one padding slot when the
// number of self-conjugate momenta is odd, rounded up to whole groups of G.
long grouped_positions(long V, const int L[3], int G) {
    const long n = V + (self_conjugate(L) & 1);
    return (n + G - 1) / G * G;
}

// Lattices whose momentum groups come in x-row runs (square 24-, 32- and
// 96-point planes: the forward FFT's last pass writes whole runs).
bool run_ordered(const int L[3]) { return L[0] == L[1] && (L[0] == 24 || L[0] == 32 || L[0] == 96); }

// Momentum groups of G positions, each closed under q -> -q.  Entry p: (momentum
// at position p, or -1 for padding; the lane within the group that holds -q).
//
// Default order: the self-conjugate momenta first, one padding slot if their
// number is odd, then the pairs (q, -q) in increasing q (a pair starts at an
// even position, so never straddles two groups), the last group padded.
//
// Run order (run_ordered lattices; Lx a multiple of 8, Ly even): for each x-row
// r = (ky, kz) whose mirror row m = (-ky, -kz) is not smaller, one run of whole
// groups: r != m: the pairs ((kx, r), (-kx, m)) for kx = 0 .. Lx-1 (2 Lx
// positions); r == m: (0, r) and (Lx/2, r) (self-conjugate), then the pairs
// ((kx, r), (-kx, r)) for kx = 1 .. Lx/2-1 (Lx positions).  xrun (optional)
// receives, for every x-row, the first group of the run that holds it.
std::vector<int2> momentum_groups(const int L[3], int G, std::vector<int> *xrun = nullptr) {
    const int V = L[0] * L[1] * L[2];
    auto neg = [&](int q) {
        const int qx = q % L[0], qy = (q / L[0]) % L[1], qz = q / (L[0] * L[1]);
        return ((L[0] - qx) % L[0]) + L[0] * (((L[1] - qy) % L[1]) + L[1] * ((L[2] - qz) % L[2]));
    };
    std::vector<int2> pos;
    auto lane = [&]() { return (int)(pos.size() % G); };
    if (run_ordered(L)) {
        const int Lx = L[0], Ly = L[1], Lz = L[2], nrow = Ly * Lz;
        auto mrow = [&](int r) { return (Ly - r % Ly) % Ly + Ly * ((Lz - r / Ly) % Lz); };
        if (xrun) xrun->assign(nrow, -1);
        for (int r = 0; r < nrow; ++r) {
            const int m = mrow(r);
            if (m < r) continue;
            if (pos.size() % G) throw std::logic_error("x-row run not aligned to a group");
            if (xrun) (*xrun)[r] = (*xrun)[m] = (int)(pos.size() / G);
            const int b = Lx * r, mb = Lx * m;
            if (m == r) {
                pos.push_back(make_int2(b, lane()));
                pos.push_back(make_int2(b + Lx / 2, lane()));
                for (int kx = 1; kx < Lx / 2; ++kx) {
                    const int l = lane();
                    pos.push_back(make_int2(b + kx, l + 1));
                    pos.push_back(make_int2(b + Lx - kx, l));
                }
            } else {
                for (int kx = 0; kx < Lx; ++kx) {
                    const int l = lane();
                    pos.push_back(make_int2(b + kx, l + 1));
                    pos.push_back(make_int2(mb + (Lx - kx) % Lx, l));
                }
            }
        }
        if ((long)pos.size() != V) throw std::logic_error("x-row runs do not cover the lattice");
        return pos;
    }
    for (int q = 0; q < V; ++q)
        if (neg(q) == q) pos.push_back(make_int2(q, lane()));
    if (pos.size() & 1) pos.push_back(make_int2(-1, lane()));
    for (int q = 0; q < V; ++q) {
        const int m = neg(q);
        if (m <= q) continue;
        const int l = lane();
        pos.push_back(make_int2(q, l + 1));
        pos.push_back(make_int2(m, l));
    }
    while (pos.size() % G) pos.push_back(make_int2(-1, lane()));
    return pos;
}

template <typename E>
hipError_t upload_vec(E **dst, const std::vector<E> &src) {
    size_t bytes = std::max<size_t>(sizeof(E), src.size() * sizeof(E));
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(E), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

namespace {
enum JobState { JOB_QUEUED = 0, JOB_RUNNING = 1, JOB_DONE = 2, JOB_CANCELLED = 3, JOB_FAILED = 4 };
using Clock = std::chrono::steady_clock;

// A propagator set resident in HBM (serving): n_t slices of both flavours.
struct PropSet {
    int L[3];
    int prec;
    int n_t;
    void *dl = nullptr, *ds = nullptr;
    size_t bytes = 0;
    int refs = 0;            // queued or running jobs using it
    bool released = false;
};

struct Job {
    uint64_t id = 0;
    PropSet *ps = nullptr;
    std::vector<int> slice, tl;
    int t0 = 0;
    std::vector<int> chans;
    int spin = 0;
    std::vector<double> energy;
    void *out = nullptr;
    double *scale = nullptr;
    DevPlan *dp = nullptr;
    size_t foot = 0;
    int state = JOB_QUEUED;
    bbc_status status = BBC_OK;
    std::string err;
    bool cancel = false;
    int next = 0, inflight = 0;
    int bypassed = 0;        // times a later job was admitted while this one waited at the head
    Clock::time_point t_submit, t_start, t_done;
};

struct Slot {
    hipStream_t st = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    Job *job = nullptr;
    bool reserved = false;        // held for a job whose workspace is being allocated
    std::deque<hipEvent_t> evs;   // one completion event per enqueued slice
    // graph replay: the slot's device copy of the current slice's arguments, and
    // one captured slice per request shape on this slot's workspace
    bbc::SliceArgs *d_args = nullptr;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    void clear_graphs() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
};

struct Server {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool running = false, stop = false;
    std::deque<Job *> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::map<uint64_t, std::unique_ptr<PropSet>> props;
    std::vector<Slot> slots;
    std::vector<hipEvent_t> evpool;
    hipStream_t cap = nullptr;    // capture stream of the slot graphs
    uint64_t next_id = 1;
    size_t committed = 0;         // resident propagators + slot workspaces
};
}  // namespace

struct bbc_context {
    int device = 0;
    Server srv;
    uint64_t budget = 0;
    std::mutex mu;
    std::map<std::pair<std::vector<int>, int>, std::unique_ptr<DevPlan>> plans;   // key: (channels, 2 spin_offset + FP32)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double *d_energy = nullptr;
    int energy_cap = 0;
    std::map<std::vector<int>, int2 *> groups;       // per (lattice, G): momentum groups
    // allocation-free entry point: this device's copy of the scratch array, and
    // host images of the momentum groups per lattice
    void *scratch = nullptr;
    std::map<std::vector<int>, std::pair<std::vector<int2>, long>> group_images;
    std::vector<double> noalloc_energy;
    std::mutex qmu;                                   // guards groups and plans for the server thread
    hipStream_t cin = nullptr, cout = nullptr;        // copy streams of the host-streamed direct path
    // direct calls share the workspace and the energy array: each call's stream
    // waits for the previous call's work (recorded on `last`), whatever streams
    // the callers use
    hipEvent_t last = nullptr;
    bool last_valid = false;
    hipEvent_t sev[8] = {};
    // graph mode: the kernel sequence of a device-resident job captured once per
    // argument tuple on gs, then replayed on the caller's stream
    std::atomic<bool> graph_mode{false};     // read by the serving thread too
    hipStream_t gs = nullptr;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    // kernel variants per request shape (lattice, precision, spin offset, channel
    // hash), set by bbc_tuning_set / bbc_autotune / a tuning file; tune_path: the
    // file bbc_autotune rewrites (from BBC_TUNING_CACHE)
    std::mutex tmu;
    std::map<std::array<uint64_t, 6>, bbc::Tuning> tuning;
    std::string tune_path;
    // concurrent time slices of one direct call: streams forked from and joined
    // back into the caller's stream (bev[0] fork, bev[1 + b] join of stream b)
    hipStream_t bstreams[bbc::kMaxSliceStreams] = {};
    hipEvent_t bev[bbc::kMaxSliceStreams + 1] = {};
    void clear_graphs() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    // profiling: event pairs recorded around kernel stages
    bool prof = false;
    struct Rec { int stage, nk; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t event() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) { e = pool.back(); pool.pop_back(); return e; }
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~bbc_context() {
        if (ws) (void)hipFree(ws);
        if (d_energy) (void)hipFree(d_energy);
        for (auto &kv : groups) (void)hipFree(kv.second);
        if (cin) (void)hipStreamDestroy(cin);
        if (cout) (void)hipStreamDestroy(cout);
        clear_graphs();
        if (gs) (void)hipStreamDestroy(gs);
        for (auto s : bstreams) if (s) (void)hipStreamDestroy(s);
        for (auto e : bev) if (e) (void)hipEventDestroy(e);
        for (auto e : sev) if (e) (void)hipEventDestroy(e);
        if (last) (void)hipEventDestroy(last);
        for (auto &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

namespace {
// Records an event pair around one kernel stage when profiling is on (ctx may be null).
struct StageTimer {
    bbc_context *ctx; hipStream_t st; int stage; hipEvent_t a = nullptr;
    int nk = 1;                      // kernels launched inside the stage
    StageTimer(bbc_context *c, hipStream_t s, int g) : ctx(c), st(s), stage(g) {
        if (ctx && ctx->prof && (a = ctx->event())) (void)hipEventRecord(a, st);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = ctx->event();
        if (!b) { ctx->pool.push_back(a); return; }
        (void)hipEventRecord(b, st);
        ctx->recs.push_back({stage, nk, a, b});
    }
};
}  // namespace

namespace {

// Orders a direct call after the previous one on the context (called with ctx->mu held).
bbc_status order_after_last(bbc_context *ctx, hipStream_t st) {
    if (!ctx->last) HIP_TRY(hipEventCreateWithFlags(&ctx->last, hipEventDisableTiming));
    if (ctx->last_valid) HIP_TRY(hipStreamWaitEvent(st, ctx->last, 0));
    return BBC_OK;
}
bbc_status mark_last(bbc_context *ctx, hipStream_t st, bbc_status s) {
    if (hipEventRecord(ctx->last, st) == hipSuccess) ctx->last_valid = true;
    return s;
}

// Appends `n` elements at a 256-byte boundary of the image; returns their offset.
template <typename E>
size_t image_put(std::vector<unsigned char> &img, const E *data, size_t n) {
    const size_t off = (img.size() + 255) & ~(size_t)255;
    img.resize(off + std::max<size_t>(1, n) * sizeof(E), 0);
    if (n) std::memcpy(img.data() + off, data, n * sizeof(E));
    return off;
}

// Plan of a channel list and spin selection (cached per context).  With
// `upload`, the table image is also copied to a device allocation of its own;
// the allocation-free entry point copies it into its scratch instead.
// Row tiles of the contraction: rows and columns (shape 1: half the columns) per
// tile, the shapes the tile kernels are instantiated for.
constexpr int kTileRows = 3, kTileCols = 4;

bbc_status get_plan(bbc_context *ctx, const std::vector<int> &chans, int spin_offset, bbc_precision prec,
                    DevPlan **out, bool upload = true, int full_sub = -1) {
    std::lock_guard<std::mutex> lock(ctx->qmu);
    auto key = std::make_pair(chans, spin_offset * 2 + (prec == BBC_F32 ? 1 : 0) + 8 * (full_sub + 1));
    auto it = ctx->plans.find(key);
    if (it == ctx->plans.end()) {
        std::unique_ptr<DevPlan> dp(new DevPlan);
        try {
            int lower[4];
            for (int i = 0; i < 4; ++i) lower[i] = (full_sub >> i) & 1;
            dp->plan = full_sub >= 0 ? bbc::build_plan(chans, 0, lower) : bbc::build_plan(chans, spin_offset);
        } catch (const std::exception &e) {
            return fail(BBC_EINVAL, std::string("planner: ") + e.what());
        }
        dp->full_sub = full_sub;
        dp->chans = chans;
        dp->spin_offset = spin_offset;
        dp->prec = (int)prec;
        dp->chash = channel_hash(chans);
        const bbc::Plan &P = dp->plan;
        // pattern runs of the component layout (components are sorted by pattern id)
        dp->pats.n = 0;
        dp->pats.any_imag = 0;
        for (uint32_t code : P.terms) dp->pats.any_imag |= (int)((code >> 13) & 1);
        for (int c = 0; c < P.ncomp;) {
            const int id = P.comp_pat[c];
            int e = c;
            while (e < P.ncomp && P.comp_pat[e] == id) ++e;
            if (dp->pats.n == bbc::kMaxBlockPatterns) return fail(BBC_EUNSUPPORTED, "too many component patterns");
            bbc::BlockPattern &bp = dp->pats.p[dp->pats.n++];
            const int sp = id / 8;
            const bbc::SpinStruct &S = bbc::spin_struct(sp);
            bp.begin = c;
            bp.end = e;
            bp.qa = (uint8_t)((id >> 2) & 1);
            bp.qb = (uint8_t)((id >> 1) & 1);
            bp.qc = (uint8_t)(id & 1);
            for (int m = 0; m < 4; ++m) {
                bp.p1[m] = (uint8_t)S.p1[m]; bp.k1[m] = (uint8_t)S.k1[m];
                bp.p2[m] = (uint8_t)S.p2[m]; bp.k2[m] = (uint8_t)S.k2[m];
            }
            bp.new_diquark = 1;
            if (dp->pats.n > 1) {
                const bbc::BlockPattern &pv = dp->pats.p[dp->pats.n - 2];
                bool same = pv.qa == bp.qa && pv.qb == bp.qb;
                for (int m = 0; m < 4; ++m) same = same && pv.p1[m] == bp.p1[m] && pv.k1[m] == bp.k1[m];
                bp.new_diquark = same ? 0 : 1;
            }
            c = e;
        }
        bbc::PairTables pt;
        try {
            // row tiles of three rows and at most 4 columns (2 in shape 1): three (FP32)
            // or four (FP64) waves per SIMD with their accumulators
            pt = bbc::build_pair_tables(P, kTileRows, kTileCols);
        } catch (const std::exception &e) {
            return fail(BBC_EUNSUPPORTED, std::string("contraction tables: ") + e.what());
        }
        // the tile kernels take exactly these shapes (a larger one would be skipped)
        for (const bbc::PTask &t : pt.tiles)
            if (t.nrow < 1 || t.nrow > kTileRows || t.np < 1 || t.np > (t.shape ? kTileCols / 2 : kTileCols))
                return fail(BBC_EUNSUPPORTED, "contraction tile outside the kernels' shapes");
        dp->ntask = (int)pt.tasks.size();
        dp->ntile = (int)pt.tiles.size();
        dp->npair = pt.npair;
        std::vector<int2> content;
        for (int ch : P.channels) {
            const auto bq = bbc::channel_baryons(ch);
            int ns = 0;
            for (int s2 = 0; s2 < 2; ++s2)
                for (int i = 0; i < 3; ++i) ns += bbc::baryon(bq[s2]).flav[i] == bbc::FS;
            content.push_back(make_int2(6 - ns, ns));
        }
        std::vector<unsigned char> &img = dp->image;
        // block kernel: terms with the diquark index ea * 12 + eb precomputed, and one
        // record per component holding its first two terms
        std::vector<uint32_t> kterms(P.terms.size());
        for (size_t t = 0; t < P.terms.size(); ++t) {
            const uint32_t code = P.terms[t];
            kterms[t] = ((code & 15) * 12 + ((code >> 4) & 15)) | (code & 0x3f00u);
        }
        std::vector<bbc::BlockComp> comps(P.ncomp);
        for (int c = 0; c < P.ncomp; ++c) {
            const int tb = P.term_begin[c], n = P.term_begin[c + 1] - tb;
            // the block kernel takes terms in pairs (every component of the
            // catalogue has 2, 8 or 24: its colour antisymmetry pairs them)
            if (n < 2 || n % 2)
                return fail(BBC_EUNSUPPORTED, "block component with " + std::to_string(n) + " terms");
            comps[c] = bbc::BlockComp{n > 0 ? kterms[tb] : 0u, n > 1 ? kterms[tb + 1] : 0u, (uint32_t)(tb + 2),
                                      (uint32_t)n};
        }
        dp->off_terms = image_put(img, kterms.data(), kterms.size());
        dp->off_comps = image_put(img, comps.data(), comps.size());
        dp->off_tasks = image_put(img, pt.tasks.data(), pt.tasks.size());
        dp->off_tiles = image_put(img, pt.tiles.data(), pt.tiles.size());
        dp->off_comb = image_put(img, pt.comb.data(), pt.comb.size());
        dp->off_comb_begin = image_put(img, pt.comb_begin.data(), pt.comb_begin.size());
        dp->off_content = image_put(img, content.data(), content.size());
        img.resize((img.size() + 255) & ~(size_t)255, 0);
        dp->table_bytes = img.size();
        it = ctx->plans.emplace(key, std::move(dp)).first;
    }
    DevPlan *dp = it->second.get();
    if (upload && !dp->d_image) {
        HIP_TRY(hipSetDevice(ctx->device));
        hipError_t e = hipMalloc(&dp->d_image, dp->image.size());
        if (e != hipSuccess) { dp->d_image = nullptr; return fail(BBC_ENOMEM, "hipMalloc of the plan tables"); }
        HIP_TRY(hipMemcpy(dp->d_image, dp->image.data(), dp->image.size(), hipMemcpyHostToDevice));
    }
    *out = dp;
    return BBC_OK;
}

// Workspace of one slice:
//   region A: the intermediates I in site space (2 spins x nc x V); once they
//             are in the momentum groups it is dead, and the contracted fields
//             Ct (n_ch x 16 x V, 16 bytes each) and, after them, the pair products
//             P (npair x 16 per grouped position, at most V + 8) reuse it;
//   region B: the momentum-grouped copy Iq (groups x 2 x nc x G, at most V + 8
//             positions);
//   then the rescale maxima of the FP32 form.
struct WsLayout {
    size_t p, a, b, total;   // byte offsets of P (inside region A), of region B, of the small tail; total
};
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
WsLayout ws_layout(long V, int nc, int n_ch, int npair, size_t csize) {
    WsLayout L;
    L.p = align256((size_t)n_ch * 16 * V * 16);   // Ct: 16 bytes per value (double2, or float-float pairs)
    const size_t ra = std::max<size_t>((size_t)2 * nc * V * csize, L.p + (size_t)npair * 16 * (V + 8) * csize);
    const size_t rb = (size_t)2 * nc * (V + 8) * csize;
    L.a = align256(ra);
    L.b = L.a + align256(rb);
    L.total = L.b + 256;
    return L;
}
size_t workspace_bytes(long V, int nc, int n_ch, int npair, size_t csize) {
    return ws_layout(V, nc, n_ch, npair, csize).total;
}

bbc_status check_lattice(const int32_t *lattice, long *V) {
    if (!lattice) return fail(BBC_EINVAL, "lattice is NULL");
    long v = 1;
    for (int i = 0; i < 3; ++i) {
        if (lattice[i] < 1) return fail(BBC_EINVAL, "lattice extent must be positive");
        if (!bbc::fft_size_supported(lattice[i]))
            return fail(BBC_EUNSUPPORTED, "lattice extent " + std::to_string(lattice[i]) +
                                              " not in {1,2,3,4,6,8,12,16,24,32,48,64,96}");
        v *= lattice[i];
    }
    if (v > (1L << 30)) return fail(BBC_EUNSUPPORTED, "lattice volume too large");
    *V = v;
    return BBC_OK;
}

// Device table of the momentum groups for precision T.
struct MomGroups {
    const int2 *pos = nullptr;
    const int *posof = nullptr;   // momentum -> position (V entries)
    const int *xrun = nullptr;    // run-ordered lattices: x-row -> first group of its run (Ly Lz entries)
    int ngroup = 0;
};
constexpr int kGroupSize = 8;                    // momenta per group

// Host image of the momentum groups of a lattice: the npos position entries,
// then the V momentum -> position entries and, for run-ordered lattices, the
// Ly Lz x-row -> run entries (as ints, two per int2).
std::vector<int2> group_image(const int L[3], long *npos_out) {
    const long V = (long)L[0] * L[1] * L[2];
    const long npos = grouped_positions(V, L, kGroupSize);
    std::vector<int> xrun;
    std::vector<int2> g = momentum_groups(L, kGroupSize, &xrun);
    std::vector<int2> all(g);
    all.resize(npos + (V + (long)xrun.size() + 1) / 2);
    int *posof = reinterpret_cast<int *>(all.data() + npos);
    for (long p = 0; p < npos; ++p)
        if (g[p].x >= 0) posof[g[p].x] = (int)p;
    std::copy(xrun.begin(), xrun.end(), posof + V);
    *npos_out = npos;
    return all;
}

MomGroups groups_at(const int2 *base, long npos, const int L[3]) {
    const int *posof = reinterpret_cast<const int *>(base + npos);
    const long V = (long)L[0] * L[1] * L[2];
    return MomGroups{base, posof, run_ordered(L) ? posof + V : nullptr, (int)(npos / kGroupSize)};
}

template <typename T>
MomGroups get_groups(bbc_context *ctx, const int L[3], bbc_status *st) {
    std::lock_guard<std::mutex> lock(ctx->qmu);
    auto key = std::vector<int>{L[0], L[1], L[2], kGroupSize};
    auto it = ctx->groups.find(key);
    long npos = 0;
    if (it == ctx->groups.end()) {
        std::vector<int2> all = group_image(L, &npos);
        int2 *d = nullptr;
        hipError_t e = upload_vec(&d, all);
        if (e != hipSuccess) {
            *st = fail(BBC_EDEVICE, std::string("momentum group upload: ") + hipGetErrorString(e));
            return MomGroups{};
        }
        it = ctx->groups.emplace(key, d).first;
    } else {
        npos = grouped_positions((long)L[0] * L[1] * L[2], L, kGroupSize);
    }
    *st = BBC_OK;
    return groups_at(it->second, npos, L);
}

using TuneKey = std::array<uint64_t, 6>;
TuneKey tune_key(const int L[3], int prec, int spin_offset, uint64_t chash) {
    return TuneKey{(uint64_t)L[0], (uint64_t)L[1], (uint64_t)L[2], (uint64_t)prec, (uint64_t)spin_offset, chash};
}

// Built-in choice for shapes without a tuning entry (the fastest variants
// measured at 16^3 and 32^3 with 52 channels): the contraction in row tiles
// staged through LDS (FP64 per set of 4 momenta), and in FP32 the LDS-staged
// channel sums, 8 x 2 block workgroups and half-size plane-pass workgroups.
// Small lattices run several slices at once (a slice alone does not fill the
// GPU), and up to 512 sites the block kernel takes 4 x 4 workgroups (4 sites x
// 2 shares would give one workgroup per CU).
bbc::Tuning default_tuning(const int L[3], int prec) {
    const long V = (long)L[0] * L[1] * L[2];
    const int sl = V <= 2048 ? 3 : V <= 4096 ? 1 : 0;
    if (prec == BBC_F32) return bbc::Tuning{5, V <= 512 ? 1 : 2, 1, sl, 2};
    return bbc::Tuning{8, V <= 512 ? 1 : 0, 0, sl, 0};
}

// Tuning of a request: the context's entry for its shape, else the built-in choice.
bbc::Tuning tuning_for(bbc_context *ctx, const int L[3], const DevPlan *dp) {
    std::lock_guard<std::mutex> lock(ctx->tmu);
    auto it = ctx->tuning.find(tune_key(L, dp->prec, dp->spin_offset, dp->chash));
    return it != ctx->tuning.end() ? it->second : default_tuning(L, dp->prec);
}

// Launches the kernel sequence of one time slice on stream st, using the
// workspace ws (layout of workspace_bytes).  Stage events are recorded only
// for the direct (profiled) path.  force: kernel variants to use instead of
// the request's tuning (the autotuner's candidates).
template <typename T>
bbc_status enqueue_slice(bbc_context *ctx, const PlanDev &pd, const int L[3], long V, void *ws, const MomGroups &mg,
                         const void *slp, const void *ssp, int n_ch, const double *d_energy, double dt, void *outp,
                         double *scale, hipStream_t st, bool timed, const bbc::Tuning *force = nullptr,
                         const bbc::SliceArgs *ia = nullptr) {
    using T2 = typename bbc::cplx_t<T>::type;
    const DevPlan *dp = pd.dp;
    const bbc::Tuning tu = force ? *force : tuning_for(ctx, L, dp);
    const bbc::Plan &P = dp->plan;
    const int nc = P.ncomp;
    const WsLayout lay = ws_layout(V, nc, n_ch, dp->npair, sizeof(T2));
    T2 *I = (T2 *)ws;
    T2 *Iq = (T2 *)((char *)ws + lay.a);
    using TC = typename bbc::ct_t<T>::type;
    TC *Ct = (TC *)ws;                            // reuses region A once Iq is written
    T2 *Pp = (T2 *)((char *)ws + lay.p);
    uint32_t *kmax = (uint32_t *)((char *)ws + lay.b);
    bbc::PairDevTables tb{mg.pos, mg.ngroup, pd.tasks, dp->ntask, pd.tiles, dp->ntile, dp->npair, pd.comb,
                          pd.comb_begin};
    const T2 *sl = (const T2 *)slp, *ss = (const T2 *)ssp;
    T2 *out = (T2 *)outp;
    const bool fp32 = sizeof(T) == 4;
    bbc_context *pc = timed ? ctx : nullptr;
    {
        StageTimer tm(pc, st, 0);
        if (fp32) bbc::launch_absmax((const float2 *)sl, (const float2 *)ss, V * 144, kmax, st, ia);
        bbc::launch_blocks<T>(sl, ss, I, (int)V, nc, P.spin_offset, pd.comps, pd.terms, dp->pats,
                              fp32 ? kmax : nullptr, tu.blocks, st, ia);
    }
    // small cubic lattices: one fused pass (FFT in LDS, written straight into the
    // groups); 24- and 32-point planes: plane passes, then the z pass writes into
    // the groups; otherwise axis passes and a separate copy into the groups
    // FP32 cubic 32-point lattices: one pass too (z in registers, x and y in LDS,
    // written into the run-ordered groups)
    const bool onepass = mg.xrun && bbc::fft3d_onepass_fits<T>(L);
    const bool fused = onepass || bbc::fft3d_grouped_fits<T>(L);
    const bool zgrouped = !fused && bbc::fft3d_zgrouped_fits<T>(L);
    {
        StageTimer tm(pc, st, 1);
        if (onepass) {
            if (bbc::launch_fft3d_onepass<T>(I, Iq, nc, L, mg.xrun, st)) return fail(BBC_EUNSUPPORTED, "FFT size");
        } else if (fused) {
            if (bbc::launch_fft3d_grouped<T>(I, Iq, nc, L, mg.ngroup, mg.pos, st))
                return fail(BBC_EUNSUPPORTED, "FFT size");
        } else if (zgrouped) {
            if ((tm.nk = bbc::launch_fft3d_zgrouped<T>(I, Iq, nc, L, mg.posof, mg.xrun, tu.planes, st)) < 0)
                return fail(BBC_EUNSUPPORTED, "FFT size");
        } else if ((tm.nk = bbc::launch_fft3d<T>(I, 2L * nc, L, -1, st)) < 0) {
            return fail(BBC_EUNSUPPORTED, "FFT size");
        }
    }
    if (!fused && !zgrouped) {
        StageTimer tm(pc, st, 2);
        bbc::launch_transpose_grouped<T>(I, Iq, nc, V, mg.ngroup, mg.pos, st);
    }
    {
        StageTimer tm(pc, st, 3);
        bbc::launch_pairs<T>(Iq, Pp, nc, tb, tu.pairs, st);
    }
    {
        StageTimer tm(pc, st, 6);
        bbc::launch_pair_combine<T>(Pp, Ct, n_ch, V, tb, tu.combine, st);
    }
    {
        StageTimer tm(pc, st, 4);
        // FP32 form: compensated float-float arithmetic for this last spatial sum
        if ((tm.nk = bbc::launch_fft3d<typename bbc::ct_real<T>::type>(Ct, 16L * n_ch, L, +1, st)) < 0)
            return fail(BBC_EUNSUPPORTED, "FFT size");
    }
    {
        StageTimer tm(pc, st, 5);
        bbc::launch_finalize<T>(Ct, out, n_ch, (int)V, d_energy, dt, 1.0 / (double)V, scale, fp32 ? kmax : nullptr,
                                pd.content, st, ia, dp->full_sub);
    }
    HIP_TRY(hipGetLastError());
    return BBC_OK;
}

// Streams and events of the concurrent-slice path (created once per context).
bbc_status slice_streams(bbc_context *ctx, int B) {
    for (int b = 0; b < B; ++b)
        if (!ctx->bstreams[b]) HIP_TRY(hipStreamCreateWithFlags(&ctx->bstreams[b], hipStreamNonBlocking));
    for (int b = 0; b <= B; ++b)
        if (!ctx->bev[b]) HIP_TRY(hipEventCreateWithFlags(&ctx->bev[b], hipEventDisableTiming));
    return BBC_OK;
}

// n device-resident slices, B of them at a time: slice i runs on stream i mod B
// (the caller's stream when B = 1) with its own workspace ws + (i mod B) stride.
// The B streams wait for the caller's earlier work and the caller's stream waits
// for all of them, so the call stays ordered on `st`; under graph capture on `st`
// the streams become parallel branches of the graph.  Each slice runs the same
// kernels on its own buffers, so the results do not depend on B.
template <typename T>
bbc_status enqueue_slices(bbc_context *ctx, const PlanDev &pd, const int L[3], long V, char *ws, size_t stride,
                          int B, const MomGroups &mg, int n, const void *const *sl, const void *const *ss, int n_ch,
                          const double *d_energy, const double *dt, void *const *out, double *const *scale,
                          hipStream_t st, bool timed, const bbc::Tuning *force = nullptr) {
    if (B <= 1) {
        for (int i = 0; i < n; ++i) {
            bbc_status s = enqueue_slice<T>(ctx, pd, L, V, ws, mg, sl[i], ss[i], n_ch, d_energy, dt[i], out[i],
                                            scale[i], st, timed, force);
            if (s) return s;
        }
        return BBC_OK;
    }
    bbc_status s = slice_streams(ctx, B);
    if (s) return s;
    HIP_TRY(hipEventRecord(ctx->bev[0], st));
    for (int b = 0; b < B; ++b) HIP_TRY(hipStreamWaitEvent(ctx->bstreams[b], ctx->bev[0], 0));
    for (int i = 0; i < n; ++i) {
        const int b = i % B;
        s = enqueue_slice<T>(ctx, pd, L, V, ws + (size_t)b * stride, mg, sl[i], ss[i], n_ch, d_energy, dt[i], out[i],
                             scale[i], ctx->bstreams[b], false, force);
        if (s) return s;
    }
    for (int b = 0; b < B; ++b) {
        HIP_TRY(hipEventRecord(ctx->bev[1 + b], ctx->bstreams[b]));
        HIP_TRY(hipStreamWaitEvent(st, ctx->bev[1 + b], 0));
    }
    return BBC_OK;
}

// Concurrent slices of a direct call: the tuning's choice, at most n_t, one when
// profiling (stage events are per stream), and as many as the budget allows.
int concurrent_slices(bbc_context *ctx, const bbc::Tuning &tu, int n_t, size_t per_slice, size_t extra) {
    int B = std::min(n_t, 1 << tu.slices);
    if (ctx->prof) B = 1;
    while (B > 1 && ctx->budget && (size_t)B * per_slice + extra > ctx->budget) B >>= 1;
    return std::max(B, 1);
}

// True unless the pointer is memory kernels may dereference directly: HIP device
// allocations (or managed memory).  Pinned host memory, and pageable memory --
// reported either as an error or as hipMemoryTypeUnregistered -- count as host
// memory and are only ever touched by copies.
bool is_host_pointer(const void *p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) { (void)hipGetLastError(); return true; }
    return !(attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
}

// Grows the context workspace to at least `need` bytes (waits for the device
// and drops the cached graphs, which hold its old address).
bbc_status ensure_workspace(bbc_context *ctx, size_t need) {
    if (ctx->ws_bytes >= need) return BBC_OK;
    HIP_TRY(hipDeviceSynchronize());
    ctx->clear_graphs();
    if (ctx->ws) { HIP_TRY(hipFree(ctx->ws)); ctx->ws = nullptr; ctx->ws_bytes = 0; }
    hipError_t e = hipMalloc(&ctx->ws, need);
    if (e != hipSuccess) { ctx->ws = nullptr; return fail(BBC_ENOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e)); }
    ctx->ws_bytes = need;
    return BBC_OK;
}

// Copies the per-channel energies to the context's device array (stream-ordered).
bbc_status upload_energy(bbc_context *ctx, const double *energy, int n_ch, hipStream_t st) {
    if (ctx->energy_cap < n_ch) {
        HIP_TRY(hipDeviceSynchronize());
        ctx->clear_graphs();
        if (ctx->d_energy) HIP_TRY(hipFree(ctx->d_energy));
        ctx->d_energy = nullptr;
        HIP_TRY(hipMalloc((void **)&ctx->d_energy, sizeof(double) * n_ch));
        ctx->energy_cap = n_ch;
    }
    HIP_TRY(hipMemcpyAsync(ctx->d_energy, energy, sizeof(double) * n_ch, hipMemcpyHostToDevice, st));
    return BBC_OK;
}

// Direct path.  Propagators and output may be device or host memory; host
// buffers (pinned memory recommended) are streamed per slice through two
// device staging buffers each, on separate copy streams, so that the transfer
// of slice n+1 in, and of slice n-1 out, overlap the kernels of slice n.
template <typename T>
bbc_status run_correlate(bbc_context *ctx, DevPlan *dp, const int L[3], long V, const void *S_light,
                         const void *S_strange, int n_t, const int32_t *t_list, int t0, int n_ch,
                         const double *energy, void *C_out, double *C_scale, hipStream_t st, bool host_in,
                         bool host_out) {
    using T2 = typename bbc::cplx_t<T>::type;
    const size_t cs = sizeof(T2);
    const size_t core = workspace_bytes(V, dp->plan.ncomp, n_ch, dp->npair, cs);
    const size_t in_slice = (size_t)V * 144 * cs, out_slice = (size_t)n_ch * V * (dp->full_sub >= 0 ? 256 : 16) * cs;
    const size_t in_stage = host_in ? 2 * 2 * in_slice : 0, out_stage = host_out ? 2 * out_slice : 0;
    // device-resident requests may run several slices at once (own workspace each)
    const bool device_path = !host_in && !host_out;
    const size_t stride = (core + 255) & ~(size_t)255;
    const int B = device_path ? concurrent_slices(ctx, tuning_for(ctx, L, dp), n_t, stride, dp->table_bytes) : 1;
    const size_t need = B > 1 ? (size_t)B * stride : core + in_stage + out_stage;
    if (ctx->budget && need + dp->table_bytes > ctx->budget)
        return fail(BBC_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the context budget");
    bbc_status s = ensure_workspace(ctx, need);
    if (s) return s;
    if (energy && (s = upload_energy(ctx, energy, n_ch, st))) return s;
    const MomGroups mg = get_groups<T>(ctx, L, &s);
    if (!mg.pos) return s;
    std::vector<const void *> vsl, vss;
    std::vector<void *> vout;
    std::vector<double *> vsc;
    std::vector<double> vdt;
    if (device_path) {
        for (int n = 0; n < n_t; ++n) {
            vsl.push_back((const T2 *)S_light + (size_t)n * V * 144);
            vss.push_back((const T2 *)S_strange + (size_t)n * V * 144);
            vout.push_back((char *)C_out + (size_t)n * out_slice);
            vsc.push_back(C_scale ? C_scale + (size_t)n * n_ch : nullptr);
            vdt.push_back((double)(t_list[n] - t0));
        }
    }
    if (ctx->graph_mode && device_path && !ctx->prof && n_t > 0) {
        // every value the captured kernels depend on
        std::vector<int64_t> key = {(int64_t)(intptr_t)dp, L[0], L[1], L[2], (int64_t)sizeof(T),
                                    (int64_t)(intptr_t)S_light, (int64_t)(intptr_t)S_strange, n_t, t0, n_ch,
                                    (int64_t)(intptr_t)(energy ? ctx->d_energy : nullptr), (int64_t)(intptr_t)C_out,
                                    (int64_t)(intptr_t)C_scale, (int64_t)(intptr_t)ctx->ws, B};
        for (int n = 0; n < n_t; ++n) key.push_back(t_list[n]);
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            if (!ctx->gs) HIP_TRY(hipStreamCreateWithFlags(&ctx->gs, hipStreamNonBlocking));
            if (ctx->graphs.size() >= 16) ctx->clear_graphs();
            HIP_TRY(hipStreamBeginCapture(ctx->gs, hipStreamCaptureModeRelaxed));
            bbc_status es = enqueue_slices<T>(ctx, plan_dev(dp, dp->d_image), L, V, (char *)ctx->ws, stride, B, mg,
                                              n_t, vsl.data(), vss.data(), n_ch,
                                              energy ? ctx->d_energy : nullptr, vdt.data(), vout.data(), vsc.data(),
                                              ctx->gs, false);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->gs, &g);
            if (es != BBC_OK) { if (g) (void)hipGraphDestroy(g); return es; }
            if (e != hipSuccess) return fail(BBC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(BBC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
            it = ctx->graphs.emplace(key, ex).first;
        }
        HIP_TRY(hipGraphLaunch(it->second, st));
        return BBC_OK;
    }
    if (device_path)
        return enqueue_slices<T>(ctx, plan_dev(dp, dp->d_image), L, V, (char *)ctx->ws, stride, B, mg, n_t,
                                 vsl.data(), vss.data(), n_ch, energy ? ctx->d_energy : nullptr, vdt.data(),
                                 vout.data(), vsc.data(), st, true);
    char *stage_in = (char *)ctx->ws + core, *stage_out = stage_in + in_stage;
    if ((host_in || host_out) && !ctx->cin) {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->cin, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&ctx->cout, hipStreamNonBlocking));
        for (auto &e : ctx->sev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    // events: [0,1] input staged, [2,3] input consumed, [4,5] output ready, [6,7] output drained
    hipEvent_t *ev = ctx->sev;
    auto stage_input = [&](int n) -> bbc_status {
        const int b = n & 1;
        char *dl = stage_in + (size_t)b * 2 * in_slice, *ds = dl + in_slice;
        if (n >= 2) HIP_TRY(hipStreamWaitEvent(ctx->cin, ev[2 + b], 0));
        HIP_TRY(hipMemcpyAsync(dl, (const char *)S_light + (size_t)n * in_slice, in_slice, hipMemcpyHostToDevice,
                               ctx->cin));
        HIP_TRY(hipMemcpyAsync(ds, (const char *)S_strange + (size_t)n * in_slice, in_slice, hipMemcpyHostToDevice,
                               ctx->cin));
        HIP_TRY(hipEventRecord(ev[b], ctx->cin));
        return BBC_OK;
    };
    if (host_in && n_t > 0) {
        HIP_TRY(hipEventRecord(ev[7], st));           // stage after earlier work on st
        HIP_TRY(hipStreamWaitEvent(ctx->cin, ev[7], 0));
        if ((s = stage_input(0))) return s;
    }
    const T2 *Sl = (const T2 *)S_light, *Ss = (const T2 *)S_strange;
    for (int n = 0; n < n_t; ++n) {
        const int b = n & 1;
        const T2 *sl = Sl + (size_t)n * V * 144, *ss = Ss + (size_t)n * V * 144;
        if (host_in) {
            if (n + 1 < n_t && (s = stage_input(n + 1))) return s;
            HIP_TRY(hipStreamWaitEvent(st, ev[b], 0));
            sl = (const T2 *)(stage_in + (size_t)b * 2 * in_slice);
            ss = (const T2 *)(stage_in + (size_t)b * 2 * in_slice + in_slice);
        }
        void *out = (char *)C_out + (size_t)n * out_slice;
        if (host_out) {
            if (n >= 2) HIP_TRY(hipStreamWaitEvent(st, ev[6 + b], 0));
            out = stage_out + (size_t)b * out_slice;
        }
        s = enqueue_slice<T>(ctx, plan_dev(dp, dp->d_image), L, V, ctx->ws, mg, sl, ss, n_ch, energy ? ctx->d_energy : nullptr,
                             (double)(t_list[n] - t0), out, C_scale ? C_scale + (size_t)n * n_ch : nullptr, st,
                             true);
        if (s) return s;
        if (host_in) HIP_TRY(hipEventRecord(ev[2 + b], st));    // staged input of slice n no longer needed
        if (host_out) {
            HIP_TRY(hipEventRecord(ev[4 + b], st));
            HIP_TRY(hipStreamWaitEvent(ctx->cout, ev[4 + b], 0));
            HIP_TRY(hipMemcpyAsync((char *)C_out + (size_t)n * out_slice, out, out_slice, hipMemcpyDeviceToHost,
                                   ctx->cout));
            HIP_TRY(hipEventRecord(ev[6 + b], ctx->cout));
        }
    }
    // the caller's stream completes only when the last outputs have left the device
    if (host_out && n_t > 0) {
        HIP_TRY(hipStreamWaitEvent(st, ev[6 + ((n_t - 1) & 1)], 0));
        if (n_t > 1) HIP_TRY(hipStreamWaitEvent(st, ev[6 + ((n_t - 2) & 1)], 0));
    }
    if (host_in && n_t > 0) HIP_TRY(hipStreamWaitEvent(st, ev[(n_t - 1) & 1], 0));
    return BBC_OK;
}

// Forward/backward (CPT) average (Sec. 6), device memory only.  Per tau the
// upper components of slice t0 + tau are written to R_out, the lower components
// of slice t0 - tau (both mod Lt) to a workspace buffer after the slice
// workspace, and the averaging kernel combines them in place.  Both parts are
// normalised by exp(E tau).
template <typename T>
bbc_status run_cpt(bbc_context *ctx, DevPlan *up, DevPlan *lo, const int L[3], long V, int Lt,
                   const void *S_light, const void *S_strange, int t0, int n_tau, const int32_t *tau_list,
                   int n_ch, const double *energy, int sign, void *R_out, double *R_scale, hipStream_t st) {
    using T2 = typename bbc::cplx_t<T>::type;
    constexpr bool fp32 = sizeof(T) == 4;
    const size_t cs = sizeof(T2);
    const size_t core = std::max(workspace_bytes(V, up->plan.ncomp, n_ch, up->npair, cs),
                                 workspace_bytes(V, lo->plan.ncomp, n_ch, lo->npair, cs));
    const size_t out_slice = (size_t)n_ch * V * 16 * cs;
    const size_t bwd_off = (core + 255) & ~(size_t)255;
    const size_t sc_off = (bwd_off + out_slice + 255) & ~(size_t)255;
    const size_t need = sc_off + 2 * sizeof(double) * n_ch;
    if (ctx->budget && need + up->table_bytes + lo->table_bytes > ctx->budget)
        return fail(BBC_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the context budget");
    bbc_status s = ensure_workspace(ctx, need);
    if (s) return s;
    if (energy && (s = upload_energy(ctx, energy, n_ch, st))) return s;
    const MomGroups mg = get_groups<T>(ctx, L, &s);
    if (!mg.pos) return s;
    T2 *bwd = (T2 *)((char *)ctx->ws + bwd_off);
    double *sf = fp32 ? (double *)((char *)ctx->ws + sc_off) : nullptr;
    double *sb = fp32 ? sf + n_ch : nullptr;
    const T2 *Sl = (const T2 *)S_light, *Ss = (const T2 *)S_strange;
    const double *de = energy ? ctx->d_energy : nullptr;
    for (int n = 0; n < n_tau; ++n) {
        const int tau = tau_list[n];
        const size_t tf = (size_t)(((t0 + tau) % Lt + Lt) % Lt), tb = (size_t)(((t0 - tau) % Lt + Lt) % Lt);
        T2 *out = (T2 *)((char *)R_out + (size_t)n * out_slice);
        s = enqueue_slice<T>(ctx, plan_dev(up, up->d_image), L, V, ctx->ws, mg, Sl + tf * V * 144, Ss + tf * V * 144, n_ch, de, (double)tau,
                             out, sf, st, true);
        if (s) return s;
        s = enqueue_slice<T>(ctx, plan_dev(lo, lo->d_image), L, V, ctx->ws, mg, Sl + tb * V * 144, Ss + tb * V * 144, n_ch, de, (double)tau,
                             bwd, sb, st, true);
        if (s) return s;
        bbc::launch_cpt_average<T>(out, bwd, V * 16, n_ch, (double)sign, sf, sb,
                                   fp32 ? R_scale + (size_t)n * n_ch : nullptr, st);
        HIP_TRY(hipGetLastError());
    }
    return BBC_OK;
}

}  // namespace

namespace {

size_t job_footprint(const Job &j) {
    const long V = (long)j.ps->L[0] * j.ps->L[1] * j.ps->L[2];
    const size_t cs = j.ps->prec == BBC_F64 ? 16 : 8;
    return workspace_bytes(V, j.dp->plan.ncomp, (int)j.chans.size(), j.dp->npair, cs) + 8 * j.chans.size() + 256;
}

// Enqueues slice j.next of a running job on its slot.  In graph mode the slot
// replays one captured slice per request shape (plan, lattice, precision,
// energies, workspace, kernel variants): a one-thread kernel first writes this
// slice's propagator, output and scale pointers and t - t0 to the slot's
// argument record, which the captured block, rescale and output kernels read.
// The same kernels run in the same order either way, so the results are the
// same bits.
template <typename T>
bbc_status server_enqueue_t(bbc_context *ctx, Slot &sl, Job &j) {
    using T2 = typename bbc::cplx_t<T>::type;
    Server &S = ctx->srv;
    const PropSet &ps = *j.ps;
    const long V = (long)ps.L[0] * ps.L[1] * ps.L[2];
    const int n_ch = (int)j.chans.size();
    bbc_status s;
    const size_t wsz = workspace_bytes(V, j.dp->plan.ncomp, n_ch, j.dp->npair, sizeof(T2));
    const double *d_energy = j.energy.empty() ? nullptr : (const double *)((char *)sl.ws + ((wsz + 255) & ~(size_t)255));
    const int n = j.next;
    const int si = j.slice[n];
    const size_t slice_elems = (size_t)V * 144;
    const double dt = (double)(j.tl[n] - j.t0);
    const MomGroups mg = get_groups<T>(ctx, ps.L, &s);
    if (!mg.pos) return s;
    const T2 *dl = (const T2 *)ps.dl + si * slice_elems, *ds = (const T2 *)ps.ds + si * slice_elems;
    T2 *out = (T2 *)j.out + (size_t)n * n_ch * V * 16;
    double *scale = sizeof(T) == 4 ? j.scale + (size_t)n * n_ch : nullptr;
    const PlanDev pd = plan_dev(j.dp, j.dp->d_image);
    if (!ctx->graph_mode || !sl.d_args)
        return enqueue_slice<T>(ctx, pd, ps.L, V, sl.ws, mg, dl, ds, n_ch, d_energy, dt, out, scale, sl.st, false);
    const bbc::Tuning tu = tuning_for(ctx, ps.L, j.dp);
    const std::vector<int64_t> key = {(int64_t)(intptr_t)j.dp, ps.L[0], ps.L[1], ps.L[2], (int64_t)sizeof(T), n_ch,
                                      d_energy ? 1 : 0, (int64_t)(intptr_t)sl.ws, tu.pairs, tu.blocks, tu.planes,
                                      tu.combine};
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
        if (!S.cap) HIP_TRY(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(S.cap, hipStreamCaptureModeRelaxed));
        const bbc_status es = enqueue_slice<T>(ctx, pd, ps.L, V, sl.ws, mg, dl, ds, n_ch, d_energy, dt, out, scale,
                                               S.cap, false, &tu, sl.d_args);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(S.cap, &g);
        if (es != BBC_OK) { if (g) (void)hipGraphDestroy(g); return es; }
        if (e != hipSuccess) return fail(BBC_EDEVICE, std::string("slot graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(BBC_EDEVICE, std::string("slot graph instantiate: ") + hipGetErrorString(e));
        it = sl.graphs.emplace(key, ex).first;
    }
    bbc::launch_slice_args(sl.d_args, bbc::SliceArgs{dl, ds, out, scale, dt}, sl.st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipGraphLaunch(it->second, sl.st));
    return BBC_OK;
}

bbc_status server_enqueue(bbc_context *ctx, Slot &sl, Job &j) {
    return j.ps->prec == BBC_F64 ? server_enqueue_t<double>(ctx, sl, j) : server_enqueue_t<float>(ctx, sl, j);
}

void release_prop_if_unused(Server &S, PropSet *ps) {
    if (ps->released && ps->refs == 0) {
        (void)hipFree(ps->dl);
        (void)hipFree(ps->ds);
        S.committed -= ps->bytes;
        for (auto it = S.props.begin(); it != S.props.end(); ++it)
            if (it->second.get() == ps) { S.props.erase(it); break; }
    }
}

void finish_job(Server &S, Job &j, int state) {
    j.state = state;
    j.t_done = Clock::now();
    j.ps->refs--;
    release_prop_if_unused(S, j.ps);
    S.done_cv.notify_all();
}

// Admission (called by the scheduler thread with S.mu held through lk).
//
// A queued job fits a free slot when the slot's workspace is large enough
// (workspaces are kept between jobs and reused), or when replacing it by one
// of the job's size keeps the committed bytes -- resident propagator sets plus
// slot workspaces -- within the context budget.  Jobs are taken in arrival
// order; when the job at the head does not fit, up to kBypassWindow later jobs
// that do may start instead, at most kMaxBypass times per head job, so a large
// job is delayed but never starved.  When nothing fits, the workspaces of idle
// slots are released; if the head job still does not fit with no job running,
// it can never run beside the resident propagator sets and is refused.
// Device allocation and release happen with S.mu unlocked (hipFree waits for
// the device); the slot is reserved for its job meanwhile.
constexpr int kBypassWindow = 8;
constexpr int kMaxBypass = 16;

bool admit_jobs(bbc_context *ctx, std::unique_lock<std::mutex> &lk) {
    Server &S = ctx->srv;
    bool progressed = false;
    auto fits = [&](const Slot &sl, const Job *j) {
        if (j->foot <= sl.ws_bytes || !ctx->budget) return true;
        return S.committed - sl.ws_bytes + j->foot <= ctx->budget;
    };
    for (;;) {
        if (S.queue.empty() || S.stop) break;
        bool any_free = false, any_busy = false;
        for (auto &sl : S.slots) (sl.job || sl.reserved ? any_busy : any_free) = true;
        if (!any_free) break;
        Job *head = S.queue.front();
        const size_t window = head->bypassed < kMaxBypass ? std::min<size_t>(S.queue.size(), 1 + kBypassWindow) : 1;
        size_t pick = window;
        Slot *slot = nullptr;
        for (size_t q = 0; q < window && !slot; ++q) {
            const Job *j = S.queue[q];
            // best fit: the smallest free workspace that holds the job, else the
            // largest free one that may be replaced within the budget
            for (auto &sl : S.slots) {
                if (sl.job || sl.reserved || !fits(sl, j)) continue;
                const bool holds = sl.ws_bytes >= j->foot;
                if (!slot) { slot = &sl; continue; }
                const bool sholds = slot->ws_bytes >= j->foot;
                if (holds && (!sholds || sl.ws_bytes < slot->ws_bytes)) slot = &sl;
                else if (!holds && !sholds && sl.ws_bytes > slot->ws_bytes) slot = &sl;
            }
            if (slot) pick = q;
        }
        if (!slot) {
            // nothing fits: release the workspaces of idle slots, then look again
            std::vector<void *> drop;
            for (auto &sl : S.slots)
                if (!sl.job && !sl.reserved && sl.ws) {
                    sl.clear_graphs();
                    drop.push_back(sl.ws);
                    S.committed -= sl.ws_bytes;
                    sl.ws = nullptr;
                    sl.ws_bytes = 0;
                }
            if (!drop.empty()) {
                lk.unlock();
                for (void *p : drop) (void)hipFree(p);
                lk.lock();
                progressed = true;
                continue;
            }
            if (!any_busy) {
                // no job runs and no idle workspace is left: the head job cannot fit
                S.queue.pop_front();
                head->status = BBC_ENOMEM;
                head->err = "job workspace does not fit the HBM budget beside the resident propagator sets";
                finish_job(S, *head, JOB_FAILED);
                progressed = true;
                continue;
            }
            break;   // wait for running jobs to free memory
        }
        Job *j = S.queue[pick];
        S.queue.erase(S.queue.begin() + (long)pick);
        if (pick > 0) head->bypassed++;
        j->state = JOB_RUNNING;
        j->t_start = Clock::now();
        slot->reserved = true;
        bool ok = true;
        // the slot is idle: its graphs may go (a new workspace, or a full cache)
        if (j->foot > slot->ws_bytes || slot->graphs.size() >= 16) slot->clear_graphs();
        if (j->foot > slot->ws_bytes) {
            void *old = slot->ws;
            S.committed += j->foot - slot->ws_bytes;
            slot->ws = nullptr;
            slot->ws_bytes = 0;
            lk.unlock();
            if (old) (void)hipFree(old);
            void *p = nullptr;
            ok = hipMalloc(&p, j->foot) == hipSuccess;
            lk.lock();
            if (ok) { slot->ws = p; slot->ws_bytes = j->foot; }
            else S.committed -= j->foot;
        }
        slot->reserved = false;
        if (!ok) {
            j->status = BBC_ENOMEM;
            j->err = "hipMalloc of a job workspace failed";
            finish_job(S, *j, JOB_FAILED);
            progressed = true;
            continue;
        }
        if (!j->energy.empty()) {
            const PropSet &ps = *j->ps;
            const long V = (long)ps.L[0] * ps.L[1] * ps.L[2];
            const size_t wsz = workspace_bytes(V, j->dp->plan.ncomp, (int)j->chans.size(), j->dp->npair,
                                               ps.prec == BBC_F64 ? 16 : 8);
            (void)hipMemcpyAsync((char *)slot->ws + ((wsz + 255) & ~(size_t)255), j->energy.data(),
                                 8 * j->energy.size(), hipMemcpyHostToDevice, slot->st);
        }
        slot->job = j;
        progressed = true;
    }
    return progressed;
}

// Continuous batching: every slot advances its job one time slice at a time
// (at most two slices in flight per slot); as soon as a slot is free, the
// next queued job is admitted if its workspace fits the context budget.
// Slots run on separate streams, so the slices of different jobs overlap on
// the device.  Results do not depend on the mix: each slice uses its own
// slot workspace and the same kernels and reduction order as when alone.
void server_loop(bbc_context *ctx) {
    Server &S = ctx->srv;
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(S.mu);
    for (;;) {
        bool progressed = false;
        for (auto &sl : S.slots) {
            Job *j = sl.job;
            if (!j) continue;
            while (!sl.evs.empty() && hipEventQuery(sl.evs.front()) == hipSuccess) {
                S.evpool.push_back(sl.evs.front());
                sl.evs.pop_front();
                j->inflight--;
                progressed = true;
            }
            while (!j->cancel && j->state == JOB_RUNNING && j->inflight < 2 && j->next < (int)j->slice.size()) {
                bbc_status st = server_enqueue(ctx, sl, *j);
                if (st != BBC_OK) {
                    j->status = st;
                    j->err = g_err;
                    j->state = JOB_FAILED;
                    break;
                }
                hipEvent_t ev = nullptr;
                if (!S.evpool.empty()) { ev = S.evpool.back(); S.evpool.pop_back(); }
                else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
                if (!ev || hipEventRecord(ev, sl.st) != hipSuccess) {
                    j->status = BBC_EDEVICE;
                    j->err = "event record failed";
                    j->state = JOB_FAILED;
                    if (ev) S.evpool.push_back(ev);
                    break;
                }
                sl.evs.push_back(ev);
                j->next++;
                j->inflight++;
                progressed = true;
            }
            if (j->inflight == 0 && (j->next == (int)j->slice.size() || j->cancel || j->state == JOB_FAILED)) {
                int final_state = j->state == JOB_FAILED ? JOB_FAILED
                                  : (j->cancel && j->next < (int)j->slice.size()) ? JOB_CANCELLED : JOB_DONE;
                finish_job(S, *j, final_state);
                sl.job = nullptr;
                progressed = true;
            }
        }
        if (admit_jobs(ctx, lk)) progressed = true;
        bool idle = S.queue.empty();
        for (auto &sl : S.slots) idle = idle && !sl.job;
        if (S.stop && idle) break;
        if (!progressed) S.cv.wait_for(lk, std::chrono::microseconds(50));
    }
}

}  // namespace

// ---------------------------------------------------------------- allocation-free entry point
namespace {
// Scratch of bbc_correlate_noalloc: a file-scope device array, one copy on every
// GPU the library runs on, held until the process ends.  In host code the
// array's name is not a device address: a GPU's copy is reached only through
// the address hipGetSymbolAddress returns with that GPU current, taken once per
// device (bbc_create) and kept here.
constexpr size_t kScratchBytes = (size_t)192 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;           // device -> address of its copy

bbc_status scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) { *out = it->second; return BBC_OK; }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(BBC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr.emplace(device, p);
    *out = p;
    return BBC_OK;
}
}  // namespace

namespace {
bbc_status load_tuning(bbc_context *ctx, const std::string &path);
}

extern "C" {

int bbc_num_channels(void) { return bbc::kNumChannels; }
int bbc_num_channels_all(void) { return bbc::kNumChannelsAll; }

const char *bbc_channel_name(int channel) {
    // names are made on first request and kept (map nodes do not move)
    static std::mutex mu;
    static std::map<int, std::string> names;
    if (!bbc::channel_valid(channel)) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = names.find(channel);
    if (it == names.end()) it = names.emplace(channel, bbc::channel_name(channel)).first;
    return it->second.c_str();
}

int bbc_num_baryons(void) { return bbc::kNumBaryons; }

const char *bbc_baryon_name(int b) {
    if (b < 0 || b >= bbc::kNumBaryons) return nullptr;
    return bbc::baryon(b).name;
}

int bbc_channel_id(int b1, int b2, int b3, int b4) {
    const int b[4] = {b1, b2, b3, b4};
    for (int i = 0; i < 4; ++i)
        if (b[i] < 0 || b[i] >= bbc::kNumBaryons) return fail(BBC_EINVAL, "baryon index out of range");
    const int id = bbc::channel_id(b);
    if (!bbc::channel_valid(id)) return fail(BBC_EINVAL, "the sink and source differ in quark content");
    return id;
}

bbc_status bbc_channel_content(int channel, int *n_light, int *n_strange) {
    if (!bbc::channel_valid(channel)) return fail(BBC_EINVAL, "channel index out of range or flavour not conserved");
    if (!n_light || !n_strange) return fail(BBC_EINVAL, "NULL output");
    const auto b = bbc::channel_baryons(channel);
    int ns = 0;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 3; ++i) ns += bbc::baryon(b[s]).flav[i] == bbc::FS;
    *n_strange = ns;
    *n_light = 6 - ns;
    return BBC_OK;
}

bbc_status bbc_source_terms(int channel, int *n3, int *n4) {
    if (!bbc::channel_valid(channel)) return fail(BBC_EINVAL, "channel index out of range or flavour not conserved");
    if (!n3 || !n4) return fail(BBC_EINVAL, "NULL output");
    const auto b = bbc::channel_baryons(channel);
    *n3 = bbc::baryon(b[2]).nterm;
    *n4 = bbc::baryon(b[3]).nterm;
    return BBC_OK;
}

bbc_status bbc_diagram_table(int channel, int term3, int term4, int max_diagrams, int *n_diagrams, int32_t *K,
                             int32_t *sign) {
    if (!bbc::channel_valid(channel)) return fail(BBC_EINVAL, "channel index out of range or flavour not conserved");
    const auto b = bbc::channel_baryons(channel);
    if (term3 < 0 || term3 >= bbc::baryon(b[2]).nterm || term4 < 0 || term4 >= bbc::baryon(b[3]).nterm)
        return fail(BBC_EINVAL, "source term index out of range");
    if (!n_diagrams) return fail(BBC_EINVAL, "NULL output");
    try {
        auto ds = bbc::classify(channel, term3, term4, nullptr, nullptr);
        *n_diagrams = (int)ds.size();
        if ((int)ds.size() > max_diagrams || !K || !sign) return fail(BBC_EINVAL, "output arrays too small");
        for (size_t i = 0; i < ds.size(); ++i) { K[i] = ds[i].K; sign[i] = ds[i].sign; }
    } catch (const std::exception &e) {
        return fail(BBC_EINVAL, e.what());
    }
    return BBC_OK;
}

bbc_status bbc_plan_stats(int n_ch, const int32_t *ch_list, int64_t *n_inter, int64_t *n_comp, int64_t *n_terms,
                          int64_t *n_iter) {
    if (n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list");
    std::vector<int> chans(ch_list, ch_list + n_ch);
    try {
        bbc::Plan P = bbc::build_plan(chans, 0);
        if (n_inter) *n_inter = (int64_t)P.inters.size();
        if (n_comp) *n_comp = 2 * (int64_t)P.ncomp;
        if (n_terms) *n_terms = (int64_t)P.diags.size();
        if (n_iter) *n_iter = P.iterations;
    } catch (const std::exception &e) {
        return fail(BBC_EINVAL, e.what());
    }
    return BBC_OK;
}

bbc_status bbc_pair_stats(int n_ch, const int32_t *ch_list, int64_t *n_pairs, int64_t *n_tasks, int64_t *items,
                          int64_t *n_weights) {
    if (n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list");
    std::vector<int> chans(ch_list, ch_list + n_ch);
    try {
        const bbc::Plan P = bbc::build_plan(chans, 0);
        const bbc::PairTables T = bbc::build_pair_tables(P);
        if (n_pairs) *n_pairs = T.npair;
        if (n_tasks) *n_tasks = (int64_t)T.tasks.size();
        if (items) *items = T.pair_items;
        if (n_weights) *n_weights = (int64_t)T.term_pair.size();
    } catch (const std::exception &e) {
        return fail(BBC_EINVAL, e.what());
    }
    return BBC_OK;
}

const char *bbc_last_error(void) { return g_err.c_str(); }

bbc_status bbc_create(int device, uint64_t budget, bbc_context **out) {
    if (!out) return fail(BBC_EINVAL, "NULL output");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(BBC_EINVAL, "no HIP device " + std::to_string(device));
    HIP_TRY(hipSetDevice(device));
    void *scr = nullptr;
    bbc_status s = scratch_address(device, &scr);   // with the device current
    if (s) return s;
    bbc_context *c = new (std::nothrow) bbc_context;
    if (!c) return fail(BBC_ENOMEM, "context allocation");
    c->device = device;
    c->budget = budget;
    c->scratch = scr;
    // tuning file: loaded if present, rewritten by bbc_autotune
    if (const char *tp = std::getenv("BBC_TUNING_CACHE")) {
        if (*tp) {
            c->tune_path = tp;
            if (std::ifstream(tp).good()) {
                bbc_status ts = load_tuning(c, tp);
                if (ts) { delete c; return ts; }
            }
        }
    }
    *out = c;
    return BBC_OK;
}

void bbc_destroy(bbc_context *ctx) {
    if (!ctx) return;
    (void)bbc_server_stop(ctx);
    (void)hipSetDevice(ctx->device);
    for (auto &kv : ctx->srv.props) { (void)hipFree(kv.second->dl); (void)hipFree(kv.second->ds); }
    ctx->srv.props.clear();
    (void)hipDeviceSynchronize();
    ctx->plans.clear();
    delete ctx;
}

bbc_status bbc_footprint(const int32_t lattice[3], bbc_precision prec, int n_ch, const int32_t *ch_list,
                         uint64_t *bytes) {
    long V;
    bbc_status s = check_lattice(lattice, &V);
    if (s) return s;
    if (n_ch <= 0 || !ch_list || !bytes) return fail(BBC_EINVAL, "bad channel list or output");
    std::vector<int> chans(ch_list, ch_list + n_ch);
    try {
        bbc::Plan P = bbc::build_plan(chans, 0);
        const bbc::PairTables pt = bbc::build_pair_tables(P);
        *bytes = workspace_bytes(V, P.ncomp, n_ch, pt.npair, prec == BBC_F64 ? 16 : 8);
    } catch (const std::exception &e) {
        return fail(BBC_EINVAL, e.what());
    }
    return BBC_OK;
}

bbc_status bbc_correlate(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, const void *S_light,
                         const void *S_strange, int n_t, const int32_t *t_list, int t0, int n_ch,
                         const int32_t *ch_list, bbc_spin spin, const double *energy, void *C_out, double *C_scale,
                         void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_lattice(lattice, &V);
    if (s) return s;
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (spin != BBC_SPIN_UPPER && spin != BBC_SPIN_LOWER && spin != BBC_SPIN_FULL)
        return fail(BBC_EINVAL, "spin selection");
    if (n_t < 0 || n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list or negative n_t");
    if (n_t > 0 && (!S_light || !S_strange || !t_list || !C_out)) return fail(BBC_EINVAL, "NULL buffer");
    if (prec == BBC_F32 && n_t > 0 && !C_scale) return fail(BBC_EINVAL, "C_scale is required in FP32 mode");
    for (int i = 0; i < n_ch; ++i)
        if (!bbc::channel_valid(ch_list[i]))
            return fail(BBC_EINVAL, "channel index " + std::to_string(ch_list[i]) + " out of range");
    if (n_t == 0) return BBC_OK;
    const bool host_in = is_host_pointer(S_light), host_out = is_host_pointer(C_out);
    if (is_host_pointer(S_strange) != host_in)
        return fail(BBC_EINVAL, "S_light and S_strange must both be host or both be device memory");
    if (C_scale && is_host_pointer(C_scale)) return fail(BBC_EINVAL, "C_scale must be device memory");
    if (spin == BBC_SPIN_FULL && host_out) return fail(BBC_EINVAL, "BBC_SPIN_FULL needs C_out in device memory");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<int> chans(ch_list, ch_list + n_ch);
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    hipStream_t st = (hipStream_t)stream;
    DevPlan *dp = nullptr;
    if (spin == BBC_SPIN_FULL) {
        // 16 evaluations, one per choice of upper or lower pair for each baryon,
        // each writing its 16 components into the 256-value layout
        if ((s = order_after_last(ctx, st))) return s;
        for (int sub = 0; sub < 16 && !s; ++sub) {
            if ((s = get_plan(ctx, chans, 0, prec, &dp, true, sub))) break;
            if (prec == BBC_F64)
                s = run_correlate<double>(ctx, dp, L, V, S_light, S_strange, n_t, t_list, t0, n_ch, energy, C_out,
                                          nullptr, st, host_in, false);
            else
                s = run_correlate<float>(ctx, dp, L, V, S_light, S_strange, n_t, t_list, t0, n_ch, energy, C_out,
                                         C_scale, st, host_in, false);
        }
        return mark_last(ctx, st, s);
    }
    s = get_plan(ctx, chans, spin == BBC_SPIN_LOWER ? 2 : 0, prec, &dp);
    if (s) return s;
    if ((s = order_after_last(ctx, st))) return s;
    if (prec == BBC_F64)
        s = run_correlate<double>(ctx, dp, L, V, S_light, S_strange, n_t, t_list, t0, n_ch, energy, C_out, nullptr,
                                  st, host_in, host_out);
    else
        s = run_correlate<float>(ctx, dp, L, V, S_light, S_strange, n_t, t_list, t0, n_ch, energy, C_out, C_scale,
                                 st, host_in, host_out);
    return mark_last(ctx, st, s);
}


bbc_status bbc_correlate_noalloc(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, const void *S_light,
                                 const void *S_strange, int n_t, const int32_t *t_list, int t0, int n_ch,
                                 const int32_t *ch_list, bbc_spin spin, const double *energy, void *C_out,
                                 double *C_scale, void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_lattice(lattice, &V);
    if (s) return s;
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (spin != BBC_SPIN_UPPER && spin != BBC_SPIN_LOWER) return fail(BBC_EINVAL, "spin selection");
    if (n_t < 0 || n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list or negative n_t");
    if (n_t > 0 && (!S_light || !S_strange || !t_list || !C_out)) return fail(BBC_EINVAL, "NULL buffer");
    if (prec == BBC_F32 && n_t > 0 && !C_scale) return fail(BBC_EINVAL, "C_scale is required in FP32 mode");
    for (int i = 0; i < n_ch; ++i)
        if (!bbc::channel_valid(ch_list[i]))
            return fail(BBC_EINVAL, "channel index " + std::to_string(ch_list[i]) + " out of range");
    if (n_t == 0) return BBC_OK;
    if (is_host_pointer(S_light) || is_host_pointer(S_strange) || is_host_pointer(C_out) ||
        (C_scale && is_host_pointer(C_scale)))
        return fail(BBC_EINVAL, "bbc_correlate_noalloc takes device memory only");
    if (!ctx->scratch) return fail(BBC_ESTATE, "no scratch address for the context's device");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<int> chans(ch_list, ch_list + n_ch);
    DevPlan *dp = nullptr;
    if ((s = get_plan(ctx, chans, spin == BBC_SPIN_LOWER ? 2 : 0, prec, &dp, false))) return s;
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    auto gk = std::vector<int>{L[0], L[1], L[2]};
    auto git = ctx->group_images.find(gk);
    if (git == ctx->group_images.end()) {
        long npos = 0;
        std::vector<int2> img = group_image(L, &npos);
        git = ctx->group_images.emplace(gk, std::make_pair(std::move(img), npos)).first;
    }
    const std::vector<int2> &gimg = git->second.first;
    const long npos = git->second.second;
    // scratch layout: plan tables, momentum groups, energies, slice workspace
    const size_t cs = prec == BBC_F64 ? 16 : 8;
    const size_t off_grp = align256(dp->image.size());
    const size_t off_en = align256(off_grp + gimg.size() * sizeof(int2));
    const size_t off_ws = align256(off_en + sizeof(double) * n_ch);
    const size_t need = off_ws + workspace_bytes(V, dp->plan.ncomp, n_ch, dp->npair, cs);
    if (need > kScratchBytes)
        return fail(BBC_ENOMEM, "request needs " + std::to_string(need) + " bytes of scratch; the allocation-free "
                                "entry point holds at most " + std::to_string(kScratchBytes) + " bytes (192 MiB)");
    char *sc = (char *)ctx->scratch;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(sc, dp->image.data(), dp->image.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sc + off_grp, gimg.data(), gimg.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    if (energy) {
        ctx->noalloc_energy.assign(energy, energy + n_ch);
        HIP_TRY(hipMemcpyAsync(sc + off_en, ctx->noalloc_energy.data(), sizeof(double) * n_ch, hipMemcpyHostToDevice,
                               st));
    }
    const PlanDev pd = plan_dev(dp, sc);
    const MomGroups mg = groups_at((const int2 *)(sc + off_grp), npos, L);
    const double *d_en = energy ? (const double *)(sc + off_en) : nullptr;
    const size_t in_slice = (size_t)V * 144, out_slice = (size_t)n_ch * V * 16;
    for (int n = 0; n < n_t; ++n) {
        const double dt = (double)(t_list[n] - t0);
        if (prec == BBC_F64) {
            const double2 *sl = (const double2 *)S_light + n * in_slice, *ss = (const double2 *)S_strange + n * in_slice;
            s = enqueue_slice<double>(ctx, pd, L, V, sc + off_ws, mg, sl, ss, n_ch, d_en, dt,
                                      (double2 *)C_out + n * out_slice, nullptr, st, false);
        } else {
            const float2 *sl = (const float2 *)S_light + n * in_slice, *ss = (const float2 *)S_strange + n * in_slice;
            s = enqueue_slice<float>(ctx, pd, L, V, sc + off_ws, mg, sl, ss, n_ch, d_en, dt,
                                     (float2 *)C_out + n * out_slice, C_scale + (size_t)n * n_ch, st, false);
        }
        if (s) return s;
    }
    return BBC_OK;
}

bbc_status bbc_correlate_cpt(bbc_context *ctx, const int32_t lattice[3], int Lt, bbc_precision prec,
                             const void *S_light, const void *S_strange, int t0, int n_tau, const int32_t *tau_list,
                             int n_ch, const int32_t *ch_list, int sign, const double *energy, void *R_out,
                             double *R_scale, void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_lattice(lattice, &V);
    if (s) return s;
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (Lt < 1) return fail(BBC_EINVAL, "Lt must be positive");
    if (sign != 1 && sign != -1) return fail(BBC_EINVAL, "sign must be +1 or -1");
    if (n_tau < 0 || n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list or negative n_tau");
    for (int i = 0; i < n_ch; ++i)
        if (!bbc::channel_valid(ch_list[i]))
            return fail(BBC_EINVAL, "channel index " + std::to_string(ch_list[i]) + " out of range");
    if (n_tau == 0) return BBC_OK;
    if (!S_light || !S_strange || !tau_list || !R_out) return fail(BBC_EINVAL, "NULL buffer");
    if (prec == BBC_F32 && !R_scale) return fail(BBC_EINVAL, "R_scale is required in FP32 mode");
    if (t0 < 0 || t0 >= Lt) return fail(BBC_EINVAL, "t0 outside [0, Lt)");
    for (int n = 0; n < n_tau; ++n)
        if (tau_list[n] < 0 || tau_list[n] >= Lt) return fail(BBC_EINVAL, "tau outside [0, Lt)");
    if (is_host_pointer(S_light) || is_host_pointer(S_strange) || is_host_pointer(R_out) ||
        (R_scale && is_host_pointer(R_scale)))
        return fail(BBC_EINVAL, "bbc_correlate_cpt takes device memory only");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<int> chans(ch_list, ch_list + n_ch);
    DevPlan *up = nullptr, *lo = nullptr;
    if ((s = get_plan(ctx, chans, 0, prec, &up))) return s;
    if ((s = get_plan(ctx, chans, 2, prec, &lo))) return s;
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(ctx, st))) return s;
    if (prec == BBC_F64)
        s = run_cpt<double>(ctx, up, lo, L, V, Lt, S_light, S_strange, t0, n_tau, tau_list, n_ch, energy, sign,
                            R_out, nullptr, st);
    else
        s = run_cpt<float>(ctx, up, lo, L, V, Lt, S_light, S_strange, t0, n_tau, tau_list, n_ch, energy, sign,
                           R_out, R_scale, st);
    return mark_last(ctx, st, s);
}

bbc_status bbc_server_start(bbc_context *ctx, int n_slots) {
    if (!ctx || n_slots < 1 || n_slots > 16) return fail(BBC_EINVAL, "n_slots must be 1..16");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.running) return fail(BBC_ESTATE, "server already running");
    HIP_TRY(hipSetDevice(ctx->device));
    S.slots.assign(n_slots, Slot());
    for (auto &sl : S.slots) {
        HIP_TRY(hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking));
        HIP_TRY(hipMalloc((void **)&sl.d_args, sizeof(bbc::SliceArgs)));
    }
    S.stop = false;
    S.running = true;
    S.th = std::thread(server_loop, ctx);
    return BBC_OK;
}

bbc_status bbc_server_stop(bbc_context *ctx) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (!S.running) return BBC_OK;
        for (Job *j : S.queue) finish_job(S, *j, JOB_CANCELLED);
        S.queue.clear();
        S.stop = true;
        S.cv.notify_all();
    }
    S.th.join();
    std::lock_guard<std::mutex> lk(S.mu);
    for (auto &sl : S.slots) {
        (void)hipStreamSynchronize(sl.st);
        for (auto e : sl.evs) (void)hipEventDestroy(e);
        sl.clear_graphs();
        (void)hipStreamDestroy(sl.st);
        if (sl.d_args) (void)hipFree(sl.d_args);
        if (sl.ws) { (void)hipFree(sl.ws); S.committed -= sl.ws_bytes; }
    }
    S.slots.clear();
    for (auto e : S.evpool) (void)hipEventDestroy(e);
    S.evpool.clear();
    if (S.cap) { (void)hipStreamDestroy(S.cap); S.cap = nullptr; }
    S.running = false;
    return BBC_OK;
}

bbc_status bbc_prop_upload(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, const void *S_light,
                           const void *S_strange, int n_t, uint64_t *handle) {
    if (!ctx || !handle || !S_light || !S_strange || n_t < 1) return fail(BBC_EINVAL, "bad prop_upload arguments");
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    long V;
    bbc_status s = check_lattice(lattice, &V);
    if (s) return s;
    Server &S = ctx->srv;
    std::unique_ptr<PropSet> ps(new PropSet);
    for (int i = 0; i < 3; ++i) ps->L[i] = lattice[i];
    ps->prec = prec;
    ps->n_t = n_t;
    const size_t one = (size_t)n_t * V * 144 * (prec == BBC_F64 ? 16 : 8);
    ps->bytes = 2 * one;
    {
        // the bytes are reserved before allocating, so concurrent uploads cannot
        // both pass the budget check
        std::lock_guard<std::mutex> lk(S.mu);
        if (ctx->budget && S.committed + ps->bytes > ctx->budget)
            return fail(BBC_ENOMEM, "propagator set exceeds the HBM budget");
        S.committed += ps->bytes;
    }
    auto unreserve = [&](bbc_status st) {
        (void)hipFree(ps->dl);
        (void)hipFree(ps->ds);
        std::lock_guard<std::mutex> lk(S.mu);
        S.committed -= ps->bytes;
        return st;
    };
    if (hipSetDevice(ctx->device) != hipSuccess) return unreserve(fail(BBC_EDEVICE, "hipSetDevice"));
    if (hipMalloc(&ps->dl, one) != hipSuccess || hipMalloc(&ps->ds, one) != hipSuccess)
        return unreserve(fail(BBC_ENOMEM, "hipMalloc of a propagator set failed"));
    const hipMemcpyKind kl = is_host_pointer(S_light) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind ks = is_host_pointer(S_strange) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpy(ps->dl, S_light, one, kl);
    if (e == hipSuccess) e = hipMemcpy(ps->ds, S_strange, one, ks);
    if (e != hipSuccess) return unreserve(fail(BBC_EDEVICE, std::string("propagator copy: ") + hipGetErrorString(e)));
    std::lock_guard<std::mutex> lk(S.mu);
    *handle = S.next_id++;
    S.props.emplace(*handle, std::move(ps));
    return BBC_OK;
}

bbc_status bbc_prop_release(bbc_context *ctx, uint64_t handle) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.props.find(handle);
    if (it == S.props.end() || it->second->released) return fail(BBC_EINVAL, "unknown propagator handle");
    it->second->released = true;
    release_prop_if_unused(S, it->second.get());
    return BBC_OK;
}

bbc_status bbc_submit(bbc_context *ctx, uint64_t prop, int n_t, const int32_t *slice_idx, const int32_t *t_list,
                      int t0, int n_ch, const int32_t *ch_list, bbc_spin spin, const double *energy, void *C_out,
                      double *C_scale, uint64_t *job) {
    if (!ctx || !job || n_t < 1 || !slice_idx || !t_list || n_ch < 1 || !ch_list || !C_out)
        return fail(BBC_EINVAL, "bad submit arguments");
    if (spin != BBC_SPIN_UPPER && spin != BBC_SPIN_LOWER) return fail(BBC_EINVAL, "spin selection");
    for (int i = 0; i < n_ch; ++i)
        if (!bbc::channel_valid(ch_list[i])) return fail(BBC_EINVAL, "channel index out of range");
    Server &S = ctx->srv;
    std::unique_ptr<Job> j(new Job);
    {
        // the reference is taken under the lock, so a concurrent bbc_prop_release
        // cannot free the set between lookup and use
        std::lock_guard<std::mutex> lk(S.mu);
        if (!S.running) return fail(BBC_ESTATE, "server not started");
        auto it = S.props.find(prop);
        if (it == S.props.end() || it->second->released) return fail(BBC_EINVAL, "unknown propagator handle");
        j->ps = it->second.get();
        j->ps->refs++;
    }
    // drops the reference on every early return
    auto drop = [&](bbc_status st) {
        std::lock_guard<std::mutex> lk(S.mu);
        j->ps->refs--;
        release_prop_if_unused(S, j->ps);
        return st;
    };
    if (j->ps->prec == BBC_F32 && !C_scale) return drop(fail(BBC_EINVAL, "C_scale is required in FP32 mode"));
    if (is_host_pointer(C_out) || (C_scale && j->ps->prec == BBC_F32 && is_host_pointer(C_scale)))
        return drop(fail(BBC_EINVAL, "C_out and C_scale of a served job must be device memory"));
    for (int i = 0; i < n_t; ++i)
        if (slice_idx[i] < 0 || slice_idx[i] >= j->ps->n_t) return drop(fail(BBC_EINVAL, "slice index out of range"));
    j->slice.assign(slice_idx, slice_idx + n_t);
    j->tl.assign(t_list, t_list + n_t);
    j->t0 = t0;
    j->chans.assign(ch_list, ch_list + n_ch);
    j->spin = spin;
    if (energy) j->energy.assign(energy, energy + n_ch);
    j->out = C_out;
    j->scale = j->ps->prec == BBC_F32 ? C_scale : nullptr;
    bbc_status s = get_plan(ctx, j->chans, spin == BBC_SPIN_LOWER ? 2 : 0, (bbc_precision)j->ps->prec, &j->dp);
    if (s) return drop(s);
    j->foot = job_footprint(*j);
    // a job that cannot fit beside its own propagator set can never run
    if (ctx->budget && j->foot + j->ps->bytes > ctx->budget)
        return drop(fail(BBC_ENOMEM, "job workspace and its propagator set exceed the HBM budget"));
    std::lock_guard<std::mutex> lk(S.mu);
    j->id = S.next_id++;
    j->t_submit = Clock::now();
    *job = j->id;
    S.queue.push_back(j.get());
    S.jobs.emplace(j->id, std::move(j));
    S.cv.notify_all();
    return BBC_OK;
}

bbc_status bbc_poll(bbc_context *ctx, uint64_t job, int *state) {
    if (!ctx || !state) return fail(BBC_EINVAL, "bad poll arguments");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.jobs.find(job);
    if (it == S.jobs.end()) return fail(BBC_EINVAL, "unknown job");
    *state = it->second->state;
    return BBC_OK;
}

bbc_status bbc_wait(bbc_context *ctx, uint64_t job, int timeout_ms) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.jobs.find(job);
    if (it == S.jobs.end()) return fail(BBC_EINVAL, "unknown job");
    Job *j = it->second.get();
    auto pred = [j] { return j->state >= JOB_DONE; };
    if (timeout_ms < 0) S.done_cv.wait(lk, pred);
    else if (!S.done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
        return fail(BBC_ETIMEOUT, "job not finished within the timeout");
    if (j->state == JOB_CANCELLED) return fail(BBC_ECANCELLED, "job cancelled");
    if (j->state == JOB_FAILED) return fail(j->status, j->err);
    return BBC_OK;
}

bbc_status bbc_cancel(bbc_context *ctx, uint64_t job) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.jobs.find(job);
    if (it == S.jobs.end()) return fail(BBC_EINVAL, "unknown job");
    Job *j = it->second.get();
    if (j->state == JOB_QUEUED) {
        for (auto q = S.queue.begin(); q != S.queue.end(); ++q)
            if (*q == j) { S.queue.erase(q); break; }
        finish_job(S, *j, JOB_CANCELLED);
    } else if (j->state == JOB_RUNNING) {
        j->cancel = true;
        S.cv.notify_all();
    }
    return BBC_OK;
}

bbc_status bbc_job_times(bbc_context *ctx, uint64_t job, double *queue_ms, double *run_ms, double *total_ms) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.jobs.find(job);
    if (it == S.jobs.end()) return fail(BBC_EINVAL, "unknown job");
    const Job &j = *it->second;
    if (j.state < JOB_DONE) return fail(BBC_ESTATE, "job not finished");
    auto ms = [](Clock::time_point a, Clock::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const bool started = j.t_start.time_since_epoch().count() != 0;
    if (queue_ms) *queue_ms = ms(j.t_submit, started ? j.t_start : j.t_done);
    if (run_ms) *run_ms = started ? ms(j.t_start, j.t_done) : 0.0;
    if (total_ms) *total_ms = ms(j.t_submit, j.t_done);
    return BBC_OK;
}

bbc_status bbc_job_forget(bbc_context *ctx, uint64_t job) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    Server &S = ctx->srv;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.jobs.find(job);
    if (it == S.jobs.end()) return fail(BBC_EINVAL, "unknown job");
    if (it->second->state < JOB_DONE) return fail(BBC_ESTATE, "job not finished");
    S.jobs.erase(it);
    return BBC_OK;
}

bbc_status bbc_graph_mode(bbc_context *ctx, int enable) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    ctx->graph_mode = enable != 0;
    if (!ctx->graph_mode) {
        HIP_TRY(hipDeviceSynchronize());
        ctx->clear_graphs();
    }
    return BBC_OK;
}

bbc_status bbc_profile_enable(bbc_context *ctx, int enable) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->prof = enable != 0;
    return BBC_OK;
}

bbc_status bbc_profile_read(bbc_context *ctx, int n_stages, double *ms, int64_t *launches) {
    if (!ctx || !ms || !launches || n_stages < 1 || n_stages > BBC_NUM_STAGES)
        return fail(BBC_EINVAL, "bad profile_read arguments");
    std::lock_guard<std::mutex> lock(ctx->mu);
    for (int i = 0; i < n_stages; ++i) { ms[i] = 0; launches[i] = 0; }
    HIP_TRY(hipSetDevice(ctx->device));
    bbc_status st = BBC_OK;
    for (auto &r : ctx->recs) {
        float t = 0;
        if (st == BBC_OK) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
            if (e != hipSuccess) st = fail(BBC_EDEVICE, std::string("profile: ") + hipGetErrorString(e));
        }
        if (r.stage < n_stages) { ms[r.stage] += t; launches[r.stage] += r.nk; }
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------- post-processing
namespace {
bbc_status check_extents(const int32_t *lattice, long *V) {
    if (!lattice) return fail(BBC_EINVAL, "lattice is NULL");
    long v = 1;
    for (int i = 0; i < 3; ++i) {
        if (lattice[i] < 1) return fail(BBC_EINVAL, "lattice extent must be positive");
        v *= lattice[i];
    }
    if (v > (1L << 30)) return fail(BBC_EUNSUPPORTED, "lattice volume too large");
    *V = v;
    return BBC_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" {

bbc_status bbc_spin_project(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_fields,
                            const void *in, int n_out, const double *W, void *out, void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_extents(lattice, &V);
    if (s) return s;
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (n_fields < 0 || n_out < 1 || n_out > 16) return fail(BBC_EINVAL, "n_fields >= 0 and 1 <= n_out <= 16");
    if (!W) return fail(BBC_EINVAL, "NULL weights");
    if (n_fields == 0) return BBC_OK;
    if (!in || !out) return fail(BBC_EINVAL, "NULL buffer");
    if (is_host_pointer(in) || is_host_pointer(out)) return fail(BBC_EINVAL, "in and out must be device memory");
    const size_t cs = prec == BBC_F64 ? 16 : 8;
    const long nsite = (long)n_fields * V;
    if (overlap(in, nsite * 16 * cs, out, nsite * n_out * cs)) return fail(BBC_EINVAL, "in and out overlap");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (prec == BBC_F64)
        bbc::launch_spin_project<double>((const double2 *)in, (double2 *)out, nsite, n_out, W, st);
    else
        bbc::launch_spin_project<float>((const float2 *)in, (float2 *)out, nsite, n_out, W, st);
    HIP_TRY(hipGetLastError());
    return BBC_OK;
}

bbc_status bbc_cubic_project(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_fields, int n_comp,
                             const void *in, int mode, void *out, void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_extents(lattice, &V);
    if (s) return s;
    if (lattice[0] != lattice[1] || lattice[1] != lattice[2])
        return fail(BBC_EUNSUPPORTED, "the cubic-group projection needs a cubic lattice");
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (mode != BBC_CUBIC_A1 && mode != BBC_CUBIC_A1_COMPLEMENT) return fail(BBC_EINVAL, "mode");
    if (n_fields < 0 || n_comp < 1) return fail(BBC_EINVAL, "n_fields >= 0 and n_comp >= 1");
    if (n_fields == 0) return BBC_OK;
    if (!in || !out) return fail(BBC_EINVAL, "NULL buffer");
    if (is_host_pointer(in) || is_host_pointer(out)) return fail(BBC_EINVAL, "in and out must be device memory");
    const size_t cs = prec == BBC_F64 ? 16 : 8;
    const size_t bytes = (size_t)n_fields * V * n_comp * cs;
    if (overlap(in, bytes, out, bytes)) return fail(BBC_EINVAL, "in and out overlap");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    const int cmp = mode == BBC_CUBIC_A1_COMPLEMENT;
    if (prec == BBC_F64)
        bbc::launch_cubic_project<double>((const double2 *)in, (double2 *)out, n_fields, lattice[0], n_comp, cmp, st);
    else
        bbc::launch_cubic_project<float>((const float2 *)in, (float2 *)out, n_fields, lattice[0], n_comp, cmp, st);
    HIP_TRY(hipGetLastError());
    return BBC_OK;
}

bbc_status bbc_central_potential(bbc_context *ctx, const int32_t lattice[3], int n_fields, int n_t, const void *R,
                                 double inv_2mu, void *V_out, void *stream) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_extents(lattice, &V);
    if (s) return s;
    if (n_fields < 0) return fail(BBC_EINVAL, "n_fields >= 0");
    if (n_t < 3) return fail(BBC_EINVAL, "the potential needs n_t >= 3 consecutive slices");
    if (n_fields == 0) return BBC_OK;
    if (!R || !V_out) return fail(BBC_EINVAL, "NULL buffer");
    if (is_host_pointer(R) || is_host_pointer(V_out)) return fail(BBC_EINVAL, "R and V must be device memory");
    if (overlap(R, (size_t)n_fields * n_t * V * 16, V_out, (size_t)n_fields * (n_t - 2) * V * 16))
        return fail(BBC_EINVAL, "R and V overlap");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    bbc::launch_central_potential((const double2 *)R, (double2 *)V_out, L, n_fields, n_t, inv_2mu,
                                  (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return BBC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Kernel variants per request shape, and the autotuner.
// ---------------------------------------------------------------------------
namespace {

bool tuning_valid(const bbc_tuning &t, bbc_precision prec) {
    const int np = prec == BBC_F64 ? bbc::kPairVariants64 : bbc::kPairVariants32;
    return t.pairs >= 0 && t.pairs < np && t.blocks >= 0 && t.blocks < bbc::kBlockVariants && t.planes >= 0 &&
           t.planes < bbc::kPlaneVariants && t.slices >= 0 && t.slices < bbc::kSliceVariants && t.combine >= 0 &&
           t.combine < bbc::kCombineVariants;
}

bbc_status check_request(const int32_t lattice[3], bbc_precision prec, int n_ch, const int32_t *ch_list,
                         bbc_spin spin, long *V) {
    bbc_status s = check_lattice(lattice, V);
    if (s) return s;
    if (prec != BBC_F64 && prec != BBC_F32) return fail(BBC_EINVAL, "precision");
    if (spin != BBC_SPIN_UPPER && spin != BBC_SPIN_LOWER) return fail(BBC_EINVAL, "spin selection");
    if (n_ch <= 0 || !ch_list) return fail(BBC_EINVAL, "empty channel list");
    for (int i = 0; i < n_ch; ++i)
        if (!bbc::channel_valid(ch_list[i]))
            return fail(BBC_EINVAL, "channel index " + std::to_string(ch_list[i]) + " out of range");
    return BBC_OK;
}

TuneKey request_key(const int32_t lattice[3], bbc_precision prec, int n_ch, const int32_t *ch_list, bbc_spin spin) {
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    return tune_key(L, (int)prec, spin == BBC_SPIN_LOWER ? 2 : 0,
                    channel_hash(std::vector<int>(ch_list, ch_list + n_ch)));
}

// Tuning file: one JSON object, {"bbc_tuning": 1, "entries": [...]}, each entry
// {"lattice": [Lx, Ly, Lz], "precision": 0|1, "spin_offset": 0|2,
//  "channel_hash": "<16 hex digits>", "pairs": p, "blocks": b, "planes": l}.
std::string tuning_json(const std::map<TuneKey, bbc::Tuning> &m) {
    std::ostringstream o;
    o << "{\"bbc_tuning\": 1, \"entries\": [";
    bool first = true;
    for (const auto &kv : m) {
        char hx[17];
        std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)kv.first[5]);
        o << (first ? "\n " : ",\n ") << "{\"lattice\": [" << kv.first[0] << ", " << kv.first[1] << ", "
          << kv.first[2] << "], \"precision\": " << kv.first[3] << ", \"spin_offset\": " << kv.first[4]
          << ", \"channel_hash\": \"" << hx << "\", \"pairs\": " << kv.second.pairs << ", \"blocks\": "
          << kv.second.blocks << ", \"planes\": " << kv.second.planes << ", \"slices\": " << kv.second.slices
          << ", \"combine\": " << kv.second.combine << "}";
        first = false;
    }
    o << "\n]}\n";
    return o.str();
}

// Integer value of "key": in text[from, to), or false.
bool json_int(const std::string &text, size_t from, size_t to, const char *key, long long *v) {
    const std::string k = std::string("\"") + key + "\":";
    size_t p = text.find(k, from);
    if (p == std::string::npos || p >= to) return false;
    p += k.size();
    while (p < to && text[p] == ' ') ++p;
    char *end = nullptr;
    *v = std::strtoll(text.c_str() + p, &end, 10);
    return end != text.c_str() + p;
}

bbc_status parse_tuning(const std::string &text, std::map<TuneKey, bbc::Tuning> *out) {
    if (text.find("\"bbc_tuning\": 1") == std::string::npos) return fail(BBC_EINVAL, "not a tuning file");
    size_t p = 0;
    while ((p = text.find("{\"lattice\": [", p)) != std::string::npos) {
        const size_t e = text.find('}', p);
        if (e == std::string::npos) return fail(BBC_EINVAL, "tuning file: unterminated entry");
        int L[3];
        if (std::sscanf(text.c_str() + p, "{\"lattice\": [%d, %d, %d]", &L[0], &L[1], &L[2]) != 3)
            return fail(BBC_EINVAL, "tuning file: lattice");
        long long prec, spin, pr, bl, pl, sl, cm;
        if (!json_int(text, p, e, "precision", &prec) || !json_int(text, p, e, "spin_offset", &spin) ||
            !json_int(text, p, e, "pairs", &pr) || !json_int(text, p, e, "blocks", &bl) ||
            !json_int(text, p, e, "planes", &pl) || !json_int(text, p, e, "slices", &sl) ||
            !json_int(text, p, e, "combine", &cm))
            return fail(BBC_EINVAL, "tuning file: missing field");
        const size_t h = text.find("\"channel_hash\": \"", p);
        if (h == std::string::npos || h > e) return fail(BBC_EINVAL, "tuning file: channel_hash");
        const uint64_t hash = std::strtoull(text.c_str() + h + 17, nullptr, 16);
        bbc_tuning t{(int32_t)pr, (int32_t)bl, (int32_t)pl, (int32_t)sl, (int32_t)cm};
        if ((prec != 0 && prec != 1) || (spin != 0 && spin != 2) || !tuning_valid(t, (bbc_precision)prec))
            return fail(BBC_EINVAL, "tuning file: value out of range");
        (*out)[tune_key(L, (int)prec, (int)spin, hash)] = bbc::Tuning{t.pairs, t.blocks, t.planes, t.slices, t.combine};
        p = e + 1;
    }
    return BBC_OK;
}

bbc_status save_tuning(bbc_context *ctx, const std::string &path) {
    std::string text;
    {
        std::lock_guard<std::mutex> lock(ctx->tmu);
        text = tuning_json(ctx->tuning);
    }
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return fail(BBC_EINVAL, "cannot write " + tmp);
        f << text;
        if (!f) return fail(BBC_EINVAL, "write failed: " + tmp);
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) return fail(BBC_EINVAL, "cannot replace " + path);
    return BBC_OK;
}

bbc_status load_tuning(bbc_context *ctx, const std::string &path) {
    std::ifstream f(path);
    if (!f) return fail(BBC_EINVAL, "cannot read " + path);
    std::stringstream ss;
    ss << f.rdbuf();
    std::map<TuneKey, bbc::Tuning> m;
    bbc_status s = parse_tuning(ss.str(), &m);
    if (s) return s;
    std::lock_guard<std::mutex> lock(ctx->tmu);
    for (const auto &kv : m) ctx->tuning[kv.first] = kv.second;
    return BBC_OK;
}

// Device time per slice of `reps` rounds of nb slices (one untimed round first)
// with the variants `tu`; every slice reads the same input, slice i writes
// outs[i].
template <typename T>
bbc_status time_variant(bbc_context *ctx, DevPlan *dp, const int L[3], long V, const MomGroups &mg, size_t stride,
                        const void *sl, const void *ss, int n_ch, int nb, void *const *outs, double *const *scales,
                        int reps, const bbc::Tuning &tu, hipStream_t st, hipEvent_t a, hipEvent_t b, float *ms) {
    const PlanDev pd = plan_dev(dp, dp->d_image);
    std::vector<const void *> vsl(nb, sl), vss(nb, ss);
    std::vector<double> dt(nb, 0.0);
    const int B = std::min(nb, 1 << tu.slices);
    auto round = [&]() {
        return enqueue_slices<T>(ctx, pd, L, V, (char *)ctx->ws, stride, B, mg, nb, vsl.data(), vss.data(), n_ch,
                                 nullptr, dt.data(), outs, scales, st, false, &tu);
    };
    bbc_status s = round();
    if (s) return s;
    HIP_TRY(hipEventRecord(a, st));
    for (int r = 0; r < reps && s == BBC_OK; ++r) s = round();
    if (s) return s;
    HIP_TRY(hipEventRecord(b, st));
    HIP_TRY(hipEventSynchronize(b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, a, b));
    *ms = e / (float)(reps * nb);
    return BBC_OK;
}

template <typename T>
bbc_status autotune(bbc_context *ctx, DevPlan *dp, const int L[3], long V, const void *sl, const void *ss, int n_ch,
                    int reps, hipStream_t st, bbc::Tuning *best, float *best_ms) {
    using T2 = typename bbc::cplx_t<T>::type;
    const size_t stride = (workspace_bytes(V, dp->plan.ncomp, n_ch, dp->npair, sizeof(T2)) + 255) & ~(size_t)255;
    // concurrent-slice candidates: workspaces within 16 GB and the budget
    int max_sv = 0;
    while (max_sv + 1 < bbc::kSliceVariants) {
        const size_t w = (size_t)(2 << max_sv) * stride;
        if (w > (16ull << 30) || (ctx->budget && w + dp->table_bytes > ctx->budget)) break;
        ++max_sv;
    }
    const int nb = 1 << max_sv;                 // slices per timed round
    bbc_status s = ensure_workspace(ctx, (size_t)nb * stride);
    if (s) return s;
    const MomGroups mg = get_groups<T>(ctx, L, &s);
    if (!mg.pos) return s;
    const size_t ob = (size_t)n_ch * 16 * V * sizeof(T2);
    char *out = nullptr;
    double *scale = nullptr;
    if (hipMalloc((void **)&out, ob * nb) != hipSuccess) return fail(BBC_ENOMEM, "autotune output buffer");
    if (hipMalloc((void **)&scale, sizeof(double) * n_ch * nb) != hipSuccess) {
        (void)hipFree(out);
        return fail(BBC_ENOMEM, "autotune scale buffer");
    }
    std::vector<void *> outs(nb);
    std::vector<double *> scales(nb);
    for (int i = 0; i < nb; ++i) { outs[i] = out + (size_t)i * ob; scales[i] = scale + (size_t)i * n_ch; }
    hipEvent_t a = nullptr, b = nullptr;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    // coordinate search from the current choice: the pair-product kernel, the plane
    // pass (only where the lattice takes one), the block kernel, the channel sums,
    // concurrent slices
    bbc::Tuning cur = tuning_for(ctx, L, dp);
    cur.slices = std::min(cur.slices, max_sv);
    float cur_ms = 0.f;
    s = time_variant<T>(ctx, dp, L, V, mg, stride, sl, ss, n_ch, nb, outs.data(), scales.data(), reps, cur, st, a, b,
                        &cur_ms);
    const bool planes = bbc::fft3d_zgrouped_fits<T>(L) && !bbc::fft3d_grouped_fits<T>(L);
    const int npv = sizeof(T) == 8 ? bbc::kPairVariants64 : bbc::kPairVariants32;
    for (int dim = 0; dim < 5 && s == BBC_OK; ++dim) {
        const int n = dim == 0 ? npv : dim == 1 ? (planes ? bbc::kPlaneVariants : 1)
                                     : dim == 2 ? bbc::kBlockVariants : dim == 3 ? bbc::kCombineVariants : max_sv + 1;
        for (int v = 0; v < n && s == BBC_OK; ++v) {
            bbc::Tuning c = cur;
            int &field = dim == 0 ? c.pairs : dim == 1 ? c.planes : dim == 2 ? c.blocks : dim == 3 ? c.combine
                                                                                                 : c.slices;
            if (field == v) continue;
            field = v;
            float ms = 0.f;
            s = time_variant<T>(ctx, dp, L, V, mg, stride, sl, ss, n_ch, nb, outs.data(), scales.data(), reps, c, st,
                                a, b, &ms);
            if (s == BBC_OK && ms < cur_ms) { cur = c; cur_ms = ms; }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(st);
    (void)hipFree(out);
    (void)hipFree(scale);
    *best = cur;
    *best_ms = cur_ms;
    return s;
}

}  // namespace

extern "C" {

bbc_status bbc_tuning_get(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_ch,
                          const int32_t *ch_list, bbc_spin spin, bbc_tuning *out, int *tuned) {
    if (!ctx || !out) return fail(BBC_EINVAL, "NULL argument");
    long V;
    bbc_status s = check_request(lattice, prec, n_ch, ch_list, spin, &V);
    if (s) return s;
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    std::lock_guard<std::mutex> lock(ctx->tmu);
    auto it = ctx->tuning.find(request_key(lattice, prec, n_ch, ch_list, spin));
    const bbc::Tuning t = it != ctx->tuning.end() ? it->second : default_tuning(L, (int)prec);
    *out = bbc_tuning{t.pairs, t.blocks, t.planes, t.slices, t.combine};
    if (tuned) *tuned = it != ctx->tuning.end();
    return BBC_OK;
}

bbc_status bbc_tuning_set(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, int n_ch,
                          const int32_t *ch_list, bbc_spin spin, const bbc_tuning *t) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_request(lattice, prec, n_ch, ch_list, spin, &V);
    if (s) return s;
    const TuneKey key = request_key(lattice, prec, n_ch, ch_list, spin);
    std::lock_guard<std::mutex> lock(ctx->tmu);
    if (!t) {
        ctx->tuning.erase(key);
        return BBC_OK;
    }
    if (!tuning_valid(*t, prec)) return fail(BBC_EINVAL, "kernel variant out of range");
    ctx->tuning[key] = bbc::Tuning{t->pairs, t->blocks, t->planes, t->slices, t->combine};
    return BBC_OK;
}

bbc_status bbc_autotune(bbc_context *ctx, const int32_t lattice[3], bbc_precision prec, const void *S_light,
                        const void *S_strange, int n_ch, const int32_t *ch_list, bbc_spin spin, int reps,
                        void *stream, bbc_tuning *out, double *ms_per_slice) {
    if (!ctx) return fail(BBC_EINVAL, "NULL context");
    long V;
    bbc_status s = check_request(lattice, prec, n_ch, ch_list, spin, &V);
    if (s) return s;
    if (reps < 1 || reps > 1000) return fail(BBC_EINVAL, "reps in [1, 1000]");
    if (!S_light || !S_strange) return fail(BBC_EINVAL, "NULL buffer");
    if (is_host_pointer(S_light) || is_host_pointer(S_strange))
        return fail(BBC_EINVAL, "bbc_autotune takes one device-resident slice");
    std::lock_guard<std::mutex> lock(ctx->mu);
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<int> chans(ch_list, ch_list + n_ch);
    DevPlan *dp = nullptr;
    if ((s = get_plan(ctx, chans, spin == BBC_SPIN_LOWER ? 2 : 0, prec, &dp))) return s;
    const int L[3] = {lattice[0], lattice[1], lattice[2]};
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_after_last(ctx, st))) return s;
    bbc::Tuning best;
    float ms = 0.f;
    if (prec == BBC_F64) s = autotune<double>(ctx, dp, L, V, S_light, S_strange, n_ch, reps, st, &best, &ms);
    else s = autotune<float>(ctx, dp, L, V, S_light, S_strange, n_ch, reps, st, &best, &ms);
    s = mark_last(ctx, st, s);
    if (s) return s;
    {
        std::lock_guard<std::mutex> tl(ctx->tmu);
        ctx->tuning[tune_key(L, (int)prec, dp->spin_offset, dp->chash)] = best;
    }
    if (out) *out = bbc_tuning{best.pairs, best.blocks, best.planes, best.slices, best.combine};
    if (ms_per_slice) *ms_per_slice = ms;
    if (!ctx->tune_path.empty()) return save_tuning(ctx, ctx->tune_path);
    return BBC_OK;
}

bbc_status bbc_tuning_save(bbc_context *ctx, const char *path) {
    if (!ctx || !path || !*path) return fail(BBC_EINVAL, "NULL argument");
    return save_tuning(ctx, path);
}

bbc_status bbc_tuning_load(bbc_context *ctx, const char *path) {
    if (!ctx || !path || !*path) return fail(BBC_EINVAL, "NULL argument");
    return load_tuning(ctx, path);
}

}  // extern "C"
