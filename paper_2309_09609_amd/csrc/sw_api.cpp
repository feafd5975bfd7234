// Host side of libswsearch: the C ABI declared in include/swsearch.h.
//
// sw_db_pack sorts subjects by length (descending, ties by index), cuts the
// sorted list into groups of 128 and interleaves each group so that one wave
// reads 4 columns of 128 subjects as 512 contiguous bytes (one dwordx2 per lane).
//
// A search is planned on the host: every group gets a lane-cooperation degree
// B (1 = one pair of subjects per lane, 64 = a whole wave on one pair) so that
// no work unit is large against a persistent wave's share of the search, units
// are bundled four to a workgroup and ordered longest first, and one persistent
// launch pulls them from an atomic counter.  The long pairs of a short query
// run on a second stream with fewer rows per lane.  Pairs whose 16-bit score
// saturates are appended to a list that a 32-bit launch consumes.  The launch
// sequence itself allocates nothing, so the batched form captures a batch
// shape that comes twice in a row as a HIP graph and replays it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/swsearch.h"
#include "sw_internal.h"

namespace sw {
hipError_t launch_sweep(bool i16, int R, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_occupancy(bool i16, int R, int* blocks_per_cu);
hipError_t launch_sweep_q2(int R, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_occupancy_q2(int R, int* blocks_per_cu);
hipError_t launch_sweep_mode(int mode, int R, const SweepArgs& a, int grid, hipStream_t st);
hipError_t launch_sweep_mode16(int mode, int R, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_occupancy_mode16(int mode, int R, int* blocks_per_cu);
hipError_t launch_align_fill(const AlignPair* pairs, int npairs, int W, const int8_t* subst, int A, int go, int ge,
                             uint8_t* dirs, int32_t* bnd, int32_t* best, int lds_max, hipStream_t st);
hipError_t launch_align_tiles(const AlignPair* pairs, const AlignTile* tiles, int ntiled, int ndiag,
                              int max_diag_tiles, const int8_t* subst, int A, int go, int ge, uint8_t* dirs,
                              int32_t* bnd, int32_t* tws, int32_t* best, hipStream_t st);
hipError_t launch_align_trace(const AlignPair* pairs, int npairs, const uint8_t* dirs, const int32_t* best, char* ops,
                              int64_t ops_stride, int64_t* info, hipStream_t st);
int align_waves(int m, int A, int lds_max);
int64_t align_dir_bytes(int m, int64_t n);
int64_t align_bnd_words(int64_t n);
hipError_t launch_profile(const int8_t* stage, int A, const QDesc* qd, int nq, const int64_t* qoff, int16_t* prof,
                          int32_t* counters, int ncounters, uint32_t* bits, int64_t nbits_words, int max_mp,
                          hipStream_t st, int add = 0);
hipError_t launch_interleave(const int8_t* res, const int64_t* soff, const int32_t* slen, int64_t n, int A,
                             const GroupRec* groups, const int64_t* gdw, int ngroups, uint32_t* image,
                             int64_t total_dw, int32_t* err, hipStream_t st);
hipError_t launch_topk_ws(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                          int64_t* top_i, void* ws, hipStream_t st);
int64_t topk_ws_bytes(int64_t n, int rows, int k);
hipError_t launch_topk(const int32_t* scores, int64_t n, int64_t row_stride, int rows, int k, int32_t* top_s,
                       int64_t* top_i, hipStream_t st);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t st);
}  // namespace sw

using namespace sw;

namespace {

thread_local std::string g_err;

sw_status fail(sw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(SW_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// Device buffer that grows on demand (contents are not preserved).  Every
// reallocation bumps *gen, which invalidates captured graphs.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t want, uint64_t* gen = nullptr) {
        if (want <= bytes && p) return hipSuccess;
        if (p) { hipFree(p); p = nullptr; bytes = 0; }
        const size_t sz = std::max<size_t>(want, 256);
        hipError_t e = hipMalloc(&p, sz);
        if (e == hipSuccess) bytes = sz;
        if (gen) ++*gen;
        return e;
    }
    void release() { if (p) hipFree(p); p = nullptr; bytes = 0; }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

constexpr int kStageRing = 4;         // pinned staging buffers per handle

// Pinned staging buffer; the event marks completion of the last copy out of it.
struct HostPinned {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    hipError_t reserve(size_t want) {
        if (pending) { hipEventSynchronize(done); pending = false; }
        if (want <= bytes && p) return hipSuccess;
        if (p) { hipHostFree(p); p = nullptr; bytes = 0; }
        const size_t sz = std::max<size_t>(want, 4096);
        hipError_t e = hipHostMalloc(&p, sz, hipHostMallocDefault);
        if (e == hipSuccess) bytes = sz;
        return e;
    }
    void release() {
        if (pending) hipEventSynchronize(done);
        if (p) hipHostFree(p);
        if (done) hipEventDestroy(done);
        p = nullptr; done = nullptr; bytes = 0; pending = false;
    }
};

// Work items of one search: the bulk at R_main rows per lane and, on a side
// stream, the long pairs of a short query at a smaller R_side.  Searches on
// the handle's own workspace read the items from device copies made once;
// searches on a caller's workspace upload them with the queries.
struct Plan {
    std::vector<WgItem> h_items;  // [main items..., side items...]
    std::vector<int2> h_pairs;    // query pairs (query a, query b or -1) when qpack
    int32_t n_main = 0, n_side = 0;
    int R_main = 16, R_side = 16;
    bool qpack = false;           // items index query pairs (two queries per lane)
    DevBuf items, qpairs;         // device copies (handle workspace only)
    bool on_device = false;
    void release() { items.release(); qpairs.release(); on_device = false; }
};

// Device pointers of the staged queries (descriptors, offsets, matrix + residues).
struct Staged {
    const QDesc* qd = nullptr;
    const int64_t* qoff = nullptr;
    const int8_t* sm_q = nullptr;
    int nq = 0;
    int max_mp = 0;
    int bias = 0;                 // 16-bit cell bias: minus the lowest substitution score, at least 0
};

struct GraphEntry {
    std::vector<int> qlens;
    int32_t go = 0, ge = 0, k = 0, bias = 0;
    const void* scores = nullptr;
    const void* top_s = nullptr;
    const void* top_i = nullptr;
    hipStream_t stream = nullptr;
    uint64_t gen = 0;
    const void* ws = nullptr;         // workspace base the sequence was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;        // recorded after every launch of exec
    bool launched = false;
    void clear() {
        if (exec && launched && done) hipEventSynchronize(done);   // the last launch may still run
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        launched = false;
        qlens.clear();
    }
};

// The inputs that decide a batched launch sequence; a shape is captured into a graph the second time
// it comes in a row (one-off shapes, e.g. served batches, are enqueued directly and never wait).
struct BatchKey {
    std::vector<int> qlens;
    int32_t go = 0, ge = 0, k = 0, bias = 0;
    const void* scores = nullptr;
    const void* top_s = nullptr;
    const void* top_i = nullptr;
    hipStream_t stream = nullptr;
    uint64_t gen = 0;
    const void* ws = nullptr;
    bool operator==(const BatchKey& o) const {
        return qlens == o.qlens && go == o.go && ge == o.ge && k == o.k && bias == o.bias && scores == o.scores &&
               top_s == o.top_s && top_i == o.top_i && stream == o.stream && gen == o.gen && ws == o.ws;
    }
};

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// 64-bit hash of offsets[0..n]: every value through the splitmix64 finaliser, combined with its
// position, so a changed, moved or swapped boundary changes it.
uint64_t offsets_hash(const int64_t* offsets, int64_t n) {
    uint64_t h = 0x243F6A8885A308D3ull ^ (uint64_t)n;
    for (int64_t k = 0; k <= n; ++k) {
        uint64_t x = (uint64_t)offsets[k] + 0x9E3779B97F4A7C15ull * (uint64_t)(k + 1);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        h = (h ^ (x ^ (x >> 31))) * 0x100000001B3ull;
    }
    return h;
}

}  // namespace

struct sw_db {
    int device = 0;
    int64_t n = 0;
    int64_t total_res = 0;
    int64_t off_first = 0, off_last = 0;
    uint64_t off_hash = 0;            // offsets_hash of the offsets the image was packed with
    int ngroups = 0;
    std::vector<int32_t> ncols;       // per group
    std::vector<int32_t> pcols;       // per pair: longest subject of the pair, rounded up to 4
    int32_t ncols_max = 0;
    // The packed image: one device allocation, the handle's own (image_own) or the caller's
    // (sw_db_pack_into), laid out by DbLayout.
    DevBuf image_own;
    bool caller_image = false;
    uint8_t* d_image = nullptr;       // interleaved residues
    GroupRec* d_groups = nullptr;
    int32_t* d_perm = nullptr;        // sorted slot -> original subject index, -1 for padding slots
    int32_t* d_pair_cols = nullptr;   // per pair: longest subject of the pair, rounded up to 4
    int32_t* d_slen = nullptr;        // subject length per sorted slot (end-to-end modes), 0 for padding
    int64_t image_bytes = 0;
    // per original subject: length and sorted slot; per group: byte offset in the image (alignments)
    std::vector<int32_t> lens, slot_of;
    std::vector<int64_t> gbase;
    DevBuf align_dirs, align_bnd, align_misc, align_tws;   // traceback workspace
    int align_tiles = 0;              // tiled traceback fill: 0 = long pairs, 1 = never, 2 = every pair
    int wg_mode = 0;                  // persistent workgroups of an end-to-end sweep
    Plan mode_plan;
    // launch geometry
    int cus = 0, wg16 = 0, wg32 = 0;  // scratch slots (workgroups) of the 16-bit sweeps; 32-bit grid
    int wgR[17] = {0};                // persistent workgroups per 16-bit instance, by R
    int wgQ[17] = {0};                // persistent workgroups per query-pair instance, by R
    int64_t slot_cap = 0;             // (column x pair) capacity of one wave's boundary slot
    hipStream_t side = nullptr;       // second stream for the long pairs of short queries
    hipStream_t side2 = nullptr;      // third stream (end-to-end modes: the 32-bit groups beside both 16-bit launches)
    hipStream_t cap = nullptr;        // stream the batched sequence is captured on
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
    // workspace of searches without a caller workspace (laid out by WsLayout)
    uint64_t gen = 1;                 // bumped on every workspace reallocation
    DevBuf ws_own;
    // pinned staging of the queries (and, on a caller's workspace, the plan), a ring so that a call
    // reuses a buffer only once the copy of the call kStageRing before it has run
    HostPinned hstage[kStageRing];
    int hstage_next = 0;
    std::map<int, Plan> plans;        // plain searches: query length -> plan
    Plan batch_plan, multi_plan;
    std::vector<int> batch_qlens;
    GraphEntry graph;                 // batched form: last captured shape
    BatchKey last_eager;              // batched form: the last shape enqueued without a graph
    // tuning knobs and test hooks
    int force_lgB = -1;               // fixed lanes per pair
    int force_R = 0;                  // fixed rows per lane (4, 8, 16)
    double unit_share = 0.25;         // largest unit / one wave's share of a search
    int32_t sat = kSat16;             // rerun threshold
    int64_t rerun_cap_hook = 0;       // test hook: list capacity of the recompute (0 = default)
    int poison = 0;                   // test hook: flagged pairs' 16-bit scores read kPoison
    int lane_pack = 1;                // 1: subject pairs per lane; 2: query pairs per lane (several queries)
    int alphabet = 20;                // residue codes 0..alphabet-1; matrices are alphabet x alphabet
    // statistics and timing
    int last_items = 0, last_rows = 16, last_grid = 0, last_side_items = 0, last_side_rows = 0;
    int64_t last_cap = 0;             // list capacity of the last search's recompute
    const int32_t* last_counters = nullptr;   // device counters of the last search (its workspace)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<int> ev_used;         // indices into ev_pool, in launch order
    std::mutex mu;
};

namespace {

// [0] bulk sweep counter, [1] flagged pairs, [2] recompute work counter, [3] side sweep counter,
// [4] second side sweep counter, [5] pairs recomputed
constexpr int kCounters = 6;
// Most entries of the recompute list; flagged pairs beyond it are found through their bits.
constexpr int64_t kRerunListMax = (int64_t)1 << 20;
constexpr int kRerunGrid = 64;
constexpr int kRerunRows = 8;  // rows per lane of the 32-bit recompute
constexpr int kMaxWgPerCu = 4; // persistent workgroups per CU (bounds the scratch slots)
const int kRowChoices[3] = {4, 8, 16};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() { if (prev >= 0) hipSetDevice(prev); }
};

sw_status apply_opts(sw_db* db, const sw_pack_opts* opts) {
    if (!opts) return SW_OK;
    const int fl = opts->force_lanes;
    if (fl < 0 || fl > 64 || (fl & (fl - 1))) return fail(SW_E_INVALID, "force_lanes must be 0 or a power of two <= 64");
    if (opts->rerun_threshold < 0) return fail(SW_E_INVALID, "rerun_threshold must be >= 0");
    const int rpl = opts->rows_per_lane;
    if (rpl != 0 && rpl != 4 && rpl != 8 && rpl != 16) return fail(SW_E_INVALID, "rows_per_lane must be 0, 4, 8 or 16");
    if (opts->lane_pack < 0 || opts->lane_pack > 2) return fail(SW_E_INVALID, "lane_pack must be 0, 1 or 2");
    if (opts->unit_share < 0 || opts->unit_share > 100000) return fail(SW_E_INVALID, "unit_share must be in 0..100000");
    if (opts->rerun_cap < 0) return fail(SW_E_INVALID, "rerun_cap must be >= 0");
    if (opts->poison != 0 && opts->poison != 1) return fail(SW_E_INVALID, "poison must be 0 or 1");
    if (opts->align_tiles < 0 || opts->align_tiles > 2) return fail(SW_E_INVALID, "align_tiles must be 0, 1 or 2");
    db->force_lgB = fl ? __builtin_ctz(fl) : -1;
    db->force_R = rpl;
    db->unit_share = opts->unit_share > 0 ? opts->unit_share / 1000.0 : 0.25;
    db->sat = opts->rerun_threshold > 0 ? std::min<int32_t>(opts->rerun_threshold, kSat16) : kSat16;
    db->lane_pack = opts->lane_pack == 2 ? 2 : 1;
    db->rerun_cap_hook = opts->rerun_cap;
    db->poison = opts->poison;
    db->align_tiles = opts->align_tiles;
    return SW_OK;
}

// ------------------------------------------------------------------ planning
// Issue slots of one unit (in half instructions): passes x steps x the step's
// instruction count, 9.5 per row of R plus loads, addressing and, with
// cooperating lanes, the shift of the bottom row.
int64_t unit_cost(int m, int ncols, int lgB, int R) {
    const int B = 1 << lgB;
    const int64_t passes = (m + (R << lgB) - 1) / (R << lgB);
    const int64_t steps = round_up(ncols + B - 1, 4);
    const int64_t per_step = 19 * R + 30 + (lgB ? 8 : 0);
    return passes * steps * per_step;
}

// Work items for queries of lengths qlens (query index = position) against all
// groups.  Every group gets the smallest lanes-per-pair B whose units cost at
// most a set fraction of a persistent wave's share of the work (0.25 by
// default: smaller units force wide lane cooperation whose pass height exceeds
// short queries, larger ones lengthen the longest-first tail) and whose
// boundary row fits a scratch slot.  Units still above that share at B = 64
// are pairs that a single wave sweeps column by column; for a single short
// query a smaller R makes them cheaper (most of a 64 x 16-row pass would be
// padding) and they go to the side list.  Items are ordered longest first.
// Overrides for sweeps other than the 16-bit ones: fixed R, their slot capacity and wave count, and
// whether the long pairs of a single short query may still go to the side list at a smaller R.
struct PlanLimits { int R; int64_t slot_cap; int64_t nwaves; bool side = false; };

// Groups [g_lo, g_hi) only (g_hi < 0: to the end).
void plan_units(const sw_db* db, const std::vector<int>& qlens, Plan* plan, std::vector<WgItem>& main_out,
                std::vector<WgItem>& side_out, const std::vector<int>* chunk = nullptr, int nchunks = 1,
                const PlanLimits* lim = nullptr, int g_lo = 0, int g_hi = -1) {
    if (g_hi < 0) g_hi = db->ngroups;
    const int64_t slot_cap = lim ? lim->slot_cap : db->slot_cap;
    const bool force_R = lim ? true : db->force_R != 0;
    // query qi covers groups chunk[qi], chunk[qi] + nchunks, ... (all groups when nchunks == 1)
    auto first_group = [&](size_t qi) { return chunk ? (*chunk)[qi] : 0; };
    struct Tmp { WgItem it; int64_t cost; };
    // The plan at R rows per lane; returns its estimated makespan in cost units per wave.
    auto plan_at = [&](int R_main, std::vector<Tmp>& items, std::vector<Tmp>& sitems, int& R_side) -> double {
        const int64_t nwaves = std::max<int64_t>(lim ? lim->nwaves : (int64_t)db->wgR[R_main] * kWaves, 1);
        int64_t total = 0;
        for (size_t qi = 0; qi < qlens.size(); ++qi)
            if (qlens[qi] > 0)
                for (int g = first_group(qi); g < db->ngroups; g += nchunks)
                    if (g >= g_lo && g < g_hi) total += unit_cost(qlens[qi], db->ncols[g], 0, R_main);
        const double cap = db->unit_share * (double)total / (double)nwaves;
        R_side = R_main;
        int64_t sum = 0, biggest = 0, sbiggest = 0;
        for (size_t qi = 0; qi < qlens.size(); ++qi) {
            const int m = qlens[qi];
            if (m <= 0) continue;
            int r_long = R_main;
            if (qlens.size() == 1 && (!force_R || (lim && lim->side)))
                for (int R : kRowChoices)
                    if (unit_cost(m, db->ncols_max, 6, R) < unit_cost(m, db->ncols_max, 6, r_long)) r_long = R;
            const int g_first = first_group(qi);
            WgItem cur{0, (int32_t)qi, 0, -1, 0, nchunks}, scur{0, (int32_t)qi, 0, -1, 0, nchunks};
            int64_t cur_cost = 0, scur_cost = 0;
            auto flush = [](std::vector<Tmp>& v, WgItem& c, int64_t& cc) {
                if (c.count > 0) v.push_back({c, cc});
                c.count = 0;
                cc = 0;
            };
            auto add = [&](std::vector<Tmp>& v, WgItem& c, int64_t& cc, int g, int k, int lgB, int64_t cost) {
                // position of (group, sub-unit) in this query's unit sequence
                const int64_t seq_g = (g - g_first) / nchunks, seq_c = (c.g0 - g_first) / nchunks;
                const bool contiguous = c.count > 0 && c.lgB == lgB && (seq_c << lgB) + c.k0 + c.count == (seq_g << lgB) + k;
                if (c.count == kWaves || !contiguous) {
                    flush(v, c, cc);
                    c.g0 = g;
                    c.k0 = (int16_t)k;
                    c.lgB = (int8_t)lgB;
                }
                c.count++;
                cc = std::max(cc, cost);
            };
            for (int g = g_first; g < db->ngroups; g += nchunks) {
                if (g < g_lo || g >= g_hi) continue;
                const int nc = db->ncols[g];
                int lgB = 0;
                for (; lgB < 6; ++lgB) {
                    const int64_t P = kGroupPairs >> lgB;
                    if ((double)unit_cost(m, nc, lgB, R_main) <= cap && (int64_t)nc * P <= slot_cap) break;
                }
                if (db->force_lgB >= 0) {
                    lgB = db->force_lgB;
                    while (lgB < 6 && (int64_t)nc * (kGroupPairs >> lgB) > slot_cap) ++lgB;
                }
                for (int k = 0; k < (1 << lgB); ++k) {
                    const int uc = db->pcols[(size_t)g * kGroupPairs + (k << (6 - lgB))];
                    const int64_t c = unit_cost(m, uc, lgB, R_main);
                    if (lgB == 6 && db->force_lgB < 0 && r_long != R_main && (double)c > cap &&
                        unit_cost(m, uc, 6, r_long) < c) {
                        const int64_t sc = unit_cost(m, uc, 6, r_long);
                        add(sitems, scur, scur_cost, g, k, 6, sc);
                        sbiggest = std::max(sbiggest, sc);
                        R_side = r_long;
                    } else {
                        add(items, cur, cur_cost, g, k, lgB, c);
                        sum += c;
                        biggest = std::max(biggest, c);
                    }
                }
            }
            flush(items, cur, cur_cost);
            flush(sitems, scur, scur_cost);
        }
        // issue time: the SIMDs share the total; a unit shares its SIMD with the other resident waves
        const double nsimd = 4.0 * db->cus, per_simd = (double)nwaves / nsimd;
        return std::max({(double)sum / nsimd, (double)biggest * per_simd, (double)sbiggest * per_simd});
    };
    std::vector<Tmp> items, sitems;
    int R_main = lim ? lim->R : db->force_R ? db->force_R : 16, R_side = R_main;
    const double t_main = plan_at(R_main, items, sitems, R_side);
    if (!force_R) {
        // fewer rows per lane pay more per cell but pad less when lanes cooperate on a short query
        std::vector<Tmp> items8, sitems8;
        int side8 = 8;
        const double t8 = plan_at(8, items8, sitems8, side8);
        if (t8 < t_main) {
            items.swap(items8);
            sitems.swap(sitems8);
            R_main = 8;
            R_side = side8;
        }
    }
    auto by_cost = [](const Tmp& a, const Tmp& b) { return a.cost > b.cost; };
    std::stable_sort(items.begin(), items.end(), by_cost);
    std::stable_sort(sitems.begin(), sitems.end(), by_cost);
    for (auto& t : items) main_out.push_back(t.it);
    for (auto& t : sitems) side_out.push_back(t.it);
    plan->R_main = R_main;
    plan->R_side = R_side;
}

// Query-pair plan: queries on the same chunk are sorted by length and paired
// neighbour with neighbour (a leftover query runs alone in its half-empty lanes);
// each pair sweeps max(m_a, m_b) rows.  A unit holds P = 64/B subjects and a
// group 2B units; B is capped at 32 (the interleaved slice is twice as large).
void plan_units_q2(const sw_db* db, const std::vector<int>& qlens, Plan* plan, std::vector<WgItem>& out,
                   std::vector<int2>& pairs, const std::vector<int>* chunk, int nchunks) {
    const int R = db->force_R == 8 ? 8 : 16;
    std::vector<int> order;
    for (int q = 0; q < (int)qlens.size(); ++q)
        if (qlens[q] > 0) order.push_back(q);
    auto ch = [&](int q) { return chunk ? (*chunk)[q] : 0; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return ch(a) != ch(b) ? ch(a) < ch(b) : qlens[a] > qlens[b];
    });
    for (size_t i = 0; i < order.size();) {
        if (i + 1 < order.size() && ch(order[i]) == ch(order[i + 1])) {
            pairs.push_back(make_int2(order[i], order[i + 1]));
            i += 2;
        } else {
            pairs.push_back(make_int2(order[i], -1));
            i += 1;
        }
    }
    auto cost = [&](int m, int nc, int lgB) {
        const int B = 1 << lgB;
        const int64_t passes = (m + (R << lgB) - 1) / (R << lgB);
        return passes * round_up(nc + B - 1, 4) * (int64_t)(17 * R + 30 + (lgB ? 8 : 0));
    };
    const int64_t nwaves = (int64_t)db->wgQ[R] * kWaves;
    int64_t total = 0;
    for (const int2& pr : pairs) {
        const int m = std::max(qlens[pr.x], pr.y >= 0 ? qlens[pr.y] : 0);
        for (int g = ch(pr.x); g < db->ngroups; g += nchunks) total += 2 * cost(m, db->ncols[g], 0);
    }
    const double cap = db->unit_share * (double)total / (double)std::max<int64_t>(nwaves, 1);
    struct Tmp { WgItem it; int64_t cost; };
    std::vector<Tmp> items;
    for (size_t pi = 0; pi < pairs.size(); ++pi) {
        const int2 pr = pairs[pi];
        const int m = std::max(qlens[pr.x], pr.y >= 0 ? qlens[pr.y] : 0);
        const int g_first = ch(pr.x);
        WgItem cur{0, (int32_t)pi, 0, -1, 0, nchunks};
        int64_t cc = 0;
        for (int g = g_first; g < db->ngroups; g += nchunks) {
            const int nc = db->ncols[g];
            int lgB = 0;
            for (; lgB < 5; ++lgB)
                if ((double)cost(m, nc, lgB) <= cap && (int64_t)nc * (kGroupPairs >> lgB) <= db->slot_cap) break;
            if (db->force_lgB >= 0) lgB = std::min(db->force_lgB, 5);
            while (lgB < 5 && (int64_t)nc * (kGroupPairs >> lgB) > db->slot_cap) ++lgB;
            const int units = 2 << lgB;
            const int P = kGroupPairs >> lgB;
            const int64_t seq_g = (g - g_first) / nchunks;
            for (int k = 0; k < units; ++k) {
                const int64_t c = cost(m, db->pcols[(size_t)g * kGroupPairs + ((k * P) >> 1)], lgB);
                const int64_t seq_c = (cur.g0 - g_first) / nchunks;
                const bool contiguous = cur.count > 0 && cur.lgB == lgB &&
                                        seq_c * units + cur.k0 + cur.count == seq_g * units + k;
                if (cur.count == kWaves || !contiguous) {
                    if (cur.count > 0) items.push_back({cur, cc});
                    cur.g0 = g;
                    cur.k0 = (int16_t)k;
                    cur.lgB = (int8_t)lgB;
                    cur.count = 0;
                    cc = 0;
                }
                cur.count++;
                cc = std::max(cc, c);
            }
        }
        if (cur.count > 0) items.push_back({cur, cc});
    }
    std::stable_sort(items.begin(), items.end(), [](const Tmp& a, const Tmp& b) { return a.cost > b.cost; });
    for (auto& t : items) out.push_back(t.it);
    plan->R_main = R;
    plan->R_side = R;
}

sw_status build_plan(sw_db* db, const std::vector<int>& qlens, Plan* p, const std::vector<int>* chunk = nullptr,
                     int nchunks = 1) {
    std::vector<WgItem> mi, si;
    std::vector<int2> pairs;
    int nonempty = 0;
    for (int m : qlens) nonempty += m > 0;
    p->qpack = db->lane_pack == 2 && nonempty >= 2;
    if (p->qpack)
        plan_units_q2(db, qlens, p, mi, pairs, chunk, nchunks);
    else
        plan_units(db, qlens, p, mi, si, chunk, nchunks);
    p->n_main = (int32_t)mi.size();
    p->n_side = (int32_t)si.size();
    mi.insert(mi.end(), si.begin(), si.end());
    p->h_items.swap(mi);
    p->h_pairs.swap(pairs);
    p->on_device = false;
    return SW_OK;
}

// Device copies of a plan's items and query pairs (searches on the handle's own workspace).
sw_status upload_plan(sw_db* db, Plan* p) {
    if (p->on_device) return SW_OK;
    HIP_TRY(p->items.reserve(std::max<size_t>(p->h_items.size(), 1) * sizeof(WgItem), &db->gen));
    if (!p->h_items.empty())
        HIP_TRY(hipMemcpy(p->items.p, p->h_items.data(), p->h_items.size() * sizeof(WgItem), hipMemcpyHostToDevice));
    if (p->qpack) {
        HIP_TRY(p->qpairs.reserve(std::max<size_t>(p->h_pairs.size(), 1) * sizeof(int2), &db->gen));
        if (!p->h_pairs.empty())
            HIP_TRY(hipMemcpy(p->qpairs.p, p->h_pairs.data(), p->h_pairs.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    p->on_device = true;
    return SW_OK;
}

sw_status get_plan(sw_db* db, int m, Plan** out) {
    auto it = db->plans.find(m);
    if (it != db->plans.end()) { *out = &it->second; return SW_OK; }
    if (db->plans.size() >= 64) {
        for (auto& kv : db->plans) kv.second.release();
        db->plans.clear();
    }
    Plan& p = db->plans[m];
    sw_status s = build_plan(db, std::vector<int>{m}, &p);
    if (s != SW_OK) { p.release(); db->plans.erase(m); return s; }
    *out = &p;
    return SW_OK;
}

void clear_caches(sw_db* db) {
    for (auto& kv : db->plans) kv.second.release();
    db->plans.clear();
    db->batch_plan.release();
    db->batch_plan.h_items.clear();
    db->batch_plan.n_main = db->batch_plan.n_side = 0;
    db->multi_plan.release();
    db->multi_plan.h_items.clear();
    db->multi_plan.n_main = db->multi_plan.n_side = 0;
    db->batch_qlens.clear();
    db->graph.clear();
    db->last_eager = BatchKey();
}

sw_status check_subst_gaps(const int8_t* subst, int32_t go, int32_t ge) {
    if (!subst) return fail(SW_E_INVALID, "substitution matrix pointer is NULL");
    if (go < 0 || ge < 0) return fail(SW_E_INVALID, "gap penalties must be >= 0 (got %d, %d)", go, ge);
    return SW_OK;
}

// Launch geometry (occupancy of every sweep instance, boundary-slot sizes), streams and events.
// Allocates no device memory.
sw_status ensure_geometry(sw_db* db) {
    if (db->wg16 == 0) {
        // a failure part way leaves wg16 at 0, so the next call sets up again (streams and events are
        // created once)
        struct Undo {
            sw_db* d;
            bool done = false;
            ~Undo() { if (!done) d->wg16 = 0; }
        } undo{db};
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, db->device));
        db->cus = prop.multiProcessorCount;
        int b32 = 0;
        db->wg16 = 0;
        for (int R : kRowChoices) {
            int b = 0;
            HIP_TRY(sweep_occupancy(true, R, &b));
            if (b < 1) return fail(SW_E_HIP, "16-bit sweep (R=%d) cannot be resident", R);
            db->wgR[R] = db->cus * std::min(b, kMaxWgPerCu);
            db->wg16 = std::max(db->wg16, db->wgR[R]);
        }
        for (int R : {8, 16}) {
            int b = 0;
            HIP_TRY(sweep_occupancy_q2(R, &b));
            if (b < 1) return fail(SW_E_HIP, "query-pair sweep (R=%d) cannot be resident", R);
            db->wgQ[R] = db->cus * std::min(b, kMaxWgPerCu);
            db->wg16 = std::max(db->wg16, db->wgQ[R]);
        }
        HIP_TRY(sweep_occupancy(false, kRerunRows, &b32));
        if (b32 < 1) return fail(SW_E_HIP, "32-bit sweep cannot be resident");
        db->wg32 = kRerunGrid;
        // a unit's boundary row is (columns x subjects-or-pairs per wave); the widest
        // query-pair unit is 2 subjects of the longest subject's width
        db->slot_cap = std::max<int64_t>(65536, 2 * (int64_t)db->ncols_max);
        if (!db->side) HIP_TRY(hipStreamCreateWithFlags(&db->side, hipStreamNonBlocking));
        if (!db->side2) HIP_TRY(hipStreamCreateWithFlags(&db->side2, hipStreamNonBlocking));
        if (!db->cap) HIP_TRY(hipStreamCreateWithFlags(&db->cap, hipStreamNonBlocking));
        if (!db->ev_fork) HIP_TRY(hipEventCreateWithFlags(&db->ev_fork, hipEventDisableTiming));
        if (!db->ev_join) HIP_TRY(hipEventCreateWithFlags(&db->ev_join, hipEventDisableTiming));
        if (!db->ev_join2) HIP_TRY(hipEventCreateWithFlags(&db->ev_join2, hipEventDisableTiming));
        for (HostPinned& h : db->hstage)
            if (!h.done) HIP_TRY(hipEventCreateWithFlags(&h.done, hipEventDisableTiming));
        undo.done = true;
    }
    return SW_OK;
}

// Layout of the staging buffer: [QDesc x nq][qoff x nq][subst, kMaxAlphabet^2 bytes][queries]
// [plan items][query pairs]; the plan parts only when the plan travels with the queries (a caller's
// workspace).
struct StageLayout { size_t off_qoff, off_sm, off_items, off_pairs, total; int64_t prof_elems; int max_mp; };

StageLayout stage_layout(const int64_t* h_qoffsets, int nq, const Plan* with_plan = nullptr) {
    StageLayout L{};
    L.off_qoff = round_up(sizeof(QDesc) * nq, 64);
    L.off_sm = L.off_qoff + round_up(sizeof(int64_t) * nq, 64);
    L.off_items = round_up(L.off_sm + kMaxAlphabet * kMaxAlphabet + (h_qoffsets[nq] - h_qoffsets[0]), 64);
    L.off_pairs = round_up(L.off_items + (with_plan ? with_plan->h_items.size() * sizeof(WgItem) : 0), 64);
    L.total = L.off_pairs + (with_plan && with_plan->qpack ? with_plan->h_pairs.size() * sizeof(int2) : 0);
    L.max_mp = kProfRowAlign;
    for (int q = 0; q < nq; ++q) {
        const int m = (int)(h_qoffsets[q + 1] - h_qoffsets[q]);
        const int mp = (int)round_up(std::max(m, 1), kProfRowAlign);
        L.prof_elems += (int64_t)kNRes * mp;
        L.max_mp = std::max(L.max_mp, mp);
    }
    return L;
}

// Capacity of the recompute list for nq queries: a flagged (query, subject
// pair) is appended once, so nq x pairs entries can never overflow; the list
// stops at kRerunListMax (or the test hook's capacity) and the pairs past it
// go through their flag bits.
int64_t rerun_capacity(const sw_db* db, int nq) {
    int64_t cap = std::min<int64_t>((int64_t)db->ngroups * kGroupPairs * std::max(nq, 1), kRerunListMax);
    if (db->rerun_cap_hook > 0) cap = std::min<int64_t>(cap, db->rerun_cap_hook);
    return std::max<int64_t>(cap, 1);
}

int64_t rerun_words(const sw_db* db, int nq) { return (int64_t)std::max(nq, 1) * db->ngroups * 2; }

// The device workspace of a launch sequence, one region laid out in this order:
// 16-bit boundary slots, 32-bit slots, counters, profiles, staging, recompute
// list, flag bits, top-k pieces, score rows (a batch that keeps only its top k).
struct WsLayout {
    StageLayout st;
    int64_t scratch16 = 0, scratch32 = 0, counters = 0, prof = 0, stage = 0, rerun = 0, bits = 0, topk = 0,
            scores = 0, total = 0;
    int64_t rerun_cap = 0, bits_words = 0;
};

WsLayout ws_layout(const sw_db* db, const int64_t* h_qoffsets, int nq, int k, bool with_scores,
                   const Plan* with_plan) {
    WsLayout L;
    L.st = stage_layout(h_qoffsets, nq, with_plan);
    L.rerun_cap = rerun_capacity(db, nq);
    L.bits_words = rerun_words(db, nq);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { const int64_t at = o; o = round_up(o + std::max<int64_t>(bytes, 1), 256); return at; };
    L.scratch16 = take((int64_t)db->wg16 * kWaves * db->slot_cap * 2 * 4);
    L.scratch32 = take((int64_t)db->wg32 * kWaves * std::max<int64_t>(db->ncols_max, 4) * 4 * 4);
    L.counters = take(kCounters * sizeof(int32_t));
    L.prof = take(L.st.prof_elems * (int64_t)sizeof(int16_t));
    L.stage = take((int64_t)L.st.total);
    L.rerun = take(L.rerun_cap * (int64_t)sizeof(WgItem));
    L.bits = take(L.bits_words * (int64_t)sizeof(uint32_t));
    L.topk = take(k > 0 ? topk_ws_bytes(db->n, nq, k) : 0);
    L.scores = take(with_scores ? (int64_t)nq * std::max<int64_t>(db->n, 1) * (int64_t)sizeof(int32_t) : 0);
    L.total = o;
    return L;
}

// Device pointers of a workspace (the handle's own or a caller's) carved by a layout, and where the
// plan's items live.
struct Work {
    WsLayout L;
    uint32_t* scratch16 = nullptr;
    uint32_t* scratch32 = nullptr;
    int32_t* counters = nullptr;
    int16_t* prof = nullptr;
    char* stage = nullptr;
    WgItem* rerun = nullptr;
    uint32_t* bits = nullptr;
    void* topk = nullptr;
    int32_t* scores = nullptr;
    const WgItem* items = nullptr;
    const int2* qpairs = nullptr;
    HostPinned* host = nullptr;       // the pinned staging buffer of this call
};

Work carve(void* base, const WsLayout& L) {
    char* b = static_cast<char*>(base);
    Work W;
    W.L = L;
    W.scratch16 = reinterpret_cast<uint32_t*>(b + L.scratch16);
    W.scratch32 = reinterpret_cast<uint32_t*>(b + L.scratch32);
    W.counters = reinterpret_cast<int32_t*>(b + L.counters);
    W.prof = reinterpret_cast<int16_t*>(b + L.prof);
    W.stage = b + L.stage;
    W.rerun = reinterpret_cast<WgItem*>(b + L.rerun);
    W.bits = reinterpret_cast<uint32_t*>(b + L.bits);
    W.topk = b + L.topk;
    W.scores = reinterpret_cast<int32_t*>(b + L.scores);
    return W;
}

// The workspace of a launch sequence: the caller's (d_ws, checked against the layout) or the
// handle's own (grown as needed); plan items from the plan's device copy or, with a caller's
// workspace, from the staging area they are uploaded to.
sw_status get_work(sw_db* db, const int64_t* h_qoffsets, int nq, int k, bool with_scores, Plan* plan, void* d_ws,
                   int64_t ws_bytes, Work* out) {
    const bool caller = d_ws != nullptr;
    const WsLayout L = ws_layout(db, h_qoffsets, nq, k, with_scores, caller ? plan : nullptr);
    if (caller) {
        if (ws_bytes < L.total)
            return fail(SW_E_SIZE, "workspace of %lld bytes < %lld needed", (long long)ws_bytes, (long long)L.total);
        if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(SW_E_INVALID, "workspace not 256-byte aligned");
        *out = carve(d_ws, L);
    } else {
        HIP_TRY(db->ws_own.reserve((size_t)L.total, &db->gen));
        *out = carve(db->ws_own.p, L);
    }
    HostPinned& hs = db->hstage[db->hstage_next];
    db->hstage_next = (db->hstage_next + 1) % kStageRing;
    HIP_TRY(hs.reserve(L.st.total));
    out->host = &hs;
    if (plan) {
        if (caller) {
            out->items = reinterpret_cast<const WgItem*>(out->stage + L.st.off_items);
            out->qpairs = plan->qpack ? reinterpret_cast<const int2*>(out->stage + L.st.off_pairs) : nullptr;
        } else {
            sw_status s = upload_plan(db, plan);
            if (s != SW_OK) return s;
            out->items = plan->items.as<WgItem>();
            out->qpairs = plan->qpack ? plan->qpairs.as<int2>() : nullptr;
        }
    }
    return SW_OK;
}

// The recompute fields of a 16-bit sweep's arguments (flagged pairs are listed, then set as bits).
void set_rerun_args(sw_db* db, SweepArgs& a, const Work& W, int32_t* ctr) {
    a.rerun = W.rerun;
    a.rerun_count = ctr + 1;
    a.rerun_cap = (int32_t)W.L.rerun_cap;
    a.rerun_bits = W.bits;
    a.rerun_groups = db->ngroups;
    a.rerun_words = W.L.bits_words;
    a.recomputed = ctr + 5;
    a.poison = db->poison;
    db->last_cap = a.rerun_cap;
}

// Arguments of the 32-bit recompute that follows sweep arguments a: every listed pair, then (when the
// list overflowed) every pair whose flag bit is set; one unit per workgroup in the 32-bit slots.
SweepArgs recompute_args(const sw_db* db, const SweepArgs& a, const Work& W, int32_t* ctr) {
    SweepArgs r = a;
    r.items = W.rerun;
    r.n_items_dev = ctr + 1;
    r.n_items = a.rerun_cap;
    r.counter = ctr + 2;
    r.scratch = W.scratch32;
    r.slot_words = (int64_t)std::max<int32_t>(db->ncols_max, 4) * 4;
    r.slot_base = 0;
    r.rerun = nullptr;              // reads rerun_bits, appends nothing
    r.rerun_count = nullptr;
    r.unit_list = 1;
    r.poison = 0;
    return r;
}

// Sweep arguments shared by every launch of a search: image, profile, queries, gaps, 16-bit slots.
SweepArgs sweep_args(const sw_db* db, const Staged& S, const Work& W, int32_t go, int32_t ge, int32_t* scores) {
    SweepArgs a{};
    a.image = db->d_image;
    a.groups = db->d_groups;
    a.perm = db->d_perm;
    a.pair_cols = db->d_pair_cols;
    a.slen = db->d_slen;
    a.prof = W.prof;
    a.qd = S.qd;
    a.go = go;
    a.ge = ge;
    a.scratch = W.scratch16;
    a.slot_words = db->slot_cap * 2;
    a.slot_base = 0;
    a.scores = scores;
    return a;
}

// Copies the queries (host) into the staging buffer on the device.  No launch.
sw_status stage_queries(sw_db* db, const Work& W, const int8_t* h_queries, const int64_t* h_qoffsets, int nq,
                        const int8_t* subst, int64_t score_row_stride, hipStream_t st, Staged* out,
                        int32_t* const* per_query_out = nullptr, const Plan* with_plan = nullptr) {
    const StageLayout& L = W.L.st;
    char* h = static_cast<char*>(W.host->p);
    int64_t prof_off = 0;
    QDesc* qd = reinterpret_cast<QDesc*>(h);
    int64_t* qo = reinterpret_cast<int64_t*>(h + L.off_qoff);
    for (int q = 0; q < nq; ++q) {
        const int m = (int)(h_qoffsets[q + 1] - h_qoffsets[q]);
        const int mp = (int)round_up(std::max(m, 1), kProfRowAlign);
        qd[q] = QDesc{prof_off, (int64_t)q * score_row_stride, per_query_out ? per_query_out[q] : nullptr, m, mp};
        prof_off += (int64_t)kNRes * mp;
        qo[q] = h_qoffsets[q] - h_qoffsets[0];
    }
    memcpy(h + L.off_sm, subst, (size_t)db->alphabet * db->alphabet);
    int lowest = 0;
    for (int e = 0; e < db->alphabet * db->alphabet; ++e) lowest = std::min<int>(lowest, subst[e]);
    out->bias = -lowest;
    const int64_t qbytes = h_qoffsets[nq] - h_qoffsets[0];
    if (qbytes) memcpy(h + L.off_sm + kMaxAlphabet * kMaxAlphabet, h_queries + h_qoffsets[0], qbytes);
    if (with_plan) {
        if (!with_plan->h_items.empty())
            memcpy(h + L.off_items, with_plan->h_items.data(), with_plan->h_items.size() * sizeof(WgItem));
        if (with_plan->qpack && !with_plan->h_pairs.empty())
            memcpy(h + L.off_pairs, with_plan->h_pairs.data(), with_plan->h_pairs.size() * sizeof(int2));
    }
    HIP_TRY(hipMemcpyAsync(W.stage, h, L.total, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(W.host->done, st));
    W.host->pending = true;
    const char* d = W.stage;
    out->qd = reinterpret_cast<const QDesc*>(d);
    out->qoff = reinterpret_cast<const int64_t*>(d + L.off_qoff);
    out->sm_q = reinterpret_cast<const int8_t*>(d + L.off_sm);
    out->nq = nq;
    out->max_mp = L.max_mp;
    return SW_OK;
}

// Timing events of the dominant launches (sw_profile_kernels): a ring of
// kTimerSlots start/stop pairs; the oldest is forgotten when it is full.
constexpr int kTimerSlots = 4096;

int record_timer_start(sw_db* db, hipStream_t st) {
    if (db->ev_used.size() >= (size_t)kTimerSlots) db->ev_used.erase(db->ev_used.begin());
    const int ev = (int)((db->ev_used.empty() ? -1 : db->ev_used.back()) + 1) % kTimerSlots;
    while ((int)db->ev_pool.size() <= ev) {
        hipEvent_t x, y;
        if (hipEventCreate(&x) != hipSuccess) return -1;
        if (hipEventCreate(&y) != hipSuccess) { hipEventDestroy(x); return -1; }
        db->ev_pool.push_back({x, y});
    }
    if (hipEventRecord(db->ev_pool[ev].first, st) != hipSuccess) return -1;
    return ev;
}

// The launch sequence of a search: profile (zeroes the counters), the side and
// bulk 16-bit sweeps, the 32-bit recompute, top-k.  Allocates nothing and never
// waits on the host, so it can be captured into a graph.
sw_status enqueue(sw_db* db, const Staged& S, const Plan& plan, const Work& W, int32_t go, int32_t ge,
                  int32_t* d_scores, int64_t n, int k, int32_t* top_s, int64_t* top_i, hipStream_t st,
                  bool time_sweep) {
    int32_t* ctr = W.counters;
    HIP_TRY(launch_profile(S.sm_q, db->alphabet, S.qd, S.nq, S.qoff, W.prof, ctr, kCounters, W.bits, W.L.bits_words,
                           S.max_mp, st));
    SweepArgs a = sweep_args(db, S, W, go, ge, d_scores);
    a.items = W.items;
    a.n_items_dev = nullptr;
    a.n_items = plan.n_main;
    a.counter = ctr + 0;
    set_rerun_args(db, a, W, ctr);
    a.unit_list = 0;
    a.bias = S.bias;
    a.sat = std::min<int32_t>(db->sat + S.bias, kSat16);
    a.qpairs = plan.qpack ? W.qpairs : nullptr;
    // the side launch takes the first slots; the bulk launch fills the rest of the GPU
    const int wg_main = plan.qpack ? db->wgQ[plan.R_main] : db->wgR[plan.R_main];
    const int grid_side = std::min(plan.n_side, std::max(1, wg_main / 8));
    const int grid_main = std::max(1, std::min(wg_main - grid_side, std::max(plan.n_main, 1)));
    if (plan.n_side > 0) {
        SweepArgs b = a;
        b.items = W.items + plan.n_main;
        b.n_items = plan.n_side;
        b.counter = ctr + 3;
        b.slot_base = grid_main;
        HIP_TRY(hipEventRecord(db->ev_fork, st));
        HIP_TRY(hipStreamWaitEvent(db->side, db->ev_fork, 0));
        HIP_TRY(launch_sweep(true, plan.R_side, b, grid_side, db->side));
        HIP_TRY(hipEventRecord(db->ev_join, db->side));
    }
    const int ev = time_sweep && db->timing ? record_timer_start(db, st) : -1;
    if (plan.n_main > 0) {
        if (plan.qpack)
            HIP_TRY(launch_sweep_q2(plan.R_main, a, grid_main, st));
        else
            HIP_TRY(launch_sweep(true, plan.R_main, a, grid_main, st));
    }
    if (plan.n_side > 0) HIP_TRY(hipStreamWaitEvent(st, db->ev_join, 0));
    if (ev >= 0) {
        HIP_TRY(hipEventRecord(db->ev_pool[ev].second, st));
        db->ev_used.push_back(ev);
    }
    // exact 32-bit recompute of saturated pairs; the count is read on the device
    const SweepArgs r = recompute_args(db, a, W, ctr);
    HIP_TRY(launch_sweep(false, kRerunRows, r, db->wg32, st));
    if (k > 0)
        HIP_TRY(launch_topk_ws(d_scores, n, n, S.nq, k, top_s, top_i, topk_ws_bytes(n, S.nq, k) > 0 ? W.topk : nullptr,
                               st));
    db->last_items = plan.n_main;
    db->last_rows = plan.R_main;
    db->last_side_items = plan.n_side;
    db->last_side_rows = plan.n_side ? plan.R_side : 0;
    db->last_grid = grid_main + (plan.n_side > 0 ? grid_side : 0);
    db->last_counters = ctr;
    return SW_OK;
}

sw_status check_db_args(sw_db* db, const int64_t* h_offsets, int64_t n) {
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if (n != db->n) return fail(SW_E_INVALID, "n = %lld but the database holds %lld subjects", (long long)n, (long long)db->n);
    if (h_offsets && n > 0 &&
        (h_offsets[0] != db->off_first || h_offsets[n] != db->off_last || offsets_hash(h_offsets, n) != db->off_hash))
        return fail(SW_E_INVALID, "offsets do not match the packed database");
    return SW_OK;
}


}  // namespace

namespace {

// Host side of packing: the length order, the groups of 128 subjects and where each subject goes.
struct PackPlan {
    std::vector<int32_t> len;         // per original subject
    std::vector<int32_t> order;       // sorted slot -> original subject
    std::vector<GroupRec> groups;
    std::vector<int64_t> gdw;         // group base in dwords
    std::vector<int32_t> perm;        // [G * 128] sorted slot -> original subject, -1 for padding slots
    std::vector<int64_t> soff;        // sorted slot -> residue offset of the subject
    std::vector<int32_t> slen;        // [G * 128] sorted slot -> length, 0 for padding slots
    std::vector<int32_t> ncols;       // per group
    std::vector<int32_t> pcols;       // per pair
    int32_t ncols_max = 0;
    int64_t image_bytes = 0;
    int G = 0;
};

sw_status plan_pack(const int64_t* h_offsets, int64_t n, PackPlan* P) {
    if (n < 0) return fail(SW_E_INVALID, "n must be >= 0");
    if (n > ((int64_t)1 << 31) - 256) return fail(SW_E_UNSUPPORTED, "more than 2^31 subjects");
    if (n > 0 && !h_offsets) return fail(SW_E_INVALID, "NULL offsets");
    if (n > 0 && h_offsets[0] < 0) return fail(SW_E_INVALID, "offsets[0] < 0");
    P->len.resize(n);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t l = h_offsets[k + 1] - h_offsets[k];
        if (l < 0) return fail(SW_E_INVALID, "offsets decrease at %lld", (long long)k);
        if (l > (1 << 24)) return fail(SW_E_UNSUPPORTED, "subject %lld longer than 2^24", (long long)k);
        P->len[k] = (int32_t)l;
    }
    P->order.resize(n);
    std::iota(P->order.begin(), P->order.end(), 0);
    std::stable_sort(P->order.begin(), P->order.end(), [&](int32_t a, int32_t b) { return P->len[a] > P->len[b]; });
    const int G = P->G = (int)((n + kGroupSubjects - 1) / kGroupSubjects);
    P->groups.resize(G);
    P->gdw.resize(G);
    P->ncols.resize(G);
    int64_t base = 0;
    for (int g = 0; g < G; ++g) {
        const int32_t nc = (int32_t)round_up(P->len[P->order[(size_t)g * kGroupSubjects]], kChunkCols);
        P->groups[g] = GroupRec{base, nc, g * kGroupSubjects};
        P->gdw[g] = base / 4;
        P->ncols[g] = nc;
        P->ncols_max = std::max(P->ncols_max, nc);
        base += (int64_t)nc * kGroupSubjects;
    }
    P->image_bytes = base;
    P->perm.assign((size_t)G * kGroupSubjects, -1);
    P->slen.assign((size_t)G * kGroupSubjects, 0);
    P->soff.resize(n);
    P->pcols.assign((size_t)G * kGroupPairs, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t o = P->order[i];
        P->pcols[(size_t)(i / 2)] = std::max<int32_t>(P->pcols[(size_t)(i / 2)], (int32_t)round_up(P->len[o], kChunkCols));
        P->perm[i] = o;
        P->soff[i] = h_offsets[o];
        P->slen[i] = P->len[o];
    }
    return SW_OK;
}

// Device layout of a packed image: interleaved residues, group table, permutation, pair widths,
// sorted lengths, then what packing alone uses (residue offsets per sorted slot, group bases, an
// error word), which may hold anything afterwards.
struct DbLayout { int64_t image, groups, perm, pair_cols, slen, soff, gdw, err, total; };

DbLayout db_layout(int64_t n, int G, int64_t image_bytes) {
    DbLayout L{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) { const int64_t at = o; o = round_up(o + std::max<int64_t>(bytes, 1), 256); return at; };
    L.image = take(std::max<int64_t>(image_bytes, 4));
    L.groups = take((int64_t)sizeof(GroupRec) * G);
    L.perm = take(4 * (int64_t)G * kGroupSubjects);
    L.pair_cols = take(4 * (int64_t)G * kGroupPairs);
    L.slen = take(4 * (int64_t)G * kGroupSubjects);
    L.soff = take(8 * std::max<int64_t>(n, 1));
    L.gdw = take(8 * (int64_t)std::max(G, 1));
    L.err = take(4);
    L.total = o;
    return L;
}

// sw_db_pack (d_db NULL: the handle allocates the image) and sw_db_pack_into (the caller's buffer).
sw_status pack_db(const int8_t* d_residues, const int64_t* h_offsets, int64_t n, const sw_pack_opts* opts, void* d_db,
                  int64_t db_bytes, hipStream_t st, sw_db** out) {
    if (!out) return fail(SW_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n > 0 && !d_residues) return fail(SW_E_INVALID, "NULL residues");
    PackPlan P;
    sw_status so = plan_pack(h_offsets, n, &P);
    if (so != SW_OK) return so;
    const DbLayout L = db_layout(n, P.G, P.image_bytes);
    if (d_db && db_bytes < L.total)
        return fail(SW_E_SIZE, "image buffer of %lld bytes < %lld needed", (long long)db_bytes, (long long)L.total);
    if (d_db && (reinterpret_cast<uintptr_t>(d_db) & 255) != 0) return fail(SW_E_INVALID, "image buffer not 256-byte aligned");
    sw_db* db = new (std::nothrow) sw_db();
    if (!db) return fail(SW_E_NOMEM, "host allocation failed");
    auto bail = [&](sw_status s) { sw_db_free(db); return s; };
    if (hipGetDevice(&db->device) != hipSuccess) return bail(fail(SW_E_HIP, "no current HIP device"));
    so = apply_opts(db, opts);
    if (so != SW_OK) return bail(so);
    if (opts && (opts->alphabet < 0 || opts->alphabet > kMaxAlphabet))
        return bail(fail(SW_E_INVALID, "alphabet must be 0 (= 20) or 1..%d", kMaxAlphabet));
    db->alphabet = (opts && opts->alphabet > 0) ? opts->alphabet : 20;
    db->n = n;
    db->off_first = n > 0 ? h_offsets[0] : 0;
    db->off_last = n > 0 ? h_offsets[n] : 0;
    db->off_hash = n > 0 ? offsets_hash(h_offsets, n) : 0;
    db->total_res = db->off_last - db->off_first;
    db->ngroups = P.G;
    db->ncols = P.ncols;
    db->pcols = P.pcols;
    db->ncols_max = P.ncols_max;
    db->image_bytes = P.image_bytes;
    db->lens = P.len;
    db->slot_of.assign(n, 0);
    for (int64_t i = 0; i < n; ++i) db->slot_of[P.order[i]] = (int32_t)i;
    db->gbase.resize(P.G);
    for (int g = 0; g < P.G; ++g) db->gbase[g] = P.groups[g].base;
    char* base = static_cast<char*>(d_db);
    if (!d_db) {
        const hipError_t e = db->image_own.reserve((size_t)L.total);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? SW_E_NOMEM : SW_E_HIP, "device allocation: %s", hipGetErrorString(e)));
        base = db->image_own.as<char>();
    }
    db->caller_image = d_db != nullptr;
    db->d_image = reinterpret_cast<uint8_t*>(base + L.image);
    db->d_groups = reinterpret_cast<GroupRec*>(base + L.groups);
    db->d_perm = reinterpret_cast<int32_t*>(base + L.perm);
    db->d_pair_cols = reinterpret_cast<int32_t*>(base + L.pair_cols);
    db->d_slen = reinterpret_cast<int32_t*>(base + L.slen);
    if (P.G > 0) {
        int64_t* d_soff = reinterpret_cast<int64_t*>(base + L.soff);
        int64_t* d_gdw = reinterpret_cast<int64_t*>(base + L.gdw);
        int32_t* d_err = reinterpret_cast<int32_t*>(base + L.err);
        int32_t zero = 0, herr = 0;
        hipError_t e = hipSuccess;
        auto step = [&](hipError_t x) { if (e == hipSuccess) e = x; };
        step(hipMemcpyAsync(db->d_groups, P.groups.data(), sizeof(GroupRec) * P.G, hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(db->d_perm, P.perm.data(), sizeof(int32_t) * P.perm.size(), hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(db->d_pair_cols, P.pcols.data(), sizeof(int32_t) * P.pcols.size(), hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(db->d_slen, P.slen.data(), sizeof(int32_t) * P.slen.size(), hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(d_soff, P.soff.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(d_gdw, P.gdw.data(), sizeof(int64_t) * P.G, hipMemcpyHostToDevice, st));
        step(hipMemcpyAsync(d_err, &zero, 4, hipMemcpyHostToDevice, st));
        step(launch_interleave(d_residues, d_soff, db->d_slen, n, db->alphabet, db->d_groups, d_gdw, P.G,
                               reinterpret_cast<uint32_t*>(db->d_image), P.image_bytes / 4, d_err, st));
        step(hipMemcpyAsync(&herr, d_err, 4, hipMemcpyDeviceToHost, st));
        step(hipStreamSynchronize(st));
        if (e != hipSuccess) return bail(fail(SW_E_HIP, "packing: %s", hipGetErrorString(e)));
        if (herr) return bail(fail(SW_E_RESIDUE, "database residue code outside 0..%d", db->alphabet - 1));
    }
    *out = db;
    return SW_OK;
}

}  // namespace

namespace {

// sw_search and sw_search_ws: the plain form, on the handle's workspace (d_ws NULL) or the caller's.
sw_status search_one(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets, int64_t n,
                     const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_scores_out, void* d_ws,
                     int64_t ws_bytes, hipStream_t st) {
    sw_status s;
    if ((s = check_db_args(db, h_offsets, n)) != SW_OK) return s;
    if ((s = check_subst_gaps(h_subst, gap_open, gap_extend)) != SW_OK) return s;
    if (qlen < 0) return fail(SW_E_INVALID, "qlen must be >= 0");
    if (qlen > 0 && !h_query) return fail(SW_E_INVALID, "query is NULL");
    if (n > 0 && !d_scores_out) return fail(SW_E_INVALID, "scores_out is NULL");
    for (int32_t i = 0; i < qlen; ++i)
        if (h_query[i] < 0 || h_query[i] >= db->alphabet)
            return fail(SW_E_RESIDUE, "query residue %d at %d outside 0..%d", h_query[i], i, db->alphabet - 1);
    if (n == 0) return SW_OK;
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    if (qlen == 0) { HIP_TRY(launch_fill(d_scores_out, n, 0, st)); return SW_OK; }
    if ((s = ensure_geometry(db)) != SW_OK) return s;
    Plan* plan = nullptr;
    if ((s = get_plan(db, qlen, &plan)) != SW_OK) return s;
    const int64_t qo[2] = {0, qlen};
    Work W;
    if ((s = get_work(db, qo, 1, 0, false, plan, d_ws, ws_bytes, &W)) != SW_OK) return s;
    Staged S;
    if ((s = stage_queries(db, W, h_query, qo, 1, h_subst, 0, st, &S, nullptr, d_ws ? plan : nullptr)) != SW_OK)
        return s;
    return enqueue(db, S, *plan, W, gap_open, gap_extend, d_scores_out, n, 0, nullptr, nullptr, st, true);
}

}  // namespace

namespace {

// The batch plan for these query lengths (kept while the lengths repeat).
sw_status plan_for(sw_db* db, const std::vector<int>& qlens, Plan** out) {
    if (qlens != db->batch_qlens) {
        if (db->batch_plan.on_device) HIP_TRY(hipDeviceSynchronize());   // a batch in flight may read its items
        db->batch_qlens.clear();
        db->batch_plan.release();
        sw_status s = build_plan(db, qlens, &db->batch_plan);
        if (s != SW_OK) return s;
        db->batch_qlens = qlens;
    }
    *out = &db->batch_plan;
    return SW_OK;
}

// sw_search_batch and sw_search_batch_ws: the batched form, on the handle's workspace (d_ws NULL) or
// the caller's.
sw_status search_batch(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                       const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t k, int32_t* d_scores,
                       int32_t* d_top_scores, int64_t* d_top_index, void* d_ws, int64_t ws_bytes, hipStream_t st) {
    sw_status s;
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if ((s = check_subst_gaps(h_subst, gap_open, gap_extend)) != SW_OK) return s;
    if (nq < 0) return fail(SW_E_INVALID, "nq must be >= 0");
    if (nq > 0 && (!h_qoffsets || !h_queries)) return fail(SW_E_INVALID, "NULL queries or offsets");
    if (k < 0 || k > 1024) return fail(SW_E_UNSUPPORTED, "k must be in 0..1024 (got %d)", k);
    if (k > 0 && (!d_top_scores || !d_top_index)) return fail(SW_E_INVALID, "NULL top-k outputs");
    if (!d_scores && k == 0) return fail(SW_E_INVALID, "no output requested (scores NULL and k == 0)");
    for (int q = 0; q < nq; ++q) {
        if (h_qoffsets[q + 1] < h_qoffsets[q]) return fail(SW_E_INVALID, "query offsets decrease at %d", q);
        if (h_qoffsets[q + 1] - h_qoffsets[q] > (1 << 24)) return fail(SW_E_UNSUPPORTED, "query %d too long", q);
    }
    if (nq > 0)
        for (int64_t i = h_qoffsets[0]; i < h_qoffsets[nq]; ++i)
            if (h_queries[i] < 0 || h_queries[i] >= db->alphabet) return fail(SW_E_RESIDUE, "query residue outside 0..%d at %lld", db->alphabet - 1, (long long)i);
    if (nq == 0) return SW_OK;
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    const int64_t n = db->n;
    if (n == 0) {
        if (k > 0) HIP_TRY(launch_topk(d_scores, 0, 0, nq, k, d_top_scores, d_top_index, st));
        return SW_OK;
    }
    if ((s = ensure_geometry(db)) != SW_OK) return s;
    std::vector<int> qlens(nq);
    for (int q = 0; q < nq; ++q) qlens[q] = (int)(h_qoffsets[q + 1] - h_qoffsets[q]);
    // On the handle's workspace the plan's device copy may still be read by the previous batch; a caller's
    // workspace receives the plan with the queries, in stream order, so nothing waits.
    if (!d_ws && qlens != db->batch_qlens) HIP_TRY(hipStreamSynchronize(st));
    Plan* plan = nullptr;
    if ((s = plan_for(db, qlens, &plan)) != SW_OK) return s;
    Work W;
    if ((s = get_work(db, h_qoffsets, nq, k, d_scores == nullptr, plan, d_ws, ws_bytes, &W)) != SW_OK) return s;
    int32_t* scores = d_scores ? d_scores : W.scores;
    // zero-length queries score 0 everywhere (outside the captured sequence)
    for (int q = 0; q < nq; ++q)
        if (qlens[q] == 0) HIP_TRY(launch_fill(scores + (int64_t)q * n, n, 0, st));
    Staged S;
    if ((s = stage_queries(db, W, h_queries, h_qoffsets, nq, h_subst, n, st, &S, nullptr, d_ws ? plan : nullptr)) != SW_OK)
        return s;
    GraphEntry& G = db->graph;
    BatchKey key;
    key.qlens = qlens;
    key.go = gap_open;
    key.ge = gap_extend;
    key.k = k;
    key.bias = S.bias;
    key.scores = scores;
    key.top_s = d_top_scores;
    key.top_i = d_top_index;
    key.stream = st;
    key.gen = db->gen;
    key.ws = W.scratch16;
    const bool hit = G.exec && G.gen == db->gen && G.ws == W.scratch16 && G.qlens == qlens && G.go == gap_open &&
                     G.ge == gap_extend && G.bias == S.bias && G.k == k && G.scores == scores &&
                     G.top_s == d_top_scores && G.top_i == d_top_index && G.stream == st;
    if (!hit && !(key == db->last_eager)) {
        db->last_eager = key;
        const int ev = db->timing ? record_timer_start(db, st) : -1;
        s = enqueue(db, S, *plan, W, gap_open, gap_extend, scores, n, k, d_top_scores, d_top_index, st, false);
        if (s != SW_OK) return s;
        if (ev >= 0) {
            HIP_TRY(hipEventRecord(db->ev_pool[ev].second, st));
            db->ev_used.push_back(ev);
        }
        return SW_OK;
    }
    if (!hit) {
        // captured on the library's own stream (the caller's may be the legacy
        // default stream, which cannot be captured); launched on the caller's
        G.clear();
        HIP_TRY(hipStreamBeginCapture(db->cap, hipStreamCaptureModeThreadLocal));
        s = enqueue(db, S, *plan, W, gap_open, gap_extend, scores, n, k, d_top_scores, d_top_index, db->cap, false);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(db->cap, &graph);
        if (s != SW_OK) { if (graph) hipGraphDestroy(graph); return s; }
        if (e != hipSuccess) return fail(SW_E_HIP, "graph capture: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { hipGraphDestroy(graph); return fail(SW_E_HIP, "graph instantiate: %s", hipGetErrorString(e)); }
        G.graph = graph;
        G.exec = exec;
        G.qlens = qlens;
        G.go = gap_open;
        G.ge = gap_extend;
        G.bias = S.bias;
        G.k = k;
        G.scores = scores;
        G.top_s = d_top_scores;
        G.top_i = d_top_index;
        G.stream = st;
        G.gen = db->gen;
        G.ws = W.scratch16;
        db->last_eager = BatchKey();
    }
    if (!G.done) HIP_TRY(hipEventCreateWithFlags(&G.done, hipEventDisableTiming));
    const int ev = db->timing ? record_timer_start(db, st) : -1;
    HIP_TRY(hipGraphLaunch(G.exec, st));
    HIP_TRY(hipEventRecord(G.done, st));
    G.launched = true;
    if (ev >= 0) {
        HIP_TRY(hipEventRecord(db->ev_pool[ev].second, st));
        db->ev_used.push_back(ev);
    }
    return SW_OK;
}


}  // namespace

namespace sw {
// Records an error for sw_last_error() from other files of the library and returns s.
sw_status report(sw_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
}  // namespace sw

// ====================================================================== C ABI
extern "C" {

const char* sw_status_str(sw_status s) {
    switch (s) {
        case SW_OK: return "SW_OK";
        case SW_E_INVALID: return "SW_E_INVALID";
        case SW_E_RESIDUE: return "SW_E_RESIDUE";
        case SW_E_NOMEM: return "SW_E_NOMEM";
        case SW_E_HIP: return "SW_E_HIP";
        case SW_E_UNSUPPORTED: return "SW_E_UNSUPPORTED";
        case SW_E_SIZE: return "SW_E_SIZE";
        default: return "SW_E_UNKNOWN";
    }
}

const char* sw_last_error(void) { return g_err.c_str(); }

sw_status sw_db_pack(const int8_t* d_residues, const int64_t* h_offsets, int64_t n, const sw_pack_opts* opts,
                     sw_stream stream, sw_db** out) {
    g_err.clear();
    return pack_db(d_residues, h_offsets, n, opts, nullptr, 0, static_cast<hipStream_t>(stream), out);
}

sw_status sw_db_pack_into(const int8_t* d_residues, const int64_t* h_offsets, int64_t n, const sw_pack_opts* opts,
                          void* d_db, int64_t db_bytes, sw_stream stream, sw_db** out) {
    g_err.clear();
    if (!d_db) return fail(SW_E_INVALID, "d_db is NULL");
    return pack_db(d_residues, h_offsets, n, opts, d_db, db_bytes, static_cast<hipStream_t>(stream), out);
}

sw_status sw_db_pack_bytes(const int64_t* h_offsets, int64_t n, const sw_pack_opts* opts, int64_t* bytes) {
    g_err.clear();
    (void)opts;                       // the image does not depend on the options
    if (!bytes) return fail(SW_E_INVALID, "bytes is NULL");
    PackPlan P;
    sw_status s = plan_pack(h_offsets, n, &P);
    if (s != SW_OK) return s;
    *bytes = db_layout(n, P.G, P.image_bytes).total;
    return SW_OK;
}

sw_status sw_db_tune(sw_db* db, const sw_pack_opts* opts) {
    g_err.clear();
    if (!db || !opts) return fail(SW_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    sw_db probe;
    sw_status s = apply_opts(&probe, opts);        // validate before touching the handle
    if (s != SW_OK) return s;
    HIP_TRY(hipDeviceSynchronize());               // no search of this handle may be in flight
    apply_opts(db, opts);
    clear_caches(db);
    return SW_OK;
}

void sw_db_free(sw_db* db) {
    if (!db) return;
    DeviceGuard dg(db->device);
    hipDeviceSynchronize();
    clear_caches(db);
    db->image_own.release();           // a caller's image stays the caller's
    db->align_dirs.release(); db->align_bnd.release(); db->align_misc.release(); db->align_tws.release();
    db->mode_plan.release();
    db->ws_own.release();
    for (HostPinned& h : db->hstage) h.release();
    for (auto& e : db->ev_pool) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
    if (db->side) hipStreamDestroy(db->side);
    if (db->side2) hipStreamDestroy(db->side2);
    if (db->cap) hipStreamDestroy(db->cap);
    if (db->graph.done) hipEventDestroy(db->graph.done);
    if (db->ev_fork) hipEventDestroy(db->ev_fork);
    if (db->ev_join) hipEventDestroy(db->ev_join);
    if (db->ev_join2) hipEventDestroy(db->ev_join2);
    delete db;
}

sw_status sw_db_info(const sw_db* db, int64_t* n, int64_t* residues, int64_t* device_bytes) {
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if (n) *n = db->n;
    if (residues) *residues = db->total_res;
    if (device_bytes) {
        // everything the handle itself allocated: its image, workspace, plan copies, alignment buffers
        size_t b = db->image_own.bytes + db->ws_own.bytes + db->align_dirs.bytes + db->align_bnd.bytes +
                   db->align_misc.bytes + db->mode_plan.items.bytes + db->batch_plan.items.bytes +
                   db->batch_plan.qpairs.bytes + db->multi_plan.items.bytes + db->multi_plan.qpairs.bytes;
        for (const auto& kv : db->plans) b += kv.second.items.bytes + kv.second.qpairs.bytes;
        *device_bytes = (int64_t)b;
    }
    return SW_OK;
}

sw_status sw_search(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets, int64_t n,
                    const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_scores_out,
                    sw_stream stream) {
    g_err.clear();
    return search_one(h_query, qlen, db, h_offsets, n, h_subst, gap_open, gap_extend, d_scores_out, nullptr, 0,
                      static_cast<hipStream_t>(stream));
}

sw_status sw_search_ws(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets, int64_t n,
                       const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_scores_out,
                       void* d_workspace, int64_t ws_bytes, sw_stream stream) {
    g_err.clear();
    if (!d_workspace) return fail(SW_E_INVALID, "workspace is NULL");
    return search_one(h_query, qlen, db, h_offsets, n, h_subst, gap_open, gap_extend, d_scores_out, d_workspace,
                      ws_bytes, static_cast<hipStream_t>(stream));
}

sw_status sw_topk(const int32_t* d_scores, int64_t n, int32_t k, int32_t* d_top_scores, int64_t* d_top_index,
                  sw_stream stream) {
    return sw_topk_ws(d_scores, n, k, d_top_scores, d_top_index, nullptr, 0, stream);
}

sw_status sw_topk_ws_bytes(int64_t n, int32_t k, int64_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(SW_E_INVALID, "bytes is NULL");
    if (n < 0) return fail(SW_E_INVALID, "n must be >= 0");
    if (k < 1 || k > 1024) return fail(SW_E_UNSUPPORTED, "k must be in 1..1024 (got %d)", k);
    *bytes = topk_ws_bytes(n, 1, k);
    return SW_OK;
}

sw_status sw_topk_ws(const int32_t* d_scores, int64_t n, int32_t k, int32_t* d_top_scores, int64_t* d_top_index,
                     void* d_workspace, int64_t ws_bytes, sw_stream stream) {
    g_err.clear();
    if (n < 0) return fail(SW_E_INVALID, "n must be >= 0");
    if (k < 1 || k > 1024) return fail(SW_E_UNSUPPORTED, "k must be in 1..1024 (got %d)", k);
    if ((n > 0 && !d_scores) || !d_top_scores || !d_top_index) return fail(SW_E_INVALID, "NULL pointer");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t need = topk_ws_bytes(n, 1, k);
    if (d_workspace && need > 0 && ws_bytes < need) return fail(SW_E_SIZE, "workspace of %lld bytes < %lld", (long long)ws_bytes, (long long)need);
    HIP_TRY(launch_topk_ws(d_scores, n, n, 1, k, d_top_scores, d_top_index, need > 0 ? d_workspace : nullptr, st));
    return SW_OK;
}

sw_status sw_search_batch(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                          const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t k, int32_t* d_scores,
                          int32_t* d_top_scores, int64_t* d_top_index, sw_stream stream) {
    g_err.clear();
    return search_batch(h_queries, h_qoffsets, nq, db, h_subst, gap_open, gap_extend, k, d_scores, d_top_scores,
                        d_top_index, nullptr, 0, static_cast<hipStream_t>(stream));
}

sw_status sw_search_batch_ws(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                             const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t k, int32_t* d_scores,
                             int32_t* d_top_scores, int64_t* d_top_index, void* d_workspace, int64_t ws_bytes,
                             sw_stream stream) {
    g_err.clear();
    if (!d_workspace) return fail(SW_E_INVALID, "workspace is NULL");
    return search_batch(h_queries, h_qoffsets, nq, db, h_subst, gap_open, gap_extend, k, d_scores, d_top_scores,
                        d_top_index, d_workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

sw_status sw_batch_workspace_bytes(sw_db* db, const int64_t* h_qoffsets, int32_t nq, int32_t k, int32_t scores_in_ws,
                                   int64_t* bytes) {
    g_err.clear();
    sw_status s;
    if (!db || !bytes) return fail(SW_E_INVALID, "NULL argument");
    if (nq < 0 || (nq > 0 && !h_qoffsets)) return fail(SW_E_INVALID, "bad query offsets");
    if (k < 0 || k > 1024) return fail(SW_E_UNSUPPORTED, "k must be in 0..1024 (got %d)", k);
    for (int q = 0; q < nq; ++q)
        if (h_qoffsets[q + 1] < h_qoffsets[q]) return fail(SW_E_INVALID, "query offsets decrease at %d", q);
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    if ((s = ensure_geometry(db)) != SW_OK) return s;
    std::vector<int> qlens(nq);
    for (int q = 0; q < nq; ++q) qlens[q] = (int)(h_qoffsets[q + 1] - h_qoffsets[q]);
    Plan* plan = nullptr;
    if ((s = plan_for(db, qlens, &plan)) != SW_OK) return s;
    const int64_t zero[1] = {0};
    *bytes = ws_layout(db, nq ? h_qoffsets : zero, nq, k, scores_in_ws != 0, plan).total;
    return SW_OK;
}

sw_status sw_search_multi(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, const int32_t* h_chunk,
                          int32_t nchunks, sw_db* db, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend,
                          int32_t* const* h_d_scores, sw_stream stream) {
    g_err.clear();
    sw_status s;
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if ((s = check_subst_gaps(h_subst, gap_open, gap_extend)) != SW_OK) return s;
    if (nq < 0 || nchunks < 1) return fail(SW_E_INVALID, "nq must be >= 0 and nchunks >= 1");
    if (nq > 0 && (!h_qoffsets || !h_queries || !h_chunk || !h_d_scores)) return fail(SW_E_INVALID, "NULL argument");
    for (int q = 0; q < nq; ++q) {
        if (h_qoffsets[q + 1] < h_qoffsets[q]) return fail(SW_E_INVALID, "query offsets decrease at %d", q);
        if (h_qoffsets[q + 1] - h_qoffsets[q] > (1 << 24)) return fail(SW_E_UNSUPPORTED, "query %d too long", q);
        if (h_chunk[q] < 0 || h_chunk[q] >= nchunks) return fail(SW_E_INVALID, "chunk %d of query %d outside 0..%d", h_chunk[q], q, nchunks - 1);
        if (db->n > 0 && !h_d_scores[q]) return fail(SW_E_INVALID, "score vector of query %d is NULL", q);
    }
    if (nq > 0)
        for (int64_t i = h_qoffsets[0]; i < h_qoffsets[nq]; ++i)
            if (h_queries[i] < 0 || h_queries[i] >= db->alphabet) return fail(SW_E_RESIDUE, "query residue outside 0..%d at %lld", db->alphabet - 1, (long long)i);
    if (nq == 0 || db->n == 0) return SW_OK;
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = ensure_geometry(db)) != SW_OK) return s;
    std::vector<int> qlens(nq), chunk(h_chunk, h_chunk + nq);
    for (int q = 0; q < nq; ++q) qlens[q] = (int)(h_qoffsets[q + 1] - h_qoffsets[q]);
    // a zero-length query scores 0 on its chunk: fill its whole vector (other chunks are 0 as well)
    for (int q = 0; q < nq; ++q)
        if (qlens[q] == 0) HIP_TRY(launch_fill(h_d_scores[q], db->n, 0, st));
    HIP_TRY(hipStreamSynchronize(st));              // the previous call may still read the plan buffer
    if ((s = build_plan(db, qlens, &db->multi_plan, &chunk, nchunks)) != SW_OK) return s;
    if (db->multi_plan.n_main + db->multi_plan.n_side == 0) return SW_OK;
    Work W;
    if ((s = get_work(db, h_qoffsets, nq, 0, false, &db->multi_plan, nullptr, 0, &W)) != SW_OK) return s;
    Staged S;
    if ((s = stage_queries(db, W, h_queries, h_qoffsets, nq, h_subst, 0, st, &S, h_d_scores)) != SW_OK) return s;
    return enqueue(db, S, db->multi_plan, W, gap_open, gap_extend, nullptr, db->n, 0, nullptr, nullptr, st, true);
}

sw_status sw_profile_kernels(sw_db* db, int32_t enable) {
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    db->timing = enable != 0;
    db->ev_used.clear();
    return SW_OK;
}

sw_status sw_kernel_times(sw_db* db, float* ms_out, int32_t cap, int32_t* count) {
    if (!db || !count || (cap > 0 && !ms_out)) return fail(SW_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    *count = 0;
    for (int i : db->ev_used) {
        HIP_TRY(hipEventSynchronize(db->ev_pool[i].second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, db->ev_pool[i].first, db->ev_pool[i].second));
        if (*count < cap) ms_out[(*count)++] = ms;
    }
    db->ev_used.clear();
    return SW_OK;
}

sw_status sw_last_stats(sw_db* db, int64_t out[8]) {
    if (!db || !out) return fail(SW_E_INVALID, "NULL argument");
    DeviceGuard dg(db->device);
    int32_t c[kCounters] = {};
    if (db->last_counters) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(c, db->last_counters, sizeof c, hipMemcpyDeviceToHost));
    }
    out[0] = db->last_items;
    out[1] = c[1];
    out[2] = db->last_rows;
    out[3] = (int64_t)db->last_grid * kWaves;
    out[4] = db->last_side_items;
    out[5] = db->last_side_rows;
    out[6] = c[5];
    out[7] = std::max<int64_t>(0, (int64_t)c[1] - db->last_cap);
    return SW_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ alignments
namespace {
constexpr int64_t kAlignBudget = (int64_t)4 << 30;   // direction bytes per round of pairs
}

sw_status sw_align_batch(const int8_t* h_queries, const int64_t* h_qoffsets, int32_t nq, sw_db* db,
                         const int64_t* h_subjects, const int64_t* h_soffsets, const int8_t* h_subst, int32_t gap_open,
                         int32_t gap_extend, sw_alignment* h_out, char* h_ops, int64_t ops_stride, sw_stream stream) {
    g_err.clear();
    sw_status s;
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if ((s = check_subst_gaps(h_subst, gap_open, gap_extend)) != SW_OK) return s;
    if (nq < 0) return fail(SW_E_INVALID, "nq must be >= 0");
    if (nq > 0 && (!h_qoffsets || !h_soffsets)) return fail(SW_E_INVALID, "NULL offsets");
    if (nq == 0) return SW_OK;
    if (h_soffsets[0] < 0) return fail(SW_E_INVALID, "subject offsets start below 0");
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t m = h_qoffsets[q + 1] - h_qoffsets[q];
        if (m < 0) return fail(SW_E_INVALID, "query offsets decrease at %d", q);
        if (m > (1 << 20)) return fail(SW_E_UNSUPPORTED, "query %d longer than 2^20 residues", q);
        if (h_soffsets[q + 1] < h_soffsets[q]) return fail(SW_E_INVALID, "subject offsets decrease at %d", q);
        if (m > 0 && !h_queries) return fail(SW_E_INVALID, "queries is NULL");
        for (int64_t i = h_qoffsets[q]; i < h_qoffsets[q + 1]; ++i)
            if (h_queries[i] < 0 || h_queries[i] >= db->alphabet)
                return fail(SW_E_RESIDUE, "query %d residue %d at %lld outside 0..%d", q, h_queries[i],
                            (long long)(i - h_qoffsets[q]), db->alphabet - 1);
    }
    const int64_t s0 = h_soffsets[0], npairs = h_soffsets[nq] - s0;
    if (npairs > 0 && (!h_subjects || !h_out || !h_ops)) return fail(SW_E_INVALID, "NULL subjects or outputs");
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t m = h_qoffsets[q + 1] - h_qoffsets[q];
        for (int64_t k = h_soffsets[q]; k < h_soffsets[q + 1]; ++k) {
            const int64_t sub = h_subjects[k - s0];
            if (sub < 0 || sub >= db->n) return fail(SW_E_INVALID, "subject index %lld outside 0..n-1", (long long)sub);
            if (ops_stride < m + db->lens[sub])
                return fail(SW_E_SIZE, "ops_stride %lld < query + subject (%lld) for query %d", (long long)ops_stride,
                            (long long)(m + db->lens[sub]), q);
            h_out[k - s0] = sw_alignment{0, 0, 0, sub, 0, 0, 0};
        }
    }
    // pairs with a non-empty query, longest first, so that the biggest fills start first
    struct Job { int64_t k; int32_t q; int32_t m; int32_t n; int64_t cost; };
    std::vector<Job> jobs;
    for (int32_t q = 0; q < nq; ++q) {
        const int32_t m = (int32_t)(h_qoffsets[q + 1] - h_qoffsets[q]);
        if (m == 0) continue;
        for (int64_t k = h_soffsets[q]; k < h_soffsets[q + 1]; ++k) {
            const int32_t n = db->lens[h_subjects[k - s0]];
            jobs.push_back({k - s0, q, m, n, align_dir_bytes(m, n)});
        }
    }
    if (jobs.empty()) return SW_OK;
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) { return a.cost > b.cost; });
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int lds_max = 0;                                // LDS a workgroup may use (64 KiB on older parts, 160 KiB on gfx950)
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, db->device));
    if ((s = ensure_geometry(db)) != SW_OK) return s;      // the side stream
    // A long pair's fill runs on one workgroup for as long as its many stages take; spread over tiles of one
    // band by tn columns (one anti-diagonal of tiles per launch) it finishes in about (bands + tiles) tile
    // sweeps instead.  Which pairs: db->align_tiles (0: both sides of the matrix at least kTileMinSide).
    constexpr int kTileMinSide = 2048;
    auto tiled = [&](const Job& J) {
        return J.n > 0 && (db->align_tiles == 2 || (db->align_tiles == 0 && J.m >= kTileMinSide && J.n >= kTileMinSide));
    };
    auto tile_cols = [](int n) { return n >= 4096 ? 256 : 128; };
    size_t j0 = 0;
    while (j0 < jobs.size()) {
        // a round: pairs whose direction bytes fit the budget (at least one pair)
        size_t j1 = j0;
        int64_t dir_total = 0, bnd_total = 0, stride = 1, tws_total = 0;
        int W = 1;
        std::vector<int32_t> qs_used;
        while (j1 < jobs.size()) {
            const Job& J = jobs[j1];
            if (j1 > j0 && dir_total + J.cost > kAlignBudget) break;
            dir_total += round_up(J.cost, 256);
            bnd_total += align_bnd_words(J.n);
            stride = std::max<int64_t>(stride, (int64_t)J.m + J.n + 1);
            qs_used.push_back(J.q);
            ++j1;
        }
        // the round's pairs filled by one workgroup each first, then the tiled ones
        std::stable_partition(jobs.begin() + j0, jobs.begin() + j1, [&](const Job& J) { return !tiled(J); });
        int nfill = 0;
        for (size_t j = j0; j < j1; ++j)
            if (!tiled(jobs[j])) {
                W = std::max(W, align_waves(jobs[j].m, db->alphabet, lds_max));
                ++nfill;
            }
        std::sort(qs_used.begin(), qs_used.end());
        qs_used.erase(std::unique(qs_used.begin(), qs_used.end()), qs_used.end());
        const int np = (int)(j1 - j0);
        const int ntiled = np - nfill;
        // misc: pairs | best (3 int32 each) | info (4 int64 each) | tiles | matrix | queries | ops
        const size_t o_pairs = 0;
        const size_t o_best = round_up(sizeof(AlignPair) * np, 256);
        const size_t o_info = o_best + round_up(12 * (size_t)np, 256);
        const size_t o_tiles = o_info + round_up(32 * (size_t)np, 256);
        const size_t o_sm = o_tiles + round_up(sizeof(AlignTile) * std::max(ntiled, 1), 256);
        const size_t o_query = o_sm + 1024;
        std::vector<int64_t> qpos(nq, -1);
        size_t qbytes = 0;
        for (int32_t q : qs_used) {
            qpos[q] = (int64_t)qbytes;
            qbytes += (size_t)round_up(h_qoffsets[q + 1] - h_qoffsets[q], 256);
        }
        const size_t o_ops = o_query + qbytes;
        const size_t misc = o_ops + (size_t)np * stride;
        std::vector<AlignPair> pairs(np);
        std::vector<AlignTile> tiles;
        int64_t dir_off = 0, bnd_off = 0;
        int ndiag = 0, max_diag_tiles = 0;
        for (int i = 0; i < np; ++i) {
            const Job& J = jobs[j0 + i];
            const int64_t sub = h_subjects[J.k];
            const int32_t slot = db->slot_of[sub];
            const int g = slot / kGroupSubjects, w = slot % kGroupSubjects;
            AlignPair& P = pairs[i];
            P.residues = db->d_image + db->gbase[g] + (int64_t)(w >> 1) * 8 + (w & 1) * 4;
            P.n = J.n;
            P.m = J.m;
            P.dir_off = dir_off;
            P.bnd_off = bnd_off;
            dir_off += round_up(J.cost, 256);
            bnd_off += align_bnd_words(J.n);
            if (i >= nfill && J.n > 0) {
                AlignTile T;
                T.pair = i;
                T.nb = (J.m + 255) / 256;
                T.tn = tile_cols(J.n);
                T.nc = (J.n + T.tn - 1) / T.tn;
                T.ws_off = tws_total;
                tws_total += round_up(2 * (int64_t)J.m + T.nb + 3 * (int64_t)T.nb * T.nc, 64);
                ndiag = std::max(ndiag, T.nb + T.nc - 1);
                max_diag_tiles = std::max(max_diag_tiles, std::min(T.nb, T.nc));
                tiles.push_back(T);
            }
        }
        HIP_TRY(db->align_dirs.reserve((size_t)std::max<int64_t>(dir_total, 256)));
        HIP_TRY(db->align_bnd.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(bnd_total, 64)));
        HIP_TRY(db->align_misc.reserve(misc));
        HIP_TRY(db->align_tws.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(tws_total, 64)));
        char* mb = db->align_misc.as<char>();
        for (int i = 0; i < np; ++i) pairs[i].query = reinterpret_cast<const int8_t*>(mb + o_query + qpos[jobs[j0 + i].q]);
        HIP_TRY(hipMemcpyAsync(mb + o_pairs, pairs.data(), sizeof(AlignPair) * np, hipMemcpyHostToDevice, st));
        if (!tiles.empty())
            HIP_TRY(hipMemcpyAsync(mb + o_tiles, tiles.data(), sizeof(AlignTile) * tiles.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(mb + o_sm, h_subst, (size_t)db->alphabet * db->alphabet, hipMemcpyHostToDevice, st));
        for (int32_t q : qs_used)
            HIP_TRY(hipMemcpyAsync(mb + o_query + qpos[q], h_queries + h_qoffsets[q], (size_t)(h_qoffsets[q + 1] - h_qoffsets[q]),
                                   hipMemcpyHostToDevice, st));
        const AlignPair* d_pairs = reinterpret_cast<AlignPair*>(mb + o_pairs);
        const int8_t* d_sm = reinterpret_cast<int8_t*>(mb + o_sm);
        int32_t* d_best = reinterpret_cast<int32_t*>(mb + o_best);
        // the one-workgroup fills on the side stream while the tiled ones run on the caller's
        const bool fork = nfill > 0 && !tiles.empty();
        const hipStream_t fs = fork ? db->side : st;
        if (fork) {
            HIP_TRY(hipEventRecord(db->ev_fork, st));
            HIP_TRY(hipStreamWaitEvent(db->side, db->ev_fork, 0));
        }
        HIP_TRY(launch_align_fill(d_pairs, nfill, W, d_sm, db->alphabet, gap_open, gap_extend, db->align_dirs.as<uint8_t>(),
                                  db->align_bnd.as<int32_t>(), d_best, lds_max, fs));
        if (fork) HIP_TRY(hipEventRecord(db->ev_join, db->side));
        HIP_TRY(launch_align_tiles(d_pairs, reinterpret_cast<AlignTile*>(mb + o_tiles), (int)tiles.size(), ndiag,
                                   max_diag_tiles, d_sm, db->alphabet, gap_open, gap_extend, db->align_dirs.as<uint8_t>(),
                                   db->align_bnd.as<int32_t>(), db->align_tws.as<int32_t>(), d_best, st));
        if (fork) HIP_TRY(hipStreamWaitEvent(st, db->ev_join, 0));
        HIP_TRY(launch_align_trace(d_pairs, np, db->align_dirs.as<uint8_t>(), d_best, mb + o_ops, stride,
                                   reinterpret_cast<int64_t*>(mb + o_info), st));
        std::vector<int32_t> best(3 * (size_t)np);
        std::vector<int64_t> info(4 * (size_t)np);
        std::vector<char> ops((size_t)np * stride);
        HIP_TRY(hipMemcpyAsync(best.data(), mb + o_best, 12 * (size_t)np, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(info.data(), mb + o_info, 32 * (size_t)np, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(ops.data(), mb + o_ops, (size_t)np * stride, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int i = 0; i < np; ++i) {
            const Job& J = jobs[j0 + i];
            if (info[4 * i + 3] != 0)
                return fail(SW_E_HIP, "inconsistent traceback for subject %lld", (long long)h_subjects[J.k]);
            sw_alignment& A = h_out[J.k];
            const int64_t len = info[4 * i + 2];
            A.score = best[3 * i];
            A.q_begin = (int32_t)info[4 * i];
            A.q_end = best[3 * i + 1];
            A.s_begin = info[4 * i + 1];
            A.s_end = best[3 * i + 2];
            A.n_ops = len;
            char* dst = h_ops + J.k * ops_stride;
            const char* src = ops.data() + (size_t)i * stride;
            for (int64_t x = 0; x < len; ++x) dst[x] = src[len - 1 - x];     // the walk wrote them last to first
        }
        j0 = j1;
    }
    return SW_OK;
}

sw_status sw_align(const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_subjects, int32_t nsub,
                   const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, sw_alignment* h_out, char* h_ops,
                   int64_t ops_stride, sw_stream stream) {
    g_err.clear();
    if (!db) return fail(SW_E_INVALID, "db is NULL");
    if (qlen < 0 || nsub < 0) return fail(SW_E_INVALID, "qlen and nsub must be >= 0");
    if (qlen > 0 && !h_query) return fail(SW_E_INVALID, "query is NULL");
    const int64_t qo[2] = {0, qlen}, so[2] = {0, nsub};
    return sw_align_batch(h_query, qo, 1, db, h_subjects, so, h_subst, gap_open, gap_extend, h_out, h_ops, ops_stride,
                          stream);
}

// ------------------------------------------------------------------ end-to-end modes
namespace {
int64_t gap_run(int64_t k, int64_t go, int64_t ge) { return k <= 0 ? 0 : -(go + (k - 1) * std::min(go, ge)); }
}

sw_status sw_search_mode(int32_t mode, const int8_t* h_query, int32_t qlen, sw_db* db, const int64_t* h_offsets,
                         int64_t n, const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_scores_out,
                         sw_stream stream) {
    if (mode == SW_LOCAL)
        return sw_search(h_query, qlen, db, h_offsets, n, h_subst, gap_open, gap_extend, d_scores_out, stream);
    g_err.clear();
    if (mode != SW_GLOBAL && mode != SW_SEMIGLOBAL) return fail(SW_E_INVALID, "mode must be 0, 1 or 2 (got %d)", mode);
    sw_status s;
    if ((s = check_db_args(db, h_offsets, n)) != SW_OK) return s;
    if ((s = check_subst_gaps(h_subst, gap_open, gap_extend)) != SW_OK) return s;
    if (qlen < 0) return fail(SW_E_INVALID, "qlen must be >= 0");
    if (qlen > 0 && !h_query) return fail(SW_E_INVALID, "query is NULL");
    if (n > 0 && !d_scores_out) return fail(SW_E_INVALID, "scores_out is NULL");
    for (int32_t i = 0; i < qlen; ++i)
        if (h_query[i] < 0 || h_query[i] >= db->alphabet)
            return fail(SW_E_RESIDUE, "query residue %d at %d outside 0..%d", h_query[i], i, db->alphabet - 1);
    // every value of the recurrence stays within +-2^29: gap runs cost at most Go + (m + n) max(Go, Ge)
    const int64_t span = (int64_t)qlen + db->ncols_max + 1;
    if ((int64_t)gap_open + span * std::max(gap_open, gap_extend) >= ((int64_t)1 << 29) || span * 127 >= ((int64_t)1 << 29))
        return fail(SW_E_UNSUPPORTED, "gap penalties x lengths too large for 32-bit end-to-end scores");
    if (n == 0) return SW_OK;
    std::lock_guard<std::mutex> lk(db->mu);
    DeviceGuard dg(db->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (qlen == 0) {
        // one gap run per subject (global) or nothing to align (semi-global)
        std::vector<int32_t> v((size_t)n);
        for (int64_t k = 0; k < n; ++k) v[k] = mode == SW_GLOBAL ? (int32_t)gap_run(db->lens[k], gap_open, gap_extend) : 0;
        HIP_TRY(hipMemcpyAsync(d_scores_out, v.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        return SW_OK;
    }
    if ((s = ensure_geometry(db)) != SW_OK) return s;
    if (db->wg_mode == 0) {
        int b1 = 0, b2 = 0;
        int b3 = 0;
        HIP_TRY(sweep_occupancy_mode16(SW_GLOBAL, 16, &b1));
        HIP_TRY(sweep_occupancy_mode16(SW_SEMIGLOBAL, 16, &b2));
        HIP_TRY(sweep_occupancy_mode16(kModeGlobalOffset, 16, &b3));
        const int b = std::min(std::min(std::min(b1, b2), b3), kMaxWgPerCu);
        if (b < 1) return fail(SW_E_HIP, "16-bit end-to-end sweep cannot be resident");
        db->wg_mode = std::min(db->cus * b, db->wg16);     // within the 16-bit boundary slots
    }
    // 16-bit cells hold values in [128 - bias, kModeTop - bias).  Semi-global H never falls below the
    // gap run down the query, g(m) = -(Go + (m - 1) Ge), so its bias is just large enough for that (at
    // most the middle of the range), which leaves the most room above for high scores.  Global mode with
    // Ge <= Go runs on column-offset cells H' = H - g(j) (g(j) the row-0 gap run to column j): every H'
    // is at least g(m) too, whatever the subject's length, so it takes the same bias; the profile then
    // carries SM + Ge, E extends for free and opens at Go - Ge, and a score is H'[m][n] + g(n).  Global
    // mode with Ge > Go keeps plain cells at the middle of the range, and so do long queries: their own
    // bias is high, and their long similar subjects are lifted by -g(n) as well, so high scorers leave
    // the range and go to the serial 32-bit recompute, where plain cells run the longest subjects in
    // 32 bits beside the 16-bit launch.  Offset cells are used while the query's bias stays within 2/5
    // of the middle one (queries up to about 3,100 residues at 10/2): there the 32-bit chain of a long
    // subject, which they remove, is the longer path (measured on the 570,000-subject workload).
    const int64_t offset_bias = 128 + (int64_t)gap_open + (int64_t)(qlen - 1) * gap_extend;
    const bool offset = mode == SW_GLOBAL && gap_extend <= gap_open && 5 * offset_bias <= 2 * (int64_t)kModeBias;
    int32_t bias = kModeBias;
    if (mode == SW_SEMIGLOBAL || offset)
        bias = (int32_t)std::min<int64_t>(kModeBias, 128 + (int64_t)gap_open + (int64_t)(qlen - 1) * gap_extend);
    // A query whose column-0 border (the gap run down its length) falls below the range runs wholly in
    // 32-bit cells; with plain global cells so do the longest subjects, whose row-0 border does (a prefix
    // of the length-sorted groups).
    const int64_t lowest = 128 - (int64_t)bias;
    int g_split = 0;                              // groups [0, g_split) run in 32-bit cells
    if (gap_run(qlen, gap_open, gap_extend) < lowest) g_split = db->ngroups;
    else if (mode == SW_GLOBAL && !offset)
        while (g_split < db->ngroups && gap_run(db->ncols[g_split], gap_open, gap_extend) < lowest) ++g_split;
    const bool use_offset = offset && g_split == 0;
    const int mode16 = use_offset ? kModeGlobalOffset : mode;      // the 16-bit kernels' form
    const int32_t sm_shift = use_offset ? gap_extend : 0;
    // 16-bit plan at 16 rows per lane; the long pairs of a short query go to a side list at 4 or 8 rows
    std::vector<WgItem> mi, si, m32, s32;
    if (g_split < db->ngroups) {
        PlanLimits lim{16, db->slot_cap, (int64_t)db->wg_mode * kWaves};
        lim.side = true;
        plan_units(db, std::vector<int>{qlen}, &db->mode_plan, mi, si, nullptr, 1, &lim, g_split, -1);
    }
    // (4 rows per lane measured no faster for the 32-bit chain of a short query, and slower for longer ones)
    constexpr int R32 = 8;
    if (g_split > 0) {
        // 32-bit units in the 32-bit boundary slots: one wave slot holds the widest subject's columns
        const PlanLimits lim32{R32, std::max<int64_t>(db->ncols_max, 4), (int64_t)db->wg32 * kWaves};
        Plan tmp;
        plan_units(db, std::vector<int>{qlen}, &tmp, m32, s32, nullptr, 1, &lim32, 0, g_split);
    }
    HIP_TRY(hipStreamSynchronize(st));            // the plan buffer may still be read by an earlier launch
    // device item list: [16-bit main..., 16-bit side..., 32-bit...]
    const size_t n16 = mi.size(), n16s = si.size(), n_items = n16 + n16s + m32.size();
    HIP_TRY(db->mode_plan.items.reserve(sizeof(WgItem) * std::max<size_t>(n_items, 1)));
    mi.insert(mi.end(), si.begin(), si.end());
    mi.insert(mi.end(), m32.begin(), m32.end());
    if (n_items) HIP_TRY(hipMemcpy(db->mode_plan.items.p, mi.data(), sizeof(WgItem) * n_items, hipMemcpyHostToDevice));
    const int64_t qo[2] = {0, qlen};
    Work W;
    if ((s = get_work(db, qo, 1, 0, false, nullptr, nullptr, 0, &W)) != SW_OK) return s;
    Staged S;
    if ((s = stage_queries(db, W, h_query, qo, 1, h_subst, 0, st, &S)) != SW_OK) return s;
    int32_t* ctr = W.counters;
    HIP_TRY(launch_profile(S.sm_q, db->alphabet, S.qd, S.nq, S.qoff, W.prof, ctr, kCounters, W.bits, W.L.bits_words,
                           S.max_mp, st, sm_shift));
    SweepArgs a = sweep_args(db, S, W, gap_open, gap_extend, d_scores_out);
    a.sm_shift = sm_shift;
    a.items = db->mode_plan.items.as<WgItem>();
    a.n_items = (int32_t)n16;
    a.counter = ctr + 0;
    set_rerun_args(db, a, W, ctr);
    a.unit_list = 0;
    // every value carries the bias; a pair whose H leaves [128, sat) is recomputed
    a.bias = bias;
    a.sat = db->sat < kSat16 ? std::min<int32_t>(bias + db->sat, kModeTop) : kModeTop;
    // the 16-bit side launch takes the first slots; the 16-bit bulk launch fills the rest
    const int grid_side = n16s ? std::min<int>((int)n16s, std::max(1, db->wg_mode / 8)) : 0;
    const int grid = std::max(1, std::min<int>(db->wg_mode - grid_side, std::max<int>((int)n16, 1)));
    if (n16s || !m32.empty()) {
        HIP_TRY(hipEventRecord(db->ev_fork, st));
        if (n16s) HIP_TRY(hipStreamWaitEvent(db->side, db->ev_fork, 0));
        if (!m32.empty()) HIP_TRY(hipStreamWaitEvent(db->side2, db->ev_fork, 0));
    }
    if (n16s) {
        // long pairs of a short query at fewer rows per lane, concurrently on the side stream
        SweepArgs b = a;
        b.items = db->mode_plan.items.as<WgItem>() + n16;
        b.n_items = (int32_t)n16s;
        b.counter = ctr + 3;
        b.slot_base = grid;
        HIP_TRY(launch_sweep_mode16(mode16, db->mode_plan.R_side, b, grid_side, db->side));
        HIP_TRY(hipEventRecord(db->ev_join, db->side));
    }
    if (!m32.empty()) {
        // the longest subjects in 32-bit cells, concurrently on the second side stream
        SweepArgs b = a;
        b.items = db->mode_plan.items.as<WgItem>() + n16 + n16s;
        b.n_items = (int32_t)m32.size();
        b.counter = ctr + 4;
        b.scratch = W.scratch32;
        b.slot_words = (int64_t)std::max<int32_t>(db->ncols_max, 4) * 4;
        b.rerun = nullptr;
        b.rerun_count = nullptr;
        b.rerun_cap = 0;
        b.poison = 0;
        b.bias = 0;
        HIP_TRY(launch_sweep_mode(mode, R32, b, std::max(1, std::min<int>(db->wg32, (int)m32.size())), db->side2));
        HIP_TRY(hipEventRecord(db->ev_join2, db->side2));
    }
    const int ev = db->timing ? record_timer_start(db, st) : -1;
    if (n16 > 0) HIP_TRY(launch_sweep_mode16(mode16, 16, a, grid, st));
    // the recompute reads the side launches' rerun entries and reuses the 32-bit slots; the timed
    // region of the sweep ends when all three launches have
    if (n16s) HIP_TRY(hipStreamWaitEvent(st, db->ev_join, 0));
    if (!m32.empty()) HIP_TRY(hipStreamWaitEvent(st, db->ev_join2, 0));
    if (ev >= 0) {
        HIP_TRY(hipEventRecord(db->ev_pool[ev].second, st));
        db->ev_used.push_back(ev);
    }
    // exact 32-bit recompute of the pairs that left the range; the count is read on the device
    SweepArgs r = recompute_args(db, a, W, ctr);
    r.bias = 0;
    HIP_TRY(launch_sweep_mode(mode, kRerunRows, r, db->wg32, st));
    db->last_items = (int)n16;
    db->last_rows = 16;
    db->last_side_items = (int)(n16s + m32.size());
    db->last_side_rows = n16s ? db->mode_plan.R_side : m32.empty() ? 0 : R32;
    db->last_grid = grid + grid_side;
    db->last_counters = ctr;
    return SW_OK;
}
