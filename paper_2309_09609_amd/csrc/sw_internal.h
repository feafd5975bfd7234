// Library-internal layout and launch descriptors shared by the host code and
// the gfx950 kernels of libswsearch.  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace sw {

// ---------------------------------------------------------------- constants
constexpr int kMaxAlphabet = 24;  // residue codes 0..alphabet-1, alphabet <= 24 (20 amino acids + B, Z, X, *)
constexpr int kNRes = kMaxAlphabet + 1;   // profile rows: padding (image code 0) and residues (codes 1..24)
constexpr int kPadCode = 0;        // image byte of padding columns (residue codes are stored + 1)
constexpr int16_t kPadScore = 0;       // substitution score of padding: never above a real score's effect
                                       // (S is unchanged), and padded cells copy real values diagonally
                                       // instead of decaying, so the 16-bit range checks of the end-to-end
                                       // modes see only values of real cells
constexpr int kGroupPairs = 64;    // subject pairs per group (one per lane of a wave)
constexpr int kGroupSubjects = 2 * kGroupPairs;
constexpr int kChunkCols = 4;      // columns per interleaved chunk (one dword per subject)
constexpr int kChunkBytes = kGroupPairs * 8;   // one chunk row of a group: 64 pairs x 2 subjects x 4 residues
constexpr int kWaves = 4;          // waves per workgroup of the sweep kernel
constexpr int kRowsMax = 16;       // most query rows per lane (R) of any sweep instance
constexpr int kSliceRows = 1024;   // largest rows-per-pass (B*R) kept in LDS: 64 lanes x 16 rows
constexpr int kProfRowAlign = 1024;    // profile row stride is a multiple of this (covers every B*R)
constexpr int16_t kSat16 = 0x7C00; // 16-bit scores at or above this are recomputed in 32 bits
// End-to-end modes in 16-bit cells: every value carries kModeBias (the middle of
// the exact range), and a pair whose H leaves [128, kModeTop) is recomputed in 32 bits.
constexpr int32_t kModeBias = 0x3E00;
constexpr int32_t kModeTop = 0x7C00 - 128;
// Test hook: what a flagged pair's 16-bit scores read until its 32-bit recompute overwrites them.
constexpr int32_t kPoison = -0x3B9ACA07;

// Packed database image, one record per group of 128 length-sorted subjects.
// Residues of group g live at image + base, as chunk rows of kChunkBytes bytes:
// byte (chunk c, pair p, half h, k) = 1 + residue (4c + k) of subject 2p + h of the group,
// or kPadCode (0) past the subject's end.  Columns are padded to a multiple of 4.
struct GroupRec {
    int64_t base;     // byte offset of the group's first chunk row
    int32_t ncols;    // padded column count (multiple of 4) = longest subject of the group, rounded up
    int32_t first;    // index of the group's first subject in length-sorted order (= 128 g)
};

// One unit of work for a wave: pairs [k*P, (k+1)*P) of group g, P = 64 >> lgB, with B = 1 << lgB
// lanes cooperating on each pair.  A workgroup item bundles up to kWaves units of one query:
// wave w takes unit k0 + w, carried into the following groups of the item's group sequence
// g0, g0 + gstep, g0 + 2 gstep, ... (gstep > 1 when a search covers every gstep-th group).
struct WgItem {
    int32_t g0;       // group of the first unit
    int32_t q;        // query index within the launch
    int16_t k0;       // sub-group index of the first unit within g0
    int8_t lgB;       // log2 of lanes per pair (0..6)
    int8_t count;     // number of valid units (1..kWaves)
    int32_t gstep;    // distance between consecutive groups of the item
};

// Per-query descriptor.
struct QDesc {
    int64_t prof_off;     // element offset of this query's profile [kNRes][mp] in the profile buffer
    int64_t out_off;      // element offset of this query's score row in the common output
    int32_t* out;         // if non-null: this query's own score vector (out_off is then ignored)
    int32_t m;            // query length (>= 1)
    int32_t mp;           // profile row stride (multiple of kProfRowAlign, >= m)
};

// Form of the 16-bit end-to-end sweep beside SW_GLOBAL (1) and SW_SEMIGLOBAL (2): global scores on
// column-offset cells (Ge <= Go).
constexpr int kModeGlobalOffset = 3;

struct SweepArgs {
    const WgItem* items;
    const int32_t* n_items_dev;   // if non-null, the item count is read here (rerun launches)
    int32_t n_items;              // item count (or capacity when n_items_dev is used)
    int32_t* counter;             // work counter, zeroed before the launch
    const uint8_t* image;
    const GroupRec* groups;
    const int32_t* perm;          // sorted slot -> original subject index, -1 for padding slots
    const int32_t* pair_cols;     // [group*64 + pair]: longest subject of the pair, rounded up to 4
    const int16_t* prof;
    const QDesc* qd;
    int32_t go, ge;
    uint32_t* scratch;            // per-wave boundary-row slots
    int64_t slot_words;           // uint32 words per wave slot
    int32_t slot_base;            // first workgroup slot of this launch (launches share the scratch)
    int32_t* scores;
    WgItem* rerun;                // 16-bit sweep: pairs that saturated are appended here
    int32_t* rerun_count;         // flagged (query, pair) count: appends attempted, listed or not
    int32_t rerun_cap;            // entries of rerun[]; a flagged pair beyond it sets its bit in rerun_bits
    uint32_t* rerun_bits;         // one bit per (query, group, pair): [q][group][2 words], zero before a search
    int32_t rerun_groups;         // groups per query row of rerun_bits (the database's group count)
    int64_t rerun_words;          // words of rerun_bits (queries x groups x 2)
    int32_t* recomputed;          // 32-bit recompute: pairs recomputed (listed and from rerun_bits)
    int32_t poison;               // test hook: a flagged pair's 16-bit scores are written as kPoison
    int32_t unit_list;            // 1: items[] holds one unit per workgroup (rerun list), 0: workgroup items
    int32_t sat;                  // 16-bit scores >= sat (biased) are recomputed with 32-bit cells
    int32_t bias;                 // 16-bit cells carry H, E, F + bias (>= minus the lowest substitution score;
                                  // end-to-end modes: the middle of the 16-bit range)
    const int2* qpairs;           // query-pair sweep: item.q indexes these (query a, query b or -1)
    const int32_t* slen;          // end-to-end modes: subject length per sorted slot (0 for padding slots)
    int32_t sm_shift;             // global mode on column-offset cells: the profile holds SM + sm_shift on
                                  // real residues; 32-bit cells subtract it again
};

// One (query, subject) pair of an alignment launch.
struct AlignPair {
    const uint8_t* residues;  // the subject's first chunk in the image (+ 8 * pair + 4 * half of its group)
    int32_t n;                // subject length
    int32_t m;                // query length (>= 1)
    const int8_t* query;      // the query's residue codes on the device
    int64_t dir_off;          // byte offset of the pair's direction bytes
    int64_t bnd_off;          // int32 offset of the pair's boundary row (H then F, n rounded up to 4 words each)
};

// A pair whose fill is spread over tiles of one band (256 query rows) by tn subject columns.
struct AlignTile {
    int32_t pair;             // index of the pair in the round's AlignPair array
    int32_t nb, nc;           // bands and column tiles
    int32_t tn;               // tile width, a multiple of 64, <= kAlignTileMax
    int64_t ws_off;           // int32 offset in the tile workspace: hcol[m] | ecol[m] | corner[nb] | ends[3 nb nc]
};
constexpr int kAlignTileMax = 256;

}  // namespace sw
