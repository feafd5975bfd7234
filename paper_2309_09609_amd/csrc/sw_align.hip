// gfx950 kernels of libswsearch: the alignment behind a score (traceback).
//
// Only the top-ranked subjects of a search need their alignment (Sec. II-B);
// it is recovered by tracing back from the cell that holds the highest H.
// On a GPU with hundreds of GB of HBM the direct way pays: one pass over the
// (query x subject) matrix of Eq. 1-3 in 32-bit cells stores one direction
// byte per cell, and one thread then walks the bytes back from the end cell.
//
// Fill.  One workgroup of up to 16 waves per (query, subject) pair.  The
// query is cut into bands of 256 rows; lane b of the wave holding a band owns
// 4 consecutive rows and at step t updates column j = t - b + 1 (1-based), so
// the 64 lanes form an anti-diagonal wavefront and the bottom row of lane b
// reaches lane b+1 through a DPP shift.  Band k goes to wave k mod W, and the
// bands run as a pipeline of 128-step stages: band k starts 2 stages after
// band k-1, whose bottom row (H and F per column, in a per-pair row buffer) it
// reads, and every W-th band waits max(0, nch - 2W) stages more (nch = stages
// per band) so that its wave has finished its previous band; a workgroup
// barrier ends every stage.  Lag 2 covers the 64 steps a column needs to
// cross a band plus one step of read-ahead.  The 4 direction bytes a lane produces per
// step form one dword, and the 64 lanes write 256 consecutive bytes per
// step: byte (band p, step t, lane b, row r) at ((p * (n + 63) + t) * 64 + b)
// * 4 + r.
//
// A long pair's fill can instead be spread over tiles of one band by 128 or
// 256 columns, one anti-diagonal of tiles per launch (k_align_tile): it writes
// the same bytes and finds the same end cell, in about (bands + column tiles)
// tile sweeps instead of the one workgroup's many stages.
//
// Walk.  One wave per pair copies the 256-byte step records of up to 128
// steps of the current band into LDS and follows the path through them until
// it leaves the copied steps; every move keeps or lowers the step index, so
// each copy serves dozens of moves.  The wave takes a run of equal moves (a
// diagonal stretch, a gap) at once: each lane checks one cell of the run and
// a ballot finds where it ends.
//
// Direction byte of cell (i, j):
//   bits 0-1  where H comes from: 0 H = 0 (an alignment starts after this
//             cell), 1 the diagonal H[i-1][j-1] + SM, 2 E, 3 F -- the first
//             that equals H in this order;
//   bit 2     E[i][j] = H[i][j-1] - Go (the horizontal gap opens at j-1);
//   bit 3     F[i][j] = H[i-1][j] - Go (the vertical gap opens at i-1).
// End cell: the first cell with H = S in row-major order.  These choices fix
// one alignment among those that reach S.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <climits>

#include <algorithm>

#include "sw_internal.h"

namespace sw {

constexpr int kAlignRows = 4;                    // query rows per lane
constexpr int kAlignPass = 64 * kAlignRows;      // query rows per band
constexpr int kAlignWaves = 16;                  // bands in flight per pair
constexpr int kAlignStage = 32;                  // iterations of 4 steps per stage
constexpr int kTraceSteps = 128;                 // steps per LDS copy of the walk

__device__ __forceinline__ uint32_t align_shr1(uint32_t v) {
    // lane l receives lane l-1's value; lane 0 receives 0
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

// (score desc, row asc, column asc): true if (s, i, j) comes before (t, k, l)
__device__ __forceinline__ bool end_before(int s, int i, int j, int t, int k, int l) {
    return s > t || (s == t && (i < k || (i == k && j < l)));
}

// The direction byte of a cell (layout above) from its values: h = max(hd, e, f, 0), e = max(eo, ee),
// f = max(fo, fe).  With nz, nd, ne = 0 when h equals 0, hd, e, the source is nz (nd (ne + 1) + 1): 0,
// then 1, 2 or 3 in the stated order; ee - eo - 1 is negative exactly when eo >= ee (a gap that opens
// here), likewise for F.  The opening bits come from sign bits rather than compare/select pairs, which
// all pass through one condition register and wait on it between compare and select: a lone wave (the
// tiled fill) gains by that (7 % on a 40,000 x 40,000 pair), while the one-workgroup fill, whose waves
// share a SIMD and hide those waits, runs its two more instructions per row 4 % slower and keeps the
// plain compare form.
__device__ __forceinline__ uint32_t dir_byte(int h, int hd, int e, int eo, int ee, int fo, int fe) {
    const uint32_t nz = min((uint32_t)h, 1u);
    const uint32_t nd = min((uint32_t)(h - hd), 1u);                 // h >= hd
    const uint32_t ne = min((uint32_t)(h - e), 1u);                  // h >= e
    const uint32_t src = nz * (nd * (ne + 1u) + 1u);
    const uint32_t eob = ((uint32_t)(ee - eo - 1) >> 31) << 2;
    const uint32_t fob = ((uint32_t)(fe - fo - 1) >> 31) << 3;
    return src | eob | fob;
}

typedef __amdgpu_buffer_rsrc_t align_rsrc;

// Raw buffer over [base, base + bytes): out-of-range loads return zeros.
__device__ __forceinline__ align_rsrc align_buffer(const void* base, uint32_t bytes) {
    const uint64_t p = (uint64_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p), hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0,
                                             (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

// Residues arrive 4 columns per dword two chunks ahead and the boundary row
// one iteration ahead, so no step waits for memory.  Dynamic LDS: the query
// profile of each wave's band, prof[c][row] for image byte c (0 = padding,
// 1..A = residue c - 1) with the rows of lane b at bytes 4b .. 4b + 3 of each
// row (W * (A + 1) * 256 bytes), built from a copy of the substitution matrix
// in LDS.  Padding scores -128.
// Every lane computes every step, also before its first column and past the
// last: there the diagonal term is H + (-128) from a zero border, so H stays
// 0 before the first column, and E may drift below 0 -- such E (and F) never
// lie on an alignment's path, which only follows positive values.  Cells past
// the last column feed no real cell (those depend only on cells to their left
// and above); they may start from stale boundary words of a padding column
// and are never taken as the end cell.  Only the direction stores past the
// band's steps and the bottom-row stores are guarded.
// A pair with fewer bands than the workgroup has waves leaves the other waves
// idle (they still take part in every barrier).
__global__ __launch_bounds__(64 * kAlignWaves) void k_align_fill(const AlignPair* pairs, const int8_t* subst, int A,
                                                                 int go, int ge, uint8_t* dirs, int32_t* bnd,
                                                                 int32_t* best) {
    extern __shared__ __attribute__((aligned(16))) int8_t align_lds[];
    __shared__ int wbest[kAlignWaves][3];
    __shared__ int8_t sm[kMaxAlphabet * kMaxAlphabet];
    const AlignPair P = pairs[blockIdx.x];
    const int wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = threadIdx.x & 63;
    const int8_t* query = P.query;
    const int m = P.m;
    int8_t* prof = align_lds + wave * ((A + 1) * kAlignPass);
    for (int e = threadIdx.x; e < A * A; e += blockDim.x) sm[e] = subst[e];
    __syncthreads();
    const int n = P.n;
    const int n4 = (n + 3) & ~3;                // columns rounded up to whole chunks
    const align_rsrc img = align_buffer(P.residues, (uint32_t)(n4 >> 2) * kChunkBytes);
    int32_t* bh = bnd + P.bnd_off;              // bottom row of the previous band, 0-based columns: H, then F
    int32_t* bf = bh + n4;
    const align_rsrc bhr = align_buffer(bh, (uint32_t)n4 * 4), bfr = align_buffer(bf, (uint32_t)n4 * 4);
    uint32_t* dir = reinterpret_cast<uint32_t*>(dirs + P.dir_off);
    const int passes = (m + kAlignPass - 1) / kAlignPass;
    const int W = min((int)(blockDim.x >> 6), passes);            // waves of this pair
    const int nsteps = n + 63;
    const int nloop = (nsteps + 3) >> 2;
    const int nch = (nloop + kAlignStage - 1) / kAlignStage;     // stages per band
    // band k starts at stage 2k + (k / W) * D: two stages after band k-1, and every W-th band D stages
    // later still, so that its wave has finished the band before (a wave's bands start max(2W, nch) apart)
    const int D = max(0, nch - 2 * W);
    const int period = 2 * W + D;
    const int nstages = 2 * (passes - 1) + ((passes - 1) / W) * D + nch;
    const int coff = (-b) >> 2, csh = (-b) & 3;  // lane b works on 0-based columns 4c - b .. 4c - b + 3 in iteration c
    auto chunk = [&](int c) { return __builtin_amdgcn_raw_buffer_load_b32(img, (uint32_t)(c * kChunkBytes), 0, 0); };
    int best_s = 0, best_i = 0, best_j = 0;     // wave-uniform after each band
    // state of the wave's band in progress
    int row0 = 0;
    bool valid[kAlignRows];
    int H[kAlignRows], E[kAlignRows], bs[kAlignRows], bj[kAlignRows];
    int diag_top = 0;                           // H of the row above this lane's block, previous column
    int up_h = 0, up_f = 0;                     // bottom row of lane b-1 at this step's column
    uint32_t rd = 0x80000000u;                  // boundary offset: only the first lane of a band > 0 reads
    uint32_t lo = 0, hi = 0, nx = 0;
    uint4 vh = {0, 0, 0, 0}, vf = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < kAlignRows; ++r) { valid[r] = false; H[r] = 0; E[r] = 0; bs[r] = 0; bj[r] = 0; }
    for (int s = 0; s < nstages; ++s) {
        // the band of this wave in stage s, if any: bands wave, wave + W, ... start at 2 wave + i period
        int p = -1, c = 0;
        if (wave < W && s >= 2 * wave) {
            const int i = (s - 2 * wave) / period;
            const int kk = wave + i * W;
            const int cc = s - (2 * wave + i * period);
            if (kk < passes && cc < nch) { p = kk; c = cc; }
        }
        if (p >= 0 && c == 0) {
            row0 = p * kAlignPass + b * kAlignRows;
#pragma unroll
            // rows past the query never become the best (their running maximum starts above every score)
            for (int r = 0; r < kAlignRows; ++r) {
                valid[r] = row0 + r < m;
                H[r] = 0;
                E[r] = 0;
                bs[r] = valid[r] ? 0 : INT_MAX;
                bj[r] = 0;
            }
            int qa[kAlignRows];                 // matrix row offset of each query row, -1 past the query
#pragma unroll
            for (int r = 0; r < kAlignRows; ++r) qa[r] = valid[r] ? query[row0 + r] * A : -1;
            *reinterpret_cast<uint32_t*>(prof + 4 * b) = 0x80808080u;          // padding: -128 on every row
            for (int d = 0; d < A; ++d) {
                uint32_t v = 0;
#pragma unroll
                for (int r = 0; r < kAlignRows; ++r)
                    if (qa[r] >= 0) v |= (uint32_t)(uint8_t)sm[qa[r] + d] << (8 * r);
                *reinterpret_cast<uint32_t*>(prof + (d + 1) * kAlignPass + 4 * b) = v;
            }
            diag_top = 0;
            up_h = 0;
            up_f = 0;
            rd = (b == 0 && p > 0) ? 0u : 0x80000000u;
            lo = chunk(coff);
            hi = chunk(coff + 1);
            nx = chunk(coff + 2);
            vh = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bhr, rd, 0, 0));
            vf = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bfr, rd, 0, 0));
        }
        __syncthreads();                        // the band's profile is in LDS
        if (p >= 0) {
            const int it1 = min(nloop, (c + 1) * kAlignStage);
            for (int it = c * kAlignStage; it < it1; ++it) {
                const uint32_t nn = chunk(coff + it + 3);
                const uint4 wh = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bhr, rd + 16u * (it + 1), 0, 0));
                const uint4 wf = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bfr, rd + 16u * (it + 1), 0, 0));
                const uint32_t rr = __builtin_amdgcn_alignbyte(hi, lo, csh);
                const int th[4] = {(int)vh.x, (int)vh.y, (int)vh.z, (int)vh.w};
                const int tf[4] = {(int)vf.x, (int)vf.y, (int)vf.z, (int)vf.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = 4 * it + u;
                    const int j = t - b + 1;    // 1-based column of this lane
                    const int htop = b == 0 ? th[u] : up_h;
                    const int ftop = b == 0 ? tf[u] : up_f;
                    const int d = (int)((rr >> (8 * u)) & 0xffu);
                    const uint32_t sv = *reinterpret_cast<const uint32_t*>(prof + d * kAlignPass + 4 * b);
                    int dg = diag_top, hu = htop, fu = ftop;
                    uint32_t bits = 0;
                    const bool real = j <= n;   // columns past the subject may read stale boundary words
#pragma unroll
                    for (int r = 0; r < kAlignRows; ++r) {
                        const int hl = H[r];                         // H[i][j-1]
                        const int eo = hl - go, ee = E[r] - ge;
                        const int e = max(eo, ee);                   // Eq. 2
                        const int fo = hu - go, fe = fu - ge;
                        const int f = max(fo, fe);                   // Eq. 3
                        const int hd = dg + (int)(int8_t)(sv >> (8 * r));
                        const int h = max(max(hd, e), max(f, 0));    // Eq. 1
                        const uint32_t src = h == 0 ? 0u : h == hd ? 1u : h == e ? 2u : 3u;
                        bits |= (src | (eo >= ee ? 4u : 0u) | (fo >= fe ? 8u : 0u)) << (8 * r);
                        if (real && h > bs[r]) { bs[r] = h; bj[r] = j; }
                        dg = hl;
                        H[r] = h;
                        E[r] = e;
                        hu = h;
                        fu = f;
                    }
                    if (t < nsteps) dir[((int64_t)p * nsteps + t) * 64 + b] = bits;   // t is the same in every lane
                    // the last lane hands the band's bottom row to the next band (columns 1..n4 only)
                    const uint32_t bo = (b == 63 && p + 1 < passes) ? (uint32_t)(j - 1) * 4u : 0x80000000u;
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)hu, bhr, bo, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)fu, bfr, bo, 0, 0);
                    diag_top = htop;
                    up_h = (int)align_shr1((uint32_t)hu);
                    up_f = (int)align_shr1((uint32_t)fu);
                }
                lo = hi;
                hi = nx;
                nx = nn;
                vh = wh;
                vf = wf;
            }
            if (c == nch - 1) {
                // this band's first end cell, then the first over the wave's bands
                int sc = 0, ci = 0, cj = 0;
#pragma unroll
                for (int r = 0; r < kAlignRows; ++r)
                    if (valid[r] && bs[r] > 0 && end_before(bs[r], row0 + r + 1, bj[r], sc, ci, cj)) {
                        sc = bs[r];
                        ci = row0 + r + 1;
                        cj = bj[r];
                    }
                for (int o = 1; o < 64; o <<= 1) {
                    const int s2 = __shfl_xor(sc, o, 64), i2 = __shfl_xor(ci, o, 64), j2 = __shfl_xor(cj, o, 64);
                    if (s2 > 0 && (sc == 0 || end_before(s2, i2, j2, sc, ci, cj))) { sc = s2; ci = i2; cj = j2; }
                }
                if (sc > 0 && (best_s == 0 || end_before(sc, ci, cj, best_s, best_i, best_j))) { best_s = sc; best_i = ci; best_j = cj; }
            }
        }
        __syncthreads();                        // this stage's bottom rows are visible to the next bands
    }
    if (b == 0 && wave < W) {
        wbest[wave][0] = best_s;
        wbest[wave][1] = best_i;
        wbest[wave][2] = best_j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int sc = 0, ci = 0, cj = 0;
        for (int w = 0; w < W; ++w) {
            const int s2 = wbest[w][0], i2 = wbest[w][1], j2 = wbest[w][2];
            if (s2 > 0 && (sc == 0 || end_before(s2, i2, j2, sc, ci, cj))) { sc = s2; ci = i2; cj = j2; }
        }
        best[3 * blockIdx.x] = sc;
        best[3 * blockIdx.x + 1] = ci;
        best[3 * blockIdx.x + 2] = cj;
    }
}

// Tiled fill for long pairs: the same cells, direction bytes and end cell as
// k_align_fill, computed by many workgroups.  The pair's matrix is cut into
// tiles of one band (256 rows) by tn columns; the tiles of one anti-diagonal
// I + J = d of the tile grid are independent, so launch d runs them all, one
// wave per tile, and launch order is the only synchronisation.  Lane b of a
// tile owns the band's rows 4b..4b+3 as in k_align_fill and writes the
// direction dword of (band step t, lane b) for the columns of its own tile
// only, so the band layout the walk reads comes out the same.  Between
// launches: the band's bottom row (H and F per column) in the pair's row
// buffer, as k_align_fill keeps it; the tile's last column (H and E per row)
// in hcol/ecol; and corner[I], the row buffer's H at the tile's last column,
// saved before the tile overwrites it (the next tile of band I+1 needs it as
// its diagonal).  Each tile writes its first end cell (score desc, row asc,
// column asc) to ends[3 * (I * nc + J)]; k_align_tile_end reduces them.

__global__ __launch_bounds__(64) void k_align_tile(const AlignPair* pairs, const AlignTile* tiles, const int8_t* subst,
                                                   int A, int go, int ge, uint8_t* dirs, int32_t* bnd, int32_t* tws,
                                                   int d, int tile0) {
    __shared__ uint32_t prof[(kMaxAlphabet + 1) * 64];          // [image byte][lane]: 4 rows' scores
    __shared__ uint8_t sres[kAlignTileMax];                      // the tile's image bytes (residue code + 1)
    __shared__ int32_t rowh[kAlignTileMax], rowf[kAlignTileMax]; // the band above: H and F of its last row
    __shared__ int32_t outh[kAlignTileMax], outf[kAlignTileMax]; // this band's last row
    __shared__ int8_t sm[kMaxAlphabet * kMaxAlphabet];
    const AlignTile T = tiles[tile0 + blockIdx.y];
    const int I = max(0, d - (T.nc - 1)) + (int)blockIdx.x;
    if (I >= T.nb || I > d) return;                              // uniform over the workgroup
    const int J = d - I;
    const AlignPair P = pairs[T.pair];
    const int b = threadIdx.x;
    const int m = P.m, n = P.n;
    const int nsteps = n + 63;
    const int j0 = J * T.tn;                                     // 0-based first column of the tile
    const int w = min(T.tn, n - j0);                             // its columns
    const int row0 = I * kAlignPass + b * kAlignRows;            // 0-based first row of this lane
    int32_t* hcol = tws + T.ws_off;
    int32_t* ecol = hcol + m;
    int32_t* corner = ecol + m;
    int32_t* ends = corner + T.nb;
    int32_t* bh = bnd + P.bnd_off;
    int32_t* bf = bh + ((n + 3) & ~3);
    uint32_t* dir = reinterpret_cast<uint32_t*>(dirs + P.dir_off);
    for (int e = b; e < A * A; e += 64) sm[e] = subst[e];
    bool valid[kAlignRows];
    int qa[kAlignRows];
#pragma unroll
    for (int r = 0; r < kAlignRows; ++r) {
        valid[r] = row0 + r < m;
        qa[r] = valid[r] ? P.query[row0 + r] * A : -1;
    }
    __syncthreads();
    // rows past the query score 0 against every residue (as in k_align_fill); they never end an alignment
    prof[b] = 0x80808080u;
    for (int c = 0; c < A; ++c) {
        uint32_t v = 0;
#pragma unroll
        for (int r = 0; r < kAlignRows; ++r)
            if (qa[r] >= 0) v |= (uint32_t)(uint8_t)sm[qa[r] + c] << (8 * r);
        prof[(c + 1) * 64 + b] = v;
    }
    for (int k = b; k < w; k += 64) {
        const int j = j0 + k;
        sres[k] = P.residues[(int64_t)(j >> 2) * kChunkBytes + (j & 3)];
        rowh[k] = I > 0 ? bh[j] : 0;
        rowf[k] = I > 0 ? bf[j] : 0;
    }
    __syncthreads();
    int H[kAlignRows], E[kAlignRows], bs[kAlignRows], bj[kAlignRows];
#pragma unroll
    for (int r = 0; r < kAlignRows; ++r) {
        H[r] = (J > 0 && valid[r]) ? hcol[row0 + r] : 0;
        E[r] = (J > 0 && valid[r]) ? ecol[row0 + r] : 0;
        bs[r] = valid[r] ? 0 : INT_MAX;
        bj[r] = 0;
    }
    // H of the row above this lane's block at the column before the tile (lane 0: the band above's last
    // row, which the tile before this one in the band saved before overwriting it)
    int diag = 0;
    if (J > 0) diag = b == 0 ? corner[I] : (row0 - 1 < m ? hcol[row0 - 1] : 0);
    int up_h = 0, up_f = 0;                                      // lane b-1's last row at this step's column
    const int nst = w + 63;
    // LDS reads run ahead of the step that uses them (the profile word one step, the residue that addresses
    // it two, the band-above row one), so no step waits on a dependent pair of reads
    auto colk = [&](int t) { return min(max(t - b, 0), w - 1); };
    uint32_t pv = prof[(int)sres[colk(0)] * 64 + b];
    int res2 = sres[colk(1)];
    int rh = rowh[colk(0)], rf = rowf[colk(0)];
    for (int t = 0; t < nst; ++t) {
        const int k = t - b;                                     // 0-based column of this lane in the tile
        const bool active = k >= 0 && k < w;
        const uint32_t pv_next = prof[res2 * 64 + b];
        const int res3 = sres[colk(t + 2)];
        const int rh_next = rowh[colk(t + 1)], rf_next = rowf[colk(t + 1)];
        const int htop = b == 0 ? rh : up_h;
        const int ftop = b == 0 ? rf : up_f;
        int hu = 0, fu = 0;
        if (active) {
            const uint32_t sv = pv;
            const int j = j0 + k + 1;                            // 1-based column
            int dg = diag;
            hu = htop;
            fu = ftop;
            uint32_t bits = 0;
#pragma unroll
            for (int r = 0; r < kAlignRows; ++r) {
                const int hl = H[r];
                const int eo = hl - go, ee = E[r] - ge;
                const int e = max(eo, ee);                       // Eq. 2
                const int fo = hu - go, fe = fu - ge;
                const int f = max(fo, fe);                       // Eq. 3
                const int hd = dg + (int)(int8_t)(sv >> (8 * r));
                const int h = max(max(hd, e), max(f, 0));        // Eq. 1
                bits |= dir_byte(h, hd, e, eo, ee, fo, fe) << (8 * r);
                if (h > bs[r]) { bs[r] = h; bj[r] = j; }
                dg = hl;
                H[r] = h;
                E[r] = e;
                hu = h;
                fu = f;
            }
            dir[((int64_t)I * nsteps + j0 + t) * 64 + b] = bits;
            if (b == 63) {
                outh[k] = hu;
                outf[k] = fu;
            }
            if (k == w - 1) {
#pragma unroll
                for (int r = 0; r < kAlignRows; ++r)
                    if (valid[r]) {
                        hcol[row0 + r] = H[r];
                        ecol[row0 + r] = E[r];
                    }
            }
            diag = htop;
        }
        up_h = (int)align_shr1((uint32_t)hu);
        up_f = (int)align_shr1((uint32_t)fu);
        pv = pv_next;
        res2 = res3;
        rh = rh_next;
        rf = rf_next;
    }
    // the tile's first end cell
    int sc = 0, ci = 0, cj = 0;
#pragma unroll
    for (int r = 0; r < kAlignRows; ++r)
        if (valid[r] && bs[r] > 0 && end_before(bs[r], row0 + r + 1, bj[r], sc, ci, cj)) {
            sc = bs[r];
            ci = row0 + r + 1;
            cj = bj[r];
        }
    for (int o = 1; o < 64; o <<= 1) {
        const int s2 = __shfl_xor(sc, o, 64), i2 = __shfl_xor(ci, o, 64), j2 = __shfl_xor(cj, o, 64);
        if (s2 > 0 && (sc == 0 || end_before(s2, i2, j2, sc, ci, cj))) { sc = s2; ci = i2; cj = j2; }
    }
    __syncthreads();
    if (b == 0) corner[I] = rowh[w - 1];                         // for the next tile of this band
    if (I + 1 < T.nb) {
        for (int k = b; k < w; k += 64) {
            bh[j0 + k] = outh[k];
            bf[j0 + k] = outf[k];
        }
    }
    if (b == 0) {
        int32_t* o = ends + 3 * ((int64_t)I * T.nc + J);
        o[0] = sc;
        o[1] = ci;
        o[2] = cj;
    }
}

// The first end cell over a tiled pair's tiles, into best[3 * pair].
__global__ __launch_bounds__(64) void k_align_tile_end(const AlignPair* pairs, const AlignTile* tiles,
                                                       const int32_t* tws, int32_t* best) {
    const AlignTile T = tiles[blockIdx.x];
    const int32_t* ends = tws + T.ws_off + 2 * (int64_t)pairs[T.pair].m + T.nb;
    const int nt = T.nb * T.nc;
    int sc = 0, ci = 0, cj = 0;
    for (int x = threadIdx.x; x < nt; x += 64) {
        const int s2 = ends[3 * x], i2 = ends[3 * x + 1], j2 = ends[3 * x + 2];
        if (s2 > 0 && (sc == 0 || end_before(s2, i2, j2, sc, ci, cj))) { sc = s2; ci = i2; cj = j2; }
    }
    for (int o = 1; o < 64; o <<= 1) {
        const int s2 = __shfl_xor(sc, o, 64), i2 = __shfl_xor(ci, o, 64), j2 = __shfl_xor(cj, o, 64);
        if (s2 > 0 && (sc == 0 || end_before(s2, i2, j2, sc, ci, cj))) { sc = s2; ci = i2; cj = j2; }
    }
    if (threadIdx.x == 0) {
        best[3 * T.pair] = sc;
        best[3 * T.pair + 1] = ci;
        best[3 * T.pair + 2] = cj;
    }
}

// One wave per pair: walk the direction bytes back from the end cell, through
// LDS copies of up to kTraceSteps step records of the band it is in, a run of
// equal moves at a time; the byte of (row rb of the band, 0-based
// column c) sits at ((c + rb / 4 - t0) * 256 + rb) in a copy that starts at
// step t0.  Operations, last to first, collect in LDS and the wave writes
// them out after each copy; begin positions and the count go to
// info[4 * pair] = (q_begin, s_begin, count, status).
constexpr int kTraceOps = 1024;                  // operations buffered in LDS per copy

__global__ __launch_bounds__(64) void k_align_trace(const AlignPair* pairs, const uint8_t* dirs, const int32_t* best,
                                                    char* ops, int64_t ops_stride, int64_t* info) {
    __shared__ __attribute__((aligned(16))) uint8_t tile[kTraceSteps * 256];
    __shared__ char obuf[kTraceOps];
    __shared__ int64_t walk[7];                 // i, j, len, state, done, status, buffered operations
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    const AlignPair P = pairs[k];
    const int n = P.n, m = P.m;
    const int nsteps = n + 63;
    const uint8_t* dir = dirs + P.dir_off;
    char* out = ops + (int64_t)k * ops_stride;
    int i = best[3 * k + 1], j = best[3 * k + 2];
    int64_t len = 0;
    int state = 0;                              // 0: H, 1: E, 2: F
    int64_t status = 0;
    bool done = best[3 * k] <= 0;
    if (done) {
        i = 0;
        j = 0;
    }
    while (!done) {                             // wave-uniform
        if (i < 1 || j < 1 || i > m || j > n || len >= ops_stride) {
            if (state != 0) status = 1;         // a gap cannot reach the border: inconsistent bytes
            break;
        }
        const int row = i - 1;
        const int p = row / kAlignPass;
        const int t = j - 1 + (row % kAlignPass) / kAlignRows;
        const int t0 = max(0, t - kTraceSteps + 1);
        // step records t0 .. t of band p: (t - t0 + 1) * 256 contiguous bytes
        const uint4* src = reinterpret_cast<const uint4*>(dir + ((int64_t)p * nsteps + t0) * 256);
        const int words = (t - t0 + 1) * 16;
        for (int x = lane; x < words; x += 64) reinterpret_cast<uint4*>(tile)[x] = src[x];
        __syncthreads();
        {
            // the wave follows runs of equal moves: lane k looks at the k-th cell of the run (down the
            // diagonal in H, along the row in E, up the column in F) and the first lane whose cell ends
            // the run, or lies outside the copy, the band, the matrix or the room left, decides
            int rb = row - p * kAlignPass;      // row within the band
            int c = j - 1;                      // 0-based column
            int cnt = 0;
            const int64_t room = ops_stride - len;
            const int cap = room < kTraceOps ? (int)room : kTraceOps;
            for (;;) {
                const int rk = state == 1 ? rb : rb - lane;
                const int ck = state == 2 ? c : c - lane;
                const int tk = ck + (rk >> 2);
                const bool ok = rk >= 0 && ck >= 0 && tk >= t0 && cnt + lane < cap;
                const uint32_t v = ok ? tile[(tk - t0) * 256 + rk] : 0u;
                const bool stop = !ok || (state == 0 ? (v & 3u) != 1u : (v & (state == 1 ? 4u : 8u)) != 0u);
                const uint64_t mask = __ballot(stop);
                const int K = mask ? (int)__builtin_ctzll(mask) : 64;
                const bool okK = K < 64 && __shfl((int)ok, K, 64) != 0;
                const uint32_t vK = (uint32_t)__shfl((int)v, K < 64 ? K : 0, 64);
                if (state == 0) {
                    if (lane < K) obuf[cnt + lane] = 'M';
                    cnt += K;
                    rb -= K;
                    c -= K;
                    if (K == 64) continue;
                    if (!okK) break;                             // the outer loop decides
                    const uint32_t sr = vK & 3u;
                    if (sr == 0) { done = true; break; }
                    state = (int)sr - 1;
                } else {
                    const char op = state == 1 ? 'D' : 'I';
                    const int moves = okK ? K + 1 : K;           // the gap's opening cell is its last move
                    if (lane < moves) obuf[cnt + lane] = op;
                    cnt += moves;
                    if (state == 1) c -= moves; else rb -= moves;
                    if (okK) state = 0;
                    else if (K < 64) break;                      // the outer loop decides
                }
            }
            if (lane == 0) {
                walk[0] = rb + p * kAlignPass + 1;
                walk[1] = c + 1;
                walk[2] = len + cnt;
                walk[3] = state;
                walk[4] = done;
                walk[5] = status;
                walk[6] = cnt;
            }
        }
        __syncthreads();
        const int cnt = (int)walk[6];
        for (int x = lane; x < cnt; x += 64) out[len + x] = obuf[x];
        i = (int)walk[0];
        j = (int)walk[1];
        len = walk[2];
        state = (int)walk[3];
        done = walk[4] != 0;
        status = walk[5];
        __syncthreads();                        // everyone has read the state and the buffer before the next copy
    }
    if (lane == 0) {
        info[4 * k] = i;
        info[4 * k + 1] = j;
        info[4 * k + 2] = len;
        info[4 * k + 3] = status;
    }
}

constexpr int kFillStaticLds = 1024;             // k_align_fill's own LDS (matrix copy, per-wave end cells), rounded up

// W = waves per workgroup: the most bands of a pair in the launch, at most 16
// and at most align_waves(., A, lds_max) allows; lds_max = LDS bytes a
// workgroup may use on the device.
hipError_t launch_align_fill(const AlignPair* pairs, int npairs, int W, const int8_t* subst, int A, int go, int ge,
                             uint8_t* dirs, int32_t* bnd, int32_t* best, int lds_max, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    const size_t lds = (size_t)W * (A + 1) * kAlignPass;
    if (W < 1 || W > kAlignWaves || lds + kFillStaticLds > (size_t)lds_max) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_align_fill, dim3(npairs), dim3(64 * W), lds, st, pairs, subst, A, go, ge, dirs, bnd, best);
    return hipGetLastError();
}

// The tiled fill of ntiled pairs (tiles[i].pair indexes pairs): one launch per anti-diagonal of the
// largest tile grid, then the end cells.  max_diag_tiles = the most tiles any pair has on one diagonal.
hipError_t launch_align_tiles(const AlignPair* pairs, const AlignTile* tiles, int ntiled, int ndiag,
                              int max_diag_tiles, const int8_t* subst, int A, int go, int ge, uint8_t* dirs,
                              int32_t* bnd, int32_t* tws, int32_t* best, hipStream_t st) {
    if (ntiled <= 0) return hipSuccess;
    constexpr int kMaxGridY = 65535;
    for (int d = 0; d < ndiag; ++d)
        for (int t0 = 0; t0 < ntiled; t0 += kMaxGridY) {
            hipLaunchKernelGGL(k_align_tile, dim3(max_diag_tiles, std::min(kMaxGridY, ntiled - t0)), dim3(64), 0, st,
                               pairs, tiles, subst, A, go, ge, dirs, bnd, tws, d, t0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    hipLaunchKernelGGL(k_align_tile_end, dim3(ntiled), dim3(64), 0, st, pairs, tiles, tws, best);
    return hipGetLastError();
}

hipError_t launch_align_trace(const AlignPair* pairs, int npairs, const uint8_t* dirs, const int32_t* best, char* ops,
                              int64_t ops_stride, int64_t* info, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_align_trace, dim3(npairs), dim3(64), 0, st, pairs, dirs, best, ops, ops_stride, info);
    return hipGetLastError();
}

// Waves per pair: one per band of 256 query rows, up to 16, with the bands'
// profiles ((A + 1) x 256 bytes each) and the kernel's own LDS within lds_max.
int align_waves(int m, int A, int lds_max) {
    const int passes = (m + kAlignPass - 1) / kAlignPass;
    const int fit = (lds_max - kFillStaticLds) / ((A + 1) * kAlignPass);
    return std::max(1, std::min(std::min(passes, kAlignWaves), fit));
}

int64_t align_bnd_words(int64_t n) { return 2 * ((n + 3) & ~(int64_t)3); }

int64_t align_dir_bytes(int m, int64_t n) {
    const int64_t passes = (m + kAlignPass - 1) / kAlignPass;
    return passes * (n + 63) * 64 * 4;
}

}  // namespace sw
