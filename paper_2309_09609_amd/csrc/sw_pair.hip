// One long pair (query x subject) scored across many workgroups: the
// intra-task parallelism of Sec. II-B (processing elements share one matrix,
// Fig. 1) taken from one wave to the whole GPU, as SW# does for one-to-one
// alignment of long sequences (Sec. III-A).
//
// Smith-Waterman with Gotoh gaps (Eq. 1-3) in int32 cells, E and F floored at
// 0 (H is unchanged by it, H >= 0 anyway).  The matrix is cut into tiles of
// kPairRows query rows by TN subject columns.  Tile (I, J) needs only what
// tiles (I-1, J), (I, J-1) and (I-1, J-1) produced, so the tiles of one
// anti-diagonal I + J = d are independent: launch d runs all of them, one wave
// per tile, and no workgroup ever waits for another (launch order on the
// stream is the only synchronisation).  Between launches the boundary goes
// through the workspace:
//   hrow[j], frow[j]  H of the last row of band I-1 at column j, and F already
//                     advanced to the first row of band I;
//   hcol[i], ecol[i]  H of row i at the last column of the previous tile of
//                     its band, and E already advanced to the next column;
//   corner[I]         H at (first row of band I - 1, first column of the tile
//                     about to run - 1), saved by the tile before it in the
//                     band from the row buffer just before it overwrote it.
// Inside a tile lane b owns rows 4b..4b+3 of the band and at step t updates
// column t - b (an anti-diagonal wavefront across the wave); the bottom row
// of lane b reaches lane b+1 through a DPP shift.  The query profile of the
// band's rows sits in LDS as [residue][lane] dwords of four int8 scores, so a
// step's lookup is conflict-free whatever the residues.  The best H of each
// tile goes to the score with one atomic maximum.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "../../include/swsearch.h"
#include "sw_internal.h"

namespace sw {
sw_status report(sw_status s, const char* fmt, ...);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t st);

constexpr int kPairLanes = 64;
constexpr int kPairRowsPerLane = 4;
constexpr int kPairRows = kPairLanes * kPairRowsPerLane;   // query rows per band (tile height)
constexpr int kPairMaxCols = 256;                          // widest tile (LDS staging)

struct PairArgs {
    const int8_t* q;        // query codes, m
    const int8_t* s;        // subject codes, n
    const int8_t* sm;       // A x A substitution scores [query residue][subject residue]
    int32_t* hrow;          // n
    int32_t* frow;          // n
    int32_t* hcol;          // m
    int32_t* ecol;          // m
    int32_t* corner;        // bands
    int32_t* best;          // the score
    int64_t m, n;
    int32_t A, go, ge;
    int32_t tn;             // tile width (columns), a multiple of 64, <= kPairMaxCols
    int32_t nb, nc;         // bands, column tiles
    int32_t d;              // the anti-diagonal of this launch
};

__device__ __forceinline__ int pair_shr1(int v) {
    // lane l receives lane l-1's value (DPP wave_shr:1); lane 0 receives 0
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

__global__ __launch_bounds__(kPairLanes) void k_pair_tile(PairArgs a) {
    __shared__ uint32_t prof[(kMaxAlphabet + 1) * kPairLanes];   // [residue code + 1][lane]; row 0 padding
    __shared__ uint8_t sres[kPairMaxCols];                       // the tile's subject residues, code + 1
    __shared__ int32_t rowh[kPairMaxCols], rowf[kPairMaxCols];   // the band above: H and advanced F
    __shared__ int32_t outh[kPairMaxCols], outf[kPairMaxCols];   // this band's bottom row
    __shared__ int8_t smat[kMaxAlphabet * kMaxAlphabet];
    const int b = threadIdx.x;
    for (int e = b; e < a.A * a.A; e += kPairLanes) smat[e] = a.sm[e];
    const int I = max(0, a.d - (a.nc - 1)) + blockIdx.x;
    const int J = a.d - I;
    const int64_t i0 = (int64_t)I * kPairRows, j0 = (int64_t)J * a.tn;
    const int w = (int)min<int64_t>(a.tn, a.n - j0);             // real columns of the tile
    const int64_t r0 = i0 + kPairRowsPerLane * b;                // this lane's first row
    // profile: padding scores -128 on every row (a padded row never raises the score), rows past m too
    int qrow[kPairRowsPerLane];                                  // matrix row offset of each of this lane's rows
#pragma unroll
    for (int r = 0; r < kPairRowsPerLane; ++r) qrow[r] = r0 + r < a.m ? a.q[r0 + r] * a.A : -1;
    __syncthreads();                                             // the matrix is in LDS
    prof[b] = 0x80808080u;
    for (int c = 0; c < a.A; ++c) {
        uint32_t v = 0;
#pragma unroll
        for (int r = 0; r < kPairRowsPerLane; ++r)
            v |= (uint32_t)(uint8_t)(qrow[r] >= 0 ? smat[qrow[r] + c] : (int8_t)-128) << (8 * r);
        prof[(c + 1) * kPairLanes + b] = v;
    }
    for (int k = b; k < w; k += kPairLanes) {
        sres[k] = (uint8_t)(a.s[j0 + k] + 1);
        rowh[k] = a.hrow[j0 + k];
        rowf[k] = a.frow[j0 + k];
    }
    __syncthreads();
    // this lane's rows at column j0 - 1: H, and E advanced to column j0
    int H[kPairRowsPerLane], E[kPairRowsPerLane];
#pragma unroll
    for (int r = 0; r < kPairRowsPerLane; ++r) {
        const bool real = r0 + r < a.m;
        H[r] = real ? a.hcol[r0 + r] : 0;
        E[r] = real ? a.ecol[r0 + r] : 0;
    }
    const int corner = a.corner[I];
    // H of the row above this lane's block at column j0 - 1
    int diag = b == 0 ? corner : (r0 - 1 < a.m ? a.hcol[r0 - 1] : 0);
    int up_h = 0, up_f = 0;                                      // lane b-1's bottom row, one column back
    int S = 0;
    const int nsteps = w + kPairLanes - 1;
    // LDS reads run ahead of the step that uses them: the profile word one step, the residue (which
    // addresses it) two steps, the band-above row one step, so no step waits on a dependent pair of loads
    auto colk = [&](int t) { return min(max(t - b, 0), w - 1); };
    uint32_t pv = prof[(int)sres[colk(0)] * kPairLanes + b];
    int res2 = sres[colk(1)];
    int rh = rowh[colk(0)], rf = rowf[colk(0)];
    for (int t = 0; t < nsteps; ++t) {
        const int k = t - b;                                     // column of this lane within the tile
        const bool active = k >= 0 && k < w;
        const uint32_t pv_next = prof[res2 * kPairLanes + b];
        const int res3 = sres[colk(t + 2)];
        const int rh_next = rowh[colk(t + 1)], rf_next = rowf[colk(t + 1)];
        const int htop = b == 0 ? rh : up_h;
        const int ftop = b == 0 ? rf : up_f;
        int hb = 0, fb = 0;
        if (active) {
            int dg = diag, F = ftop;
#pragma unroll
            for (int r = 0; r < kPairRowsPerLane; ++r) {
                const int hd = dg + (int)(int8_t)(pv >> (8 * r));
                const int h = max(max(hd, E[r]), F);             // E, F >= 0: the local floor
                S = max(S, h);
                const int hgo = h - a.go;
                E[r] = max(max(E[r] - a.ge, hgo), 0);
                F = max(max(F - a.ge, hgo), 0);
                dg = H[r];
                H[r] = h;
            }
            diag = htop;
            hb = H[kPairRowsPerLane - 1];
            fb = F;
            if (b == kPairLanes - 1) {
                outh[k] = hb;
                outf[k] = fb;
            }
            if (k == w - 1) {
                // this lane's rows at the tile's last column, for the next tile of the band
#pragma unroll
                for (int r = 0; r < kPairRowsPerLane; ++r)
                    if (r0 + r < a.m) {
                        a.hcol[r0 + r] = H[r];
                        a.ecol[r0 + r] = E[r];
                    }
            }
        }
        up_h = pair_shr1(hb);
        up_f = pair_shr1(fb);
        pv = pv_next;
        res2 = res3;
        rh = rh_next;
        rf = rf_next;
    }
    for (int o = 32; o >= 1; o >>= 1) S = max(S, __shfl_xor(S, o, 64));
    __syncthreads();
    // the bottom row for the band below; the next tile of this band takes its corner from the row
    // buffer's value just before it is overwritten (the last column of this tile)
    const bool last_band = I == a.nb - 1;
    if (!last_band)
        for (int kx = b; kx < w; kx += kPairLanes) {
            a.hrow[j0 + kx] = outh[kx];
            a.frow[j0 + kx] = outf[kx];
        }
    if (b == 0) {
        a.corner[I] = rowh[w - 1];
        if (S > 0) atomicMax(a.best, S);
    }
}

}  // namespace sw

using namespace sw;

namespace {

struct PairLayout { int64_t q, s, sm, hrow, frow, hcol, ecol, corner, fill_words, total; };

int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }

PairLayout pair_layout(int64_t m, int64_t n) {
    PairLayout L{};
    const int64_t nb = (m + kPairRows - 1) / kPairRows;
    L.hrow = 0;                                       // the int32 region first: one fill zeroes it
    L.frow = L.hrow + 4 * n;
    L.hcol = L.frow + 4 * n;
    L.ecol = L.hcol + 4 * m;
    L.corner = L.ecol + 4 * m;
    L.fill_words = (L.corner + 4 * nb) / 4;
    L.q = up256(L.corner + 4 * nb);
    L.s = up256(L.q + m);
    L.sm = up256(L.s + n);
    L.total = up256(L.sm + kMaxAlphabet * kMaxAlphabet);
    return L;
}

int pair_tile_cols(int64_t m, int64_t n) {
    // Wider tiles pay less per tile (the 63-step ramp of each wave) but give fewer tiles per
    // anti-diagonal; 256 columns keeps hundreds of tiles in flight for pairs of tens of thousands.
    (void)m;
    return n >= 4096 ? 256 : 128;
}

}  // namespace

extern "C" {

sw_status sw_pair_workspace_bytes(int64_t qlen, int64_t slen, int64_t* bytes) {
    report(SW_OK, "");
    if (!bytes) return report(SW_E_INVALID, "bytes is NULL");
    if (qlen < 0 || slen < 0) return report(SW_E_INVALID, "lengths must be >= 0");
    if (qlen > ((int64_t)1 << 31) || slen > ((int64_t)1 << 31)) return report(SW_E_UNSUPPORTED, "longer than 2^31");
    *bytes = pair_layout(qlen, slen).total;
    return SW_OK;
}

sw_status sw_pair(const int8_t* h_query, int64_t qlen, const int8_t* h_subject, int64_t slen, int32_t alphabet,
                  const int8_t* h_subst, int32_t gap_open, int32_t gap_extend, int32_t* d_score, void* d_workspace,
                  int64_t ws_bytes, sw_stream stream) {
    report(SW_OK, "");
    if (!d_score) return report(SW_E_INVALID, "score is NULL");
    if (qlen < 0 || slen < 0) return report(SW_E_INVALID, "lengths must be >= 0");
    if ((qlen > 0 && !h_query) || (slen > 0 && !h_subject) || !h_subst) return report(SW_E_INVALID, "NULL input");
    if (qlen > ((int64_t)1 << 31) || slen > ((int64_t)1 << 31)) return report(SW_E_UNSUPPORTED, "longer than 2^31");
    const int A = alphabet > 0 ? alphabet : 20;
    if (A > kMaxAlphabet) return report(SW_E_INVALID, "alphabet must be 0 (= 20) or 1..%d", kMaxAlphabet);
    if (gap_open < 0 || gap_extend < 0) return report(SW_E_INVALID, "gap penalties must be >= 0");
    // int32 cells: the score is at most 127 x min(m, n)
    if (127 * std::min(qlen, slen) >= ((int64_t)1 << 31) - 1) return report(SW_E_UNSUPPORTED, "score may exceed int32");
    for (int64_t i = 0; i < qlen; ++i)
        if (h_query[i] < 0 || h_query[i] >= A) return report(SW_E_RESIDUE, "query residue at %lld outside 0..%d", (long long)i, A - 1);
    for (int64_t i = 0; i < slen; ++i)
        if (h_subject[i] < 0 || h_subject[i] >= A) return report(SW_E_RESIDUE, "subject residue at %lld outside 0..%d", (long long)i, A - 1);
    const PairLayout L = pair_layout(qlen, slen);
    if (qlen > 0 && slen > 0 && (!d_workspace || ws_bytes < L.total))
        return report(SW_E_SIZE, "workspace of %lld bytes < %lld needed", (long long)ws_bytes, (long long)L.total);
    if (d_workspace && (reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0)
        return report(SW_E_INVALID, "workspace not 256-byte aligned");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_fill(d_score, 1, 0, st);
    if (e != hipSuccess) return report(SW_E_HIP, "fill: %s", hipGetErrorString(e));
    if (qlen == 0 || slen == 0) return SW_OK;
    char* base = static_cast<char*>(d_workspace);
    PairArgs a{};
    a.q = reinterpret_cast<const int8_t*>(base + L.q);
    a.s = reinterpret_cast<const int8_t*>(base + L.s);
    a.sm = reinterpret_cast<const int8_t*>(base + L.sm);
    a.hrow = reinterpret_cast<int32_t*>(base + L.hrow);
    a.frow = reinterpret_cast<int32_t*>(base + L.frow);
    a.hcol = reinterpret_cast<int32_t*>(base + L.hcol);
    a.ecol = reinterpret_cast<int32_t*>(base + L.ecol);
    a.corner = reinterpret_cast<int32_t*>(base + L.corner);
    a.best = d_score;
    a.m = qlen;
    a.n = slen;
    a.A = A;
    a.go = gap_open;
    a.ge = gap_extend;
    a.tn = pair_tile_cols(qlen, slen);
    a.nb = (int)((qlen + kPairRows - 1) / kPairRows);
    a.nc = (int)((slen + a.tn - 1) / a.tn);
    if ((e = hipMemcpyAsync(base + L.q, h_query, qlen, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(base + L.s, h_subject, slen, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(base + L.sm, h_subst, (size_t)A * A, hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = launch_fill(reinterpret_cast<int32_t*>(base), L.fill_words, 0, st)) != hipSuccess)
        return report(SW_E_HIP, "set-up: %s", hipGetErrorString(e));
    for (int d = 0; d < a.nb + a.nc - 1; ++d) {
        a.d = d;
        const int lo = std::max(0, d - (a.nc - 1)), hi = std::min(d, a.nb - 1);
        hipLaunchKernelGGL(k_pair_tile, dim3(hi - lo + 1), dim3(kPairLanes), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return report(SW_E_HIP, "tile launch: %s", hipGetErrorString(e));
    }
    return SW_OK;
}

}  // extern "C"
