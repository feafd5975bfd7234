// gfx950 kernels of libswsearch: the alignment behind a score (traceback).
//
// Only the top-ranked subjects of a search need their alignment (Sec. II-B);
// it is recovered by tracing back from the cell that holds the highest H.
// On a GPU with hundreds of GB of HBM the direct way pays: one pass over the
// (query x subject) matrix of Eq. 1-3 in 32-bit cells stores one direction
// byte per cell, and one thread then walks the bytes back from the end cell.
//
// Fill.  One wave per (query, subject) pair.  Lane b owns 4 consecutive query
// rows of each pass of 256 rows and at step t updates column j = t - b + 1
// (1-based), so the 64 lanes form an anti-diagonal wavefront; the bottom row
// of lane b reaches lane b+1 through a DPP shift, and the bottom row of the
// pass goes to the next pass through a per-pair boundary buffer.  The 4
// direction bytes a lane produces per step form one dword, and the 64 lanes
// write 256 consecutive bytes per step: byte (pass p, step t, lane b, row r)
// at ((p * (n + 63) + t) * 64 + b) * 4 + r.
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

#include "sw_internal.h"

namespace sw {

constexpr int kAlignRows = 4;                    // query rows per lane
constexpr int kAlignPass = 64 * kAlignRows;      // query rows per pass

__device__ __forceinline__ uint32_t align_shr1(uint32_t v) {
    // lane l receives lane l-1's value; lane 0 receives 0
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}

// (score desc, row asc, column asc): true if (s, i, j) comes before (t, k, l)
__device__ __forceinline__ bool end_before(int s, int i, int j, int t, int k, int l) {
    return s > t || (s == t && (i < k || (i == k && j < l)));
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
// one chunk ahead, so no step waits for memory.
__global__ __launch_bounds__(64) void k_align_fill(const AlignPair* pairs, const int8_t* query, int m,
                                                   const int8_t* subst, int A, int go, int ge, uint8_t* dirs,
                                                   int32_t* bnd, int32_t* best) {
    // query profile of the current pass: prof[d][row], rows of lane b at bytes 4b .. 4b + 3 of each residue row
    __shared__ __attribute__((aligned(16))) int8_t prof[kMaxAlphabet * kAlignPass];
    const AlignPair P = pairs[blockIdx.x];
    const int b = threadIdx.x;
    const int n = P.n;
    const int n4 = (n + 3) & ~3;                // columns rounded up to whole chunks
    const align_rsrc img = align_buffer(P.residues, (uint32_t)(n4 >> 2) * kChunkBytes);
    int32_t* bh = bnd + P.bnd_off;              // last row of the previous pass, 0-based columns: H, then F
    int32_t* bf = bh + n4;
    const align_rsrc bhr = align_buffer(bh, (uint32_t)n4 * 4), bfr = align_buffer(bf, (uint32_t)n4 * 4);
    uint32_t* dir = reinterpret_cast<uint32_t*>(dirs + P.dir_off);
    int best_s = 0, best_i = 0, best_j = 0;     // wave-uniform after each pass
    const int passes = (m + kAlignPass - 1) / kAlignPass;
    const int nsteps = n + 63;
    const int nloop = (nsteps + 3) >> 2;
    const int coff = (-b) >> 2, csh = (-b) & 3;  // lane b works on 0-based columns 4c - b .. 4c - b + 3 in iteration c
    auto chunk = [&](int c) { return __builtin_amdgcn_raw_buffer_load_b32(img, (uint32_t)(c * kChunkBytes), 0, 0); };
    for (int p = 0; p < passes; ++p) {
        const int row0 = p * kAlignPass + b * kAlignRows;     // 0-based first row of this lane
        bool valid[kAlignRows];
#pragma unroll
        for (int r = 0; r < kAlignRows; ++r) valid[r] = row0 + r < m;
        __syncthreads();                        // the previous pass is done with the profile
        for (int e = b; e < A * kAlignPass; e += 64) {
            const int d = e / kAlignPass, row = p * kAlignPass + (e - d * kAlignPass);
            prof[e] = row < m ? subst[query[row] * A + d] : (int8_t)0;
        }
        __syncthreads();
        int H[kAlignRows], E[kAlignRows], bs[kAlignRows], bj[kAlignRows];
#pragma unroll
        for (int r = 0; r < kAlignRows; ++r) { H[r] = 0; E[r] = 0; bs[r] = 0; bj[r] = 0; }
        int diag_top = 0;                       // H of the row above this lane's block, previous column
        int up_h = 0, up_f = 0;                 // bottom row of lane b-1 at this step's column
        const uint32_t rd = (b == 0 && p > 0) ? 0u : 0x80000000u;   // only the first lane reads the boundary
        uint32_t lo = chunk(coff), hi = chunk(coff + 1), nx = chunk(coff + 2);
        uint4 vh = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bhr, rd, 0, 0));
        uint4 vf = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bfr, rd, 0, 0));
        for (int c = 0; c < nloop; ++c) {
            const uint32_t nn = chunk(coff + c + 3);
            const uint4 wh = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bhr, rd + 16u * (c + 1), 0, 0));
            const uint4 wf = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(bfr, rd + 16u * (c + 1), 0, 0));
            const uint32_t rr = __builtin_amdgcn_alignbyte(hi, lo, csh);
            const int th[4] = {(int)vh.x, (int)vh.y, (int)vh.z, (int)vh.w};
            const int tf[4] = {(int)vf.x, (int)vf.y, (int)vf.z, (int)vf.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = 4 * c + u;
                const int j = t - b + 1;        // 1-based column of this lane
                const bool active = j >= 1 && j <= n;
                const int htop = b == 0 ? th[u] : up_h;
                const int ftop = b == 0 ? tf[u] : up_f;
                int hbot = 0, fbot = 0;
                if (active) {
                    const int d = (int)((rr >> (8 * u)) & 0xffu) - 1;
                    const uint32_t sv = *reinterpret_cast<const uint32_t*>(prof + d * kAlignPass + 4 * b);
                    int dg = diag_top, hu = htop, fu = ftop;
                    uint32_t bits = 0;
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
                        bits |= (src | (e == eo ? 4u : 0u) | (f == fo ? 8u : 0u)) << (8 * r);
                        if (valid[r] && h > bs[r]) { bs[r] = h; bj[r] = j; }
                        dg = hl;
                        H[r] = h;
                        E[r] = e;
                        hu = h;
                        fu = f;
                    }
                    dir[((int64_t)p * nsteps + t) * 64 + b] = bits;
                    hbot = hu;
                    fbot = fu;
                    if (b == 63 && p + 1 < passes) { bh[j - 1] = hbot; bf[j - 1] = fbot; }
                }
                diag_top = htop;
                up_h = (int)align_shr1((uint32_t)hbot);
                up_f = (int)align_shr1((uint32_t)fbot);
            }
            lo = hi;
            hi = nx;
            nx = nn;
            vh = wh;
            vf = wf;
        }
        // this pass's first end cell, then the first over all passes
        int s = 0, ci = 0, cj = 0;
#pragma unroll
        for (int r = 0; r < kAlignRows; ++r)
            if (bs[r] > 0 && end_before(bs[r], row0 + r + 1, bj[r], s, ci, cj)) { s = bs[r]; ci = row0 + r + 1; cj = bj[r]; }
        for (int o = 1; o < 64; o <<= 1) {
            const int s2 = __shfl_xor(s, o, 64), i2 = __shfl_xor(ci, o, 64), j2 = __shfl_xor(cj, o, 64);
            if (s2 > 0 && (s == 0 || end_before(s2, i2, j2, s, ci, cj))) { s = s2; ci = i2; cj = j2; }
        }
        if (s > 0 && (best_s == 0 || end_before(s, ci, cj, best_s, best_i, best_j))) { best_s = s; best_i = ci; best_j = cj; }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");   // boundary row visible to the next pass
        __syncthreads();
    }
    if (b == 0) {
        best[3 * blockIdx.x] = best_s;
        best[3 * blockIdx.x + 1] = best_i;
        best[3 * blockIdx.x + 2] = best_j;
    }
}

// One thread per pair: walk the direction bytes back from the end cell.
// Operations are written last to first; begin positions and the count go to
// info[4 * pair] = (q_begin, s_begin, count, status).
__global__ void k_align_trace(const AlignPair* pairs, int npairs, int m, const uint8_t* dirs, const int32_t* best,
                              char* ops, int64_t ops_stride, int64_t* info) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const AlignPair P = pairs[k];
    const int n = P.n;
    const int nsteps = n + 63;
    const uint8_t* dir = dirs + P.dir_off;
    char* out = ops + (int64_t)k * ops_stride;
    int i = best[3 * k + 1], j = best[3 * k + 2];
    int64_t len = 0;
    int state = 0;                              // 0: H, 1: E, 2: F
    int64_t status = 0;
    auto byte_at = [&](int ii, int jj) -> uint32_t {
        const int row = ii - 1;
        const int p = row / kAlignPass, b = (row % kAlignPass) / kAlignRows, r = row % kAlignRows;
        const int t = jj - 1 + b;
        return dir[(((int64_t)p * nsteps + t) * 64 + b) * 4 + r];
    };
    if (best[3 * k] > 0) {
        for (;;) {
            if (i < 1 || j < 1 || i > m || j > n || len >= ops_stride) {
                if (state != 0) status = 1;     // a gap cannot reach the border: inconsistent bytes
                break;
            }
            const uint32_t v = byte_at(i, j);
            if (state == 0) {
                const uint32_t src = v & 3u;
                if (src == 0) break;
                if (src == 1) { out[len++] = 'M'; --i; --j; }
                else state = (int)src - 1;
            } else if (state == 1) {
                out[len++] = 'D';
                if (v & 4u) state = 0;
                --j;
            } else {
                out[len++] = 'I';
                if (v & 8u) state = 0;
                --i;
            }
        }
    } else {
        i = 0;
        j = 0;
    }
    info[4 * k] = i;
    info[4 * k + 1] = j;
    info[4 * k + 2] = len;
    info[4 * k + 3] = status;
}

hipError_t launch_align(const AlignPair* pairs, int npairs, const int8_t* query, int m, const int8_t* subst, int A, int go,
                        int ge, uint8_t* dirs, int32_t* bnd, int32_t* best, char* ops, int64_t ops_stride,
                        int64_t* info, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_align_fill, dim3(npairs), dim3(64), 0, st, pairs, query, m, subst, A, go, ge, dirs, bnd, best);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_align_trace, dim3((npairs + 63) / 64), dim3(64), 0, st, pairs, npairs, m, dirs, best, ops,
                       ops_stride, info);
    return hipGetLastError();
}

int64_t align_bnd_words(int64_t n) { return 2 * ((n + 3) & ~(int64_t)3); }

int64_t align_dir_bytes(int m, int64_t n) {
    const int64_t passes = (m + kAlignPass - 1) / kAlignPass;
    return passes * (n + 63) * 64 * 4;
}

}  // namespace sw
